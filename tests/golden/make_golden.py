"""Write tests/golden/config1_oracle.json: the oracle's ELBO, per-source objectives and
gradient on the 1-star + 1-galaxy workload.  Calls only oracle/ and the seeded generator.
The paper prints no worked numeric example of the objective, so this file is a regression
pin of the oracle itself (it catches unintended changes to its arithmetic), not an
external value.

Run from the repository root:  python -m tests.golden.make_golden
"""
import json
import os

from oracle import elbo as E
from synth import gen

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    prob = gen.config1()
    m = E.Model(prob)
    total, local, grad = E.elbo_total_and_grad(m, prob.theta0)
    out = dict(workload=prob.name, seed=gen.SEED_BASE + 1, elbo_total=total, elbo_local=local.tolist(),
               grad=grad.tolist())
    with open(os.path.join(HERE, "config1_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
