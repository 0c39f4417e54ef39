"""A hash of a generated problem's inputs (images, patches, pixels, priors, initial
parameters), stored beside the oracle values so that a change of the generator is caught
before stored values are compared with anything."""
import hashlib

import numpy as np

FIELDS = ("img_band", "img_H", "img_W", "img_npsf", "img_psf", "img_A", "img_b", "img_iota", "img_sky_qh",
          "img_sky_qw", "img_sky_off", "sky_knots", "patch_src", "patch_img", "patch_x0", "patch_y0", "patch_w",
          "patch_h", "patch_off", "pixels", "prior_r", "prior_cw", "prior_cmean", "prior_ccov", "prior_radius",
          "prior_profile", "prior_axis", "exp_alpha", "exp_tau", "dev_alpha", "dev_tau", "theta0")


def inputs_hash(prob):
    h = hashlib.sha256()
    h.update(str(int(prob.n_sources)).encode())
    h.update(repr(float(prob.prior_a)).encode())
    for f in FIELDS:
        a = np.ascontiguousarray(getattr(prob, f))
        h.update(f.encode())
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def load_golden(name, prob):
    """The stored oracle values tests/golden/<name>, after checking that they were made from
    the same generated inputs as `prob`."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), name)
    with np.load(path, allow_pickle=False) as z:
        ref = {k: z[k] for k in z.files}
    if str(ref["input_sha256"]) != inputs_hash(prob):
        raise AssertionError(f"{name}: the generator no longer produces the inputs these values were made from")
    return ref
