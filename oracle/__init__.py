"""FP64 CPU reference ("oracle") for the VI objective of Regier et al., "Approximate
Inference for Constructing Astronomical Catalogs from Images" (arXiv 1803.00113).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its Python
binding) may import, call or link anything here; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path; the only common
input is the seeded problem generator in `synth/`, which holds no method arithmetic.

Modules:
  elbo    -- variational objective (Section 4.2, Supplement A) and its derivatives by
             reverse-mode autodiff in float64
  newton  -- trust-region Newton block step, graph colouring and block coordinate ascent
             (Sections 4.3-4.4)
  likelihood -- Poisson log-likelihood at point values of the latent variables, the
             likelihood factor of the MCMC procedure's target (Sections 3 and 3.1)

Parity status per function is listed in each function's docstring ("pinned by ..." or
"parity unpinned").
"""
