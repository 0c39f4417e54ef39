"""MI355X (gfx950) implementation of the variational-inference objective of Regier et al.,
"Approximate Inference for Constructing Astronomical Catalogs from Images"
(arXiv 1803.00113): the ELBO and its gradient over each source's active pixels,
trust-region Newton block steps and block coordinate ascent, behind the C ABI of
include/celmi.h (libcelmi.so).

Submodules:
  api       Context / Plan and the calls elbo_eval, elbo_grad, elbo_grad_plain,
            newton_step, sweep (ctypes marshalling only)
  autograd  ElboFunction: torch.autograd.Function over elbo_eval / elbo_grad
  serve     continuous-batching request loop
  build     compiles libcelmi.so for gfx950
The HIP library is required: importing `api` raises ImportError when libcelmi.so is
missing; there is no CPU fallback.
"""
