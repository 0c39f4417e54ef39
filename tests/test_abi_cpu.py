"""The C-ABI library loads and exports every function include/celmi.h declares (no GPU
needed: nothing is called)."""
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "celmi.h")).read()
    return sorted(set(re.findall(r"^\s*(?:cel_status|void|const char\*)\s+(cel_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_function():
    lib = os.path.join(ROOT, "paper_1803_00113_amd", "libcelmi.so")
    if not os.path.exists(lib):
        from paper_1803_00113_amd import build
        build.build()
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (cel_\w+)$", out, re.M))
    declared = _declared()
    assert len(declared) >= 10
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    from paper_1803_00113_amd import _ffi
    assert set(_ffi.EXPORTED) == set(declared)


def test_image_records_match_the_problem():
    """The cel_image records handed to cel_prepare carry every field of every image."""
    import ctypes as C
    import numpy as np
    from paper_1803_00113_amd import api, _ffi as F
    from synth import gen
    prob = gen.config4()
    images = api.host_tables(prob)[0]
    assert images.dtype.itemsize == C.sizeof(F.CelImage)
    recs = C.cast(images.ctypes.data, C.POINTER(F.CelImage))
    for n in range(len(prob.img_band)):
        im = recs[n]
        assert (im.band, im.H, im.W, im.n_psf) == (prob.img_band[n], prob.img_H[n], prob.img_W[n], prob.img_npsf[n])
        assert np.array_equal(np.array([list(r) for r in im.psf]), prob.img_psf[n, :F.MAX_PSF])
        assert np.array_equal(np.array([list(r) for r in im.A]), prob.img_A[n]) and list(im.b) == list(prob.img_b[n])
        assert im.iota == prob.img_iota[n]
        assert (im.sky_qh, im.sky_qw, im.sky_off) == (prob.img_sky_qh[n], prob.img_sky_qw[n], prob.img_sky_off[n])
