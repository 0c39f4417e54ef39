"""Host logic of the serving loop (no GPU): merging requests and footprint estimates."""
import numpy as np

from synth import gen


def test_merge_offsets_and_footprint():
    from paper_1803_00113_amd import serve
    a = gen.config5_request(11, n_sources=3)
    b = gen.config5_request(12, n_sources=5)
    m = serve.merge([a, b])
    assert m.n_sources == 8
    assert len(m.img_band) == len(a.img_band) + len(b.img_band)
    assert np.array_equal(m.patch_src[:a.n_patches], a.patch_src)
    assert np.array_equal(m.patch_src[a.n_patches:], b.patch_src + 3)
    assert np.array_equal(m.patch_img[a.n_patches:], b.patch_img + len(a.img_band))
    assert np.array_equal(m.patch_off[a.n_patches:], b.patch_off + len(a.pixels))
    assert np.array_equal(m.img_sky_off[len(a.img_band):], b.img_sky_off + len(a.sky_knots))
    assert np.array_equal(m.theta0, np.vstack([a.theta0, b.theta0]))
    assert serve.footprint_bytes(b) > serve.footprint_bytes(a) > 0
