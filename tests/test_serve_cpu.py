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


def _as_problem(m, probs):
    import dataclasses
    f = {x.name: getattr(m, x.name) for x in dataclasses.fields(gen.Problem) if hasattr(m, x.name)}
    f["pixels"] = np.concatenate([p.pixels for p in probs])
    return gen.Problem(**f)


def test_merged_requests_keep_their_objectives():
    """Merging is exact: the oracle's per-source objectives of the merged problem equal each
    request's own (requests of one survey share the prior)."""
    from oracle import elbo as E
    from paper_1803_00113_amd import serve
    a = gen.crop_patches(gen.config5_request(21, n_sources=3), 20)
    b = gen.crop_patches(gen.config5_request(22, n_sources=2), 20)
    assert serve.same_model(a, b)
    m = _as_problem(serve.merge([a, b]), [a, b])
    loc_m = E.elbo(E.Model(m), m.theta0, with_total=False)[1].numpy()
    loc_a = E.elbo(E.Model(a), a.theta0, with_total=False)[1].numpy()
    loc_b = E.elbo(E.Model(b), b.theta0, with_total=False)[1].numpy()
    assert np.allclose(loc_m, np.concatenate([loc_a, loc_b]), rtol=1e-13, atol=0)


def test_merge_rejects_different_priors():
    import pytest
    from paper_1803_00113_amd import serve
    a = gen.config5_request(11, n_sources=2)
    b = gen.config2(n_sources=2)
    assert not serve.same_model(a, b)
    with pytest.raises(ValueError):
        serve.merge([a, b])
