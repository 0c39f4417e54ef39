"""The lane schedule of the kernels' many-value wavefront sums (csrc/pixmath.h, wave_sums and
wave_sums_slot / wave_sums_lane), restated over 64 emulated lanes: at each lane offset
32, 16, ... a lane keeps half of its values and adds its partner lane's copies of them; a
lone value finishes by butterfly.  Checked here: each of M values ends in exactly one owner
lane (the one wave_sums_lane names), and its sum is bitwise the butterfly sum that one
wavefront sum per value would give, for float32 inputs (widened before the first addition)
and float64 inputs.  Host logic only: the GPU suite checks the kernels' outputs."""
import numpy as np
import pytest

LANES = np.arange(64)


def butterfly(v):
    v = v.astype(np.float64)
    for o in (32, 16, 8, 4, 2, 1):
        v = v + v[LANES ^ o]
    return v


def wave_sums(V, O=32):
    M = V.shape[1]
    if M == 1:
        x = V[:, 0].astype(np.float64)
        while O >= 1:
            x = x + x[LANES ^ O]
            O >>= 1
        return x
    A = (M + 1) // 2
    B = M - A
    hi = (LANES & O) != 0
    W = np.zeros((64, A))
    for i in range(A):
        f = V[:, i]
        s = V[:, A + i] if i < B else np.zeros(64, V.dtype)
        send = np.where(hi, f, s)
        keep = np.where(hi, s, f)
        W[:, i] = keep.astype(np.float64) + send[LANES ^ O].astype(np.float64)
    return wave_sums(W, O // 2)


def slot(M, O, lane):
    if M == 1:
        return 0 if (O == 0 or (lane & (2 * O - 1)) == 0) else -1
    A = (M + 1) // 2
    B = M - A
    r = slot(A, O // 2, lane)
    if r < 0:
        return -1
    if lane & O:
        return A + r if r < B else -1
    return r


def owner_lane(M, q, O=32):
    if M == 1:
        return 0
    A = (M + 1) // 2
    return owner_lane(A, q, O // 2) if q < A else O + owner_lane(A, q - A, O // 2)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_schedule_matches_butterfly_bitwise(dtype):
    rng = np.random.default_rng(7)
    for M in range(1, 65):
        # magnitudes over 16 decades and mixed signs, so that the addition order shows
        V = (rng.standard_normal((64, M)) * 10.0 ** rng.integers(-8, 8, (64, M))).astype(dtype)
        s = wave_sums(V)
        owners = {}
        for lane in range(64):
            q = slot(M, 32, lane)
            if q < 0:
                continue
            assert q not in owners
            owners[q] = lane
            assert s[lane] == butterfly(V[:, q])[0]
        assert sorted(owners) == list(range(M))
        assert all(owner_lane(M, q) == owners[q] for q in range(M))
