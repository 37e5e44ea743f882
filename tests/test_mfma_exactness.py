"""Host-side proofs of the preconditions the matrix-core kernels rely on for
bit-exactness (see the header of kernels_mfma.hip): worst-case ranges of
every intermediate over all 8-bit blocks and all retention masks, and the
float32 rounding of the final numerator."""
import numpy as np

from oracle import codec
from oracle import transform as tf


def _box_max(K, lo=-128, hi=127):
    pos = np.where(K > 0, K, 0)
    neg = np.where(K < 0, K, 0)
    mx = (pos * hi + neg * lo).sum(axis=(-2, -1))
    mn = (pos * lo + neg * hi).sum(axis=(-2, -1))
    return float(np.maximum(np.abs(mx), np.abs(mn)).max())


import pytest


@pytest.mark.parametrize("name,mat,umax_want,nmax_want", [("T", tf.T, 212544, 1648452),
                                                       ("WHT", tf.wht(), 208464, 1327662)])
def test_intermediate_ranges_all_masks(name, mat, umax_want, nmax_want):
    T = mat.astype(np.float64)
    w = tf.inverse_weights(mat).astype(np.float64)
    KP = np.einsum("fb,ia->ifab", T, np.eye(16))           # P = Xc T^T
    KZ = np.einsum("ua,vb->uvab", T, T)                    # Z = T Xc T^T
    assert _box_max(KP) <= 2048                            # fp16-exact
    assert _box_max(KZ) <= 32768
    masks = [codec.mask_none()] + [codec.mask_zonal(r) for r in range(1, 17)] + \
            [codec.mask_zigzag(r) for r in range(1, 257)]
    umax = nmax = 0.0
    for M in masks:
        KU = np.einsum("u,ui,uf,ufab->ifab", w, T, M.astype(float), KZ)
        KN = np.einsum("f,fj,ifab->ijab", w, T, KU)
        umax = max(umax, _box_max(KU))
        nmax = max(nmax, _box_max(KN))
    # 1536 + U 2^-11 must stay inside [1024, 2048), where fp16 steps by 1.
    assert umax / 2048 < 512
    # N 2^-11 (with the stage-4 partial sums) must stay below 1024 so that a
    # multiple of 2^-11 is exact in float32; N itself far below 2^24.
    assert nmax / 2048 + 96 < 1024 and nmax < 2**24
    assert umax == umax_want and nmax == nmax_want
    # the final rounding below is proven for |N| <= 1648452
    assert nmax <= 1648452
    # collapsed products: G = T^T diag(w m) T is integer with |G| <= 68, so
    # G 2^-11 is exact in fp16
    for r in range(1, 17):
        g = T.T @ np.diag(w * (np.arange(16) < r)) @ T
        assert np.abs(g).max() <= 68 and np.array_equal(g, np.rint(g))


def test_final_rounding_is_exact():
    n = np.arange(-1648452, 1648453, dtype=np.int64)
    s = n.astype(np.longdouble) / 2048                      # exact in float32 too
    c = np.longdouble(np.float32(8.0 / 9.0))
    off = np.longdouble(np.float32(128.0 + 1.0 / 4096.0))
    t = (s * c + off).astype(np.float32)                    # one rounding: the FMA
    got = np.clip(np.rint(t), 0, 255).astype(np.int64)      # cvt_pk_u8: nearest-even, saturating
    want = np.clip(np.floor_divide(n + 1152, 2304) + 128, 0, 255)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("name,mat", [("T", tf.T), ("WHT", tf.wht())])
def test_int8_round_trip_ranges(name, mat):
    """The int8 round trip (N = G Xc G, G = T^T diag(w m) T for r x r masks)
    needs G in int8, |Xc G| small enough for two signed base-256 digits
    (top digit in int8), and every int32 sum exact."""
    T = mat.astype(np.int64)
    w = tf.inverse_weights(mat).astype(np.int64)
    for r in range(1, 17):
        g = T.T @ np.diag(w * (np.arange(16) < r)) @ T
        assert np.abs(g).max() <= 48
        vmax = 128 * np.abs(g).sum(axis=0).max()          # |Xc G| over the pixel box
        assert vmax <= 13312
        assert (vmax + 128) >> 8 <= 127 and (-vmax + 128) >> 8 >= -128
        # digit products |G^T s| <= 128 sum |G|; N = s0 G + 256 s1 G below 2^31
        assert 128 * np.abs(g).sum(axis=0).max() * 257 < 2**31
        assert _box_max(np.einsum("ia,bj->ijab", g, g)) <= 1648452   # |N|: the proven rounding range


def test_int8_digits_reassemble():
    rng = np.random.default_rng(3)
    v = np.concatenate([np.arange(-13312, 13313), rng.integers(-13312, 13313, 1000)])
    s0 = ((v & 255) ^ 128) - 128       # the low byte read as int8
    s1 = (v + 128) >> 8                # byte 1 of v + 128
    assert np.array_equal(256 * s1 + s0, v)
    assert s0.min() >= -128 and s0.max() <= 127 and s1.min() >= -128 and s1.max() <= 127


def test_wave_sum_digits_recombine():
    """The 64-bit wavefront sum adds the 24-, 24- and 16-bit digits of the 64
    lane values separately (each digit sum below 2^30, so 32-bit adds do not
    overflow) and recombines them: the result equals the plain sum modulo
    2^64, for random values and for the extremes."""
    rng = np.random.default_rng(64)
    cases = [rng.integers(0, 2**63, size=64, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=64, dtype=np.uint64)
             for _ in range(200)]
    cases += [np.full(64, 2**64 - 1, dtype=np.uint64), np.zeros(64, dtype=np.uint64),
              np.full(64, 2**24 - 1, dtype=np.uint64), np.full(64, 2**48 - 1, dtype=np.uint64)]
    for v in cases:
        vals = [int(x) for x in v]
        d0 = sum(x & 0xFFFFFF for x in vals)
        d1 = sum((x >> 24) & 0xFFFFFF for x in vals)
        d2 = sum(x >> 48 for x in vals)
        assert max(d0, d1, d2) < 2**32
        assert (d0 + (d1 << 24) + (d2 << 48)) % 2**64 == sum(vals) % 2**64
