"""Pins of the CPU oracle against what the paper prints and what the
mathematics fixes.  No expected value here comes from the HIP path.

Each pin is written as a function returning the list of failures, so that
``test_pins_catch_planted_mistakes`` can plant plausible mistakes in a copy
of the oracle (on the CPU) and show that some pin fails for each of them.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import codec, metrics
from oracle import transform as tf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ----------------------------------------------------------------------------
# Pins written as functions of an oracle-like namespace.

def pin_orthogonality(T):
    """Section 2: T T^T is diagonal and its diagonal is the printed 1/S^2."""
    bad = []
    g = T @ T.T
    if np.count_nonzero(g - np.diag(np.diag(g))):
        bad.append("T T^T not diagonal")
    want = np.array(_golden("s_diag.json")["inv_sqrt_of"])
    if not np.array_equal(np.diag(g), want):
        bad.append("diag(T T^T) != printed S^-2")
    return bad


def pin_table2(T, C):
    """Table 2: d2, epsilon, MSE, Cg, eta of S T and of the exact DCT at the
    printed number of decimals."""
    bad = []
    n = np.diag(T @ T.T).astype(np.float64)
    ch = (1.0 / np.sqrt(n))[:, None] * T.astype(np.float64)
    rows = _golden("table2.json")["rows"]
    for name, mat in (("Proposed", ch), ("DCT", C)):
        got = metrics.table2_row(C, mat)
        for k, txt in rows[name].items():
            dec = len(txt.split(".")[1]) if "." in txt else 0
            if abs(got[k] - float(txt)) > 0.5 * 10.0 ** (-dec) + 1e-12:
                bad.append(f"{name}.{k}: {got[k]} vs printed {txt}")
    return bad


def pin_forward_bruteforce(forward, seed=3, nblk=4):
    """Z[u,v] = sum_a sum_b T[u,a] A[a,b] T[v,b], with T taken from the
    factorisation's product (independent of the literal) and the sums
    written out as Python loops."""
    P = np.eye(16, dtype=np.int64)
    for f in tf.factors():
        P = f @ P
    rng = np.random.default_rng(seed)
    blocks = rng.integers(-300, 300, size=(nblk, 16, 16))
    got = forward(blocks)
    bad = []
    for k in range(nblk):
        A = blocks[k].tolist()
        for u in range(16):
            for v in range(16):
                s = 0
                for a in range(16):
                    for b in range(16):
                        s += int(P[u, a]) * A[a][b] * int(P[v, b])
                if s != int(got[k, u, v]):
                    bad.append((k, u, v))
    return bad


def pin_inverse_identity(inverse_num, forward):
    """Orthogonality of C_hat: with nothing discarded the round trip
    reconstructs the block exactly (numerator = 2304 * A)."""
    rng = np.random.default_rng(11)
    a = rng.integers(0, 256, size=(32, 16, 16))
    num = inverse_num(forward(a))
    return [] if np.array_equal(num, 2304 * a) else ["round trip numerator != 2304 A"]


# ----------------------------------------------------------------------------
# Matrix facts.

def test_T_orthogonality_and_S():
    assert pin_orthogonality(tf.T) == []
    ch = tf.c_hat()
    assert np.max(np.abs(ch @ ch.T - np.eye(16))) < 1e-15
    assert np.max(np.abs(ch.T @ ch - np.eye(16))) < 1e-15
    # T^T T itself is not diagonal: only the scaled matrix is orthogonal.
    g = tf.T.T @ tf.T
    assert np.count_nonzero(g - np.diag(np.diag(g))) > 0


def test_T_entries_and_symmetry():
    assert set(np.unique(tf.T).tolist()) == {-1, 0, 1}
    # Only row 0 has a non-zero sum: a flat block has only a DC coefficient.
    assert tf.T.sum(axis=1).tolist() == [16] + [0] * 15
    # Even rows are symmetric, odd rows antisymmetric, like the DCT's.
    for i in range(16):
        r = tf.T[i]
        assert np.array_equal(r[::-1], r if i % 2 == 0 else -r)


def test_factorisation_product_is_T():
    P = np.eye(16, dtype=np.int64)
    for f in tf.factors():
        P = f @ P
    assert np.array_equal(P, tf.T)


def test_p2_reading():
    # The printed cycles repeat their first element; the chosen reading
    # maps a -> b within each cycle.  The opposite direction fails.
    sig = tf.p2_sigma()
    assert sig.tolist() == [0, 8, 4, 11, 3, 9, 5, 12, 1, 13, 7, 10, 2, 14, 6, 15]
    rev = [list(reversed(c)) for c in tf.P2_CYCLES]
    fs = tf.factors()
    fs[-1] = tf.factor_P2(rev)
    P = np.eye(16, dtype=np.int64)
    for f in fs:
        P = f @ P
    assert not np.array_equal(P, tf.T)


def test_addition_count_table1():
    want = _golden("table1.json")["proposed"]
    per = [tf.additions(f) for f in tf.factors()]
    assert per == [16, 0, 16, 24, 4, 0]
    assert sum(per) == want["additions"] == 60
    # No factor multiplies: all entries are in {0, +1, -1}.
    for f in tf.factors():
        assert set(np.unique(f).tolist()) <= {-1, 0, 1}
    # Every row of every factor has a +1 (no negation-only output).
    for f in tf.factors():
        assert np.all((f == 1).any(axis=1))
    # The transposed factorisation (inverse transform) also costs 60.
    assert sum(tf.additions(f.T) for f in tf.factors()) == 60


def test_table2_reproduces():
    assert pin_table2(tf.T, tf.dct_matrix()) == []


def test_table2_wht_row():
    # Third, independent matrix for the measures: the Walsh-Hadamard
    # transform in natural (Sylvester) order, scaled to be orthonormal.
    from scipy.linalg import hadamard
    h = hadamard(16) / 4.0
    got = metrics.table2_row(tf.dct_matrix(), h)
    for k, txt in _golden("table2.json")["rows"]["WHT"].items():
        dec = len(txt.split(".")[1])
        assert abs(got[k] - float(txt)) <= 0.5 * 10.0 ** (-dec) + 1e-12, k


def test_wht_matrix_and_round_trip():
    # Natural (Sylvester) order equals scipy's Hadamard; H H^T = 16 I, so
    # S = I / 4 and every inverse weight is 3 (A' = 9 H^T Z H / 2304).
    from scipy.linalg import hadamard
    h = tf.wht()
    assert np.array_equal(h, hadamard(16))
    assert np.array_equal(h @ h.T, 16 * np.eye(16, dtype=np.int64))
    assert np.array_equal(tf.inverse_weights(h), np.full(16, 3))
    rng = np.random.default_rng(9)
    a = rng.integers(0, 256, size=(32, 16, 16))
    z = tf.forward_int(a, h)
    assert np.array_equal(tf.inverse_int_numerator(z, h), 2304 * a)   # lossless
    # the natural-order WHT coefficient (u, v) of a block is the sum of the
    # pixels weighted by (-1)^(popcount(u & i) + popcount(v & j))
    for u, v in ((0, 0), (3, 5), (15, 9)):
        sgn = np.array([[(-1) ** (bin(u & i).count("1") + bin(v & j).count("1")) for j in range(16)] for i in range(16)])
        assert np.array_equal(z[:, u, v], np.einsum("bij,ij->b", a, sgn))


def test_dct_matrix_against_library():
    from scipy.fft import dct
    c = tf.dct_matrix()
    lib = dct(np.eye(16), type=2, norm="ortho", axis=0)
    assert np.max(np.abs(c - lib)) < 1e-14
    assert np.max(np.abs(c @ c.T - np.eye(16))) < 1e-14


# ----------------------------------------------------------------------------
# Blockwise transform.

def test_forward_bruteforce():
    assert pin_forward_bruteforce(tf.forward_int) == []


def test_forward_unit_blocks_and_constant():
    # A block with a single 1 at (a, b) gives the outer product T[:, a] T[:, b]^T.
    for a, b in [(0, 0), (3, 11), (15, 7)]:
        e = np.zeros((1, 16, 16), dtype=np.int64)
        e[0, a, b] = 1
        assert np.array_equal(tf.forward_int(e)[0], np.outer(tf.T[:, a], tf.T[:, b]))
    for c in (0, 1, 128, 255):
        z = tf.forward_int(np.full((1, 16, 16), c))[0]
        want = np.zeros((16, 16), dtype=np.int64)
        want[0, 0] = 256 * c
        assert np.array_equal(z, want)


def test_forward_extreme_ranges():
    # uint8 blocks reach DC 65280 and AC +-32640; centred int8 fits int16.
    t = tf.T
    hi = np.where(np.outer(t[1], t[1]) > 0, 255, 0)
    lo = np.where(np.outer(t[1], t[1]) > 0, 0, 255)
    z = tf.forward_int(np.stack([np.full((16, 16), 255), hi, lo]))
    assert z[0, 0, 0] == 65280
    assert z[1, 1, 1] == 32640 and z[2, 1, 1] == -32640
    zc = tf.forward_int(np.stack([hi - 128, lo - 128]))
    assert zc.max() <= 32767 and zc.min() >= -32768
    # Uncentred minus centred is 32768 at DC only.
    d = tf.forward_int(hi[None]) - tf.forward_int((hi - 128)[None])
    want = np.zeros((16, 16), dtype=np.int64)
    want[0, 0] = 32768
    assert np.array_equal(d[0], want)


def test_scaled_coefficients_are_orthonormal():
    rng = np.random.default_rng(5)
    a = rng.integers(0, 256, size=(16, 16, 16))
    b = tf.scale(tf.forward_int(a))
    assert np.max(np.abs(b - tf.forward_real(a))) < 1e-9
    # Parseval: an orthogonal transform keeps the energy of every block.
    assert np.allclose(np.sum(b * b, axis=(1, 2)), np.sum(a.astype(float) ** 2, axis=(1, 2)), rtol=1e-13)


def test_inverse_integer_form_equals_paper_form():
    assert pin_inverse_identity(tf.inverse_int_numerator, tf.forward_int) == []
    rng = np.random.default_rng(7)
    a = rng.integers(0, 256, size=(64, 16, 16))
    z = tf.forward_int(a)
    for keep in (codec.mask_zonal(2), codec.mask_zonal(8), codec.mask_zigzag(16), codec.mask_zigzag(100)):
        zk = np.where(keep[None], z, 0)
        exact = tf.inverse_int_numerator(zk) / 2304.0
        paper = tf.inverse_real(tf.scale(zk))
        assert np.max(np.abs(exact - paper)) < 1e-9


def test_inverse_numerator_range_int32():
    # Worst case over the +-1 sign patterns of T rows for the zonal masks:
    # the exact numerator stays far inside int32.
    w = tf.inverse_weights()
    for r in (1, 2, 4, 6, 8, 16):
        keep = codec.mask_zonal(r)
        # |N_ij| <= sum_uv |T[u,i] w_u w_v T[v,j]| * max|Z_uv| with |Z| <= 65280
        bound = np.abs(tf.T.T) @ (np.outer(w, w) * keep) @ np.abs(tf.T) * 65280
        assert bound.max() < 2**31


def test_rounding_matches_exact_rationals():
    nums = np.arange(-20000, 700000, 97, dtype=np.int64)
    got = codec.int_recon_u8(nums)
    for n, g in zip(nums.tolist(), got.tolist()):
        v = math.floor(Fraction(n, 2304) + Fraction(1, 2))
        assert g == min(255, max(0, v))


# ----------------------------------------------------------------------------
# Retention masks and the zig-zag scan.

def test_zigzag_scan():
    order = codec.zigzag_order()
    assert len(order) == 256 and len(set(order)) == 256
    assert order[:10] == [(0, 0), (0, 1), (1, 0), (2, 0), (1, 1), (0, 2), (0, 3), (1, 2), (2, 1), (3, 0)]
    assert order[-1] == (15, 15)
    for (u0, v0), (u1, v1) in zip(order, order[1:]):
        d0, d1 = u0 + v0, u1 + v1
        assert d1 in (d0, d0 + 1)
        if d1 == d0:  # within a diagonal, one step along it
            assert abs(u1 - u0) == 1 and abs(v1 - v0) == 1
    for r in (1, 16, 50, 256):
        assert codec.mask_zigzag(r).sum() == r
    # The 16th coefficient opens diagonal 5 at (0, 5).
    assert codec.mask_zigzag(16)[0, 5] and not codec.mask_zigzag(16)[5, 0]
    assert codec.mask_zonal(4).sum() == 16 and codec.mask_zonal(16).all()


# ----------------------------------------------------------------------------
# Uniform quantiser.

def test_uniform_multipliers_closed_forms():
    m = codec.uniform_multipliers(1)
    n = tf.row_norms()
    for u in range(16):
        for v in range(16):
            nn = int(n[u] * n[v])
            if nn == 256:
                assert m[u, v] == np.float32(1 / 16)
            elif nn == 64:
                assert m[u, v] == np.float32(1 / 8)
            elif nn == 144:
                assert m[u, v] == np.float32(1 / 12)
    for q, k in ((8, 3), (16, 4), (32, 5)):
        assert np.array_equal(codec.uniform_multipliers(q), m / np.float32(2 ** k))


def test_uniform_levels_against_ideal():
    rng = np.random.default_rng(9)
    a = rng.integers(-255, 256, size=(500, 16, 16))
    z = tf.forward_int(a)
    for q in (1, 8, 16, 32):
        lv = codec.quantise_uniform(z, q)
        ideal = codec.quantise_uniform_ideal(z, q)
        diff = lv != ideal
        # The float32 decision may differ from the float64 ideal only at an
        # exact rounding tie of the real value (Z / (sqrt(n_u n_v) q) with a
        # rational scale), where the two float evaluations break the tie
        # differently.
        y = tf.scale(z) / q
        frac = np.abs(np.abs(y - np.floor(y)) - 0.5)
        assert np.all(frac[diff] < 1e-9)
        # Where s_u s_v is a power of two the decision is an exact division.
        n = tf.row_norms()
        exact = np.isin(np.outer(n, n), (64, 256))
        want = np.rint(z[:, exact] / (np.sqrt(np.outer(n, n))[exact] * q))
        assert np.array_equal(lv[:, exact], want)


# ----------------------------------------------------------------------------
# Quality measures.

def test_deadzone_scales_and_steps():
    # Each quantisation scale times its reconstruction scale is 2^20 to
    # within 0.01 %, so quantising and reconstructing keeps the amplitude;
    # the step doubles every six QP, and QP 4 is the unit step.
    for qs, ds in zip(codec.QUANT_SCALE, codec.DEQUANT_SCALE):
        assert abs(qs * ds / 2.0 ** 20 - 1.0) < 1e-4
    for qp in range(0, 58):
        assert codec.deadzone_step(qp + 6) == 2 * codec.deadzone_step(qp)
    assert codec.deadzone_step(4) == 1.0
    n = tf.row_norms()
    m = codec.deadzone_multipliers(4)
    for u in range(16):
        for v in range(16):
            # M = 1 / sqrt(n_u n_v) at QP 4 (unit step): S folded, nothing else
            assert abs(float(m[u, v]) * math.sqrt(float(n[u] * n[v])) - 1.0) < 2e-7


def test_deadzone_levels_against_exact_rationals():
    # Away from float32 rounding, L = sign(Y) floor(|Y| / step + f) with Y = S Z S.
    rng = np.random.default_rng(7)
    z = rng.integers(-40000, 40000, size=(64, 16, 16))
    for qp, inter in ((4, False), (22, False), (27, True), (37, True)):
        got = codec.quantise_deadzone(z, qp, inter)
        step = codec.deadzone_step(qp)
        y = np.abs(tf.scale(z)) / step + (1.0 / 6.0 if inter else 1.0 / 3.0)
        want = np.sign(z) * np.floor(y)
        near = np.abs(y - np.rint(y)) < 1e-3
        assert np.array_equal(got[~near], want[~near].astype(np.int64))
        # dead zone: |Y| below (1 - f) steps gives level 0
        small = np.abs(tf.scale(z)) < (1.0 - (1.0 / 6.0 if inter else 1.0 / 3.0)) * step * (1 - 1e-6)
        assert np.all(got[small] == 0)


def test_se_code_lengths_against_written_codes():
    # Build each code word: k + 1 in binary, preceded by (bits - 1) zeros.
    for v in range(-300, 301):
        k = 2 * v - 1 if v > 0 else -2 * v
        word = "0" * ((k + 1).bit_length() - 1) + format(k + 1, "b")
        assert codec.se_code_length(v) == len(word)
    assert [codec.se_code_length(v) for v in (0, 1, -1, 2, -2, 3, -3, 4)] == [1, 3, 3, 5, 5, 5, 5, 7]
    assert codec.rate_bits(np.array([[0, 1], [-1, 4]])) == 1 + 3 + 3 + 7


def test_psnr_closed_forms():
    a = np.full((48, 32), 100, dtype=np.uint8)
    assert codec.psnr(a, a) == math.inf
    b = a + 1
    assert abs(codec.psnr(a, b) - 20 * math.log10(255)) < 1e-12
    c = a.astype(np.int16) - 10
    assert abs(codec.psnr(a, c) - (20 * math.log10(255) - 20)) < 1e-12
    assert codec.sse(a, c) == 100 * a.size


def test_ssim_closed_forms():
    rng = np.random.default_rng(1)
    x = rng.integers(0, 256, size=(40, 40)).astype(np.uint8)
    assert abs(codec.ssim(x, x) - 1.0) < 1e-12
    a, b = 100.0, 140.0
    c1 = (0.01 * 255) ** 2
    s = codec.ssim(np.full((20, 20), a), np.full((20, 20), b))
    assert abs(s - (2 * a * b + c1) / (a * a + b * b + c1)) < 1e-12


def test_blocking_round_trip_and_edge_extension():
    rng = np.random.default_rng(2)
    img = rng.integers(0, 256, size=(37, 50)).astype(np.uint8)
    blk = codec.image_to_blocks(img)
    assert blk.shape == (3 * 4, 16, 16)
    assert np.array_equal(codec.blocks_to_image(blk, 37, 50), img)
    # Padding repeats the last row/column.
    full = codec.blocks_to_image(blk, 48, 64)
    assert np.array_equal(full[37:, :50], np.repeat(img[-1:, :], 11, axis=0))
    assert np.array_equal(full[:37, 50:], np.repeat(img[:, -1:], 14, axis=1))


def test_lossless_and_zonal_experiment():
    from synth import ar1_image
    img = ar1_image(0x16060556 + 1, 128, 96)
    rec, s, p = codec.compress_kept(img, codec.mask_zonal(16))
    assert s == 0 and p == math.inf and np.array_equal(rec, img)
    ps = [codec.compress_kept(img, codec.mask_zonal(r))[2] for r in (2, 4, 8)]
    assert ps[0] < ps[1] < ps[2]
    # Energy compaction: keeping more coefficients never hurts on this image,
    # and the exact DCT compacts better than the approximation at r = 4.
    _, pd = codec.compress_dct_kept(img, codec.mask_zonal(4))
    assert pd > ps[1]


# ----------------------------------------------------------------------------
# Pins of the image-level codec functions: SSIM, the dequantised
# reconstructions, the reconstruction rounding and APE.  Each is a function
# of the codec module as it stands, so that a planted mistake in that module
# (test_codec_pins_catch_planted_mistakes) shows up as a failure here.

def _norm_products():
    """n_u n_v from the printed S (Section 2), not from the oracle's T."""
    n = np.array(_golden("s_diag.json")["inv_sqrt_of"], dtype=np.float64)
    return np.outer(n, n)


def _gauss_1d(size, sigma):
    """The 1-D factor of the SSIM window of the Wang et al. reading: samples
    of exp(-t^2 / (2 sigma^2)) at integer t centred on the window, normalised
    to sum 1 (the 2-D window is the outer product)."""
    t = [k - (size - 1) / 2.0 for k in range(size)]
    g = [math.exp(-x * x / (2.0 * sigma * sigma)) for x in t]
    tot = sum(g)
    return [x / tot for x in g]


def _checkerboard(h, w, mu, d):
    i, j = np.indices((h, w))
    return mu + d * np.where((i + j) % 2 == 0, 1.0, -1.0)


def _ssim_of_checkerboards(h, w, mu1, d1, mu2, d2, size=11, sigma=1.5, peak=255.0):
    """Closed form of the mean SSIM of two checkerboards x = mu1 + d1 (-1)^(i+j)
    and y = mu2 + d2 (-1)^(i+j).  With c = sum_k g_k (-1)^k, a window whose
    corner has parity s = (-1)^(p+q) sees mu_x = mu1 + s d1 c^2,
    var_x = d1^2 (1 - c^4), var_y = d2^2 (1 - c^4) and cov_xy = d1 d2 (1 - c^4)
    (population moments under the window weights)."""
    g = _gauss_1d(size, sigma)
    c = sum(gk * (-1) ** k for k, gk in enumerate(g))
    c1, c2 = (0.01 * peak) ** 2, (0.03 * peak) ** 2
    vx, vy, cxy = d1 * d1 * (1 - c ** 4), d2 * d2 * (1 - c ** 4), d1 * d2 * (1 - c ** 4)
    tot, cnt = 0.0, 0
    for p_ in range(h - size + 1):
        for q_ in range(w - size + 1):
            s = 1 if (p_ + q_) % 2 == 0 else -1
            mx, my = mu1 + s * d1 * c * c, mu2 + s * d2 * c * c
            tot += ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
            cnt += 1
    return tot / cnt


def _ssim_bruteforce(x, y, size=11, sigma=1.5, peak=255.0):
    """Mean SSIM with every window's weighted sums written out as loops."""
    g = _gauss_1d(size, sigma)
    c1, c2 = (0.01 * peak) ** 2, (0.03 * peak) ** 2
    h, w = x.shape
    vals = []
    for p_ in range(h - size + 1):
        for q_ in range(w - size + 1):
            sx = sy = sxx = syy = sxy = 0.0
            for k in range(size):
                for l_ in range(size):
                    wt = g[k] * g[l_]
                    a, b = float(x[p_ + k, q_ + l_]), float(y[p_ + k, q_ + l_])
                    sx += wt * a
                    sy += wt * b
                    sxx += wt * a * a
                    syy += wt * b * b
                    sxy += wt * a * b
            vx, vy, cv = sxx - sx * sx, syy - sy * sy, sxy - sx * sy
            vals.append(((2 * sx * sy + c1) * (2 * cv + c2)) / ((sx * sx + sy * sy + c1) * (vx + vy + c2)))
    return sum(vals) / len(vals)


def pin_ssim():
    bad = []
    for (h, w, mu1, d1, mu2, d2) in ((30, 37, 120.0, 50.0, 120.0, 0.0),   # checkerboard against flat
                                     (24, 24, 100.0, 40.0, 130.0, -30.0),  # anti-correlated checkerboards
                                     (13, 12, 60.0, 20.0, 70.0, 45.0)):    # correlated, 3 x 2 windows
        x = _checkerboard(h, w, mu1, d1)
        y = _checkerboard(h, w, mu2, d2)
        got, want = codec.ssim(x, y), _ssim_of_checkerboards(h, w, mu1, d1, mu2, d2)
        if not abs(got - want) < 1e-12:
            bad.append(f"ssim checkerboard {h}x{w}: {got} vs closed form {want}")
    rng = np.random.default_rng(31)
    for (h, w) in ((11, 11), (12, 13)):
        x = rng.integers(0, 256, size=(h, w)).astype(np.float64)
        y = np.clip(x + rng.integers(-40, 41, size=(h, w)), 0, 255)
        got, want = codec.ssim(x, y), _ssim_bruteforce(x, y)
        if not abs(got - want) < 1e-12:
            bad.append(f"ssim brute force {h}x{w}: {got} vs {want}")
    return bad


# Reconstruction steps of the deadzone reading, worked by hand from
# D = {40, 45, 51, 57, 64, 72} and step(QP) = D[QP mod 6] 2^(QP div 6) / 64.
DEADZONE_STEPS = {4: 1.0, 10: 2.0, 22: 8.0, 27: 14.25, 37: 45.0, 0: 0.625}


def pin_dequantised_reconstruction():
    """C_hat is orthogonal (Section 2), so for every block the unrounded
    reconstruction error equals the coefficient error (Parseval):
    ||A' - A||^2 = sum_uv (B_uv - step L_uv)^2 with B = Z / sqrt(n_u n_v),
    whatever the levels L are.  The DC level alone rebuilds a flat block of
    step L / 16 (row 0 of T is all ones and S_00 = 1/4)."""
    bad = []
    rng = np.random.default_rng(41)
    nn = _norm_products()
    for k in range(12):
        a = rng.integers(-255, 256, size=(16, 16)) if k % 2 else rng.integers(0, 256, size=(16, 16))
        z = codec.forward_image(a)[0]
        b = z / np.sqrt(nn)
        lv = rng.integers(-40, 41, size=(1, 16, 16))
        for q in (1, 8, 16, 32):
            rec = codec.reconstruct_uniform(lv, q, 16, 16, np.int16, rounded=False)
            lhs = float(np.sum((rec - a) ** 2))
            rhs = float(np.sum((b - q * lv[0]) ** 2))
            if not abs(lhs - rhs) <= 1e-9 * max(1.0, rhs):
                bad.append(f"uniform Parseval q={q}: {lhs} vs {rhs}")
        for qp, step in DEADZONE_STEPS.items():
            # reconstruct_deadzone rounds; compare the rounding of the
            # Parseval-checked real reconstruction A_r = C_hat^T (step L) C_hat.
            rec = codec.reconstruct_deadzone(lv, qp, 16, 16, np.int16).astype(np.float64)
            real = codec.reconstruct_uniform(lv, 1, 16, 16, np.int16, rounded=False) * step
            if np.max(np.abs(rec - real)) > 0.5 + 1e-9:
                bad.append(f"deadzone QP {qp}: reconstruction off the step {step}")
            lhs = float(np.sum((real - a) ** 2))
            rhs = float(np.sum((b - step * lv[0]) ** 2))
            if not abs(lhs - rhs) <= 1e-9 * max(1.0, rhs):
                bad.append(f"deadzone Parseval QP {qp}: {lhs} vs {rhs}")
    for q in (1, 8, 32):
        dc = np.zeros((1, 16, 16), dtype=np.int64)
        dc[0, 0, 0] = 7
        rec = codec.reconstruct_uniform(dc, q, 16, 16, np.int16, rounded=False)
        if np.max(np.abs(rec - q * 7 / 16.0)) > 1e-12:
            bad.append(f"uniform DC closed form q={q}")
    return bad


def pin_rounding_half_up():
    """floor(x + 1/2) then clamp (u8) or saturate (int16), checked against
    exact rationals on halves, quarters and values just off a half."""
    bad = []
    xs = [Fraction(k, 4) for k in range(-131080, 131081, 3)]
    xs += [Fraction(k, 2) for k in (-65537, -65536, -5, -3, -1, 1, 3, 5, 509, 511, 65533, 65535)]
    eps = Fraction(1, 2 ** 30)
    xs += [Fraction(2 * k + 1, 2) + e for k in (-7, 0, 7, 200) for e in (-eps, eps)]
    arr = np.array([float(x) for x in xs])
    u8, i16 = codec.round_half_up_u8(arr), codec.round_half_up_i16(arr)
    for x, g8, g16 in zip(xs, u8.tolist(), i16.tolist()):
        r = math.floor(x + Fraction(1, 2))
        if g8 != min(255, max(0, r)):
            bad.append(f"u8 rounding of {x}: {g8}")
        if g16 != min(32767, max(-32768, r)):
            bad.append(f"i16 rounding of {x}: {g16}")
    return bad


def pin_ape():
    """Section 4's absolute percentage error of a measure with respect to the
    exact DCT, 100 |x - x_dct| / |x_dct|, on the Lena PSNRs the paper prints
    (27.13 dB proposed, 28.55 dB exact DCT at 16 retained coefficients),
    worked as exact rationals."""
    bad = []
    cases = ((Fraction(2713, 100), Fraction(2855, 100)), (Fraction(2855, 100), Fraction(2713, 100)),
             (Fraction(95, 100), Fraction(97, 100)), (Fraction(-3, 2), Fraction(-2, 1)))
    for x, ref in cases:
        want = 100 * abs(x - ref) / abs(ref)
        got = codec.ape(float(x), float(ref))
        if not abs(got - float(want)) <= 1e-12 * float(want):
            bad.append(f"ape({float(x)}, {float(ref)}) = {got}, want {float(want)}")
    if not abs(codec.ape(27.13, 28.55) - 4.97373029772329) < 1e-9:
        bad.append("ape of the printed Lena PSNRs")
    return bad


def _codec_pins():
    return pin_ssim() + pin_dequantised_reconstruction() + pin_rounding_half_up() + pin_ape()


def test_ssim_checkerboard_and_bruteforce():
    assert pin_ssim() == []


def test_dequantised_reconstruction_parseval():
    assert pin_dequantised_reconstruction() == []


def test_reconstruction_rounding_half_up():
    assert pin_rounding_half_up() == []


def test_ape_worked_values():
    assert pin_ape() == []


# ----------------------------------------------------------------------------
# Planted mistakes: each plausible error in the oracle trips some pin.

def _mutants():
    t_sign = tf.T.copy()
    t_sign[6, 3] *= -1
    t_swap = tf.T.copy()
    t_swap[[4, 5]] = t_swap[[5, 4]]
    yield "sign flip in T", t_sign, tf.forward_int, tf.inverse_int_numerator
    yield "two rows of T swapped", t_swap, tf.forward_int, tf.inverse_int_numerator
    yield "transposed operand in forward", tf.T, (lambda a: tf.T @ np.swapaxes(np.asarray(a, np.int64), 1, 2) @ tf.T.T), tf.inverse_int_numerator
    yield "dropped T^T in forward", tf.T, (lambda a: tf.T @ np.asarray(a, np.int64)), tf.inverse_int_numerator
    w = tf.inverse_weights()
    yield "weights applied once", tf.T, tf.forward_int, (lambda z: tf.T.T @ (w[:, None] * np.asarray(z, np.int64)) @ tf.T * 48)


@pytest.mark.parametrize("name,T,fwd,inv", list(_mutants()), ids=[m[0] for m in _mutants()])
def test_pins_catch_planted_mistakes(name, T, fwd, inv):
    failures = (pin_orthogonality(T) + pin_table2(T, tf.dct_matrix())
                + pin_forward_bruteforce(fwd, nblk=1) + pin_inverse_identity(inv, fwd))
    assert failures, f"planted mistake '{name}' went undetected"


def _codec_mutants():
    n_win = 121.0

    def sample_cov(x, y, g, _orig=codec._local_moments):
        mx, my, sxx, syy, sxy = _orig(x, y, g)
        f = n_win / (n_win - 1.0)
        return mx, my, sxx * f, syy * f, sxy * f

    sv = 1.0 / np.sqrt(_norm_products())
    return [
        ("SSIM window sigma 1.0", "_gauss_window", lambda size=11, sigma=1.5, _o=codec._gauss_window: _o(size, 1.0)),
        ("SSIM window 7x7", "_gauss_window", lambda size=11, sigma=1.5, _o=codec._gauss_window: _o(7, sigma)),
        ("SSIM sample covariance", "_local_moments", sample_cov),
        ("dequantisation without q", "dequantise_uniform", lambda lv, q: np.asarray(lv, dtype=np.float64)),
        ("S applied twice", "dequantise_uniform", lambda lv, q: float(q) * np.asarray(lv, dtype=np.float64) * sv),
        ("deadzone step dropped", "deadzone_step", lambda qp: 1.0),
        ("deadzone step off by one QP", "deadzone_step",
         lambda qp, _o=codec.deadzone_step: _o(qp + 1) if qp + 1 < 64 else _o(qp)),
        ("half-even rounding u8", "round_half_up_u8",
         lambda a: np.clip(np.rint(np.asarray(a, dtype=np.float64)), 0, 255).astype(np.uint8)),
        ("half-away-from-zero rounding i16", "round_half_up_i16",
         lambda a: np.clip(np.sign(a) * np.floor(np.abs(np.asarray(a, dtype=np.float64)) + 0.5),
                           -32768, 32767).astype(np.int16)),
        ("truncating rounding i16", "round_half_up_i16",
         lambda a: np.clip(np.trunc(np.asarray(a, dtype=np.float64) + 0.5), -32768, 32767).astype(np.int16)),
        ("APE divided by x", "ape", lambda x, ref: 100.0 * abs(x - ref) / abs(x)),
        ("APE without the factor 100", "ape", lambda x, ref: abs(x - ref) / abs(ref)),
    ]


@pytest.mark.parametrize("name,attr,fn", _codec_mutants(), ids=[m[0] for m in _codec_mutants()])
def test_codec_pins_catch_planted_mistakes(name, attr, fn, monkeypatch):
    monkeypatch.setattr(codec, attr, fn)
    assert _codec_pins(), f"planted mistake '{name}' went undetected"


def test_oracle_header_declares_test_infrastructure():
    assert "TEST INFRASTRUCTURE ONLY" in oracle.__doc__
