"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: integer coefficients, retained coefficients, levels and zonal
reconstructions bit-exact; float outputs within 1e-6 relative of the float64
oracle; PSNR within 1e-3 dB (+inf equals +inf).  Rounded reconstructions of
the uniform quantiser come from a float64 inverse on both sides (different
summation order), so a pixel may differ by one only where the oracle's
value lies within 1e-9 of a rounding tie; every other pixel must match.
"""
import math
import warnings

import numpy as np
import pytest

from oracle import codec
from oracle import transform as tf
from synth import BASE_SEED, ar1_image, luma_frame, mixed_image, random_blocks_u8, residual_plane

from batch_util import Batch

pytestmark = pytest.mark.gpu

PSNR_TOL_DB = 1e-3
FLOAT_RTOL = 1e-6


def A():
    import paper_1606_05562_amd as mod
    return mod


def torch():
    import torch as t
    return t


def _images_u8():
    rng = np.random.default_rng(5)
    ims = [ar1_image(BASE_SEED + 1, 512, 512),            # the paper's 512x512 shape
           luma_frame(BASE_SEED + 2, 0, 64, 1040),        # several strips, ragged strip tail
           rng.integers(0, 256, (37, 50)).astype(np.uint8),  # ragged in both directions
           rng.integers(0, 256, (16, 16)).astype(np.uint8),
           rng.integers(0, 256, (1, 1)).astype(np.uint8),
           rng.integers(0, 256, (17, 130)).astype(np.uint8),
           rng.integers(0, 256, (200, 7)).astype(np.uint8)]
    # extremes of the forward ranges: flat 255 (DC 65280), sign patterns of
    # rows of T (AC +-32640)
    t = tf.T
    ext = np.zeros((32, 48), dtype=np.uint8)
    ext[:16, :16] = 255
    ext[:16, 16:32] = np.where(np.outer(t[1], t[1]) > 0, 255, 0)
    ext[:16, 32:48] = np.where(np.outer(t[1], t[1]) > 0, 0, 255)
    ext[16:, :16] = np.where(np.outer(t[7], t[13]) > 0, 255, 0)
    ext[16:, 16:32] = 0
    ext[16:, 32:48] = np.where(np.outer(t[15], t[2]) < 0, 255, 0)
    ims.append(ext)
    return ims


def _images_i16():
    rng = np.random.default_rng(6)
    return [residual_plane(BASE_SEED + 5, 0, 0, 96, 160),
            residual_plane(BASE_SEED + 5, 0, 1, 48, 80),
            rng.integers(-255, 256, (33, 47)).astype(np.int16),
            np.full((16, 32), 255, dtype=np.int16),
            np.full((16, 32), -255, dtype=np.int16)]


@pytest.fixture(scope="module")
def batch_u8():
    return Batch(_images_u8())


@pytest.fixture(scope="module")
def batch_i16():
    return Batch(_images_i16())


def _oracle_z(images):
    return [codec.forward_image(im) for im in images]


# ----------------------------------------------------------------------------
# Forward

@pytest.mark.parametrize("backend", [1])
def test_forward_i32_u8(batch_u8, backend):
    T = torch()
    plan = batch_u8.plan(coef_dtype=A().I32, backend=backend)
    coef = batch_u8.coef_tensor(T.int32)
    plan.forward(batch_u8.dev, coef)
    T.cuda.synchronize()
    for got, want in zip(batch_u8.split_coef(coef), _oracle_z(batch_u8.images)):
        assert np.array_equal(got.astype(np.int64), want)


def test_forward_i16_centred(batch_u8):
    T = torch()
    plan = batch_u8.plan(coef_dtype=A().I16)
    coef = batch_u8.coef_tensor(T.int16)
    plan.forward(batch_u8.dev, coef)
    T.cuda.synchronize()
    for got, want in zip(batch_u8.split_coef(coef), _oracle_z(batch_u8.images)):
        want = want.copy()
        want[:, 0, 0] -= 32768
        assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("which", ["u8", "i16"])
def test_forward_f32_scaled(batch_u8, batch_i16, which):
    T = torch()
    b = batch_u8 if which == "u8" else batch_i16
    plan = b.plan(coef_dtype=A().F32)
    coef = b.coef_tensor(T.float32)
    plan.forward(b.dev, coef)
    T.cuda.synchronize()
    for got, z in zip(b.split_coef(coef), _oracle_z(b.images)):
        want = tf.scale(z)
        assert np.all(np.abs(got - want) <= FLOAT_RTOL * np.abs(want))


def test_forward_i32_i16(batch_i16):
    T = torch()
    plan = batch_i16.plan(coef_dtype=A().I32)
    coef = batch_i16.coef_tensor(T.int32)
    plan.forward(batch_i16.dev, coef)
    T.cuda.synchronize()
    for got, want in zip(batch_i16.split_coef(coef), _oracle_z(batch_i16.images)):
        assert np.array_equal(got.astype(np.int64), want)


# ----------------------------------------------------------------------------
# Retention and quantiser

@pytest.mark.parametrize("qmode,r", [(2, 1), (2, 16), (2, 50), (2, 256), (1, 2), (1, 8), (1, 16), (0, 16)])
def test_quantise_masks(batch_u8, qmode, r):
    T = torch()
    plan = batch_u8.plan(coef_dtype=A().I32, qmode=qmode, r=r)
    coef = batch_u8.coef_tensor(T.int32)
    qc = batch_u8.coef_tensor(T.int32)
    plan.forward(batch_u8.dev, coef)
    plan.quantise(coef, qc)
    T.cuda.synchronize()
    keep = {0: codec.mask_none(), 1: codec.mask_zonal(r), 2: codec.mask_zigzag(r)}[qmode]
    for got, z in zip(batch_u8.split_coef(qc), _oracle_z(batch_u8.images)):
        assert np.array_equal(got.astype(np.int64), np.where(keep[None], z, 0))


@pytest.mark.parametrize("q", [1, 8, 16, 32])
@pytest.mark.parametrize("coef", ["i32", "i16"])
def test_quantise_uniform_levels(batch_u8, q, coef):
    T = torch()
    cd = A().I32 if coef == "i32" else A().I16
    plan = batch_u8.plan(coef_dtype=cd, qmode=A().Q_UNIFORM, q=q, qcoef_dtype=A().I32)
    c = batch_u8.coef_tensor(T.int32 if coef == "i32" else T.int16)
    lv = batch_u8.coef_tensor(T.int32)
    plan.forward(batch_u8.dev, c)
    plan.quantise(c, lv)
    T.cuda.synchronize()
    for got, z in zip(batch_u8.split_coef(lv), _oracle_z(batch_u8.images)):
        assert np.array_equal(got.astype(np.int64), codec.quantise_uniform(z, q))


# ----------------------------------------------------------------------------
# Inverse

@pytest.mark.parametrize("qmode,r", [(0, 16), (1, 2), (1, 6), (2, 16), (2, 100)])
def test_inverse_mask_u8(batch_u8, qmode, r):
    T = torch()
    plan = batch_u8.plan(coef_dtype=A().I32, qmode=qmode, r=r)
    coef = batch_u8.coef_tensor(T.int32)
    out = batch_u8.empty_like_images(np.uint8, 77)
    plan.forward(batch_u8.dev, coef)
    plan.quantise(coef, coef)
    plan.inverse(coef, out)
    T.cuda.synchronize()
    keep = {0: codec.mask_none(), 1: codec.mask_zonal(r), 2: codec.mask_zigzag(r)}[qmode]
    for got, im in zip(batch_u8.unpack(out), batch_u8.images):
        want, _, _ = codec.compress_kept(im, keep)
        assert np.array_equal(got, want)
        if qmode == 0:
            assert np.array_equal(got, im)  # lossless round trip


def test_inverse_mask_centred_i16_and_f32(batch_u8):
    T = torch()
    plan = batch_u8.plan(coef_dtype=A().I16, qmode=A().Q_ZONAL, r=4, out_dtype=A().F32)
    coef = batch_u8.coef_tensor(T.int16)
    out = batch_u8.empty_like_images(np.float32)
    plan.forward(batch_u8.dev, coef)
    plan.quantise(coef, coef)
    plan.inverse(coef, out)
    T.cuda.synchronize()
    keep = codec.mask_zonal(4)
    for got, im in zip(batch_u8.unpack(out), batch_u8.images):
        h, w = im.shape
        z = codec.forward_image(im)
        want = codec.blocks_to_image(tf.inverse_real(tf.scale(np.where(keep[None], z, 0))), h, w)
        assert np.all(np.abs(got - want) <= FLOAT_RTOL * np.abs(want) + 1e-9)


def _check_near_tie_rounding(got, real, lo=-32768, hi=32767):
    """Rounded float64 reconstructions: equal except where the oracle's
    real value is within 1e-9 of a tie, and then off by at most one."""
    want = np.clip(np.floor(real + 0.5), lo, hi)
    diff = got.astype(np.int64) - want.astype(np.int64)
    bad = diff != 0
    tie = np.abs(real - np.floor(real) - 0.5) < 1e-9
    assert np.all(np.abs(diff) <= 1)
    assert np.all(tie[bad]), f"{bad.sum()} mismatches away from ties"


@pytest.mark.parametrize("q", [8, 32])
def test_inverse_uniform(batch_i16, q):
    T = torch()
    plan = batch_i16.plan(coef_dtype=A().I32, qmode=A().Q_UNIFORM, q=q, qcoef_dtype=A().I16, out_dtype=A().I16)
    coef = batch_i16.coef_tensor(T.int32)
    lv = batch_i16.coef_tensor(T.int16)
    out = batch_i16.empty_like_images(np.int16)
    plan.forward(batch_i16.dev, coef)
    plan.quantise(coef, lv)
    plan.inverse(lv, out)
    T.cuda.synchronize()
    levels = batch_i16.split_coef(lv)
    for got, lvl, im in zip(batch_i16.unpack(out), levels, batch_i16.images):
        h, w = im.shape
        assert np.array_equal(lvl.astype(np.int64), codec.quantise_uniform(codec.forward_image(im), q))
        real = codec.reconstruct_uniform(lvl.astype(np.int64), q, h, w, rounded=False)
        _check_near_tie_rounding(got, real)


# ----------------------------------------------------------------------------
# Fused forward -> retention/quantiser -> inverse -> PSNR

def _psnr_close(a, b):
    if math.isinf(b):
        return math.isinf(a) and a > 0
    return abs(a - b) <= PSNR_TOL_DB


@pytest.mark.parametrize("r", [2, 4, 6, 8, 16])
def test_fused_zonal_u8(batch_u8, r):
    T = torch()
    plan = batch_u8.plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=r, qcoef_dtype=A().I16)
    out = batch_u8.empty_like_images(np.uint8, 3)
    qc = batch_u8.coef_tensor(T.int16)
    sse = T.zeros(len(batch_u8.images), dtype=T.int64, device="cuda")
    psnr = T.zeros(len(batch_u8.images), dtype=T.float64, device="cuda")
    plan.compress_and_measure(batch_u8.dev, out, qc, sse, psnr)
    T.cuda.synchronize()
    keep = codec.mask_zonal(r)
    qcs = batch_u8.split_coef(qc)
    for i, (got, im) in enumerate(zip(batch_u8.unpack(out), batch_u8.images)):
        want, s, p = codec.compress_kept(im, keep)
        assert np.array_equal(got, want)
        assert int(sse[i]) == s
        assert _psnr_close(float(psnr[i]), p)
        zc = np.where(keep[None], codec.forward_image(im), 0)
        zc[:, 0, 0] -= 32768
        assert np.array_equal(qcs[i].astype(np.int64), zc)


def test_fused_zigzag_and_none(batch_u8):
    T = torch()
    for qmode, r, keep in ((A().Q_ZIGZAG, 16, codec.mask_zigzag(16)), (A().Q_NONE, 16, codec.mask_none())):
        plan = batch_u8.plan(coef_dtype=A().I32, qmode=qmode, r=r)
        out = batch_u8.empty_like_images(np.uint8)
        psnr = T.zeros(len(batch_u8.images), dtype=T.float64, device="cuda")
        plan.compress_and_measure(batch_u8.dev, out, None, None, psnr)
        T.cuda.synchronize()
        for i, (got, im) in enumerate(zip(batch_u8.unpack(out), batch_u8.images)):
            want, s, p = codec.compress_kept(im, keep)
            assert np.array_equal(got, want)
            assert _psnr_close(float(psnr[i]), p)


@pytest.mark.parametrize("q", [8, 16, 32])
def test_fused_uniform_residual(batch_i16, q):
    T = torch()
    plan = batch_i16.plan(coef_dtype=A().I32, qmode=A().Q_UNIFORM, q=q, qcoef_dtype=A().I16, out_dtype=A().I16)
    out = batch_i16.empty_like_images(np.int16)
    lv = batch_i16.coef_tensor(T.int16)
    sse = T.zeros(len(batch_i16.images), dtype=T.int64, device="cuda")
    psnr = T.zeros(len(batch_i16.images), dtype=T.float64, device="cuda")
    plan.compress_and_measure(batch_i16.dev, out, lv, sse, psnr)
    T.cuda.synchronize()
    for i, (got, lvl, im) in enumerate(zip(batch_i16.unpack(out), batch_i16.split_coef(lv), batch_i16.images)):
        h, w = im.shape
        want_lv = codec.quantise_uniform(codec.forward_image(im), q)
        assert np.array_equal(lvl.astype(np.int64), want_lv)
        real = codec.reconstruct_uniform(want_lv, q, h, w, rounded=False)
        _check_near_tie_rounding(got, real)
        assert int(sse[i]) == codec.sse(im, got)
        want_rec = codec.reconstruct_uniform(want_lv, q, h, w, out_dtype=np.int16)
        assert _psnr_close(float(psnr[i]), codec.psnr_from_sse(codec.sse(im, want_rec), h * w))


def test_fused_uniform_u8(batch_u8):
    T = torch()
    q = 16
    plan = batch_u8.plan(coef_dtype=A().I32, qmode=A().Q_UNIFORM, q=q, qcoef_dtype=A().I32)
    out = batch_u8.empty_like_images(np.uint8)
    lv = batch_u8.coef_tensor(T.int32)
    plan.compress_and_measure(batch_u8.dev, out, lv, None, None)
    T.cuda.synchronize()
    for got, lvl, im in zip(batch_u8.unpack(out), batch_u8.split_coef(lv), batch_u8.images):
        h, w = im.shape
        want_lv = codec.quantise_uniform(codec.forward_image(im), q)
        assert np.array_equal(lvl.astype(np.int64), want_lv)
        real = codec.reconstruct_uniform(want_lv, q, h, w, rounded=False)
        _check_near_tie_rounding(got, real, lo=0, hi=255)


def test_fused_zonal_i16(batch_i16):
    T = torch()
    plan = batch_i16.plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=6, out_dtype=A().I16)
    out = batch_i16.empty_like_images(np.int16)
    sse = T.zeros(len(batch_i16.images), dtype=T.int64, device="cuda")
    plan.compress_and_measure(batch_i16.dev, out, None, sse, None)
    T.cuda.synchronize()
    for i, (got, im) in enumerate(zip(batch_i16.unpack(out), batch_i16.images)):
        want, s, _ = codec.compress_kept(im, codec.mask_zonal(6))
        assert np.array_equal(got, want)
        assert int(sse[i]) == s


def test_measure(batch_u8):
    T = torch()
    plan = batch_u8.plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=4)
    coef = batch_u8.coef_tensor(T.int32)
    out = batch_u8.empty_like_images(np.uint8)
    plan.forward(batch_u8.dev, coef)
    plan.quantise(coef, coef)
    plan.inverse(coef, out)
    sse = T.zeros(len(batch_u8.images), dtype=T.int64, device="cuda")
    psnr = T.zeros(len(batch_u8.images), dtype=T.float64, device="cuda")
    plan.measure(batch_u8.dev, out, sse, psnr)
    T.cuda.synchronize()
    for i, (got, im) in enumerate(zip(batch_u8.unpack(out), batch_u8.images)):
        assert int(sse[i]) == codec.sse(im, got)
        assert _psnr_close(float(psnr[i]), codec.psnr(im, got))


# ----------------------------------------------------------------------------
# Ragged batch (mixed content, sizes not multiples of 16), determinism, graphs

def test_ragged_fused_r8_deterministic():
    T = torch()
    rng = np.random.default_rng(12)
    sizes = [(int(a), int(b)) for a, b in rng.integers(16, 420, size=(9, 2))]
    ims = [mixed_image(BASE_SEED + 4, k, h, w) for k, (h, w) in enumerate(sizes)]
    b = Batch(ims)
    plan = b.plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=8)
    outs, sses = [], []
    for _ in range(2):
        out = b.empty_like_images(np.uint8)
        sse = T.zeros(len(ims), dtype=T.int64, device="cuda")
        psnr = T.zeros(len(ims), dtype=T.float64, device="cuda")
        plan.compress_and_measure(b.dev, out, None, sse, psnr)
        T.cuda.synchronize()
        outs.append(out.cpu().numpy())
        sses.append(sse.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(sses[0], sses[1])
    for i, (got, im) in enumerate(zip(b.unpack(T.from_numpy(outs[0]).cuda()), ims)):
        want, s, p = codec.compress_kept(im, codec.mask_zonal(8))
        assert np.array_equal(got, want)
        assert sses[0][i] == s
        assert _psnr_close(float(psnr[i]), p)


def test_graph_replays_match_eager(batch_u8):
    T = torch()
    plan = batch_u8.plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=4)
    out_e = batch_u8.empty_like_images(np.uint8)
    sse_e = T.zeros(len(batch_u8.images), dtype=T.int64, device="cuda")
    plan.compress_and_measure(batch_u8.dev, out_e, None, sse_e, None)
    out_g = batch_u8.empty_like_images(np.uint8)
    sse_g = T.full((len(batch_u8.images),), 99, dtype=T.int64, device="cuda")
    psnr_g = T.zeros(len(batch_u8.images), dtype=T.float64, device="cuda")
    g = plan.graph(batch_u8.dev, out_g, None, sse_g, psnr_g)
    want = batch_u8.unpack(out_e)
    for rep in range(4):
        out_g.fill_(rep)
        g.launch()
        T.cuda.synchronize()
        assert all(np.array_equal(a, b) for a, b in zip(batch_u8.unpack(out_g), want)), f"replay {rep}"
        assert T.equal(sse_g, sse_e), f"replay {rep}"
        _ = (out_g.float().sum() + 1).item()  # eager work between replays
    g.close()


@pytest.mark.parametrize("n_images", [1, 3, 16, 17])
def test_valu_repeated_calls_and_replays(n_images):
    """The vector fused kernel accumulates SSE in per-image slots that the
    finishing kernel sums and clears: repeated calls and graph replays give
    the oracle's reconstruction, SSE and PSNR every time."""
    T = torch()
    ims = [mixed_image(BASE_SEED + 11, k, 40 + 8 * (k % 3), 72 + 16 * (k % 4)) for k in range(n_images)]
    b = Batch(ims, 16)
    plan = b.plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=5, backend=A().BACKEND_VALU)
    want = [codec.compress_kept(im, codec.mask_zonal(5)) for im in ims]
    out = b.empty_like_images(np.uint8)
    sse = T.zeros(n_images, dtype=T.int64, device="cuda")
    psnr = T.zeros(n_images, dtype=T.float64, device="cuda")

    def check(tag):
        T.cuda.synchronize()
        recs, s, p = b.unpack(out), sse.cpu().numpy(), psnr.cpu().numpy()
        for i, (got, (wr, ws, wp)) in enumerate(zip(recs, want)):
            assert np.array_equal(got, wr) and s[i] == ws, f"{tag}, image {i}"
            assert (math.isinf(wp) and math.isinf(p[i])) or abs(p[i] - wp) <= 1e-3, f"{tag}, image {i}"

    for rep in range(3):
        sse.fill_(7)
        psnr.fill_(0)
        plan.compress_and_measure(b.dev, out, None, sse, psnr)
        check(f"call {rep}")
    g = plan.graph(b.dev, out, None, sse, psnr)
    for rep in range(3):
        sse.fill_(7)
        psnr.fill_(0)
        g.launch()
        check(f"replay {rep}")
        _ = (out.float().sum() + 1).item()  # eager work between replays
    g.close()


@pytest.mark.parametrize("n", [1, 63, 64, 65, 10000])
def test_one_d_api(n):
    """Whole 64-vector groups go through the LDS-regrouped path, the rest
    one per lane; both directions against the oracle's T."""
    T = torch()
    rng = np.random.default_rng(3 + n)
    x = rng.integers(-100000, 100000, size=(n, 16)).astype(np.int32)
    xd = T.from_numpy(x).cuda()
    y = T.empty_like(xd)
    A().forward_1d(xd, y)
    yi = T.empty_like(xd)
    A().inverse_1d(xd, yi)
    T.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy().astype(np.int64), x.astype(np.int64) @ tf.T.T)
    assert np.array_equal(yi.cpu().numpy().astype(np.int64), x.astype(np.int64) @ tf.T)
    A().forward_1d(xd[:0], y[:0])  # empty input is a no-op


def test_one_d_api_large():
    """More groups than the launch has wavefronts (each wavefront loops),
    plus a ragged tail; sampled rows against the oracle's T."""
    T = torch()
    n = 64 * (4 << 16) + 64 * 3 + 5
    g = T.Generator(device="cpu").manual_seed(77)
    xd = T.randint(-(1 << 20), 1 << 20, (n, 16), dtype=T.int32, generator=g).cuda()
    y = T.empty_like(xd)
    A().forward_1d(xd, y)
    T.cuda.synchronize()
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([np.arange(64), np.arange(n - 200, n), rng.integers(0, n, 20000)]))
    idx = T.from_numpy(rows).cuda()
    xs = xd[idx].cpu().numpy().astype(np.int64)
    ys = y[idx].cpu().numpy().astype(np.int64)
    assert np.array_equal(ys, xs @ tf.T.T)


def test_random_blocks_worst_case():
    T = torch()
    blocks = random_blocks_u8(BASE_SEED + 9, 4096)
    img = blocks.reshape(64, 64, 16, 16).transpose(0, 2, 1, 3).reshape(1024, 1024)
    b = Batch([img])
    plan = b.plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=3)
    out = b.empty_like_images(np.uint8)
    coef = b.coef_tensor(T.int32)
    plan.forward(b.dev, coef)
    plan.compress_and_measure(b.dev, out)
    T.cuda.synchronize()
    assert np.array_equal(b.split_coef(coef)[0].astype(np.int64), tf.forward_int(blocks))
    want, _, _ = codec.compress_kept(img, codec.mask_zonal(3))
    assert np.array_equal(b.unpack(out)[0], want)


# ----------------------------------------------------------------------------
# Full size: 256 luma frames 1920x1088 in the benchmark's launch
# configuration; sampled frames are checked completely against the oracle.

def test_full_size_luma_batch_sampled():
    from synth import luma_batch
    T = torch()
    import paper_1606_05562_amd as mod
    n, h, w = 256, 1088, 1920
    frames = luma_batch(BASE_SEED + 2, n, h, w)
    dev = T.from_numpy(frames.reshape(-1)).cuda()
    plan = mod.Plan([h] * n, [w] * n, [w] * n, [i * h * w for i in range(n)], in_dtype=mod.U8,
                    coef_dtype=mod.I32, qmode=mod.Q_ZONAL, r=8, backend=mod.BACKEND_VALU)
    out = T.empty_like(dev)
    sse = T.zeros(n, dtype=T.int64, device="cuda")
    psnr = T.zeros(n, dtype=T.float64, device="cuda")
    plan.compress_and_measure(dev, out, None, sse, psnr)
    T.cuda.synchronize()
    keep = codec.mask_zonal(8)
    for t in (0, 137, 255):
        got = out[t * h * w:(t + 1) * h * w].cpu().numpy().reshape(h, w)
        want, s, p = codec.compress_kept(frames[t], keep)
        assert np.array_equal(got, want), f"frame {t}"
        assert int(sse[t]) == s and _psnr_close(float(psnr[t]), p)
    # every frame: SSE consistent with the reconstruction actually written
    m = T.zeros(n, dtype=T.int64, device="cuda")
    plan.measure(dev, out, m)
    T.cuda.synchronize()
    assert T.equal(m, sse)


# ----------------------------------------------------------------------------
# Deadzone quantiser (QP-scaled step) and the rate proxy

@pytest.mark.parametrize("qp,inter", [(4, False), (22, False), (27, True), (37, False), (51, True)])
def test_fused_deadzone_residual(batch_i16, qp, inter):
    T = torch()
    plan = batch_i16.plan(coef_dtype=A().I32, qmode=A().Q_DEADZONE, q=qp, qcoef_dtype=A().I16, out_dtype=A().I16,
                          flags=A().FLAG_DEADZONE_INTER if inter else 0)
    out = batch_i16.empty_like_images(np.int16)
    lv = batch_i16.coef_tensor(T.int16)
    sse = T.zeros(len(batch_i16.images), dtype=T.int64, device="cuda")
    psnr = T.zeros(len(batch_i16.images), dtype=T.float64, device="cuda")
    bits = T.zeros(len(batch_i16.images), dtype=T.int64, device="cuda")
    plan.compress_and_measure(batch_i16.dev, out, lv, sse, psnr)
    plan.rate(lv, bits)
    T.cuda.synchronize()
    for i, (got, lvl, im) in enumerate(zip(batch_i16.unpack(out), batch_i16.split_coef(lv), batch_i16.images)):
        h, w = im.shape
        want_lv = codec.quantise_deadzone(codec.forward_image(im), qp, inter)
        assert np.array_equal(lvl.astype(np.int64), want_lv)
        assert int(bits[i]) == codec.rate_bits(want_lv)
        real = tf.inverse_real(codec.deadzone_step(qp) * want_lv.astype(np.float64))
        _check_near_tie_rounding(got, codec.blocks_to_image(real, h, w))
        assert int(sse[i]) == codec.sse(im, got)
        want_rec = codec.reconstruct_deadzone(want_lv, qp, h, w, out_dtype=np.int16)
        assert _psnr_close(float(psnr[i]), codec.psnr_from_sse(codec.sse(im, want_rec), h * w))


@pytest.mark.parametrize("lv_dtype", ["i16", "i32"])
def test_deadzone_unfused_u8(batch_u8, lv_dtype):
    # forward -> quantise -> inverse through HBM, levels in either dtype
    T = torch()
    qp = 30
    plan = batch_u8.plan(coef_dtype=A().I32, qmode=A().Q_DEADZONE, q=qp,
                         qcoef_dtype=A().I16 if lv_dtype == "i16" else A().I32)
    coef = batch_u8.coef_tensor(T.int32)
    lv = batch_u8.coef_tensor(T.int16 if lv_dtype == "i16" else T.int32)
    out = batch_u8.empty_like_images(np.uint8)
    bits = T.zeros(len(batch_u8.images), dtype=T.int64, device="cuda")
    plan.forward(batch_u8.dev, coef)
    plan.quantise(coef, lv)
    plan.inverse(lv, out)
    plan.rate(lv, bits)
    T.cuda.synchronize()
    for i, (got, lvl, im) in enumerate(zip(batch_u8.unpack(out), batch_u8.split_coef(lv), batch_u8.images)):
        h, w = im.shape
        want_lv = codec.quantise_deadzone(codec.forward_image(im), qp)
        assert np.array_equal(lvl.astype(np.int64), want_lv)
        assert int(bits[i]) == codec.rate_bits(want_lv)
        real = tf.inverse_real(codec.deadzone_step(qp) * want_lv.astype(np.float64))
        _check_near_tie_rounding(got, codec.blocks_to_image(real, h, w), 0, 255)


def test_rate_rejects_mask_plans(batch_u8):
    plan = batch_u8.plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=4)
    T = torch()
    with pytest.raises(A().Adct16Error) as e:
        plan.rate(batch_u8.coef_tensor(T.int32), T.zeros(len(batch_u8.images), dtype=T.int64, device="cuda"))
    assert e.value.status == A().E_STATE


# ----------------------------------------------------------------------------
# Section 4's comparison: exact DCT-II round trip, SSIM and APE

@pytest.mark.parametrize("qmode,r", [(1, 4), (2, 16), (2, 100), (0, 16)])
def test_dct_roundtrip_and_ape(batch_u8, qmode, r):
    T = torch()
    keep = {0: codec.mask_none(), 1: codec.mask_zonal(r), 2: codec.mask_zigzag(r)}[qmode]
    plan = batch_u8.plan(coef_dtype=A().I32, qmode=qmode, r=r)
    out = batch_u8.empty_like_images(np.uint8, 9)
    sse = T.zeros(len(batch_u8.images), dtype=T.int64, device="cuda")
    psnr = T.zeros(len(batch_u8.images), dtype=T.float64, device="cuda")
    plan.dct_compress_and_measure(batch_u8.dev, out, sse, psnr)
    out_a = batch_u8.empty_like_images(np.uint8, 9)
    psnr_a = T.zeros(len(batch_u8.images), dtype=T.float64, device="cuda")
    plan.compress_and_measure(batch_u8.dev, out_a, None, None, psnr_a)
    T.cuda.synchronize()
    for i, (got, im) in enumerate(zip(batch_u8.unpack(out), batch_u8.images)):
        h, w = im.shape
        real = codec.blocks_to_image(tf.dct_inverse(np.where(keep[None], tf.dct_forward(codec.image_to_blocks(im)), 0.0)),
                                     h, w)
        _check_near_tie_rounding(got, real, 0, 255)
        assert int(sse[i]) == codec.sse(im, got)
        want_rec, want_psnr = codec.compress_dct_kept(im, keep)
        assert _psnr_close(float(psnr[i]), codec.psnr(im, got))
        if not math.isinf(want_psnr):
            ape_gpu = codec.ape(float(psnr_a[i]), float(psnr[i]))
            _, _, p_approx = codec.compress_kept(im, keep)
            assert abs(ape_gpu - codec.ape(p_approx, want_psnr)) < 1e-3


def test_ssim_against_oracle(batch_u8):
    T = torch()
    plan = batch_u8.plan(coef_dtype=A().I32, qmode=A().Q_ZIGZAG, r=20)
    out = batch_u8.empty_like_images(np.uint8, 5)
    plan.compress_and_measure(batch_u8.dev, out)
    s = T.zeros(len(batch_u8.images), dtype=T.float64, device="cuda")
    s_same = T.zeros(len(batch_u8.images), dtype=T.float64, device="cuda")
    plan.ssim(batch_u8.dev, out, s)
    plan.ssim(batch_u8.dev, batch_u8.dev, s_same)
    T.cuda.synchronize()
    for i, (got, im) in enumerate(zip(batch_u8.unpack(out), batch_u8.images)):
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            want = codec.ssim(im, got) if min(im.shape) >= 11 else float("nan")
        if math.isnan(want):
            assert math.isnan(float(s[i])) and math.isnan(float(s_same[i]))
        else:
            assert abs(float(s[i]) - want) < 1e-10, (i, float(s[i]), want)
            assert abs(float(s_same[i]) - 1.0) < 1e-12


# ----------------------------------------------------------------------------
# The same kernels with the Walsh-Hadamard matrix (a comparison transform of
# Table 2) in place of T

@pytest.mark.parametrize("backend", ["valu", "mfma"])
@pytest.mark.parametrize("qmode,r", [(0, 16), (1, 4), (2, 50)])
def test_wht_fused_u8(batch_u8, backend, qmode, r):
    T = torch()
    be = A().BACKEND_VALU if backend == "valu" else A().BACKEND_MFMA
    plan = batch_u8.plan(coef_dtype=A().I32, qmode=qmode, r=r, backend=be, matrix=A().MATRIX_WHT)
    out = batch_u8.empty_like_images(np.uint8, 7)
    sse = T.zeros(len(batch_u8.images), dtype=T.int64, device="cuda")
    plan.compress_and_measure(batch_u8.dev, out, None, sse)
    T.cuda.synchronize()
    keep = {0: codec.mask_none(), 1: codec.mask_zonal(r), 2: codec.mask_zigzag(r)}[qmode]
    for i, (got, im) in enumerate(zip(batch_u8.unpack(out), batch_u8.images)):
        want, s, _ = codec.compress_kept(im, keep, tf.wht())
        assert np.array_equal(got, want), f"image {i}"
        assert int(sse[i]) == s
        if qmode == 0:
            assert np.array_equal(got, im)


@pytest.mark.parametrize("backend,int8", [("valu", False), ("mfma", False), ("mfma", True)])
def test_wht_forward(batch_u8, backend, int8):
    T = torch()
    be = A().BACKEND_VALU if backend == "valu" else A().BACKEND_MFMA
    plan = batch_u8.plan(coef_dtype=A().I32, backend=be, matrix=A().MATRIX_WHT,
                         flags=A().FLAG_MFMA_INT8 if int8 else 0)
    coef = batch_u8.coef_tensor(T.int32)
    plan.forward(batch_u8.dev, coef)
    T.cuda.synchronize()
    for got, im in zip(batch_u8.split_coef(coef), batch_u8.images):
        assert np.array_equal(got.astype(np.int64), codec.forward_image(im, tf.wht()))


def test_wht_uniform_residual(batch_i16):
    T = torch()
    q = 16
    plan = batch_i16.plan(coef_dtype=A().I32, qmode=A().Q_UNIFORM, q=q, qcoef_dtype=A().I16, out_dtype=A().I16,
                          matrix=A().MATRIX_WHT)
    out = batch_i16.empty_like_images(np.int16)
    lv = batch_i16.coef_tensor(T.int16)
    plan.compress_and_measure(batch_i16.dev, out, lv)
    T.cuda.synchronize()
    h16 = tf.wht()
    for got, lvl, im in zip(batch_i16.unpack(out), batch_i16.split_coef(lv), batch_i16.images):
        h, w = im.shape
        want_lv = codec.quantise_uniform(codec.forward_image(im, h16), q, h16)
        assert np.array_equal(lvl.astype(np.int64), want_lv)
        real = codec.reconstruct_uniform(want_lv, q, h, w, rounded=False, t=h16)
        _check_near_tie_rounding(got, real)
