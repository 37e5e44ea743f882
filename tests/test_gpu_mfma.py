"""Matrix-core forms: the int-exact FP16 contractions must be bit-exact with
the oracle (and therefore with the adder kernel); the exact DCT-II on BF16 /
F16 operands is compared with the float64 DCT within an error bound derived
from the operand rounding."""
import math

import numpy as np
import pytest

from oracle import codec
from oracle import transform as tf
from synth import BASE_SEED, luma_batch, mixed_image, random_blocks_u8

from batch_util import Batch
from test_gpu_parity import _images_i16, _images_u8

pytestmark = pytest.mark.gpu


def A():
    import paper_1606_05562_amd as mod
    return mod


def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def batch_u8():
    return Batch(_images_u8())


@pytest.fixture(scope="module")
def batch_worst():
    # uniformly random blocks plus sign patterns of every pair of rows of T
    # (the blocks that reach the extreme coefficients)
    rnd = random_blocks_u8(BASE_SEED + 11, 1024)
    t = tf.T
    pats = [np.where(np.outer(t[u], t[v]) > 0, 255, 0).astype(np.uint8) for u in range(16) for v in range(16)]
    pats += [255 - p for p in pats]
    blocks = np.concatenate([rnd, np.stack(pats)])            # 1536 blocks
    img = blocks.reshape(24, 64, 16, 16).transpose(0, 2, 1, 3).reshape(24 * 16, 64 * 16)
    return Batch([img])


@pytest.mark.parametrize("int8", [False, True])
@pytest.mark.parametrize("cd", ["i32", "i16"])
def test_mfma_forward_bit_exact(batch_u8, cd, int8):
    # int8: int8 products with int32 accumulation on hi/lo digit planes;
    # otherwise exact FP16 products
    T = torch()
    plan = batch_u8.plan(coef_dtype=A().I32 if cd == "i32" else A().I16, backend=A().BACKEND_MFMA,
                         flags=A().FLAG_MFMA_INT8 if int8 else 0)
    coef = batch_u8.coef_tensor(T.int32 if cd == "i32" else T.int16)
    plan.forward(batch_u8.dev, coef)
    T.cuda.synchronize()
    for got, im in zip(batch_u8.split_coef(coef), batch_u8.images):
        want = codec.forward_image(im)
        if cd == "i16":
            want = want.copy()
            want[:, 0, 0] -= 32768
        assert np.array_equal(got.astype(np.int64), want)


def _fused(batch, backend, qmode, r, flags=0):
    T = torch()
    plan = batch.plan(coef_dtype=A().I32, qmode=qmode, r=r, backend=backend, flags=flags)
    out = batch.empty_like_images(np.uint8, 1)
    sse = T.zeros(len(batch.images), dtype=T.int64, device="cuda")
    psnr = T.zeros(len(batch.images), dtype=T.float64, device="cuda")
    plan.compress_and_measure(batch.dev, out, None, sse, psnr)
    T.cuda.synchronize()
    return batch.unpack(out), sse.cpu().numpy(), psnr.cpu().numpy()


CASES = [(1, r) for r in (1, 2, 3, 5, 8, 9, 12, 16)] + [(0, 16)] + [(2, r) for r in (1, 16, 100, 181, 256)]


@pytest.mark.parametrize("explicit", [False, True])
@pytest.mark.parametrize("qmode,r", CASES)
def test_mfma_fused_bit_exact(batch_u8, qmode, r, explicit):
    # explicit: coefficients formed per block; otherwise separable masks use
    # the single contraction with G = T^T diag(w m) T.
    keep = {0: codec.mask_none(), 1: codec.mask_zonal(r), 2: codec.mask_zigzag(r)}[qmode]
    recs, sse, psnr = _fused(batch_u8, A().BACKEND_MFMA, qmode, r, A().FLAG_EXPLICIT_COEF if explicit else 0)
    for i, (got, im) in enumerate(zip(recs, batch_u8.images)):
        want, s, p = codec.compress_kept(im, keep)
        assert np.array_equal(got, want), f"image {i}"
        assert sse[i] == s
        assert (math.isinf(p) and math.isinf(psnr[i])) or abs(psnr[i] - p) <= 1e-3


@pytest.mark.parametrize("explicit", [False, True])
@pytest.mark.parametrize("qmode,r", [(1, 8), (1, 16), (2, 181), (1, 1), (0, 16)])
def test_mfma_equals_adder_kernel_on_extremes(batch_worst, qmode, r, explicit):
    a = _fused(batch_worst, A().BACKEND_MFMA, qmode, r, A().FLAG_EXPLICIT_COEF if explicit else 0)
    b = _fused(batch_worst, A().BACKEND_VALU, qmode, r)
    assert np.array_equal(a[0][0], b[0][0]) and np.array_equal(a[1], b[1])
    keep = {0: codec.mask_none(), 1: codec.mask_zonal(r), 2: codec.mask_zigzag(r)}[qmode]
    want, s, _ = codec.compress_kept(batch_worst.images[0], keep)
    assert np.array_equal(a[0][0], want) and a[1][0] == s


# ----------------------------------------------------------------------------
# The round trip as int8 products (flag MFMA_INT8, separable masks):
# N = G Xc G with G = T^T diag(w m) T, the intermediate Xc G on signed
# base-256 digit planes.

INT8_CASES = [(1, r) for r in (1, 2, 3, 5, 8, 9, 12, 16)] + [(0, 16)]


@pytest.mark.parametrize("qmode,r", INT8_CASES)
def test_mfma_int8_fused_bit_exact(batch_u8, qmode, r):
    keep = {0: codec.mask_none(), 1: codec.mask_zonal(r)}[qmode]
    plan = batch_u8.plan(coef_dtype=A().I32, qmode=qmode, r=r, backend=A().BACKEND_MFMA, flags=A().FLAG_MFMA_INT8)
    import json
    assert json.loads(plan.info())["fused_form"] == "int8"
    recs, sse, psnr = _fused(batch_u8, A().BACKEND_MFMA, qmode, r, A().FLAG_MFMA_INT8)
    for i, (got, im) in enumerate(zip(recs, batch_u8.images)):
        want, s, p = codec.compress_kept(im, keep)
        assert np.array_equal(got, want), f"image {i}"
        assert sse[i] == s
        assert (math.isinf(p) and math.isinf(psnr[i])) or abs(psnr[i] - p) <= 1e-3


@pytest.fixture(scope="module")
def batch_int8_worst():
    """The extreme blocks of batch_worst plus, for every r x r mask and every
    column n of G_r = T^T diag(w m_r) T, the block whose rows all follow the
    sign pattern of G_r[:, n] (and its complement): these reach the largest
    |Xc G| = 128 sum_j |G_r[j][n]| (13312 at most)."""
    t = tf.T.astype(np.int64)
    w = tf.inverse_weights(tf.T).astype(np.int64)
    pats = []
    for r in range(1, 17):
        g = t.T @ np.diag(w * (np.arange(16) < r)) @ t
        for n in range(16):
            row = np.where(g[:, n] > 0, 255, 0).astype(np.uint8)
            pats.append(np.tile(row, (16, 1)))
            pats.append(255 - np.tile(row, (16, 1)))
    rnd = random_blocks_u8(BASE_SEED + 11, 1024)
    tp = [np.where(np.outer(t[u], t[v]) > 0, 255, 0).astype(np.uint8) for u in range(16) for v in range(16)]
    tp += [255 - p for p in tp]
    blocks = np.concatenate([rnd, np.stack(tp), np.stack(pats)])  # 1536 + 512 blocks
    img = blocks.reshape(32, 64, 16, 16).transpose(0, 2, 1, 3).reshape(32 * 16, 64 * 16)
    return Batch([img])


@pytest.mark.parametrize("qmode,r", [(1, 1), (1, 3), (1, 8), (1, 13), (1, 16), (0, 16)])
def test_mfma_int8_equals_adder_kernel_on_extremes(batch_int8_worst, qmode, r):
    a = _fused(batch_int8_worst, A().BACKEND_MFMA, qmode, r, A().FLAG_MFMA_INT8)
    b = _fused(batch_int8_worst, A().BACKEND_VALU, qmode, r)
    assert np.array_equal(a[0][0], b[0][0]) and np.array_equal(a[1], b[1])
    keep = {0: codec.mask_none(), 1: codec.mask_zonal(r)}[qmode]
    want, s, _ = codec.compress_kept(batch_int8_worst.images[0], keep)
    assert np.array_equal(a[0][0], want) and a[1][0] == s


@pytest.mark.parametrize("align", [16, 128])
def test_mfma_int8_ragged_and_wht(align):
    # ragged edges (both task tables' edge strips), and the Walsh-Hadamard
    # matrix through the same int8 kernel against the adder kernel
    rng = np.random.default_rng(23)
    sizes = [(int(x), int(y)) for x, y in rng.integers(16, 300, size=(6, 2))] + [(272, 384), (33, 2050)]
    ims = [mixed_image(BASE_SEED + 4, k, h, w) for k, (h, w) in enumerate(sizes)]
    b = Batch(ims, align)
    recs, sse, _ = _fused(b, A().BACKEND_MFMA, A().Q_ZONAL, 6, A().FLAG_MFMA_INT8)
    for i, (got, im) in enumerate(zip(recs, ims)):
        want, s, _ = codec.compress_kept(im, codec.mask_zonal(6))
        assert np.array_equal(got, want) and sse[i] == s, f"image {i} {sizes[i]}"
    T = torch()
    outs = []
    for be, fl in ((A().BACKEND_MFMA, A().FLAG_MFMA_INT8), (A().BACKEND_VALU, 0)):
        plan = b.plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=5, backend=be, flags=fl, matrix=A().MATRIX_WHT)
        out = b.empty_like_images(np.uint8, 1)
        sse2 = T.zeros(len(ims), dtype=T.int64, device="cuda")
        plan.compress_and_measure(b.dev, out, None, sse2, None)
        T.cuda.synchronize()
        outs.append((out.cpu().numpy(), sse2.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_mfma_int8_full_size():
    """The 256-frame 1920x1088 batch at r = 8 through the int8 round trip:
    sampled frames against the oracle, every pixel and SSE against the FP16
    matrix-core form."""
    T = torch()
    mod = A()
    n, h, w = 256, 1088, 1920
    frames = luma_batch(BASE_SEED + 2, n, h, w)
    dev = T.from_numpy(frames.reshape(-1)).cuda()
    offs = [i * h * w for i in range(n)]
    res = []
    for fl in (mod.FLAG_MFMA_INT8, 0):
        plan = mod.Plan([h] * n, [w] * n, [w] * n, offs, in_dtype=mod.U8, coef_dtype=mod.I32, qmode=mod.Q_ZONAL,
                        r=8, backend=mod.BACKEND_MFMA, flags=fl)
        out = T.empty_like(dev)
        sse = T.zeros(n, dtype=T.int64, device="cuda")
        plan.compress_and_measure(dev, out, None, sse, None)
        T.cuda.synchronize()
        res.append((out, sse))
    out, sse = res[0]
    for t in (1, 254):
        got = out[t * h * w:(t + 1) * h * w].cpu().numpy().reshape(h, w)
        want, s, _ = codec.compress_kept(frames[t], codec.mask_zonal(8))
        assert np.array_equal(got, want) and int(sse[t]) == s
    assert T.equal(out, res[1][0]) and T.equal(sse, res[1][1])


@pytest.mark.parametrize("int8", [False, True])
def test_mfma_forward_extremes(batch_worst, int8):
    # sign patterns of the rows of T reach |P| = 2048 and the extreme Z
    T = torch()
    plan = batch_worst.plan(coef_dtype=A().I32, backend=A().BACKEND_MFMA, flags=A().FLAG_MFMA_INT8 if int8 else 0)
    coef = batch_worst.coef_tensor(T.int32)
    plan.forward(batch_worst.dev, coef)
    T.cuda.synchronize()
    got = batch_worst.split_coef(coef)[0]
    assert np.array_equal(got.astype(np.int64), codec.forward_image(batch_worst.images[0]))


@pytest.mark.parametrize("align", [16, 128])
def test_mfma_ragged(align):
    # align 128: whole-cache-line rows, the streaming (non-temporal) variant
    rng = np.random.default_rng(21)
    sizes = [(int(x), int(y)) for x, y in rng.integers(16, 300, size=(7, 2))]
    sizes += [(272, 384), (32, 128)]  # widths that are whole strips
    ims = [mixed_image(BASE_SEED + 4, k, h, w) for k, (h, w) in enumerate(sizes)]
    b = Batch(ims, align)
    recs, sse, _ = _fused(b, A().BACKEND_MFMA, A().Q_ZONAL, 8)
    for i, (got, im) in enumerate(zip(recs, ims)):
        want, s, _ = codec.compress_kept(im, codec.mask_zonal(8))
        assert np.array_equal(got, want) and sse[i] == s


@pytest.mark.parametrize("strips", [1, 2, 3, 4, 16])
def test_mfma_task_sizes(monkeypatch, strips):
    """The task tables (equal runs of at most 1, 2, 3, 4 or 16 strips of a block
    row), on images whose block rows hold fewer and more strips than a run
    and split into runs of unequal length (2050 pixels: 17 strips, 8 + 9 or
    3 + 3 + 4 + 3 + 4), through the fused kernel and both forward forms."""
    monkeypatch.setenv("ADCT16_TASK_STRIPS", str(strips))
    T = torch()
    sizes = [(48, 16), (40, 130), (33, 2050), (20, 4000), (272, 384), (70, 1920), (16, 2048), (24, 3840)]
    ims = [mixed_image(BASE_SEED + 6, k, h, w) for k, (h, w) in enumerate(sizes)]
    b = Batch(ims, 128)
    plan = b.plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=6, backend=A().BACKEND_MFMA)
    import json
    assert json.loads(plan.info())["task_strips"] == strips
    recs, sse, _ = _fused(b, A().BACKEND_MFMA, A().Q_ZONAL, 6)
    for i, (got, im) in enumerate(zip(recs, ims)):
        want, s, _ = codec.compress_kept(im, codec.mask_zonal(6))
        assert np.array_equal(got, want) and sse[i] == s, f"image {i} {sizes[i]}"
    for int8 in (False, True):
        p = b.plan(coef_dtype=A().I32, backend=A().BACKEND_MFMA, flags=A().FLAG_MFMA_INT8 if int8 else 0)
        coef = b.coef_tensor(T.int32)
        p.forward(b.dev, coef)
        T.cuda.synchronize()
        for i, (got, im) in enumerate(zip(b.split_coef(coef), ims)):
            assert np.array_equal(got.astype(np.int64), codec.forward_image(im)), f"int8={int8} image {i}"


def test_mfma_full_size_sampled():
    T = torch()
    mod = A()
    n, h, w = 256, 1088, 1920
    frames = luma_batch(BASE_SEED + 2, n, h, w)
    dev = T.from_numpy(frames.reshape(-1)).cuda()
    plan = mod.Plan([h] * n, [w] * n, [w] * n, [i * h * w for i in range(n)], in_dtype=mod.U8,
                    coef_dtype=mod.I32, qmode=mod.Q_ZONAL, r=8, backend=mod.BACKEND_MFMA)
    out = T.empty_like(dev)
    sse = T.zeros(n, dtype=T.int64, device="cuda")
    plan.compress_and_measure(dev, out, None, sse, None)
    T.cuda.synchronize()
    for t in (3, 200):
        got = out[t * h * w:(t + 1) * h * w].cpu().numpy().reshape(h, w)
        want, s, _ = codec.compress_kept(frames[t], codec.mask_zonal(8))
        assert np.array_equal(got, want) and int(sse[t]) == s
    ref = mod.Plan([h] * n, [w] * n, [w] * n, [i * h * w for i in range(n)], in_dtype=mod.U8,
                   coef_dtype=mod.I32, qmode=mod.Q_ZONAL, r=8, backend=mod.BACKEND_VALU)
    out2 = T.empty_like(dev)
    sse2 = T.zeros(n, dtype=T.int64, device="cuda")
    ref.compress_and_measure(dev, out2, None, sse2, None)
    T.cuda.synchronize()
    assert T.equal(out, out2) and T.equal(sse, sse2)


def test_full_size_bench_configuration():
    """The default benchmark's call, exactly as bench.py makes it (256 luma
    frames 1920x1088, zonal r = 8, backend and launch shape chosen by the
    autotuner): sampled frames completely against the oracle, and every
    pixel, SSE and PSNR of the batch against the vector adder kernel."""
    import json
    T = torch()
    mod = A()
    n, h, w = 256, 1088, 1920
    frames = luma_batch(BASE_SEED + 2, n, h, w)  # the benchmark's frames
    dev = T.from_numpy(frames.reshape(-1)).cuda()
    offs = [i * h * w for i in range(n)]
    plan = mod.Plan([h] * n, [w] * n, [w] * n, offs, in_dtype=mod.U8, coef_dtype=mod.I32, qmode=mod.Q_ZONAL,
                    r=8, backend=mod.BACKEND_AUTO, flags=mod.FLAG_AUTOTUNE)
    info = json.loads(plan.info())
    out = T.empty_like(dev)
    sse = T.zeros(n, dtype=T.int64, device="cuda")
    psnr = T.zeros(n, dtype=T.float64, device="cuda")
    for _ in range(2):  # a replay sees the state the first call left
        plan.compress_and_measure(dev, out, None, sse, psnr)
    T.cuda.synchronize()
    keep = codec.mask_zonal(8)
    for t in (0, 131, 255):
        got = out[t * h * w:(t + 1) * h * w].cpu().numpy().reshape(h, w)
        want, s, p = codec.compress_kept(frames[t], keep)
        assert np.array_equal(got, want), f"frame {t} ({info})"
        assert int(sse[t]) == s and abs(float(psnr[t]) - p) <= 1e-3, f"frame {t}"
    ref = mod.Plan([h] * n, [w] * n, [w] * n, offs, in_dtype=mod.U8, coef_dtype=mod.I32, qmode=mod.Q_ZONAL,
                   r=8, backend=mod.BACKEND_VALU)
    out2 = T.empty_like(dev)
    sse2 = T.zeros(n, dtype=T.int64, device="cuda")
    psnr2 = T.zeros(n, dtype=T.float64, device="cuda")
    ref.compress_and_measure(dev, out2, None, sse2, psnr2)
    T.cuda.synchronize()
    assert T.equal(out, out2) and T.equal(sse, sse2) and T.equal(psnr, psnr2)


# ----------------------------------------------------------------------------
# Exact DCT-II on BF16 / F16 operands (comparison transform).

def _dct_bound(xc, eps):
    """|Y_gpu - C Xc C^T| <= ((1+eps)^3 - 1 + 2^-20) |C| |Xc| |C|^T elementwise:
    C rounded once (both sides), the row-pass result rounded once, FP32
    accumulation error far below the operand rounding."""
    c = np.abs(tf.dct_matrix())
    mag = c @ np.abs(xc) @ c.T
    return ((1 + eps) ** 3 - 1 + 2.0 ** -20) * mag


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_dct_mfma_error_bound(batch_u8, prec):
    T = torch()
    mod = A()
    plan = batch_u8.plan(coef_dtype=mod.I32)
    y = batch_u8.coef_tensor(T.float32)
    plan.dct_forward(batch_u8.dev, y, mod.F16 if prec == "f16" else mod.BF16)
    T.cuda.synchronize()
    eps = 2.0 ** -11 if prec == "f16" else 2.0 ** -8
    worst_abs, worst_rel = 0.0, 0.0
    for got, im in zip(batch_u8.split_coef(y), batch_u8.images):
        xc = codec.image_to_blocks(im).astype(np.float64) - 128.0
        ref = tf.dct_forward(xc)
        err = np.abs(got - ref)
        assert np.all(err <= _dct_bound(xc, eps))
        worst_abs = max(worst_abs, float(err.max()))
        worst_rel = max(worst_rel, float(err.max() / max(1.0, np.abs(ref).max())))
    print(f"DCT-II {prec}: max abs error {worst_abs:.4g}, relative to max|Y| {worst_rel:.3g}")


@pytest.mark.parametrize("kw", [dict(in_dtype=2, coef_dtype=4, out_dtype=2), dict(coef_dtype=4, out_dtype=4)])
def test_mfma_unsupported_plans_rejected(kw):
    # no call of these plans has a matrix-core form (float coefficients, and
    # no fused matrix-core call for the mode or dtypes)
    mod = A()
    args = dict(in_dtype=mod.U8, coef_dtype=mod.I32, qmode=mod.Q_ZONAL, r=8, backend=mod.BACKEND_MFMA)
    args.update(kw)
    with pytest.raises(mod.Adct16Error) as e:
        mod.Plan([32], [32], [32], [0], **args)
    assert e.value.status == mod.E_MODE


def test_mfma_backend_per_call():
    """A matrix-core plan runs each call that has a matrix-core form there;
    the others (here the quantiser's fused call) run on the vector ALUs."""
    import json
    mod = A()
    p = mod.Plan([32], [32], [32], [0], in_dtype=mod.I16, coef_dtype=mod.I32, qmode=mod.Q_UNIFORM, q=8,
                 qcoef_dtype=mod.I16, out_dtype=mod.I16, backend=mod.BACKEND_MFMA)
    info = json.loads(p.info())
    assert info["forward_backend"] == "mfma" and info["fused_backend"] == "valu"
    p = mod.Plan([32], [32], [32], [0], in_dtype=mod.U8, coef_dtype=mod.I32, qmode=mod.Q_ZONAL, r=8,
                 backend=mod.BACKEND_MFMA)
    info = json.loads(p.info())
    assert info["forward_backend"] == "mfma" and info["fused_backend"] == "mfma"


def _images_i16_full():
    """Residual planes plus full-range 16-bit content: uniform samples, the
    extreme values, and the sign patterns of pairs of rows of T at +-32767 /
    -32768, which reach the extreme coefficients; widths and heights give
    interior strips, partial strips and partial blocks."""
    rng = np.random.default_rng(16)
    ims = list(_images_i16())
    ims.append(rng.integers(-32768, 32768, (48, 300)).astype(np.int16))
    ims.append(rng.integers(-32768, 32768, (32, 256)).astype(np.int16))
    ims.append(np.full((20, 130), -32768, dtype=np.int16))
    ims.append(np.full((16, 144), 32767, dtype=np.int16))
    t = tf.T
    pats = [np.where(np.outer(t[u], t[v]) > 0, 32767, -32768).astype(np.int16) for u in range(16) for v in range(16)]
    ims.append(np.concatenate([np.concatenate(pats[k * 16:(k + 1) * 16], axis=1) for k in range(16)], axis=0))
    return ims


@pytest.mark.parametrize("align,strips", [(16, 4), (128, 1), (128, 4), (128, 16)])
def test_mfma_forward_i16_bit_exact(monkeypatch, align, strips):
    """16-bit input through the int8 form with three base-64 digits per value
    (both passes): bit-exact with the oracle and the vector-ALU forward on
    the whole int16 range."""
    monkeypatch.setenv("ADCT16_TASK_STRIPS", str(strips))
    T = torch()
    mod = A()
    ims = _images_i16_full()
    b = Batch(ims, align)
    coefs = {}
    for be in (mod.BACKEND_MFMA, mod.BACKEND_VALU):
        plan = b.plan(coef_dtype=mod.I32, out_dtype=mod.I16, backend=be)
        coef = b.coef_tensor(T.int32)
        plan.forward(b.dev, coef)
        T.cuda.synchronize()
        coefs[be] = b.split_coef(coef)
    for i, im in enumerate(ims):
        want = codec.forward_image(im)
        assert np.array_equal(coefs[mod.BACKEND_MFMA][i].astype(np.int64), want), f"image {i} {im.shape}"
        assert np.array_equal(coefs[mod.BACKEND_MFMA][i], coefs[mod.BACKEND_VALU][i])


def test_mfma_fused_needs_32bit_offsets():
    """The line stores of the strip kernel address a strip row through a
    32-bit buffer range: plans whose images reach 2^31 bytes, or whose rows
    reach 2^24 bytes, keep the vector kernel for the fused call (geometry
    only; nothing is launched)."""
    import json
    mod = A()
    def fused_backend(h, pitch):
        plan = mod.Plan([h], [64], [pitch], [0], in_dtype=mod.U8, coef_dtype=mod.I32, qmode=mod.Q_ZONAL, r=8,
                        backend=mod.BACKEND_MFMA)
        return json.loads(plan.info())["fused_backend"]
    assert fused_backend(16, (1 << 24) - 128) == "mfma"    # rows just below 16 MiB
    assert fused_backend(16, 1 << 24) == "valu"            # 16 MiB rows
    assert fused_backend(16383, 1 << 17) == "mfma"         # just below 2 GiB
    assert fused_backend(16384, 1 << 17) == "valu"         # 2 GiB


@pytest.mark.parametrize("strips", [1, 2, 3, 4, 16])
def test_mfma_unaligned_rows_line_stores(monkeypatch, strips):
    """Rows at 16-byte pitches and offsets (not whole cache lines): the
    strip kernel writes whole aligned lines, each from two consecutive strips
    of a run plus a tail after the run's last interior strip.  Every image
    byte equals the oracle's, and no byte outside the images (row padding,
    gaps between images) is written.  Widths give every shift of a row in its
    line, runs of 1 to 16 strips, and edge strips after interior ones."""
    monkeypatch.setenv("ADCT16_TASK_STRIPS", str(strips))
    T = torch()
    sizes = [(48, 1040), (33, 2050), (16, 2048), (40, 1936), (17, 1000), (64, 3856), (20, 272), (32, 128)]
    ims = [mixed_image(BASE_SEED + 9, k, h, w) for k, (h, w) in enumerate(sizes)]
    b = Batch(ims, 16)
    fill = 0xA5
    plan = b.plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=6, backend=A().BACKEND_MFMA)
    import json
    info = json.loads(plan.info())
    assert info["rows_line_aligned"] is False and info["task_strips"] == strips
    out = b.empty_like_images(np.uint8, fill)
    sse = T.zeros(len(ims), dtype=T.int64, device="cuda")
    plan.compress_and_measure(b.dev, out, None, sse, None)
    T.cuda.synchronize()
    flat = out.cpu().numpy()
    inside = np.zeros(len(flat), dtype=bool)
    for i, (im, h, w, p, o) in enumerate(zip(ims, b.h, b.w, b.p, b.o)):
        want, s, _ = codec.compress_kept(im, codec.mask_zonal(6))
        got = flat[o:o + h * p].reshape(h, p)[:, :w]
        assert np.array_equal(got, want) and int(sse[i]) == s, f"image {i} {sizes[i]}"
        inside[o:o + h * p].reshape(h, p)[:, :w] = True
    assert np.all(flat[~inside] == fill)
