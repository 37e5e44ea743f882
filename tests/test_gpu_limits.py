"""Parity at the limits of the batch description (Section 4's blockwise
2-D transform applied to every image of a batch).

* images at the largest width and height the C ABI accepts (65536), and one
  pixel short of it (ragged in both directions);
* the largest image count (2^20), every image a single pixel;
* a batch whose pixel offsets pass 2^31 elements and whose coefficient
  offsets pass 2^31 elements (2^33 bytes), sampled frames checked completely
  against the oracle, every frame through properties that hold at any size.

Bars as in the other parity tests: integers and rounded pixels bit-exact,
PSNR within 1e-3 dB."""
import math

import numpy as np
import pytest

from oracle import codec
from synth import BASE_SEED, ar1_image, luma_batch, residual_plane

from batch_util import Batch

pytestmark = pytest.mark.gpu

PSNR_TOL_DB = 1e-3


def A():
    import paper_1606_05562_amd as mod
    return mod


def torch():
    import torch as t
    return t


def _psnr_close(got, want):
    if math.isinf(want):
        return math.isinf(got)
    return abs(got - want) <= PSNR_TOL_DB


LIMIT_SHAPES = [(16, 65536), (65536, 16), (17, 65535), (65535, 17)]


@pytest.fixture(scope="module")
def batch_limits():
    return Batch([ar1_image(BASE_SEED + 40 + k, h, w) for k, (h, w) in enumerate(LIMIT_SHAPES)])


def _backend(name):
    return {"valu": A().BACKEND_VALU, "mfma": A().BACKEND_MFMA}[name]


@pytest.mark.parametrize("backend", ["valu", "mfma"])
@pytest.mark.parametrize("qmode,r", [(1, 8), (2, 100)])
def test_limit_shapes_fused(batch_limits, backend, qmode, r):
    T = torch()
    b = batch_limits
    plan = b.plan(coef_dtype=A().I32, qmode=qmode, r=r, backend=_backend(backend))
    out = b.empty_like_images(np.uint8, 7)
    sse = T.zeros(len(b.images), dtype=T.int64, device="cuda")
    psnr = T.zeros(len(b.images), dtype=T.float64, device="cuda")
    plan.compress_and_measure(b.dev, out, None, sse, psnr)
    T.cuda.synchronize()
    keep = codec.mask_zonal(r) if qmode == 1 else codec.mask_zigzag(r)
    for i, (got, im) in enumerate(zip(b.unpack(out), b.images)):
        want, s, p = codec.compress_kept(im, keep)
        assert np.array_equal(got, want), f"image {i} {im.shape}"
        assert int(sse[i]) == s and _psnr_close(float(psnr[i]), p)


def test_limit_shapes_levels_written(batch_limits):
    # the fused call that also writes the retained coefficients (centred int16)
    T = torch()
    b = batch_limits
    plan = b.plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=4, qcoef_dtype=A().I16)
    out = b.empty_like_images(np.uint8)
    qc = b.coef_tensor(T.int16)
    plan.compress_and_measure(b.dev, out, qc, None, None)
    T.cuda.synchronize()
    keep = codec.mask_zonal(4)
    for i, (got_c, got, im) in enumerate(zip(b.split_coef(qc), b.unpack(out), b.images)):
        zc = np.where(keep[None], codec.forward_image(im), 0)
        zc[:, 0, 0] -= 32768
        assert np.array_equal(got_c.astype(np.int64), zc), f"image {i}"
        assert np.array_equal(got, codec.compress_kept(im, keep)[0])


@pytest.mark.parametrize("backend,flags", [("valu", 0), ("mfma", 0), ("mfma", "int8")])
def test_limit_shapes_forward_and_inverse(batch_limits, backend, flags):
    T = torch()
    b = batch_limits
    fl = A().FLAG_MFMA_INT8 if flags == "int8" else 0
    plan = b.plan(coef_dtype=A().I32, qmode=A().Q_ZIGZAG, r=37, backend=_backend(backend), flags=fl)
    coef = b.coef_tensor(T.int32)
    plan.forward(b.dev, coef)
    kept = b.coef_tensor(T.int32)
    plan.quantise(coef, kept)
    out = b.empty_like_images(np.uint8)
    plan.inverse(kept, out)
    T.cuda.synchronize()
    keep = codec.mask_zigzag(37)
    for i, (z, zk, got, im) in enumerate(zip(b.split_coef(coef), b.split_coef(kept), b.unpack(out), b.images)):
        want = codec.forward_image(im)
        assert np.array_equal(z.astype(np.int64), want), f"image {i}"
        assert np.array_equal(zk.astype(np.int64), np.where(keep[None], want, 0))
        assert np.array_equal(got, codec.compress_kept(im, keep)[0])


def test_limit_shapes_residual_uniform():
    T = torch()
    ims = [residual_plane(BASE_SEED + 44, 0, 0, 16, 65536), residual_plane(BASE_SEED + 45, 0, 0, 65535, 17)]
    b = Batch(ims)
    q = 16
    plan = b.plan(coef_dtype=A().I32, qmode=A().Q_UNIFORM, q=q, qcoef_dtype=A().I16, out_dtype=A().I16)
    out = b.empty_like_images(np.int16)
    lv = b.coef_tensor(T.int16)
    sse = T.zeros(len(ims), dtype=T.int64, device="cuda")
    plan.compress_and_measure(b.dev, out, lv, sse, None)
    T.cuda.synchronize()
    for i, (got, lvl, im) in enumerate(zip(b.unpack(out), b.split_coef(lv), ims)):
        h, w = im.shape
        want_lv = codec.quantise_uniform(codec.forward_image(im), q)
        assert np.array_equal(lvl.astype(np.int64), want_lv), f"image {i}"
        real = codec.reconstruct_uniform(want_lv, q, h, w, rounded=False)
        want = np.clip(np.floor(real + 0.5), -32768, 32767)
        diff = got.astype(np.int64) - want.astype(np.int64)
        tie = np.abs(real - np.floor(real) - 0.5) < 1e-9
        assert np.all(np.abs(diff) <= 1) and np.all(tie[diff != 0])
        assert int(sse[i]) == codec.sse(im, got)
    # the matrix-core forward of 16-bit input
    mplan = b.plan(coef_dtype=A().I32, out_dtype=A().I16, backend=A().BACKEND_MFMA)
    coef = b.coef_tensor(T.int32)
    mplan.forward(b.dev, coef)
    T.cuda.synchronize()
    for i, (z, im) in enumerate(zip(b.split_coef(coef), ims)):
        assert np.array_equal(z.astype(np.int64), codec.forward_image(im)), f"image {i}"


# ----------------------------------------------------------------------------
# 2^20 images of one pixel each.  Edge extension makes every block constant,
# so only the DC coefficient 256 v is non-zero and every retention mask
# reconstructs the pixel exactly: SSE 0 and PSNR +inf for every image.

@pytest.mark.parametrize("backend", ["valu", "mfma"])
def test_max_image_count(backend):
    T = torch()
    mod = A()
    n = 1 << 20
    vals = np.random.default_rng([BASE_SEED, 0x1F1]).integers(0, 256, n, dtype=np.uint8)
    buf = np.zeros(n * 16, dtype=np.uint8)
    buf[::16] = vals
    dev = T.from_numpy(buf).cuda()
    plan = mod.Plan([1] * n, [1] * n, [16] * n, [16 * i for i in range(n)], in_dtype=mod.U8,
                    coef_dtype=mod.I32, qmode=mod.Q_ZONAL, r=2, backend=_backend(backend))
    assert plan.num_blocks == n
    out = T.full_like(dev, 3)
    sse = T.full((n,), -1, dtype=T.int64, device="cuda")
    psnr = T.zeros(n, dtype=T.float64, device="cuda")
    plan.compress_and_measure(dev, out, None, sse, psnr)
    T.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(got[::16], vals)
    assert int(T.count_nonzero(sse)) == 0
    assert bool(T.isinf(psnr).all())
    # sampled images through the oracle, and the coefficients of every block
    for i in (0, 1, n // 2 + 3, n - 1):
        want, s, p = codec.compress_kept(vals[i].reshape(1, 1), codec.mask_zonal(2))
        assert got[16 * i] == want[0, 0] and s == 0 and math.isinf(p)
    coef = T.zeros(n * 256, dtype=T.int32, device="cuda")
    plan.forward(dev, coef)
    T.cuda.synchronize()
    c = coef.view(n, 256)
    assert T.equal(c[:, 0].cpu(), T.from_numpy(vals.astype(np.int32) * 256))
    assert int(T.count_nonzero(c[:, 1:])) == 0
    assert np.array_equal(coef[:256].cpu().numpy().reshape(1, 16, 16),
                          codec.forward_image(vals[:1].reshape(1, 1)).astype(np.int32))


# ----------------------------------------------------------------------------
# 1040 frames of 1920x1088: 2.17e9 pixels (past 2^31 elements) and 8.5e6
# blocks, so int32 coefficients pass 2^31 elements (8.7 GB).  Frame t is
# luma frame t mod 4 rotated by t columns: every frame differs.

N_BIG, H_BIG, W_BIG = 1040, 1088, 1920
SAMPLED = (0, 257, 514, 1027, 1028, 1039)  # coefficient bytes pass 2^31, 2^32; pixels and elements pass 2^31


def _big_frame(base, t):
    return np.roll(base[t % len(base)], t, axis=1)


@pytest.fixture(scope="module")
def big_batch():
    T = torch()
    assert N_BIG * H_BIG * W_BIG > 2 ** 31 and N_BIG * (H_BIG // 16) * (W_BIG // 16) * 256 > 2 ** 31
    base = luma_batch(BASE_SEED + 46, 4, H_BIG, W_BIG)
    bd = T.from_numpy(base).cuda()
    dev = T.empty(N_BIG * H_BIG * W_BIG, dtype=T.uint8, device="cuda")
    view = dev.view(N_BIG, H_BIG, W_BIG)
    for t in range(N_BIG):
        view[t] = T.roll(bd[t % 4], shifts=t, dims=1)
    T.cuda.synchronize()
    return base, dev


def _big_plan(**kw):
    mod = A()
    n, h, w = N_BIG, H_BIG, W_BIG
    return mod.Plan([h] * n, [w] * n, [w] * n, [i * h * w for i in range(n)], in_dtype=mod.U8, **kw)


@pytest.mark.parametrize("backend", ["valu", "mfma"])
def test_batch_past_2_31_fused(big_batch, backend):
    T = torch()
    base, dev = big_batch
    n, hw = N_BIG, H_BIG * W_BIG
    plan = _big_plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=8, backend=_backend(backend))
    out = T.empty_like(dev)
    sse = T.zeros(n, dtype=T.int64, device="cuda")
    psnr = T.zeros(n, dtype=T.float64, device="cuda")
    plan.compress_and_measure(dev, out, None, sse, psnr)
    T.cuda.synchronize()
    keep = codec.mask_zonal(8)
    for t in SAMPLED:
        got = out[t * hw:(t + 1) * hw].cpu().numpy().reshape(H_BIG, W_BIG)
        want, s, p = codec.compress_kept(_big_frame(base, t), keep)
        assert np.array_equal(got, want), f"frame {t}"
        assert int(sse[t]) == s and _psnr_close(float(psnr[t]), p), f"frame {t}"
    # every frame: the SSE equals that of the reconstruction written
    m = T.zeros(n, dtype=T.int64, device="cuda")
    plan.measure(dev, out, m)
    T.cuda.synchronize()
    assert T.equal(m, sse)
    del out


def test_batch_past_2_31_forward_and_unfused(big_batch):
    T = torch()
    base, dev = big_batch
    n, hw = N_BIG, H_BIG * W_BIG
    nb = (H_BIG // 16) * (W_BIG // 16)
    keep = codec.mask_zonal(8)
    ref = None
    for backend in ("valu", "mfma"):
        plan = _big_plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=8, backend=_backend(backend))
        coef = T.empty(n * nb * 256, dtype=T.int32, device="cuda")
        plan.forward(dev, coef)
        T.cuda.synchronize()
        for t in SAMPLED:
            got = coef[t * nb * 256:(t + 1) * nb * 256].cpu().numpy().reshape(nb, 16, 16)
            assert np.array_equal(got.astype(np.int64), codec.forward_image(_big_frame(base, t))), \
                f"{backend} frame {t}"
        if ref is None:
            ref = coef
        else:
            assert T.equal(ref, coef)
            del coef
    # quantise + inverse of the valu coefficients equal the fused call, every frame
    plan = _big_plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=8, backend=A().BACKEND_VALU)
    kept = T.empty_like(ref)
    plan.quantise(ref, kept)
    del ref
    out = T.empty_like(dev)
    plan.inverse(kept, out)
    fused = T.empty_like(dev)
    plan.compress_and_measure(dev, fused, None, None, None)
    T.cuda.synchronize()
    assert T.equal(out, fused)
    t = SAMPLED[-1]
    assert np.array_equal(out[t * hw:(t + 1) * hw].cpu().numpy().reshape(H_BIG, W_BIG),
                          codec.compress_kept(_big_frame(base, t), keep)[0])
