"""The allocation-free fused call, adct16_compress_and_measure_static,
through the C ABI: on two calls in a row (the second with a smaller batch)
its outputs equal those of adct16_compress_and_measure on the same plan and
input, bit for bit (reconstructions, levels, SSE) and PSNR for PSNR; both
kernels (matrix-core and vector) and both SSE destinations (caller's buffer,
the library's scratch) are covered.
"""
import numpy as np
import pytest

from synth import BASE_SEED, ar1_image, luma_frame, residual_plane

from batch_util import Batch

pytestmark = pytest.mark.gpu


def A():
    import paper_1606_05562_amd as mod
    return mod


def _u8_batches():
    rng = np.random.default_rng(11)
    big = [luma_frame(BASE_SEED + 2, t, 1088, 1920) for t in range(3)] + [
        ar1_image(BASE_SEED + 1, 512, 512), rng.integers(0, 256, (37, 50)).astype(np.uint8),
        rng.integers(0, 256, (200, 7)).astype(np.uint8)]
    small = [rng.integers(0, 256, (17, 130)).astype(np.uint8), ar1_image(BASE_SEED + 3, 64, 96)]
    return big, small


def _run_pair(b: Batch, plan, *, out_dtype, levels, sse_given):
    import torch
    n = len(b.images)
    res = []
    for fn in (plan.compress_and_measure, plan.compress_and_measure_static):
        out = b.empty_like_images(out_dtype, fill=7)
        lv = torch.full((b.n_blocks * 256,), 3, dtype=torch.int16, device="cuda") if levels else None
        sse = torch.full((n,), -5, dtype=torch.int64, device="cuda") if sse_given else None
        psnr = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
        fn(b.dev, out, lv, sse, psnr)
        torch.cuda.synchronize()
        res.append((out.cpu().numpy(), None if lv is None else lv.cpu().numpy(),
                    None if sse is None else sse.cpu().numpy(), psnr.cpu().numpy()))
    (o1, l1, s1, p1), (o2, l2, s2, p2) = res
    assert np.array_equal(o1, o2)
    if levels:
        assert np.array_equal(l1, l2)
    if sse_given:
        assert np.array_equal(s1, s2)
        assert (s1 >= 0).all()
    assert np.array_equal(p1, p2)  # same kernels, same integer SSE: identical doubles (inf == inf)
    return p1


@pytest.mark.parametrize("backend_name", ["mfma", "valu"])
@pytest.mark.parametrize("sse_given", [True, False])
def test_static_matches_fused_u8(backend_name, sse_given):
    big, small = _u8_batches()
    backend = {"mfma": A().BACKEND_MFMA, "valu": A().BACKEND_VALU}[backend_name]
    for ims in (big, small):  # second call: smaller batch
        b = Batch(ims)
        plan = b.plan(coef_dtype=A().I32, qmode=A().Q_ZONAL, r=8, backend=backend)
        psnr = _run_pair(b, plan, out_dtype=np.uint8, levels=False, sse_given=sse_given)
        assert np.isfinite(psnr).all()


def test_static_matches_fused_residual_levels():
    big = [residual_plane(BASE_SEED + 5, 0, 0, 272, 480), residual_plane(BASE_SEED + 5, 1, 1, 136, 240)]
    small = [residual_plane(BASE_SEED + 5, 2, 0, 40, 72)]
    for ims in (big, small):
        b = Batch(ims)
        plan = b.plan(coef_dtype=A().I32, qmode=A().Q_UNIFORM, q=16, qcoef_dtype=A().I16, out_dtype=A().I16)
        _run_pair(b, plan, out_dtype=np.int16, levels=True, sse_given=True)
        _run_pair(b, plan, out_dtype=np.int16, levels=False, sse_given=False)


def test_static_rejects_batches_beyond_scratch():
    import torch
    n = 600_000  # 1x1 images: the vector kernel's accumulators need 8 bytes each, 4.8 MB > 4 MiB
    a = A()
    plan = a.Plan([1] * n, [1] * n, [16] * n, [16 * i for i in range(n)], in_dtype=a.U8, coef_dtype=a.I32,
                  qmode=a.Q_ZONAL, r=8, backend=a.BACKEND_VALU)
    x = torch.zeros(16 * n, dtype=torch.uint8, device="cuda")
    with pytest.raises(a.Adct16Error) as ei:
        plan.compress_and_measure_static(x, None, None, None, None)
    assert ei.value.status == a.E_SHAPE
    assert "scratch" in str(ei.value)
