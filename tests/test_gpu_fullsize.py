"""Full-size parity in the benchmark's own launch configurations: the
ragged batch (64 images, sides 64..3840) and one 4:2:0 residual frame
(Y 3840x2160, U and V 1920x1080), each planned exactly as bench.py plans
it (autotuned backend and launch shape; the residual frame replayed from a
HIP graph).  Sampled images or every plane go through the oracle; the
whole ragged batch is also compared with the vector adder kernel.

Bars as in the other parity tests: integers and rounded retention pixels
bit-exact, PSNR within 1e-3 dB; uniform-quantiser reconstructions equal
except where the float64 value lies within 1e-9 of a rounding tie."""
import math

import numpy as np
import pytest

from oracle import codec
from synth import BASE_SEED, pack_images, ragged_batch, yuv420_residual_frame

pytestmark = pytest.mark.gpu


def A():
    import paper_1606_05562_amd as mod
    return mod


def torch():
    import torch as t
    return t


def _unpack(flat, h, w, p, o):
    return flat[o:o + h * p].reshape(h, p)[:, :w]


def test_full_size_ragged_bench_configuration():
    T = torch()
    mod = A()
    ims = ragged_batch(BASE_SEED + 4, 64)  # the benchmark's batch
    buf, hs, ws, ps, offs = pack_images(ims, align_elems=128, pitch_multiple=128)
    dev = T.from_numpy(buf).cuda()
    n = len(ims)
    plan = mod.Plan(hs, ws, ps, offs, in_dtype=mod.U8, coef_dtype=mod.I32, qmode=mod.Q_ZONAL, r=8,
                    backend=mod.BACKEND_AUTO, flags=mod.FLAG_AUTOTUNE)
    out = T.zeros_like(dev)
    sse = T.zeros(n, dtype=T.int64, device="cuda")
    psnr = T.zeros(n, dtype=T.float64, device="cuda")
    for _ in range(2):
        plan.compress_and_measure(dev, out, None, sse, psnr)
    T.cuda.synchronize()
    flat = out.cpu().numpy()
    # the smallest, a middle and the largest image, completely
    by_size = sorted(range(n), key=lambda i: hs[i] * ws[i])
    keep = codec.mask_zonal(8)
    for i in (by_size[0], by_size[n // 2], by_size[-1]):
        want, s, p = codec.compress_kept(ims[i], keep)
        got = _unpack(flat, hs[i], ws[i], ps[i], offs[i])
        assert np.array_equal(got, want), f"image {i} {hs[i]}x{ws[i]}"
        assert int(sse[i]) == s and abs(float(psnr[i]) - p) <= 1e-3, f"image {i}"
    # every image against the vector adder kernel (padding columns untouched by both)
    ref = mod.Plan(hs, ws, ps, offs, in_dtype=mod.U8, coef_dtype=mod.I32, qmode=mod.Q_ZONAL, r=8,
                   backend=mod.BACKEND_VALU)
    out2 = T.zeros_like(dev)
    sse2 = T.zeros(n, dtype=T.int64, device="cuda")
    ref.compress_and_measure(dev, out2, None, sse2, None)
    T.cuda.synchronize()
    assert T.equal(out, out2) and T.equal(sse, sse2)


def test_full_size_residual_frame_bench_configuration():
    T = torch()
    mod = A()
    q = 16
    planes = yuv420_residual_frame(BASE_SEED + 5, 0)  # the benchmark's first frame
    buf, hs, ws, ps, offs = pack_images(planes)
    dev = T.from_numpy(buf).cuda()
    rec = T.zeros_like(dev)
    plan = mod.Plan(hs, ws, ps, offs, in_dtype=mod.I16, coef_dtype=mod.I32, qmode=mod.Q_UNIFORM, q=q,
                    qcoef_dtype=mod.I16, out_dtype=mod.I16, flags=mod.FLAG_AUTOTUNE)
    lv = T.zeros(plan.num_blocks * 256, dtype=T.int16, device="cuda")
    sse = T.zeros(len(hs), dtype=T.int64, device="cuda")
    psnr = T.zeros(len(hs), dtype=T.float64, device="cuda")
    g = plan.graph(dev, rec, lv, sse, psnr)
    for _ in range(2):
        g.launch()
    T.cuda.synchronize()
    flat = rec.cpu().numpy()
    levels = lv.cpu().numpy().reshape(-1, 16, 16)
    first = 0
    for i, im in enumerate(planes):
        h, w = im.shape
        nb = ((h + 15) // 16) * ((w + 15) // 16)
        want_lv = codec.quantise_uniform(codec.forward_image(im), q)
        assert np.array_equal(levels[first:first + nb].astype(np.int64), want_lv), f"plane {i}"
        first += nb
        real = codec.reconstruct_uniform(want_lv, q, h, w, rounded=False)
        got = _unpack(flat, hs[i], ws[i], ps[i], offs[i])
        want = np.clip(np.floor(real + 0.5), -32768, 32767)
        diff = got.astype(np.int64) - want.astype(np.int64)
        tie = np.abs(real - np.floor(real) - 0.5) < 1e-9
        assert np.all(np.abs(diff) <= 1) and np.all(tie[diff != 0]), f"plane {i}"
        s = codec.sse(im, got)
        assert int(sse[i]) == s
        p = codec.psnr_from_sse(s, h * w)
        assert (math.isinf(p) and math.isinf(float(psnr[i]))) or abs(float(psnr[i]) - p) <= 1e-3
