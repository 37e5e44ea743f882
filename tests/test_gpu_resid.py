"""The matrix-core round trip of 16-bit residuals (flag RESIDUAL_RANGE,
MFMA backend): levels bit-exact with the oracle, reconstructions equal to the
oracle's float64 inverse except within 1e-9 of a rounding tie (and then off
by one), SSE exact against the returned reconstruction, PSNR within 1e-3 dB
of the oracle's wherever no tie was rounded the other way; and the same
levels as the vector adder kernel on the same input.

Exact half-integer reconstructions occur only where the terms in sqrt(2),
sqrt(3) and sqrt(6) of the inverse vanish; the extreme sign-pattern blocks
below produce many, and both float64 evaluations may round them either
way."""
import json
import math

import numpy as np
import pytest

from oracle import codec
from oracle import transform as tf
from synth import BASE_SEED, residual_plane, yuv420_residual_frame

from batch_util import Batch
from test_gpu_parity import _check_near_tie_rounding, _psnr_close

pytestmark = pytest.mark.gpu


def A():
    import paper_1606_05562_amd as mod
    return mod


def torch():
    import torch as t
    return t


def _extreme_residual_blocks():
    """Blocks at the ends of the domain: constant -256 and 255, and the sign
    patterns of every pair of rows of T at +-256 / 255 (the largest |Z|, and
    |L| = 512 at q = 8)."""
    t = tf.T
    pats = [np.full((16, 16), -256, np.int16), np.full((16, 16), 255, np.int16)]
    for u in range(16):
        for v in range(0, 16, 3):
            s = np.outer(t[u], t[v])
            pats.append(np.where(s > 0, 255, -256).astype(np.int16))
            pats.append(np.where(s > 0, -256, 255).astype(np.int16))
    n = len(pats) // 8 * 8
    blocks = np.stack(pats[:n])
    return blocks.reshape(n // 8, 8, 16, 16).transpose(0, 2, 1, 3).reshape(n // 8 * 16, 128)


def _images():
    rng = np.random.default_rng(31)
    return [residual_plane(BASE_SEED + 5, 0, 0, 96, 384),          # whole strips
            residual_plane(BASE_SEED + 5, 0, 1, 136, 240),         # ragged strip tail, partial block row
            rng.integers(-256, 256, (33, 47)).astype(np.int16),   # ragged in both directions
            rng.integers(-256, 256, (17, 130)).astype(np.int16),
            rng.integers(-256, 256, (1, 1)).astype(np.int16),
            _extreme_residual_blocks()]


@pytest.fixture(scope="module")
def batch_res():
    return Batch(_images(), 128)


def _check_recon(got, real, im, sse_i, psnr_i, want_rec):
    """Tie rule on the reconstruction, exact SSE of it, and PSNR: that of the
    returned reconstruction, and the oracle's where they agree pixel for
    pixel."""
    h, w = im.shape
    _check_near_tie_rounding(got, real)
    assert int(sse_i) == codec.sse(im, got)
    assert _psnr_close(float(psnr_i), codec.psnr_from_sse(codec.sse(im, got), h * w))
    if np.array_equal(got, want_rec):
        assert _psnr_close(float(psnr_i), codec.psnr_from_sse(codec.sse(im, want_rec), h * w))


def _run(batch, backend, qmode, q, flags=0, levels="i16", out=True):
    T = torch()
    mod = A()
    lv_dt = {"i16": mod.I16, "i32": mod.I32}[levels]
    plan = batch.plan(coef_dtype=mod.I32, qmode=qmode, q=q, qcoef_dtype=lv_dt, out_dtype=mod.I16, backend=backend,
                      flags=flags)
    rec = batch.empty_like_images(np.int16, 77) if out else None
    lv = batch.coef_tensor(T.int16 if levels == "i16" else T.int32)
    sse = T.zeros(len(batch.images), dtype=T.int64, device="cuda")
    psnr = T.zeros(len(batch.images), dtype=T.float64, device="cuda")
    plan.compress_and_measure(batch.dev, rec, lv, sse, psnr)
    T.cuda.synchronize()
    info = json.loads(plan.info())
    return (batch.unpack(rec) if out else None), batch.split_coef(lv), sse.cpu().numpy(), psnr.cpu().numpy(), info


@pytest.mark.parametrize("q", [8, 16, 32, 100])
def test_resid_mfma_uniform_against_oracle(batch_res, q):
    recs, lvs, sse, psnr, info = _run(batch_res, A().BACKEND_MFMA, A().Q_UNIFORM, q, A().FLAG_RESIDUAL_RANGE)
    assert info["levels_backend"] == "mfma" and info["fused_form"] == "fp16-residual-classes"
    for i, (got, lvl, im) in enumerate(zip(recs, lvs, batch_res.images)):
        h, w = im.shape
        want_lv = codec.quantise_uniform(codec.forward_image(im), q)
        assert np.array_equal(lvl.astype(np.int64), want_lv), f"image {i}"
        real = codec.reconstruct_uniform(want_lv, q, h, w, rounded=False)
        want_rec = codec.reconstruct_uniform(want_lv, q, h, w, out_dtype=np.int16)
        _check_recon(got, real, im, sse[i], psnr[i], want_rec)


@pytest.mark.parametrize("strips", [1, 2, 3, 4, 16])
def test_resid_mfma_task_sizes(monkeypatch, batch_res, strips):
    """The task tables (runs of at most 1, 2, 3, 4 or 16 strips)."""
    monkeypatch.setenv("ADCT16_TASK_STRIPS", str(strips))
    recs, lvs, sse, psnr, info = _run(batch_res, A().BACKEND_MFMA, A().Q_UNIFORM, 16, A().FLAG_RESIDUAL_RANGE)
    assert info["levels_backend"] == "mfma" and info["levels_task_strips"] == strips
    for i, (got, lvl, im) in enumerate(zip(recs, lvs, batch_res.images)):
        h, w = im.shape
        want_lv = codec.quantise_uniform(codec.forward_image(im), 16)
        assert np.array_equal(lvl.astype(np.int64), want_lv), f"image {i}"
        real = codec.reconstruct_uniform(want_lv, 16, h, w, rounded=False)
        want_rec = codec.reconstruct_uniform(want_lv, 16, h, w, out_dtype=np.int16)
        _check_recon(got, real, im, sse[i], psnr[i], want_rec)


@pytest.mark.parametrize("qp,inter", [(22, False), (27, True), (32, True), (37, False), (51, True)])
def test_resid_mfma_deadzone_against_oracle(batch_res, qp, inter):
    flags = A().FLAG_RESIDUAL_RANGE | (A().FLAG_DEADZONE_INTER if inter else 0)
    recs, lvs, sse, psnr, info = _run(batch_res, A().BACKEND_MFMA, A().Q_DEADZONE, qp, flags)
    assert info["levels_backend"] == "mfma"
    for i, (got, lvl, im) in enumerate(zip(recs, lvs, batch_res.images)):
        h, w = im.shape
        want_lv = codec.quantise_deadzone(codec.forward_image(im), qp, inter)
        assert np.array_equal(lvl.astype(np.int64), want_lv), f"image {i}"
        real = codec.blocks_to_image(tf.inverse_real(codec.deadzone_step(qp) * want_lv.astype(np.float64)), h, w)
        want_rec = codec.reconstruct_deadzone(want_lv, qp, h, w, out_dtype=np.int16)
        _check_recon(got, real, im, sse[i], psnr[i], want_rec)


@pytest.mark.parametrize("qmode,q", [(3, 8), (3, 16), (3, 32), (4, 22), (4, 37)])
def test_resid_mfma_equals_adder_kernel(batch_res, qmode, q):
    a = _run(batch_res, A().BACKEND_MFMA, qmode, q, A().FLAG_RESIDUAL_RANGE)
    b = _run(batch_res, A().BACKEND_VALU, qmode, q)
    assert a[4]["levels_backend"] == "mfma" and b[4]["levels_backend"] == "valu"
    for i in range(len(batch_res.images)):
        assert np.array_equal(a[1][i], b[1][i]), f"levels of image {i}"
    # two float64 evaluations of the same real numbers: equal except where
    # the value lies within 1e-9 of a tie (the oracle's, from the levels)
    for i, (ga, gb, im) in enumerate(zip(a[0], b[0], batch_res.images)):
        h, w = im.shape
        lv = a[1][i].astype(np.int64)
        real = codec.reconstruct_uniform(lv, q, h, w, rounded=False) if qmode == 3 else codec.blocks_to_image(
            tf.inverse_real(codec.deadzone_step(q) * lv.astype(np.float64)), h, w)
        diff = ga != gb
        assert np.abs(ga.astype(np.int64) - gb.astype(np.int64)).max() <= 1
        assert np.all(np.abs(real - np.floor(real) - 0.5)[diff] < 1e-9), f"image {i}"
        if not diff.any():
            assert abs(a[3][i] - b[3][i]) <= 1e-3 or (math.isinf(a[3][i]) and math.isinf(b[3][i]))


def test_resid_mfma_levels_int32_and_no_output(batch_res):
    q = 16
    a = _run(batch_res, A().BACKEND_MFMA, A().Q_UNIFORM, q, A().FLAG_RESIDUAL_RANGE, levels="i32")
    b = _run(batch_res, A().BACKEND_MFMA, A().Q_UNIFORM, q, A().FLAG_RESIDUAL_RANGE, levels="i16", out=False)
    for i, im in enumerate(batch_res.images):
        want_lv = codec.quantise_uniform(codec.forward_image(im), q)
        assert np.array_equal(a[1][i].astype(np.int64), want_lv) and np.array_equal(b[1][i].astype(np.int64), want_lv)
    assert np.array_equal(a[2], b[2])  # SSE does not depend on writing the reconstruction


def test_resid_mfma_without_levels(batch_res):
    T = torch()
    mod = A()
    plan = batch_res.plan(coef_dtype=mod.I32, qmode=mod.Q_UNIFORM, q=8, out_dtype=mod.I16, backend=mod.BACKEND_MFMA,
                          flags=mod.FLAG_RESIDUAL_RANGE)
    assert json.loads(plan.info())["fused_backend"] == "mfma"
    rec = batch_res.empty_like_images(np.int16)
    sse = T.zeros(len(batch_res.images), dtype=T.int64, device="cuda")
    plan.compress_and_measure(batch_res.dev, rec, None, sse, None)
    T.cuda.synchronize()
    ref = _run(batch_res, mod.BACKEND_MFMA, mod.Q_UNIFORM, 8, mod.FLAG_RESIDUAL_RANGE)
    for got, want in zip(batch_res.unpack(rec), ref[0]):
        assert np.array_equal(got, want)
    assert np.array_equal(sse.cpu().numpy(), ref[2])


def test_resid_out_of_range_is_reported():
    """A sample outside [-256, 255] marks its image (SSE -1, PSNR NaN); the
    other images of the batch are unaffected."""
    rng = np.random.default_rng(5)
    good = residual_plane(BASE_SEED + 5, 3, 0, 64, 256)
    bad = rng.integers(-256, 256, (48, 200)).astype(np.int16)
    bad[17, 33] = 300
    bad2 = rng.integers(-256, 256, (32, 32)).astype(np.int16)
    bad2[31, 31] = -257
    b = Batch([good, bad, bad2], 128)
    recs, lvs, sse, psnr, _ = _run(b, A().BACKEND_MFMA, A().Q_UNIFORM, 16, A().FLAG_RESIDUAL_RANGE)
    assert sse[1] == -1 and math.isnan(psnr[1]) and sse[2] == -1 and math.isnan(psnr[2])
    want_lv = codec.quantise_uniform(codec.forward_image(good), 16)
    assert np.array_equal(lvs[0].astype(np.int64), want_lv)
    assert sse[0] == codec.sse(good, recs[0]) and not math.isnan(psnr[0])


def test_resid_requires_flag_and_step():
    """Without the range flag, or with a step below 8, 16-bit plans keep the
    vector kernel for the fused call."""
    b = Batch([residual_plane(BASE_SEED + 5, 0, 0, 32, 128)], 128)
    mod = A()
    for flags, q in ((0, 16), (mod.FLAG_RESIDUAL_RANGE, 4)):
        plan = b.plan(coef_dtype=mod.I32, qmode=mod.Q_UNIFORM, q=q, qcoef_dtype=mod.I16, out_dtype=mod.I16,
                      backend=mod.BACKEND_MFMA, flags=flags)
        info = json.loads(plan.info())
        assert info["fused_backend"] == "valu" and info["levels_backend"] == "valu"


def test_resid_mfma_needs_32bit_offsets():
    """The matrix-core kernel addresses samples by 32-bit byte offsets from
    the image start: plans whose images reach 2^31 bytes, or whose rows
    reach 2^24 bytes, keep the vector kernel for the fused call (geometry
    only; nothing is launched)."""
    mod = A()
    def levels_backend(h, pitch):
        plan = mod.Plan([h], [64], [pitch], [0], in_dtype=mod.I16, coef_dtype=mod.I32, qmode=mod.Q_UNIFORM, q=16,
                        qcoef_dtype=mod.I16, out_dtype=mod.I16, backend=mod.BACKEND_MFMA,
                        flags=mod.FLAG_RESIDUAL_RANGE)
        return json.loads(plan.info())["levels_backend"]
    assert levels_backend(16, (1 << 23) - 64) == "mfma"    # rows just below 16 MiB
    assert levels_backend(16, 1 << 23) == "valu"           # 16 MiB rows
    assert levels_backend(1023, 1 << 20) == "mfma"         # just below 2 GiB
    assert levels_backend(1024, 1 << 20) == "valu"         # 2 GiB


def test_resid_graph_replays_match_eager():
    T = torch()
    mod = A()
    b = Batch(yuv420_residual_frame(BASE_SEED + 5, 1, 272, 480), 128)
    plan = b.plan(coef_dtype=mod.I32, qmode=mod.Q_UNIFORM, q=16, qcoef_dtype=mod.I16, out_dtype=mod.I16,
                  backend=mod.BACKEND_MFMA, flags=mod.FLAG_RESIDUAL_RANGE)
    n = len(b.images)
    rec, lv = b.empty_like_images(np.int16), b.coef_tensor(T.int16)
    sse, psnr = T.zeros(n, dtype=T.int64, device="cuda"), T.zeros(n, dtype=T.float64, device="cuda")
    plan.compress_and_measure(b.dev, rec, lv, sse, psnr)
    T.cuda.synchronize()
    want = (rec.clone(), lv.clone(), sse.clone(), psnr.clone())
    g = plan.graph(b.dev, rec, lv, sse, psnr)
    for _ in range(3):
        rec.fill_(0)
        lv.fill_(0)
        sse.fill_(0)
        g.launch()
        T.cuda.synchronize()
        assert T.equal(rec, want[0]) and T.equal(lv, want[1]) and T.equal(sse, want[2]) and T.equal(psnr, want[3])


def test_resid_full_frame():
    """One 3840x2160 4:2:0 residual frame (the residual stream's shape):
    the Y plane's levels against the oracle, every level and sample against
    the vector kernel."""
    T = torch()
    mod = A()
    planes = yuv420_residual_frame(BASE_SEED + 5, 0)
    b = Batch(planes, 128)
    a = _run(b, mod.BACKEND_MFMA, mod.Q_UNIFORM, 16, mod.FLAG_RESIDUAL_RANGE)
    v = _run(b, mod.BACKEND_VALU, mod.Q_UNIFORM, 16)
    want_lv = codec.quantise_uniform(codec.forward_image(planes[1]), 16)
    assert np.array_equal(a[1][1].astype(np.int64), want_lv)
    for i in range(3):
        assert np.array_equal(a[1][i], v[1][i])
        h, w = planes[i].shape
        real = codec.reconstruct_uniform(a[1][i].astype(np.int64), 16, h, w, rounded=False)
        diff = a[0][i] != v[0][i]
        assert np.abs(a[0][i].astype(np.int64) - v[0][i].astype(np.int64)).max() <= 1
        assert np.all(np.abs(real - np.floor(real) - 0.5)[diff] < 1e-9)
        assert abs(a[3][i] - v[3][i]) <= 1e-3
