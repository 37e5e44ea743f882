"""Image-level pieces of the compression experiment of Section 4 (oracle;
test infrastructure only).

Readings taken where the paper is silent (each listed in the design notes):
* Images whose sides are not multiples of 16 are extended by repeating the
  last row/column before blocking; measures use only the true pixels.
* Blocks are numbered in raster order; within a block, index u (rows of T
  applied down the columns) is the vertical frequency and v the horizontal
  one: Z[u, v] = sum_a sum_b T[u, a] A[a, b] T[v, b].
* The reconstruction is rounded half up, floor(A' + 1/2), then clamped to
  [0, 255] for 8-bit images or saturated to int16 for residual planes.
* PSNR uses peak 255 for both 8-bit images and residual planes, is computed
  per image over its h*w true pixels, and is +inf when the SSE is 0.
* The uniform quantiser folds S into one float32 multiplier per coefficient
  (Section 2 says S can be absorbed into the quantisation step without
  fixing how): M_uv = fl32(1 / (sqrt(n_u n_v) q)),
  L_uv = round_half_even(fl32(fl32(Z_uv) * M_uv)).  Dequantisation gives
  B'_uv = q L_uv in the orthonormal domain.
"""
from __future__ import annotations

import math

import numpy as np

from . import transform as tf

BLK = 16


# ----------------------------------------------------------------------------
# Blocking (Section 4: 16x16 disjoint blocks).

def grid(h: int, w: int) -> tuple[int, int]:
    return (h + BLK - 1) // BLK, (w + BLK - 1) // BLK


def image_to_blocks(img: np.ndarray) -> np.ndarray:
    """(h, w) image -> (nblocks, 16, 16) blocks in raster order, edge-extended."""
    h, w = img.shape
    by, bx = grid(h, w)
    ext = np.pad(img, ((0, by * BLK - h), (0, bx * BLK - w)), mode="edge")
    return ext.reshape(by, BLK, bx, BLK).transpose(0, 2, 1, 3).reshape(by * bx, BLK, BLK)


def blocks_to_image(blocks: np.ndarray, h: int, w: int) -> np.ndarray:
    by, bx = grid(h, w)
    full = np.asarray(blocks).reshape(by, bx, BLK, BLK).transpose(0, 2, 1, 3).reshape(by * BLK, bx * BLK)
    return full[:h, :w]


# ----------------------------------------------------------------------------
# Retention masks (Section 4 keeps the first r coefficients in zig-zag order).

def mask_none() -> np.ndarray:
    return np.ones((BLK, BLK), dtype=bool)


def mask_zonal(r: int) -> np.ndarray:
    """Keep the top-left r x r square of coefficients."""
    m = np.zeros((BLK, BLK), dtype=bool)
    m[:r, :r] = True
    return m


def zigzag_order(n: int = BLK) -> list[tuple[int, int]]:
    """Zig-zag scan of an n x n block, extended from the 8x8 JPEG scan:
    anti-diagonals d = u + v in increasing order; odd d are walked with the
    row index increasing, even d with it decreasing, so the scan begins
    (0,0), (0,1), (1,0), (2,0), (1,1), (0,2), ..."""
    order = []
    for d in range(2 * n - 1):
        rows = range(max(0, d - n + 1), min(d, n - 1) + 1)
        if d % 2 == 0:
            rows = reversed(rows)
        order.extend((u, d - u) for u in rows)
    return order


def mask_zigzag(r: int) -> np.ndarray:
    """Keep the first r coefficients of the zig-zag scan (1 <= r <= 256)."""
    m = np.zeros((BLK, BLK), dtype=bool)
    for u, v in zigzag_order()[:r]:
        m[u, v] = True
    return m


# ----------------------------------------------------------------------------
# Uniform quantiser with S folded in (float32 decision, see module notes).

def uniform_multipliers(q: int, t: np.ndarray = tf.T) -> np.ndarray:
    n = tf.row_norms(t)
    m = np.empty((BLK, BLK), dtype=np.float32)
    for u in range(BLK):
        for v in range(BLK):
            m[u, v] = np.float32(1.0 / (math.sqrt(float(n[u] * n[v])) * float(q)))
    return m


def quantise_uniform(z: np.ndarray, q: int, t: np.ndarray = tf.T) -> np.ndarray:
    zf = np.asarray(z).astype(np.float32)
    prod = (zf * uniform_multipliers(q, t)).astype(np.float32)
    return np.rint(prod).astype(np.int64)


def quantise_uniform_ideal(z: np.ndarray, q: int) -> np.ndarray:
    """round(B / q) in float64 (diagnostic only: the ideal levels)."""
    return np.rint(tf.scale(z) / float(q)).astype(np.int64)


def dequantise_uniform(levels: np.ndarray, q: int) -> np.ndarray:
    return float(q) * np.asarray(levels, dtype=np.float64)


# ----------------------------------------------------------------------------
# Deadzone quantiser with a QP-scaled step.  The paper embeds the transform in
# a video coder (Section 5.3) without giving that coder's quantiser; this is
# the usual form of one: six steps per doubling given by integer scales,
# S folded into one float32 multiplier per coefficient, a rounding offset f
# below 1/2 (the dead zone), and a matching reconstruction step.

QUANT_SCALE = (26214, 23302, 20560, 18396, 16384, 14564)
DEQUANT_SCALE = (40, 45, 51, 57, 64, 72)


def deadzone_multipliers(qp: int) -> np.ndarray:
    """M_uv = fl32(Q[qp mod 6] / (sqrt(n_u n_v) 2^(14 + qp // 6)))."""
    n = tf.row_norms()
    m = np.empty((BLK, BLK), dtype=np.float32)
    for u in range(BLK):
        for v in range(BLK):
            m[u, v] = np.float32(math.ldexp(QUANT_SCALE[qp % 6] / math.sqrt(float(n[u] * n[v])), -(14 + qp // 6)))
    return m


def deadzone_offset(inter: bool = False) -> np.float32:
    return np.float32(1.0 / 6.0) if inter else np.float32(1.0 / 3.0)


def quantise_deadzone(z: np.ndarray, qp: int, inter: bool = False) -> np.ndarray:
    """L = sign(Z) floor(fl32(fl32(fl32(|Z|) M) + f)), float32 multiply and
    add each rounded on its own."""
    z = np.asarray(z)
    a = (np.abs(z).astype(np.float32) * deadzone_multipliers(qp)).astype(np.float32)
    b = (a + deadzone_offset(inter)).astype(np.float32)
    return (np.sign(z) * np.floor(b)).astype(np.int64)


def deadzone_step(qp: int) -> float:
    """Reconstruction step D[qp mod 6] 2^(qp // 6) / 64 (exact in float64)."""
    return math.ldexp(float(DEQUANT_SCALE[qp % 6]), qp // 6 - 6)


def reconstruct_deadzone(levels: np.ndarray, qp: int, h: int, w: int, out_dtype=np.uint8) -> np.ndarray:
    a = tf.inverse_real(deadzone_step(qp) * np.asarray(levels, dtype=np.float64))
    rec = round_half_up_u8(a) if out_dtype == np.uint8 else round_half_up_i16(a)
    return blocks_to_image(rec, h, w)


def compress_deadzone(img: np.ndarray, qp: int, inter: bool = False):
    """Forward, deadzone quantiser, inverse, measure: (levels, recon, sse, psnr)."""
    h, w = img.shape
    lv = quantise_deadzone(forward_image(img), qp, inter)
    rec = reconstruct_deadzone(lv, qp, h, w, np.uint8 if img.dtype == np.uint8 else np.int16)
    s = sse(img, rec)
    return lv, rec, s, psnr_from_sse(s, h * w)


def se_code_length(v: int) -> int:
    """Bits of the signed Exp-Golomb code se(v): code number k = 2v - 1 for
    v > 0 and -2v otherwise, written as k + 1 in binary preceded by as many
    zeros as it has bits after the leading one."""
    k = 2 * v - 1 if v > 0 else -2 * v
    return 2 * ((k + 1).bit_length() - 1) + 1


def rate_bits(levels: np.ndarray) -> int:
    """Rate proxy: total se(v) length of the levels."""
    vals, counts = np.unique(np.asarray(levels, dtype=np.int64), return_counts=True)
    return int(sum(se_code_length(int(v)) * int(c) for v, c in zip(vals, counts)))


# ----------------------------------------------------------------------------
# Reconstruction rounding.

def round_half_up_u8(a: np.ndarray) -> np.ndarray:
    return np.clip(np.floor(np.asarray(a, dtype=np.float64) + 0.5), 0, 255).astype(np.uint8)


def round_half_up_i16(a: np.ndarray) -> np.ndarray:
    return np.clip(np.floor(np.asarray(a, dtype=np.float64) + 0.5), -32768, 32767).astype(np.int16)


def int_recon_u8(numerator: np.ndarray) -> np.ndarray:
    """floor(N/2304 + 1/2) clamped to [0, 255], in exact integer arithmetic."""
    return np.clip(np.floor_divide(np.asarray(numerator, dtype=np.int64) + 1152, 2304), 0, 255).astype(np.uint8)


def int_recon_i16(numerator: np.ndarray) -> np.ndarray:
    return np.clip(np.floor_divide(np.asarray(numerator, dtype=np.int64) + 1152, 2304),
                   -32768, 32767).astype(np.int16)


# ----------------------------------------------------------------------------
# Quality measures (Section 4).

def sse(a: np.ndarray, b: np.ndarray) -> int:
    d = np.asarray(a, dtype=np.int64) - np.asarray(b, dtype=np.int64)
    return int(np.sum(d * d))


def psnr_from_sse(s: int, npix: int, peak: float = 255.0) -> float:
    if s == 0:
        return math.inf
    return 10.0 * math.log10(peak * peak * npix / s)


def psnr(a: np.ndarray, b: np.ndarray, peak: float = 255.0) -> float:
    return psnr_from_sse(sse(a, b), np.asarray(a).size, peak)


def ape(x: float, ref: float) -> float:
    """Absolute percentage error 100 |x - ref| / |ref| (Section 4)."""
    return 100.0 * abs(x - ref) / abs(ref)


def _gauss_window(size: int = 11, sigma: float = 1.5) -> np.ndarray:
    ax = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-(ax[:, None] ** 2 + ax[None, :] ** 2) / (2.0 * sigma * sigma))
    return g / g.sum()


def _local_moments(x: np.ndarray, y: np.ndarray, g: np.ndarray):
    """Weighted means, variances and covariance of x and y over every window
    position fully inside the image (population moments: E[xy] - E[x]E[y]
    under the normalised window weights)."""
    from scipy.signal import correlate2d

    def f(z):
        return correlate2d(z, g, mode="valid")

    mx, my = f(x), f(y)
    return mx, my, f(x * x) - mx * mx, f(y * y) - my * my, f(x * y) - mx * my


def ssim(a: np.ndarray, b: np.ndarray, peak: float = 255.0) -> float:
    """Mean SSIM index of Wang, Bovik, Sheikh and Simoncelli (the measure
    Section 4 cites): 11x11 Gaussian window (sigma 1.5), K1 = 0.01,
    K2 = 0.03, statistics over every window position fully inside the image.
    The paper prints no SSIM of an image available here; the window, sigma
    and population moments are pinned by closed forms (checkerboards against
    flat and against other checkerboards) and by brute force on an 11x11
    image."""
    x = np.asarray(a, dtype=np.float64)
    y = np.asarray(b, dtype=np.float64)
    c1 = (0.01 * peak) ** 2
    c2 = (0.03 * peak) ** 2
    mx, my, sxx, syy, sxy = _local_moments(x, y, _gauss_window())
    m = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    return float(m.mean())


# ----------------------------------------------------------------------------
# The compression experiment of Section 4, per image.

def forward_image(img: np.ndarray, t: np.ndarray = tf.T) -> np.ndarray:
    """Integer coefficients Z of every block, (nblocks, 16, 16) int64."""
    return tf.forward_int(image_to_blocks(img), t)


def reconstruct_kept(z: np.ndarray, keep: np.ndarray, h: int, w: int, out_dtype=np.uint8,
                     t: np.ndarray = tf.T) -> np.ndarray:
    """Zero the coefficients outside ``keep`` and invert exactly."""
    zk = np.where(keep[None, :, :], z, 0)
    num = tf.inverse_int_numerator(zk, t)
    rec = int_recon_u8(num) if out_dtype == np.uint8 else int_recon_i16(num)
    return blocks_to_image(rec, h, w)


def reconstruct_uniform(levels: np.ndarray, q: int, h: int, w: int, out_dtype=np.uint8,
                        rounded: bool = True, t: np.ndarray = tf.T) -> np.ndarray:
    a = tf.inverse_real(dequantise_uniform(levels, q), t)
    if not rounded:
        return blocks_to_image(a, h, w)
    rec = round_half_up_u8(a) if out_dtype == np.uint8 else round_half_up_i16(a)
    return blocks_to_image(rec, h, w)


def compress_kept(img: np.ndarray, keep: np.ndarray, t: np.ndarray = tf.T):
    """Forward, retain ``keep``, inverse, measure: (recon, sse, psnr)."""
    h, w = img.shape
    rec = reconstruct_kept(forward_image(img, t), keep, h, w,
                           np.uint8 if img.dtype == np.uint8 else np.int16, t)
    s = sse(img, rec)
    return rec, s, psnr_from_sse(s, h * w)


def compress_uniform(img: np.ndarray, q: int, t: np.ndarray = tf.T):
    """Forward, uniform quantiser, inverse, measure: (levels, recon, sse, psnr)."""
    h, w = img.shape
    lv = quantise_uniform(forward_image(img, t), q, t)
    rec = reconstruct_uniform(lv, q, h, w, np.uint8 if img.dtype == np.uint8 else np.int16, t=t)
    s = sse(img, rec)
    return lv, rec, s, psnr_from_sse(s, h * w)


def compress_dct_kept(img: np.ndarray, keep: np.ndarray):
    """Same experiment with the exact DCT-II (comparison transform):
    returns (rounded recon, psnr)."""
    h, w = img.shape
    b = tf.dct_forward(image_to_blocks(img))
    a = tf.dct_inverse(np.where(keep[None], b, 0.0))
    rec = blocks_to_image(round_half_up_u8(a), h, w)
    return rec, psnr(img, rec)
