"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only produces input data.  It holds no part of the transform,
the quantiser, the inverse or the quality measures: both the oracle and the
HIP path receive the bytes made here and nothing else.

Workload shapes follow the paper's experiments:

* Section 4 codes 512x512 8-bit grayscale images cut into 16x16 blocks.  The
  image bank itself is not available, so images are drawn from the
  first-order Markov (AR(1)) model that Section 3.2 adopts for natural image
  data (correlation R_ij = rho^|i-j|, rho = 0.95), applied separably along
  rows and columns.
* Section 5.3 embeds the transform in a video coder, where it is applied to
  motion-compensated prediction residuals.  ``residual_frame`` produces such
  residuals from AR(1) frames and per-16x16-block motion vectors.

Every generator takes an explicit seed; frames are derived from
``numpy.random.default_rng([seed, index])`` so that any frame can be
regenerated on its own and in parallel.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

BASE_SEED = 0x16060556


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _ar1_axis0(e: np.ndarray, rho: float) -> np.ndarray:
    """Stationary unit-variance AR(1) recursion down axis 0 of ``e``."""
    c = np.float32(np.sqrt(1.0 - rho * rho))
    r = np.float32(rho)
    x = np.empty_like(e)
    x[0] = e[0]
    for i in range(1, e.shape[0]):
        np.multiply(x[i - 1], r, out=x[i])
        x[i] += c * e[i]
    return x


def ar1_field(rng: np.random.Generator, h: int, w: int, rho: float) -> np.ndarray:
    """Zero-mean, unit-variance separable AR(1) field of shape (h, w), float32."""
    e = rng.standard_normal((h, w), dtype=np.float32)
    x = _ar1_axis0(e, rho)
    x = _ar1_axis0(np.ascontiguousarray(x.T), rho)
    return np.ascontiguousarray(x.T)


def _to_u8(x: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(x), 0, 255).astype(np.uint8)


def ar1_image(seed: int, h: int = 512, w: int = 512, rho: float = 0.95,
              sigma: float = 40.0, mean: float = 128.0) -> np.ndarray:
    """One uint8 image: mean + sigma * AR(1) field, rounded and clipped."""
    rng = np.random.default_rng([seed, 0])
    return _to_u8(mean + sigma * ar1_field(rng, h, w, rho))


def _rect_params(seed: int, h: int, w: int, count: int = 8, side: int = 64):
    rng = np.random.default_rng([seed, 0x7EC7])
    y0 = rng.integers(0, max(1, h - side), count)
    x0 = rng.integers(0, max(1, w - side), count)
    vy = rng.integers(-6, 7, count)
    vx = rng.integers(-6, 7, count)
    level = rng.integers(0, 256, count)
    return y0, x0, vy, vx, level


def luma_frame(seed: int, t: int, h: int = 1088, w: int = 1920,
               rho: float = 0.95, sigma: float = 40.0, mean: float = 128.0,
               n_rect: int = 8, side: int = 64) -> np.ndarray:
    """Frame ``t`` of a luma sequence: an AR(1) field plus ``n_rect``
    piecewise-constant side x side rectangles that translate from frame to
    frame (constant per-rectangle velocity, wrapping at the borders)."""
    rng = np.random.default_rng([seed, 1 + t])
    f = mean + sigma * ar1_field(rng, h, w, rho)
    y0, x0, vy, vx, level = _rect_params(seed, h, w, n_rect, side)
    for k in range(n_rect):
        yy = int(y0[k] + vy[k] * t) % max(1, h - side)
        xx = int(x0[k] + vx[k] * t) % max(1, w - side)
        f[yy:yy + side, xx:xx + side] = level[k]
    return _to_u8(f)


def luma_batch(seed: int, n: int, h: int = 1088, w: int = 1920,
               out: np.ndarray | None = None) -> np.ndarray:
    """``n`` frames from ``luma_frame`` stacked into an (n, h, w) uint8 array."""
    if out is None:
        out = np.empty((n, h, w), dtype=np.uint8)

    def one(t):
        out[t] = luma_frame(seed, t, h, w)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(one, range(n)))
    return out


def ragged_sizes(seed: int, n: int = 64, lo: int = 64, hi: int = 3840,
                 multiple: int = 16) -> list[tuple[int, int]]:
    """Image sizes with each side uniform in [lo, hi], rounded up to
    ``multiple`` (``multiple=1`` leaves them unrounded)."""
    rng = np.random.default_rng([seed, 0x5E5])
    hw = rng.integers(lo, hi + 1, size=(n, 2))
    if multiple > 1:
        hw = (hw + multiple - 1) // multiple * multiple
    return [(int(a), int(b)) for a, b in hw]


def _voronoi(rng: np.random.Generator, h: int, w: int, cells: int = 32) -> np.ndarray:
    cy = rng.uniform(0, h, cells)
    cx = rng.uniform(0, w, cells)
    lv = rng.integers(0, 256, cells).astype(np.uint8)
    out = np.empty((h, w), dtype=np.uint8)
    xs = np.arange(w, dtype=np.float32)
    band = 64
    for y in range(0, h, band):
        ys = np.arange(y, min(h, y + band), dtype=np.float32)
        d = (ys[:, None, None] - cy[None, None, :]) ** 2 + (xs[None, :, None] - cx[None, None, :]) ** 2
        out[y:y + len(ys)] = lv[np.argmin(d, axis=2)]
    return out


def mixed_image(seed: int, k: int, h: int, w: int) -> np.ndarray:
    """Image ``k`` of a ragged batch.  The content class is drawn per image:
    40% AR(1) with rho ~ U[0.85, 0.98], 30% Gaussian noise sigma=20 around
    128, 30% Voronoi regions with 32 cells of uniform grey level."""
    rng = np.random.default_rng([seed, 100 + k])
    u = rng.uniform()
    if u < 0.4:
        rho = rng.uniform(0.85, 0.98)
        return _to_u8(128.0 + 40.0 * ar1_field(rng, h, w, rho))
    if u < 0.7:
        return _to_u8(128.0 + 20.0 * rng.standard_normal((h, w), dtype=np.float32))
    return _voronoi(rng, h, w, 32)


def ragged_batch(seed: int, n: int = 64, lo: int = 64, hi: int = 3840,
                 multiple: int = 16) -> list[np.ndarray]:
    sizes = ragged_sizes(seed, n, lo, hi, multiple)
    with ThreadPoolExecutor(_threads()) as ex:
        return list(ex.map(lambda kv: mixed_image(seed, kv[0], *kv[1]), enumerate(sizes)))


def residual_plane(seed: int, t: int, plane: int, h: int, w: int,
                   max_mv: int = 8, rho: float = 0.95) -> np.ndarray:
    """int16 residual F_t - MC(F_{t-1}) for one plane, values in [-255, 255].

    F_t and F_{t-1} are independent AR(1) uint8 frames (sigma 40, mean 128);
    MC shifts every 16x16 block of F_{t-1} by its own motion vector, uniform
    in [-max_mv, max_mv]^2, clamping source coordinates at the borders."""
    f_prev = _to_u8(128.0 + 40.0 * ar1_field(np.random.default_rng([seed, 7, plane, t]), h, w, rho))
    f_cur = _to_u8(128.0 + 40.0 * ar1_field(np.random.default_rng([seed, 7, plane, t + 1]), h, w, rho))
    rng = np.random.default_rng([seed, 9, plane, t])
    by, bx = (h + 15) // 16, (w + 15) // 16
    mv = rng.integers(-max_mv, max_mv + 1, size=(by, bx, 2))
    yy = np.arange(h)[:, None]
    xx = np.arange(w)[None, :]
    dy = np.repeat(np.repeat(mv[:, :, 0], 16, 0), 16, 1)[:h, :w]
    dx = np.repeat(np.repeat(mv[:, :, 1], 16, 0), 16, 1)[:h, :w]
    sy = np.clip(yy + dy, 0, h - 1)
    sx = np.clip(xx + dx, 0, w - 1)
    pred = f_prev[sy, sx]
    return (f_cur.astype(np.int16) - pred.astype(np.int16))


def yuv420_residual_frame(seed: int, t: int, h: int = 2160, w: int = 3840,
                          chroma_pad_to: int = 16) -> list[np.ndarray]:
    """Y, U, V residual planes of one 4:2:0 frame.  Chroma planes are
    (h/2, w/2); their true size is kept (padding, if any, is the library's
    business)."""
    y = residual_plane(seed, t, 0, h, w)
    u = residual_plane(seed, t, 1, h // 2, w // 2)
    v = residual_plane(seed, t, 2, h // 2, w // 2)
    return [y, u, v]


def random_blocks_u8(seed: int, n: int) -> np.ndarray:
    """n uniformly random 16x16 uint8 blocks (worst-case texture)."""
    return np.random.default_rng([seed, 0xB10C]).integers(0, 256, size=(n, 16, 16), dtype=np.uint8)


def pack_images(images: list[np.ndarray], align_elems: int = 16,
                pitch_multiple: int = 16) -> tuple[np.ndarray, list[int], list[int], list[int], list[int]]:
    """Pack 2-D images of one dtype into one flat buffer.

    Returns (buffer, heights, widths, pitches, offsets).  Each row pitch is
    the width rounded up to ``pitch_multiple`` elements and each image starts
    at an element offset that is a multiple of ``align_elems``; padding
    columns are filled by repeating each row's last pixel so that the buffer
    is fully initialised."""
    dt = images[0].dtype
    hs, ws, ps, offs = [], [], [], []
    total = 0
    for im in images:
        h, w = im.shape
        p = (w + pitch_multiple - 1) // pitch_multiple * pitch_multiple
        total = (total + align_elems - 1) // align_elems * align_elems
        hs.append(h); ws.append(w); ps.append(p); offs.append(total)
        total += h * p
    total = (total + align_elems - 1) // align_elems * align_elems
    buf = np.zeros(total, dtype=dt)
    for im, h, w, p, o in zip(images, hs, ws, ps, offs):
        v = buf[o:o + h * p].reshape(h, p)
        v[:, :w] = im
        if p > w:
            v[:, w:] = im[:, w - 1:w]
    return buf, hs, ws, ps, offs
