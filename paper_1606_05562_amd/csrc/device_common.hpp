// Device building blocks: the 16-point butterflies of Eq. (1), the LDS
// transposition buffer between the row and column passes, and the strip
// scheduler shared by the persistent kernels.
#pragma once

#include "adct16_internal.hpp"

namespace adct16 {

typedef unsigned short us2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// y = T x by the factorisation T = P2 M4 M3 M2 P1 M1 of Eq. (1): 16 + 16 +
// 24 + 4 additions, the permutations P1 and P2 being register renames.
// T is any type with + and - : packed 2 x uint16 (modular arithmetic, exact
// whenever the true result's range is known), int32 or float64.
template <class T>
__device__ __forceinline__ void t_fwd(T (&x)[16]) {
  T y[16];
#pragma unroll
  for (int k = 0; k < 8; ++k) {  // M1 = [[I, J], [J, -I]]
    y[k] = x[k] + x[15 - k];
    y[8 + k] = x[7 - k] - x[8 + k];
  }
  // P1 keeps 0..8 and reorders 9..15.
  T z[16] = {y[0], y[1], y[2], y[3], y[4], y[5], y[6], y[7], y[8],
             y[11], y[12], y[15], y[14], y[13], y[10], y[9]};
  T u[16];
#pragma unroll
  for (int o = 0; o < 16; o += 8) {  // M2: two 8-point butterflies
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      u[o + k] = z[o + k] + z[o + 7 - k];
      u[o + 4 + k] = z[o + 3 - k] - z[o + 4 + k];
    }
  }
  T v[16];  // M3: four 4x4 blocks
  v[0] = u[0] + u[3];
  v[1] = u[1] + u[2];
  v[2] = u[2] - u[1];
  v[3] = u[0] - u[3];
  v[4] = u[5] + u[6] + u[7];
  v[5] = u[7] - u[4] - u[5];
  v[6] = u[5] - u[4] - u[6];
  v[7] = u[4] - u[6] + u[7];
  v[8] = u[8] + u[11];
  v[9] = u[9] + u[10];
  v[10] = u[10] - u[9];
  v[11] = u[11] - u[8];
  v[12] = u[13] + u[14] + u[15];
  v[13] = u[12] + u[13] - u[15];
  v[14] = u[12] - u[13] + u[14];
  v[15] = u[12] - u[14] + u[15];
  // M4 on (0,1) and (8,9), then P2: output i is stage-4 value sigma(i),
  // sigma = [0,8,4,11,3,9,5,12,1,13,7,10,2,14,6,15].
  const T w0 = v[0] + v[1], w1 = v[0] - v[1], w8 = v[8] + v[9], w9 = v[8] - v[9];
  x[0] = w0;    x[1] = w8;    x[2] = v[4];  x[3] = v[11];
  x[4] = v[3];  x[5] = w9;    x[6] = v[5];  x[7] = v[12];
  x[8] = w1;    x[9] = v[13]; x[10] = v[7]; x[11] = v[10];
  x[12] = v[2]; x[13] = v[14]; x[14] = v[6]; x[15] = v[15];
}

// y = T^T x = M1^T P1^T M2^T M3^T M4^T P2^T x (M1, M2, M4 are symmetric):
// also 60 additions.
template <class T>
__device__ __forceinline__ void t_inv(T (&x)[16]) {
  // P2^T: stage-4 value sigma(i) = x[i]
  T w[16];
  w[0] = x[0];  w[8] = x[1];  w[4] = x[2];  w[11] = x[3];
  w[3] = x[4];  w[9] = x[5];  w[5] = x[6];  w[12] = x[7];
  w[1] = x[8];  w[13] = x[9]; w[7] = x[10]; w[10] = x[11];
  w[2] = x[12]; w[14] = x[13]; w[6] = x[14]; w[15] = x[15];
  T v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = w[k];
  v[0] = w[0] + w[1];  // M4
  v[1] = w[0] - w[1];
  v[8] = w[8] + w[9];
  v[9] = w[8] - w[9];
  T u[16];  // M3^T
  u[0] = v[0] + v[3];
  u[1] = v[1] - v[2];
  u[2] = v[1] + v[2];
  u[3] = v[0] - v[3];
  u[4] = v[7] - v[5] - v[6];
  u[5] = v[4] - v[5] + v[6];
  u[6] = v[4] - v[6] - v[7];
  u[7] = v[4] + v[5] + v[7];
  u[8] = v[8] - v[11];
  u[9] = v[9] - v[10];
  u[10] = v[9] + v[10];
  u[11] = v[8] + v[11];
  u[12] = v[13] + v[14] + v[15];
  u[13] = v[12] + v[13] - v[14];
  u[14] = v[12] + v[14] - v[15];
  u[15] = v[12] - v[13] + v[15];
  T z[16];
#pragma unroll
  for (int o = 0; o < 16; o += 8) {  // M2
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      z[o + k] = u[o + k] + u[o + 7 - k];
      z[o + 4 + k] = u[o + 3 - k] - u[o + 4 + k];
    }
  }
  // P1^T
  T y[16] = {z[0], z[1], z[2], z[3], z[4], z[5], z[6], z[7], z[8],
             z[15], z[14], z[9], z[10], z[13], z[12], z[11]};
#pragma unroll
  for (int k = 0; k < 8; ++k) {  // M1
    x[k] = y[k] + y[15 - k];
    x[8 + k] = y[7 - k] - y[8 + k];
  }
}

// The Walsh-Hadamard transform in natural (Sylvester) order, y = H x, by
// four radix-2 stages (64 additions); H is symmetric, so it is its own
// inverse pass (H^T = H).
template <class T>
__device__ __forceinline__ void wht_fwd(T (&x)[16]) {
#pragma unroll
  for (int len = 1; len < 16; len <<= 1) {
#pragma unroll
    for (int i = 0; i < 16; i += 2 * len) {
#pragma unroll
      for (int j = 0; j < len; ++j) {
        const T a = x[i + j], b = x[i + j + len];
        x[i + j] = a + b;
        x[i + j + len] = a - b;
      }
    }
  }
}


template <int MAT, class T>
__device__ __forceinline__ void m_fwd(T (&x)[16]) {
  if constexpr (MAT == MAT_WHT) wht_fwd(x); else t_fwd(x);
}

template <int MAT, class T>
__device__ __forceinline__ void m_inv(T (&x)[16]) {
  if constexpr (MAT == MAT_WHT) wht_fwd(x); else t_inv(x);
}

// ---------------------------------------------------------------------------
// Transposition buffer (Section 5.1's row-parallel transpose, in LDS).
// Each wavefront owns 4 slots of 16 x 16 dwords, one per lane group p.
// Element (i, c) of slot s sits at s * kSlot + i * kRow + c; the padding
// makes both the row accesses
// (4 x 16-byte per lane) and the column accesses (16 x 4-byte per lane)
// bank-conflict free for a wavefront laid out as lane = 16 * p + x.
constexpr int kRow = 20;
constexpr int kSlot = 16 * kRow + 16;
constexpr int kWaveLds = 4 * kSlot;  // dwords per wavefront (slot p = lanes 16p..16p+15)

// Orders this wavefront's LDS accesses (all lanes) at this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T>
__device__ __forceinline__ void lds_put_row(int* lds, int slot, int x, const T (&r)[16]) {
  static_assert(sizeof(T) == 4, "32-bit elements");
  int4* p = reinterpret_cast<int4*>(lds + slot * kSlot + x * kRow);
  const int* ri = reinterpret_cast<const int*>(r);
#pragma unroll
  for (int m = 0; m < 4; ++m) p[m] = make_int4(ri[4 * m], ri[4 * m + 1], ri[4 * m + 2], ri[4 * m + 3]);
}

template <class T>
__device__ __forceinline__ void lds_get_row(const int* lds, int slot, int x, T (&r)[16]) {
  static_assert(sizeof(T) == 4, "32-bit elements");
  const int4* p = reinterpret_cast<const int4*>(lds + slot * kSlot + x * kRow);
  int* ri = reinterpret_cast<int*>(r);
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    int4 q = p[m];
    ri[4 * m] = q.x; ri[4 * m + 1] = q.y; ri[4 * m + 2] = q.z; ri[4 * m + 3] = q.w;
  }
}

template <class T>
__device__ __forceinline__ void lds_put_col(int* lds, int slot, int x, const T (&c)[16]) {
  static_assert(sizeof(T) == 4, "32-bit elements");
  const int* ci = reinterpret_cast<const int*>(c);
#pragma unroll
  for (int i = 0; i < 16; ++i) lds[slot * kSlot + i * kRow + x] = ci[i];
}

template <class T>
__device__ __forceinline__ void lds_get_col(const int* lds, int slot, int x, T (&c)[16]) {
  static_assert(sizeof(T) == 4, "32-bit elements");
  int* ci = reinterpret_cast<int*>(c);
#pragma unroll
  for (int i = 0; i < 16; ++i) ci[i] = lds[slot * kSlot + i * kRow + x];
}

// Rows -> columns of one slot: lane x holds row x before, column x after.
template <class T>
__device__ __forceinline__ void transpose_rows_to_cols(int* lds, int slot, int x, T (&v)[16]) {
  lds_put_row(lds, slot, x, v);
  wave_lds_sync();
  lds_get_col(lds, slot, x, v);
  wave_lds_sync();
}

template <class T>
__device__ __forceinline__ void transpose_cols_to_rows(int* lds, int slot, int x, T (&v)[16]) {
  lds_put_col(lds, slot, x, v);
  wave_lds_sync();
  lds_get_row(lds, slot, x, v);
  wave_lds_sync();
}

// float64 through the 32-bit buffer: low and high words in turn.
__device__ __forceinline__ void transpose_cols_to_rows_f64(int* lds, int slot, int x, double (&v)[16]) {
  int lo[16], hi[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    unsigned long long b = __double_as_longlong(v[i]);
    lo[i] = (int)(unsigned)b;
    hi[i] = (int)(unsigned)(b >> 32);
  }
  transpose_cols_to_rows(lds, slot, x, lo);
  transpose_cols_to_rows(lds, slot, x, hi);
#pragma unroll
  for (int i = 0; i < 16; ++i)
    v[i] = __longlong_as_double((long long)(((unsigned long long)(unsigned)hi[i] << 32) | (unsigned)lo[i]));
}

// ---------------------------------------------------------------------------
// Strip scheduling.  Wavefront g of G takes strips [g*S/G, (g+1)*S/G): equal
// shares of equal-area work, contiguous in memory.  The image containing
// the first strip is found by binary search; later strips advance it.
struct StripCursor {
  int64_t s, s_end;
  int img;
  int32_t sy, sxi;       // block-row index and strip index within the row
  ImageDesc d;
};

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffff));
  int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return ((int64_t)hi << 32) | (unsigned)lo;
}

__device__ __forceinline__ ImageDesc load_desc(const ImageDesc* images, int i) {
  ImageDesc d = images[i];
  d.offset = uniform_i64(d.offset);
  d.block_begin = uniform_i64(d.block_begin);
  d.strip_begin = uniform_i64(d.strip_begin);
  d.h = uniform_int(d.h); d.w = uniform_int(d.w); d.pitch = uniform_int(d.pitch);
  d.bx = uniform_int(d.bx); d.by = uniform_int(d.by); d.sx = uniform_int(d.sx);
  return d;
}

// The hardware hands workgroup b to XCD b mod 8.  When the grid is a
// multiple of 8, workgroup b takes slot (b mod 8) (G / 8) + b / 8 (a
// bijection), so that each XCD works through one contiguous eighth of the
// strips instead of every eighth group of four waves.
__device__ __forceinline__ int xcd_slot(int b, int G) {
  return (G & 7) ? b : (b & 7) * (G >> 3) + (b >> 3);
}

__device__ __forceinline__ bool cursor_init(StripCursor& c, const Params& P) {
  const int wave = uniform_int(threadIdx.x >> 6);
  const int64_t g = (int64_t)xcd_slot(blockIdx.x, gridDim.x) * kWavesPerGroup + wave;
  const int64_t G = (int64_t)gridDim.x * kWavesPerGroup;
  c.s = P.n_strips * g / G;
  c.s_end = P.n_strips * (g + 1) / G;
  if (c.s >= c.s_end) return false;
  int lo = 0, hi = P.n_images - 1;  // last image with strip_begin <= s
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (uniform_i64(P.images[mid].strip_begin) <= c.s) lo = mid; else hi = mid - 1;
  }
  c.img = uniform_int(lo);
  c.d = load_desc(P.images, c.img);
  const int64_t local = c.s - c.d.strip_begin;
  c.sy = (int32_t)(local / c.d.sx);
  c.sxi = (int32_t)(local - (int64_t)c.sy * c.d.sx);
  return true;
}

// Advance to the next strip; returns true when the image changed.
__device__ __forceinline__ bool cursor_next(StripCursor& c, const Params& P) {
  ++c.s;
  if (c.s >= c.s_end) return false;
  if (++c.sxi == c.d.sx) {
    c.sxi = 0;
    if (++c.sy == c.d.by) {
      c.sy = 0;
      ++c.img;
      c.d = load_desc(P.images, c.img);
      return true;
    }
  }
  return false;
}

// ---------------------------------------------------------------------------
// Wave reductions and small helpers.
// Sum of a 32-bit value over the 64 lanes with DPP row shifts and row
// broadcasts (no LDS traffic); the total is returned uniform.
__device__ __forceinline__ unsigned wave_sum_u32(unsigned v) {
  v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, false);  // row_shr:8 (lane 15 of a row: row sum)
  v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
  v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
  return __builtin_amdgcn_readlane(v, 63);
}

// Sum of a 64-bit value over the 64 lanes, modulo 2^64 like the plain sum:
// its 24-, 24- and 16-bit digits are summed separately (64 digits of 24 bits
// stay below 2^30, so no digit sum carries out of 32 bits) and recombined
// in scalars.  Three DPP reductions instead of six rounds of lane exchange
// through LDS.
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  const unsigned long long d0 = wave_sum_u32((unsigned)v & 0xFFFFFFu);
  const unsigned long long d1 = wave_sum_u32((unsigned)(v >> 24) & 0xFFFFFFu);
  const unsigned long long d2 = wave_sum_u32((unsigned)(v >> 48));
  return d0 + (d1 << 24) + (d2 << 48);
}

// SSE and PSNR of image blockIdx.x from its task partials (a workgroup of
// kFinishThreads threads, four loads in flight per thread): 32-bit
// partials, or 64-bit ones (WIDE) where ~0 marks a task that saw a sample
// outside the kernel's domain (SSE -1, PSNR NaN).
constexpr int kFinishThreads = 256;

template <bool WIDE>
__device__ __forceinline__ void finish_image(const Params& P) {
  __shared__ unsigned long long part[kFinishThreads / 64];
  __shared__ int part_bad[kFinishThreads / 64];
  const int i = blockIdx.x, tid = threadIdx.x;
  const int64_t b = P.task_first[i], e = P.task_first[i + 1];
  unsigned long long v = 0;
  bool bad = false;
  auto take = [&](int64_t t) {
    if constexpr (WIDE) {
      const unsigned long long s = P.task_sse64[t];
      bad |= s == ~0ull;
      v += s;
    } else {
      v += P.task_sse[t];
    }
  };
  int64_t t = b + tid;
  for (; t + 3 * kFinishThreads < e; t += 4 * kFinishThreads) {
#pragma unroll
    for (int u = 0; u < 4; ++u) take(t + u * kFinishThreads);
  }
  for (; t < e; t += kFinishThreads) take(t);
  v = wave_sum_u64(v);
  const bool wbad = __builtin_amdgcn_ballot_w64(bad) != 0;
  if ((tid & 63) == 0) {
    part[tid >> 6] = v;
    part_bad[tid >> 6] = wbad;
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long sum = 0;
    bool any_bad = false;
#pragma unroll
    for (int w = 0; w < kFinishThreads / 64; ++w) {
      sum += part[w];
      any_bad |= part_bad[w] != 0;
    }
    P.sse[i] = any_bad ? ~0ull : sum;
    if (P.psnr) {
      const ImageDesc& d = P.images[i];
      P.psnr[i] = any_bad ? __builtin_nan("")
                          : sum == 0 ? __builtin_huge_val()
                                     : 10.0 * log10(65025.0 * (double)d.h * (double)d.w / (double)sum);
    }
  }
}

__device__ __forceinline__ unsigned byte_of(const uint4& q, int k) {
  const unsigned w = k < 4 ? q.x : k < 8 ? q.y : k < 12 ? q.z : q.w;
  return (w >> (8 * (k & 3))) & 0xffu;
}

// Repeat byte (n-1) into bytes n..15 (edge extension of a partial block row).
__device__ __forceinline__ uint4 extend_bytes(uint4 q, int n) {
  unsigned b[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) b[k] = byte_of(q, k);
  unsigned last = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) last = (k == n - 1) ? b[k] : last;
#pragma unroll
  for (int k = 0; k < 16; ++k) b[k] = (k < n) ? b[k] : last;
  uint4 r;
  r.x = b[0] | (b[1] << 8) | (b[2] << 16) | (b[3] << 24);
  r.y = b[4] | (b[5] << 8) | (b[6] << 16) | (b[7] << 24);
  r.z = b[8] | (b[9] << 8) | (b[10] << 16) | (b[11] << 24);
  r.w = b[12] | (b[13] << 8) | (b[14] << 16) | (b[15] << 24);
  return r;
}

// Keep bytes 0..n-1, zero the rest.
__device__ __forceinline__ uint4 keep_bytes(uint4 q, int n) {
  auto m = [n](int k0) -> unsigned {
    unsigned r = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) r |= (k0 + j < n) ? (0xffu << (8 * j)) : 0u;
    return r;
  };
  q.x &= m(0); q.y &= m(4); q.z &= m(8); q.w &= m(12);
  return q;
}

// ---------------------------------------------------------------------------
// SSE accumulation per wavefront, flushed with one 64-bit atomic per image.
// Per-image SSE of the vector kernels: each wavefront adds its (nonzero)
// sums atomically into one of P.sse_slots accumulators of the image, chosen
// by the wavefront's index, so that the wavefronts working on one image do
// not all contend for one address; a finishing kernel sums the slots.
struct SseAcc {
  unsigned long long lane = 0;
  int slot = 0;
  __device__ __forceinline__ void init(const Params& P) {
    slot = uniform_int((int)((blockIdx.x * kWavesPerGroup + (threadIdx.x >> 6)) % (unsigned)P.sse_slots));
  }
  __device__ __forceinline__ void flush(const Params& P, int img) {
    const unsigned long long t = wave_sum_u64(lane);
    if ((threadIdx.x & 63) == 0 && t) atomicAdd(P.sse + (int64_t)img * P.sse_slots + slot, t);
    lane = 0;
  }
};

}  // namespace adct16
