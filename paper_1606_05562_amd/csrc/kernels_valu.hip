// Vector-ALU kernels: the 60-addition butterflies of Eq. (1) applied to the
// rows of 16x16 blocks, an LDS transpose, and the columns (Section 5.1's
// row / transpose / column structure), plus retention, the uniform
// quantiser, the inverse and the PSNR reduction of Section 4.
//
// Work layout.  A wavefront processes one strip (16 rows x 8 blocks) at a
// time.  Lane l = 16 p + x works on blocks p and p + 4 of the strip: in the
// row layout it holds row x of both blocks, in the column layout column x.
// 8-bit pixels are transformed as packed pairs of 16-bit lanes (block p in
// the low half, block p + 4 in the high half): every forward output lies in
// a known range narrower than 2^16 (AC in [-32640, 32640], DC in [0, 65280]),
// so modular 16-bit arithmetic recovers it exactly and each v_pk_add/sub
// does two of the paper's additions.  Inverses run in int32 (exact) or
// float64 (uniform quantiser).
#include <algorithm>

#include "device_common.hpp"

namespace adct16 {

__device__ __forceinline__ us2 as_us2(unsigned v) { return __builtin_bit_cast(us2, v); }
__device__ __forceinline__ unsigned as_u32(us2 v) { return __builtin_bit_cast(unsigned, v); }

struct LaneGeom {
  bool full;       // the strip is 8 whole blocks wide (the same in every lane): no column is extended
  bool rowok;      // this lane's row (row layout) lies inside the image
  int na, nb;      // valid columns of blocks a / b (0: block absent)
  int64_t rowoff;  // element offset of the (clamped) row
  int xa, xb;      // first column of blocks a / b
  int64_t blka, blkb;  // block indices in coefficient buffers
};

__device__ __forceinline__ LaneGeom lane_geom(const StripCursor& c, int x, int p) {
  LaneGeom g;
  g.full = (c.sxi + 1) * (16 * kStripBlocks) <= c.d.w;
  const int y0 = c.sy * 16;
  g.rowok = (y0 + x) < c.d.h;
  const int y = min(y0 + x, c.d.h - 1);
  const int ba = c.sxi * kStripBlocks + p, bb = ba + 4;
  g.xa = ba * 16;
  g.xb = bb * 16;
  g.na = ba < c.d.bx ? min(16, c.d.w - g.xa) : 0;
  g.nb = bb < c.d.bx ? min(16, c.d.w - g.xb) : 0;
  g.rowoff = c.d.offset + (int64_t)y * c.d.pitch;
  const int64_t rowblk = c.d.block_begin + (int64_t)c.sy * c.d.bx;
  g.blka = rowblk + ba;
  g.blkb = rowblk + bb;
  return g;
}

// ---------------------------------------------------------------------------
// Loads of one block row (16 samples), edge-extended past the image width.
__device__ __forceinline__ uint4 load_row_u8(const uint8_t* img, int64_t off, int n) {
  if (n <= 0) return make_uint4(0, 0, 0, 0);
  uint4 q = *reinterpret_cast<const uint4*>(img + off);
  if (n < 16) q = extend_bytes(q, n);
  return q;
}

// 16 int16 samples from two raw 16-byte words; when 0 < n < 16 the row is
// extended by its last valid sample (n >= 16: no extension).  `full` (the
// same in every lane) says that no lane has n < 16, which skips the
// extension's selects altogether.
__device__ __forceinline__ void unpack_i16(const uint4& q0, const uint4& q1, int n, int (&v)[16],
                                           bool full = false) {
  const unsigned w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[2 * k] = (int)(short)(w[k] & 0xffffu);
    v[2 * k + 1] = ((int)w[k]) >> 16;
  }
  if (!full && n < 16) {
    int last = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) last = (k == n - 1) ? v[k] : last;
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = (k < n) ? v[k] : last;
  }
}

__device__ __forceinline__ void load_row_i16(const int16_t* img, int64_t off, int n, int (&v)[16]) {
  if (n <= 0) {
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = 0;
    return;
  }
  const uint4* q = reinterpret_cast<const uint4*>(img + off);
  unpack_i16(q[0], q[1], n, v);
}

// Raw rows of blocks a and b (32 bytes each; zero for absent blocks), so
// that the next strip's loads can be in flight while this one is computed.
// Block rows are 16-byte aligned (validated pitches, offsets and buffers).
// The loads are unconditional, an absent block reading column 0 of the
// same row: loads under a branch would each be waited for at its join.
struct RawI16 { uint4 a0, a1, b0, b1; };

__device__ __forceinline__ const uint4* row_ptr16(const void* row, int64_t byte_off) {
  return reinterpret_cast<const uint4*>(
      __builtin_assume_aligned(reinterpret_cast<const uint8_t*>(row) + byte_off, 16));
}

__device__ __forceinline__ RawI16 load_rows_i16(const int16_t* img, const LaneGeom& g) {
  const uint4 z = make_uint4(0, 0, 0, 0);
  const int16_t* row = img + g.rowoff;
  const uint4* pa = row_ptr16(row, 2 * (int64_t)(g.na > 0 ? g.xa : 0));
  const uint4* pb = row_ptr16(row, 2 * (int64_t)(g.nb > 0 ? g.xb : 0));
  const uint4 a0 = pa[0], a1 = pa[1], b0 = pb[0], b1 = pb[1];
  RawI16 r;
  r.a0 = g.na > 0 ? a0 : z;
  r.a1 = g.na > 0 ? a1 : z;
  r.b0 = g.nb > 0 ? b0 : z;
  r.b1 = g.nb > 0 ? b1 : z;
  return r;
}

// (a[k], b[k]) byte pairs -> packed 16-bit pairs.
__device__ __forceinline__ void pair_bytes(const uint4& a, const uint4& b, us2 (&X)[16]) {
  const unsigned aw[4] = {a.x, a.y, a.z, a.w};
  const unsigned bw[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const unsigned j = k & 3;
    const unsigned sel = j | (0x0cu << 8) | ((4u + j) << 16) | (0x0cu << 24);
    X[k] = as_us2(__builtin_amdgcn_perm(bw[k >> 2], aw[k >> 2], sel));
  }
}

// ---------------------------------------------------------------------------
// Forward transform of the strip; results in the column layout.
struct ColsU8 { us2 z[16]; };       // packed (block a, block b) modulo 2^16
struct ColsI32 { int a[16], b[16]; };

// Raw 16-byte row loads of blocks a and b (zero for absent blocks); the
// edge extension is applied where the rows are consumed, so that loads for
// the next strip can be in flight while the current one is computed.
__device__ __forceinline__ void load_rows_u8(const uint8_t* img, const LaneGeom& g, uint4& ra, uint4& rb) {
  const uint8_t* row = img + g.rowoff;
  const uint4 a = *row_ptr16(row, g.na > 0 ? g.xa : 0), b = *row_ptr16(row, g.nb > 0 ? g.xb : 0);
  ra = g.na > 0 ? a : make_uint4(0, 0, 0, 0);
  rb = g.nb > 0 ? b : make_uint4(0, 0, 0, 0);
}

__device__ __forceinline__ void fix_edges_u8(const LaneGeom& g, uint4& ra, uint4& rb) {
  if (g.full) return;
  if (g.na > 0 && g.na < 16) ra = extend_bytes(ra, g.na);
  if (g.nb > 0 && g.nb < 16) rb = extend_bytes(rb, g.nb);
}

// Forward transform of rows already loaded (and edge-extended).
template <int MAT>
__device__ __forceinline__ void forward_u8_rows(int* lds, int x, int p, const uint4& ra, const uint4& rb,
                                                us2 (&Z)[16]) {
  pair_bytes(ra, rb, Z);
  m_fwd<MAT>(Z);                                 // row pass
  transpose_rows_to_cols(lds, p, x, Z);     // transposition buffer
  m_fwd<MAT>(Z);                                 // column pass: Z[u] = (Za[u][x], Zb[u][x])
}

template <int MAT>
__device__ __forceinline__ void forward_u8(const uint8_t* img, const LaneGeom& g, int* lds, int x,
                                           int p, uint4& ra, uint4& rb, us2 (&Z)[16]) {
  ra = load_row_u8(img, g.rowoff + g.xa, g.na);
  rb = load_row_u8(img, g.rowoff + g.xb, g.nb);
  pair_bytes(ra, rb, Z);
  m_fwd<MAT>(Z);                                 // row pass
  transpose_rows_to_cols(lds, p, x, Z);     // transposition buffer
  m_fwd<MAT>(Z);                                 // column pass: Z[u] = (Za[u][x], Zb[u][x])
}

// Exact int32 coefficients from the packed 16-bit residues: AC values are
// the signed residues, DC (u = v = 0, lane x = 0) the unsigned one.
__device__ __forceinline__ void widen_u8(const us2 (&Z)[16], int x, int (&za)[16], int (&zb)[16]) {
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const unsigned w = as_u32(Z[u]);
    za[u] = (int)(short)(w & 0xffffu);
    zb[u] = ((int)w) >> 16;
  }
  const unsigned w0 = as_u32(Z[0]);
  za[0] = (x == 0) ? (int)(w0 & 0xffffu) : za[0];
  zb[0] = (x == 0) ? (int)(w0 >> 16) : zb[0];
}

template <int MAT>
__device__ __forceinline__ void forward_i16_rows(const RawI16& r, const LaneGeom& g, int* lds, int x, int p,
                                                 int (&za)[16], int (&zb)[16]) {
  unpack_i16(r.a0, r.a1, g.na, za, g.full);
  unpack_i16(r.b0, r.b1, g.nb, zb, g.full);
  m_fwd<MAT>(za);
  m_fwd<MAT>(zb);
  transpose_rows_to_cols(lds, p, x, za);
  transpose_rows_to_cols(lds, p, x, zb);
  m_fwd<MAT>(za);
  m_fwd<MAT>(zb);
}

template <int MAT>
__device__ __forceinline__ void forward_i16(const int16_t* img, const LaneGeom& g, int* lds, int x,
                                            int p, int (&za)[16], int (&zb)[16]) {
  forward_i16_rows<MAT>(load_rows_i16(img, g), g, lds, x, p, za, zb);
}

// ---------------------------------------------------------------------------
// Inverses, column layout in, row layout out.

// Mask modes: t = T^T (W .* Z) T + 1152 exactly in int32 (W = w w^T .* keep
// already applied by the caller).  `rnd` adds 1152 at (0,0), which adds 1152
// to every output because row 0 of T is all ones.
template <int MAT>
__device__ __forceinline__ void inverse_int(int* lds, int x, int p, int (&a)[16], int (&b)[16], bool rnd) {
  if (rnd && x == 0) { a[0] += 1152; b[0] += 1152; }
  m_inv<MAT>(a);
  m_inv<MAT>(b);
  transpose_cols_to_rows(lds, p, x, a);
  transpose_cols_to_rows(lds, p, x, b);
  m_inv<MAT>(a);
  m_inv<MAT>(b);
}

template <int MAT>
__device__ __forceinline__ void inverse_f64(int* lds, int x, int p, double (&a)[16], double (&b)[16]) {
  m_inv<MAT>(a);
  m_inv<MAT>(b);
  transpose_cols_to_rows_f64(lds, p, x, a);
  transpose_cols_to_rows_f64(lds, p, x, b);
  m_inv<MAT>(a);
  m_inv<MAT>(b);
}

// floor((N + 1152) / 2304) clamped to [0, 255], given t = N + 1152: for
// 0 <= t <= 589823, floor(t / 2304) = (t * 1864136) >> 32 (24-bit multiply).
__device__ __forceinline__ unsigned pix_u8_from_t(int t) {
  const unsigned tc = (unsigned)min(max(t, 0), 589823);
  return (unsigned)(((unsigned long long)tc * 1864136ull) >> 32);
}

// floor(t / 2304) saturated to [-32768, 32767].  With t clamped to
// [-32768 * 2304, 32767 * 2304 + 2303], u = t + 32768 * 2304 lies in
// [0, 2^28); floor(u / 2304) = (u * 3817748708) >> 43 for every u < 2^33,
// since 3817748708 = ceil(2^43 / 2304) exceeds 2^43 / 2304 by 1024 / 2304.
__device__ __forceinline__ int pix_i16_from_t(int t) {
  const unsigned u = (unsigned)(min(max(t, -75497472), 75497471) + 75497472);
  return (int)(__umulhi(u, 3817748708u) >> 11) - 32768;
}

__device__ __forceinline__ int sat16(long long v) { return (int)min(max(v, -32768ll), 32767ll); }

__device__ __forceinline__ uint4 pack_u8(const unsigned (&v)[16]) {
  uint4 r;
  r.x = v[0] | (v[1] << 8) | (v[2] << 16) | (v[3] << 24);
  r.y = v[4] | (v[5] << 8) | (v[6] << 16) | (v[7] << 24);
  r.z = v[8] | (v[9] << 8) | (v[10] << 16) | (v[11] << 24);
  r.w = v[12] | (v[13] << 8) | (v[14] << 16) | (v[15] << 24);
  return r;
}

// Sum of squared byte differences over the first n bytes of two rows.
__device__ __forceinline__ unsigned sse_u8(uint4 o, uint4 r, int n) {
  if (n < 16) { o = keep_bytes(o, n); r = keep_bytes(r, n); }
  const unsigned ow[4] = {o.x, o.y, o.z, o.w}, rw[4] = {r.x, r.y, r.z, r.w};
  unsigned oo = 0, rr = 0, orr = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    oo = __builtin_amdgcn_udot4(ow[m], ow[m], oo, false);
    rr = __builtin_amdgcn_udot4(rw[m], rw[m], rr, false);
    orr = __builtin_amdgcn_udot4(ow[m], rw[m], orr, false);
  }
  return oo + rr - 2u * orr;
}

// Whole block rows of the reconstruction are stored non-temporally (written
// once, never read back in the pass).
typedef unsigned v4u_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void store_row_u8(uint8_t* img, int64_t off, int n, uint4 v) {
  if (n >= 16) {
    const v4u_t w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<v4u_t*>(img + off));
  } else {
    for (int k = 0; k < n; ++k) img[off + k] = (uint8_t)byte_of(v, k);
  }
}

__device__ __forceinline__ void store_row_i16(int16_t* img, int64_t off, int n, const int (&v)[16]) {
  if (n >= 16) {
    uint4* q = reinterpret_cast<uint4*>(img + off);
    unsigned w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = ((unsigned)v[2 * k] & 0xffffu) | ((unsigned)v[2 * k + 1] << 16);
    const v4u_t s0 = {w[0], w[1], w[2], w[3]}, s1 = {w[4], w[5], w[6], w[7]};
    __builtin_nontemporal_store(s0, reinterpret_cast<v4u_t*>(q));
    __builtin_nontemporal_store(s1, reinterpret_cast<v4u_t*>(q) + 1);
  } else {
    for (int k = 0; k < n; ++k) img[off + k] = (int16_t)v[k];
  }
}

// ---------------------------------------------------------------------------
// Block-major coefficient buffers (256 values per block, [u][v]) to and
// from the column layout, through the transposition buffer: lane group p
// puts its column-layout values of one block into slot p, and each global
// access instruction then moves one whole block from row chunks (lane l:
// row l / 4, columns 4 (l % 4) .. + 3), 1 KB of 32-bit or 512 B of 16-bit
// values contiguously.  `first` is the block held by lane group 0 and `nb`
// how many of the four (consecutive) blocks exist; both are the same for
// the whole wavefront.  32-bit kinds: CF_I32, CF_L32 and CF_F32 (float
// bits); 16-bit: CF_I16C (DC centred by -32768) and CF_L16 (saturated).
typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef unsigned v2u_t __attribute__((ext_vector_type(2)));

// The stores are non-temporal: each instruction writes whole cache lines of
// a block (1 KB or 512 B at a multiple of that offset) that nothing reads
// again in the same pass.
template <int CF>
__device__ __forceinline__ void store_blocks(void* buf, int* lds, int p, int x, int lane, int64_t first, int nb,
                                             const int (&z)[16]) {
  lds_put_col(lds, p, x, z);
  wave_lds_sync();
  const int u = lane >> 2, j = lane & 3;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    if (m < nb) {
      int4 v = *reinterpret_cast<const int4*>(lds + m * kSlot + u * kRow + 4 * j);
      const int64_t off = (first + m) * 256 + u * 16 + 4 * j;
      if constexpr (CF == CF_I32 || CF == CF_L32 || CF == CF_F32) {
        const v4i_t w = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(w, reinterpret_cast<v4i_t*>(reinterpret_cast<int*>(buf) + off));
      } else {
        if constexpr (CF == CF_I16C) {
          if (lane == 0) v.x -= 32768;
        } else {
          v = make_int4(sat16(v.x), sat16(v.y), sat16(v.z), sat16(v.w));
        }
        const v2u_t w = {((unsigned)v.x & 0xffffu) | ((unsigned)v.y << 16),
                         ((unsigned)v.z & 0xffffu) | ((unsigned)v.w << 16)};
        __builtin_nontemporal_store(w, reinterpret_cast<v2u_t*>(reinterpret_cast<int16_t*>(buf) + off));
      }
    }
  }
  wave_lds_sync();
}

// The converse, in two steps so that the loads of the next strip can be in
// flight while this one is computed: fetch_blocks issues the loads (zeros
// where a block does not exist), blocks_to_cols regroups them into column
// x of the lane group's block.
// The loads are unconditional (a missing block reads block `safe`, which
// exists, and is zeroed afterwards): loads under a branch would each be
// waited for before the branch joins.  Like the stores above they are
// non-temporal (whole lines, read once).
template <int CF>
__device__ __forceinline__ void fetch_blocks(const void* buf, int lane, int64_t first, int nb, int64_t safe,
                                             int4 (&v)[4]) {
  const int u = lane >> 2, j = lane & 3;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int64_t off = (m < nb ? first + m : safe) * 256 + u * 16 + 4 * j;
    int4 t;
    if constexpr (CF == CF_I32 || CF == CF_L32) {
      const v4i_t w = __builtin_nontemporal_load(reinterpret_cast<const v4i_t*>(reinterpret_cast<const int*>(buf) + off));
      t = make_int4(w.x, w.y, w.z, w.w);
    } else {
      const v2u_t w = __builtin_nontemporal_load(reinterpret_cast<const v2u_t*>(reinterpret_cast<const int16_t*>(buf) + off));
      t = make_int4((int)(short)(w.x & 0xffffu), ((int)w.x) >> 16, (int)(short)(w.y & 0xffffu), ((int)w.y) >> 16);
      if constexpr (CF == CF_I16C) {
        if (lane == 0) t.x += 32768;
      }
    }
    v[m] = m < nb ? t : make_int4(0, 0, 0, 0);
  }
}

__device__ __forceinline__ void blocks_to_cols(int* lds, int p, int x, int lane, const int4 (&v)[4], int (&z)[16]) {
  const int u = lane >> 2, j = lane & 3;
#pragma unroll
  for (int m = 0; m < 4; ++m) *reinterpret_cast<int4*>(lds + m * kSlot + u * kRow + 4 * j) = v[m];
  wave_lds_sync();
  lds_get_col(lds, p, x, z);
  wave_lds_sync();
}

// Blocks of the strip's lane-group halves: a = blocks 0..3, b = 4..7.
__device__ __forceinline__ int blocks_a(const StripCursor& c) { return min(4, max(0, c.d.bx - c.sxi * kStripBlocks)); }
__device__ __forceinline__ int blocks_b(const StripCursor& c) { return min(4, max(0, c.d.bx - c.sxi * kStripBlocks - 4)); }

// ---------------------------------------------------------------------------
// Kernels.

template <int MAT, int IN, int CF>
__global__ __launch_bounds__(kGroupThreads) void k_forward(Params P) {
  __shared__ __attribute__((aligned(16))) int lds_all[kWavesPerGroup * kWaveLds];
  int* lds = lds_all + (threadIdx.x >> 6) * kWaveLds;
  const int lane = threadIdx.x & 63, x = lane & 15, p = lane >> 4;
  float ysc[16];
  if constexpr (CF == CF_F32) {
#pragma unroll
    for (int u = 0; u < 16; ++u) ysc[u] = P.tables->yscale[u * 16 + x];
  }
  StripCursor c;
  if (!cursor_init(c, P)) return;
  do {
    const LaneGeom g = lane_geom(c, x, p);
    int za[16], zb[16];
    if constexpr (IN == IN_U8) {
      uint4 ra, rb;
      us2 Z[16];
      forward_u8<MAT>(reinterpret_cast<const uint8_t*>(P.in), g, lds, x, p, ra, rb, Z);
      widen_u8(Z, x, za, zb);
    } else {
      forward_i16<MAT>(reinterpret_cast<const int16_t*>(P.in), g, lds, x, p, za, zb);
    }
    if constexpr (CF == CF_F32) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        za[u] = __float_as_int((float)za[u] * ysc[u]);
        zb[u] = __float_as_int((float)zb[u] * ysc[u]);
      }
    }
    store_blocks<CF>(P.coef, lds, p, x, lane, g.blka - p, blocks_a(c), za);
    store_blocks<CF>(P.coef, lds, p, x, lane, g.blkb - p, blocks_b(c), zb);
  } while (cursor_next(c, P), c.s < c.s_end);
}

// Quantisation level of one integer coefficient Z with its multiplier M
// (S and the step folded in).  Uniform: round-half-even(fl32(fl32(Z) M)).
// Deadzone: sign(Z) floor(fl32(fl32(fl32(|Z|) M) + f)); the separate
// rounded multiply and add (no fused multiply-add) are part of the
// definition.
template <int MODE>
__device__ __forceinline__ int level_of(int z, float m, float f) {
  if constexpr (MODE == MODE_UNIFORM) {
    return (int)__builtin_rintf((float)z * m);
  } else {
    const float a = __fmul_rn((float)abs(z), m);
    const int l = (int)floorf(__fadd_rn(a, f));
    return z < 0 ? -l : l;
  }
}

// Row norms n_u of the plan's matrix fall into three classes (16, 12, 8)
// for T and one (16) for the Walsh-Hadamard matrix.  The quantiser's
// multipliers depend on (u, v) only through n_u n_v, so a lane (fixed v)
// keeps one value per class instead of sixteen.
constexpr int kNormClasses = 3;

template <int MAT>
__device__ __forceinline__ constexpr int norm_class(int u) {
  if constexpr (MAT == MAT_WHT) {
    return 0;
  } else {
    constexpr int cls[16] = {0, 0, 1, 2, 2, 0, 1, 1, 0, 1, 1, 2, 2, 1, 1, 1};  // n_u = 16, 12, 8
    return cls[u];
  }
}

// A row u of each class.
__device__ __forceinline__ constexpr int class_row(int c) { return c == 0 ? 0 : c == 1 ? 2 : 3; }

// Per-lane constants of the quantisers: the level multipliers M_uv and the
// reconstruction factors (step) s_u s_v, one per norm class of u.
struct QuantLane {
  float m[kNormClasses];
  double d[kNormClasses];
};

__device__ __forceinline__ QuantLane quant_lane(const Tables* tb, int x) {
  QuantLane q;
#pragma unroll
  for (int c = 0; c < kNormClasses; ++c) {
    q.m[c] = tb->qmul[class_row(c) * 16 + x];
    q.d[c] = tb->deqc[x] * tb->sdiag[class_row(c)];
  }
  return q;
}

// Quantiser reconstruction of one block (column layout in, this lane's row
// out): V = step s_u s_v L in float64, T^T V T by the butterflies and the
// transposition buffer, then rounded half up and clamped to the input's range.
template <int MAT, int IN>
__device__ __forceinline__ void dequant_inverse_block(int* lds, int x, int p, const QuantLane& ql,
                                                      const int (&l)[16], int (&pix)[16]) {
  double f[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) f[u] = (double)l[u] * ql.d[norm_class<MAT>(u)];
  m_inv<MAT>(f);
  transpose_cols_to_rows_f64(lds, p, x, f);
  m_inv<MAT>(f);
  constexpr int lo = IN == IN_U8 ? 0 : -32768, hi = IN == IN_U8 ? 255 : 32767;
#pragma unroll
  for (int k = 0; k < 16; ++k) pix[k] = min(max((int)floor(f[k] + 0.5), lo), hi);
}

// Retention / quantiser of the column-layout coefficients of one lane, and
// the inverse.  Mask modes multiply by W = w_u w_v keep(u, v) (the inverse
// weights; the masked coefficients themselves are kept for an optional
// qcoef output) and return t = N + 1152 (N for float output).  Quantisers
// return the rounded reconstruction pixels.  |A'| stays far inside the
// int32 range (within 8 q of the 16-bit input), so the conversion is exact.
template <int MAT, int IN, int MODE, int QOUT, int OUT>
__device__ __forceinline__ void quant_and_inverse(const Params& P, const LaneGeom& g, int nba, int nbb, int* lds,
                                                  int x, int p, int lane, const int (&W)[16], const QuantLane& ql,
                                                  int (&za)[16], int (&zb)[16], int (&oa)[16],
                                                  int (&ob)[16]) {
  if constexpr (MODE == MODE_MASK) {
    if constexpr (QOUT != CF_NONE) {
      int ka[16], kb[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        ka[u] = W[u] ? za[u] : 0;
        kb[u] = W[u] ? zb[u] : 0;
      }
      store_blocks<QOUT>(P.qcoef, lds, p, x, lane, g.blka - p, nba, ka);
      store_blocks<QOUT>(P.qcoef, lds, p, x, lane, g.blkb - p, nbb, kb);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      za[u] = __mul24(za[u], W[u]);
      zb[u] = __mul24(zb[u], W[u]);
    }
    inverse_int<MAT>(lds, x, p, za, zb, OUT != OUT_F32);
#pragma unroll
    for (int k = 0; k < 16; ++k) { oa[k] = za[k]; ob[k] = zb[k]; }
  } else {
    const float f = P.tables->qoff;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      za[u] = level_of<MODE>(za[u], ql.m[norm_class<MAT>(u)], f);
      zb[u] = level_of<MODE>(zb[u], ql.m[norm_class<MAT>(u)], f);
    }
    if constexpr (QOUT != CF_NONE) {
      store_blocks<QOUT>(P.qcoef, lds, p, x, lane, g.blka - p, nba, za);
      store_blocks<QOUT>(P.qcoef, lds, p, x, lane, g.blkb - p, nbb, zb);
    }
    // one block at a time: half the float64 registers live
    dequant_inverse_block<MAT, IN>(lds, x, p, ql, za, oa);
    dequant_inverse_block<MAT, IN>(lds, x, p, ql, zb, ob);
  }
}

// Row-layout epilogue: reconstruction pixels of this lane's rows.
template <int MODE, int OUT>
__device__ __forceinline__ void recon_u8(const int (&t)[16], const double (&f)[16], unsigned (&pix)[16]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if constexpr (MODE == MODE_MASK) {
      pix[k] = pix_u8_from_t(t[k]);
    } else {
      const double r = floor(f[k] + 0.5);
      pix[k] = (unsigned)fmin(fmax(r, 0.0), 255.0);
    }
  }
}

template <int MODE>
__device__ __forceinline__ void recon_i16(const int (&t)[16], const double (&f)[16], int (&pix)[16]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    if constexpr (MODE == MODE_MASK) {
      pix[k] = pix_i16_from_t(t[k]);
    } else {
      const double r = floor(f[k] + 0.5);
      pix[k] = (int)fmin(fmax(r, -32768.0), 32767.0);
    }
  }
}

template <int MAT, int IN, int MODE, int QOUT, int OUT>
__global__ __launch_bounds__(kGroupThreads, ADCT16_VALU_MIN_WG) void k_fused(Params P) {
  __shared__ __attribute__((aligned(16))) int lds_all[kWavesPerGroup * kWaveLds];
  int* lds = lds_all + (threadIdx.x >> 6) * kWaveLds;
  const int lane = threadIdx.x & 63, x = lane & 15, p = lane >> 4;
  int W[16];
  QuantLane ql;
  if constexpr (MODE == MODE_MASK) {
#pragma unroll
    for (int u = 0; u < 16; ++u) W[u] = P.tables->wkeep[u * 16 + x];
  } else {
    ql = quant_lane(P.tables, x);
  }
  StripCursor c;
  if (!cursor_init(c, P)) return;
  SseAcc acc;
  acc.init(P);
  int since_flush = 0;
  const uint8_t* in8 = reinterpret_cast<const uint8_t*>(P.in);
  const int16_t* in16 = reinterpret_cast<const int16_t*>(P.in);
  LaneGeom gn = lane_geom(c, x, p);
  uint4 na = make_uint4(0, 0, 0, 0), nb = na;
  RawI16 nr;
  if constexpr (IN == IN_U8) load_rows_u8(in8, gn, na, nb);
  else nr = load_rows_i16(in16, gn);
  for (;;) {
    const LaneGeom g = gn;
    const int nba = blocks_a(c), nbb = blocks_b(c);
    int za[16], zb[16];
    uint4 ra = na, rb = nb;
    const RawI16 rr = nr;
    const int img = c.img;
    const bool changed = cursor_next(c, P);
    const bool done = c.s >= c.s_end;
    // prefetch the next strip, unconditionally: past the last strip the
    // cursor still describes the current one, which is read again
    gn = lane_geom(c, x, p);
    if constexpr (IN == IN_U8) load_rows_u8(in8, gn, na, nb);
    else nr = load_rows_i16(in16, gn);
    if constexpr (IN == IN_U8) {
      us2 Z[16];
      fix_edges_u8(g, ra, rb);
      forward_u8_rows<MAT>(lds, x, p, ra, rb, Z);
      widen_u8(Z, x, za, zb);
    } else {
      forward_i16_rows<MAT>(rr, g, lds, x, p, za, zb);
    }
    int ta[16], tb[16];
    quant_and_inverse<MAT, IN, MODE, QOUT, OUT>(P, g, nba, nbb, lds, x, p, lane, W, ql, za, zb, ta, tb);
    if constexpr (IN == IN_U8) {
      unsigned pa[16], pb[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        pa[k] = MODE == MODE_MASK ? pix_u8_from_t(ta[k]) : (unsigned)ta[k];
        pb[k] = MODE == MODE_MASK ? pix_u8_from_t(tb[k]) : (unsigned)tb[k];
      }
      const uint4 qa = pack_u8(pa), qb = pack_u8(pb);
      if (g.rowok) {
        if constexpr (OUT == OUT_U8) {
          uint8_t* o = reinterpret_cast<uint8_t*>(P.out);
          if (g.na > 0) store_row_u8(o, g.rowoff + g.xa, g.na, qa);
          if (g.nb > 0) store_row_u8(o, g.rowoff + g.xb, g.nb, qb);
        }
        if (g.full) acc.lane += sse_u8(ra, qa, 16) + sse_u8(rb, qb, 16);
        else acc.lane += (g.na > 0 ? sse_u8(ra, qa, g.na) : 0u) + (g.nb > 0 ? sse_u8(rb, qb, g.nb) : 0u);
      }
    } else {
      int pa[16], pb[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        pa[k] = MODE == MODE_MASK ? pix_i16_from_t(ta[k]) : ta[k];
        pb[k] = MODE == MODE_MASK ? pix_i16_from_t(tb[k]) : tb[k];
      }
      if (g.rowok) {
        // the error against the input rows, read again (cache-resident;
        // holding them across the inverse costs more in occupancy)
        int ia[16], ib[16];
        const RawI16 er = load_rows_i16(in16, g);
        unpack_i16(er.a0, er.a1, 16, ia);
        unpack_i16(er.b0, er.b1, 16, ib);
        if constexpr (OUT == OUT_I16) {
          int16_t* o = reinterpret_cast<int16_t*>(P.out);
          if (g.na > 0) store_row_i16(o, g.rowoff + g.xa, g.na, pa);
          if (g.nb > 0) store_row_i16(o, g.rowoff + g.xb, g.nb, pb);
        }
        // |error| < 2^16, so its square is the low 32 bits of a 24-bit product
        unsigned long long s = 0;
        if (g.full) {
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            s += (unsigned)__mul24(ia[k] - pa[k], ia[k] - pa[k]);
            s += (unsigned)__mul24(ib[k] - pb[k], ib[k] - pb[k]);
          }
        } else {
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            const int da = (k < g.na) ? ia[k] - pa[k] : 0;
            const int db = (k < g.nb) ? ib[k] - pb[k] : 0;
            s += (unsigned)__mul24(da, da);
            s += (unsigned)__mul24(db, db);
          }
        }
        acc.lane += s;
      }
    }
    if (changed || done || ++since_flush == 1024) {
      acc.flush(P, img);
      since_flush = 0;
    }
    if (done) break;
  }
}

// Inverse of block-major coefficients or levels.
template <int MAT, int CFIN, int MODE, int OUT>
__global__ __launch_bounds__(kGroupThreads) void k_inverse(Params P) {
  __shared__ __attribute__((aligned(16))) int lds_all[kWavesPerGroup * kWaveLds];
  int* lds = lds_all + (threadIdx.x >> 6) * kWaveLds;
  const int lane = threadIdx.x & 63, x = lane & 15, p = lane >> 4;
  int W[16];
  double Dc = 0.0;
  if constexpr (MODE == MODE_MASK) {
#pragma unroll
    for (int u = 0; u < 16; ++u) W[u] = P.tables->wall[u * 16 + x];
  } else {
    Dc = P.tables->deqc[x];
  }
  StripCursor c;
  if (!cursor_init(c, P)) return;
  LaneGeom gn = lane_geom(c, x, p);
  int4 va[4], vb[4];
  fetch_blocks<CFIN>(P.qcoef, lane, gn.blka - p, blocks_a(c), gn.blka - p, va);
  fetch_blocks<CFIN>(P.qcoef, lane, gn.blkb - p, blocks_b(c), gn.blka - p, vb);
  for (;;) {
    const LaneGeom g = gn;
    const int4 ca[4] = {va[0], va[1], va[2], va[3]}, cb[4] = {vb[0], vb[1], vb[2], vb[3]};
    cursor_next(c, P);
    const bool more = c.s < c.s_end;
    // the next strip's coefficients, loaded unconditionally: past the last
    // strip the cursor still describes the current one, read again
    gn = lane_geom(c, x, p);
    fetch_blocks<CFIN>(P.qcoef, lane, gn.blka - p, blocks_a(c), gn.blka - p, va);
    fetch_blocks<CFIN>(P.qcoef, lane, gn.blkb - p, blocks_b(c), gn.blka - p, vb);
    int za[16], zb[16];
    blocks_to_cols(lds, p, x, lane, ca, za);
    blocks_to_cols(lds, p, x, lane, cb, zb);
    int ta[16], tb[16];
    double fa[16], fb[16];
    if constexpr (MODE == MODE_MASK) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        za[u] = __mul24(za[u], W[u]);
        zb[u] = __mul24(zb[u], W[u]);
      }
      inverse_int<MAT>(lds, x, p, za, zb, OUT != OUT_F32);
#pragma unroll
      for (int k = 0; k < 16; ++k) { ta[k] = za[k]; tb[k] = zb[k]; }
    } else {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        fa[u] = ((double)za[u] * Dc) * P.tables->sdiag[u];
        fb[u] = ((double)zb[u] * Dc) * P.tables->sdiag[u];
      }
      inverse_f64<MAT>(lds, x, p, fa, fb);
    }
    if (!g.rowok) {
      // rows past the image height: nothing to store
    } else if constexpr (OUT == OUT_U8) {
      unsigned pa[16], pb[16];
      recon_u8<MODE, OUT>(ta, fa, pa);
      recon_u8<MODE, OUT>(tb, fb, pb);
      uint8_t* o = reinterpret_cast<uint8_t*>(P.out);
      if (g.na > 0) store_row_u8(o, g.rowoff + g.xa, g.na, pack_u8(pa));
      if (g.nb > 0) store_row_u8(o, g.rowoff + g.xb, g.nb, pack_u8(pb));
    } else if constexpr (OUT == OUT_I16) {
      int pa[16], pb[16];
      recon_i16<MODE>(ta, fa, pa);
      recon_i16<MODE>(tb, fb, pb);
      int16_t* o = reinterpret_cast<int16_t*>(P.out);
      if (g.na > 0) store_row_i16(o, g.rowoff + g.xa, g.na, pa);
      if (g.nb > 0) store_row_i16(o, g.rowoff + g.xb, g.nb, pb);
    } else {
      float* o = reinterpret_cast<float*>(P.out);
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        float fva, fvb;
        if constexpr (MODE == MODE_MASK) {
          fva = (float)((double)ta[k] / 2304.0);
          fvb = (float)((double)tb[k] / 2304.0);
        } else {
          fva = (float)fa[k];
          fvb = (float)fb[k];
        }
        if (k < g.na) o[g.rowoff + g.xa + k] = fva;
        if (k < g.nb) o[g.rowoff + g.xb + k] = fvb;
      }
    }
    if (!more) break;
  }
}

// Retention or uniform quantisation of block-major coefficients: thread t
// handles the 16 coefficients of row u = t mod 16 of block t / 16.
template <int CFIN, int MODE, int QOUT>
__global__ __launch_bounds__(256) void k_quantise(Params P) {
  const int64_t nrows = P.n_blocks * 16;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nrows;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int u = (int)(t & 15);
    int z[16];
    if constexpr (CFIN == CF_I32) {
      const int4* s = reinterpret_cast<const int4*>(reinterpret_cast<const int*>(P.coef) + t * 16);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int4 q = s[m];
        z[4 * m] = q.x; z[4 * m + 1] = q.y; z[4 * m + 2] = q.z; z[4 * m + 3] = q.w;
      }
    } else {
      const uint4* s = reinterpret_cast<const uint4*>(reinterpret_cast<const int16_t*>(P.coef) + t * 16);
      const uint4 q0 = s[0], q1 = s[1];
      const unsigned w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        z[2 * k] = (int)(short)(w[k] & 0xffffu);
        z[2 * k + 1] = ((int)w[k]) >> 16;
      }
    }
    int r[16];
    if constexpr (MODE == MODE_MASK) {
#pragma unroll
      for (int v = 0; v < 16; ++v) r[v] = P.tables->wkeep[u * 16 + v] ? z[v] : 0;
    } else {
      if constexpr (CFIN == CF_I16C) z[0] += (u == 0) ? 32768 : 0;
#pragma unroll
      for (int v = 0; v < 16; ++v) r[v] = level_of<MODE>(z[v], P.tables->qmul[u * 16 + v], P.tables->qoff);
    }
    if constexpr (QOUT == CF_I32 || QOUT == CF_L32) {
      int4* d = reinterpret_cast<int4*>(reinterpret_cast<int*>(P.qcoef) + t * 16);
#pragma unroll
      for (int m = 0; m < 4; ++m) d[m] = make_int4(r[4 * m], r[4 * m + 1], r[4 * m + 2], r[4 * m + 3]);
    } else {
      unsigned w[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int lo = (QOUT == CF_L16) ? sat16(r[2 * k]) : r[2 * k];
        const int hi = (QOUT == CF_L16) ? sat16(r[2 * k + 1]) : r[2 * k + 1];
        w[k] = ((unsigned)lo & 0xffffu) | ((unsigned)hi << 16);
      }
      uint4* d = reinterpret_cast<uint4*>(reinterpret_cast<int16_t*>(P.qcoef) + t * 16);
      d[0] = make_uint4(w[0], w[1], w[2], w[3]);
      d[1] = make_uint4(w[4], w[5], w[6], w[7]);
    }
  }
}

// Per-image SSE between P.in (IN) and P.in2 (OUT type).
template <int IN>
__global__ __launch_bounds__(kGroupThreads) void k_measure(Params P) {
  const int lane = threadIdx.x & 63, x = lane & 15, p = lane >> 4;
  StripCursor c;
  if (!cursor_init(c, P)) return;
  SseAcc acc;
  acc.init(P);
  int since_flush = 0;
  for (;;) {
    const LaneGeom g = lane_geom(c, x, p);
    if (g.rowok) {
      if constexpr (IN == IN_U8) {
        const uint8_t* a = reinterpret_cast<const uint8_t*>(P.in);
        const uint8_t* b = reinterpret_cast<const uint8_t*>(P.in2);
        if (g.na > 0) acc.lane += sse_u8(load_row_u8(a, g.rowoff + g.xa, 16), load_row_u8(b, g.rowoff + g.xa, 16), g.na);
        if (g.nb > 0) acc.lane += sse_u8(load_row_u8(a, g.rowoff + g.xb, 16), load_row_u8(b, g.rowoff + g.xb, 16), g.nb);
      } else {
        const int16_t* a = reinterpret_cast<const int16_t*>(P.in);
        const int16_t* b = reinterpret_cast<const int16_t*>(P.in2);
        int va[16], vb[16];
        unsigned long long s = 0;
        if (g.na > 0) {
          load_row_i16(a, g.rowoff + g.xa, 16, va);
          load_row_i16(b, g.rowoff + g.xa, 16, vb);
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            const long long d = (k < g.na) ? (long long)(va[k] - vb[k]) : 0;
            s += (unsigned long long)(d * d);
          }
        }
        if (g.nb > 0) {
          load_row_i16(a, g.rowoff + g.xb, 16, va);
          load_row_i16(b, g.rowoff + g.xb, 16, vb);
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            const long long d = (k < g.nb) ? (long long)(va[k] - vb[k]) : 0;
            s += (unsigned long long)(d * d);
          }
        }
        acc.lane += s;
      }
    }
    const int img = c.img;
    const bool changed = cursor_next(c, P);
    const bool done = c.s >= c.s_end;
    if (changed || done || ++since_flush == 1024) {
      acc.flush(P, img);
      since_flush = 0;
    }
    if (done) break;
  }
}

// Hashed noise for the autotuner's scratch input (the chip's clock follows
// its power draw, which depends on the data: a constant input would favour
// launch shapes that are slow on real data).  Bytes: the full 8-bit range;
// 16-bit samples: [-512, 511], the range of prediction residuals.
// Hashed noise for the autotuner's scratch input: kind 0 any bytes, 1 int16
// pairs in [-512, 511], 2 int16 pairs in [-256, 255].
__global__ void k_fill_noise(uint32_t* p, int64_t n, int kind) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t h = (uint32_t)i * 0x9E3779B1u;
    h ^= h >> 15;
    h *= 0x85EBCA77u;
    h ^= h >> 13;
    h *= 0xC2B2AE3Du;
    h ^= h >> 16;
    if (kind == 1) h = (((h & 0x3ffu) - 512u) & 0xffffu) | ((((h >> 16) & 0x3ffu) - 512u) << 16);
    if (kind == 2) h = (((h & 0x1ffu) - 256u) & 0xffffu) | ((((h >> 16) & 0x1ffu) - 256u) << 16);
    p[i] = h;
  }
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// Per-image SSE from the accumulator slots (written to `sse` when given)
// and PSNR = 10 log10(255^2 h w / SSE), +inf for SSE = 0 (Section 4).  One
// wavefront per image, a lane per slot; the slots are cleared after they
// are read, so that every call leaves them at zero for the next one.
__global__ __launch_bounds__(64) void k_sse_finalize(Params P, unsigned long long* sse) {
  const int i = blockIdx.x, l = threadIdx.x;
  unsigned long long* slots = P.sse + (int64_t)i * P.sse_slots;
  unsigned long long v = 0;
  for (int k = l; k < P.sse_slots; k += 64) {
    v += slots[k];
    slots[k] = 0;
  }
  v = wave_sum_u64(v);
  if (l == 0) {
    if (sse) sse[i] = v;
    if (P.psnr) {
      const ImageDesc& d = P.images[i];
      P.psnr[i] = v == 0 ? __builtin_huge_val() : 10.0 * log10(65025.0 * (double)d.h * (double)d.w / (double)v);
    }
  }
}

// Per-image SSE from the per-task partials of the matrix-core fused kernel
// (one workgroup per image; an image's tasks are contiguous), and PSNR.
__global__ __launch_bounds__(kFinishThreads) void k_task_sse_reduce(Params P) { finish_image<false>(P); }

// 1-D transforms of int32 vectors of 16.  A wavefront moves 64 vectors
// (4 KB) per step: each load or store instruction covers 1 KB of
// consecutive bytes (lane l, instruction m: bytes 1024 m + 16 l), and the
// LDS regroups them so that each lane holds one whole vector (rows of 80
// bytes, 16 of them padding, keep the accesses free of bank conflicts).
// The data is streamed once, so the accesses are non-temporal.  Vectors
// past the last whole group of 64 are taken one per lane by wavefront 0.
typedef int v4i __attribute__((ext_vector_type(4)));

template <bool INV>
__device__ __forceinline__ void t_1d(int (&v)[16]) {
  if constexpr (INV) t_inv(v); else t_fwd(v);
}

template <bool INV>
__global__ __launch_bounds__(256) void k_1d(const int32_t* __restrict__ x, int32_t* __restrict__ y, int64_t n) {
  __shared__ v4i lds_all[kWavesPerGroup][64 * 5];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  v4i* L = lds_all[w];
  const int64_t groups = n / 64;
  for (int64_t c = (int64_t)blockIdx.x * kWavesPerGroup + w; c < groups; c += (int64_t)gridDim.x * kWavesPerGroup) {
    const v4i* src = reinterpret_cast<const v4i*>(x) + c * 256;
    v4i q[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) q[m] = __builtin_nontemporal_load(src + m * 64 + l);
#pragma unroll
    for (int m = 0; m < 4; ++m) L[(m * 16 + (l >> 2)) * 5 + (l & 3)] = q[m];
    wave_lds_sync();
    int v[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const v4i t = L[l * 5 + k];
      v[4 * k] = t.x; v[4 * k + 1] = t.y; v[4 * k + 2] = t.z; v[4 * k + 3] = t.w;
    }
    t_1d<INV>(v);
#pragma unroll
    for (int k = 0; k < 4; ++k) L[l * 5 + k] = v4i{v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]};
    wave_lds_sync();
    v4i* dst = reinterpret_cast<v4i*>(y) + c * 256;
#pragma unroll
    for (int m = 0; m < 4; ++m) __builtin_nontemporal_store(L[(m * 16 + (l >> 2)) * 5 + (l & 3)], dst + m * 64 + l);
    wave_lds_sync();
  }
  const int64_t i = groups * 64 + l;
  if (blockIdx.x == 0 && w == 0 && i < n) {
    int v[16];
    const int4* src = reinterpret_cast<const int4*>(x + i * 16);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int4 q = src[m];
      v[4 * m] = q.x; v[4 * m + 1] = q.y; v[4 * m + 2] = q.z; v[4 * m + 3] = q.w;
    }
    t_1d<INV>(v);
    int4* dst = reinterpret_cast<int4*>(y + i * 16);
#pragma unroll
    for (int m = 0; m < 4; ++m) dst[m] = make_int4(v[4 * m], v[4 * m + 1], v[4 * m + 2], v[4 * m + 3]);
  }
}

// ---------------------------------------------------------------------------
// Launchers.
#define ADCT16_LAUNCH(kernel, grid, s, P)                                     \
  do {                                                                        \
    hipLaunchKernelGGL((kernel), dim3(grid), dim3(kGroupThreads), 0, (s), (P)); \
    return hipGetLastError();                                                 \
  } while (0)

hipError_t launch_fill_noise(void* p, int64_t bytes, int kind, hipStream_t s) {
  const int64_t n = bytes / 4;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(k_fill_noise, dim3(grid), dim3(256), 0, s, reinterpret_cast<uint32_t*>(p), n, kind);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u64, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_task_sse_reduce(const Params& P, hipStream_t s) {
  hipLaunchKernelGGL(k_task_sse_reduce, dim3(P.n_images), dim3(kFinishThreads), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_sse_finalize(const Params& P, unsigned long long* sse, hipStream_t s) {
  hipLaunchKernelGGL(k_sse_finalize, dim3(P.n_images), dim3(64), 0, s, P, sse);
  return hipGetLastError();
}

template <int MAT>
static hipError_t valu_forward_m(int in_kind, int coef_kind, const Params& P, int grid, hipStream_t s) {
  if (in_kind == IN_U8) {
    switch (coef_kind) {
      case CF_I32: ADCT16_LAUNCH((k_forward<MAT, IN_U8, CF_I32>), grid, s, P);
      case CF_I16C: ADCT16_LAUNCH((k_forward<MAT, IN_U8, CF_I16C>), grid, s, P);
      case CF_F32: ADCT16_LAUNCH((k_forward<MAT, IN_U8, CF_F32>), grid, s, P);
    }
  } else {
    switch (coef_kind) {
      case CF_I32: ADCT16_LAUNCH((k_forward<MAT, IN_I16, CF_I32>), grid, s, P);
      case CF_F32: ADCT16_LAUNCH((k_forward<MAT, IN_I16, CF_F32>), grid, s, P);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_valu_forward(int mat, int in_kind, int coef_kind, const Params& P, int grid, hipStream_t s) {
  return mat == MAT_WHT ? valu_forward_m<MAT_WHT>(in_kind, coef_kind, P, grid, s)
                        : valu_forward_m<MAT_APPROX>(in_kind, coef_kind, P, grid, s);
}

template <int MAT, int IN, int MODE, int QOUT>
static hipError_t fused_out(int out_kind, const Params& P, int grid, hipStream_t s) {
  constexpr int OUTK = IN == IN_U8 ? OUT_U8 : OUT_I16;
  if (out_kind == OUT_NONE) ADCT16_LAUNCH((k_fused<MAT, IN, MODE, QOUT, OUT_NONE>), grid, s, P);
  if (out_kind == OUTK) ADCT16_LAUNCH((k_fused<MAT, IN, MODE, QOUT, OUTK>), grid, s, P);
  return hipErrorInvalidValue;
}

template <int MAT, int IN>
static hipError_t fused_in(int mode, int qout, int out_kind, const Params& P, int grid, hipStream_t s) {
  if (mode == MODE_MASK) {
    if (qout == CF_NONE) return fused_out<MAT, IN, MODE_MASK, CF_NONE>(out_kind, P, grid, s);
    if (qout == CF_I32) return fused_out<MAT, IN, MODE_MASK, CF_I32>(out_kind, P, grid, s);
    if (IN == IN_U8 && qout == CF_I16C) return fused_out<MAT, IN, MODE_MASK, CF_I16C>(out_kind, P, grid, s);
  } else if (mode == MODE_UNIFORM) {
    if (qout == CF_NONE) return fused_out<MAT, IN, MODE_UNIFORM, CF_NONE>(out_kind, P, grid, s);
    if (qout == CF_L16) return fused_out<MAT, IN, MODE_UNIFORM, CF_L16>(out_kind, P, grid, s);
    if (qout == CF_L32) return fused_out<MAT, IN, MODE_UNIFORM, CF_L32>(out_kind, P, grid, s);
  } else {
    if (qout == CF_NONE) return fused_out<MAT, IN, MODE_DEADZONE, CF_NONE>(out_kind, P, grid, s);
    if (qout == CF_L16) return fused_out<MAT, IN, MODE_DEADZONE, CF_L16>(out_kind, P, grid, s);
    if (qout == CF_L32) return fused_out<MAT, IN, MODE_DEADZONE, CF_L32>(out_kind, P, grid, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_valu_fused(int mat, int in_kind, int mode, int qout_kind, int out_kind, const Params& P,
                             int grid, hipStream_t s) {
  if (mat == MAT_WHT) {
    if (in_kind == IN_U8) return fused_in<MAT_WHT, IN_U8>(mode, qout_kind, out_kind, P, grid, s);
    return fused_in<MAT_WHT, IN_I16>(mode, qout_kind, out_kind, P, grid, s);
  }
  if (in_kind == IN_U8) return fused_in<MAT_APPROX, IN_U8>(mode, qout_kind, out_kind, P, grid, s);
  return fused_in<MAT_APPROX, IN_I16>(mode, qout_kind, out_kind, P, grid, s);
}

template <int MAT, int CFIN, int MODE>
static hipError_t inverse_out(int out_kind, const Params& P, int grid, hipStream_t s) {
  switch (out_kind) {
    case OUT_U8: ADCT16_LAUNCH((k_inverse<MAT, CFIN, MODE, OUT_U8>), grid, s, P);
    case OUT_I16: ADCT16_LAUNCH((k_inverse<MAT, CFIN, MODE, OUT_I16>), grid, s, P);
    case OUT_F32: ADCT16_LAUNCH((k_inverse<MAT, CFIN, MODE, OUT_F32>), grid, s, P);
  }
  return hipErrorInvalidValue;
}

template <int MAT>
static hipError_t valu_inverse_m(int coef_kind, int mode, int out_kind, const Params& P, int grid, hipStream_t s) {
  if (mode == MODE_MASK) {
    if (coef_kind == CF_I32) return inverse_out<MAT, CF_I32, MODE_MASK>(out_kind, P, grid, s);
    if (coef_kind == CF_I16C) return inverse_out<MAT, CF_I16C, MODE_MASK>(out_kind, P, grid, s);
  } else {
    if (coef_kind == CF_L32) return inverse_out<MAT, CF_L32, MODE_UNIFORM>(out_kind, P, grid, s);
    if (coef_kind == CF_L16) return inverse_out<MAT, CF_L16, MODE_UNIFORM>(out_kind, P, grid, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_valu_inverse(int mat, int coef_kind, int mode, int out_kind, const Params& P, int grid,
                               hipStream_t s) {
  return mat == MAT_WHT ? valu_inverse_m<MAT_WHT>(coef_kind, mode, out_kind, P, grid, s)
                        : valu_inverse_m<MAT_APPROX>(coef_kind, mode, out_kind, P, grid, s);
}

hipError_t launch_quantise(int coef_kind, int mode, int qout_kind, const Params& P, hipStream_t s) {
  const int64_t rows = P.n_blocks * 16;
  const int grid = (int)std::min<int64_t>((rows + 255) / 256, 1 << 16);
#define ADCT16_QLAUNCH(K)                                                \
  do {                                                                   \
    hipLaunchKernelGGL((K), dim3(grid), dim3(256), 0, s, P);             \
    return hipGetLastError();                                            \
  } while (0)
  if (mode == MODE_MASK) {
    if (coef_kind == CF_I32 && qout_kind == CF_I32) ADCT16_QLAUNCH((k_quantise<CF_I32, MODE_MASK, CF_I32>));
    if (coef_kind == CF_I16C && qout_kind == CF_I16C) ADCT16_QLAUNCH((k_quantise<CF_I16C, MODE_MASK, CF_I16C>));
  } else if (mode == MODE_UNIFORM) {
    if (coef_kind == CF_I32 && qout_kind == CF_L16) ADCT16_QLAUNCH((k_quantise<CF_I32, MODE_UNIFORM, CF_L16>));
    if (coef_kind == CF_I32 && qout_kind == CF_L32) ADCT16_QLAUNCH((k_quantise<CF_I32, MODE_UNIFORM, CF_L32>));
    if (coef_kind == CF_I16C && qout_kind == CF_L16) ADCT16_QLAUNCH((k_quantise<CF_I16C, MODE_UNIFORM, CF_L16>));
    if (coef_kind == CF_I16C && qout_kind == CF_L32) ADCT16_QLAUNCH((k_quantise<CF_I16C, MODE_UNIFORM, CF_L32>));
  } else {
    if (coef_kind == CF_I32 && qout_kind == CF_L16) ADCT16_QLAUNCH((k_quantise<CF_I32, MODE_DEADZONE, CF_L16>));
    if (coef_kind == CF_I32 && qout_kind == CF_L32) ADCT16_QLAUNCH((k_quantise<CF_I32, MODE_DEADZONE, CF_L32>));
    if (coef_kind == CF_I16C && qout_kind == CF_L16) ADCT16_QLAUNCH((k_quantise<CF_I16C, MODE_DEADZONE, CF_L16>));
    if (coef_kind == CF_I16C && qout_kind == CF_L32) ADCT16_QLAUNCH((k_quantise<CF_I16C, MODE_DEADZONE, CF_L32>));
  }
#undef ADCT16_QLAUNCH
  return hipErrorInvalidValue;
}

hipError_t launch_measure(int in_kind, int out_kind, const Params& P, int grid, hipStream_t s) {
  if (in_kind == IN_U8 && out_kind == OUT_U8) ADCT16_LAUNCH((k_measure<IN_U8>), grid, s, P);
  if (in_kind == IN_I16 && out_kind == OUT_I16) ADCT16_LAUNCH((k_measure<IN_I16>), grid, s, P);
  return hipErrorInvalidValue;
}

// Rate proxy: the length of the signed Exp-Golomb code se(v) of a level v
// (v > 0 maps to code number 2v - 1, v <= 0 to -2v; code number k takes
// 2 floor(log2(k + 1)) + 1 bits).
__device__ __forceinline__ unsigned se_bits(int v) {
  const unsigned k = v > 0 ? 2u * (unsigned)v - 1u : 2u * (unsigned)(-v);
  return 2u * (31u - (unsigned)__builtin_clz(k + 1u)) + 1u;
}

// Per-image sum of se(v) lengths over the block-major levels: one wavefront
// per strip of 8 blocks' worth of levels at a time, walking the image table.
template <int LK>
__global__ __launch_bounds__(256) void k_rate(Params P, unsigned long long* bits) {
  const int lane = threadIdx.x & 63;
  StripCursor c;
  if (!cursor_init(c, P)) return;
  unsigned long long acc = 0;
  int img = c.img;
  for (;;) {
    const int b0 = c.sxi * kStripBlocks;
    const int nb = min(kStripBlocks, c.d.bx - b0);
    const int64_t blk = c.d.block_begin + (int64_t)c.sy * c.d.bx + b0;
    // nb blocks x 256 levels; lane handles 32 consecutive levels per block pair
    unsigned s = 0;
    for (int b = 0; b < nb; ++b) {
      const int64_t base = (blk + b) * 256 + lane * 4;
      int v[4];
      if constexpr (LK == CF_L32) {
        const int4 q = *reinterpret_cast<const int4*>(reinterpret_cast<const int*>(P.qcoef) + base);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
      } else {
        const uint2 q = *reinterpret_cast<const uint2*>(reinterpret_cast<const int16_t*>(P.qcoef) + base);
        v[0] = (int)(short)(q.x & 0xffffu); v[1] = ((int)q.x) >> 16;
        v[2] = (int)(short)(q.y & 0xffffu); v[3] = ((int)q.y) >> 16;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) s += se_bits(v[k]);
    }
    acc += s;
    const bool changed = cursor_next(c, P);
    const bool done = c.s >= c.s_end;
    if (changed || done) {
      const unsigned long long t = wave_sum_u64(acc);
      if (lane == 0) atomicAdd(bits + img, t);
      acc = 0;
      img = c.img;
    }
    if (done) break;
  }
}

hipError_t launch_rate(int level_kind, const Params& P, unsigned long long* bits, hipStream_t s) {
  hipError_t e = launch_zero_u64(bits, P.n_images, s);
  if (e != hipSuccess) return e;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((P.n_strips + kWavesPerGroup - 1) / kWavesPerGroup, 2048));
  if (level_kind == CF_L32) hipLaunchKernelGGL((k_rate<CF_L32>), dim3(grid), dim3(kGroupThreads), 0, s, P, bits);
  else if (level_kind == CF_L16) hipLaunchKernelGGL((k_rate<CF_L16>), dim3(grid), dim3(kGroupThreads), 0, s, P, bits);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_1d(bool inverse, const int32_t* x, int32_t* y, int64_t n, hipStream_t s) {
  const int64_t groups = n / 64;  // whole 64-vector groups, one per wavefront step
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((groups + kWavesPerGroup - 1) / kWavesPerGroup, 1 << 16));
  if (inverse) hipLaunchKernelGGL(k_1d<true>, dim3(grid), dim3(256), 0, s, x, y, n);
  else hipLaunchKernelGGL(k_1d<false>, dim3(grid), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

}  // namespace adct16
