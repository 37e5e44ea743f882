// Matrix-core round trip of 16-bit prediction residuals (the transform
// applied to residual planes, Section 5.3) with the uniform quantiser
// (Section 2: S absorbed into the step) or the deadzone quantiser.
//
// Domain: samples x in [-256, 255] (the difference of two 8-bit samples)
// and a step of at least 8 (uniform q >= 8, deadzone QP >= 22).  Then
// |Y_uv| = |Z_uv| / sqrt(n_u n_v) <= 256 * 16 and every level has |L| <= 512.
// Every stage below is exact; only the final combination rounds, in float64.
//
// Stages for one 16x16 block (lane l = 16 g + q; the operand layout of
// kernels_mfma.hip: lane l holds row q of A and column q of B in the g-th
// quarter of K, the accumulator rows 4g..4g+3 of column q):
//
//   F1  P = (X + 1280) T^T - 20480 e_0.  X + 1280 lies in [1024, 1535],
//       where fp16 steps by 1: its bits are x + 0x6500 (one packed 16-bit
//       add per two samples), and a sample outside [-256, 255] shows in the
//       top 7 bits (the range check).  |P| <= 4096.
//   F2  Z^T = P^T T^T on the two fp16 digits of P (a = fp16_rtz(P), b = P - a
//       in {-1, 0, 1}), one K = 32 product.  |Z| <= 65536.  Lane 16g + q
//       holds Z[q][4g..4g+3].
//   Q   the quantiser's own float32 definition: uniform
//       L = round_half_even(fl32(Z) M), deadzone
//       L = sign(Z) floor(fl32(fl32(|Z|) M) + f) (no fused multiply-add).
//   I1  Y_c = L T_c for four classes c of the rows of T: norm 16 (rows 0, 1,
//       5, 8), the first and the second half of the norm-12 rows (2, 6, 7, 9;
//       10, 13, 14, 15) and norm 8 (3, 4, 11, 12); T_c keeps the rows of
//       class c.  Four rows each: |Y_c| <= 4 * 512 = 2048, fp16-exact.
//   I2  The inverse A' = C_hat^T (step L) C_hat with C_hat = S T is
//           A'/step = sum_{u,v} T[u][i] L[u][v] T[v][j] / sqrt(n_u n_v)
//                   = R0 / 48 + R2 / sqrt(128) + R3 / sqrt(192) + R6 / sqrt(96)
//       with integers R_k: the pairs of equal norm (n_u n_v = 256, 144, 64,
//       1/sqrt(n_u n_v) = w_u / 48 with w = 48 / n = 3, 4, 6) form R0, the
//       mixed pairs (16, 8), (16, 12) and (12, 8) form R2, R3 and R6:
//           R_k[i][j] = sum_u T[u][i] sum_c coef_k(class(u), c) Y_c[u][j].
//       Seven K = 32 products (two Y_c per product); every partial sum is an
//       integer below 2^24.  Lane 16g + q ends with R_k[q][4g..4g+3], four
//       consecutive pixels of row q.
//   x   float64: x = 0.5 + R0 step/48 + R2 step/sqrt(128) + R3 step/sqrt(192)
//       + R6 step/sqrt(96) (fused multiply-adds), pixel = saturate_int16(
//       floor(x)), the rounding half up of the reconstruction.  The error of
//       x is a few units in the last place of terms below 2^18: far below
//       1e-9.
//   SSE sum (x - pixel)^2 with packed 16-bit differences (|difference| <=
//       256 + 8192: the reconstruction of a block has at most twice the
//       energy of the block, Section 2's orthogonality) and dot2.
//
// Memory side: strips of 16 rows x 128 samples, 4 row loads of 16 bytes per
// lane (4 rows x 256 bytes per instruction), regrouped through LDS (272-byte
// rows) into the operand layout and back for the stores.  The next strip's
// rows are requested one strip ahead, unconditionally, from addresses
// clamped into its image (rows past the height read the last row); each
// strip ends with an explicit wait for everything but its own stores.  Edge
// strips (a partial last block, rows past the height) extend their rows in
// LDS and store sample by sample.
#include <type_traits>

#include "mfma_stages.hpp"
#include "task_stream.hpp"

namespace adct16 {

constexpr int kResRow = 68;                  // LDS dwords per strip row (256 B + 16 B)
constexpr int kResWaveLds = 16 * kResRow;    // row dwords per wavefront
// levels of the 8 blocks of a strip staged in LDS: 128 (int16) or 256
// (int32) dwords per block, lane 16g + q at 2 (or 4) dwords per block
template <int QOUT>
constexpr int res_level_dwords() { return QOUT == CF_L16 ? 8 * 128 : QOUT == CF_L32 ? 8 * 256 : 0; }
#ifndef ADCT16_RESID_NB
#define ADCT16_RESID_NB 2
#endif
constexpr int kResNB = ADCT16_RESID_NB;      // blocks carried through the stages together

// Second-pass products: {output k, class pair}.  Pair 0 = (Y_16, Y_8),
// pair 1 = (Y_12a, Y_12b); R2 needs no pair-1 product (a norm-12 Y never
// meets rows of norm 16 or 8 in the (16, 8) class pair).
struct ResidConsts {
  uint2 tq;       // T[q][4g..4g+3]: F1 and F2 B
  float c1;       // F1 accumulator start: -20480 in column 0
  float m[4];     // quantiser multipliers M[q][4g+v]
  uint2 yb[4];    // I1 B per class c: [class(4g+v) == c] T[4g+v][q]
  uint4 rb[7];    // I2 B: R0 p0, R0 p1, R2 p0, R3 p0, R3 p1, R6 p0, R6 p1
};

// The per-lane constants, read from the plan's table (built on the host:
// resid_lane_consts in api.hip), 11 coalesced 16-byte loads per lane.
__device__ __forceinline__ ResidConsts load_resid_consts(int lane, const Tables* tb) {
  uint32_t w[4 * Tables::kResConstGroups];
#pragma unroll
  for (int i = 0; i < Tables::kResConstGroups; ++i) {
    const uint4 v = *reinterpret_cast<const uint4*>(tb->rconst[i][lane]);
    w[4 * i] = v.x;
    w[4 * i + 1] = v.y;
    w[4 * i + 2] = v.z;
    w[4 * i + 3] = v.w;
  }
  ResidConsts k;
  k.tq = make_uint2(w[0], w[1]);
  k.c1 = __builtin_bit_cast(float, w[2]);
#pragma unroll
  for (int v = 0; v < 4; ++v) k.m[v] = __builtin_bit_cast(float, w[3 + v]);
#pragma unroll
  for (int c = 0; c < 4; ++c) k.yb[c] = make_uint2(w[7 + 2 * c], w[8 + 2 * c]);
#pragma unroll
  for (int i = 0; i < 7; ++i) k.rb[i] = make_uint4(w[15 + 4 * i], w[16 + 4 * i], w[17 + 4 * i], w[18 + 4 * i]);
  return k;
}

template <int MODE>
__device__ __forceinline__ float level_f(float z, float m, float f) {
  if constexpr (MODE == MODE_UNIFORM) {
    return __builtin_rintf(z * m);
  } else {
    const float a = floorf(__fadd_rn(__fmul_rn(fabsf(z), m), f));
    return __builtin_copysignf(a, z);
  }
}

// Levels of block b of a strip, lane 16g + q: L[q][4g..4g+3], to the LDS
// staging area (interior strips, written to HBM at the end of the strip)
template <int QOUT>
__device__ __forceinline__ void stage_levels(int* lv, int b, int q, int g, const float (&l)[4]) {
  if constexpr (QOUT == CF_L16) {
    *reinterpret_cast<uint2*>(lv + b * 128 + 8 * q + 2 * g) =
        make_uint2(__builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pk_i16((int)l[0], (int)l[1])),
                   __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pk_i16((int)l[2], (int)l[3])));
  } else if constexpr (QOUT == CF_L32) {
    *reinterpret_cast<int4*>(lv + b * 256 + 16 * q + 4 * g) = make_int4((int)l[0], (int)l[1], (int)l[2], (int)l[3]);
  }
}

// ... read back by the same lane (no synchronisation needed) ...
template <int QOUT>
__device__ __forceinline__ uint4 read_levels(const int* lv, int b, int q, int g) {
  if constexpr (QOUT == CF_L16) {
    const uint2 w = *reinterpret_cast<const uint2*>(lv + b * 128 + 8 * q + 2 * g);
    return make_uint4(w.x, w.y, 0u, 0u);
  } else {
    const int4 w = *reinterpret_cast<const int4*>(lv + b * 256 + 16 * q + 4 * g);
    return make_uint4((unsigned)w.x, (unsigned)w.y, (unsigned)w.z, (unsigned)w.w);
  }
}

// ... and stored to the block-major level buffer.
template <int QOUT, bool NT>
__device__ __forceinline__ void write_levels(void* qcoef, int64_t blk, int q, int g, const uint4& w) {
  const int64_t base = blk * 256 + q * 16 + 4 * g;
  if constexpr (QOUT == CF_L16) {
    typedef unsigned v2u __attribute__((ext_vector_type(2)));
    const v2u v = {w.x, w.y};
    v2u* p = reinterpret_cast<v2u*>(reinterpret_cast<int16_t*>(qcoef) + base);
    if constexpr (NT) __builtin_nontemporal_store(v, p); else *p = v;
  } else {
    const v4u v = {w.x, w.y, w.z, w.w};
    v4u* p = reinterpret_cast<v4u*>(reinterpret_cast<int32_t*>(qcoef) + base);
    if constexpr (NT) __builtin_nontemporal_store(v, p); else *p = v;
  }
}

template <int QOUT, bool NT>
__device__ __forceinline__ void store_levels(void* qcoef, int64_t blk, int q, int g, const float (&l)[4]) {
  const int64_t base = blk * 256 + q * 16 + 4 * g;
  if constexpr (QOUT == CF_L16) {
    typedef unsigned v2u __attribute__((ext_vector_type(2)));
    const v2u v = {__builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pk_i16((int)l[0], (int)l[1])),
                   __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pk_i16((int)l[2], (int)l[3]))};
    v2u* p = reinterpret_cast<v2u*>(reinterpret_cast<int16_t*>(qcoef) + base);
    if constexpr (NT) __builtin_nontemporal_store(v, p); else *p = v;
  } else if constexpr (QOUT == CF_L32) {
    const v4u v = {(unsigned)(int)l[0], (unsigned)(int)l[1], (unsigned)(int)l[2], (unsigned)(int)l[3]};
    v4u* p = reinterpret_cast<v4u*>(reinterpret_cast<int32_t*>(qcoef) + base);
    if constexpr (NT) __builtin_nontemporal_store(v, p); else *p = v;
  }
}

// The round trip of kResNB blocks (blocks b0 .. b0 + kResNB - 1 of the
// strip): operand bits xop[b] (x + 0x6500, dword pair of row q, columns
// 4g..4g+3) -> reconstruction rec[b] (int16 pairs, same layout); levels
// staged in LDS (interior strips) or stored for the blocks b < nstore (EDGE
// strips).
template <int MODE, int QOUT, bool NT, bool EDGE>
__device__ __forceinline__ void resid_blocks(const uint2* xop, uint2* rec, const ResidConsts& k, const double (&cmb)[4],
                                             float f, void* qcoef, int* lv, int b0, int64_t blk0, int nstore, int q,
                                             int g) {
  constexpr int NB = kResNB;
  const f4 zero = {0, 0, 0, 0};
  const f4 c1 = {k.c1, k.c1, k.c1, k.c1};
  f4 z[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) z[b] = mma16(xop[b], k.tq, c1);  // P[4g+v][q]
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const unsigned a0 = h2bits(z[b][0], z[b][1]), a1 = h2bits(z[b][2], z[b][3]);
    const unsigned b0 = residual_pair(a0, z[b][0], z[b][1]), b1 = residual_pair(a1, z[b][2], z[b][3]);
    z[b] = mma32(make_uint4(a0, a1, b0, b1), make_uint4(k.tq.x, k.tq.y, k.tq.x, k.tq.y), zero);  // Z[q][4g+v]
  }
  uint2 lh[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    float l[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) l[v] = level_f<MODE>(z[b][v], k.m[v], f);
    if constexpr (QOUT != CF_NONE) {
      if constexpr (EDGE) {
        if (b < nstore) store_levels<QOUT, NT>(qcoef, blk0 + b, q, g, l);
      } else {
        stage_levels<QOUT>(lv, b0 + b, q, g, l);
      }
    }
    lh[b] = make_uint2(pack_h(l[0], l[1]), pack_h(l[2], l[3]));  // |L| <= 512: exact
  }
  // I1: Y_c[4g+v][q] for the four classes, packed to fp16 (|Y_c| <= 2048)
  uint4 p0[NB], p1[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const f4 y16 = mma16(lh[b], k.yb[0], zero), y12a = mma16(lh[b], k.yb[1], zero);
    const f4 y12b = mma16(lh[b], k.yb[2], zero), y8 = mma16(lh[b], k.yb[3], zero);
    p0[b] = make_uint4(pack_h(y16[0], y16[1]), pack_h(y16[2], y16[3]), pack_h(y8[0], y8[1]), pack_h(y8[2], y8[3]));
    p1[b] = make_uint4(pack_h(y12a[0], y12a[1]), pack_h(y12a[2], y12a[3]), pack_h(y12b[0], y12b[1]),
                       pack_h(y12b[2], y12b[3]));
  }
  // I2 and the float64 combination, one output class at a time
  double x[NB][4];
  {
    f4 r[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) r[b] = mma32(p1[b], k.rb[1], mma32(p0[b], k.rb[0], zero));
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) x[b][v] = __builtin_fma((double)r[b][v], cmb[0], 0.5);
  }
  {
    f4 r[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) r[b] = mma32(p0[b], k.rb[2], zero);
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) x[b][v] = __builtin_fma((double)r[b][v], cmb[1], x[b][v]);
  }
  {
    f4 r[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) r[b] = mma32(p1[b], k.rb[4], mma32(p0[b], k.rb[3], zero));
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) x[b][v] = __builtin_fma((double)r[b][v], cmb[2], x[b][v]);
  }
  {
    f4 r[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) r[b] = mma32(p1[b], k.rb[6], mma32(p0[b], k.rb[5], zero));
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) x[b][v] = __builtin_fma((double)r[b][v], cmb[3], x[b][v]);
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    int px[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) px[v] = (int)__builtin_floor(x[b][v]);
    rec[b] = make_uint2(__builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pk_i16(px[0], px[1])),
                        __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pk_i16(px[2], px[3])));
  }
}

typedef short s2v __attribute__((ext_vector_type(2)));

// sum of squared differences of two int16 pairs (no overflow: |x - rec|
// <= 8448)
__device__ __forceinline__ int sqdiff2(unsigned x, unsigned r) {
  const s2v d = __builtin_bit_cast(s2v, x) - __builtin_bit_cast(s2v, r);
  return __builtin_amdgcn_sdot2(d, d, 0, false);
}

// Samples x in [-256, 255] have operand bits x + 0x6500 in [0x6400, 0x65ff]:
// the top 7 bits of every half are 0x64 >> 1.  The check keeps the OR and
// the AND of all operand dwords of a task.
constexpr unsigned kRangeMask = 0xFE00FE00u, kRangeBits = 0x64006400u;

template <int MODE, int QOUT, int OUT, bool NT>
#ifndef ADCT16_RESID_MIN_WG
#define ADCT16_RESID_MIN_WG 3
#endif
__global__ __launch_bounds__(kGroupThreads, ADCT16_RESID_MIN_WG) void k_mfma_resid(Params P, const ImageDesc* __restrict__ images,
                                                                  const RowTask* __restrict__ rows) {
  constexpr int kWaveDw = kResWaveLds + res_level_dwords<QOUT>();
  __shared__ __attribute__((aligned(16))) int lds_all[kWavesPerGroup * kWaveDw];
  int* lds = lds_all + (threadIdx.x >> 6) * kWaveDw;
  int* lvl = lds + kResWaveLds;  // level staging (interior strips)
  const int lane = threadIdx.x & 63, q = lane & 15, g = lane >> 4, rr = lane >> 4, cc = lane & 15;
  const int64_t W = (int64_t)gridDim.x * kWavesPerGroup;
  int64_t t0 = (int64_t)blockIdx.x * kWavesPerGroup + uniform_int(threadIdx.x >> 6);
  if (t0 >= P.n_rows) return;  // before any load: launches with few tasks leave many wavefronts idle
  const ResidConsts k = load_resid_consts(lane, P.tables);
  const double cmb[4] = {P.tables->rcomb[0], P.tables->rcomb[1], P.tables->rcomb[2], P.tables->rcomb[3]};
  const float f = P.tables->qoff;
  const int16_t* in = reinterpret_cast<const int16_t*>(P.in);
  int16_t* outp = reinterpret_cast<int16_t*>(P.out);
  TaskRegs tr = gather_tasks(images, rows, t0, W, P.n_rows, lane);
  int kk = 0;
  int sy = __builtin_amdgcn_readlane(tr.sy, 0);
  const int run0 = __builtin_amdgcn_readlane(tr.run, 0);
  int sxi = task_run_first(run0);
  ImgGeom d = task_geom(tr, 0);
  int sxe = min(sxi + task_run_count(run0), d.sx);
  auto interior = [](const ImgGeom& dd, int ssy, int ssxi) {
    return (ssxi + 1) * (16 * kStripBlocks) <= dd.w && ssy * 16 + 16 <= dd.h;
  };
  // This lane's 16 bytes of strip (ssy, ssxi) in row load i: row
  // 16 ssy + 4i + rr, samples 8 cc .. 8 cc + 7, clamped into the image: rows
  // past the height read the last row, and a block past the last reads the
  // same half of block 0 (computed on, neither stored nor counted).  Every
  // address lies inside the image, so the loads are unconditional.  The
  // offset is in bytes from the image's first sample: the plan admits this
  // kernel only for images below 2^31 bytes with rows below 2^24 bytes, so
  // one 24-bit multiply-add forms it, against a uniform 64-bit base.
  auto lane_off = [&](const ImgGeom& dd, int ssy, int ssxi, int i) -> unsigned {
    const int y = min(ssy * 16 + 4 * i + rr, dd.h - 1);
    const int blk = ssxi * kStripBlocks + (cc >> 1);
    const int col = (blk < dd.bx ? 16 * blk : 0) + 8 * (cc & 1);
    return __umul24((unsigned)y, 2u * (unsigned)dd.pitch) + 2u * (unsigned)col;
  };
  auto load4 = [&](const ImgGeom& dd, int ssy, int ssxi, uint4 (&v)[4]) {
    const uint8_t* base = reinterpret_cast<const uint8_t*>(in + dd.offset);
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = ld_row16<NT>(base + lane_off(dd, ssy, ssxi, i));
  };
  // LDS rows of a strip: lane (rr, cc) writes its 16 bytes of rows 4i + rr.
  // Called right after an explicit vmcnt(0): the empty asm statements mark
  // the loaded registers as redefined there, so that the compiler's wait
  // tracking no longer holds their loads pending (it would otherwise wait
  // on them, and in hardware on every later store, where the registers are
  // next reused).
  auto rows_to_lds = [&](uint4 (&v)[4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      asm volatile("" : "+v"(v[i].x), "+v"(v[i].y), "+v"(v[i].z), "+v"(v[i].w));
      *reinterpret_cast<uint4*>(lds + (4 * i + rr) * kResRow + 4 * cc) = v[i];
    }
  };
  uint4 nr[4];
  load4(d, sy, sxi, nr);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), other counters unchanged
  rows_to_lds(nr);
  wave_lds_sync();
  unsigned long long lane_sse = 0;
  unsigned r_or = 0u, r_and = 0xFFFFFFFFu;
  int64_t tcur = t0;
  // One strip: its rows (in LDS) through the round trip kResNB blocks at a
  // time.  EDGE strips extend the row past the width, and store and count
  // only the samples inside the image; interior strips store unconditionally.
  auto strip = [&](auto edge_tag, int64_t rowblk, int nb) {
    constexpr bool EDGE = decltype(edge_tag)::value;
    if constexpr (EDGE) {
      // columns past the width repeat column w - 1 of the same row
      const int wl = d.w - sxi * (16 * kStripBlocks);  // columns of this strip inside the image (>= 1)
      if (wl < 16 * kStripBlocks) {
        const int16_t* lrow = reinterpret_cast<const int16_t*>(lds + q * kResRow);
        const unsigned last = (uint16_t)lrow[wl - 1];
#pragma unroll
        for (int b = 0; b < kStripBlocks; ++b) {
          uint2* slot = reinterpret_cast<uint2*>(lds + q * kResRow + 8 * b + 2 * g);
          uint2 v = *slot;
          const int x0 = 16 * b + 4 * g;
          if (x0 + 0 >= wl) v.x = (v.x & 0xffff0000u) | last;
          if (x0 + 1 >= wl) v.x = (v.x & 0x0000ffffu) | (last << 16);
          if (x0 + 2 >= wl) v.y = (v.y & 0xffff0000u) | last;
          if (x0 + 3 >= wl) v.y = (v.y & 0x0000ffffu) | (last << 16);
          *slot = v;
        }
      }
    }
#pragma unroll
    for (int b0 = 0; b0 < kStripBlocks; b0 += kResNB) {
      uint2 xd[kResNB], xop[kResNB], rec[kResNB];
#pragma unroll
      for (int b = 0; b < kResNB; ++b) {
        xd[b] = *reinterpret_cast<const uint2*>(lds + q * kResRow + 8 * (b0 + b) + 2 * g);
        // packed 16-bit adds: no carry between the halves
        xop[b].x = __builtin_bit_cast(unsigned, __builtin_bit_cast(s2v, xd[b].x) + (s2v){0x6500, 0x6500});
        xop[b].y = __builtin_bit_cast(unsigned, __builtin_bit_cast(s2v, xd[b].y) + (s2v){0x6500, 0x6500});
        r_or |= xop[b].x | xop[b].y;
        r_and &= xop[b].x & xop[b].y;
      }
      resid_blocks<MODE, QOUT, NT, EDGE>(xop, rec, k, cmb, f, P.qcoef, lvl, b0, rowblk + b0, nb - b0, q, g);
      // squared error over the samples inside the image (at most 4 kResNB
      // samples of 8448^2 per partial: below 2^31 for kResNB <= 4)
      int part = 0;
      if constexpr (!EDGE) {
#pragma unroll
        for (int b = 0; b < kResNB; ++b) part += sqdiff2(xd[b].x, rec[b].x) + sqdiff2(xd[b].y, rec[b].y);
      } else if (sy * 16 + q < d.h) {
#pragma unroll
        for (int b = 0; b < kResNB; ++b) {
          const int x0 = (sxi * kStripBlocks + b0 + b) * 16 + 4 * g;
          const int n = b0 + b < nb ? min(4, d.w - x0) : 0;  // samples of this lane inside the image
          const unsigned mlo = n >= 2 ? 0xffffffffu : n == 1 ? 0xffffu : 0u;
          const unsigned mhi = n >= 4 ? 0xffffffffu : n == 3 ? 0xffffu : 0u;
          part += sqdiff2(xd[b].x & mlo, rec[b].x & mlo) + sqdiff2(xd[b].y & mhi, rec[b].y & mhi);
        }
      }
      lane_sse += (unsigned)part;
      if constexpr (OUT == OUT_I16) {
        if constexpr (!EDGE) {
#pragma unroll
          for (int b = 0; b < kResNB; ++b) *reinterpret_cast<uint2*>(lds + q * kResRow + 8 * (b0 + b) + 2 * g) = rec[b];
        } else {
          const int y = sy * 16 + q;
          if (y < d.h) {
            int16_t* row = outp + d.offset + (int64_t)y * d.pitch;
#pragma unroll
            for (int b = 0; b < kResNB; ++b) {
              const int x0 = (sxi * kStripBlocks + b0 + b) * 16 + 4 * g;
              const unsigned v[4] = {rec[b].x & 0xffffu, rec[b].x >> 16, rec[b].y & 0xffffu, rec[b].y >> 16};
#pragma unroll
              for (int j = 0; j < 4; ++j)
                if (b0 + b < nb && x0 + j < d.w) row[x0 + j] = (int16_t)v[j];
            }
          }
        }
      }
    }
  };
  // The end of a strip of either kind.  The explicit vmcnt(0) completes the
  // next strip's row loads (issued when this strip began, so it costs
  // little) together with the previous strip's stores, and those rows go to
  // LDS right after it, before any store.  It sits on the one path that both
  // strip kinds share: the compiler's own count ignores stores, so a path
  // around it would leave the row loads pending at the loop head and make
  // the next strip wait there for every store of this one.  An interior
  // strip stores its reconstruction and levels here, from LDS.
  auto strip_end = [&](bool inner, int64_t rowblk) {
    __builtin_amdgcn_s_waitcnt(0x0F70);
    wave_lds_sync();
    uint4 orow[4], lw[kStripBlocks];
    if (inner) {
      if constexpr (OUT == OUT_I16) {
#pragma unroll
        for (int i = 0; i < 4; ++i) orow[i] = *reinterpret_cast<const uint4*>(lds + (4 * i + rr) * kResRow + 4 * cc);
      }
      if constexpr (QOUT != CF_NONE) {
#pragma unroll
        for (int b = 0; b < kStripBlocks; ++b) lw[b] = read_levels<QOUT>(lvl, b, q, g);
      }
      wave_lds_sync();
    }
    rows_to_lds(nr);
    if (inner) {
      if constexpr (OUT == OUT_I16) {  // byte offsets from the image's first sample, as for the loads
        uint8_t* base = reinterpret_cast<uint8_t*>(outp + d.offset);
        const unsigned pb = 2u * (unsigned)d.pitch;
        const unsigned o = __umul24((unsigned)(sy * 16 + rr), pb) + 2u * (unsigned)(sxi * (16 * kStripBlocks) + 8 * cc);
#pragma unroll
        for (int i = 0; i < 4; ++i) st_row16<NT>(base + o + 4u * i * pb, orow[i]);
      }
      if constexpr (QOUT != CF_NONE) {
#pragma unroll
        for (int b = 0; b < kStripBlocks; ++b) write_levels<QOUT, NT>(P.qcoef, rowblk + b, q, g, lw[b]);
      }
    }
  };
  for (;;) {
    const bool task_end = sxi + 1 == sxe;
    int nsy = sy, nsxi = sxi + 1, nsxe = sxe;
    ImgGeom nd = d;
    bool more = true;
    if (task_end) {
      if (++kk == 64) {
        kk = 0;
        t0 += 64 * W;
        tr = gather_tasks(images, rows, t0, W, P.n_rows, lane);
      }
      more = t0 + kk * W < P.n_rows;
      if (more) {
        nsy = __builtin_amdgcn_readlane(tr.sy, kk);
        const int nrun = __builtin_amdgcn_readlane(tr.run, kk);
        nsxi = task_run_first(nrun);
        nd = task_geom(tr, kk);
        nsxe = min(nsxi + task_run_count(nrun), nd.sx);
      } else {
        nsxi = sxi;  // past the last task the rows of this strip are loaded again
      }
    }
    // the next strip's rows requested (this strip's are in LDS)
    load4(nd, nsy, nsxi, nr);
    const int64_t rowblk = d.block_begin + (int64_t)sy * d.bx + sxi * kStripBlocks;
    const bool inner = interior(d, sy, sxi);
    if (inner) {
      strip(std::integral_constant<bool, false>(), rowblk, kStripBlocks);
    } else {
      strip(std::integral_constant<bool, true>(), rowblk, min(kStripBlocks, d.bx - sxi * kStripBlocks));
    }
    strip_end(inner, rowblk);
    wave_lds_sync();
    if (task_end) {
      const unsigned long long task_sum = wave_sum_u64(lane_sse);
      const bool bad = ((r_or & kRangeMask) != kRangeBits) || ((r_and & kRangeMask) != kRangeBits);
      const bool any_bad = __builtin_amdgcn_ballot_w64(bad) != 0;
      if (lane == 0) P.task_sse64[tcur] = any_bad ? ~0ull : task_sum;
      lane_sse = 0;
      r_or = 0u;
      r_and = 0xFFFFFFFFu;
      tcur = t0 + kk * W;
    }
    if (!more) break;
    sy = nsy;
    sxi = nsxi;
    sxe = nsxe;
    d = nd;
  }
}

// Per-image SSE and PSNR from 64-bit task partials; a task that saw a
// sample outside [-256, 255] marks its image (SSE -1, PSNR NaN).
__global__ __launch_bounds__(kFinishThreads) void k_task_sse_reduce64(Params P) { finish_image<true>(P); }

#define ADCT16_RLAUNCH(kernel, grid, s, ...)                                            \
  do {                                                                                 \
    hipLaunchKernelGGL((kernel), dim3(grid), dim3(kGroupThreads), 0, (s), __VA_ARGS__); \
    return hipGetLastError();                                                          \
  } while (0)

template <int MODE, int QOUT, bool NT>
static hipError_t resid_out(int out_kind, const Params& P, int grid, hipStream_t s) {
  if (out_kind == OUT_I16) ADCT16_RLAUNCH((k_mfma_resid<MODE, QOUT, OUT_I16, NT>), grid, s, P, P.images, P.rows);
  if (out_kind == OUT_NONE) ADCT16_RLAUNCH((k_mfma_resid<MODE, QOUT, OUT_NONE, NT>), grid, s, P, P.images, P.rows);
  return hipErrorInvalidValue;
}

template <int MODE, bool NT>
static hipError_t resid_q(int qout_kind, int out_kind, const Params& P, int grid, hipStream_t s) {
  switch (qout_kind) {
    case CF_NONE: return resid_out<MODE, CF_NONE, NT>(out_kind, P, grid, s);
    case CF_L16: return resid_out<MODE, CF_L16, NT>(out_kind, P, grid, s);
    case CF_L32: return resid_out<MODE, CF_L32, NT>(out_kind, P, grid, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mfma_resid(int mode, int qout_kind, int out_kind, bool nt, const Params& P, int grid,
                             hipStream_t s) {
  if (mode == MODE_UNIFORM)
    return nt ? resid_q<MODE_UNIFORM, true>(qout_kind, out_kind, P, grid, s)
              : resid_q<MODE_UNIFORM, false>(qout_kind, out_kind, P, grid, s);
  if (mode == MODE_DEADZONE)
    return nt ? resid_q<MODE_DEADZONE, true>(qout_kind, out_kind, P, grid, s)
              : resid_q<MODE_DEADZONE, false>(qout_kind, out_kind, P, grid, s);
  return hipErrorInvalidValue;
}

hipError_t launch_task_sse_reduce64(const Params& P, hipStream_t s) {
  hipLaunchKernelGGL(k_task_sse_reduce64, dim3(P.n_images), dim3(kFinishThreads), 0, s, P);
  return hipGetLastError();
}

}  // namespace adct16
