// Matrix-core stages of the 16x16 round trip (see kernels_mfma.hip for the
// exactness argument).
#pragma once

#include "device_common.hpp"

namespace adct16 {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __fp16 fp16x2 __attribute__((ext_vector_type(2)));

// The integer matrix (T of Section 2, or the Walsh-Hadamard matrix) and the
// inverse weights w_u = 48 / n_u come from the plan's tables (Tables::tmat,
// Tables::wvec), read once per lane when the constant operands are built.

__device__ __forceinline__ unsigned h2bits(float lo, float hi) {
  return __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(lo, hi));
}

// Pack two fp16-exact values.
__device__ __forceinline__ unsigned pack_h(float lo, float hi) { return h2bits(lo, hi); }

// b = z - a for the two halves of the fp16 pair a (a = fp16_rtz(z)).  The
// differences are exact in fp32 and fp16-representable (|b| below the fp16
// step of a), so the repacking is exact too.
__device__ __forceinline__ unsigned residual_pair(unsigned a, float z0, float z1) {
  const fp16x2 ah = __builtin_bit_cast(fp16x2, a);
  return h2bits(z0 - (float)ah[0], z1 - (float)ah[1]);
}

__device__ __forceinline__ f4 mma16(uint2 a, uint2 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4, a), __builtin_bit_cast(h4, b), c, 0, 0, 0);
}

__device__ __forceinline__ f4 mma32(uint4 a, uint4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
}

// Per-lane constant operands of the round trip.
struct MfmaConsts {
  uint2 tq;      // T[q][4g..4g+3] with row q zeroed when q is not retained (stage-1 B, stage-2 A)
  float c1;      // stage-1 accumulator start: -18432 in column 0
  uint4 w3;      // stage-3 B: w_u T[u][q] 2^-11 for u = 4g..4g+3, twice (one per digit)
  uint2 w4;      // stage-4 A: w_f T[f][q] for f = 4g..4g+3
  f4 c4;         // stage-4 accumulator start: -1536 sum_f w_f T[f][j], j = 4g+v
  uint2 gq;      // collapsed stages 2-3: G[q][4g..4g+3] 2^-11, G = T^T diag(w m) T
};

__device__ __forceinline__ MfmaConsts make_consts(int q, int g, int r_sep, const Tables* tb) {
  const signed char* tm = tb->tmat;  // tm[u * 16 + k] = T[u][k]
  const signed char* kW = tb->wvec;
  auto kT = [tm](int u, int kk) { return (int)tm[u * 16 + kk]; };
  MfmaConsts k;
  const bool keep_q = q < r_sep;
  float t[4], w3[4], w4[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int kk = 4 * g + m;
    t[m] = keep_q ? (float)kT(q, kk) : 0.0f;
    w3[m] = (float)(kW[kk] * kT(kk, q)) * (1.0f / 2048.0f);
    w4[m] = (float)(kW[kk] * kT(kk, q));
  }
  k.tq = make_uint2(pack_h(t[0], t[1]), pack_h(t[2], t[3]));
  k.c1 = (q == 0) ? -18432.0f : 0.0f;
  const unsigned w30 = pack_h(w3[0], w3[1]), w31 = pack_h(w3[2], w3[3]);
  k.w3 = make_uint4(w30, w31, w30, w31);
  k.w4 = make_uint2(pack_h(w4[0], w4[1]), pack_h(w4[2], w4[3]));
  // G = T^T diag(w m) T (m: retained rows / columns of a separable mask) is
  // a symmetric integer matrix with |G| <= 68 (48 for the Walsh-Hadamard
  // matrix); G 2^-11 is exact in fp16.
  float gv[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int kk = 4 * g + m;
    int acc = 0;
    for (int u = 0; u < r_sep; ++u) acc += kW[u] * kT(u, q) * kT(u, kk);
    gv[m] = (float)acc * (1.0f / 2048.0f);
  }
  k.gq = make_uint2(pack_h(gv[0], gv[1]), pack_h(gv[2], gv[3]));
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int j = 4 * g + v;
    int s = 0;
    for (int f = 0; f < 16; ++f) s += kW[f] * kT(f, j);
    k.c4[v] = -1536.0f * (float)s;
  }
  return k;
}

// 4 pixels (one dword) -> (x + 1024) as 4 fp16 values.
__device__ __forceinline__ uint2 bytes_to_h4(unsigned x) {
  return make_uint2(__builtin_amdgcn_perm(0x64646464u, x, 0x04010400u),
                    __builtin_amdgcn_perm(0x64646464u, x, 0x04030402u));
}

// pixel = clamp(floor(N / 2304 + 1/2) + 128, 0, 255) from s = N / 2048
__device__ __forceinline__ unsigned round_pack(f4 s) {
  constexpr float c = 8.0f / 9.0f;           // fl32(2048 / 2304)
  constexpr float off = 128.0f + 1.0f / 4096.0f;
  unsigned r = 0;
  r = __builtin_amdgcn_cvt_pk_u8_f32(__builtin_fmaf(s[0], c, off), 0, r);
  r = __builtin_amdgcn_cvt_pk_u8_f32(__builtin_fmaf(s[1], c, off), 1, r);
  r = __builtin_amdgcn_cvt_pk_u8_f32(__builtin_fmaf(s[2], c, off), 2, r);
  r = __builtin_amdgcn_cvt_pk_u8_f32(__builtin_fmaf(s[3], c, off), 3, r);
  return r;
}

// The batched forms below carry NB blocks through each stage together: the
// NB products of a stage are independent, so each one's latency is covered
// by the others.

// Stage 4 and the rounding for NB blocks, from U' = 1536 + U 2^-11 in v
// (v[b][j] = U'[q][4g+j]).  U' lies in [1024, 2048), where fp16 steps by 1:
// A = floor(U') (the round-toward-zero pack) and B = fract(U') (a multiple
// of 2^-11 in [0, 1)) are both exact in fp16, and
// s = sum_f w_f T[f][j] (A - 1536) + sum_f w_f T[f][j] B = N[q][4g+j] / 2048.
// Two chained products, integer digit first.  One K = 32 product would let
// the hardware add the integer terms (|sum| up to 16 * 6 * 2048) and the
// 2^-11 terms in any order, and such partial sums need 29 significand bits;
// chained, every partial sum stays an integer below 2^24 or a multiple of
// 2^-11 below 2^12.  (Stage 3's K = 32 product is exact: all its terms are
// multiples of 2^-11 and their magnitudes sum below 2^12.)
template <int NB>
__device__ __forceinline__ void stage4_round(f4 (&v)[NB], unsigned* out, const MfmaConsts& k) {
  uint2 lo[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    lo[b] = make_uint2(h2bits(__builtin_amdgcn_fractf(v[b][0]), __builtin_amdgcn_fractf(v[b][1])),
                       h2bits(__builtin_amdgcn_fractf(v[b][2]), __builtin_amdgcn_fractf(v[b][3])));
    v[b] = mma16(k.w4, make_uint2(h2bits(v[b][0], v[b][1]), h2bits(v[b][2], v[b][3])), k.c4);
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) v[b] = mma16(k.w4, lo[b], v[b]);
#pragma unroll
  for (int b = 0; b < NB; ++b) out[b] = round_pack(v[b]);
}

// Forward stages 1-2 for NB blocks: z[b][j] = Z_c[4g+j][q] of block b (fp32, exact).
template <int NB>
__device__ __forceinline__ void fwd_blocks(const unsigned* x, f4 (&z)[NB], const MfmaConsts& k) {
  const f4 c1 = {k.c1, k.c1, k.c1, k.c1};
  const f4 zero = {0, 0, 0, 0};
#pragma unroll
  for (int b = 0; b < NB; ++b) z[b] = mma16(bytes_to_h4(x[b]), k.tq, c1);
#pragma unroll
  for (int b = 0; b < NB; ++b) z[b] = mma16(k.tq, make_uint2(pack_h(z[b][0], z[b][1]), pack_h(z[b][2], z[b][3])), zero);
}

// Inverse stages 3-4 and the rounding for NB blocks of (masked) Z_c.
template <int NB>
__device__ __forceinline__ void inv_blocks(f4 (&z)[NB], unsigned* out, const MfmaConsts& k) {
  const f4 c3 = {1536.0f, 1536.0f, 1536.0f, 1536.0f};
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const unsigned a0 = h2bits(z[b][0], z[b][1]), a1 = h2bits(z[b][2], z[b][3]);
    const unsigned b0 = residual_pair(a0, z[b][0], z[b][1]), b1 = residual_pair(a1, z[b][2], z[b][3]);
    z[b] = mma32(make_uint4(a0, a1, b0, b1), k.w3, c3);
  }
  stage4_round<NB>(z, out, k);
}

// ---------------------------------------------------------------------------
// The round trip as int8 products with int32 accumulation (separable masks).
// With G = T^T diag(w m) T (symmetric, |G| <= 48 for every r x r mask, so
// int8) the exact numerator is N = G Xc G for the centred block Xc = X - 128
// (int8):
//
//   stage 1  V   = Xc G               |V| <= 128 max_n sum_j |G[j][n]| = 13312
//   digits   V   = 256 s1 + s0, s0 = the low byte of V as int8 in
//            [-128, 127], s1 = (V + 128) >> 8 in [-52, 52]
//   stage 2  N^T = s0^T G + 256 s1^T G          (two products, int32)
//
// Every product and sum is an integer below 2^31: exact.  Stage 1 carries
// the 16 pixels of a row in the K slots of lane groups 0 and 1 (the other 16
// slots zero); stage 2 carries one digit of V[4g..4g+3][q] in slots 0..3 of
// lane group g against G[4g..4g+3][q] (slots 4..7 zero), so that lane
// 16g + q ends with N[q][4g..4g+3], four consecutive pixels of row q.
typedef int i4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ i4v mma_i8(uint2 a, uint2 b, i4v c) {
  const long av = (long)(((uint64_t)a.y << 32) | a.x), bv = (long)(((uint64_t)b.y << 32) | b.x);
  return __builtin_amdgcn_mfma_i32_16x16x32_i8(av, bv, c, 0, 0, 0);
}

struct I8Consts {
  uint2 g1;   // stage-1 B: G[8g..8g+7][q] for g < 2, zero otherwise
  uint2 g2;   // stage-2 B: G[4g..4g+3][q] in slots 0..3, zero in slots 4..7
  float c;    // rounding: fl32(8/9) 2^-11 (pixel = fma(N, c, 128 + 2^-12), as round_pack)
};

__device__ __forceinline__ I8Consts make_consts_i8(int q, int g, int r_sep, const Tables* tb) {
  const signed char* tm = tb->tmat;
  const signed char* kW = tb->wvec;
  auto gent = [&](int a, int b) {  // G[a][b]
    int acc = 0;
    for (int u = 0; u < r_sep; ++u) acc += kW[u] * tm[u * 16 + a] * tm[u * 16 + b];
    return acc;
  };
  auto bytes4 = [&](int k0) {
    unsigned r = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) r |= (unsigned)(uint8_t)(signed char)gent(k0 + j, q) << (8 * j);
    return r;
  };
  I8Consts k;
  k.g1 = g < 2 ? make_uint2(bytes4(8 * g), bytes4(8 * g + 4)) : make_uint2(0u, 0u);
  k.g2 = make_uint2(bytes4(4 * g), 0u);
  k.c = (8.0f / 9.0f) * (1.0f / 2048.0f);
  return k;
}

// Bytes `b` (0 or 1) of four int32 values, in order, as one dword.
__device__ __forceinline__ unsigned gather_byte(int v0, int v1, int v2, int v3, unsigned sel) {
  const unsigned lo = __builtin_amdgcn_perm((unsigned)v1, (unsigned)v0, sel);
  const unsigned hi = __builtin_amdgcn_perm((unsigned)v3, (unsigned)v2, sel);
  return __builtin_amdgcn_perm(hi, lo, 0x05040100u);
}

// pixel = clamp(floor(N / 2304 + 1/2) + 128, 0, 255) for integer N: the
// float32 conversion is exact (|N| < 2^24) and fma(N, fl32(8/9) 2^-11, off)
// equals round_pack's fma(N 2^-11, fl32(8/9), off) bit for bit (the factor
// 2^-11 only moves the exponent).
__device__ __forceinline__ unsigned round_pack_i(i4v n, float c) {
  constexpr float off = 128.0f + 1.0f / 4096.0f;
  unsigned r = 0;
  r = __builtin_amdgcn_cvt_pk_u8_f32(__builtin_fmaf((float)n[0], c, off), 0, r);
  r = __builtin_amdgcn_cvt_pk_u8_f32(__builtin_fmaf((float)n[1], c, off), 1, r);
  r = __builtin_amdgcn_cvt_pk_u8_f32(__builtin_fmaf((float)n[2], c, off), 2, r);
  r = __builtin_amdgcn_cvt_pk_u8_f32(__builtin_fmaf((float)n[3], c, off), 3, r);
  return r;
}

// NB blocks from their stage-1 operands xi (raw pixel bytes of row q,
// columns 8g..8g+7, in lanes of groups 0 and 1) to four rounded pixels of
// row q per lane (out[b], the layout of round_pack).
template <int NB>
__device__ __forceinline__ void collapsed_blocks_i8(const uint2* xi, unsigned* out, const I8Consts& k) {
  const i4v zero = {0, 0, 0, 0};
  i4v v[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b)  // centred: flipping the top bit of a byte subtracts 128
    v[b] = mma_i8(make_uint2(xi[b].x ^ 0x80808080u, xi[b].y ^ 0x80808080u), k.g1, zero);
  i4v n0[NB], n1[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const unsigned d0 = gather_byte(v[b][0], v[b][1], v[b][2], v[b][3], 0x0c0c0400u);
    const unsigned d1 = gather_byte(v[b][0] + 128, v[b][1] + 128, v[b][2] + 128, v[b][3] + 128, 0x0c0c0501u);
    n0[b] = mma_i8(make_uint2(d0, 0u), k.g2, zero);
    n1[b] = mma_i8(make_uint2(d1, 0u), k.g2, zero);
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    i4v n;
#pragma unroll
    for (int j = 0; j < 4; ++j) n[j] = (n1[b][j] << 8) + n0[b][j];
    out[b] = round_pack_i(n, k.c);
  }
}

// Separable masks, NB blocks: forward row pass, then U^T = P^T G^T in one
// contraction (the forward column pass, the retention and the inverse column
// pass together: T^T diag(w m) T P = T^T (w .* m .* T P)), then stage 4 and
// the rounding.
template <int NB>
__device__ __forceinline__ void collapsed_blocks(const unsigned* x, unsigned* out, const MfmaConsts& k) {
  const f4 c1 = {k.c1, k.c1, k.c1, k.c1};
  const f4 c3 = {1536.0f, 1536.0f, 1536.0f, 1536.0f};
  f4 v[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) v[b] = mma16(bytes_to_h4(x[b]), k.tq, c1);  // P_c[4g+v][q], columns masked
#pragma unroll
  for (int b = 0; b < NB; ++b)                                               // 1536 + U[q][4g+v] 2^-11
    v[b] = mma16(make_uint2(pack_h(v[b][0], v[b][1]), pack_h(v[b][2], v[b][3])), k.gq, c3);
  stage4_round<NB>(v, out, k);
}

}  // namespace adct16
