// Matrix-core kernels.
//
// 1. The approximate DCT as exact FP16 contractions with FP32 accumulation.
//    T has entries in {0, +1, -1}, so every product below is exact; the
//    argument for exactness of each sum is that every partial sum is an
//    integer (or a multiple of 2^-11) of magnitude below 2^24, whatever the
//    order in which the matrix core adds the terms.  For 8-bit input X
//    (centred Xc = X - 128, |Xc| <= 128) and every retention mask the worst
//    cases (linear programs over the pixel box) are |P| <= 2048 after the row
//    pass, |Z| <= 32768 after the column pass, |U| <= 212544 after the first
//    inverse pass and |N| <= 1648452 for the final numerator.
//
//    stage 1  P  = (X + 1024) T^T - 18432 e_0     (X + 1024 is one v_perm
//             away from the bytes: fp16 bits 0x64xx; the accumulator starts
//             at -18432 in column 0, removing the 1024 offset and centring)
//    stage 2  Z  = T P                      (P is fp16-exact: |P| <= 2048)
//    split    Z  = a + b, a = fp16_rtz(Z), b = Z - a, |b| <= 15
//    stage 3  U' = 1536 + 2^-11 sum_u w_u T[u][i] Z'[u][f]   (both digits)
//    split    U' = A + B, A = fp16_rtz(U') = floor(U') since U' lies in
//             [1024, 2048) where fp16 steps by 1; B in [0, 1), a multiple
//             of 2^-11
//    stage 4  s  = sum_f w_f T[f][j] (A - 1536), then + sum_f w_f T[f][j] B
//             = N 2^-11 with N = T^T (w w^T .* Z') T, the exact numerator of
//             the inverse (the weights w = 48/n come from C_hat = S T)
//    round    pixel = cvt_pk_u8(fma(s, fl32(8/9), 128 + 2^-12)) which equals
//             clamp(floor(N / 2304 + 1/2) + 128, 0, 255) exactly (the bias
//             exceeds the fp32 error and stays below 1/2304 minus it).
//
//    Zonal masks are separable, so they are applied for free by zeroing rows
//    of the constant operands; zig-zag masks are applied to Z.
//
// 2. The exact DCT-II comparison transform on BF16 / F16 matrix cores.
//
// Operand layout (16x16xK, checked on the hardware): lane l = 16 g + q
// holds row q of A and column q of B restricted to the g-th quarter of K;
// the accumulator holds rows 4g..4g+3 of column q.
#include <type_traits>

#include "mfma_stages.hpp"
#include "task_stream.hpp"

namespace adct16 {

// One dword of block row q (columns 4g..4g+3), edge-extended.
__device__ __forceinline__ unsigned load_dword_u8(const uint8_t* img, const ImageDesc& d, int y, int x0) {
  const int64_t off = d.offset + (int64_t)y * d.pitch;
  if (x0 + 3 < d.w) return *reinterpret_cast<const unsigned*>(img + off + x0);
  unsigned r = 0;
  for (int k = 0; k < 4; ++k) r |= (unsigned)img[off + min(x0 + k, d.w - 1)] << (8 * k);
  return r;
}

// Reconstruct the 8 blocks of a strip from their dwords (all lanes busy),
// ADCT16_MFMA_BATCH blocks at a time.
template <bool ZIGZAG, bool COLLAPSE>
__device__ __forceinline__ void roundtrip8(const unsigned (&x)[kStripBlocks], unsigned (&out)[kStripBlocks],
                                           const MfmaConsts& k, const bool (&keepz)[4]) {
  constexpr int NB = ADCT16_MFMA_BATCH;
#pragma unroll
  for (int b0 = 0; b0 < kStripBlocks; b0 += NB) {
    if constexpr (COLLAPSE) {
      collapsed_blocks<NB>(&x[b0], &out[b0], k);
    } else {
      f4 z[NB];
      fwd_blocks<NB>(&x[b0], z, k);
      if constexpr (ZIGZAG) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) z[b][v] = keepz[v] ? z[b][v] : 0.0f;
      }
      inv_blocks<NB>(z, &out[b0], k);
    }
  }
}

__device__ __forceinline__ unsigned sse4(unsigned a, unsigned r) {
  return __builtin_amdgcn_udot4(a, a, 0u, false) + __builtin_amdgcn_udot4(r, r, 0u, false) -
         2u * __builtin_amdgcn_udot4(a, r, 0u, false);
}

// Row-wise 16-byte accesses of interior strips: in half h (0, 1) lane
// 8r + c holds bytes 16c..16c+15 of strip row 8h + r, i.e. row 8h + r of
// block c, so one load or store instruction covers 8 rows x 128 contiguous
// bytes (whole cache lines).  A transpose through LDS (layout L[g][q][b] =
// dword g of row q of block b, 512 dwords per wave) turns this into the
// operand layout (lane 16g + q: dword g of row q of every block) and back;
// the b32 accesses touch 64 consecutive dwords, the b128 ones 2-way at most.
// The row half of the transpose: the strip's rows into LDS.  The kernel
// calls it before issuing the next strip's loads, so that those loads can
// take the registers the rows were in (no register copies per strip).
__device__ __forceinline__ void rows_to_lds(int* lds, int r, int c, const uint4 (&rows)[2]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int o = (8 * h + r) * kStripBlocks + c;
    lds[o] = (int)rows[h].x;
    lds[128 + o] = (int)rows[h].y;
    lds[256 + o] = (int)rows[h].z;
    lds[384 + o] = (int)rows[h].w;
  }
}

// ... and the operand half, after rows_to_lds
__device__ __forceinline__ void lds_to_operands(int* lds, int g, int q, unsigned (&x)[kStripBlocks]) {
  wave_lds_sync();
  const int4* p = reinterpret_cast<const int4*>(lds + g * 128 + q * kStripBlocks);
  const int4 a = p[0], b = p[1];
  x[0] = (unsigned)a.x; x[1] = (unsigned)a.y; x[2] = (unsigned)a.z; x[3] = (unsigned)a.w;
  x[4] = (unsigned)b.x; x[5] = (unsigned)b.y; x[6] = (unsigned)b.z; x[7] = (unsigned)b.w;
  wave_lds_sync();
}

__device__ __forceinline__ void rows_to_operands(int* lds, int r, int c, int g, int q, const uint4 (&rows)[2],
                                                 unsigned (&x)[kStripBlocks]) {
  rows_to_lds(lds, r, c, rows);
  lds_to_operands(lds, g, q, x);
}

__device__ __forceinline__ void operands_to_rows(int* lds, int r, int c, int g, int q, const unsigned (&o)[kStripBlocks],
                                                 uint4 (&rows)[2]) {
  int4* p = reinterpret_cast<int4*>(lds + g * 128 + q * kStripBlocks);
  p[0] = make_int4((int)o[0], (int)o[1], (int)o[2], (int)o[3]);
  p[1] = make_int4((int)o[4], (int)o[5], (int)o[6], (int)o[7]);
  wave_lds_sync();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = (8 * h + r) * kStripBlocks + c;
    rows[h] = make_uint4((unsigned)lds[i], (unsigned)lds[128 + i], (unsigned)lds[256 + i], (unsigned)lds[384 + i]);
  }
  wave_lds_sync();
}

// Both operand layouts of the int8 round trip from the same rows: x[b] =
// dword g of row q of block b (the layout of the rounded output, for the
// error), and for lane groups g < 2 xi[b] = dwords 2g, 2g + 1 of row q (the
// stage-1 operand; zero for g >= 2).
__device__ __forceinline__ void lds_to_operands_i8x(int* lds, int g, int q, unsigned (&x)[kStripBlocks],
                                                    uint2 (&xi)[kStripBlocks]) {
  wave_lds_sync();
  const int4* p = reinterpret_cast<const int4*>(lds + g * 128 + q * kStripBlocks);
  const int4 a = p[0], b = p[1];
  x[0] = (unsigned)a.x; x[1] = (unsigned)a.y; x[2] = (unsigned)a.z; x[3] = (unsigned)a.w;
  x[4] = (unsigned)b.x; x[5] = (unsigned)b.y; x[6] = (unsigned)b.z; x[7] = (unsigned)b.w;
#pragma unroll
  for (int k = 0; k < kStripBlocks; ++k) xi[k] = make_uint2(0u, 0u);
  if (g < 2) {
    const int4* p0 = reinterpret_cast<const int4*>(lds + (2 * g) * 128 + q * kStripBlocks);
    const int4* p1 = reinterpret_cast<const int4*>(lds + (2 * g + 1) * 128 + q * kStripBlocks);
    const int4 a0 = p0[0], a1 = p0[1], c0 = p1[0], c1 = p1[1];
    const int lo[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
    const int hi[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
    for (int k = 0; k < kStripBlocks; ++k) xi[k] = make_uint2((unsigned)lo[k], (unsigned)hi[k]);
  }
  wave_lds_sync();
}

// The per-lane constants and the per-strip work of the fused kernel in its
// three forms: FP16 products (collapsed or explicit Z, zig-zag masks on Z)
// or int8 products (collapsed, separable masks).
template <bool ZIGZAG, bool COLLAPSE, bool I8>
struct RoundTrip {
  static_assert(!I8 || (COLLAPSE && !ZIGZAG), "the int8 form covers separable masks (collapsed)");
  typename std::conditional<I8, I8Consts, MfmaConsts>::type k;
  bool keepz[4];
  __device__ __forceinline__ RoundTrip(int q, int g, const Tables* tb) {
    if constexpr (I8) k = make_consts_i8(q, g, tb->rsep, tb);
    else k = make_consts(q, g, tb->rsep, tb);
#pragma unroll
    for (int v = 0; v < 4; ++v) keepz[v] = tb->wkeep[(4 * g + v) * 16 + q] != 0;
  }
  // the strip's rows (written to LDS by rows_to_lds) -> x (input pixels)
  // and out (rounded reconstruction), dword g of row q of each block
  __device__ __forceinline__ void run(int* lds, int g, int q, unsigned (&x)[kStripBlocks],
                                      unsigned (&out)[kStripBlocks]) const {
    if constexpr (I8) {
      uint2 xi[kStripBlocks];
      lds_to_operands_i8x(lds, g, q, x, xi);
      constexpr int NB = ADCT16_MFMA_BATCH;
#pragma unroll
      for (int b0 = 0; b0 < kStripBlocks; b0 += NB) collapsed_blocks_i8<NB>(&xi[b0], &out[b0], k);
    } else {
      lds_to_operands(lds, g, q, x);
      roundtrip8<ZIGZAG, COLLAPSE>(x, out, k, keepz);
    }
  }
};

// Work distribution: wavefront w of W takes tasks w, w + W, w + 2W, ... of
// the batch (the task table lists equal runs of at most 4 or 16 strips of
// one block row, image by image and row by row) and walks each task
// strip by strip, so that at any time the wavefronts of the chip stream
// through one contiguous window of the batch, while short tasks keep the
// work per wavefront even.  The rows of the next interior strip (possibly
// of the next task) are loaded one strip ahead; the stores of interior
// strips are unconditional, and each branch ends with an explicit wait for
// everything but its own stores, so that the loads of the next strip never
// wait for the stores of the previous one.
template <bool ZIGZAG, bool COLLAPSE, int OUT, bool NT, bool I8>
__global__ __launch_bounds__(kGroupThreads, ADCT16_MFMA_MIN_WG) void k_mfma_fused(
    Params P, const ImageDesc* __restrict__ images, const RowTask* __restrict__ rows) {
  // rows that are not whole cache lines (NT false) keep two strips' areas:
  // the line-aligned stores below combine a strip's output with the
  // previous strip's
  constexpr bool REALIGN = !NT && OUT == OUT_U8;
  constexpr int kAreas = REALIGN ? 2 : 1;
  __shared__ int lds_all[kWavesPerGroup * 512 * kAreas];
  int* const lds_w = lds_all + (threadIdx.x >> 6) * 512 * kAreas;
  int* lds = lds_w;
  const int lane = threadIdx.x & 63, q = lane & 15, g = lane >> 4, r = lane >> 3, c = lane & 7;
  const int64_t W = (int64_t)gridDim.x * kWavesPerGroup;
  int64_t t0 = (int64_t)blockIdx.x * kWavesPerGroup + uniform_int(threadIdx.x >> 6);
  if (t0 >= P.n_rows) return;  // before any load: launches with few tasks leave many wavefronts idle
  const RoundTrip<ZIGZAG, COLLAPSE, I8> rt(q, g, P.tables);
  const uint8_t* in = reinterpret_cast<const uint8_t*>(P.in);
  uint8_t* outp = reinterpret_cast<uint8_t*>(P.out);
  TaskRegs tr = gather_tasks(images, rows, t0, W, P.n_rows, lane);
  int kk = 0;  // current task: t0 + kk W
  int sy = __builtin_amdgcn_readlane(tr.sy, 0);
  const int run0 = __builtin_amdgcn_readlane(tr.run, 0);
  int sxi = task_run_first(run0);
  ImgGeom d = task_geom(tr, 0);
  int sxe = min(sxi + task_run_count(run0), d.sx);  // end of the current task
  int sxf = sxi;                                     // first strip of the current task
  auto interior = [](const ImgGeom& dd, int ssy, int ssxi) {
    return (ssxi + 1) * (16 * kStripBlocks) <= dd.w && ssy * 16 + 16 <= dd.h;
  };
  // this lane's 16 bytes of strip (ssy, ssxi) in half hh: row 16 ssy + 8 hh + r,
  // block 8 ssxi + c.  Edge strips read inside the image: rows past the
  // height read the last row (its edge extension), and a block past the last
  // reads the row's first block (its result is neither stored nor counted).
  // The offset is from the image's first pixel: the plan admits this kernel
  // for images below 2^31 bytes with rows below 2^24 bytes, so one 24-bit
  // multiply-add forms it, against a uniform 64-bit base.
  auto lane_off = [&](const ImgGeom& dd, int ssy, int ssxi, int hh) -> unsigned {
    const int y = min(ssy * 16 + 8 * hh + r, dd.h - 1);
    const int blk = ssxi * kStripBlocks + c;
    return __umul24((unsigned)y, (unsigned)dd.pitch) + (blk < dd.bx ? 16u * (unsigned)blk : 0u);
  };
  uint4 nr[2];
  nr[0] = ld_row16<NT>(in + d.offset + lane_off(d, sy, sxi, 0));
  nr[1] = ld_row16<NT>(in + d.offset + lane_off(d, sy, sxi, 1));
  // complete these loads here rather than at the loop head, where the wait
  // would also cover the previous strip's stores
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), other counters unchanged
  // SSE: per lane over the current task, reduced across the wavefront at
  // the end of the task and stored as that task's partial (at most 16
  // strips x 2048 pixels x 255^2 < 2^32); a second kernel sums the partials
  // of each image.  No atomics: tasks of one image run on many wavefronts at
  // once, and contended atomics would serialise them.
  unsigned lane_sse = 0, sum_aa = 0, sum_rr = 0, sum_ar = 0;
  int64_t tcur = t0;  // index of the current task
  for (;;) {
    // the strip after this one
    const bool task_end = sxi + 1 == sxe;
    int nsy = sy, nsxi = sxi + 1, nsxe = sxe, nsxf = sxf;
    ImgGeom nd = d;
    bool more = true;
    if (task_end) {
      if (++kk == 64) {  // next 64 tasks
        kk = 0;
        t0 += 64 * W;
        tr = gather_tasks(images, rows, t0, W, P.n_rows, lane);
      }
      more = t0 + kk * W < P.n_rows;
      if (more) {
        nsy = __builtin_amdgcn_readlane(tr.sy, kk);
        const int nrun = __builtin_amdgcn_readlane(tr.run, kk);
        nsxi = task_run_first(nrun);
        nsxf = nsxi;
        nd = task_geom(tr, kk);
        nsxe = min(nsxi + task_run_count(nrun), nd.sx);
      }
    }
    const uint4 cr[2] = {nr[0], nr[1]};
    // issued inside each branch below, so that no load is outstanding where
    // the branches join
    auto prefetch = [&]() {
      if (more) {
        nr[0] = ld_row16<NT>(in + nd.offset + lane_off(nd, nsy, nsxi, 0));
        nr[1] = ld_row16<NT>(in + nd.offset + lane_off(nd, nsy, nsxi, 1));
      }
    };
    int* const prev_area = lds;
    if constexpr (REALIGN) lds = lds_w + 512 * (lds == lds_w ? 1 : 0);  // this strip's area
    if (interior(d, sy, sxi)) {
      rows_to_lds(lds, r, c, cr);
      prefetch();
      unsigned x[kStripBlocks], out[kStripBlocks];
      rt.run(lds, g, q, x, out);
      if constexpr (REALIGN) {
        // Rows that are not whole cache lines: a strip's 128-byte row piece
        // straddles two lines, and storing the pieces as they lie leaves
        // every line written in two parts (by this strip and the next),
        // which HBM serves far slower.  Instead each lane writes one
        // 16-byte chunk of a whole aligned line: the line where this
        // strip's piece begins takes its first s chunks (s = the row's
        // offset in the line, in chunks) from the previous strip of the run
        // and the rest from this one; after the run's last interior strip
        // the line it ends in takes that strip's last s chunks.  Stores are
        // unconditional buffer stores, chunks that are not this run's get an
        // offset past the buffer range (the hardware drops them), so that
        // exactly two or four stores follow the prefetch loads.
        int4* p = reinterpret_cast<int4*>(lds + g * 128 + q * kStripBlocks);
        p[0] = make_int4((int)out[0], (int)out[1], (int)out[2], (int)out[3]);
        p[1] = make_int4((int)out[4], (int)out[5], (int)out[6], (int)out[7]);
        wave_lds_sync();
        const bool first_in_run = sxi == sxf;
        const bool tail = task_end || !interior(d, sy, sxi + 1);
        // buffer range: the strip row's 16 rows, from one line before its
        // first row (a line may begin before its row)
        const int64_t row0 = d.offset + (int64_t)sy * 16 * d.pitch;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(outp + row0 - 128, 0, 16 * d.pitch + 256, 0x00020000);
        constexpr unsigned kOffNone = 0x80000000u;  // past the range: dropped
        v4u tl[2];
        unsigned toff[2];
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int rho = 8 * hh + r;
          const int64_t rowb = (int64_t)rho * d.pitch;                 // row start, from row0
          // chunks of the row's first cache line before the row starts
          const int sh = (int)((((uintptr_t)outp + (uint64_t)(row0 + rowb)) & 127) >> 4);
          const int64_t line = rowb + 128 * sxi - 16 * sh;              // this strip's first line, from row0
          const int i0 = rho * kStripBlocks;
          // chunk c of the line: this strip's chunk c - sh, or the previous strip's chunk c + 8 - sh
          const bool own = c >= sh;
          const int* src = own ? lds + i0 + (c - sh) : prev_area + i0 + (c + 8 - sh);
          const v4u v = {(unsigned)src[0], (unsigned)src[128], (unsigned)src[256], (unsigned)src[384]};
          const unsigned off = (own || !first_in_run) ? (unsigned)(line + 128 + 16 * c) : kOffNone;
          __builtin_amdgcn_raw_buffer_store_b128(v, rs, off, 0, 0);
          // the line this strip ends in: its chunks c < sh are this strip's last
          const int* t = lds + i0 + ((c + 8 - sh) & 7);
          tl[hh] = v4u{(unsigned)t[0], (unsigned)t[128], (unsigned)t[256], (unsigned)t[384]};
          toff[hh] = c < sh ? (unsigned)(line + 256 + 16 * c) : kOffNone;
        }
        if (tail) {
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) __builtin_amdgcn_raw_buffer_store_b128(tl[hh], rs, toff[hh], 0, 0);
        }
        // the prefetched rows were issued before these stores: vmcnt(2)
        // completes them (with the tail's two stores it also waits for the
        // first two, which is correct)
        __builtin_amdgcn_s_waitcnt(0x0F72);
      } else if constexpr (OUT == OUT_U8) {
        uint4 orow[2];
        operands_to_rows(lds, r, c, g, q, out, orow);
        st_row16<NT>(outp + d.offset + lane_off(d, sy, sxi, 0), orow[0]);
        st_row16<NT>(outp + d.offset + lane_off(d, sy, sxi, 1), orow[1]);
        // the prefetched rows were issued before these two stores: wait for
        // everything but the stores (vmcnt(2))
        __builtin_amdgcn_s_waitcnt(0x0F72);
      } else {
        __builtin_amdgcn_s_waitcnt(0x0F70);
      }
      // sum (a - r)^2 = sum a^2 + sum r^2 - 2 sum a r, each accumulated in
      // the dot product's own addend
#pragma unroll
      for (int b = 0; b < kStripBlocks; ++b) {
        sum_aa = __builtin_amdgcn_udot4(x[b], x[b], sum_aa, false);
        sum_rr = __builtin_amdgcn_udot4(out[b], out[b], sum_rr, false);
        sum_ar = __builtin_amdgcn_udot4(x[b], out[b], sum_ar, false);
      }
    } else {
      // edge strip: fewer than 8 blocks, a partial last block and / or rows
      // past the height.  The rows were loaded as for interior strips; the
      // partial block's row is extended by its last pixel, and only pixels
      // inside the image are stored and counted.
      const int blk = sxi * kStripBlocks + c;
      const int nvalid = d.w - 16 * blk;  // pixels of this lane's block row inside the image
      uint4 er[2] = {cr[0], cr[1]};
      if (nvalid > 0 && nvalid < 16) {
        er[0] = extend_bytes(er[0], nvalid);
        er[1] = extend_bytes(er[1], nvalid);
      }
      rows_to_lds(lds, r, c, er);
      prefetch();
      unsigned x[kStripBlocks], out[kStripBlocks];
      rt.run(lds, g, q, x, out);
      if constexpr (OUT == OUT_U8) {
        uint4 orow[2];
        operands_to_rows(lds, r, c, g, q, out, orow);
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int y = sy * 16 + 8 * hh + r;
          if (y < d.h && nvalid > 0) {
            uint8_t* o = outp + d.offset + (int64_t)y * d.pitch + 16 * blk;
            if (nvalid >= 16) {
              *reinterpret_cast<uint4*>(o) = orow[hh];
            } else {
              for (int j = 0; j < nvalid; ++j) o[j] = (uint8_t)byte_of(orow[hh], j);
            }
          }
        }
      }
      // SSE over the pixels inside the image, in the operand layout (lane
      // 16 g + q: row q, columns 4g..4g+3 of each block)
      if (sy * 16 + q < d.h) {
#pragma unroll
        for (int b = 0; b < kStripBlocks; ++b) {
          const int n = min(4, d.w - ((sxi * kStripBlocks + b) * 16 + 4 * g));
          if (n > 0) {
            const unsigned m = n >= 4 ? 0xffffffffu : ((1u << (8 * n)) - 1u);
            lane_sse += sse4(x[b] & m, out[b] & m);
          }
        }
      }
      __builtin_amdgcn_s_waitcnt(0x0F70);
    }
    if (task_end) {
      // modular arithmetic: the true lane total is below 2^32
      const unsigned task_sum = wave_sum_u32(lane_sse + sum_aa + sum_rr - 2u * sum_ar);
      if (lane == 0) P.task_sse[tcur] = task_sum;
      lane_sse = sum_aa = sum_rr = sum_ar = 0;
      tcur = t0 + kk * W;
    }
    if (!more) break;
    sy = nsy;
    sxi = nsxi;
    sxe = nsxe;
    sxf = nsxf;
    d = nd;
  }
}

// ---------------------------------------------------------------------------
// Forward transform as int8 products with int32 accumulation (exact: every
// operand is a small integer and int32 sums do not round).
//
//   row pass     P = Xc T^T, Xc = X - 128 in int8 (the pixel byte with its
//                top bit flipped); K = 16 of the instruction's 32 slots
//                carry data, the rest are zero.  |P| <= 2048.
//   column pass  Z^T = P^T T^T with P split into signed base-64 digits,
//                P = 64 hi + lo, lo = P & 63 in [0, 63], hi = P >> 6 in
//                [-32, 31]; each lane packs the digits of the four P values
//                it holds (rows 4g..4g+3 of column q) into its 8 K slots, and
//                the constant operand carries T and 64 T in the same slots,
//                so one instruction forms T P.  Stage 2 runs transposed:
//                lane 16g + q ends with Z[q][4g..4g+3].
//   DC           Z = Zc + 32768 at (0, 0) for int32 output (accumulator
//                start); the centred int16 form is Zc itself.

// Bytes 0 of four int32 values, in order, as one dword.
__device__ __forceinline__ unsigned pack_low_bytes(int a, int b, int c, int d) {
  const unsigned ab = __builtin_amdgcn_perm((unsigned)b, (unsigned)a, 0x0c0c0400u);
  const unsigned cd = __builtin_amdgcn_perm((unsigned)d, (unsigned)c, 0x0c0c0400u);
  return __builtin_amdgcn_perm(cd, ab, 0x05040100u);
}

__device__ __forceinline__ unsigned t_bytes(const signed char* tm, int row, int c0, int scale = 1) {
  unsigned r = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) r |= (unsigned)(uint8_t)(scale * tm[row * 16 + c0 + j]) << (8 * j);
  return r;
}

// ---------------------------------------------------------------------------
// Forward only: Z (int32) or the centred int16 form, block-major, in the
// FP16 form (stages 1 and 2 above, stage 2 transposed: Z^T = P^T T^T) or
// the int8 form.  Either way lane 16g + q ends with Z[q][4g..4g+3] of each
// block, so one store instruction writes a whole block (1 KB of int32 or
// 512 B of int16) contiguously.  Strips are read and scheduled as in the
// fused kernel: 8 rows x 128 bytes per load instruction, regrouped through
// LDS, tasks dealt out cyclically, rows loaded a strip ahead.
enum FwdForm { FWD_F16 = 0, FWD_I8 = 1 };

// Int8 operands: lanes 16g + q with g < 2 take dwords 2g and 2g + 1 of row
// q of every block (8 bytes of the K = 32 slots), the others zero.
__device__ __forceinline__ void rows_to_operands_i8(int* lds, int r, int c, int g, int q, const uint4 (&rows)[2],
                                                    uint2 (&x)[kStripBlocks]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int o = (8 * h + r) * kStripBlocks + c;
    lds[o] = (int)rows[h].x;
    lds[128 + o] = (int)rows[h].y;
    lds[256 + o] = (int)rows[h].z;
    lds[384 + o] = (int)rows[h].w;
  }
  wave_lds_sync();
#pragma unroll
  for (int b = 0; b < kStripBlocks; ++b) x[b] = make_uint2(0u, 0u);
  if (g < 2) {
    const int4* p0 = reinterpret_cast<const int4*>(lds + (2 * g) * 128 + q * kStripBlocks);
    const int4* p1 = reinterpret_cast<const int4*>(lds + (2 * g + 1) * 128 + q * kStripBlocks);
    const int4 a0 = p0[0], a1 = p0[1], c0 = p1[0], c1 = p1[1];
    const int lo[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
    const int hi[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
    for (int b = 0; b < kStripBlocks; ++b) x[b] = make_uint2((unsigned)lo[b], (unsigned)hi[b]);
  }
  wave_lds_sync();
}

struct FwdConsts {
  MfmaConsts k;  // FP16 form
  uint2 b1, b2;  // int8 form: stage-1 and stage-2 B operands
};

template <int FORM>
__device__ __forceinline__ FwdConsts fwd_consts(int q, int g, const Tables* tb) {
  FwdConsts f;
  if constexpr (FORM == FWD_F16) {
    f.k = make_consts(q, g, 16, tb);
  } else {
    // stage-1 B: T[q][8g..8g+7] for g < 2 (K = image column), zero otherwise;
    // stage-2 B: column u = q; slots j < 4: T[q][4g + j], slots j >= 4: 64 T[q][4g + j - 4]
    const signed char* tm = tb->tmat;
    f.b1 = g < 2 ? make_uint2(t_bytes(tm, q, 8 * g), t_bytes(tm, q, 8 * g + 4)) : make_uint2(0u, 0u);
    f.b2 = make_uint2(t_bytes(tm, q, 4 * g), t_bytes(tm, q, 4 * g, 64));
  }
  return f;
}

// Z[q][4g..4g+3] of one block from its operand (FP16 form: dword g of row q;
// int8 form: the raw bytes, centred here).
template <int FORM, int CF>
__device__ __forceinline__ int4 fwd_z(unsigned x, uint2 xi, const FwdConsts& f, int q, int g) {
  if constexpr (FORM == FWD_F16) {
    const f4 c1 = {f.k.c1, f.k.c1, f.k.c1, f.k.c1};
    const f4 p = mma16(bytes_to_h4(x), f.k.tq, c1);  // P_c[4g+v][q]
    const uint2 ph = make_uint2(pack_h(p[0], p[1]), pack_h(p[2], p[3]));
    const f4 zero = {0, 0, 0, 0};
    const f4 zt = mma16(ph, f.k.tq, zero);  // Z_c[q][4g+v]
    int4 z = make_int4((int)zt[0], (int)zt[1], (int)zt[2], (int)zt[3]);
    if (CF == CF_I32 && q == 0 && g == 0) z.x += 32768;  // undo the centring at (0, 0)
    return z;
  } else {
    const uint2 xc = g < 2 ? make_uint2(xi.x ^ 0x80808080u, xi.y ^ 0x80808080u) : make_uint2(0u, 0u);
    const i4v zero = {0, 0, 0, 0};
    const i4v p = mma_i8(xc, f.b1, zero);  // P[4g+v][q]
    const uint2 digits = make_uint2(pack_low_bytes(p[0], p[1], p[2], p[3]) & 0x3f3f3f3fu,
                                    pack_low_bytes(p[0] >> 6, p[1] >> 6, p[2] >> 6, p[3] >> 6));
    i4v init = {0, 0, 0, 0};
    if (CF == CF_I32 && q == 0 && g == 0) init[0] = 32768;
    const i4v z = mma_i8(digits, f.b2, init);  // Z[q][4g+v]
    return make_int4(z[0], z[1], z[2], z[3]);
  }
}

template <int CF, bool NT>
__device__ __forceinline__ void store_z(void* coef, int64_t blk, int q, int g, int4 z) {
  const int64_t base = blk * 256 + q * 16 + 4 * g;
  if constexpr (CF == CF_I32) {
    v4u* p = reinterpret_cast<v4u*>(reinterpret_cast<int*>(coef) + base);
    const v4u v = {(unsigned)z.x, (unsigned)z.y, (unsigned)z.z, (unsigned)z.w};
    if constexpr (NT) __builtin_nontemporal_store(v, p); else *p = v;
  } else {
    typedef unsigned v2u __attribute__((ext_vector_type(2)));
    v2u* p = reinterpret_cast<v2u*>(reinterpret_cast<int16_t*>(coef) + base);
    const v2u v = {((unsigned)z.x & 0xffffu) | ((unsigned)z.y << 16), ((unsigned)z.z & 0xffffu) | ((unsigned)z.w << 16)};
    if constexpr (NT) __builtin_nontemporal_store(v, p); else *p = v;
  }
}

template <int FORM, int CF, bool NT>
__global__ __launch_bounds__(kGroupThreads) void k_mfma_forward(Params P, const ImageDesc* __restrict__ images,
                                                                const RowTask* __restrict__ rows) {
  __shared__ int lds_all[kWavesPerGroup * 512];
  int* lds = lds_all + (threadIdx.x >> 6) * 512;
  const int lane = threadIdx.x & 63, q = lane & 15, g = lane >> 4, r = lane >> 3, c = lane & 7;
  const int64_t W = (int64_t)gridDim.x * kWavesPerGroup;
  int64_t t0 = (int64_t)blockIdx.x * kWavesPerGroup + uniform_int(threadIdx.x >> 6);
  if (t0 >= P.n_rows) return;  // before any load
  const FwdConsts f = fwd_consts<FORM>(q, g, P.tables);
  const uint8_t* in = reinterpret_cast<const uint8_t*>(P.in);
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
  auto lane_off = [&](const ImgGeom& dd, int ssy, int ssxi) {
    return dd.offset + (int64_t)(ssy * 16 + r) * dd.pitch + ssxi * (16 * kStripBlocks) + 16 * c;
  };
  uint4 nr[2] = {make_uint4(0, 0, 0, 0), make_uint4(0, 0, 0, 0)};
  if (interior(d, sy, sxi)) {
    const int64_t o = lane_off(d, sy, sxi);
    nr[0] = ld_row16<NT>(in + o);
    nr[1] = ld_row16<NT>(in + o + 8 * (int64_t)d.pitch);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), other counters unchanged
  }
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
      }
    }
    const uint4 cr[2] = {nr[0], nr[1]};
    auto prefetch = [&]() {
      if (more && interior(nd, nsy, nsxi)) {
        const int64_t o = lane_off(nd, nsy, nsxi);
        nr[0] = ld_row16<NT>(in + o);
        nr[1] = ld_row16<NT>(in + o + 8 * (int64_t)nd.pitch);
      }
    };
    const int64_t rowblk = d.block_begin + (int64_t)sy * d.bx + sxi * kStripBlocks;
    if (interior(d, sy, sxi)) {
      prefetch();
      unsigned x[kStripBlocks] = {};
      uint2 xi[kStripBlocks] = {};
      if constexpr (FORM == FWD_F16) rows_to_operands(lds, r, c, g, q, cr, x);
      else rows_to_operands_i8(lds, r, c, g, q, cr, xi);
#pragma unroll
      for (int b = 0; b < kStripBlocks; ++b) store_z<CF, NT>(P.coef, rowblk + b, q, g, fwd_z<FORM, CF>(x[b], xi[b], f, q, g));
      // the prefetched rows were issued before the 8 stores: wait for
      // everything but the stores (vmcnt(8))
      __builtin_amdgcn_s_waitcnt(0x0F78);
    } else {
      prefetch();
      // edge strip: dword loads, the last column / row repeated
      const int y = min(sy * 16 + q, d.h - 1);
      const int b0 = sxi * kStripBlocks;
      const int nb = min(kStripBlocks, d.bx - b0);
      unsigned x[kStripBlocks];
      uint2 xi[kStripBlocks];
#pragma unroll
      for (int b = 0; b < kStripBlocks; ++b) {
        x[b] = 0u;
        xi[b] = make_uint2(0u, 0u);
        if (b < nb) {
          if constexpr (FORM == FWD_F16) {
            x[b] = load_dword_edge(in, d, y, (b0 + b) * 16 + 4 * g);
          } else if (g < 2) {
            const int x0 = (b0 + b) * 16 + 8 * g;
            xi[b] = make_uint2(load_dword_edge(in, d, y, x0), load_dword_edge(in, d, y, x0 + 4));
          }
        }
      }
#pragma unroll
      for (int b = 0; b < kStripBlocks; ++b)
        if (b < nb) store_z<CF, false>(P.coef, rowblk + b, q, g, fwd_z<FORM, CF>(x[b], xi[b], f, q, g));
      __builtin_amdgcn_s_waitcnt(0x0F70);
    }
    if (!more) break;
    sy = nsy;
    sxi = nsxi;
    sxe = nsxe;
    d = nd;
  }
}

// ---------------------------------------------------------------------------
// Forward transform of 16-bit input (any int16 sample, e.g. prediction
// residuals) as int8 products with int32 accumulation, exact.  Every value
// is split into three base-64 digits, v = 4096 d2 + 64 d1 + d0 with d0, d1
// in [0, 63] and d2 = v >> 12 signed:
//
//   row pass     X: d2 in [-8, 7].  One K = 32 product takes d0 (slots of
//                lane groups g < 2) and d1 (g >= 2) against [T | 64 T], a
//                second takes d2 against T; P = first + (second << 12).
//                |P| <= 524288.
//   column pass  P: d2 in [-128, 127]; the same two products with the
//                forward kernel's operand layout (lane 16g + q holds the
//                digits of P[4g..4g+3][q]); Z = first + (second << 12),
//                |Z| <= 2^23.
//
// Strips are 16 rows x 128 samples (256 bytes per row); a load instruction
// covers 4 rows x 256 bytes (lane l: row l / 16, 16-byte chunk l % 16).  The
// LDS regroups the rows (272-byte rows: conflict-free reads) so that lane
// 16g + q holds the 8 samples of row q, columns 8 (g & 1) .. + 7 of a block.
constexpr int kI16Row = 68;                  // LDS dwords per strip row (256 B + 16 B)
constexpr int kI16WaveLds = 16 * kI16Row;    // dwords per wavefront

// Bytes 0 and 2 of four dwords, in order (the low bytes of 8 packed
// 16-bit values).
__device__ __forceinline__ uint2 even_bytes(unsigned a, unsigned b, unsigned c, unsigned d) {
  return make_uint2(__builtin_amdgcn_perm(b, a, 0x06040200u), __builtin_amdgcn_perm(d, c, 0x06040200u));
}

// Row-pass operands of 8 samples (packed 16-bit pairs in `w`): the first
// product's digit (d0, or d1 when `sh` = 6) and the second's (d2, or zero
// for lane groups g >= 2).
__device__ __forceinline__ void i16_row_digits(const uint4& w, int sh, bool top, uint2& a1, uint2& a2) {
  const unsigned m = 0x003F003Fu;
  a1 = even_bytes((w.x >> sh) & m, (w.y >> sh) & m, (w.z >> sh) & m, (w.w >> sh) & m);
  typedef short s2 __attribute__((ext_vector_type(2)));
  auto hi = [](unsigned v) { return __builtin_bit_cast(unsigned, __builtin_bit_cast(s2, v) >> (short)12); };
  const uint2 d2 = even_bytes(hi(w.x), hi(w.y), hi(w.z), hi(w.w));
  a2 = top ? d2 : make_uint2(0u, 0u);
}

template <bool NT>
__global__ __launch_bounds__(kGroupThreads) void k_mfma_forward_i16(Params P, const ImageDesc* __restrict__ images,
                                                                    const RowTask* __restrict__ rows) {
  __shared__ __attribute__((aligned(16))) int lds_all[kWavesPerGroup * kI16WaveLds];
  int* lds = lds_all + (threadIdx.x >> 6) * kI16WaveLds;
  const int lane = threadIdx.x & 63, q = lane & 15, g = lane >> 4, rr = lane >> 4, cc = lane & 15;
  const signed char* tm = P.tables->tmat;
  // row pass B: lane (n = q, g): T[n][8 (g & 1) + j], times 64 for g >= 2
  const uint2 b1 = make_uint2(t_bytes(tm, q, 8 * (g & 1), g < 2 ? 1 : 64), t_bytes(tm, q, 8 * (g & 1) + 4, g < 2 ? 1 : 64));
  // column pass B (as in the 8-bit int8 form): slots j < 4 T[q][4g + j], j >= 4 64 T[q][4g + j - 4]
  const uint2 b2 = make_uint2(t_bytes(tm, q, 4 * g), t_bytes(tm, q, 4 * g, 64));
  const int sh = g < 2 ? 0 : 6;
  const int16_t* in = reinterpret_cast<const int16_t*>(P.in);
  const int64_t W = (int64_t)gridDim.x * kWavesPerGroup;
  int64_t t0 = (int64_t)blockIdx.x * kWavesPerGroup + uniform_int(threadIdx.x >> 6);
  if (t0 >= P.n_rows) return;
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
  // this lane's first 16 bytes of strip (ssy, ssxi): row 16 ssy + rr, chunk cc (elements)
  auto lane_off = [&](const ImgGeom& dd, int ssy, int ssxi) {
    return dd.offset + (int64_t)(ssy * 16 + rr) * dd.pitch + ssxi * (16 * kStripBlocks) + 8 * cc;
  };
  auto load4 = [&](const ImgGeom& dd, int ssy, int ssxi, uint4 (&v)[4]) {
    const int64_t o = lane_off(dd, ssy, ssxi);
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = ld_row16<NT>(reinterpret_cast<const uint8_t*>(in + o + 4 * i * (int64_t)dd.pitch));
  };
  uint4 nr[4] = {};
  if (interior(d, sy, sxi)) {
    load4(d, sy, sxi, nr);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), other counters unchanged
  }
  // Z[q][4g..4g+3] of one block from its 8 samples of row q (columns 8 (g & 1) ..)
  auto block_z = [&](const uint4& w) {
    uint2 a1, a2;
    i16_row_digits(w, sh, g < 2, a1, a2);
    const i4v zero = {0, 0, 0, 0};
    const i4v p1 = mma_i8(a1, b1, zero), p2 = mma_i8(a2, b1, zero);
    int pv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) pv[v] = p1[v] + (p2[v] << 12);  // P[4g+v][q]
    const uint2 c1 = make_uint2(pack_low_bytes(pv[0] & 63, pv[1] & 63, pv[2] & 63, pv[3] & 63),
                                pack_low_bytes((pv[0] >> 6) & 63, (pv[1] >> 6) & 63, (pv[2] >> 6) & 63, (pv[3] >> 6) & 63));
    const uint2 c2 = make_uint2(pack_low_bytes(pv[0] >> 12, pv[1] >> 12, pv[2] >> 12, pv[3] >> 12), 0u);
    const i4v z1 = mma_i8(c1, b2, zero), z2 = mma_i8(c2, b2, zero);
    return make_int4(z1[0] + (z2[0] << 12), z1[1] + (z2[1] << 12), z1[2] + (z2[2] << 12), z1[3] + (z2[3] << 12));
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
      }
    }
    const uint4 cr[4] = {nr[0], nr[1], nr[2], nr[3]};
    auto prefetch = [&]() {
      if (more && interior(nd, nsy, nsxi)) load4(nd, nsy, nsxi, nr);
    };
    const int64_t rowblk = d.block_begin + (int64_t)sy * d.bx + sxi * kStripBlocks;
    if (interior(d, sy, sxi)) {
      prefetch();
#pragma unroll
      for (int i = 0; i < 4; ++i)
        *reinterpret_cast<uint4*>(lds + (4 * i + rr) * kI16Row + 4 * cc) = cr[i];
      wave_lds_sync();
      uint4 w[kStripBlocks];
#pragma unroll
      for (int b = 0; b < kStripBlocks; ++b)
        w[b] = *reinterpret_cast<const uint4*>(lds + q * kI16Row + 4 * (2 * b + (g & 1)));
      wave_lds_sync();
#pragma unroll
      for (int b = 0; b < kStripBlocks; ++b) store_z<CF_I32, NT>(P.coef, rowblk + b, q, g, block_z(w[b]));
      __builtin_amdgcn_s_waitcnt(0x0F78);  // all but the 8 stores: the prefetched rows are in
    } else {
      prefetch();
      // edge strip: row q (the last row repeated), columns past the width
      // repeat the last one
      const int y = min(sy * 16 + q, d.h - 1);
      const int b0 = sxi * kStripBlocks;
      const int nb = min(kStripBlocks, d.bx - b0);
      const int16_t* row = in + d.offset + (int64_t)y * d.pitch;
#pragma unroll
      for (int b = 0; b < kStripBlocks; ++b) {
        if (b < nb) {
          const int x0 = (b0 + b) * 16 + 8 * (g & 1);
          unsigned v[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const unsigned lo = (uint16_t)row[min(x0 + 2 * j, d.w - 1)];
            const unsigned hi = (uint16_t)row[min(x0 + 2 * j + 1, d.w - 1)];
            v[j] = lo | (hi << 16);
          }
          store_z<CF_I32, false>(P.coef, rowblk + b, q, g, block_z(make_uint4(v[0], v[1], v[2], v[3])));
        }
      }
      __builtin_amdgcn_s_waitcnt(0x0F70);
    }
    if (!more) break;
    sy = nsy;
    sxi = nsxi;
    sxe = nsxe;
    d = nd;
  }
}

// ---------------------------------------------------------------------------
// Exact DCT-II comparison transform, Y = C X C^T, operands rounded to BF16
// or F16, FP32 accumulation.  Stage 2 runs transposed for row-wise stores.
__device__ __forceinline__ float dct_c(int k, int m) {
  const float a = k == 0 ? 0.25f : 0.35355339059327373f;
  return a * cospif((float)((2 * m + 1) * k) / 32.0f);
}

template <int PREC>
__device__ __forceinline__ unsigned pack2(float a, float b) {
  if constexpr (PREC == ADCT16_F16) {
    const _Float16 ha = (_Float16)a, hb = (_Float16)b;  // round to nearest
    return (unsigned)__builtin_bit_cast(unsigned short, ha) | ((unsigned)__builtin_bit_cast(unsigned short, hb) << 16);
  } else {
    const __bf16 ha = (__bf16)a, hb = (__bf16)b;  // round to nearest
    return (unsigned)__builtin_bit_cast(unsigned short, ha) | ((unsigned)__builtin_bit_cast(unsigned short, hb) << 16);
  }
}

template <int PREC>
__device__ __forceinline__ f4 mma_p(uint2 a, uint2 b, f4 c) {
  if constexpr (PREC == ADCT16_F16)
    return __builtin_amdgcn_mfma_f32_16x16x16f16(__builtin_bit_cast(h4, a), __builtin_bit_cast(h4, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a), __builtin_bit_cast(s4, b), c, 0, 0, 0);
}

template <int IN, int PREC>
__global__ __launch_bounds__(kGroupThreads) void k_dct(Params P, float* Y) {
  const int lane = threadIdx.x & 63, q = lane & 15, g = lane >> 4;
  // C[q][4g..4g+3] rounded to the operand type: stage-1 B (C^T) and stage-2 B.
  const uint2 cq = make_uint2(pack2<PREC>(dct_c(q, 4 * g), dct_c(q, 4 * g + 1)),
                              pack2<PREC>(dct_c(q, 4 * g + 2), dct_c(q, 4 * g + 3)));
  StripCursor c;
  if (!cursor_init(c, P)) return;
  do {
    const int y = min(c.sy * 16 + q, c.d.h - 1);
    const int b0 = c.sxi * kStripBlocks;
    const int nb = min(kStripBlocks, c.d.bx - b0);
    const int64_t rowblk = c.d.block_begin + (int64_t)c.sy * c.d.bx + b0;
    for (int b = 0; b < nb; ++b) {
      const int x0 = (b0 + b) * 16 + 4 * g;
      float xv[4];
      if constexpr (IN == IN_U8) {
        const unsigned xd = load_dword_u8(reinterpret_cast<const uint8_t*>(P.in), c.d, y, x0);
#pragma unroll
        for (int m = 0; m < 4; ++m) xv[m] = (float)((xd >> (8 * m)) & 0xffu) - 128.0f;
      } else {
        const int16_t* img = reinterpret_cast<const int16_t*>(P.in);
        const int64_t off = c.d.offset + (int64_t)y * c.d.pitch;
#pragma unroll
        for (int m = 0; m < 4; ++m) xv[m] = (float)img[off + min(x0 + m, c.d.w - 1)];
      }
      const uint2 a = make_uint2(pack2<PREC>(xv[0], xv[1]), pack2<PREC>(xv[2], xv[3]));
      const f4 zero = {0, 0, 0, 0};
      const f4 p = mma_p<PREC>(a, cq, zero);  // P[4g+v][q] = (X C^T)
      const uint2 ph = make_uint2(pack2<PREC>(p[0], p[1]), pack2<PREC>(p[2], p[3]));
      const f4 yt = mma_p<PREC>(ph, cq, zero);  // Y[q][4g+v]
      *reinterpret_cast<float4*>(Y + (rowblk + b) * 256 + q * 16 + 4 * g) = make_float4(yt[0], yt[1], yt[2], yt[3]);
    }
  } while (cursor_next(c, P), c.s < c.s_end);
}

// ---------------------------------------------------------------------------
#define ADCT16_MLAUNCH(kernel, grid, s, ...)                                           \
  do {                                                                                 \
    hipLaunchKernelGGL((kernel), dim3(grid), dim3(kGroupThreads), 0, (s), __VA_ARGS__); \
    return hipGetLastError();                                                          \
  } while (0)

template <int FORM, bool NT>
static hipError_t launch_mfma_forward_form(int coef_kind, const Params& P, int grid, hipStream_t s) {
  if (coef_kind == CF_I32) ADCT16_MLAUNCH((k_mfma_forward<FORM, CF_I32, NT>), grid, s, P, P.images, P.rows);
  if (coef_kind == CF_I16C) ADCT16_MLAUNCH((k_mfma_forward<FORM, CF_I16C, NT>), grid, s, P, P.images, P.rows);
  return hipErrorInvalidValue;
}

hipError_t launch_mfma_forward_i8(int coef_kind, bool nt, const Params& P, int grid, hipStream_t s) {
  return nt ? launch_mfma_forward_form<FWD_I8, true>(coef_kind, P, grid, s)
            : launch_mfma_forward_form<FWD_I8, false>(coef_kind, P, grid, s);
}

hipError_t launch_mfma_forward_i16(bool nt, const Params& P, int grid, hipStream_t s) {
  if (nt) ADCT16_MLAUNCH((k_mfma_forward_i16<true>), grid, s, P, P.images, P.rows);
  ADCT16_MLAUNCH((k_mfma_forward_i16<false>), grid, s, P, P.images, P.rows);
}

hipError_t launch_mfma_forward(int coef_kind, bool nt, const Params& P, int grid, hipStream_t s) {
  return nt ? launch_mfma_forward_form<FWD_F16, true>(coef_kind, P, grid, s)
            : launch_mfma_forward_form<FWD_F16, false>(coef_kind, P, grid, s);
}

template <bool NT>
hipError_t launch_mfma_fused_nt(bool zigzag, bool collapse, bool i8, int out_kind, const Params& P, int grid,
                                hipStream_t s) {
  if (i8) {
    if (zigzag || !collapse) return hipErrorInvalidValue;
    if (out_kind == OUT_U8) ADCT16_MLAUNCH((k_mfma_fused<false, true, OUT_U8, NT, true>), grid, s, P, P.images, P.rows);
    if (out_kind == OUT_NONE) ADCT16_MLAUNCH((k_mfma_fused<false, true, OUT_NONE, NT, true>), grid, s, P, P.images, P.rows);
  } else if (zigzag) {
    if (out_kind == OUT_U8) ADCT16_MLAUNCH((k_mfma_fused<true, false, OUT_U8, NT, false>), grid, s, P, P.images, P.rows);
    if (out_kind == OUT_NONE) ADCT16_MLAUNCH((k_mfma_fused<true, false, OUT_NONE, NT, false>), grid, s, P, P.images, P.rows);
  } else if (collapse) {
    if (out_kind == OUT_U8) ADCT16_MLAUNCH((k_mfma_fused<false, true, OUT_U8, NT, false>), grid, s, P, P.images, P.rows);
    if (out_kind == OUT_NONE) ADCT16_MLAUNCH((k_mfma_fused<false, true, OUT_NONE, NT, false>), grid, s, P, P.images, P.rows);
  } else {
    if (out_kind == OUT_U8) ADCT16_MLAUNCH((k_mfma_fused<false, false, OUT_U8, NT, false>), grid, s, P, P.images, P.rows);
    if (out_kind == OUT_NONE) ADCT16_MLAUNCH((k_mfma_fused<false, false, OUT_NONE, NT, false>), grid, s, P, P.images, P.rows);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mfma_fused(bool zigzag, bool collapse, bool i8, int out_kind, bool nt, const Params& P, int grid,
                             hipStream_t s) {
  return nt ? launch_mfma_fused_nt<true>(zigzag, collapse, i8, out_kind, P, grid, s)
            : launch_mfma_fused_nt<false>(zigzag, collapse, i8, out_kind, P, grid, s);
}

hipError_t launch_dct_mfma(int in_kind, int precision, const Params& P, float* y, int grid, hipStream_t s) {
  if (in_kind == IN_U8 && precision == ADCT16_F16) ADCT16_MLAUNCH((k_dct<IN_U8, ADCT16_F16>), grid, s, P, y);
  if (in_kind == IN_U8 && precision == ADCT16_BF16) ADCT16_MLAUNCH((k_dct<IN_U8, ADCT16_BF16>), grid, s, P, y);
  if (in_kind == IN_I16 && precision == ADCT16_F16) ADCT16_MLAUNCH((k_dct<IN_I16, ADCT16_F16>), grid, s, P, y);
  if (in_kind == IN_I16 && precision == ADCT16_BF16) ADCT16_MLAUNCH((k_dct<IN_I16, ADCT16_BF16>), grid, s, P, y);
  return hipErrorInvalidValue;
}

}  // namespace adct16
