// Internal definitions shared by the host API and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adct16.h"

namespace adct16 {

// A strip is the unit of work of one wavefront: 16 image rows by 8 blocks
// (128 columns) of one image.  Images are covered by whole strips; the last
// strip of a block row may hold fewer than 8 blocks.
constexpr int kStripBlocks = 8;
constexpr int kWavesPerGroup = 4;
constexpr int kGroupThreads = 64 * kWavesPerGroup;

// Minimum resident workgroups per CU requested from the compiler for the
// fused kernels (bounds their VGPR use); tuned on the target.
#ifndef ADCT16_VALU_MIN_WG
#define ADCT16_VALU_MIN_WG 1
#endif
#ifndef ADCT16_MFMA_MIN_WG
#define ADCT16_MFMA_MIN_WG 1
#endif
// Blocks of a strip carried through the matrix-core stages together.
#ifndef ADCT16_MFMA_BATCH
#define ADCT16_MFMA_BATCH 8
#endif

struct ImageDesc {
  int64_t offset;       // element offset of row 0 in the packed image buffer
  int64_t block_begin;  // index of the image's first block in coefficient buffers
  int64_t strip_begin;  // index of the image's first strip
  int32_t h, w, pitch;  // true size and row pitch (elements)
  int32_t bx, by;       // blocks across / down
  int32_t sx;           // strips across = ceil(bx / 8)
  int64_t pad;
};
static_assert(sizeof(ImageDesc) == 56, "ImageDesc layout");

// A run of consecutive strips of one block row of one image: the unit of
// work that the matrix-core kernels deal out to wavefronts cyclically.
// Each block row of sx strips is split into k = ceil(sx / N) runs of equal
// length (within one strip): run j covers strips j sx / k .. (j + 1) sx / k
// - 1.  Plans hold the tables for N = 4 and N = 16 (whole rows of images up
// to 2048 pixels wide, two runs of 15 strips for 3840); the autotuner picks.
// Equal runs keep the wavefronts that share a row in step.
constexpr int kTaskStripsUnit = 1, kTaskStripsPair = 2, kTaskStripsTriple = 3, kTaskStripsShort = 4,
              kTaskStripsLong = 16;
constexpr int kTaskTables = 5;  // tasks of at most 4, 16, 1, 2 and 3 strips
struct RowTask {
  int32_t img;
  int16_t sy;
  int16_t run;  // first strip (bits 0-9, sx0 < 512) | strip count << 10 (1..16)
};
__host__ __device__ constexpr int task_run_first(int run) { return run & 1023; }
__host__ __device__ constexpr int task_run_count(int run) { return run >> 10; }
static_assert(sizeof(RowTask) == 8, "RowTask layout");

// Per-plan constant tables, indexed u * 16 + v.
struct Tables {
  int32_t wkeep[256];  // w_u w_v keep(u, v): inverse weights with the retention mask
  int32_t wall[256];   // w_u w_v: inverse weights (w = 48 / n)
  float qmul[256];     // M_uv = fl32(1 / (sqrt(n_u n_v) q))
  float yscale[256];   // K_uv = fl32(1 / sqrt(n_u n_v))
  double deqc[16];     // q s_v, per horizontal frequency v
  int32_t rsep;        // retained r x r square for separable masks (16 = all; zig-zag masks use wkeep)
  float qoff;          // deadzone quantiser rounding offset f
  int32_t pad[2];
  double dctc[256];    // orthonormal DCT-II C[k][m] (comparison transform), float64
  double gauss[11];    // SSIM window: normalised 1-D Gaussian, sigma 1.5
  double pad2;
  double sdiag[16];    // s_u = 1 / sqrt(n_u) of the plan's matrix
  signed char tmat[256];  // the plan's integer matrix, tmat[u * 16 + k] (T or Walsh-Hadamard)
  signed char wvec[16];   // inverse weights w_u = 48 / n_u
  // Matrix-core residual round trip (T only): class of each row of T
  // (0: norm 16, 1: first four rows of norm 12, 2: the other four, 3: norm 8)
  // and the float64 factors of R0, R2, R3, R6 (step / 48, step / sqrt(128),
  // step / sqrt(192), step / sqrt(96)).
  signed char rcls[16];
  double rcomb[4];
  // ... and its per-lane constant operands, built on the host: entry
  // [i][lane] is dword group i (4 dwords) of lane 16 g + q, in the order
  // T[q][4g..4g+3] (2 dwords, fp16), the accumulator start, the quantiser
  // multipliers M[q][4g..4g+3], the four first-pass B operands (2 dwords
  // each) and the seven second-pass B operands (4 dwords each), 43 dwords
  // padded to 44.
  static constexpr int kResConstGroups = 11;
  uint32_t rconst[kResConstGroups][64][4];
};

// The integer matrix of a plan: MAT_APPROX is T of the proposed transform,
// MAT_WHT the Walsh-Hadamard matrix in natural order.
enum MatKind { MAT_APPROX = 0, MAT_WHT = 1 };
enum InKind { IN_U8 = 0, IN_I16 = 1 };
enum CoefKind { CF_I32 = 0, CF_I16C = 1, CF_F32 = 2, CF_L16 = 3, CF_L32 = 4, CF_NONE = 5 };
enum OutKind { OUT_NONE = 0, OUT_U8 = 1, OUT_I16 = 2, OUT_F32 = 3 };
enum ModeKind { MODE_MASK = 0, MODE_UNIFORM = 1, MODE_DEADZONE = 2 };

struct Params {
  const ImageDesc* images;
  int32_t n_images;
  int32_t sse_slots;    // per-image SSE accumulators (vector kernels): sse[img * sse_slots + slot]
  int64_t n_strips;
  int64_t n_blocks;
  const Tables* tables;
  const void* in;
  const void* in2;      // second image batch (measure)
  void* out;
  void* coef;
  void* qcoef;
  unsigned long long* sse;
  double* psnr;
  const RowTask* rows;  // the batch's strips in tasks, image by image, row by row
  int64_t n_rows;
  uint32_t* task_sse;   // per-task SSE partials (matrix-core fused kernel)
  unsigned long long* task_sse64;  // the same buffer as 64-bit partials (matrix-core residual kernel)
  const int64_t* task_first;  // index of each image's first task (n_images + 1 entries)
  int32_t task_strips;  // longest run of the task table (4, 16, 1, 2 or 3)
  int32_t pad1;
};

// Launchers (return hipSuccess or the launch error).  `grid` is the number
// of workgroups of kGroupThreads threads for the persistent strip kernels.
hipError_t launch_zero_u64(unsigned long long* p, int n, hipStream_t s);
hipError_t launch_fill_noise(void* p, int64_t bytes, int kind, hipStream_t s);
hipError_t launch_sse_finalize(const Params& P, unsigned long long* sse, hipStream_t s);
hipError_t launch_task_sse_reduce(const Params& P, hipStream_t s);
hipError_t launch_valu_forward(int mat, int in_kind, int coef_kind, const Params& P, int grid, hipStream_t s);
hipError_t launch_valu_fused(int mat, int in_kind, int mode, int qout_kind, int out_kind, const Params& P,
                             int grid, hipStream_t s);
hipError_t launch_valu_inverse(int mat, int coef_kind, int mode, int out_kind, const Params& P, int grid,
                               hipStream_t s);
hipError_t launch_quantise(int coef_kind, int mode, int qout_kind, const Params& P, hipStream_t s);
hipError_t launch_measure(int in_kind, int out_kind, const Params& P, int grid, hipStream_t s);
hipError_t launch_1d(bool inverse, const int32_t* x, int32_t* y, int64_t n, hipStream_t s);
hipError_t launch_rate(int level_kind, const Params& P, unsigned long long* bits, hipStream_t s);
hipError_t launch_dct_roundtrip(const Params& P, int grid, hipStream_t s);
hipError_t launch_ssim(const Params& P, const int64_t* tile_begin, int64_t n_tiles, const void* a, const void* b,
                       double* ssim, hipStream_t s);

hipError_t launch_mfma_forward(int coef_kind, bool nt, const Params& P, int grid, hipStream_t s);
hipError_t launch_mfma_forward_i8(int coef_kind, bool nt, const Params& P, int grid, hipStream_t s);
hipError_t launch_mfma_forward_i16(bool nt, const Params& P, int grid, hipStream_t s);
hipError_t launch_mfma_fused(bool zigzag, bool collapse, bool i8, int out_kind, bool nt, const Params& P, int grid,
                             hipStream_t s);
hipError_t launch_dct_mfma(int in_kind, int precision, const Params& P, float* y, int grid,
                           hipStream_t s);
hipError_t launch_mfma_resid(int mode, int qout_kind, int out_kind, bool nt, const Params& P, int grid,
                             hipStream_t s);
hipError_t launch_task_sse_reduce64(const Params& P, hipStream_t s);

}  // namespace adct16
