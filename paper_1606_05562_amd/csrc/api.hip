// C ABI: plan creation and validation, dispatch to the kernels, HIP graphs,
// kernel-choice autotuning and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "adct16_internal.hpp"

using namespace adct16;

namespace {

thread_local std::string g_last_error;

adct16_status fail(adct16_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

adct16_status hip_fail(hipError_t e, const char* what) {
  return fail(ADCT16_E_LAUNCH, "%s: %s", what, hipGetErrorString(e));
}

// Section 2: n_i = (T T^T)_ii, the squared row norms of T; S = diag(1/sqrt(n)).
// Section 2: the matrix T (its squared row norms are 16, 16, 12, 8, 8, 16,
// 12, 12, 16, 12, 12, 8, 8, 12, 12, 12).
constexpr signed char kTHost[16][16] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {1, 1, 1, 1, 1, 1, 1, 1, -1, -1, -1, -1, -1, -1, -1, -1},
    {1, 1, 1, 0, 0, -1, -1, -1, -1, -1, -1, 0, 0, 1, 1, 1},
    {1, 1, 0, 0, 0, 0, -1, -1, 1, 1, 0, 0, 0, 0, -1, -1},
    {1, 0, 0, -1, -1, 0, 0, 1, 1, 0, 0, -1, -1, 0, 0, 1},
    {1, 1, -1, -1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1},
    {1, 0, -1, -1, 1, 1, 0, -1, -1, 0, 1, 1, -1, -1, 0, 1},
    {0, 0, -1, 1, 1, -1, -1, 1, -1, 1, 1, -1, -1, 1, 0, 0},
    {1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1},
    {1, -1, -1, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 1, 1, -1},
    {1, -1, 0, 1, -1, 0, 1, -1, -1, 1, 0, -1, 1, 0, -1, 1},
    {0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0},
    {0, -1, 1, 0, 0, 1, -1, 0, 0, -1, 1, 0, 0, 1, -1, 0},
    {1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1},
    {0, -1, 1, -1, 1, -1, 1, 0, 0, 1, -1, 1, -1, 1, -1, 0},
    {1, -1, 0, 0, -1, 1, -1, 1, -1, 1, -1, 1, 0, 0, 1, -1},
};
// Deadzone quantiser scales per QP mod 6 (the six steps per doubling of the
// video-coding standards; quant_scale x dequant_scale ~ 2^20).
constexpr int kQuantScale[6] = {26214, 23302, 20560, 18396, 16384, 14564};
constexpr int kDequantScale[6] = {40, 45, 51, 57, 64, 72};
constexpr int kMaxQp = 63;

// Section 4: 16x16 zig-zag scan, anti-diagonal by anti-diagonal starting
// (0,0), (0,1), (1,0), ...; rank[u*16+v] = scan position.
void zigzag_rank(int (&rank)[256]) {
  int u = 0, v = 0;
  for (int k = 0; k < 256; ++k) {
    rank[u * 16 + v] = k;
    if ((u + v) % 2 == 0) {  // moving up-right
      if (v == 15) ++u;
      else if (u == 0) ++v;
      else { --u; ++v; }
    } else {                 // moving down-left
      if (u == 15) ++v;
      else if (v == 0) ++u;
      else { ++u; --v; }
    }
  }
}

bool is_int_dtype_for_in(int dt) { return dt == ADCT16_U8 || dt == ADCT16_I16; }

int esize(int dt) {
  switch (dt) {
    case ADCT16_U8: return 1;
    case ADCT16_I16: return 2;
    default: return 4;
  }
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// fp16 bits of an integer of magnitude at most 2048 (exact).
uint32_t f16_of_int(int v) {
  if (v == 0) return 0;
  const uint32_t sign = v < 0 ? 0x8000u : 0u;
  const uint32_t a = (uint32_t)(v < 0 ? -v : v);
  const int e = 31 - __builtin_clz(a);
  return sign | ((uint32_t)(e + 15) << 10) | ((a << (10 - e)) & 0x3ffu);
}

uint32_t f16_pair(int lo, int hi) { return f16_of_int(lo) | (f16_of_int(hi) << 16); }

// Coefficient of the first-pass class c's row u in the residual kernel's
// output R_k: k = 0 pairs rows of equal norm (weight w_u = 48 / n_u),
// k = 1, 2, 3 the norm pairs (16, 8), (16, 12), (12, 8).  Classes: 0 norm
// 16, 1 and 2 norm 12, 3 norm 8.
int resid_coef(int k, int cu, int c, int wu) {
  auto base = [](int x) { return x == 2 ? 1 : x; };
  const int a = base(cu), b = base(c);
  switch (k) {
    case 0: return a == b ? wu : 0;
    case 1: return (a == 0 && b == 3) || (a == 3 && b == 0);
    case 2: return (a == 0 && b == 1) || (a == 1 && b == 0);
    default: return (a == 1 && b == 3) || (a == 3 && b == 1);
  }
}

// Per-lane constant operands of the matrix-core residual kernel (the layout
// of Tables::rconst): lane 16 g + q holds T[q][4g..4g+3], the accumulator
// start, M[q][4g..4g+3], the first-pass B operands [class(4g+v) == c]
// T[4g+v][q] and the second-pass B operands coef_k(class(u), c) T[u][q] for
// u = 4g..4g+3 and the two classes of each product.
void resid_lane_consts(Tables& t) {
  auto T = [&](int u, int k) { return (int)t.tmat[u * 16 + k]; };
  const int prod_k[7] = {0, 0, 1, 2, 2, 3, 3};
  const int prod_p[7] = {0, 1, 0, 0, 1, 0, 1};
  for (int lane = 0; lane < 64; ++lane) {
    const int q = lane & 15, g = lane >> 4;
    uint32_t w[4 * Tables::kResConstGroups] = {};
    w[0] = f16_pair(T(q, 4 * g), T(q, 4 * g + 1));
    w[1] = f16_pair(T(q, 4 * g + 2), T(q, 4 * g + 3));
    const float c1 = q == 0 ? -20480.0f : 0.0f;
    memcpy(&w[2], &c1, 4);
    for (int v = 0; v < 4; ++v) memcpy(&w[3 + v], &t.qmul[q * 16 + 4 * g + v], 4);
    for (int c = 0; c < 4; ++c) {
      int y[4];
      for (int v = 0; v < 4; ++v) y[v] = t.rcls[4 * g + v] == c ? T(4 * g + v, q) : 0;
      w[7 + 2 * c] = f16_pair(y[0], y[1]);
      w[8 + 2 * c] = f16_pair(y[2], y[3]);
    }
    for (int i = 0; i < 7; ++i) {
      const int ca = prod_p[i] == 0 ? 0 : 1, cb = prod_p[i] == 0 ? 3 : 2;
      int h[8];
      for (int v = 0; v < 4; ++v) {
        const int u = 4 * g + v;
        h[v] = resid_coef(prod_k[i], t.rcls[u], ca, t.wvec[u]) * T(u, q);
        h[4 + v] = resid_coef(prod_k[i], t.rcls[u], cb, t.wvec[u]) * T(u, q);
      }
      for (int j = 0; j < 4; ++j) w[15 + 4 * i + j] = f16_pair(h[2 * j], h[2 * j + 1]);
    }
    for (int j = 0; j < 4 * Tables::kResConstGroups; ++j) t.rconst[j / 4][lane][j % 4] = w[j];
  }
}

}  // namespace

// Scratch of adct16_compress_and_measure_static: every GPU the library runs
// on holds one copy of this array (kStaticScratchBytes) until the process
// ends.  Host code never uses the name as an address: static_scratch()
// resolves each device's copy once, with that device current.
constexpr uint64_t kStaticScratchBytes = 4ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::vector<unsigned char*> g_scratch_ptr;  // device address of `scratch`, per device id

// The current device's copy of `scratch` (resolved on its first use).
adct16_status static_scratch(int device, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e, "static scratch address");
    g_scratch_ptr[device] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return ADCT16_OK;
}

}  // namespace

struct adct16_plan_s {
  adct16_desc d{};
  std::vector<ImageDesc> images;
  int device = 0;
  int cu_count = 0;
  int in_kind = IN_U8, coef_kind = CF_I32, qcoef_kind = CF_I32, out_kind = OUT_U8, mode = MODE_MASK;
  int64_t n_blocks = 0, n_strips = 0;
  ImageDesc* d_images = nullptr;
  Tables* d_tables = nullptr;
  // Task tables of the matrix-core kernels: [0] 4-strip, [1] 16-strip, [2]
  // 1-strip, [3] 2-strip and [4] 3-strip tasks.  The 4 wavefronts of a
  // workgroup start on 4 consecutive tasks, so short runs put a workgroup on
  // adjacent stretches of one block row at the same time (which HBM serves
  // faster), and launches with few strips per wavefront finish sooner.
  struct TaskTable {
    RowTask* d_rows = nullptr;
    int64_t* d_first = nullptr;  // each image's first task, n_images + 1 entries
    int64_t n_rows = 0;
    int strips = 0;
  } tasks[kTaskTables];
  int task_sel = 0;     // table of the calls without level output
  int task_sel_lv = 0;  // table of the calls with level output
  uint32_t* d_task_sse = nullptr;  // per-task SSE partials of the matrix-core fused kernel
  int64_t* d_ssim_tiles = nullptr;  // SSIM: first tile of each image (n_images + 1 entries)
  int64_t n_ssim_tiles = 0;
  bool lines_aligned = false;       // every pitch and image offset a multiple of 128 bytes
  bool small_images = false;        // every image below 2^31 bytes, every row below 2^24 bytes
  int mat = MAT_APPROX;             // integer matrix of the transform (T or Walsh-Hadamard)
  // n_images x sse_slots accumulators of the vector kernels, zero between
  // calls (cleared at creation, and by the finishing kernel of every call)
  unsigned long long* d_sse_ws = nullptr;
  unsigned long long* d_sse_out = nullptr;  // per-image SSE when the caller passes none
  int sse_slots = 1;
  int grid = 0;           // persistent workgroups for the strip kernels
  int backend = ADCT16_BACKEND_VALU;   // resolved backend of the fused/forward calls
  std::string tuned;      // how the choice was made
  // Fused calls that also write the retained coefficients or levels run
  // the vector kernel with its own launch shape.
  int grid_lv = 0;
  int backend_lv = ADCT16_BACKEND_VALU;  // backend of the fused calls with level output
  std::string tuned_lv;
  // Launch timing (adct16_plan_time_fused): event pairs recorded around the
  // persistent kernel of the next prof_ev.size() / 2 fused calls.
  std::vector<hipEvent_t> prof_ev;
  int prof_used = 0;
};

struct adct16_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

Params base_params(const adct16_plan_s* p) {
  Params P{};
  P.images = p->d_images;
  P.n_images = (int32_t)p->images.size();
  P.n_strips = p->n_strips;
  P.n_blocks = p->n_blocks;
  P.tables = p->d_tables;
  const auto& tt = p->tasks[p->task_sel];
  P.rows = tt.d_rows;
  P.n_rows = tt.n_rows;
  P.task_first = tt.d_first;
  P.task_strips = tt.strips;
  P.task_sse = p->d_task_sse;
  P.sse_slots = p->sse_slots;
  return P;
}

adct16_status check_plan(adct16_plan p) {
  if (!p) return fail(ADCT16_E_NULL, "plan is NULL");
  return ADCT16_OK;
}

bool mfma_supported(const adct16_plan_s* p);

// Device memory a fused call uses besides its inputs and outputs: the
// per-task SSE partials of the matrix-core kernels (8 bytes per task), the per-image accumulator
// slots of the vector kernel (zero on entry unless `clear_slots`), and the
// per-image SSE when the caller passes none.
struct Workspace {
  uint32_t* task_sse;
  unsigned long long* sse_slots;
  unsigned long long* sse_out;
  bool clear_slots;
};

Workspace plan_workspace(const adct16_plan_s* p) {
  return Workspace{p->d_task_sse, p->d_sse_ws, p->d_sse_out, false};
}

// The matrix-core fused kernel's number format: int8 products (flag
// ADCT16_FLAG_MFMA_INT8) for separable masks without explicit coefficients,
// FP16 products otherwise.
bool fused_int8(const adct16_plan_s* p) {
  return (p->d.flags & ADCT16_FLAG_MFMA_INT8) && p->d.qmode != ADCT16_Q_ZIGZAG &&
         !(p->d.flags & ADCT16_FLAG_EXPLICIT_COEF);
}

// Whether a fused call runs the matrix-core kernel (else the vector kernel).
bool resid_supported(const adct16_plan_s* p);

bool fused_on_mfma(const adct16_plan_s* p, int backend, bool levels) {
  return backend == ADCT16_BACKEND_MFMA && mfma_supported(p) && (!levels || resid_supported(p));
}

// Event pair i brackets this call's fused kernel (i = -1: not timed).  Calls
// captured into a graph are not timed.
hipError_t prof_begin(adct16_plan_s* p, hipStream_t s, int& i) {
  i = -1;
  if (p->prof_used * 2 >= (int)p->prof_ev.size()) return hipSuccess;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &cs);
  if (e != hipSuccess || cs != hipStreamCaptureStatusNone) return e;
  e = hipEventRecord(p->prof_ev[2 * p->prof_used], s);
  if (e == hipSuccess) i = p->prof_used++;
  return e;
}

hipError_t prof_end(adct16_plan_s* p, hipStream_t s, int i) {
  return i < 0 ? hipSuccess : hipEventRecord(p->prof_ev[2 * i + 1], s);
}

adct16_status compress_impl(adct16_plan_s* p, int backend, int grid, int tsel, const Workspace& ws,
                            const void* d_in, void* d_out, void* d_qcoef, int64_t* d_sse, double* d_psnr,
                            hipStream_t s) {
  Params P = base_params(p);
  P.task_sse = ws.task_sse;
  P.rows = p->tasks[tsel].d_rows;
  P.n_rows = p->tasks[tsel].n_rows;
  P.task_first = p->tasks[tsel].d_first;
  P.task_strips = p->tasks[tsel].strips;
  P.in = d_in;
  P.out = d_out;
  P.qcoef = d_qcoef;
  P.psnr = d_psnr;
  unsigned long long* const out_sse = reinterpret_cast<unsigned long long*>(d_sse);
  const int qk = d_qcoef ? p->qcoef_kind : CF_NONE;
  const int ok = d_out ? p->out_kind : OUT_NONE;
  hipError_t e;
  // The matrix-core fused kernel writes reconstructions and per-task SSE
  // partials, which a second kernel sums per image (SSE and PSNR); a call
  // that also asks for the retained coefficients runs the vector kernel,
  // which accumulates per image directly.
  if (fused_on_mfma(p, backend, qk != CF_NONE)) {
    P.sse = out_sse ? out_sse : ws.sse_out;  // the reduce writes final sums
    // whole-cache-line rows: streaming (non-temporal) accesses pay off
    const bool nt = p->lines_aligned && (reinterpret_cast<uintptr_t>(d_in) & 127) == 0 &&
                    (!d_out || (reinterpret_cast<uintptr_t>(d_out) & 127) == 0);
    int ti;
    if ((e = prof_begin(p, s, ti)) != hipSuccess) return hip_fail(e, "timing event");
    const bool resid = p->in_kind == IN_I16;
    P.task_sse64 = reinterpret_cast<unsigned long long*>(ws.task_sse);
    if (resid)
      e = launch_mfma_resid(p->mode, qk, ok, nt, P, grid, s);
    else
      e = launch_mfma_fused(p->d.qmode == ADCT16_Q_ZIGZAG, !(p->d.flags & ADCT16_FLAG_EXPLICIT_COEF), fused_int8(p),
                            ok, nt, P, grid, s);
    if (e != hipSuccess) return hip_fail(e, "fused kernel");
    if ((e = prof_end(p, s, ti)) != hipSuccess) return hip_fail(e, "timing event");
    e = resid ? launch_task_sse_reduce64(P, s) : launch_task_sse_reduce(P, s);
    if (e != hipSuccess) return hip_fail(e, "SSE reduction kernel");
    return ADCT16_OK;
  }
  P.sse = ws.sse_slots;  // accumulator slots (zero on entry)
  if (ws.clear_slots) {
    e = launch_zero_u64(ws.sse_slots, P.n_images * P.sse_slots, s);
    if (e != hipSuccess) return hip_fail(e, "clearing kernel");
  }
  int ti;
  if ((e = prof_begin(p, s, ti)) != hipSuccess) return hip_fail(e, "timing event");
  e = launch_valu_fused(p->mat, p->in_kind, p->mode, qk, ok, P, grid, s);
  if (e != hipSuccess) return hip_fail(e, "fused kernel");
  if ((e = prof_end(p, s, ti)) != hipSuccess) return hip_fail(e, "timing event");
  e = launch_sse_finalize(P, out_sse, s);  // also clears the slots
  if (e != hipSuccess) return hip_fail(e, "SSE / PSNR kernel");
  return ADCT16_OK;
}

// The matrix-core fused kernels cover 8-bit input with retention masks, and
// 16-bit residuals in [-256, 255] (declared by ADCT16_FLAG_RESIDUAL_RANGE)
// with a quantiser step of at least 8 (levels output included), in images
// below 2 GiB with rows below 16 MiB (32-bit offsets within an image or a
// strip row); the
// matrix-core forward covers 8-bit input to int32 or centred int16
// coefficients, and 16-bit input to int32.
bool resid_supported(const adct16_plan_s* p) {
  return p->in_kind == IN_I16 && p->mat == MAT_APPROX && (p->d.flags & ADCT16_FLAG_RESIDUAL_RANGE) &&
         p->out_kind == OUT_I16 && p->small_images &&
         ((p->mode == MODE_UNIFORM && p->d.q >= 8) || (p->mode == MODE_DEADZONE && p->d.q >= 22));
}

bool mfma_supported(const adct16_plan_s* p) {
  return (p->in_kind == IN_U8 && p->mode == MODE_MASK && p->out_kind == OUT_U8 && p->small_images) ||
         resid_supported(p);
}

bool mfma_forward_supported(const adct16_plan_s* p) {
  return (p->in_kind == IN_U8 && p->coef_kind != CF_F32) || (p->in_kind == IN_I16 && p->coef_kind == CF_I32);
}

// Autotuning: time the fused call for each candidate (backend, workgroups
// per CU) on a scratch batch of the plan's own geometry filled with noise,
// keep the fastest.
// Results are cached per process and, if ADCT16_TUNE_CACHE names a file,
// across processes (key: device arch, CU count, call shape, mask kind).
std::mutex g_tune_mu;

std::string tune_key(const adct16_plan_s* p, const char* arch, bool levels) {
  std::ostringstream k;
  k << arch << "/cu" << p->cu_count << "/b" << p->d.backend << "/t" << p->mat << "/in" << p->in_kind << "/m" << p->mode << "/q" << p->d.qmode
    << "/o" << p->out_kind << "/f"
    << (p->d.flags & (ADCT16_FLAG_EXPLICIT_COEF | ADCT16_FLAG_MFMA_INT8 | ADCT16_FLAG_RESIDUAL_RANGE))
    << "/lv" << (levels ? p->qcoef_kind : -1)
    << "/strips" << (p->n_strips >= (1 << 16) ? 1 << 16 : p->n_strips) << "/a" << (p->lines_aligned ? 1 : 0)
    << "/v8";
  return k.str();
}

bool tune_cache_get(const std::string& key, int& backend, int& wgpc, int& tsel) {
  const char* path = getenv("ADCT16_TUNE_CACHE");
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream in(line);
    std::string k;
    int b, w, t;
    if ((in >> k >> b >> w >> t) && k == key) {
      backend = b;
      wgpc = w;
      tsel = t;
      found = true;
    }
  }
  return found;
}

void tune_cache_put(const std::string& key, int backend, int wgpc, int tsel) {
  const char* path = getenv("ADCT16_TUNE_CACHE");
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << backend << " " << wgpc << " " << tsel << "\n";
}

int grid_for(const adct16_plan_s* p, int wgpc) {
  return (int)std::min<int64_t>((int64_t)p->cu_count * wgpc, (p->n_strips + kWavesPerGroup - 1) / kWavesPerGroup);
}

// Tunes one call shape: without (levels = false) or with the coefficient /
// level output, whose stores change the kernel's best occupancy.
adct16_status tune_shape(adct16_plan_s* p, const char* arch, bool levels, int& best_b, int& best_w, int& best_t,
                         std::string& how) {
  const std::string key = tune_key(p, arch, levels);
  best_b = ADCT16_BACKEND_VALU;
  best_w = 2;
  best_t = 0;
  if (tune_cache_get(key, best_b, best_w, best_t)) {
    how = "cache";
    return ADCT16_OK;
  }
  // Scratch input / output covering the packed batch extent.
  int64_t in_elems = 0;
  for (size_t i = 0; i < p->images.size(); ++i)
    in_elems = std::max<int64_t>(in_elems, p->images[i].offset + (int64_t)p->images[i].h * p->images[i].pitch);
  const size_t bytes = (size_t)in_elems * esize(p->d.in_dtype);
  const size_t qbytes = levels ? (size_t)p->n_blocks * 256 *
                                     ((p->qcoef_kind == CF_I16C || p->qcoef_kind == CF_L16) ? 2 : 4)
                               : 0;
  // Resources released on every exit.
  struct Scratch {
    void *din = nullptr, *dout = nullptr, *dq = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Scratch() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      if (s) (void)hipStreamDestroy(s);
      if (din) (void)hipFree(din);
      if (dout) (void)hipFree(dout);
      if (dq) (void)hipFree(dq);
    }
  } w;
  if (hipMalloc(&w.din, bytes + 64) != hipSuccess || hipMalloc(&w.dout, bytes + 64) != hipSuccess ||
      (levels && hipMalloc(&w.dq, qbytes) != hipSuccess))
    return fail(ADCT16_E_NOMEM, "autotune scratch");
  hipError_t e = hipStreamCreateWithFlags(&w.s, hipStreamNonBlocking);
  // noise over the input's range: 8-bit, 16-bit in [-512, 511], or
  // residuals in [-256, 255] (the matrix-core residual kernel's domain)
  const int noise = p->in_kind == IN_U8 ? 0 : (p->d.flags & ADCT16_FLAG_RESIDUAL_RANGE) ? 2 : 1;
  if (e == hipSuccess) e = launch_fill_noise(w.din, (int64_t)bytes, noise, w.s);
  if (e == hipSuccess) e = hipEventCreate(&w.e0);
  if (e == hipSuccess) e = hipEventCreate(&w.e1);
  if (e != hipSuccess) return hip_fail(e, "autotune set-up");
  // Candidates are timed round-robin, one launch at a time: clocks drift
  // over a few milliseconds of sustained load, and a sequential sweep would
  // favour whichever ran first (12 to 64 rounds, by the length of a round:
  // about 80 ms of timed work).  Each is ranked by the median of its
  // launches, which tracks sustained throughput; the fastest single launch
  // picked configurations that won short bursts at a high clock and lost
  // under sustained load.
  // (matrix-core candidates also choose the task size)
  struct Cand { int backend, wgpc, grid, tsel; std::vector<float> ms; };
  std::vector<Cand> cands;
  const bool mfma_ok = mfma_supported(p) && (!levels || resid_supported(p));
  if (p->d.backend != ADCT16_BACKEND_MFMA || !mfma_ok)
    for (int wg : {1, 2, 3, 4, 6, 8, 12}) cands.push_back({ADCT16_BACKEND_VALU, wg, grid_for(p, wg), 0, {}});
  if (p->d.backend != ADCT16_BACKEND_VALU && mfma_ok)
    for (int ts = 0; ts < kTaskTables; ++ts)
      for (int wg : {1, 2, 3, 4, 6, 8, 12}) cands.push_back({ADCT16_BACKEND_MFMA, wg, grid_for(p, wg), ts, {}});
  void* const tout = p->out_kind == OUT_F32 ? nullptr : w.dout;
  // Warm-up (code objects, and the engine clock, which ramps up under load):
  // passes over all candidates until about 20 ms of work has run.  Short
  // launches then get more timed rounds, so that the timed rounds cover
  // about 80 ms of sustained load.
  float warm_ms = 0, pass_ms = 0;
  for (int pass = 0; pass < 64 && warm_ms < 20.0f; ++pass) {
    e = hipEventRecord(w.e0, w.s);
    if (e != hipSuccess) return hip_fail(e, "autotune event");
    for (const Cand& c : cands) {
      adct16_status st = compress_impl(p, c.backend, c.grid, c.tsel, plan_workspace(p), w.din, tout, w.dq, nullptr, nullptr, w.s);
      if (st != ADCT16_OK) return st;
    }
    e = hipEventRecord(w.e1, w.s);
    if (e == hipSuccess) e = hipEventSynchronize(w.e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&pass_ms, w.e0, w.e1);
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    warm_ms += pass_ms;
  }
  const int rounds = std::max(12, std::min(64, (int)(80.0f / std::max(pass_ms, 1e-3f))));
  for (int round = 0; round < rounds; ++round) {
    for (Cand& c : cands) {
      e = hipEventRecord(w.e0, w.s);
      if (e != hipSuccess) return hip_fail(e, "autotune event");
      adct16_status st = compress_impl(p, c.backend, c.grid, c.tsel, plan_workspace(p), w.din, tout, w.dq, nullptr, nullptr, w.s);
      if (st != ADCT16_OK) return st;
      e = hipEventRecord(w.e1, w.s);
      if (e == hipSuccess) e = hipEventSynchronize(w.e1);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, w.e0, w.e1);
      if (e != hipSuccess) return hip_fail(e, "autotune timing");
      c.ms.push_back(ms);
    }
  }
  float best = 1e30f;
  for (Cand& c : cands) {
    std::sort(c.ms.begin(), c.ms.end());
    const size_t n = c.ms.size();
    const float med = n % 2 ? c.ms[n / 2] : 0.5f * (c.ms[n / 2 - 1] + c.ms[n / 2]);
    if (med < best) { best = med; best_b = c.backend; best_w = c.wgpc; best_t = c.tsel; }
  }
  std::ostringstream t;
  t << "timed:" << best_w << "wg/cu";
  how = t.str();
  tune_cache_put(key, best_b, best_w, best_t);
  return ADCT16_OK;
}

adct16_status autotune(adct16_plan_s* p, const char* arch) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  int b, wg, ts;
  adct16_status st = tune_shape(p, arch, false, b, wg, ts, p->tuned);
  if (st != ADCT16_OK) return st;
  // a requested matrix-core backend stays the forward's, whatever runs the fused call
  p->backend = p->d.backend == ADCT16_BACKEND_MFMA ? ADCT16_BACKEND_MFMA : b;
  p->grid = grid_for(p, wg);
  p->task_sel = ts;
  st = tune_shape(p, arch, true, b, wg, ts, p->tuned_lv);
  if (st != ADCT16_OK) return st;
  p->grid_lv = grid_for(p, wg);
  p->backend_lv = b;
  p->task_sel_lv = ts;
  return ADCT16_OK;
}

}  // namespace

namespace adct16 {
void set_last_error(const char* msg) { g_last_error = msg; }
}  // namespace adct16

extern "C" {

const char* adct16_status_string(adct16_status st) {
  switch (st) {
    case ADCT16_OK: return "ok";
    case ADCT16_E_NULL: return "null pointer";
    case ADCT16_E_SHAPE: return "invalid shape";
    case ADCT16_E_DTYPE: return "unsupported dtype";
    case ADCT16_E_MODE: return "invalid mode or parameter";
    case ADCT16_E_ALIGN: return "misaligned pointer, offset or pitch";
    case ADCT16_E_NOMEM: return "out of memory";
    case ADCT16_E_DEVICE: return "no usable gfx950 device";
    case ADCT16_E_LAUNCH: return "kernel launch failed";
    case ADCT16_E_STATE: return "call not valid for this plan";
  }
  return "unknown status";
}

const char* adct16_last_error_string(void) { return g_last_error.c_str(); }

adct16_status adct16_plan_create(const adct16_desc* d, adct16_plan* out) {
  if (!out) return fail(ADCT16_E_NULL, "out is NULL");
  *out = nullptr;
  if (!d) return fail(ADCT16_E_NULL, "desc is NULL");
  if (d->n_images < 1 || d->n_images > (1 << 20))
    return fail(ADCT16_E_SHAPE, "n_images = %d outside [1, 2^20]", d->n_images);
  if (!d->height || !d->width || !d->pitch || !d->offset) return fail(ADCT16_E_NULL, "image arrays are NULL");
  // dtypes
  if (!is_int_dtype_for_in(d->in_dtype)) return fail(ADCT16_E_DTYPE, "in_dtype must be U8 or I16");
  const bool in_u8 = d->in_dtype == ADCT16_U8;
  if (!(d->coef_dtype == ADCT16_I32 || d->coef_dtype == ADCT16_F32 || (in_u8 && d->coef_dtype == ADCT16_I16)))
    return fail(ADCT16_E_DTYPE, "coef_dtype must be I32, F32 or (U8 input) I16");
  if (!(d->out_dtype == ADCT16_I16 || d->out_dtype == ADCT16_F32 || (in_u8 && d->out_dtype == ADCT16_U8)))
    return fail(ADCT16_E_DTYPE, "out_dtype must be I16, F32 or (U8 input) U8");
  if (d->qmode < ADCT16_Q_NONE || d->qmode > ADCT16_Q_DEADZONE) return fail(ADCT16_E_MODE, "qmode %d", d->qmode);
  const bool uniform = d->qmode == ADCT16_Q_UNIFORM, deadzone = d->qmode == ADCT16_Q_DEADZONE;
  const bool levels = uniform || deadzone;
  if (levels) {
    if (!(d->qcoef_dtype == ADCT16_I16 || d->qcoef_dtype == ADCT16_I32))
      return fail(ADCT16_E_DTYPE, "quantisation levels must be I16 or I32");
    if (uniform && (d->q < 1 || d->q > 65535)) return fail(ADCT16_E_MODE, "q = %d outside [1, 65535]", d->q);
    if (deadzone && (d->q < 0 || d->q > kMaxQp)) return fail(ADCT16_E_MODE, "QP = %d outside [0, %d]", d->q, kMaxQp);
  } else {
    if (!(d->qcoef_dtype == ADCT16_I32 || (in_u8 && d->qcoef_dtype == ADCT16_I16)))
      return fail(ADCT16_E_DTYPE, "retained coefficients must be I32 or (U8 input) I16");
    if (d->qmode == ADCT16_Q_ZONAL && (d->r < 1 || d->r > 16)) return fail(ADCT16_E_MODE, "zonal r = %d outside [1, 16]", d->r);
    if (d->qmode == ADCT16_Q_ZIGZAG && (d->r < 1 || d->r > 256)) return fail(ADCT16_E_MODE, "zig-zag r = %d outside [1, 256]", d->r);
  }
  if (d->backend < ADCT16_BACKEND_AUTO || d->backend > ADCT16_BACKEND_MFMA)
    return fail(ADCT16_E_MODE, "backend %d", d->backend);
  if (!(d->matrix == ADCT16_MATRIX_APPROX || d->matrix == ADCT16_MATRIX_T || d->matrix == ADCT16_MATRIX_WHT))
    return fail(ADCT16_E_MODE, "matrix %d: the kernels take the proposed transform or the Walsh-Hadamard matrix",
                d->matrix);
  // geometry
  const int es = esize(d->in_dtype);
  std::vector<ImageDesc> images(d->n_images);
  int64_t blocks = 0, strips = 0;
  for (int i = 0; i < d->n_images; ++i) {
    const int h = d->height[i], w = d->width[i], pt = d->pitch[i];
    const int64_t off = d->offset[i];
    if (h < 1 || w < 1 || h > 65536 || w > 65536) return fail(ADCT16_E_SHAPE, "image %d: size %dx%d", i, h, w);
    const int w16 = (w + 15) / 16 * 16;
    if (pt < w16) return fail(ADCT16_E_SHAPE, "image %d: pitch %d < width rounded up to 16 (%d)", i, pt, w16);
    if (off < 0) return fail(ADCT16_E_SHAPE, "image %d: negative offset", i);
    if (((int64_t)pt * es) % 16 || (off * es) % 16)
      return fail(ADCT16_E_ALIGN, "image %d: pitch/offset not 16-byte aligned", i);
    ImageDesc& g = images[i];
    memset(&g, 0, sizeof g);
    g.offset = off;
    g.h = h; g.w = w; g.pitch = pt;
    g.bx = (w + 15) / 16;
    g.by = (h + 15) / 16;
    g.sx = (g.bx + kStripBlocks - 1) / kStripBlocks;
    g.block_begin = blocks;
    g.strip_begin = strips;
    blocks += (int64_t)g.bx * g.by;
    strips += (int64_t)g.sx * g.by;
  }
  if (blocks > ((int64_t)1 << 36)) return fail(ADCT16_E_SHAPE, "batch too large");
  // device
  int dev = 0, ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(ADCT16_E_DEVICE, "no HIP device");
  if (hipGetDevice(&dev) != hipSuccess) return fail(ADCT16_E_DEVICE, "hipGetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return fail(ADCT16_E_DEVICE, "hipGetDeviceProperties failed");
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(ADCT16_E_DEVICE, "device %d is %s, not gfx950", dev, prop.gcnArchName);

  auto* p = new adct16_plan_s();
  p->d = *d;
  p->d.height = p->d.width = p->d.pitch = nullptr;
  p->d.offset = nullptr;
  p->images = images;
  p->device = dev;
  p->cu_count = prop.multiProcessorCount;
  p->in_kind = in_u8 ? IN_U8 : IN_I16;
  p->coef_kind = d->coef_dtype == ADCT16_I32 ? CF_I32 : d->coef_dtype == ADCT16_I16 ? CF_I16C : CF_F32;
  if (levels) p->qcoef_kind = d->qcoef_dtype == ADCT16_I16 ? CF_L16 : CF_L32;
  else p->qcoef_kind = d->qcoef_dtype == ADCT16_I16 ? CF_I16C : CF_I32;
  p->out_kind = d->out_dtype == ADCT16_U8 ? OUT_U8 : d->out_dtype == ADCT16_I16 ? OUT_I16 : OUT_F32;
  p->mode = uniform ? MODE_UNIFORM : deadzone ? MODE_DEADZONE : MODE_MASK;
  p->n_blocks = blocks;
  p->n_strips = strips;
  p->lines_aligned = true;
  p->small_images = true;
  for (const ImageDesc& g : images) {
    if (((int64_t)g.pitch * es) % 128 || (g.offset * es) % 128) p->lines_aligned = false;
    if ((int64_t)g.pitch * es >= ((int64_t)1 << 24) || (int64_t)g.h * g.pitch * es >= ((int64_t)1 << 31))
      p->small_images = false;
  }

  // the integer matrix, its squared row norms n_u and the weights 48 / n_u
  p->mat = d->matrix == ADCT16_MATRIX_WHT ? MAT_WHT : MAT_APPROX;
  int tmat[16][16], norm[16];
  for (int u = 0; u < 16; ++u) {
    norm[u] = 0;
    for (int k = 0; k < 16; ++k) {
      tmat[u][k] = p->mat == MAT_WHT ? ((__builtin_popcount(u & k) & 1) ? -1 : 1) : kTHost[u][k];
      norm[u] += tmat[u][k] * tmat[u][k];
    }
  }

  // constant tables
  Tables t;
  memset(&t, 0, sizeof t);
  int zz[256];
  zigzag_rank(zz);
  for (int u = 0; u < 16; ++u) {
    for (int v = 0; v < 16; ++v) {
      const int nn = norm[u] * norm[v];
      const int wuv = (48 / norm[u]) * (48 / norm[v]);
      bool keep = true;
      if (d->qmode == ADCT16_Q_ZONAL) keep = u < d->r && v < d->r;
      if (d->qmode == ADCT16_Q_ZIGZAG) keep = zz[u * 16 + v] < d->r;
      t.wall[u * 16 + v] = wuv;
      t.wkeep[u * 16 + v] = keep ? wuv : 0;
      t.yscale[u * 16 + v] = (float)(1.0 / std::sqrt((double)nn));
      if (uniform) t.qmul[u * 16 + v] = (float)(1.0 / (std::sqrt((double)nn) * (double)d->q));
      // deadzone: M = quant_scale[QP mod 6] / (sqrt(n_u n_v) 2^(14 + QP / 6)); sqrt and
      // the division are correctly rounded, the power of two is exact
      if (deadzone)
        t.qmul[u * 16 + v] = (float)(std::ldexp((double)kQuantScale[d->q % 6] / std::sqrt((double)nn), -(14 + d->q / 6)));
    }
    if (uniform) t.deqc[u] = (double)d->q / std::sqrt((double)norm[u]);
    // deadzone reconstruction step: dequant_scale[QP mod 6] 2^(QP / 6) / 64 (exact)
    if (deadzone) t.deqc[u] = std::ldexp((double)kDequantScale[d->q % 6], d->q / 6 - 6) / std::sqrt((double)norm[u]);
    t.sdiag[u] = 1.0 / std::sqrt((double)norm[u]);
    t.wvec[u] = (signed char)(48 / norm[u]);
    for (int k = 0; k < 16; ++k) t.tmat[u * 16 + k] = (signed char)tmat[u][k];
  }
  t.qoff = (d->flags & ADCT16_FLAG_DEADZONE_INTER) ? (float)(1.0 / 6.0) : (float)(1.0 / 3.0);
  // matrix-core residual kernel: row classes of T (norm 16; the first and
  // the other four rows of norm 12; norm 8) and the float64 factors of its
  // four integer partial inverses
  {
    int seen12 = 0;
    for (int u = 0; u < 16; ++u)
      t.rcls[u] = (signed char)(norm[u] == 16 ? 0 : norm[u] == 8 ? 3 : (seen12++ < 4 ? 1 : 2));
    const double step = uniform ? (double)d->q
                                : deadzone ? std::ldexp((double)kDequantScale[d->q % 6], d->q / 6 - 6) : 1.0;
    t.rcomb[0] = step / 48.0;
    t.rcomb[1] = step / std::sqrt(128.0);
    t.rcomb[2] = step / std::sqrt(192.0);
    t.rcomb[3] = step / std::sqrt(96.0);
    resid_lane_consts(t);
  }
  // comparison transform and SSIM window
  for (int k = 0; k < 16; ++k)
    for (int m = 0; m < 16; ++m)
      t.dctc[k * 16 + m] = (k == 0 ? 0.25 : 1.0 / std::sqrt(8.0)) * std::cos(M_PI * (2 * m + 1) * k / 32.0);
  {
    double gs = 0.0;
    for (int k = 0; k < 11; ++k) gs += (t.gauss[k] = std::exp(-(double)((k - 5) * (k - 5)) / (2.0 * 1.5 * 1.5)));
    for (int k = 0; k < 11; ++k) t.gauss[k] /= gs;
  }
  std::vector<int64_t> ssim_tiles(images.size() + 1, 0);
  for (size_t i = 0; i < images.size(); ++i) {
    const int oh = images[i].h - 10, ow = images[i].w - 10;
    ssim_tiles[i + 1] = ssim_tiles[i] + (oh > 0 && ow > 0 ? (int64_t)((oh + 15) / 16) * ((ow + 31) / 32) : 0);
  }
  p->n_ssim_tiles = ssim_tiles.back();
  t.rsep = d->qmode == ADCT16_Q_ZONAL ? d->r : 16;
  std::vector<RowTask> rows[kTaskTables];
  std::vector<int64_t> first[kTaskTables];
  for (int ts = 0; ts < kTaskTables; ++ts) {
    const int n = ts == 0   ? kTaskStripsShort
                  : ts == 1 ? kTaskStripsLong
                  : ts == 2 ? kTaskStripsUnit
                  : ts == 3 ? kTaskStripsPair
                            : kTaskStripsTriple;
    p->tasks[ts].strips = n;
    for (size_t i = 0; i < images.size(); ++i) {
      first[ts].push_back((int64_t)rows[ts].size());
      // k = ceil(sx / n) runs of equal length (within one strip) per block row
      const int sx = images[i].sx, k = (sx + n - 1) / n;
      for (int sy = 0; sy < images[i].by; ++sy)
        for (int j = 0; j < k; ++j) {
          const int a = (int)((int64_t)j * sx / k), b = (int)((int64_t)(j + 1) * sx / k);
          rows[ts].push_back(RowTask{(int32_t)i, (int16_t)sy, (int16_t)(a | ((b - a) << 10))});
        }
    }
    first[ts].push_back((int64_t)rows[ts].size());
    p->tasks[ts].n_rows = (int64_t)rows[ts].size();
  }
  // SSE accumulator slots per image: fewer images are each worked on by
  // more wavefronts at once (at most 2^20 accumulators in all)
  p->sse_slots = images.size() <= 1024 ? 64 : images.size() <= 16384 ? 8 : 1;
  bool ok = hipMalloc(&p->d_images, sizeof(ImageDesc) * images.size()) == hipSuccess &&
            hipMalloc(&p->d_tables, sizeof(Tables)) == hipSuccess;
  size_t max_rows = 0;
  for (int ts = 0; ts < kTaskTables; ++ts) {
    max_rows = std::max(max_rows, rows[ts].size());
    ok = ok && hipMalloc(&p->tasks[ts].d_rows, sizeof(RowTask) * rows[ts].size()) == hipSuccess &&
         hipMalloc(&p->tasks[ts].d_first, sizeof(int64_t) * first[ts].size()) == hipSuccess &&
         hipMemcpy(p->tasks[ts].d_rows, rows[ts].data(), sizeof(RowTask) * rows[ts].size(), hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemcpy(p->tasks[ts].d_first, first[ts].data(), sizeof(int64_t) * first[ts].size(), hipMemcpyHostToDevice) ==
             hipSuccess;
  }
  ok = ok && hipMalloc(&p->d_task_sse, sizeof(unsigned long long) * max_rows) == hipSuccess &&
            hipMalloc(&p->d_ssim_tiles, sizeof(int64_t) * ssim_tiles.size()) == hipSuccess &&
            hipMalloc(&p->d_sse_ws, sizeof(unsigned long long) * images.size() * p->sse_slots) == hipSuccess &&
            hipMalloc(&p->d_sse_out, sizeof(unsigned long long) * images.size()) == hipSuccess;
  ok = ok && hipMemset(p->d_sse_ws, 0, sizeof(unsigned long long) * images.size() * p->sse_slots) == hipSuccess;
  ok = ok && hipMemcpy(p->d_images, images.data(), sizeof(ImageDesc) * images.size(), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(p->d_tables, &t, sizeof t, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(p->d_ssim_tiles, ssim_tiles.data(), sizeof(int64_t) * ssim_tiles.size(), hipMemcpyHostToDevice) ==
           hipSuccess;
  if (!ok) {
    adct16_plan_destroy(p);
    return fail(ADCT16_E_NOMEM, "plan allocation failed");
  }
  // kernel choice
  // Persistent grid: workgroups per CU (ADCT16_WG_PER_CU overrides the
  // default; the autotuner may replace it).
  const int64_t max_groups = (strips + kWavesPerGroup - 1) / kWavesPerGroup;
  int wgpc = 4;
  if (const char* env = getenv("ADCT16_WG_PER_CU")) wgpc = std::max(1, std::min(64, atoi(env)));
  p->grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)p->cu_count * wgpc, max_groups));
  // task size of the matrix-core kernels (ADCT16_TASK_STRIPS = 1, 2, 3, 4 or 16 overrides the
  // default 4; the autotuner may replace it)
  if (const char* env = getenv("ADCT16_TASK_STRIPS")) {
    const int n = atoi(env);
    p->task_sel = n >= kTaskStripsLong ? 1 : n <= kTaskStripsUnit ? 2 : n == kTaskStripsPair ? 3 : n == kTaskStripsTriple ? 4 : 0;
  }
  if (d->backend == ADCT16_BACKEND_MFMA && !mfma_supported(p) && !mfma_forward_supported(p)) {
    adct16_plan_destroy(p);
    return fail(ADCT16_E_MODE,
                "MFMA backend supports, for images below 2 GiB with rows below 16 MiB, U8 input with retention "
                "modes and U8 output, or I16 residuals with ADCT16_FLAG_RESIDUAL_RANGE, a step of at least 8 "
                "and I16 output (fused call); or U8 input to I32/I16 coefficients and I16 input to I32 "
                "coefficients (forward)");
  }
  p->grid_lv = p->grid;
  p->task_sel_lv = p->task_sel;
  p->tuned_lv = "default";
  p->backend_lv = d->backend == ADCT16_BACKEND_MFMA && resid_supported(p) ? ADCT16_BACKEND_MFMA : ADCT16_BACKEND_VALU;
  if (d->flags & ADCT16_FLAG_AUTOTUNE) {
    // a requested backend restricts the search to its launch shapes
    adct16_status st = autotune(p, prop.gcnArchName);
    if (st != ADCT16_OK) {
      adct16_plan_destroy(p);
      return st;
    }
  } else if (d->backend == ADCT16_BACKEND_MFMA || d->backend == ADCT16_BACKEND_VALU) {
    p->backend = d->backend;
    p->tuned = "requested";
  } else {
    p->backend = ADCT16_BACKEND_VALU;
    p->tuned = "default";
  }
  *out = p;
  return ADCT16_OK;
}

adct16_status adct16_plan_destroy(adct16_plan p) {
  if (!p) return fail(ADCT16_E_NULL, "plan is NULL");
  // nothing useful can be done about a failed free on teardown
  if (p->d_images) (void)hipFree(p->d_images);
  if (p->d_tables) (void)hipFree(p->d_tables);
  for (auto& tt : p->tasks) {
    if (tt.d_rows) (void)hipFree(tt.d_rows);
    if (tt.d_first) (void)hipFree(tt.d_first);
  }
  if (p->d_task_sse) (void)hipFree(p->d_task_sse);
  if (p->d_ssim_tiles) (void)hipFree(p->d_ssim_tiles);
  if (p->d_sse_ws) (void)hipFree(p->d_sse_ws);
  if (p->d_sse_out) (void)hipFree(p->d_sse_out);
  for (hipEvent_t ev : p->prof_ev) (void)hipEventDestroy(ev);
  delete p;
  return ADCT16_OK;
}

adct16_status adct16_plan_time_fused(adct16_plan p, int32_t n_calls) {
  if (adct16_status st = check_plan(p)) return st;
  if (n_calls < 0 || n_calls > (1 << 16)) return fail(ADCT16_E_SHAPE, "n_calls must be in 0..65536");
  for (hipEvent_t ev : p->prof_ev) (void)hipEventDestroy(ev);
  p->prof_ev.clear();
  p->prof_used = 0;
  for (int i = 0; i < 2 * n_calls; ++i) {
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess) {
      for (hipEvent_t e2 : p->prof_ev) (void)hipEventDestroy(e2);
      p->prof_ev.clear();
      return fail(ADCT16_E_NOMEM, "timing events");
    }
    p->prof_ev.push_back(ev);
  }
  return ADCT16_OK;
}

adct16_status adct16_plan_fused_times(adct16_plan p, float* ms, int32_t cap, int32_t* n_out) {
  if (adct16_status st = check_plan(p)) return st;
  if (!n_out || (cap > 0 && !ms)) return fail(ADCT16_E_NULL, "ms / n_out is NULL");
  const int n = std::min<int>(p->prof_used, std::max(0, cap));
  for (int i = 0; i < n; ++i) {
    hipError_t e = hipEventSynchronize(p->prof_ev[2 * i + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms[i], p->prof_ev[2 * i], p->prof_ev[2 * i + 1]);
    if (e != hipSuccess) return hip_fail(e, "timing event");
  }
  *n_out = p->prof_used;
  p->prof_used = 0;
  return ADCT16_OK;
}

adct16_status adct16_plan_num_blocks(adct16_plan p, int64_t* n) {
  if (adct16_status st = check_plan(p)) return st;
  if (!n) return fail(ADCT16_E_NULL, "num_blocks is NULL");
  *n = p->n_blocks;
  return ADCT16_OK;
}

adct16_status adct16_plan_info(adct16_plan p, char* buf, int32_t len) {
  if (adct16_status st = check_plan(p)) return st;
  if (!buf || len < 1) return fail(ADCT16_E_NULL, "buffer is NULL");
  std::ostringstream o;
  o << "{\"backend\": \"" << (p->backend == ADCT16_BACKEND_MFMA ? "mfma" : "valu") << "\", \"grid\": " << p->grid
    << ", \"threads\": " << kGroupThreads << ", \"strips\": " << p->n_strips << ", \"blocks\": " << p->n_blocks
    << ", \"cus\": " << p->cu_count << ", \"rows_line_aligned\": " << (p->lines_aligned ? "true" : "false")
    << ", \"fused_backend\": \"" << (p->backend == ADCT16_BACKEND_MFMA && mfma_supported(p) ? "mfma" : "valu")
    << "\", \"fused_form\": \""
    << (p->backend == ADCT16_BACKEND_MFMA && mfma_supported(p)
            ? (p->in_kind == IN_I16 ? "fp16-residual-classes"
               : fused_int8(p)      ? "int8"
               : (p->d.qmode == ADCT16_Q_ZIGZAG || (p->d.flags & ADCT16_FLAG_EXPLICIT_COEF)) ? "fp16-explicit"
                                                                                             : "fp16-collapsed")
            : "butterflies")
    << "\", \"forward_backend\": \""
    << (p->backend == ADCT16_BACKEND_MFMA && mfma_forward_supported(p) ? "mfma" : "valu") << "\""
    << ", \"task_strips\": " << p->tasks[p->task_sel].strips
    << ", \"choice\": \"" << p->tuned << "\", \"levels_backend\": \""
    << (p->backend_lv == ADCT16_BACKEND_MFMA ? "mfma" : "valu") << "\", \"levels_grid\": " << p->grid_lv
    << ", \"levels_task_strips\": " << p->tasks[p->task_sel_lv].strips
    << ", \"levels_choice\": \"" << p->tuned_lv << "\"}";
  const std::string s = o.str();
  if ((int32_t)s.size() + 1 > len) return fail(ADCT16_E_SHAPE, "buffer too small (%d needed)", (int)s.size() + 1);
  memcpy(buf, s.c_str(), s.size() + 1);
  return ADCT16_OK;
}

adct16_status adct16_forward(adct16_plan p, const void* d_in, void* d_coef, void* stream) {
  if (adct16_status st = check_plan(p)) return st;
  if (!d_in || !d_coef) return fail(ADCT16_E_NULL, "d_in / d_coef is NULL");
  if (!aligned16(d_in) || !aligned16(d_coef)) return fail(ADCT16_E_ALIGN, "d_in / d_coef not 16-byte aligned");
  Params P = base_params(p);
  P.in = d_in;
  P.coef = d_coef;
  hipError_t e;
  if (p->backend == ADCT16_BACKEND_MFMA && mfma_forward_supported(p)) {
    // whole-cache-line rows and block-aligned coefficients: streaming accesses
    const bool nt = p->lines_aligned && (reinterpret_cast<uintptr_t>(d_in) & 127) == 0 &&
                    (reinterpret_cast<uintptr_t>(d_coef) & 127) == 0;
    if (p->in_kind == IN_I16)  // 16-bit input: the int8 form with three digits per value
      e = launch_mfma_forward_i16(nt, P, p->grid, (hipStream_t)stream);
    else if (p->d.flags & ADCT16_FLAG_MFMA_INT8)
      e = launch_mfma_forward_i8(p->coef_kind, nt, P, p->grid, (hipStream_t)stream);
    else
      e = launch_mfma_forward(p->coef_kind, nt, P, p->grid, (hipStream_t)stream);
  } else
    e = launch_valu_forward(p->mat, p->in_kind, p->coef_kind, P, p->grid, (hipStream_t)stream);
  return e == hipSuccess ? ADCT16_OK : hip_fail(e, "forward kernel");
}

adct16_status adct16_quantise(adct16_plan p, const void* d_coef, void* d_qcoef, void* stream) {
  if (adct16_status st = check_plan(p)) return st;
  if (!d_coef || !d_qcoef) return fail(ADCT16_E_NULL, "d_coef / d_qcoef is NULL");
  if (!aligned16(d_coef) || !aligned16(d_qcoef)) return fail(ADCT16_E_ALIGN, "d_coef / d_qcoef not 16-byte aligned");
  if (p->coef_kind == CF_F32) return fail(ADCT16_E_STATE, "quantise needs integer coefficients (coef_dtype I32 or I16)");
  if (p->mode == MODE_MASK && p->qcoef_kind != p->coef_kind)
    return fail(ADCT16_E_STATE, "retention keeps the coefficient dtype: qcoef_dtype must equal coef_dtype");
  Params P = base_params(p);
  P.coef = const_cast<void*>(d_coef);
  P.qcoef = d_qcoef;
  hipError_t e = launch_quantise(p->coef_kind, p->mode, p->qcoef_kind, P, (hipStream_t)stream);
  return e == hipSuccess ? ADCT16_OK : hip_fail(e, "quantise kernel");
}

adct16_status adct16_inverse(adct16_plan p, const void* d_qcoef, void* d_out, void* stream) {
  if (adct16_status st = check_plan(p)) return st;
  if (!d_qcoef || !d_out) return fail(ADCT16_E_NULL, "d_qcoef / d_out is NULL");
  if (!aligned16(d_qcoef) || !aligned16(d_out)) return fail(ADCT16_E_ALIGN, "d_qcoef / d_out not 16-byte aligned");
  Params P = base_params(p);
  P.qcoef = const_cast<void*>(d_qcoef);
  P.out = d_out;
  // the deadzone levels are reconstructed like uniform ones (step in the tables)
  hipError_t e = launch_valu_inverse(p->mat, p->qcoef_kind, p->mode == MODE_DEADZONE ? MODE_UNIFORM : p->mode, p->out_kind,
                                     P, p->grid, (hipStream_t)stream);
  return e == hipSuccess ? ADCT16_OK : hip_fail(e, "inverse kernel");
}

adct16_status adct16_dct_compress_and_measure(adct16_plan p, const void* d_in, void* d_out, int64_t* d_sse,
                                              double* d_psnr, void* stream) {
  if (adct16_status st = check_plan(p)) return st;
  if (!d_in) return fail(ADCT16_E_NULL, "d_in is NULL");
  if (p->in_kind != IN_U8 || (d_out && p->out_kind != OUT_U8))
    return fail(ADCT16_E_DTYPE, "the DCT-II round trip takes U8 input and writes U8 output");
  if (p->mode != MODE_MASK) return fail(ADCT16_E_STATE, "the DCT-II round trip uses retention masks only");
  Params P = base_params(p);
  P.in = d_in;
  P.out = d_out;
  P.sse = p->d_sse_ws;
  P.psnr = d_psnr;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_dct_roundtrip(P, p->grid, s);
  if (e == hipSuccess) e = launch_sse_finalize(P, reinterpret_cast<unsigned long long*>(d_sse), s);
  return e == hipSuccess ? ADCT16_OK : hip_fail(e, "DCT-II round trip");
}

adct16_status adct16_ssim(adct16_plan p, const void* d_a, const void* d_b, double* d_ssim, void* stream) {
  if (adct16_status st = check_plan(p)) return st;
  if (!d_a || !d_b || !d_ssim) return fail(ADCT16_E_NULL, "d_a / d_b / d_ssim is NULL");
  if (p->in_kind != IN_U8 || p->out_kind != OUT_U8) return fail(ADCT16_E_DTYPE, "SSIM compares U8 images");
  if (reinterpret_cast<uintptr_t>(d_ssim) & 7) return fail(ADCT16_E_ALIGN, "d_ssim not 8-byte aligned");
  Params P = base_params(p);
  hipError_t e = launch_ssim(P, p->d_ssim_tiles, p->n_ssim_tiles, d_a, d_b, d_ssim, (hipStream_t)stream);
  return e == hipSuccess ? ADCT16_OK : hip_fail(e, "SSIM kernels");
}

adct16_status adct16_rate(adct16_plan p, const void* d_qcoef, int64_t* d_bits, void* stream) {
  if (adct16_status st = check_plan(p)) return st;
  if (p->mode == MODE_MASK) return fail(ADCT16_E_STATE, "the plan's qmode produces no levels");
  if (!d_qcoef || !d_bits) return fail(ADCT16_E_NULL, "d_qcoef / d_bits is NULL");
  if (!aligned16(d_qcoef) || (reinterpret_cast<uintptr_t>(d_bits) & 7))
    return fail(ADCT16_E_ALIGN, "d_qcoef not 16-byte / d_bits not 8-byte aligned");
  Params P = base_params(p);
  P.qcoef = const_cast<void*>(d_qcoef);
  hipError_t e = launch_rate(p->qcoef_kind, P, reinterpret_cast<unsigned long long*>(d_bits), (hipStream_t)stream);
  return e == hipSuccess ? ADCT16_OK : hip_fail(e, "rate kernel");
}

adct16_status adct16_measure(adct16_plan p, const void* d_a, const void* d_b, int64_t* d_sse, double* d_psnr,
                             void* stream) {
  if (adct16_status st = check_plan(p)) return st;
  if (!d_a || !d_b || !d_sse) return fail(ADCT16_E_NULL, "d_a / d_b / d_sse is NULL");
  if (!aligned16(d_a) || !aligned16(d_b)) return fail(ADCT16_E_ALIGN, "d_a / d_b not 16-byte aligned");
  if (p->out_kind == OUT_F32) return fail(ADCT16_E_STATE, "measure compares integer images (out_dtype U8 or I16)");
  if ((p->in_kind == IN_U8) != (p->out_kind == OUT_U8))
    return fail(ADCT16_E_STATE, "measure needs in_dtype == out_dtype");
  Params P = base_params(p);
  P.in = d_a;
  P.in2 = d_b;
  P.sse = p->d_sse_ws;
  P.psnr = d_psnr;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_measure(p->in_kind, p->out_kind, P, p->grid, s);
  if (e == hipSuccess) e = launch_sse_finalize(P, reinterpret_cast<unsigned long long*>(d_sse), s);
  return e == hipSuccess ? ADCT16_OK : hip_fail(e, "measure kernels");
}

adct16_status adct16_compress_and_measure(adct16_plan p, const void* d_in, void* d_out, void* d_qcoef,
                                          int64_t* d_sse, double* d_psnr, void* stream) {
  if (adct16_status st = check_plan(p)) return st;
  if (!d_in) return fail(ADCT16_E_NULL, "d_in is NULL");
  if (!aligned16(d_in) || (d_out && !aligned16(d_out)) || (d_qcoef && !aligned16(d_qcoef)))
    return fail(ADCT16_E_ALIGN, "buffers must be 16-byte aligned");
  if (d_out && p->out_kind == OUT_F32)
    return fail(ADCT16_E_STATE, "the fused call writes rounded reconstructions (out_dtype U8 or I16)");
  if (d_qcoef)
    return compress_impl(p, p->backend_lv, p->grid_lv, p->task_sel_lv, plan_workspace(p), d_in, d_out, d_qcoef,
                         d_sse, d_psnr, (hipStream_t)stream);
  return compress_impl(p, p->backend, p->grid, p->task_sel, plan_workspace(p), d_in, d_out, d_qcoef, d_sse, d_psnr,
                       (hipStream_t)stream);
}

adct16_status adct16_compress_and_measure_static(adct16_plan p, const void* d_in, void* d_out, void* d_qcoef,
                                                 int64_t* d_sse, double* d_psnr, void* stream) {
  if (adct16_status st = check_plan(p)) return st;
  if (!d_in) return fail(ADCT16_E_NULL, "d_in is NULL");
  if (!aligned16(d_in) || (d_out && !aligned16(d_out)) || (d_qcoef && !aligned16(d_qcoef)))
    return fail(ADCT16_E_ALIGN, "buffers must be 16-byte aligned");
  if (d_out && p->out_kind == OUT_F32)
    return fail(ADCT16_E_STATE, "the fused call writes rounded reconstructions (out_dtype U8 or I16)");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail(ADCT16_E_DEVICE, "the plan's device (%d) must be current (current: %d)", p->device, dev);
  const bool levels = d_qcoef != nullptr;
  const int backend = levels ? p->backend_lv : p->backend;
  const int grid = levels ? p->grid_lv : p->grid;
  const int tsel = levels ? p->task_sel_lv : p->task_sel;
  // carve the call's workspace out of the array, 256-byte aligned pieces
  auto up = [](uint64_t b) { return (b + 255) & ~uint64_t(255); };
  uint64_t need = 0, o_task = 0, o_slots = 0, o_out = 0;
  if (fused_on_mfma(p, backend, levels)) {
    o_task = need;
    need += up(sizeof(unsigned long long) * (uint64_t)p->tasks[tsel].n_rows);
    o_out = need;
    if (!d_sse) need += up(sizeof(unsigned long long) * p->images.size());
  } else {
    o_slots = need;
    need += up(sizeof(unsigned long long) * p->images.size() * (uint64_t)p->sse_slots);
  }
  if (need > kStaticScratchBytes)
    return fail(ADCT16_E_SHAPE, "the batch needs %llu bytes of scratch; the static scratch holds %llu",
                (unsigned long long)need, (unsigned long long)kStaticScratchBytes);
  unsigned char* base = nullptr;
  if (adct16_status st = static_scratch(dev, &base)) return st;
  const Workspace ws{reinterpret_cast<uint32_t*>(base + o_task), reinterpret_cast<unsigned long long*>(base + o_slots),
                     reinterpret_cast<unsigned long long*>(base + o_out), true};
  return compress_impl(p, backend, grid, tsel, ws, d_in, d_out, d_qcoef, d_sse, d_psnr, (hipStream_t)stream);
}

adct16_status adct16_dct_forward(adct16_plan p, const void* d_in, float* d_y, int32_t precision, void* stream) {
  if (adct16_status st = check_plan(p)) return st;
  if (!d_in || !d_y) return fail(ADCT16_E_NULL, "d_in / d_y is NULL");
  if (!aligned16(d_in) || !aligned16(d_y)) return fail(ADCT16_E_ALIGN, "d_in / d_y not 16-byte aligned");
  if (precision != ADCT16_BF16 && precision != ADCT16_F16) return fail(ADCT16_E_MODE, "precision must be BF16 or F16");
  Params P = base_params(p);
  P.in = d_in;
  hipError_t e = launch_dct_mfma(p->in_kind, precision, P, d_y, p->grid, (hipStream_t)stream);
  return e == hipSuccess ? ADCT16_OK : hip_fail(e, "DCT kernel");
}

adct16_status adct16_forward_1d(const int32_t* d_x, int32_t* d_y, int64_t n, void* stream) {
  if (n < 0) return fail(ADCT16_E_SHAPE, "n < 0");
  if (n == 0) return ADCT16_OK;
  if (!d_x || !d_y) return fail(ADCT16_E_NULL, "d_x / d_y is NULL");
  if (!aligned16(d_x) || !aligned16(d_y)) return fail(ADCT16_E_ALIGN, "d_x / d_y not 16-byte aligned");
  hipError_t e = launch_1d(false, d_x, d_y, n, (hipStream_t)stream);
  return e == hipSuccess ? ADCT16_OK : hip_fail(e, "1-D kernel");
}

adct16_status adct16_inverse_1d(const int32_t* d_x, int32_t* d_y, int64_t n, void* stream) {
  if (n < 0) return fail(ADCT16_E_SHAPE, "n < 0");
  if (n == 0) return ADCT16_OK;
  if (!d_x || !d_y) return fail(ADCT16_E_NULL, "d_x / d_y is NULL");
  if (!aligned16(d_x) || !aligned16(d_y)) return fail(ADCT16_E_ALIGN, "d_x / d_y not 16-byte aligned");
  hipError_t e = launch_1d(true, d_x, d_y, n, (hipStream_t)stream);
  return e == hipSuccess ? ADCT16_OK : hip_fail(e, "1-D kernel");
}

adct16_status adct16_graph_create(adct16_plan p, const void* d_in, void* d_out, void* d_qcoef, int64_t* d_sse,
                                  double* d_psnr, adct16_graph* out) {
  if (!out) return fail(ADCT16_E_NULL, "out is NULL");
  *out = nullptr;
  if (adct16_status st = check_plan(p)) return st;
  if (!d_in) return fail(ADCT16_E_NULL, "d_in is NULL");
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(ADCT16_E_LAUNCH, "capture stream");
  auto* g = new adct16_graph_s();
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  adct16_status st = ADCT16_OK;
  if (e == hipSuccess) {
    st = adct16_compress_and_measure(p, d_in, d_out, d_qcoef, d_sse, d_psnr, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
    if (st == ADCT16_OK && e2 != hipSuccess) st = hip_fail(e2, "end capture");
  } else {
    st = hip_fail(e, "begin capture");
  }
  if (st == ADCT16_OK) {
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) st = hip_fail(e, "graph instantiate");
  }
  (void)hipStreamDestroy(cs);
  if (st != ADCT16_OK) {
    adct16_graph_destroy(g);
    return st;
  }
  *out = g;
  return ADCT16_OK;
}

adct16_status adct16_graph_launch(adct16_graph g, void* stream) {
  if (!g) return fail(ADCT16_E_NULL, "graph is NULL");
  hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  return e == hipSuccess ? ADCT16_OK : hip_fail(e, "graph launch");
}

adct16_status adct16_graph_destroy(adct16_graph g) {
  if (!g) return fail(ADCT16_E_NULL, "graph is NULL");
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return ADCT16_OK;
}

}  // extern "C"
