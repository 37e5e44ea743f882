// Streaming of strips for the persistent matrix-core kernels: the task
// table (runs of strips of one block row) dealt out to wavefronts, the image
// geometry of the current task held in scalars, and 16-byte row accesses
// with optional non-temporal hints.
#pragma once

#include "adct16_internal.hpp"

namespace adct16 {

// Streaming accesses: every byte of the batch is read once and written
// once, so when the row segments are whole cache lines (128-byte aligned
// pitches, offsets and buffers) the 16-byte row accesses carry the
// non-temporal hint.  With unaligned rows a segment straddles two lines that
// neighbouring strips share, and the hint would make them fetch it twice.
typedef unsigned v4u __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ uint4 ld_row16(const uint8_t* p) {
  if constexpr (NT) {
    const v4u v = __builtin_nontemporal_load(reinterpret_cast<const v4u*>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
  } else {
    return *reinterpret_cast<const uint4*>(p);
  }
}
template <bool NT>
__device__ __forceinline__ void st_row16(uint8_t* p, const uint4& v) {
  if constexpr (NT) {
    const v4u w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<v4u*>(p));
  } else {
    *reinterpret_cast<uint4*>(p) = v;
  }
}

// The fields of an image that the fused kernel uses, held in scalars.
struct ImgGeom {
  int64_t offset;
  int32_t h, w, pitch, bx, sx;
  int64_t block_begin;
};

// One dword of block row q (columns 4g..4g+3), edge-extended.
__device__ __forceinline__ unsigned load_dword_edge(const uint8_t* img, const ImgGeom& d, int y, int x0) {
  const int64_t off = d.offset + (int64_t)y * d.pitch;
  if (x0 + 3 < d.w) return *reinterpret_cast<const unsigned*>(img + off + x0);
  unsigned r = 0;
  for (int k = 0; k < 4; ++k) r |= (unsigned)img[off + min(x0 + k, d.w - 1)] << (8 * k);
  return r;
}

// Task registers: lane k of a wavefront holds the table entry and the image
// geometry of its task t0 + k W (the k-th of its next 64 tasks), gathered
// with one set of vector loads; the task in use is read back with readlane.
// The table latency is paid once per 64 tasks instead of once per task.
struct TaskRegs {
  int sy, run, off_lo, off_hi, h, w, pitch, bx, sx, bb_lo, bb_hi;
};

__device__ __forceinline__ TaskRegs gather_tasks(const ImageDesc* __restrict__ images,
                                                 const RowTask* __restrict__ rows, int64_t t0, int64_t W,
                                                 int64_t n, int lane) {
  TaskRegs tr = {0, 0, 0, 0, 1, 1, 0, 0, 1, 0, 0};
  const int64_t tk = t0 + (int64_t)lane * W;
  if (tk < n) {
    const RowTask e = rows[tk];
    const ImageDesc* d = images + e.img;
    const int64_t off = d->offset;
    tr.sy = e.sy;
    tr.run = e.run;
    tr.off_lo = (int)(uint32_t)off;
    tr.off_hi = (int)(off >> 32);
    tr.h = d->h;
    tr.w = d->w;
    tr.pitch = d->pitch;
    tr.bx = d->bx;
    tr.sx = d->sx;
    const int64_t bb = d->block_begin;
    tr.bb_lo = (int)(uint32_t)bb;
    tr.bb_hi = (int)(bb >> 32);
  }
  // complete the gather here, so that reading a task (every few strips)
  // never waits on memory; vmcnt(0), other counters unchanged
  __builtin_amdgcn_s_waitcnt(0x0F70);
  return tr;
}

__device__ __forceinline__ ImgGeom task_geom(const TaskRegs& tr, int k) {
  ImgGeom m;
  m.offset = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(tr.off_hi, k) << 32) |
                       (uint32_t)__builtin_amdgcn_readlane(tr.off_lo, k));
  m.h = __builtin_amdgcn_readlane(tr.h, k);
  m.w = __builtin_amdgcn_readlane(tr.w, k);
  m.pitch = __builtin_amdgcn_readlane(tr.pitch, k);
  m.bx = __builtin_amdgcn_readlane(tr.bx, k);
  m.sx = __builtin_amdgcn_readlane(tr.sx, k);
  m.block_begin = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(tr.bb_hi, k) << 32) |
                            (uint32_t)__builtin_amdgcn_readlane(tr.bb_lo, k));
  return m;
}

}  // namespace adct16
