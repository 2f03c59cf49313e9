// Device helpers shared by the libpic kernels.
#pragma once
#include "pic_internal.h"

namespace pic {

// Wrap an index into [0, n) when it is at most one period outside.
__device__ __forceinline__ int wrap1(int i, int n) {
  i = i < 0 ? i + n : i;
  return i >= n ? i - n : i;
}

// Storage index along one axis of a sample with lattice index i, for a
// quantity node-located (st = 0) or half-way (st = 1) along that axis;
// -1 when outside the domain of an open axis.  Periodic axes wrap (any
// number of periods: a tile's LDS region may be wider than a small grid).
__device__ __forceinline__ int axis_slot(int i, int n, int open, int st) {
  if (!open) {
    if (i >= 0 && i < n) return i;
    if (i < 0 && i >= -n) return i + n;
    if (i >= n && i < 2 * n) return i - n;
    const int m = i % n;
    return m < 0 ? m + n : m;
  }
  return (i < 0 || i > n - 1 - st) ? -1 : i;
}

// Storage offsets along one axis of the sample at lattice index i, for a
// node-located (s[0]) and a staggered (s[1]) quantity, already multiplied
// by the axis stride; -1 outside the domain of an open axis.  Region loops
// form them once per sample and share them over the field components.
__device__ __forceinline__ void axis_slots(int i, int n, int open, int stride, int* s) {
  if (!open) {
    s[0] = s[1] = axis_slot(i, n, 0, 0) * stride;
    return;
  }
  s[0] = (i < 0 || i > n - 1) ? -1 : i * stride;
  s[1] = (i < 0 || i > n - 2) ? -1 : i * stride;
}

// True when the samples lo .. lo+w-1 of an axis need no wrap and no open
// boundary handling for either staggering (a region's fast path).
__device__ __forceinline__ bool axis_inside(int lo, int w, int n, int open) {
  return lo >= 0 && lo + w <= n - open;
}

template <typename R>
__device__ __forceinline__ void atomic_add(R* p, R v) {
  atomicAdd(p, v);
}

__device__ __forceinline__ void raise_flag(DevFlags* f, unsigned bit) {
  atomicOr(&f->flags, bit);
}

}  // namespace pic
