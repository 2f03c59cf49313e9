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
    const int m = i % n;
    return m < 0 ? m + n : m;
  }
  return (i < 0 || i > n - 1 - st) ? -1 : i;
}

template <typename R>
__device__ __forceinline__ void atomic_add(R* p, R v) {
  atomicAdd(p, v);
}

__device__ __forceinline__ void raise_flag(DevFlags* f, unsigned bit) {
  atomicOr(&f->flags, bit);
}

}  // namespace pic
