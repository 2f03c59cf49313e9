// LDS throughput probe for gfx950 (not part of the PIC step).
//
// Measures how many LDS lane-operations per second the chip sustains for
// the access kinds the push/deposit kernel issues (32- and 64-bit reads,
// integer and floating-point atomic adds without return), with the 64 lanes
// of every wavefront at addresses `stride` elements apart.  stride = 1 is
// the conflict-free case whose rate is the peak the push kernel's LDS
// atomics are compared against; larger strides expose the bank structure
// (lanes whose addresses share a bank serialize).
//
// Each workgroup (1024 threads, 16 wavefronts: one per SIMD slot as in the
// push kernel) owns a 64 KB LDS array; wavefront w uses base address
// w * 64 * stride + iteration * 64 * stride (modulo the array), so its 64
// lanes never share an address and the bank pattern inside every
// instruction is that of the stride alone.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int NT = 1024;
constexpr int LDS_BYTES = 64 * 1024;
constexpr int UNROLL = 8;

enum Op { READ_B32 = 0, READ_B64 = 1, ADD_U32 = 2, ADD_U64 = 3, ADD_F32 = 4, ADD_F64 = 5 };

template <int OP>
struct Elem;
template <> struct Elem<READ_B32> { using T = uint32_t; };
template <> struct Elem<READ_B64> { using T = uint64_t; };
template <> struct Elem<ADD_U32> { using T = uint32_t; };
template <> struct Elem<ADD_U64> { using T = unsigned long long; };
template <> struct Elem<ADD_F32> { using T = float; };
template <> struct Elem<ADD_F64> { using T = double; };

template <int OP>
__global__ void __launch_bounds__(NT) k_lds_rate(int stride, int iters, uint64_t* sink) {
  using T = typename Elem<OP>::T;
  constexpr int N = LDS_BYTES / sizeof(T);  // elements, a power of two
  __shared__ T lds[N];
  for (int i = threadIdx.x; i < N; i += NT) lds[i] = T(0);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned lane_off = (unsigned)(lane * stride);
  unsigned base = (unsigned)(wave * 64 * stride);
  const unsigned step = (unsigned)(64 * stride);
  uint64_t acc = 0;
  for (int it = 0; it < iters; it += UNROLL) {
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const unsigned e = (base + lane_off + (unsigned)u * step) & (unsigned)(N - 1);
      if constexpr (OP == READ_B32 || OP == READ_B64)
        acc += (uint64_t)lds[e];
      else
        atomicAdd(&lds[e], T(1));
    }
    base += UNROLL * step;
  }
  __syncthreads();
  if constexpr (OP != READ_B32 && OP != READ_B64) acc = (uint64_t)lds[threadIdx.x & (N - 1)];
  if (acc == 0x9e3779b97f4a7c15ull) sink[0] = acc;  // keeps the reads alive
}

template <int OP>
int launch(int stride, int iters, int blocks, uint64_t* sink, hipStream_t s) {
  k_lds_rate<OP><<<dim3((unsigned)blocks), dim3(NT), 0, s>>>(stride, iters, sink);
  return (int)hipGetLastError();
}

}  // namespace

extern "C" {

/* Run the probe once on `stream` and return the time it took in *ms (HIP
 * events on that stream; synchronises it).  op: 0 ds_read_b32, 1
 * ds_read_b64, 2 ds_add_u32, 3 ds_add_u64, 4 ds_add_f32, 5 ds_add_f64.
 * Every one of the blocks x 1024 threads issues `iters` operations (a
 * multiple of 8); `sink` is a device word the kernel may write.  Returns 0 or
 * a HIP error code; -1 for bad arguments. */
int lds_probe_run(int op, int stride, int iters, int blocks, void* sink, void* stream,
                  float* ms) {
  if (op < 0 || op > 5 || stride < 1 || stride > 1024 || iters < 8 || iters % UNROLL ||
      blocks < 1 || !sink || !ms)
    return -1;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return -2;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return -2;
  }
  int err = (int)hipEventRecord(a, s);
  uint64_t* k = (uint64_t*)sink;
  if (!err) {
    switch (op) {
      case READ_B32: err = launch<READ_B32>(stride, iters, blocks, k, s); break;
      case READ_B64: err = launch<READ_B64>(stride, iters, blocks, k, s); break;
      case ADD_U32: err = launch<ADD_U32>(stride, iters, blocks, k, s); break;
      case ADD_U64: err = launch<ADD_U64>(stride, iters, blocks, k, s); break;
      case ADD_F32: err = launch<ADD_F32>(stride, iters, blocks, k, s); break;
      default: err = launch<ADD_F64>(stride, iters, blocks, k, s); break;
    }
  }
  if (!err) err = (int)hipEventRecord(b, s);
  if (!err) err = (int)hipEventSynchronize(b);
  if (!err) err = (int)hipEventElapsedTime(ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return err;
}

}  // extern "C"
