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

#include <type_traits>

namespace {

constexpr int NT = 1024;
constexpr int LDS_BYTES = 64 * 1024;
constexpr int UNROLL = 8;

enum Op { READ_B32 = 0, READ_B64 = 1, ADD_U32 = 2, ADD_U64 = 3, ADD_F32 = 4, ADD_F64 = 5, READ2_ADJ = 6 };

template <int OP>
struct Elem;
template <> struct Elem<READ_B32> { using T = uint32_t; };
template <> struct Elem<READ_B64> { using T = uint64_t; };
template <> struct Elem<ADD_U32> { using T = uint32_t; };
template <> struct Elem<ADD_U64> { using T = unsigned long long; };
template <> struct Elem<ADD_F32> { using T = float; };
template <> struct Elem<ADD_F64> { using T = double; };
template <> struct Elem<READ2_ADJ> { using T = uint32_t; };

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
      else if constexpr (OP == READ2_ADJ) {  // two neighbouring words per lane (ds_read2_b32)
        const unsigned h = e & (unsigned)(N / 2 - 1);
        acc += (uint64_t)(lds[h] ^ lds[h + 1]);
      }
      else
        atomicAdd(&lds[e], T(1));
    }
    base += UNROLL * step;
  }
  __syncthreads();
  if constexpr (OP != READ_B32 && OP != READ_B64 && OP != READ2_ADJ) acc = (uint64_t)lds[threadIdx.x & (N - 1)];
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
 * ds_read_b64, 2 ds_add_u32, 3 ds_add_u64, 4 ds_add_f32, 5 ds_add_f64, 6 two
 * neighbouring 32-bit words per lane (ds_read2_b32, lane-ops count the pairs).
 * Every one of the blocks x 1024 threads issues `iters` operations (a
 * multiple of 8); `sink` is a device word the kernel may write.  Returns 0 or
 * a HIP error code; -1 for bad arguments. */
int lds_probe_run(int op, int stride, int iters, int blocks, void* sink, void* stream,
                  float* ms) {
  if (op < 0 || op > 6 || stride < 1 || stride > 1024 || iters < 8 || iters % UNROLL ||
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
      case ADD_F64: err = launch<ADD_F64>(stride, iters, blocks, k, s); break;
      default: err = launch<READ2_ADJ>(stride, iters, blocks, k, s); break;
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

// ---------------------------------------------------------------------------
// Access patterns of the push kernel's gather and deposit (quadratic 3D, 8^3
// tiles: field and current regions 13 x 13 x 13), replayed with lane
// layouts given by the caller: lanes[w * 64 + l] = cell of lane l of
// wavefront pattern w in the region (x + 13 (y + 13 z)), with the cell's
// class (bit d: offset >= 1/2 along d) in bits 16..18.  Wavefront v of the
// grid replays pattern v mod npat.  Mode 0: the single-precision gather (six
// components, 27 reads each at the component's own stencil); 1: the double
// one; 2: the single form's current deposit (54 ds_add_u64 of one virtual
// segment); 3: the double form's (ds_add_f64); 4: the single-precision gather
// with one ds_read_b32 per value; 5: the double one with one ds_read_b64 per
// value.
namespace {

constexpr int RX = 13, RV = RX * RX * RX;

template <int MODE>
__global__ void __launch_bounds__(NT) k_lds_pattern(const int* __restrict__ lanes, int npat,
                                                    int iters, uint64_t* sink) {
  // modes 4, 5: the gather with one read per value (reads through a
  // volatile LDS pointer are not paired into ds_read2)
  using T = typename std::conditional<MODE == 0 || MODE == 4, float,
            typename std::conditional<MODE == 2, unsigned long long, double>::type>::type;
  constexpr bool GATHER = MODE < 2 || MODE >= 4;
  constexpr int COMPS = GATHER ? 6 : 3;
  __shared__ T lds[COMPS * RV];
  for (int i = threadIdx.x; i < COMPS * RV; i += NT) lds[i] = T(i & 7);
  __syncthreads();
  const int wave = (int)((blockIdx.x * (NT / 64) + (threadIdx.x >> 6)) % (unsigned)npat);
  const int v = lanes[wave * 64 + (threadIdx.x & 63)];
  const int cell = v & 0xffff, cls = v >> 16;
  const int cb[3] = {cls & 1, (cls >> 1) & 1, (cls >> 2) & 1};
  int base[COMPS];
#pragma unroll
  for (int c = 0; c < COMPS; ++c) {
    // first stencil node relative to the cell (quadratic): a node-centred
    // axis starts at -1 + class bit, a staggered one at -1
    int sh = 0;
    const int e = c % 3;
    const bool isb = c >= 3;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const bool stag = GATHER ? (isb ? d != e : d == e) : false;
      const int str = d == 0 ? 1 : d == 1 ? RX : RX * RX;
      sh += ((stag ? 0 : cb[d]) - 1) * str;
    }
    base[c] = c * RV + cell + sh;
  }
  // nine independent sums (one per stencil row), so the adds do not form
  // one long dependency chain
  T acc9[9] = {};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < COMPS; ++c) {
      if constexpr (MODE >= 4) {
        typedef __attribute__((address_space(3))) const volatile T lf;
        lf* p = (lf*)(lds + base[c]);
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) acc9[3 * k + j] += p[i + RX * (j + RX * k)];
      } else if constexpr (MODE < 2) {
        const T* p = lds + base[c];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) acc9[3 * k + j] += p[i + RX * (j + RX * k)];
      } else {
        T* p = lds + base[c];
        // J_c: 2 nodes along c, 3 x 3 across
        const int sc = c == 0 ? 1 : c == 1 ? RX : RX * RX;
        const int sa = c == 0 ? RX : c == 1 ? RX * RX : 1;
        const int sb = c == 0 ? RX * RX : c == 1 ? 1 : RX;
#pragma unroll
        for (int ib = 0; ib < 3; ++ib)
#pragma unroll
          for (int ia = 0; ia < 3; ++ia)
#pragma unroll
            for (int ic = 0; ic < 2; ++ic) atomicAdd(&p[ic * sc + ia * sa + ib * sb], T(1));
      }
    }
  }
  T acc = T(0);
#pragma unroll
  for (int r = 0; r < 9; ++r) acc += acc9[r];
  if constexpr (!GATHER) {
    __syncthreads();
    acc = lds[threadIdx.x];
  }
  if (acc == T(12345)) sink[0] = 1;
}

template <int MODE>
int launch_pattern(const int* lanes, int npat, int iters, int blocks, uint64_t* sink, hipStream_t s) {
  k_lds_pattern<MODE><<<dim3((unsigned)blocks), dim3(NT), 0, s>>>(lanes, npat, iters, sink);
  return (int)hipGetLastError();
}

}  // namespace

extern "C" {

/* Replay the push kernel's LDS accesses (mode 0..5, see above) for `iters`
 * particle batches per wavefront with the lane layouts `lanes` (device,
 * npat x 64 ints: cell in the 13^3 region, class in bits 16..18; every
 * stencil stays inside the region for cells with coordinates 1..11) and
 * return the time in *ms (synchronises `stream`).  0 or a HIP error code;
 * -1 for bad arguments. */
int lds_probe_pattern(int mode, const void* lanes, int npat, int iters, int blocks, void* sink,
                      void* stream, float* ms) {
  if (mode < 0 || mode > 5 || !lanes || npat < 1 || iters < 1 || blocks < 1 || !sink || !ms)
    return -1;
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return -2;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return -2;
  }
  const int* L = (const int*)lanes;
  uint64_t* k = (uint64_t*)sink;
  int err = (int)hipEventRecord(a, s);
  if (!err) {
    switch (mode) {
      case 0: err = launch_pattern<0>(L, npat, iters, blocks, k, s); break;
      case 1: err = launch_pattern<1>(L, npat, iters, blocks, k, s); break;
      case 2: err = launch_pattern<2>(L, npat, iters, blocks, k, s); break;
      case 3: err = launch_pattern<3>(L, npat, iters, blocks, k, s); break;
      case 4: err = launch_pattern<4>(L, npat, iters, blocks, k, s); break;
      default: err = launch_pattern<5>(L, npat, iters, blocks, k, s); break;
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
