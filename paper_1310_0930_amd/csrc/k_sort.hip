// Tile sort of the SoA particle arrays: counting sort on the tile of each
// particle's cell (absorbed particles go to a last, dead bin).
//
// Not a step of the paper's method: it is the data layout that makes the
// fused push/deposit local (one workgroup per tile, fields and currents in
// LDS), the GPU counterpart of the paper's per-node particle partition
// (Sec. 3) and of its answer to deposit write conflicts (Sec. 3.1, Sec. 5.2).
//
// Particles that share a tile are mostly contiguous already (they were
// sorted before and drift slowly), so both the histogram and the scatter
// aggregate runs of equal keys inside a wavefront: one global atomic per
// run instead of one per particle, and each run keeps its order.
#include "k_common.h"

namespace pic {

struct SortParams {
  int n[3];
  int T[3];      // cells per tile (powers of two)
  int lgT[3];
  int ntile[3];
  int ntiles;
  int dims;
  FastDiv dn0, dn1;
};

__device__ __forceinline__ int tile_key(const SortParams& S, int cl, int ncell) {
  if (cl < 0 || cl >= ncell) return S.ntiles;  // dead bin
  const uint32_t rest = S.dn0.div((uint32_t)cl);
  const int cx = cl - (int)rest * S.n[0];
  int cy, cz;
  if (S.dims == 3) {
    const uint32_t r2 = S.dn1.div(rest);
    cy = (int)(rest - r2 * S.n[1]);
    cz = (int)r2;
  } else {
    cy = (int)rest;
    cz = 0;
  }
  return (cx >> S.lgT[0]) + S.ntile[0] * ((cy >> S.lgT[1]) + S.ntile[1] * (cz >> S.lgT[2]));
}

// Run structure of the keys held by one wavefront: a lane starts a run when
// its key differs from the previous lane's.  Returns the run's first lane and
// its length (for the first lane).
__device__ __forceinline__ void wave_runs(int key, int& head_lane, int& run_len) {
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(key, 1, 64);
  const bool boundary = lane == 0 || key != prev;
  const unsigned long long b = __ballot(boundary);
  // first lane of my run: highest boundary at or below me
  const unsigned long long below = lane == 63 ? b : (b & ((2ull << lane) - 1));
  head_lane = 63 - __clzll(below);
  // next boundary above my run head
  const unsigned long long above = head_lane == 63 ? 0ull : (b & ~((2ull << head_lane) - 1));
  const int next = above ? __ffsll(above) - 1 : 64;
  run_len = next - head_lane;
}

__global__ void k_sort_count(SortParams S, const int* __restrict__ cell, long np, int ncell,
                             int* __restrict__ counts, DevFlags* flg) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p == 0) flg->qmax = 0u;  // the scatter (next launch) takes the new maximum
  const int key = p < np ? tile_key(S, cell[p], ncell) : -1;
  int head, len;
  wave_runs(key, head, len);
  if ((int)(threadIdx.x & 63) == head && key >= 0) atomicAdd(&counts[key], len);
}

// Exclusive scan of counts[0..nb) into starts[0..nb] with one workgroup;
// the cursors (counts) are reset to the starts for the scatter.
__global__ void __launch_bounds__(1024) k_sort_scan(int* __restrict__ counts, int* __restrict__ starts, int nb) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int chunk = (nb + 1023) / 1024;
  const int lo = t * chunk;
  const int hi = min(lo + chunk, nb);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += counts[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;  // exclusive prefix of this chunk
  for (int i = lo; i < hi; ++i) {
    const int c = counts[i];
    starts[i] = run;
    counts[i] = run;
    run += c;
  }
  if (t == 1023) starts[nb] = part[1023];
}

template <typename R>
struct SortArrays {
  const int* cell;
  const R* off[3];
  const R* u[3];
  const R* q;
  const int* id;
  int* t_cell;
  R* t_off[3];
  R* t_u[3];
  R* t_q;
  int* t_id;
};

template <typename R>
__global__ void k_sort_scatter(SortParams S, SortArrays<R> A, long np, int ncell,
                               int* __restrict__ cursor, DevFlags* flg) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int cl = p < np ? A.cell[p] : 0;
  const int key = p < np ? tile_key(S, cl, ncell) : -1;
  int head, len;
  wave_runs(key, head, len);
  const int lane = threadIdx.x & 63;
  int base = 0;
  if (lane == head && key >= 0) base = atomicAdd(&cursor[key], len);
  base = __shfl(base, head, 64);
  if (A.q) {
    // largest |q| as a float bit pattern (non-negative floats order as
    // unsigned integers), rounded up so that it bounds every |q| of type R
    unsigned m = 0u;
    if (p < np) {
      const R qa = fabs(A.q[p]);
      float f = (float)qa;
      if ((R)f < qa) f = nextafterf(f, INFINITY);
      m = __float_as_uint(f);
    }
    for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o, 64));
    if (lane == 0) atomicMax(&flg->qmax, m);
  }
  if (p >= np) return;
  const long dst = (long)base + (lane - head);
  A.t_cell[dst] = (cl >= 0 && cl < ncell) ? cl : -1;
  for (int d = 0; d < S.dims; ++d) A.t_off[d][dst] = A.off[d][p];
  for (int c = 0; c < 3; ++c) A.t_u[c][dst] = A.u[c][p];
  if (A.id) A.t_id[dst] = A.id[p];
  if (A.q) A.t_q[dst] = A.q[p];
}

template <typename R>
__global__ void k_sort_copyback(SortArrays<R> A, long np, int dims) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < np; i += (long)gridDim.x * blockDim.x) {
    const_cast<int*>(A.cell)[i] = A.t_cell[i];
    for (int d = 0; d < dims; ++d) const_cast<R*>(A.off[d])[i] = A.t_off[d][i];
    for (int c = 0; c < 3; ++c) const_cast<R*>(A.u[c])[i] = A.t_u[c][i];
    if (A.q) const_cast<R*>(A.q)[i] = A.t_q[i];
    if (A.id) const_cast<int*>(A.id)[i] = A.t_id[i];
  }
}

__global__ void k_fill_int(int* a, long n, int v) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    a[i] = v;
}

template <typename R>
static int launch_sort_t(const pic_ctx* ctx, const pic_particles* p, void* ws, hipStream_t s) {
  SortParams S;
  const pic_config& c = ctx->cfg;
  S.dims = c.dims;
  for (int d = 0; d < 3; ++d) {
    S.n[d] = d < c.dims ? c.n[d] : 1;
    S.T[d] = ctx->tile[d];
    int lg = 0;
    while ((1 << lg) < S.T[d]) ++lg;
    S.lgT[d] = lg;
    S.ntile[d] = ctx->ntile[d];
  }
  S.ntiles = ctx->ntiles;
  S.dn0.init((uint32_t)S.n[0]);
  S.dn1.init((uint32_t)S.n[1]);
  const int ncell = S.n[0] * S.n[1] * S.n[2];
  const long np = p->np;
  WsLayout L = ws_layout(ctx, np);
  char* w = (char*)ws;
  int* counts = (int*)(w + L.counts);
  int* starts = (int*)(w + L.starts);
  const int nb = S.ntiles + 1;  // + dead bin
  k_fill_int<<<dim3((nb + 255) / 256), dim3(256), 0, s>>>(counts, nb + 1, 0);
  if (np == 0) {
    k_fill_int<<<dim3((nb + 256) / 256), dim3(256), 0, s>>>(starts, nb + 1, 0);
    return (int)hipGetLastError();
  }
  const unsigned grid = (unsigned)((np + 255) / 256);
  DevFlags* flg = (DevFlags*)(w + L.flags);
  k_sort_count<<<dim3(grid), dim3(256), 0, s>>>(S, p->cell, np, ncell, counts, flg);
  k_sort_scan<<<dim3(1), dim3(1024), 0, s>>>(counts, starts, nb);
  SortArrays<R> A;
  A.cell = p->cell;
  R* tr = (R*)(w + L.tmp_real);
  for (int d = 0; d < 3; ++d) {
    A.off[d] = (const R*)p->off[d];
    A.u[d] = (const R*)p->u[d];
    A.t_off[d] = tr + (size_t)d * np;
    A.t_u[d] = tr + (size_t)(3 + d) * np;
  }
  A.q = (const R*)p->q;
  A.t_q = tr + (size_t)6 * np;
  A.id = p->id;
  A.t_cell = (int*)(w + L.tmp_cell);
  A.t_id = (int*)(w + L.tmp_id);
  k_sort_scatter<R><<<dim3(grid), dim3(256), 0, s>>>(S, A, np, ncell, counts, flg);
  const unsigned g2 = grid < 8192 ? grid : 8192;
  k_sort_copyback<R><<<dim3(g2), dim3(256), 0, s>>>(A, np, c.dims);
  return (int)hipGetLastError();
}

int launch_sort(const pic_ctx* ctx, const pic_particles* p, void* ws, hipStream_t s) {
  return ctx->cfg.real_bytes == 8 ? launch_sort_t<double>(ctx, p, ws, s)
                                  : launch_sort_t<float>(ctx, p, ws, s);
}

}  // namespace pic
