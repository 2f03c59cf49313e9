// Tile sort of the SoA particle arrays: counting sort on (tile of the
// particle's cell, rank of the particle within its cell); absorbed
// particles go to a last, dead bin.
//
// Not a step of the paper's method: it is the data layout that makes the
// fused push/deposit local (one workgroup per tile, fields and currents in
// LDS), the GPU counterpart of the paper's per-node particle partition
// (Sec. 3) and of its answer to deposit write conflicts (Sec. 3.1, Sec. 5.2).
//
// Inside a tile the particles come rank by rank: first one particle of
// every cell, then a second one of every cell that has two, and so on, so a
// wavefront's 64 lanes sit in different cells and their LDS accesses spread
// over the banks.  Ranks come from per-cell counters (clamped to RB - 1).
// Particles with equal keys are mostly contiguous already (they were
// sorted before and drift slowly), so the rank counters, the histogram and
// the scatter aggregate runs of equal values inside a wavefront: one global
// atomic per run instead of one per particle.
#include "k_common.h"

namespace pic {

constexpr int RB = SORT_RANKS;

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

// Rank within the cell (run-aggregated per-cell counters), bin key
// tile * RB + min(rank, RB - 1), and the histogram of the keys.
__global__ void k_sort_count(SortParams S, const int* __restrict__ cell, long np, int ncell,
                             int* __restrict__ cellcnt, int* __restrict__ keys,
                             int* __restrict__ counts, DevFlags* flg) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p == 0) flg->qmax = 0u;  // the scatter (next launch) takes the new maximum
  const int lane = threadIdx.x & 63;
  const int cl = p < np ? cell[p] : -1;
  const bool live = cl >= 0 && cl < ncell;
  int head, len;
  wave_runs(live ? cl : -1 - (int)(p < np), head, len);
  int rank = 0;
  if (live && lane == head) rank = atomicAdd(&cellcnt[cl], len);
  rank = __shfl(rank, head, 64) + (lane - head);
  const int key = p >= np ? -1 : live ? tile_key(S, cl, ncell) * RB + min(rank, RB - 1) : S.ntiles * RB;
  if (p < np) keys[p] = key;
  wave_runs(key, head, len);
  if (lane == head && key >= 0) atomicAdd(&counts[key], len);
}

// Exclusive scan of counts[0..nb) in three passes: per-block sums, a scan of
// the block sums (one workgroup), and per-block scans with their offsets.
// starts[i] = cursor[i] = sum of counts[0..i); starts[nb] = total.
constexpr int SCAN_B = 1024;

__device__ __forceinline__ int block_incl_scan(int v, int* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_B; off <<= 1) {
    const int a = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  return sh[t];
}

__global__ void __launch_bounds__(SCAN_B) k_scan_sums(const int* __restrict__ counts, int nb,
                                                      int* __restrict__ bsum) {
  __shared__ int sh[SCAN_B];
  const int i = blockIdx.x * SCAN_B + threadIdx.x;
  const int v = i < nb ? counts[i] : 0;
  const int incl = block_incl_scan(v, sh);
  if (threadIdx.x == SCAN_B - 1) bsum[blockIdx.x] = incl;
}

// one workgroup: exclusive scan of the nblk block sums in place
__global__ void __launch_bounds__(SCAN_B) k_scan_blocks(int* __restrict__ bsum, int nblk) {
  __shared__ int sh[SCAN_B];
  int carry = 0;
  for (int base = 0; base < nblk; base += SCAN_B) {
    const int i = base + threadIdx.x;
    const int v = i < nblk ? bsum[i] : 0;
    const int incl = block_incl_scan(v, sh);
    if (i < nblk) bsum[i] = carry + incl - v;
    carry += sh[SCAN_B - 1];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(SCAN_B) k_scan_apply(int* __restrict__ counts, int nb,
                                                       const int* __restrict__ bsum,
                                                       int* __restrict__ starts) {
  __shared__ int sh[SCAN_B];
  const int i = blockIdx.x * SCAN_B + threadIdx.x;
  const int v = i < nb ? counts[i] : 0;
  const int incl = block_incl_scan(v, sh);
  const int ex = bsum[blockIdx.x] + incl - v;
  if (i < nb) {
    starts[i] = ex;
    counts[i] = ex;  // cursor for the scatter
  }
  if (i == nb - 1) starts[nb] = ex + v;
}

// Tile starts for the push: tstart[t] = first particle of tile t
// (t = ntiles: first absorbed particle), tstart[ntiles + 1] = np.
__global__ void k_tile_starts(const int* __restrict__ bstart, int ntiles, int* __restrict__ tstart) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t <= ntiles) tstart[t] = bstart[t * RB];
  if (t == ntiles + 1) tstart[t] = bstart[ntiles * RB + 1];
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
__global__ void k_sort_scatter(SortArrays<R> A, long np, int ncell, int dims,
                               const int* __restrict__ keys, int* __restrict__ cursor,
                               DevFlags* flg) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const bool in = p < np;
  // the payload is loaded first, so that its latency overlaps the cursor
  // atomic's round trip
  const int cl = in ? A.cell[p] : 0;
  const int key = in ? keys[p] : -1;
  R o[3] = {R(0), R(0), R(0)}, u[3] = {R(0), R(0), R(0)}, qv = R(0);
  int idv = 0;
  if (in) {
    for (int d = 0; d < dims; ++d) o[d] = A.off[d][p];
    for (int c = 0; c < 3; ++c) u[c] = A.u[c][p];
    if (A.q) qv = A.q[p];
    if (A.id) idv = A.id[p];
  }
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
    if (in) {
      const R qa = fabs(qv);
      float f = (float)qa;
      if ((R)f < qa) f = nextafterf(f, INFINITY);
      m = __float_as_uint(f);
    }
    for (int sh = 32; sh > 0; sh >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, sh, 64));
    if (lane == 0) atomicMax(&flg->qmax, m);
  }
  if (!in) return;
  const long dst = (long)base + (lane - head);
  A.t_cell[dst] = (cl >= 0 && cl < ncell) ? cl : -1;
  for (int d = 0; d < dims; ++d) A.t_off[d][dst] = o[d];
  for (int c = 0; c < 3; ++c) A.t_u[c][dst] = u[c];
  if (A.id) A.t_id[dst] = idv;
  if (A.q) A.t_q[dst] = qv;
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
  int* bstart = (int*)(w + L.bstart);
  int* bsum = (int*)(w + L.bsum);
  int* cellcnt = (int*)(w + L.cellcnt);
  int* keys = (int*)(w + L.keys);
  const int nb = S.ntiles * RB + 1;  // + dead bin
  const int nblk = (nb + SCAN_B - 1) / SCAN_B;
  if (np == 0) {
    k_fill_int<<<dim3((S.ntiles + 2 + 255) / 256), dim3(256), 0, s>>>(starts, S.ntiles + 2, 0);
    return (int)hipGetLastError();
  }
  auto fill_grid = [](long n) { return dim3((unsigned)((n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384)); };
  k_fill_int<<<fill_grid(nb), dim3(256), 0, s>>>(counts, nb, 0);
  k_fill_int<<<fill_grid(ncell), dim3(256), 0, s>>>(cellcnt, ncell, 0);
  const unsigned grid = (unsigned)((np + 255) / 256);
  DevFlags* flg = (DevFlags*)(w + L.flags);
  k_sort_count<<<dim3(grid), dim3(256), 0, s>>>(S, p->cell, np, ncell, cellcnt, keys, counts, flg);
  k_scan_sums<<<dim3(nblk), dim3(SCAN_B), 0, s>>>(counts, nb, bsum);
  k_scan_blocks<<<dim3(1), dim3(SCAN_B), 0, s>>>(bsum, nblk);
  k_scan_apply<<<dim3(nblk), dim3(SCAN_B), 0, s>>>(counts, nb, bsum, bstart);
  k_tile_starts<<<dim3((S.ntiles + 2 + 255) / 256), dim3(256), 0, s>>>(bstart, S.ntiles, starts);
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
  k_sort_scatter<R><<<dim3(grid), dim3(256), 0, s>>>(A, np, ncell, c.dims, keys, counts, flg);
  const unsigned g2 = grid < 8192 ? grid : 8192;
  k_sort_copyback<R><<<dim3(g2), dim3(256), 0, s>>>(A, np, c.dims);
  return (int)hipGetLastError();
}

int launch_sort(const pic_ctx* ctx, const pic_particles* p, void* ws, hipStream_t s) {
  return ctx->cfg.real_bytes == 8 ? launch_sort_t<double>(ctx, p, ws, s)
                                  : launch_sort_t<float>(ctx, p, ws, s);
}

}  // namespace pic
