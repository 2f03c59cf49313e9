// Tile sort of the SoA particle arrays, in two levels: a counting sort on
// the tile of the particle's cell (absorbed particles go to a last, dead
// bin, which is dropped: the live particles are compacted to the front),
// then, inside every tile, a placement by class and bank residue.
//
// Not a step of the paper's method: it is the data layout that makes the
// fused push/deposit local (one workgroup per tile, fields and currents in
// LDS), the GPU counterpart of the paper's per-node particle partition
// (Sec. 3) and of its answer to deposit write conflicts (Sec. 3.1, Sec. 5.2).
//
// Inside a tile the particles come class by class.  The class is the half
// of the cell the particle sits in along each axis (offset >= 1/2 or not),
// which fixes the first stencil node of every field and current component
// relative to the cell, so that the 64 lanes of a wavefront read and add at
// their cells' bases plus one common offset.  Within a class the particles
// cycle through the LDS bank residues of their cells (k_sort_place), so that
// those bases fall on distinct banks.  Particles move between sorts and the
// layout decays, so the class and cell used for the placement are those a
// straight-line estimate gives half a sort interval ahead (the particle's
// tile is still that of its present cell); the layout is then best in the
// middle of the interval rather than at its start.  The tile-level pass aggregates runs
// of equal tiles inside a wavefront (particles stay in their tile for many
// steps), one global atomic per run; the placement runs in LDS, one
// workgroup per tile.
#include <type_traits>

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
  // row and plane strides (elements) of the push kernel's LDS region whose
  // element indices decide the lanes' banks (region_strides_t)
  int rs1, rs2;
  // placement estimate: cells moved per unit of u_d over half a sort
  // interval, ((sort_every - 1) / 2) dt / dx_d
  double hdx[3];
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
template <typename K>
__device__ __forceinline__ void wave_runs(K key, int& head_lane, int& run_len) {
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

// Workgroup b of n takes chunk (b * M) mod n (M prime; a permutation of
// the chunks unless M divides n).  Sorted particles of one tile are
// contiguous, so in block order the wavefronts running together would all
// add to the same bin counter or cursor, and same-address device atomics
// serialize; in this order they spread over many tiles.
__device__ __forceinline__ long spread_block(unsigned b, unsigned n) {
  constexpr unsigned long long M = 1000003ull;
  return n % M == 0 ? (long)b : (long)(((unsigned long long)b * M) % n);
}

// Tile key of every particle (ntiles: dead) and the histogram of the keys.
// A workgroup takes COUNT_PER consecutive particles (chunks spread as
// above); runs of the chunk's first key, which after a sort is the tile of
// nearly the whole chunk, are summed in LDS and added with one global
// atomic, other runs add their own.
constexpr int COUNT_NT = 256, COUNT_PER = 8;
__global__ void __launch_bounds__(COUNT_NT) k_sort_count(SortParams S, const int* __restrict__ cell,
                                                         long np, int ncell, int* __restrict__ keys,
                                                         int* __restrict__ counts, DevFlags* flg) {
  __shared__ int acc;
  const long c0 = spread_block(blockIdx.x, gridDim.x) * (long)(COUNT_NT * COUNT_PER);
  if (c0 == 0 && threadIdx.x == 0) {
    flg->qmax = 0u;  // the scatter takes the new maximum
    flg->ndefer = 0u;  // a new sort interval starts
    flg->since_sort = 0ull;
  }
  const int lane = threadIdx.x & 63;
  const int key0 = c0 < np ? tile_key(S, cell[c0], ncell) : -1;
  if (threadIdx.x == 0) acc = 0;
  __syncthreads();
  int mine = 0;  // this thread's run lengths of key0
#pragma unroll
  for (int k = 0; k < COUNT_PER; ++k) {
    const long p = c0 + k * COUNT_NT + threadIdx.x;
    const int key = p < np ? tile_key(S, cell[p], ncell) : -1;
    if (p < np) keys[p] = key;
    if (__ballot(key == key0) == ~0ull) {  // the whole wavefront in key0's tile (the usual case)
      if (lane == 0) mine += 64;
      continue;
    }
    int head, len;
    wave_runs(key, head, len);
    if (lane == head && key >= 0) {
      if (key == key0)
        mine += len;
      else
        atomicAdd(&counts[key], len);
    }
  }
  if (mine) atomicAdd(&acc, mine);
  __syncthreads();
  if (threadIdx.x == 0 && acc) atomicAdd(&counts[key0], acc);
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
  if (t <= ntiles + 1) tstart[t] = bstart[t];
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

// Cells of a tile (at most; 8^3 in 3D, 16^2 in 2D).
constexpr int TILE_CELLS_MAX = 512;

// In-tile placement key of a live particle of tile t: its class (the half
// of the cell along each axis) and its cell within the tile, both of the
// position a straight line gives half a sort interval ahead,
// x_d + clamp(u_d, -1, 1) hdx_d (|u_d| for the speed below c, its bound
// above), rounded operation by operation in double so that a host can
// restate it exactly; the present cell and offsets when that cell leaves
// the tile.
template <typename R>
__device__ __forceinline__ int placement_key(const SortParams& S, int t, int cl, const R* o,
                                             const R* u) {
  const int tx = t % S.ntile[0], ty = (t / S.ntile[0]) % S.ntile[1], tz = t / (S.ntile[0] * S.ntile[1]);
  const uint32_t rest = S.dn0.div((uint32_t)cl);
  const int cx = cl - (int)rest * S.n[0];
  int cy = (int)rest, cz = 0;
  if (S.dims == 3) {
    const uint32_t r2 = S.dn1.div(rest);
    cy = (int)(rest - r2 * S.n[1]);
    cz = (int)r2;
  }
  const int lc[3] = {cx - tx * S.T[0], cy - ty * S.T[1], cz - tz * S.T[2]};
  int lp[3] = {lc[0], lc[1], lc[2]};
  double op[3] = {0.0, 0.0, 0.0};
  bool in = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d < S.dims) {
      const double v = fmin(fmax((double)u[d], -1.0), 1.0);
      const double x = __dadd_rn((double)o[d], __dmul_rn(v, S.hdx[d]));
      const double f = floor(x);
      lp[d] = lc[d] + (int)f;
      op[d] = x - f;
      in = in && lp[d] >= 0 && lp[d] < S.T[d];
    }
  }
  if (!in) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lp[d] = lc[d];
      op[d] = (double)o[d];
    }
  }
  int cls = (op[0] >= 0.5 ? 1 : 0) | (op[1] >= 0.5 ? 2 : 0);
  if (S.dims == 3) cls |= op[2] >= 0.5 ? 4 : 0;
  return cls * TILE_CELLS_MAX + lp[0] + S.T[0] * (lp[1] + S.T[1] * lp[2]);
}

// Copies every particle to its tile's range of the scratch arrays (in the
// order the atomics give) and records its in-tile placement key there.
template <typename R>
__global__ void k_sort_scatter(SortArrays<R> A, SortParams S, long np, int ncell,
                               const int* __restrict__ keys, int* __restrict__ cursor,
                               int* __restrict__ pkey, DevFlags* flg) {
  const int dims = S.dims;
  const long p = spread_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
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
  int head = 0, len = 64;
  if (__ballot(key == __builtin_amdgcn_readfirstlane(key)) != ~0ull)  // else one run (usual)
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
    // every wavefront's atomic on the one word would serialize: skip it when
    // the maximum so far (a possibly stale read, which can only cost an
    // extra atomic) already covers this wavefront's
    if (lane == 0 && m > __hip_atomic_load(&flg->qmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(&flg->qmax, m);
  }
  if (!in) return;
  const long dst = (long)base + (lane - head);
  const bool live = cl >= 0 && cl < ncell;
  if (live) pkey[dst] = placement_key<R>(S, key, cl, o, u);
  A.t_cell[dst] = live ? cl : -1;
  for (int d = 0; d < dims; ++d) A.t_off[d][dst] = o[d];
  for (int c = 0; c < 3; ++c) A.t_u[c][dst] = u[c];
  if (A.id) A.t_id[dst] = idv;
  if (A.q) A.t_q[dst] = qv;
}

// One particle's payload in registers: every load first, then every store
// (a store to one array may alias a later load of another as far as the
// compiler knows, which would serialize the round trips), and batched
// copies keep all loads of a batch in flight together.
template <typename R>
struct PVal {
  int cl, id;
  R o[3], u[3], q;
  __device__ __forceinline__ void load(const SortArrays<R>& A, long i, int dims) {
    cl = A.t_cell[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) o[d] = d < dims ? A.t_off[d][i] : R(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = A.t_u[c][i];
    q = A.q ? A.t_q[i] : R(0);
    id = A.id ? A.t_id[i] : 0;
  }
  __device__ __forceinline__ void store(const SortArrays<R>& A, long j, int dims) const {
    const_cast<int*>(A.cell)[j] = cl;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (d < dims) const_cast<R*>(A.off[d])[j] = o[d];
#pragma unroll
    for (int c = 0; c < 3; ++c) const_cast<R*>(A.u[c])[j] = u[c];
    if (A.q) const_cast<R*>(A.q)[j] = q;
    if (A.id) const_cast<int*>(A.id)[j] = id;
  }
};

// Bank residues of a tile's cells.  In the push every LDS access of a
// wavefront is the lanes' cell base addresses plus one offset common to
// the lanes of one class (one stencil shape).  The LDS has 32 four-byte
// banks and serves a wavefront's 4-byte accesses 32 lanes per cycle and its
// 8-byte accesses (the current tile's atomics, the double-precision field
// reads) 16 lanes per cycle, two banks each.  Lanes in one such group go
// through without conflict when their cells' element indices in the region
// differ modulo the group size; 32 consecutive distinct residues
// modulo 32 are also 16 distinct residues modulo 16 in each half, so the
// residue is taken modulo 32 in both precisions (replayed access patterns:
// modulo 16 costs the double-precision gather and deposit 18 % more LDS
// cycles).  One workgroup lists the tile's cells by residue:
// order[0 .. ncells) = cells sorted by (residue, cell),
// order[TILE_CELLS_MAX + r] = first entry of residue r (r <= RES).
constexpr int ORDER_NT = 512;
constexpr int RES = 32;
static_assert(RES <= 32, "residue masks are 32-bit words");
__device__ __forceinline__ int cell_residue(const SortParams& S, int lc) {
  const int lx = lc % S.T[0], ly = (lc / S.T[0]) % S.T[1], lz = lc / (S.T[0] * S.T[1]);
  return (lx + S.rs1 * ly + S.rs2 * lz) % RES;
}

__global__ void __launch_bounds__(ORDER_NT) k_sort_order(SortParams S, int* __restrict__ order) {
  __shared__ int cnt[RES];
  __shared__ int res[ORDER_NT];
  const int ncells = S.T[0] * S.T[1] * S.T[2];
  const int lc = threadIdx.x;
  if (lc < RES) cnt[lc] = 0;
  int r = 0;
  if (lc < ncells) {
    r = cell_residue(S, lc);
    res[lc] = r;
  }
  __syncthreads();
  if (lc < ncells) atomicAdd(&cnt[r], 1);
  __syncthreads();
  if (lc < ncells) {
    int pos = 0;
    for (int q = 0; q < r; ++q) pos += cnt[q];
    for (int c = 0; c < lc; ++c) pos += res[c] == r;
    order[pos] = lc;
  }
  if (lc <= RES) {
    int st = 0;
    for (int q = 0; q < lc; ++q) st += cnt[q];
    order[TILE_CELLS_MAX + lc] = st;
  }
}

// Placement of one tile's particles (one workgroup per tile) from the
// scatter's copy back into the particle arrays.  Pass 1 gives every particle
// its class and its rank among the particles of its (cell, class), from LDS
// counters; class and cell are those of the placement key the scatter
// recorded (placement_key: the position estimated half a sort interval
// ahead).  Within a class the particles are ranked by (k, r): r is the
// residue of the particle's cell, k the number of the class's particles of
// the same residue before it (cells in cell order, a cell's particles in
// rank order).  The class cycles through the residues it holds, so any RES
// consecutive lanes of a full cycle fall on distinct banks, and particles of
// one cell sit a whole cycle apart.  One thread per (class, residue) walks
// that residue's cells for the first k of every cell; pass 2 puts each
// particle at its class's start plus its rank in the class.
constexpr int PLACE_NT = 1024;
constexpr int PLACE_SRC_MAX = 8192;
template <typename R>
__global__ void __launch_bounds__(PLACE_NT) k_sort_place(SortArrays<R> A, SortParams S,
                                                          const int* __restrict__ tstart,
                                                          const int* __restrict__ order,
                                                          int* __restrict__ scratch, int dims) {
  constexpr int NC = 8;                           // classes (2^dims)
  // counters of passes 1-2, then (pass 3) one particle array of the tile
  constexpr size_t POOL = 2 * sizeof(int) * NC * TILE_CELLS_MAX > sizeof(R) * PLACE_SRC_MAX
                              ? 2 * sizeof(int) * NC * TILE_CELLS_MAX
                              : sizeof(R) * PLACE_SRC_MAX;
  __shared__ __align__(16) unsigned char pool[POOL];
  int* const cnt = (int*)pool;                   // particles per (class, cell)
  int* const kb = cnt + NC * TILE_CELLS_MAX;     // k of the first of them
  // particles per (class, residue), rows padded so that the lanes of one
  // wavefront reading one residue of different classes hit different banks
  __shared__ int cntr[NC][RES + 1];
  __shared__ int ctot[NC];                        // particles per class
  __shared__ int cls0[NC + 1];                    // first slot of each class
  // per (class, level k < KT): slots of the levels below k, and the
  // residues that reach level k (bit mask)
  constexpr int KT = 64;
  __shared__ int lvl0[NC][KT];
  __shared__ unsigned lvlm[NC][KT];
  __shared__ int ord[TILE_CELLS_MAX + RES + 1];
  __shared__ unsigned char res[TILE_CELLS_MAX];
  __shared__ int src[PLACE_SRC_MAX];  // source of each slot of the tile
  const int t = blockIdx.x;
  const int beg = tstart[t], end = tstart[t + 1];
  if (beg == end) return;
  const int ncells = S.T[0] * S.T[1] * S.T[2];
  for (int i = threadIdx.x; i < ncells; i += PLACE_NT) {
    ord[i] = order[i];
    res[i] = (unsigned char)cell_residue(S, i);
  }
  for (int i = threadIdx.x; i <= RES; i += PLACE_NT) ord[TILE_CELLS_MAX + i] = order[TILE_CELLS_MAX + i];
  for (int i = threadIdx.x; i < NC * TILE_CELLS_MAX; i += PLACE_NT) cnt[i] = 0;
  __syncthreads();
  // pass 1: rank of every particle among those of its (class, cell), from
  // the placement keys the scatter recorded (batches of PB1 per thread, all
  // loads of a batch in flight together); scratch = rank, class, cell
  constexpr int PB1 = 4;
  for (int i0 = beg + threadIdx.x; i0 < end; i0 += PB1 * PLACE_NT) {
    int kv[PB1];
#pragma unroll
    for (int k = 0; k < PB1; ++k) {
      const int i = i0 + k * PLACE_NT;
      kv[k] = i < end ? scratch[i] : 0;
    }
#pragma unroll
    for (int k = 0; k < PB1; ++k) {
      const int i = i0 + k * PLACE_NT;
      if (i < end) {
        const int rank = atomicAdd(&cnt[kv[k]], 1);
        scratch[i] = (rank << 12) | kv[k];
      }
    }
  }
  __syncthreads();
  // first k of every (class, cell) and the (class, residue) totals: one
  // thread per (class, residue) walks the residue's cells in cell order
  const int ncls = 1 << dims;
  if (threadIdx.x < ncls * RES) {
    const int cls = threadIdx.x / RES, r = threadIdx.x % RES;
    int k = 0;
    for (int i = ord[TILE_CELLS_MAX + r]; i < ord[TILE_CELLS_MAX + r + 1]; ++i) {
      const int key = cls * TILE_CELLS_MAX + ord[i];
      kb[key] = k;
      k += cnt[key];
    }
    cntr[cls][r] = k;
    // class total: a class is RES = 32 consecutive lanes of one wavefront
    int t = k;
#pragma unroll
    for (int m = RES / 2; m >= 1; m >>= 1) t += __shfl_xor(t, m, RES);
    if (r == 0) ctot[cls] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = beg;
    for (int c = 0; c < ncls; ++c) {
      cls0[c] = acc;
      acc += ctot[c];
    }
    cls0[ncls] = acc;
  }
  // per (class, level): slots of the levels below and the residues present
  for (int t = threadIdx.x; t < ncls * KT; t += PLACE_NT) {
    const int cls = t / KT, k = t % KT;
    int below = 0;
    unsigned m = 0u;
#pragma unroll
    for (int q = 0; q < RES; ++q) {
      const int c = cntr[cls][q];
      below += min(c, k);
      m |= (c > k ? 1u : 0u) << q;
    }
    lvl0[cls][k] = below;
    lvlm[cls][k] = m;
  }
  __syncthreads();
  const int n = end - beg;
  const bool staged = n <= PLACE_SRC_MAX;
  // Slots.  When the tile fits, pass 2 records the source of every slot in
  // LDS and pass 3 moves the particle arrays one at a time through LDS:
  // coalesced loads of the tile's copy, coalesced stores in slot order
  // (gathered loads from the copy straight out of memory had each touched a
  // cache line per lane); a larger tile stores directly.
  //
  // Slot of a particle: rank of (k, r) in the class: every residue with more
  // than k particles fills levels 0..k, those below r also level k
  auto slot = [&](int v) {
    const int key = v & 4095, cls = key / TILE_CELLS_MAX, lc = key % TILE_CELLS_MAX;
    const int k = kb[key] + (v >> 12), r = res[lc];
    if (k < KT)  // levels below k, then the residues below r that reach level k
      return cls0[cls] + lvl0[cls][k] + (int)__popc(lvlm[cls][k] & ((1u << r) - 1u));
    int pos = 0;
#pragma unroll
    for (int q = 0; q < RES; ++q) {
      const int c = cntr[cls][q];
      pos += min(c, k) + (q < r && c > k ? 1 : 0);
    }
    return cls0[cls] + pos;
  };
  if (!staged) {
    for (int i = beg + threadIdx.x; i < end; i += PLACE_NT) {
      const int j = slot(scratch[i]);
      PVal<R> pv;
      pv.load(A, i, dims);
      pv.store(A, j, dims);
    }
    return;
  }
  // every thread issues all of its loads before it uses any (few
  // workgroups per CU: their memory latency is not hidden by others)
  constexpr int PER = PLACE_SRC_MAX / PLACE_NT;
  {
    int v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = beg + threadIdx.x + k * PLACE_NT;
      if (i < end) v[k] = scratch[i];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int i = beg + threadIdx.x + k * PLACE_NT;
      if (i < end) src[slot(v[k]) - beg] = i;
    }
  }
  __syncthreads();
  // pass 3: the arrays of one element type one after the other through the
  // pool; the loads of the next array are in flight while the current one
  // is placed
  // (`arr(a)` gives array a's destination and copy; a is a compile-time
  // index after unrolling)
  auto pipeline = [&](auto arr, int count) {
    using T = typename std::remove_pointer<decltype(arr(0).first)>::type;
    constexpr int MAXA = 7;
    T* stg = (T*)pool;
    T nx[PER], w[PER];
    {
      const T* f = arr(0).second;
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int i = threadIdx.x + k * PLACE_NT;
        if (i < n) nx[k] = f[beg + i];
      }
    }
#pragma unroll
    for (int a = 0; a < MAXA; ++a) {
      if (a >= count) break;
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int i = threadIdx.x + k * PLACE_NT;
        if (i < n) stg[i] = nx[k];
      }
      __syncthreads();
      if (a + 1 < count) {
        const T* f = arr(a + 1).second;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
          const int i = threadIdx.x + k * PLACE_NT;
          if (i < n) nx[k] = f[beg + i];
        }
      }
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int j = threadIdx.x + k * PLACE_NT;
        if (j < n) w[k] = stg[src[j] - beg];
      }
      T* d = arr(a).first;
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int j = threadIdx.x + k * PLACE_NT;
        if (j < n) d[beg + j] = w[k];
      }
      __syncthreads();
    }
  };
  struct IntArr {
    int* first;
    const int* second;
  };
  struct RArr {
    R* first;
    const R* second;
  };
  pipeline(
      [&](int a) {
        return a == 0 ? IntArr{const_cast<int*>(A.cell), A.t_cell} : IntArr{const_cast<int*>(A.id), A.t_id};
      },
      A.id ? 2 : 1);
  // offsets (dims of them), momenta, then the charges when per particle
  pipeline(
      [&](int a) {
        const int d = a < 3 ? a : 2, b = a - dims < 0 ? 0 : (a - dims > 2 ? 2 : a - dims);
        if (a < dims) return RArr{const_cast<R*>(A.off[d]), A.t_off[d]};
        if (a - dims < 3) return RArr{const_cast<R*>(A.u[b]), A.t_u[b]};
        return RArr{const_cast<R*>(A.q), A.t_q};
      },
      dims + 3 + (A.q ? 1 : 0));
}

__global__ void k_fill_int(int* a, long n, int v) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    a[i] = v;
}

// The region whose banks the placement balances: the field region in single
// precision (the gather's 6 (n+1)^D four-byte reads outweigh the deposit's
// 8-byte adds), the current region in double (its double adds take twice the
// LDS cycles of the 64-bit integer adds); the two share their strides at
// even orders.
template <int DIMS, int ORDER, typename R>
static void region_strides_t(SortParams& S) {
  using G = Geo<DIMS, ORDER, R>;
  constexpr int rx = sizeof(R) == 4 ? G::ex : G::jx;
  S.rs1 = rx;
  S.rs2 = DIMS == 3 ? rx * rx : 0;
}

template <typename R>
static void region_strides(int dims, int order, SortParams& S) {
#define PIC_RS(DD, OO) \
  if (dims == DD && order == OO) return region_strides_t<DD, OO, R>(S);
  PIC_RS(2, 1) PIC_RS(2, 2) PIC_RS(2, 3) PIC_RS(2, 4)
  PIC_RS(3, 1) PIC_RS(3, 2) PIC_RS(3, 3) PIC_RS(3, 4)
#undef PIC_RS
  S.rs1 = 1;
  S.rs2 = 1;
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
  for (int d = 0; d < 3; ++d) S.hdx[d] = d < c.dims ? 0.5 * (c.sort_every - 1) * c.dt / c.dx[d] : 0.0;
  region_strides<R>(c.dims, c.order, S);
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
  int* keys = (int*)(w + L.keys);
  const int nb = S.ntiles + 1;  // + dead bin
  const int nblk = (nb + SCAN_B - 1) / SCAN_B;
  if (np == 0) {
    k_fill_int<<<dim3((S.ntiles + 2 + 255) / 256), dim3(256), 0, s>>>(starts, S.ntiles + 2, 0);
    return (int)hipGetLastError();
  }
  auto fill_grid = [](long n) { return dim3((unsigned)((n + 255) / 256 < 16384 ? (n + 255) / 256 : 16384)); };
  k_fill_int<<<fill_grid(nb), dim3(256), 0, s>>>(counts, nb, 0);
  const unsigned grid = (unsigned)((np + 255) / 256);
  DevFlags* flg = (DevFlags*)(w + L.flags);
  const long cchunk = (long)COUNT_NT * COUNT_PER;
  k_sort_count<<<dim3((unsigned)((np + cchunk - 1) / cchunk)), dim3(COUNT_NT), 0, s>>>(
      S, p->cell, np, ncell, keys, counts, flg);
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
  int* pkey = (int*)(w + L.pkey);
  k_sort_scatter<R><<<dim3(grid), dim3(256), 0, s>>>(A, S, np, ncell, keys, counts, pkey, flg);
  int* order = (int*)(w + L.order);
  k_sort_order<<<dim3(1), dim3(ORDER_NT), 0, s>>>(S, order);
  k_sort_place<R><<<dim3((unsigned)S.ntiles), dim3(PLACE_NT), 0, s>>>(A, S, starts, order, pkey, c.dims);
  // absorbed particles (the dead bin) are not copied back: the caller lowers
  // np to the live count, starts[ntiles]
  return (int)hipGetLastError();
}

int launch_sort(const pic_ctx* ctx, const pic_particles* p, void* ws, hipStream_t s) {
  return ctx->cfg.real_bytes == 8 ? launch_sort_t<double>(ctx, p, ws, s)
                                  : launch_sort_t<float>(ctx, p, ws, s);
}

}  // namespace pic
