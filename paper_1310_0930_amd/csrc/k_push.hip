// Fused gather + relativistic Boris push + move + trajectory split +
// charge-conserving (Esirkepov) deposit, tile by tile (persistent
// workgroups, one tile at a time each).
//
// This is the per-particle body of the PIC loop (Sec. 2) in the order of the
// paper's vector algorithm (Sec. 5.2, steps i-v).  The paper vectorises it
// over 4/8 SIMD lanes, emulates the field gather with serial loads and
// shuffles, and avoids write conflicts with a serial scatter of the virtual
// particles (or per-thread copies of the current grid, Sec. 3.1).  Here each
// 64-wide wavefront lane owns a particle; the workgroup stages the E and B
// samples of its tile (plus halo) in LDS once, so the gather is a set of
// LDS reads at compile-time offsets, and accumulates the current of every
// virtual segment into an LDS tile with LDS atomics (exact 64-bit fixed
// point in the single-precision form, double in the double form) before one
// coalesced flush with global atomics where tile halos overlap.
//
// Positions are an integer cell plus an offset in [0,1) normalised to the
// cell (Sec. 5.1); all shape arguments are formed from the stored offsets
// without rounding, and the shape differences of the deposit are formed in
// factored form, so that single precision keeps charge conservation at the
// level of the stored positions.
#include "k_particle.h"

namespace pic {

// ------------------------------------------------------------------ kernels
// Workgroup queue of the particles whose path crosses a stencil-switch
// plane.  A path that stays in one piece of the shape along every axis is a
// single virtual segment whose ends are the particle's old and new offsets
// in that piece's frame (nearly every particle of a thermal plasma); a
// crossing path is split into up to DIMS+1 segments (Sec. 5.2 step iv).
// About one particle in thirty crosses in a warm plasma, which puts a
// crossing in almost every 64-lane wavefront: splitting in place would run
// the split logic and the extra segments' deposit for the whole wavefront
// each time.  Instead the main loop deposits only single-segment paths, and
// crossing paths go to a queue (structure of arrays in LDS) shared by the
// workgroup's wavefronts, which is split and deposited after the tile's
// batches in whole 64-lane rounds, each lane splitting its own path (with
// per-wavefront queues a wavefront collected only about nine paths per tile
// and drained them in a mostly idle round).  Paths beyond the queue's
// capacity are split in place.  Used where the queue still fits next to the
// tile's field and current regions.
template <int DIMS, int ORDER, typename R>
struct CrossQueue {
  using G = Geo<DIMS, ORDER, R>;
  static constexpr int NW = G::NT / 64;
  static constexpr size_t room = 160 * 1024 - G::lds_bytes - 64;  // LDS left by the regions
  // full records: cell word, o0[D], o1[D], q, q v_z
  static constexpr int NV = DIMS + 2;  // the values besides o0
  static constexpr size_t full_rec = sizeof(int) + (DIMS + NV) * sizeof(R);
  // compact records (3D): cell word, particle index, o0[3]; the drain reads
  // o1 and q back from the particle arrays, where the main loop stored them
  // (the 3D current has no q v_z term)
  static constexpr size_t compact_rec = 2 * sizeof(int) + DIMS * sizeof(R);
  static constexpr int full_cap = 96 * NW;
  static constexpr bool compact = DIMS == 3 && full_cap * full_rec > room;
  static constexpr int CAP = compact ? (int)(room / compact_rec) : full_cap;
  static constexpr bool on = compact ? CAP >= 64 : full_cap * full_rec <= room;
  static constexpr int LEN = on ? CAP : 1;
  static constexpr int LENV = on && !compact ? CAP : 1;  // full records only
  static constexpr int LENI = on && compact ? CAP : 1;   // compact records only
};

// A queued path: its old cell in the current region and its cell shifts,
// packed into one word (2 bits per axis above 24 bits of cell).
__device__ __forceinline__ int pack_path(int pbase, const int* sh) {
  return pbase | ((sh[0] + 1) << 24) | ((sh[1] + 1) << 26) | ((sh[2] + 1) << 28);
}
__device__ __forceinline__ int unpack_path(int w, int* sh) {
  sh[0] = ((w >> 24) & 3) - 1;
  sh[1] = ((w >> 26) & 3) - 1;
  sh[2] = ((w >> 28) & 3) - 1;
  return w & 0xffffff;
}

// Charge-conserving current of a whole path into the LDS current tile:
// split at the stencil-switch planes, then each virtual segment on its own
// stencil.  fz = q v_z (2D: the out-of-plane current per unit time,
// already on the tile's scale).
template <int DIMS, int ORDER, typename R>
__device__ __forceinline__ void deposit_path_lds(double* s_j, int pbase, const R* jf, const R* o0,
                                                 const int* sh, const R* o1, R q, R fz) {
  Split<DIMS, R> S;
  split_path<DIMS, ORDER, R>(S, o0, sh, o1);
  LdsCurrent<DIMS, ORDER, R> sink{s_j, pbase, s_j};
  for (int sg = 0; sg <= S.m; ++sg) {
    R xa[3], xb[3], ft;
    int base[3];
    segment_ends<DIMS, ORDER, R>(S, sg, xa, xb, base, ft);
    sink.segment(base);
    deposit_segment<DIMS, ORDER, R>(sink, jf, xa, xb, q, fz * ft);
  }
}

// Tiles for persistent workgroups.  Tiles are split into 8 contiguous
// ranges, one per XCD: a workgroup takes tiles from its own XCD's range
// first (neighbouring tiles share halo samples in that XCD's L2; dispatch
// places workgroup b on XCD b mod 8) and then from the other ranges in
// turn; `xk` counts the ranges it has found used up.  A claim is one atomic
// increment of a range counter, issued early so that its latency overlaps
// other work, and resolved later (one thread does both).
__device__ inline unsigned claim_issue(DevFlags* flg, int xk) {
  return xk < 8 ? atomicAdd(&flg->tile_next[(blockIdx.x + xk) & 7], 1u) : 0u;
}

// Resolves a claim to a non-empty tile (claiming again past empty tiles and
// used-up ranges); returns -1 once every range is used up.
__device__ inline int claim_resolve(unsigned local, const int* __restrict__ starts, DevFlags* flg,
                                    int per_xcd, int ntiles, int& xk, int& beg, int& end) {
  while (xk < 8) {
    const int t = (int)((blockIdx.x + xk) & 7) * per_xcd + (int)local;
    if (local >= (unsigned)per_xcd || t >= ntiles) {
      ++xk;
    } else {
      beg = starts[t];
      end = starts[t + 1];
      if (beg != end) return t;
    }
    local = claim_issue(flg, xk);
  }
  return -1;
}

// Claims of the re-binned pass: one counter over the destination tiles
// listed by the sorted pass (each holds at least one particle).
__device__ inline unsigned rb_claim_issue(DevFlags* flg) { return atomicAdd(&flg->rb_next, 1u); }
__device__ inline int rb_claim_resolve(unsigned v, const DevFlags* flg, const Rebin& rb, int& beg,
                                       int& end) {
  if (v >= flg->rb_m) return -1;
  const int t = rb.nl[v];
  beg = rb.base[v];
  end = beg + rb.cnt[t];
  return t;
}

// Tile of a cell (the sort's tile numbering).
template <int DIMS, int ORDER, typename R>
__device__ __forceinline__ int cell_tile(const KParams<R>& P, const int* c3) {
  using G = Geo<DIMS, ORDER, R>;
  const int tz = DIMS == 3 ? c3[2] / G::TZ : 0;
  return c3[0] / G::T + P.ntile[0] * (c3[1] / G::T + P.ntile[1] * tz);
}

// The low 48 bits of a fixed-point tile sum, sign-extended (the sum itself).
__device__ __forceinline__ long long sext48(long long x) {
  return (long long)((unsigned long long)x << 16) >> 16;
}

// First particle of batch b for this lane.
__device__ __forceinline__ int pbase_of_batch(int pbeg, int b, int lane) { return pbeg + 64 * b + lane; }

// Next batch of 64 particles of the current tile for this wavefront.
__device__ __forceinline__ int take_batch(int* ctr) {
  int b = 0;
  if ((threadIdx.x & 63) == 0) b = atomicAdd(ctr, 1);
  return __builtin_amdgcn_readfirstlane(b);
}

// Tile kernel: persistent workgroups, each taking tiles until none is left;
// particles within the drift allowance of the tile run out of LDS.  The
// sorted pass (RB = false) takes the tiles of the last sort; a particle that
// has drifted beyond its tile's allowance (or moves half a cell or more in
// one step, or carries a charge above the sort's bound) is left untouched
// and appended to the deferred list.  The re-binned pass (RB = true) takes
// the deferred particles grouped by the tile of their current cell
// (k_rebin_count, k_rebin_scatter), so that those that drifted run out of
// LDS too; what it cannot take either is left untouched for
// k_push_deferred.  The tiles of one workgroup are software-pipelined: a
// wavefront that has finished its particles issues the loads of the next
// tile's fields (into registers) while the other wavefronts finish, and
// the flush of the current tile's current runs while they are in flight.
template <int DIMS, int ORDER, typename R, bool RB>
__global__ void __launch_bounds__((Geo<DIMS, ORDER, R>::NT)) k_push_tile(
    KParams<R> P, DParts<R> pa, DFields<R> F, const int* __restrict__ starts,
    int* __restrict__ deferred, DevFlags* flg, Rebin rb) {
  using G = Geo<DIMS, ORDER, R>;
  using Q = CrossQueue<DIMS, ORDER, R>;
  __shared__ R s_eb[6 * G::e_vol];
  __shared__ double s_j[3 * G::j_vol];
  __shared__ int q_path[Q::LEN];
  __shared__ R q_o0[DIMS][Q::LEN];  // the path's old offsets
  __shared__ R q_val[Q::NV][Q::LENV];  // full records: o1, q, q v_z
  __shared__ int q_idx[Q::LENI];    // compact records: the particle
  // Tile ids two deep: while tile i runs, slot (i+1)&1 holds tile i+1
  // (tile id, first and end particle) and thread 0 resolves tile i+2 into
  // slot i&1, which nobody reads until the next tile.
  __shared__ int s_q[2][3];
  __shared__ int s_batch;  // next batch of the current tile
  __shared__ int s_qn;     // paths in the crossing queue

  const int open0 = P.bc[0] == PIC_BC_OPEN, open1 = P.bc[1] == PIC_BC_OPEN;
  const int open2 = DIMS == 3 && P.bc[2] == PIC_BC_OPEN;
  const int str1 = P.n[0], str2 = P.n[0] * P.n[1];
  int xk = 0;           // thread 0: ranges used up
  unsigned claim = 0u;  // thread 0: claim in flight
  auto issue = [&]() -> unsigned {
    if constexpr (RB)
      return rb_claim_issue(flg);
    else
      return claim_issue(flg, xk);
  };
  auto resolve = [&](unsigned c, int& b, int& e) -> int {
    if constexpr (RB)
      return rb_claim_resolve(c, flg, rb, b, e);
    else
      return claim_resolve(c, starts, flg, P.per_xcd, P.ntiles, xk, b, e);
  };
  if (threadIdx.x == 0) {
    int b = 0, e = 0;
    const int t0 = resolve(issue(), b, e);
    s_q[0][0] = t0;
    s_q[0][1] = b;
    s_q[0][2] = e;
    const int t1 = t0 < 0 ? -1 : resolve(issue(), b, e);
    s_q[1][0] = t1;
    s_q[1][1] = b;
    s_q[1][2] = e;
  }
  __syncthreads();
  int tile = __builtin_amdgcn_readfirstlane(s_q[0][0]);
  if (tile < 0) return;
  int pbeg = __builtin_amdgcn_readfirstlane(s_q[0][1]);
  int pend = __builtin_amdgcn_readfirstlane(s_q[0][2]);
  constexpr int NR = (G::e_vol + G::NT - 1) / G::NT;
  R stage[NR][6];
  int org[3];
  tile_origin<DIMS, ORDER, R>(P, tile, org);
  stage_load<DIMS, ORDER, R, NR>(P, F, org, stage);
  for (int idx = threadIdx.x; idx < 3 * G::j_vol; idx += G::NT) s_j[idx] = 0.0;

  // the staged fields of the next tile from registers into LDS
  auto write_eb = [&]() {
    const int tid = opaque_tid();
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int r = tid + k * G::NT;
      if (r < G::e_vol) {
#pragma unroll
        for (int c = 0; c < 6; ++c) s_eb[c * G::e_vol + r] = stage[k][c];
      }
    }
  };
  // Where there is a crossing queue, the next tile's fields go to LDS right
  // after the barrier that ends the batches, which frees their registers for
  // the drain (held through it, they spilled in the double forms' batch
  // loop; single precision gains 1 %).
  constexpr bool early_eb = Q::on;
  if constexpr (early_eb) write_eb();  // (the first tile's; the loop writes the next ones at its end)
  for (int it = 0;; ++it) {
    if constexpr (!early_eb) write_eb();
    const int nslot = (it + 1) & 1;
    const int next = __builtin_amdgcn_readfirstlane(s_q[nslot][0]);
    const int nbeg = __builtin_amdgcn_readfirstlane(s_q[nslot][1]);
    const int nend = __builtin_amdgcn_readfirstlane(s_q[nslot][2]);
    if (threadIdx.x == 0) {
      s_batch = 0;
      s_qn = 0;
      if (next >= 0) claim = issue();  // for tile i+2
    }

    // Scales of the fixed-point current tile (single form).  A contribution
    // to J_c is q jfac_c P A with |P| <= |move along c| < 1/2 and 0 <= A <= 1
    // (P is a difference of the cumulative shape, A an average of products
    // of weights), so |contribution| < qmax |jfac_c| / 2; in 2D J_z is
    // q v_z f A with |v_z| < 1, f <= 1, so qmax bounds it.  A tile sample
    // receives at most (DIMS+1) contributions per particle of the tile
    // (2^g bounds their number).  The power-of-two scale 2^K keeps every
    // sum below 2^47 and so every scaled contribution below 2^(47-g):
    // contributions round to integers at 2^-(48-g) of the bound (about
    // 2^-34 for the 3D 8^3 tiles at 8 particles per cell, far below single
    // precision) and the 48-bit tile sums are exact.  A particle whose |q|
    // exceeds the bound the sort recorded (charges changed since) takes the
    // global-memory path.
    R jf[3] = {P.jfac[0], P.jfac[1], P.jfac[2]};
    R zs = R(1);
    int Ks[3] = {0, 0, 0};
    const float qmax = pa.q ? __uint_as_float(flg->qmax) : fabsf((float)P.q_const);
    const bool qmax_ok = qmax <= 3.0e38f;
    if constexpr (G::fixed) {
      const unsigned ncontrib = (unsigned)(DIMS + 1) * (unsigned)(pend - pbeg);
      const int g = 32 - __clz((int)(ncontrib - 1u));  // ncontrib <= 2^g
      const int top = 47 - g;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const bool z2 = DIMS == 2 && c == 2;
        int e = 0;
        frexpf(z2 ? qmax : qmax * fabsf((float)P.jfac[c]) * 0.5f, &e);  // bound < 2^e
        // uniform over the workgroup: keep the scales in scalar registers
        Ks[c] = __builtin_amdgcn_readfirstlane(qmax_ok ? top - e : 0);
        const float sc = ldexpf(z2 ? 1.0f : (float)P.jfac[c], Ks[c]);
        const float su = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(sc)));
        if (z2)
          zs = su;
        else
          jf[c] = su;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // tile i+2 (wavefront 0 starts its particles later)
      int t2 = -1, b = 0, e = 0;
      if (next >= 0) t2 = resolve(claim, b, e);
      s_q[it & 1][0] = t2;
      s_q[it & 1][1] = b;
      s_q[it & 1][2] = e;
    }
    const int lane = threadIdx.x & 63;
    // The crossing queue, whole 64-path rounds dealt round-robin to the
    // wavefronts; every lane splits its path and deposits all of its
    // segments.  It is drained after the barrier that ends the tile's
    // batches, once the next tile's fields (loaded meanwhile) are in LDS.
    auto drain = [&](int total) {
      for (int r0 = (threadIdx.x >> 6) * 64; r0 < total; r0 += G::NT) {
        const int r = r0 + lane;
        if (r < total) {
          int shq[3];
          const int pb = unpack_path(q_path[r], shq);
          R a0[3] = {R(0), R(0), R(0)}, a1[3] = {R(0), R(0), R(0)};
#pragma unroll
          for (int d = 0; d < DIMS; ++d) a0[d] = q_o0[d][r];
          if constexpr (Q::compact) {
            const int pp = q_idx[r];
#pragma unroll
            for (int d = 0; d < 3; ++d) a1[d] = pa.off[d][pp];
            deposit_path_lds<DIMS, ORDER, R>(s_j, pb, jf, a0, shq, a1,
                                             pa.q ? pa.q[pp] : P.q_const, R(0));
          } else {
#pragma unroll
            for (int d = 0; d < DIMS; ++d) a1[d] = q_val[d][r];
            deposit_path_lds<DIMS, ORDER, R>(s_j, pb, jf, a0, shq, a1, q_val[DIMS][r],
                                             q_val[DIMS + 1][r]);
          }
        }
      }
    };
    // Wavefronts take batches of 64 consecutive particles from a counter in
    // LDS, so that the wavefronts the SIMD arbiter serves first take more
    // and all finish together.  The loop is uniform per wavefront (lanes
    // past the end are idle) so that the queue's ballot sees every lane.
    // The next batch is taken, and its particle state loaded, one iteration
    // ahead.
    // (p: position in the tile's range; pi: the particle, through the list
    // in the re-binned pass)
    int p = pbase_of_batch(pbeg, take_batch(&s_batch), lane), pn;
    int qn = RB ? (p < pend ? rb.list[p] : 0) : p;
    PState<R> nxt;
    if (p < pend) nxt = load_particle<DIMS, R>(pa, qn, P.q_const);
    for (; p - lane < pend; p = pn) {
      const int pi = qn;
      PState<R> s = nxt;
      pn = pbase_of_batch(pbeg, take_batch(&s_batch), lane);
      qn = RB ? (pn < pend ? rb.list[pn] : 0) : pn;
      if (pn < pend) nxt = load_particle<DIMS, R>(pa, qn, P.q_const);
      bool valid = p < pend && s.cl >= 0;
      int c3[3] = {0, 0, 0};
      if (valid) valid = decode<DIMS, R>(P, s, c3, flg);
      // position relative to the tile origin (periodic image inside the window)
      int l[3] = {0, 0, 0};
      bool fast = true;
#pragma unroll
      for (int d = 0; d < DIMS; ++d) {
        const int Td = d == 2 ? G::TZ : G::T;
        const int Ad = d == 2 ? G::AZ : G::A;
        int v = c3[d] - org[d];
        if (P.bc[d] == PIC_BC_PERIODIC) {
          v = v < 0 ? v + P.n[d] : v;
          if (v >= Td + Ad) v -= P.n[d];
        }
        l[d] = v;
        fast = fast && v >= -Ad && v < Td + Ad;
      }
      R o1[3] = {R(0), R(0), R(0)}, vz = R(0);
      int sh[3] = {0, 0, 0};
      if (G::fixed && pa.q && !(fabs(s.q) <= qmax && qmax_ok)) fast = false;
      if (valid && !fast) {  // leave the state as it was; a later pass redoes it
        if constexpr (RB)
          rb.defer2[atomicAdd(&flg->ndefer2, 1u)] = pi;
        else
          deferred[atomicAdd(&flg->ndefer, 1u)] = pi;
        valid = false;
      }
      if (valid) {
        LdsFields<DIMS, ORDER, R> acc{
            (lds_ptr<const R>)s_eb, ((l[2] - G::e_lo_z) * G::ex + (l[1] - G::e_lo)) * G::ex + (l[0] - G::e_lo)};
        R Ep[3], Bp[3];
        gather<DIMS, ORDER, R>(acc, s.o, Ep, Bp);
        bool small = false;
        if (!push_move<DIMS, R>(P, s, Ep, Bp, sh, o1, vz, small, flg)) {
          pa.cell[pi] = -1;
          valid = false;
        } else if (!small) {
          if constexpr (RB)
            rb.defer2[atomicAdd(&flg->ndefer2, 1u)] = pi;
          else
            deferred[atomicAdd(&flg->ndefer, 1u)] = pi;
          valid = false;
        }
      }
      const int pbase = ((l[2] - G::j_lo_z) * G::jx + (l[1] - G::j_lo)) * G::jx + (l[0] - G::j_lo);
      // A path that stays in the same piece of the shape along every axis is
      // one virtual segment from the old to the new offset in that piece's
      // frame, on the stencil of the old cell's piece.
      R xa[3] = {R(0), R(0), R(0)}, xb[3] = {R(0), R(0), R(0)};
      int base[3] = {0, 0, 0};
      bool single = valid;
#pragma unroll
      for (int d = 0; d < DIMS; ++d) {
        const int k0 = piece_node<ORDER>(s.o[d], xa[d]);
        const int k1 = sh[d] + piece_node<ORDER>(o1[d], xb[d]);
        single = single && k0 == k1;
        base[d] = k0 - ORDER / 2;
      }
      const bool cross = valid && !single;
      const R fz = s.q * vz * zs;
      if (single) {
        LdsCurrent<DIMS, ORDER, R> sink{s_j, pbase, s_j};
        sink.segment(base);
        deposit_segment<DIMS, ORDER, R>(sink, jf, xa, xb, s.q, fz);
      }
      if (valid) store_particle<DIMS, R>(pa, pi, s, o1, new_cell<DIMS, R>(P, c3, sh));
      // paths that cross a stencil-switch plane
      const unsigned long long cm = __ballot(cross);
      if (cm == 0ull) continue;
      if constexpr (Q::on) {
        int q0 = 0;
        if (lane == 0) q0 = atomicAdd(&s_qn, (int)__popcll(cm));
        const int pos = __builtin_amdgcn_readfirstlane(q0) + (int)__popcll(cm & ((1ull << lane) - 1ull));
        if (cross && pos < Q::LEN) {
          q_path[pos] = pack_path(pbase, sh);
#pragma unroll
          for (int d = 0; d < DIMS; ++d) q_o0[d][pos] = s.o[d];
          if constexpr (Q::compact) {
            q_idx[pos] = pi;
          } else {
#pragma unroll
            for (int d = 0; d < DIMS; ++d) q_val[d][pos] = o1[d];
            q_val[DIMS][pos] = s.q;
            q_val[DIMS + 1][pos] = fz;
          }
        } else if (cross) {  // queue full: split in place
          deposit_path_lds<DIMS, ORDER, R>(s_j, pbase, jf, s.o, sh, o1, s.q, fz);
        }
      } else {  // no room for a queue: split in place
        if (cross) deposit_path_lds<DIMS, ORDER, R>(s_j, pbase, jf, s.o, sh, o1, s.q, fz);
      }
    }
    // (the opaque copy keeps the compiler from forming the next tile's
    // addresses before the particle loop, where registers are scarce)
    int nt = next;
    asm volatile("" : "+s"(nt));
    if (nt >= 0) {  // the next tile's fields, in flight during the flush
      int norg[3];
      tile_origin<DIMS, ORDER, R>(P, nt, norg);
      stage_load<DIMS, ORDER, R, NR>(P, F, norg, stage);
    } else {  // (defining stage on both paths ends the current values' life here)
#pragma unroll
      for (int k = 0; k < NR; ++k)
#pragma unroll
        for (int c = 0; c < 6; ++c) stage[k][c] = R(0);
    }
    __syncthreads();
    if constexpr (early_eb) {
      // (the next tile reads s_eb after the barrier at the top of the loop;
      // the flush needs one more barrier only after a drain)
      write_eb();
      const int total = min(s_qn, Q::LEN);
      if (total > 0) {
        drain(total);
        __syncthreads();
      }
    }

    // flush the LDS current tile (its halo overlaps the neighbouring
    // tiles') and clear it for the next tile
    const int jbx = org[0] + G::j_lo, jby = org[1] + G::j_lo, jbz = org[2] + G::j_lo_z;
    if (axis_inside(jbx, G::jx, P.n[0], open0) && axis_inside(jby, G::jx, P.n[1], open1) &&
        (DIMS == 2 || axis_inside(jbz, G::jz, P.n[2], open2))) {
      const int base = (DIMS == 3 ? jbz * str2 : 0) + jby * str1 + jbx;
      for (int r = opaque_tid(); r < G::j_vol; r += G::NT) {
        const int lx = r % G::jx, ly = (r / G::jx) % G::jx, lz = r / (G::jx * G::jx);
        const int o = base + (DIMS == 3 ? lz * str2 : 0) + ly * str1 + lx;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          R v;
          if constexpr (G::fixed)
            v = (R)ldexp((double)sext48(((const long long*)s_j)[c * G::j_vol + r]), -Ks[c]);
          else
            v = (R)s_j[c * G::j_vol + r];
          s_j[c * G::j_vol + r] = 0.0;
          if (v != R(0)) atomic_add(&F.J[c][o], v);
        }
      }
    } else {
      for (int r = opaque_tid(); r < G::j_vol; r += G::NT) {
        const int lx = r % G::jx, ly = (r / G::jx) % G::jx, lz = r / (G::jx * G::jx);
        int sx[2], sy[2], sz[2] = {0, 0};
        axis_slots(org[0] + G::j_lo + lx, P.n[0], open0, 1, sx);
        axis_slots(org[1] + G::j_lo + ly, P.n[1], open1, str1, sy);
        if (DIMS == 3) axis_slots(org[2] + G::j_lo_z + lz, P.n[2], open2, str2, sz);
#pragma unroll
        for (int c = 0; c < 3; ++c) {  // J_c staggered along c
          R v;
          if constexpr (G::fixed)
            v = (R)ldexp((double)sext48(((const long long*)s_j)[c * G::j_vol + r]), -Ks[c]);
          else
            v = (R)s_j[c * G::j_vol + r];
          s_j[c * G::j_vol + r] = 0.0;
          const int ix = sx[c == 0], iy = sy[c == 1], iz = sz[c == 2];
          if (v != R(0) && ix >= 0 && iy >= 0 && iz >= 0) atomic_add(&F.J[c][ix + iy + iz], v);
        }
      }
    }
    if (next < 0) break;
    tile = next;
    pbeg = nbeg;
    pend = nend;
    tile_origin<DIMS, ORDER, R>(P, tile, org);
  }
}

// Tile of the current cell of deferred particle i (the decomposition of
// decode()).
template <int DIMS, int ORDER, typename R>
__device__ __forceinline__ int deferred_tile(const KParams<R>& P, const int* __restrict__ cell,
                                             const int* __restrict__ deferred, int i) {
  const uint32_t cl = (uint32_t)cell[deferred[i]];
  const uint32_t rest = P.dn0.div(cl);
  int c3[3] = {(int)cl - (int)rest * P.n[0], (int)rest, 0};
  if (DIMS == 3) {
    const uint32_t r2 = P.dn1.div(rest);
    c3[1] = (int)(rest - r2 * P.n[1]);
    c3[2] = (int)r2;
  }
  return cell_tile<DIMS, ORDER, R>(P, c3);
}

// Counts the deferred particles of the sorted pass per destination tile
// (the tile of their current cell), giving each its rank there and listing
// the destination tiles in order of their first particle; the last
// workgroup to finish turns the counts into first list positions
// (exclusive prefix sum in the order of rb.nl).  Consecutive entries of the
// list mostly come from one tile and go to one, so the lanes of a
// wavefront that share a destination take their ranks with one atomic.
// Every thread fences its own writes before its workgroup counts itself as
// finished.
constexpr int RB_NT = 256;
template <int DIMS, int ORDER, typename R>
__global__ void __launch_bounds__(RB_NT) k_rebin_count(KParams<R> P, const int* __restrict__ cell,
                                                       const int* __restrict__ deferred, Rebin rb,
                                                       DevFlags* flg) {
  __shared__ int sc[2 * RB_NT];
  __shared__ int s_last;
  const int nd = (int)flg->ndefer;
  if (nd == 0) return;  // (nothing to re-bin: the re-binned pass finds no tile)
  const int lane = threadIdx.x & 63;
  for (int i0 = blockIdx.x * RB_NT + (threadIdx.x & ~63); i0 < nd; i0 += gridDim.x * RB_NT) {
    const int i = i0 + lane;
    const bool act = i < nd;
    const int t = act ? deferred_tile<DIMS, ORDER, R>(P, cell, deferred, i) : -1;
    unsigned long long todo = __ballot(act);
    while (todo) {
      const int l0 = __ffsll((long long)todo) - 1;
      const int t0 = __shfl(t, l0, 64);
      const unsigned long long same = __ballot(act && t == t0);
      int r0 = 0;
      if (lane == l0) {
        r0 = atomicAdd(&rb.cnt[t0], (int)__popcll(same));
        if (r0 == 0) {
          const unsigned v = atomicAdd(&flg->rb_m, 1u);
          rb.nl[v] = t0;
          rb.tv[t0] = (int)v;
        }
      }
      r0 = __shfl(r0, l0, 64);
      if (act && t == t0) rb.rank[i] = r0 + (int)__popcll(same & ((1ull << lane) - 1ull));
      todo &= ~same;
    }
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicAdd(&flg->rb_done, 1u) == gridDim.x - 1 ? 1 : 0;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  const int m = (int)__hip_atomic_load(&flg->rb_m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int tid = threadIdx.x;
  int run = 0;
  for (int c0 = 0; c0 < m; c0 += RB_NT) {
    const int v = c0 + tid;
    int n = 0;
    if (v < m) {
      const int t = __hip_atomic_load(&rb.nl[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      n = __hip_atomic_load(&rb.cnt[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    sc[tid] = n;
    __syncthreads();
    int pin = 0;
    for (int o = 1; o < RB_NT; o <<= 1) {
      int x = sc[pin * RB_NT + tid];
      if (tid >= o) x += sc[pin * RB_NT + tid - o];
      sc[(1 - pin) * RB_NT + tid] = x;
      pin ^= 1;
      __syncthreads();
    }
    if (v < m) rb.base[v] = run + sc[pin * RB_NT + tid] - n;
    run += sc[pin * RB_NT + RB_NT - 1];
    __syncthreads();
  }
}

// Groups the deferred particles of the sorted pass by destination tile: each
// goes to its tile's first list position plus its rank there.
template <int DIMS, int ORDER, typename R>
__global__ void __launch_bounds__(256) k_rebin_scatter(KParams<R> P, const int* __restrict__ cell,
                                                       const int* __restrict__ deferred, Rebin rb,
                                                       DevFlags* flg) {
  const int nd = (int)flg->ndefer;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += gridDim.x * blockDim.x) {
    const int t = deferred_tile<DIMS, ORDER, R>(P, cell, deferred, i);
    rb.list[rb.base[rb.tv[t]] + rb.rank[i]] = deferred[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && nd > 0) atomicAdd(&flg->rebinned, (unsigned long long)nd);
}

// Global-memory kernel for the deferred particles: the same gather, push,
// move and deposit with fields read from and currents added to global
// memory.  The list length is read on the device.
template <int DIMS, int ORDER, typename R>
__global__ void __launch_bounds__(256) k_push_deferred(KParams<R> P, DParts<R> pa, DFields<R> F,
                                                       const int* __restrict__ deferred,
                                                       const unsigned* __restrict__ count,
                                                       DevFlags* flg) {
  const int nd = (int)*count;
  const int open0 = P.bc[0] == PIC_BC_OPEN, open1 = P.bc[1] == PIC_BC_OPEN;
  const int open2 = DIMS == 3 && P.bc[2] == PIC_BC_OPEN;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nd; t += gridDim.x * blockDim.x) {
    const int p = deferred[t];
    PState<R> s = load_particle<DIMS, R>(pa, p, P.q_const);
    int c3[3];
    if (!decode<DIMS, R>(P, s, c3, flg)) continue;
    GlobalFields<R> acc{F.E, F.B, c3[0], c3[1], c3[2], P.n[0], P.n[1], P.n[2],
                        open0, open1, open2, DIMS};
    R Ep[3], Bp[3], o1[3], vz = R(0);
    int sh[3];
    bool small;
    gather<DIMS, ORDER, R>(acc, s.o, Ep, Bp);
    if (!push_move<DIMS, R>(P, s, Ep, Bp, sh, o1, vz, small, flg)) {
      pa.cell[p] = -1;
      continue;
    }
    GlobalCurrent<R> sink{F.J, c3[0], c3[1], c3[2], P.n[0], P.n[1], P.n[2],
                          open0, open1, open2, DIMS, 0, 0, 0};
    deposit<DIMS, ORDER, R>(sink, P.jfac, s.o, sh, o1, s.q, vz);
    store_particle<DIMS, R>(pa, p, s, o1, new_cell<DIMS, R>(P, c3, sh));
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && nd > 0) atomicAdd(&flg->slowpath, (unsigned long long)nd);
}

// Zero J (n = 0: keep it, another species adds its current), the
// deferred-list lengths, the tile counters and the re-binned pass's counts
// before a push.
template <typename R>
__global__ void k_push_prologue(R* a, R* b, R* c, long n, DevFlags* flg, int* rb_cnt, int ntiles) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    flg->since_sort += flg->ndefer;
    flg->ndefer = 0u;
    flg->ndefer2 = 0u;
    flg->rb_m = 0u;
    flg->rb_next = 0u;
    flg->rb_done = 0u;
  }
  if (blockIdx.x == 0 && threadIdx.x < 8) flg->tile_next[threadIdx.x] = 0u;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ntiles; i += gridDim.x * blockDim.x)
    rb_cnt[i] = 0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    a[i] = R(0);
    b[i] = R(0);
    c[i] = R(0);
  }
}

static int device_cus() {
  static int cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cache[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cache[dev] = n;
  }
  return cache[dev];
}

// Workgroups of the persistent tile kernel: as many as are resident at once
// (compute units x workgroups per unit), at most 8 x the XCD range length.
template <int DIMS, int ORDER, typename R, bool RB>
static unsigned tile_grid(const KParams<R>& P) {
  using G = Geo<DIMS, ORDER, R>;
  static int occ = 0;
  if (occ == 0) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_push_tile<DIMS, ORDER, R, RB>, G::NT, 0) !=
            hipSuccess ||
        b < 1)
      b = 1;
    occ = b;
  }
  const long want = 8L * P.per_xcd, have = (long)device_cus() * occ;
  return (unsigned)(want < have ? want : have);
}

template <int DIMS, int ORDER, typename R>
static int launch_pd(const pic_ctx* ctx, const pic_particles* p, const pic_fields* f, void* ws,
                     hipStream_t s, bool accumulate) {
  using G = Geo<DIMS, ORDER, R>;
  KParams<R> P = make_params<R>(ctx);
  WsLayout L = ws_layout(ctx, p->np);
  char* w = (char*)ws;
  DParts<R> pa;
  pa.cell = p->cell;
  for (int d = 0; d < 3; ++d) {
    pa.off[d] = (R*)p->off[d];
    pa.u[d] = (R*)p->u[d];
  }
  pa.q = (R*)p->q;
  pa.id = p->id;
  DFields<R> F;
  for (int c = 0; c < 3; ++c) {
    F.E[c] = (R*)f->E[c];
    F.B[c] = (R*)f->B[c];
    F.J[c] = (R*)f->J[c];
  }
  DevFlags* flg = (DevFlags*)(w + L.flags);
  // the sort's scratch is free during a push: deferred list, re-binning
  int* deferred = (int*)(w + L.tmp_cell);
  Rebin rb;
  rb.cnt = (int*)(w + L.counts);
  rb.tv = (int*)(w + L.rb_tv);
  rb.nl = (int*)(w + L.rb_nl);
  rb.base = (int*)(w + L.bstart);
  rb.rank = (int*)(w + L.keys);
  rb.list = (int*)(w + L.tmp_id);
  rb.defer2 = (int*)(w + L.tmp_real);
  const long ncell = accumulate ? 0L : (long)P.n[0] * P.n[1] * P.n[2];
  const long nz = ncell > P.ntiles ? ncell : (long)P.ntiles;
  const long fb = (nz + 255) / 256;
  k_push_prologue<R><<<dim3((unsigned)(fb < 1 ? 1 : fb < 4096 ? fb : 4096)), dim3(256), 0, s>>>(
      F.J[0], F.J[1], F.J[2], ncell, flg, rb.cnt, P.ntiles);
  k_push_tile<DIMS, ORDER, R, false><<<dim3(tile_grid<DIMS, ORDER, R, false>(P)), dim3(G::NT), 0, s>>>(
      P, pa, F, (const int*)(w + L.starts), deferred, flg, rb);
  if (ctx->rebin) {
    k_rebin_count<DIMS, ORDER, R><<<dim3(256), dim3(RB_NT), 0, s>>>(P, pa.cell, deferred, rb, flg);
    k_rebin_scatter<DIMS, ORDER, R><<<dim3(512), dim3(256), 0, s>>>(P, pa.cell, deferred, rb, flg);
    k_push_tile<DIMS, ORDER, R, true><<<dim3(tile_grid<DIMS, ORDER, R, true>(P)), dim3(G::NT), 0, s>>>(
        P, pa, F, (const int*)(w + L.starts), deferred, flg, rb);
    k_push_deferred<DIMS, ORDER, R><<<dim3(1024), dim3(256), 0, s>>>(P, pa, F, rb.defer2, &flg->ndefer2,
                                                                      flg);
  } else {
    k_push_deferred<DIMS, ORDER, R><<<dim3(1024), dim3(256), 0, s>>>(P, pa, F, deferred, &flg->ndefer,
                                                                      flg);
  }
  return (int)hipGetLastError();
}

int launch_push_deposit(const pic_ctx* ctx, const pic_particles* p, const pic_fields* f, void* ws,
                        hipStream_t s, bool accumulate) {
  const int D = ctx->cfg.dims, O = ctx->cfg.order;
  const bool dbl = ctx->cfg.real_bytes == 8;
#define PIC_PD(DD, OO)                                                            \
  if (D == DD && O == OO)                                                         \
    return dbl ? launch_pd<DD, OO, double>(ctx, p, f, ws, s, accumulate)         \
               : launch_pd<DD, OO, float>(ctx, p, f, ws, s, accumulate);
  PIC_PD(2, 1) PIC_PD(2, 2) PIC_PD(2, 3) PIC_PD(2, 4)
  PIC_PD(3, 1) PIC_PD(3, 2) PIC_PD(3, 3) PIC_PD(3, 4)
#undef PIC_PD
  return (int)hipErrorInvalidValue;
}

}  // namespace pic
