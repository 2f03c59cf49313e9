// FP64 diagnostics, kept off the timed loop: charge density from the stored
// cells and offsets, Gauss's-law and continuity residuals, field and kinetic
// energies.
//
// Charge conservation is the property the paper's deposit is chosen for
// (Sec. 5.2: a charge-conserving method for the virtual trajectories); these
// residuals measure it in double precision against the positions the push
// actually stored, whatever precision the push ran in.
#include "k_common.h"

namespace pic {

struct DiagParams {
  int n[3];
  int open[3];
  int dims, order, margin;
  double dx[3], dt, dV;
  FastDiv dn0, dn1;
  int ncell;
};

// Node-centred B-spline weights in double (same polynomials as the push).
template <int ORDER>
__device__ __forceinline__ int node_weights(double o, double* w) {
  double xi;
  int k;
  if (ORDER & 1) {
    k = 0;
    xi = o;
  } else {
    k = o >= 0.5;
    xi = k ? o - 1.0 : o;
  }
  if (ORDER == 1) {
    w[0] = 1.0 - xi;
    w[1] = xi;
  } else if (ORDER == 2) {
    const double a = 0.5 - xi, b = 0.5 + xi;
    w[0] = 0.5 * a * a;
    w[1] = 0.75 - xi * xi;
    w[2] = 0.5 * b * b;
  } else if (ORDER == 3) {
    const double s = 1.0 - xi, t2 = xi * xi, t3 = t2 * xi;
    w[0] = s * s * s / 6.0;
    w[1] = (4.0 - 6.0 * t2 + 3.0 * t3) / 6.0;
    w[2] = (1.0 + 3.0 * xi + 3.0 * t2 - 3.0 * t3) / 6.0;
    w[3] = t3 / 6.0;
  } else {
    const double a = 1.0 - 2.0 * xi, b = 1.0 + 2.0 * xi, t2 = xi * xi;
    w[0] = a * a * a * a / 384.0;
    w[1] = (19.0 + xi * (-44.0 + xi * (24.0 + xi * (16.0 - 16.0 * xi)))) / 96.0;
    w[2] = (115.0 + t2 * (-120.0 + 48.0 * t2)) / 192.0;
    w[3] = (19.0 + xi * (44.0 + xi * (24.0 + xi * (-16.0 - 16.0 * xi)))) / 96.0;
    w[4] = b * b * b * b / 384.0;
  }
  return k - ORDER / 2;
}

template <int DIMS, int ORDER, typename R>
__global__ void k_deposit_rho(DiagParams P, const int* __restrict__ cell, const R* o0, const R* o1,
                              const R* o2, const R* q, double qc, long np, double* __restrict__ rho) {
  const long p = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int cl = cell[p];
  if (cl < 0 || cl >= P.ncell) return;
  const R* off[3] = {o0, o1, o2};
  const double qp = q ? (double)q[p] : qc;
  const uint32_t rest = P.dn0.div((uint32_t)cl);
  int c3[3];
  c3[0] = cl - (int)rest * P.n[0];
  c3[1] = DIMS == 3 ? (int)(rest - P.dn1.div(rest) * P.n[1]) : (int)rest;
  c3[2] = DIMS == 3 ? (int)P.dn1.div(rest) : 0;
  constexpr int M = ORDER + 1;
  double w[3][M];
  int b[3] = {0, 0, 0};
  for (int d = 0; d < DIMS; ++d) {
    const double o = (double)off[d][p];
    if (!(o >= 0.0 && o < 1.0)) return;
    b[d] = node_weights<ORDER>(o, w[d]);
  }
  constexpr int MZ = DIMS == 3 ? M : 1;
  for (int k = 0; k < MZ; ++k) {
    const int iz = DIMS == 3 ? axis_slot(c3[2] + b[2] + k, P.n[2], P.open[2], 0) : 0;
    if (iz < 0) continue;
    const double wz = DIMS == 3 ? w[2][k] : 1.0;
    for (int j = 0; j < M; ++j) {
      const int iy = axis_slot(c3[1] + b[1] + j, P.n[1], P.open[1], 0);
      if (iy < 0) continue;
      for (int i = 0; i < M; ++i) {
        const int ix = axis_slot(c3[0] + b[0] + i, P.n[0], P.open[0], 0);
        if (ix < 0) continue;
        atomicAdd(&rho[ix + P.n[0] * (iy + P.n[1] * iz)], qp * w[0][i] * w[1][j] * wz);
      }
    }
  }
}

// The same charge density for particles binned by the last sort, one
// workgroup per tile: the tile's charges are summed in an LDS region (the
// tile, the push's drift allowance around it and the stencil reach) with
// double-precision LDS atomics and added to rho once per region node, so
// the global atomics fall from (n+1)^D per particle to one per region node.
// Particles that drifted beyond the allowance add to rho directly.
struct RhoTiles {
  int ntile[3];
  const int* starts;  // tile t holds particles starts[t] .. starts[t+1]-1
};

template <int DIMS, int ORDER, typename R>
__global__ void __launch_bounds__(256) k_rho_tile(DiagParams P, RhoTiles Tl,
                                                  const int* __restrict__ cell, const R* o0,
                                                  const R* o1, const R* o2, const R* q, double qc,
                                                  double* __restrict__ rho) {
  using G = Geo<DIMS, ORDER, R>;
  // nodes a particle reaches relative to its cell: LO .. HI
  constexpr int LO = -(ORDER / 2), HI = ORDER / 2 + 1;
  constexpr int RX = G::T + 2 * G::A + ORDER + 1;
  constexpr int RZ = DIMS == 3 ? G::TZ + 2 * G::AZ + ORDER + 1 : 1;
  static_assert(HI - LO <= ORDER + 1, "the region holds every node a particle reaches");
  __shared__ double reg[RX * RX * RZ];
  const int t = blockIdx.x;
  const int beg = Tl.starts[t], end = Tl.starts[t + 1];
  if (beg == end) return;
  const int org[3] = {(t % Tl.ntile[0]) * G::T, ((t / Tl.ntile[0]) % Tl.ntile[1]) * G::T,
                      DIMS == 3 ? (t / (Tl.ntile[0] * Tl.ntile[1])) * G::TZ : 0};
  const int rlo[3] = {org[0] - G::A + LO, org[1] - G::A + LO, DIMS == 3 ? org[2] - G::AZ + LO : 0};
  for (int r = threadIdx.x; r < RX * RX * RZ; r += blockDim.x) reg[r] = 0.0;
  __syncthreads();
  const R* off[3] = {o0, o1, o2};
  constexpr int M = ORDER + 1;
  constexpr int MZ = DIMS == 3 ? M : 1;
  for (int p = beg + threadIdx.x; p < end; p += blockDim.x) {
    const int cl = cell[p];
    if (cl < 0 || cl >= P.ncell) continue;
    const double qp = q ? (double)q[p] : qc;
    const uint32_t rest = P.dn0.div((uint32_t)cl);
    int c3[3];
    c3[0] = cl - (int)rest * P.n[0];
    c3[1] = DIMS == 3 ? (int)(rest - P.dn1.div(rest) * P.n[1]) : (int)rest;
    c3[2] = DIMS == 3 ? (int)P.dn1.div(rest) : 0;
    double w[3][M];
    int b[3] = {0, 0, 0};
    bool ok = true;
    for (int d = 0; d < DIMS; ++d) {
      const double o = (double)off[d][p];
      ok = ok && o >= 0.0 && o < 1.0;
      if (ok) b[d] = node_weights<ORDER>(o, w[d]);
    }
    if (!ok) continue;
    if (DIMS == 2) w[2][0] = 1.0;
    // cell relative to the tile (periodic image inside the allowance)
    int l[3] = {0, 0, 0};
    bool inside = true;
    for (int d = 0; d < DIMS; ++d) {
      const int Td = d == 2 ? G::TZ : G::T, Ad = d == 2 ? G::AZ : G::A;
      int v = c3[d] - org[d];
      if (!P.open[d]) {
        v = v < 0 ? v + P.n[d] : v;
        if (v >= Td + Ad) v -= P.n[d];
      }
      l[d] = v;
      inside = inside && v >= -Ad && v < Td + Ad;
    }
    for (int k = 0; k < MZ; ++k)
      for (int j = 0; j < M; ++j)
        for (int i = 0; i < M; ++i) {
          const double v = qp * w[0][i] * w[1][j] * w[2][k];
          if (inside) {
            const int rx = l[0] + G::A - LO + b[0] + i;
            const int ry = l[1] + G::A - LO + b[1] + j;
            const int rz = DIMS == 3 ? l[2] + G::AZ - LO + b[2] + k : 0;
            atomicAdd(&reg[(rz * RX + ry) * RX + rx], v);
          } else {
            const int iz = DIMS == 3 ? axis_slot(c3[2] + b[2] + k, P.n[2], P.open[2], 0) : 0;
            const int iy = axis_slot(c3[1] + b[1] + j, P.n[1], P.open[1], 0);
            const int ix = axis_slot(c3[0] + b[0] + i, P.n[0], P.open[0], 0);
            if (ix >= 0 && iy >= 0 && iz >= 0) atomicAdd(&rho[ix + P.n[0] * (iy + P.n[1] * iz)], v);
          }
        }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < RX * RX * RZ; r += blockDim.x) {
    const double v = reg[r];
    if (v == 0.0) continue;
    const int rx = r % RX, ry = (r / RX) % RX, rz = r / (RX * RX);
    const int ix = axis_slot(rlo[0] + rx, P.n[0], P.open[0], 0);
    const int iy = axis_slot(rlo[1] + ry, P.n[1], P.open[1], 0);
    const int iz = DIMS == 3 ? axis_slot(rlo[2] + rz, P.n[2], P.open[2], 0) : 0;
    if (ix >= 0 && iy >= 0 && iz >= 0) atomicAdd(&rho[ix + P.n[0] * (iy + P.n[1] * iz)], v);
  }
}

// Per-block partials: [max|G|, max|rho|, sum C^2, max|C|, sum drho^2, sum E^2+B^2, -, -]
constexpr int NPART = 8;

template <typename R>
__global__ void __launch_bounds__(256) k_diag_fields(DiagParams P, const R* E0, const R* E1, const R* E2, const R* B0,
                              const R* B1, const R* B2, const R* J0, const R* J1, const R* J2,
                              const double* __restrict__ rho, const double* __restrict__ rho_prev,
                              const double* __restrict__ gref, double* __restrict__ gout,
                              double* __restrict__ part) {
  __shared__ double red[NPART][256];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  double v[NPART] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (idx < P.ncell) {
    const uint32_t rest = P.dn0.div((uint32_t)idx);
    int L[3];
    L[0] = idx - (int)rest * P.n[0];
    L[1] = P.dims == 3 ? (int)(rest - P.dn1.div(rest) * P.n[1]) : (int)rest;
    L[2] = P.dims == 3 ? (int)P.dn1.div(rest) : 0;
    const R* E[3] = {E0, E1, E2};
    const R* B[3] = {B0, B1, B2};
    const R* J[3] = {J0, J1, J2};
    bool interior = true;
    for (int d = 0; d < P.dims; ++d)
      if (P.open[d] && (L[d] < P.margin || L[d] > P.n[d] - 1 - P.margin)) interior = false;
    // Yee divergence at the node (backward differences)
    double divE = 0.0, divJ = 0.0;
    for (int d = 0; d < P.dims; ++d) {
      int M[3] = {L[0], L[1], L[2]};
      M[d] -= 1;
      if (M[d] < 0) {
        if (P.open[d]) continue;  // not interior; value unused
        M[d] += P.n[d];
      }
      const int im = M[0] + P.n[0] * (M[1] + P.n[1] * M[2]);
      divE += ((double)E[d][idx] - (double)E[d][im]) / P.dx[d];
      divJ += ((double)J[d][idx] - (double)J[d][im]) / P.dx[d];
    }
    const double r = rho[idx];
    double G = divE - r - (gref ? gref[idx] : 0.0);
    if (gout) gout[idx] = interior ? G : 0.0;
    v[1] = fabs(r);
    if (interior) {
      v[0] = fabs(G);
      if (rho_prev) {
        const double dr = (r - rho_prev[idx]) / P.dt;
        const double C = dr + divJ;
        v[2] = C * C;
        v[3] = fabs(C);
        v[4] = dr * dr;
      }
    }
    double wf = 0.0;
    for (int c = 0; c < 3; ++c) {
      bool ie = true, ib = true;
      for (int d = 0; d < P.dims; ++d) {
        if (!P.open[d]) continue;
        if (L[d] > P.n[d] - 1 - (d == c ? 1 : 0)) ie = false;
        if (L[d] > P.n[d] - 1 - (d != c ? 1 : 0)) ib = false;
      }
      if (ie) wf += (double)E[c][idx] * (double)E[c][idx];
      if (ib) wf += (double)B[c][idx] * (double)B[c][idx];
    }
    v[5] = wf;
  }
  for (int k = 0; k < NPART; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + s]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + s]);
      red[2][threadIdx.x] += red[2][threadIdx.x + s];
      red[3][threadIdx.x] = fmax(red[3][threadIdx.x], red[3][threadIdx.x + s]);
      red[4][threadIdx.x] += red[4][threadIdx.x + s];
      red[5][threadIdx.x] += red[5][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < NPART; ++k) part[(long)blockIdx.x * NPART + k] = red[k][0];
}

// Per-block partials: [sum m (gamma-1), live count] with the macro-particle
// mass density m = |q| / |q/m| (minv = 1 / |q/m|)
template <typename R>
__global__ void __launch_bounds__(256) k_diag_particles(const int* __restrict__ cell, const R* u0, const R* u1,
                                 const R* u2, const R* q, double qc, double minv, long np,
                                 double* __restrict__ part) {
  __shared__ double red[2][256];
  double wk = 0.0, alive = 0.0;
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < np; p += (long)gridDim.x * blockDim.x) {
    if (cell[p] < 0) continue;
    const double ux = u0[p], uy = u1[p], uz = u2[p];
    const double g = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
    wk += fabs(q ? (double)q[p] : qc) * minv * (g - 1.0);
    alive += 1.0;
  }
  red[0][threadIdx.x] = wk;
  red[1][threadIdx.x] = alive;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = red[0][0];
    part[2 * blockIdx.x + 1] = red[1][0];
  }
}

__global__ void k_fill_d(double* a, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    a[i] = 0.0;
}

static DiagParams diag_params(const pic_ctx* ctx) {
  const pic_config& c = ctx->cfg;
  DiagParams P;
  P.dims = c.dims;
  P.order = c.order;
  P.margin = 1 + c.order / 2;
  P.dV = 1.0;
  for (int d = 0; d < 3; ++d) {
    P.n[d] = d < c.dims ? c.n[d] : 1;
    P.open[d] = d < c.dims && c.bc[d] == PIC_BC_OPEN;
    P.dx[d] = c.dx[d];
    if (d < c.dims) P.dV *= c.dx[d];
  }
  P.dt = c.dt;
  P.dn0.init((uint32_t)P.n[0]);
  P.dn1.init((uint32_t)P.n[1]);
  P.ncell = P.n[0] * P.n[1] * P.n[2];
  return P;
}

template <int DIMS, int ORDER, typename R>
static void rho_t(const DiagParams& P, const pic_particles* p, double qc, double* rho,
                  const RhoTiles* tiles, int ntiles, hipStream_t s) {
  const long np = p->np;
  if (np == 0) return;
  if (tiles) {
    k_rho_tile<DIMS, ORDER, R><<<dim3((unsigned)ntiles), dim3(256), 0, s>>>(
        P, *tiles, p->cell, (const R*)p->off[0], (const R*)p->off[1], (const R*)p->off[2],
        (const R*)p->q, qc, rho);
    return;
  }
  k_deposit_rho<DIMS, ORDER, R><<<dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s>>>(
      P, p->cell, (const R*)p->off[0], (const R*)p->off[1], (const R*)p->off[2], (const R*)p->q, qc,
      np, rho);
}

int launch_deposit_rho(const pic_ctx* ctx, const pic_particles* p, double* rho, void* ws,
                       hipStream_t s, bool accumulate) {
  DiagParams P = diag_params(ctx);
  // the tile kernel needs the bins of a sort of these very arrays in this
  // workspace (the particles may have moved since)
  RhoTiles T;
  const bool binned = ws && ctx->sorted_cell == p->cell && ctx->sorted_ws == ws &&
                      ctx->sorted_np == p->np;
  if (binned) {
    for (int d = 0; d < 3; ++d) T.ntile[d] = ctx->ntile[d];
    T.starts = (const int*)((const char*)ws + ws_layout(ctx, p->np).starts);
  }
  const RhoTiles* tiles = binned ? &T : nullptr;
  if (!accumulate)
    k_fill_d<<<dim3((unsigned)((P.ncell + 255) / 256 < 4096 ? (P.ncell + 255) / 256 : 4096)),
               dim3(256), 0, s>>>(rho, P.ncell);
  const bool dbl = ctx->cfg.real_bytes == 8;
  const int D = P.dims, O = P.order;
  const double qc = ctx->cfg.q_const;
#define PIC_RHO(DD, OO)                                              \
  if (D == DD && O == OO) {                                          \
    if (dbl)                                                         \
      rho_t<DD, OO, double>(P, p, qc, rho, tiles, ctx->ntiles, s);   \
    else                                                             \
      rho_t<DD, OO, float>(P, p, qc, rho, tiles, ctx->ntiles, s);    \
  }
  PIC_RHO(2, 1) PIC_RHO(2, 2) PIC_RHO(2, 3) PIC_RHO(2, 4)
  PIC_RHO(3, 1) PIC_RHO(3, 2) PIC_RHO(3, 3) PIC_RHO(3, 4)
#undef PIC_RHO
  return (int)hipGetLastError();
}

// Diagnostics of one or more species sharing the fields: rho is the sum of
// the species' charge densities; the kinetic energy sums every species'
// mass density (q over q/m) times gamma - 1.  Each species' particle
// partials go to the diagnostics scratch of its own workspace.
template <typename R>
static int diag_t(int ns, const pic_ctx* const* ctx, const pic_particles* const* p,
                  void* const* ws, const pic_fields* f, const double* rho_prev,
                  const double* gauss_ref, double* rho_out, double* gauss_out, pic_diag* out,
                  hipStream_t s) {
  DiagParams P = diag_params(ctx[0]);
  for (int k = 0; k < ns; ++k) {
    int err = launch_deposit_rho(ctx[k], p[k], rho_out, ws[k], s, k > 0);
    if (err) return err;
  }
  WsLayout L0 = ws_layout(ctx[0], p[0]->np);
  double* part = (double*)((char*)ws[0] + L0.diag);
  const unsigned gf = (unsigned)((P.ncell + 255) / 256);
  k_diag_fields<R><<<dim3(gf), dim3(256), 0, s>>>(
      P, (const R*)f->E[0], (const R*)f->E[1], (const R*)f->E[2], (const R*)f->B[0],
      (const R*)f->B[1], (const R*)f->B[2], (const R*)f->J[0], (const R*)f->J[1],
      (const R*)f->J[2], rho_out, rho_prev, gauss_ref, gauss_out, part);
  const unsigned gp = 1024;
  for (int k = 0; k < ns; ++k) {
    WsLayout Lk = ws_layout(ctx[k], p[k]->np);
    double* ppart = (double*)((char*)ws[k] + Lk.diag) + (size_t)gf * NPART;
    const double minv = 1.0 / fabs(ctx[k]->cfg.q_over_m);
    k_diag_particles<R><<<dim3(gp), dim3(256), 0, s>>>(
        p[k]->cell, (const R*)p[k]->u[0], (const R*)p[k]->u[1], (const R*)p[k]->u[2],
        (const R*)p[k]->q, ctx[k]->cfg.q_const, minv, p[k]->np, ppart);
  }
  int err = (int)hipGetLastError();
  if (err) return err;
  const size_t nfp = (size_t)gf * NPART + 2 * gp;
  double* host = (double*)malloc(nfp * sizeof(double));
  if (!host) return (int)hipErrorOutOfMemory;
  double gmax = 0, rmax = 0, c2 = 0, cmax = 0, d2 = 0, wf = 0, wk = 0, alive = 0;
  for (int k = 0; k < ns && !err; ++k) {
    WsLayout Lk = ws_layout(ctx[k], p[k]->np);
    const double* src = (const double*)((const char*)ws[k] + Lk.diag);
    // species 0 brings the field partials as well
    const size_t off = k == 0 ? 0 : (size_t)gf * NPART;
    err = (int)hipMemcpyAsync(host + off, src + off, (nfp - off) * sizeof(double),
                              hipMemcpyDeviceToHost, s);
    if (!err) err = (int)hipStreamSynchronize(s);
    if (err) break;
    if (k == 0) {
      for (unsigned b = 0; b < gf; ++b) {
        const double* v = host + (size_t)b * NPART;
        gmax = fmax(gmax, v[0]);
        rmax = fmax(rmax, v[1]);
        c2 += v[2];
        cmax = fmax(cmax, v[3]);
        d2 += v[4];
        wf += v[5];
      }
    }
    for (unsigned b = 0; b < gp; ++b) {
      wk += host[(size_t)gf * NPART + 2 * b];
      alive += host[(size_t)gf * NPART + 2 * b + 1];
    }
  }
  free(host);
  if (err) return err;
  out->gauss_max = gmax;
  out->rho_max = rmax;
  out->gauss_rel = rmax > 0 ? gmax / rmax : 0.0;
  out->cont_max = rho_prev ? cmax : 0.0;
  out->cont_rel_l2 = (rho_prev && d2 > 0) ? sqrt(c2 / d2) : 0.0;
  out->cont_rel_inf = (rho_prev && rmax > 0) ? cmax / (rmax / P.dt) : 0.0;
  out->w_field = 0.5 * wf * P.dV;
  out->w_kin = wk * P.dV;
  out->n_alive = (int64_t)alive;
  return 0;
}

int launch_diagnostics(int ns, const pic_ctx* const* ctx, const pic_particles* const* p,
                       void* const* ws, const pic_fields* f, const double* rho_prev,
                       const double* gauss_ref, double* rho_out, double* gauss_out, pic_diag* out,
                       hipStream_t s) {
  return ctx[0]->cfg.real_bytes == 8
             ? diag_t<double>(ns, ctx, p, ws, f, rho_prev, gauss_ref, rho_out, gauss_out, out, s)
             : diag_t<float>(ns, ctx, p, ws, f, rho_prev, gauss_ref, rho_out, gauss_out, out, s);
}

long diag_len(const pic_config& cf) {
  long ncell = 1;
  for (int d = 0; d < cf.dims; ++d) ncell *= cf.n[d];
  return ((ncell + 255) / 256) * NPART + 2 * 1024;
}

}  // namespace pic
