// FP64 CPU oracle of one explicit, fully relativistic EM-PIC step.
//
// TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the CPU
// baseline of bench.py; never by the product library.  Plain loops in the
// order of the paper's PIC loop (Sec. 2) and of its vector algorithm
// (Sec. 5.2, steps i-v), written for readability, not speed.
//
// Every routine is templated on the scalar type R so that the same code runs
// in double and in a forward-mode dual number (value + one directional
// derivative), which yields exact JVPs of the discrete step for checking the
// hand-written adjoint.  Branch decisions (floor, crossing tests) use the
// value part only, so the JVP is the derivative of the branch taken.
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- dual number
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}  // NOLINT: constants promote with zero derivative
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
inline Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
inline Dual operator+(double a, Dual b) { return {a + b.v, b.d}; }
inline Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
inline Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
inline Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
inline Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
inline Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
inline Dual operator/(double a, Dual b) { return Dual(a) / b; }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return {s, a.d / (2.0 * s)};
}
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
using std::sqrt;

// ---------------------------------------------------------------- grid
struct Grid {
  int dims, order;
  long n[3];
  double dx[3], dt, qm;
  int bc[3];
  explicit Grid(const oracle_config& c) {
    dims = c.dims;
    order = c.order;
    for (int d = 0; d < 3; ++d) {
      n[d] = c.n[d];
      dx[d] = c.dx[d];
      bc[d] = c.bc[d];
    }
    if (dims == 2) {
      n[2] = 1;
      bc[2] = ORACLE_PERIODIC;
    }
    dt = c.dt;
    qm = c.q_over_m;
  }
  long ncell() const { return n[0] * n[1] * n[2]; }
  long idx(long i, long j, long k) const { return i + n[0] * (j + n[1] * k); }
  bool open(int d) const { return d < dims && bc[d] == ORACLE_OPEN; }
  double cell_volume() const {
    double v = 1.0;
    for (int d = 0; d < dims; ++d) v *= dx[d];
    return v;
  }
  // Storage index along axis d of the sample with lattice index i, for a
  // quantity node-located (st = 0) or half-way between nodes (st = 1) along
  // d.  Periodic axes wrap; on open axes a sample at position p = i + st/2 is
  // inside iff 0 <= p <= n-1, otherwise -1.  In 2D the z axis is one plane.
  long axis_index(int d, long i, int st) const {
    if (d >= dims) return 0;
    if (bc[d] == ORACLE_PERIODIC) {
      long m = i % n[d];
      return m < 0 ? m + n[d] : m;
    }
    long last = n[d] - 1 - st;
    return (i < 0 || i > last) ? -1 : i;
  }
};

// Staggering of the Yee components: E_c (and J_c) half-way along c; B_c
// half-way along the two other axes.  Standard Yee layout (the paper only
// notes that components sit at different positions in the cell, Sec. 5.1).
inline int stag_e(int c, int d) { return d == c ? 1 : 0; }
inline int stag_b(int c, int d) { return d == c ? 0 : 1; }

// ---------------------------------------------------------------- shapes
// Index of the piece of the order-n B-spline that contains X: the node
// stencil switches at integer planes for odd orders and at half-integer
// planes for even orders.
inline long piece_index(int order, double X) {
  return (order % 2 == 1) ? (long)std::floor(X) : (long)std::floor(X + 0.5);
}
inline long stencil_base(int order, double X) {
  return piece_index(order, X) - order / 2;
}

// B-spline weights of order 1..4 on the nodes base..base+order, evaluated at
// X (the polynomial piece belonging to that stencil; used also at the closed
// ends of the piece, where the spline is continuous).  Order 4 is the quartic
// spline of Table 3's fourth benchmark: with t = X - (base + 2), the distance
// to the centre node, the five weights are the quartic B-spline at distances
// t + 2, t + 1, t, 1 - t, 2 - t.
template <class R>
void shape_on_base(int order, R X, long base, R* w) {
  if (order == 4) {
    R t = X - (double)(base + 2);
    R t2 = t * t, t3 = t2 * t, t4 = t2 * t2;
    R a = 1.0 - 2.0 * t, b = 1.0 + 2.0 * t;
    w[0] = a * a * a * a / 384.0;
    w[1] = (19.0 - 44.0 * t + 24.0 * t2 + 16.0 * t3 - 16.0 * t4) / 96.0;
    w[2] = (115.0 - 120.0 * t2 + 48.0 * t4) / 192.0;
    w[3] = (19.0 + 44.0 * t + 24.0 * t2 - 16.0 * t3 - 16.0 * t4) / 96.0;
    w[4] = b * b * b * b / 384.0;
    return;
  }
  if (order == 1) {
    R t = X - (double)base;
    w[0] = 1.0 - t;
    w[1] = t;
  } else if (order == 2) {
    R dlt = X - (double)(base + 1);
    R a = 0.5 - dlt, b = 0.5 + dlt;
    w[0] = 0.5 * a * a;
    w[1] = 0.75 - dlt * dlt;
    w[2] = 0.5 * b * b;
  } else {
    R t = X - (double)(base + 1);
    R s = 1.0 - t;
    R t2 = t * t, t3 = t2 * t;
    w[0] = s * s * s / 6.0;
    w[1] = (4.0 - 6.0 * t2 + 3.0 * t3) / 6.0;
    w[2] = (1.0 + 3.0 * t + 3.0 * t2 - 3.0 * t3) / 6.0;
    w[3] = t3 / 6.0;
  }
}

// ---------------------------------------------------------------- gather
// Field component F (storage layout of the grid) interpolated at X with
// order-n weights taken at the component's own staggered position.
template <class R>
R interp(const Grid& g, const R* F, const int st[3], const R X[3]) {
  long base[3];
  R w[3][5];
  int cnt[3];
  for (int d = 0; d < 3; ++d) {
    if (d < g.dims) {
      R P = X[d] - 0.5 * st[d];
      base[d] = stencil_base(g.order, val(P));
      shape_on_base(g.order, P, base[d], w[d]);
      cnt[d] = g.order + 1;
    } else {
      base[d] = 0;
      w[d][0] = R(1.0);
      cnt[d] = 1;
    }
  }
  R s(0.0);
  for (int k = 0; k < cnt[2]; ++k) {
    long kk = g.axis_index(2, base[2] + k, st[2]);
    if (kk < 0) continue;
    for (int j = 0; j < cnt[1]; ++j) {
      long jj = g.axis_index(1, base[1] + j, st[1]);
      if (jj < 0) continue;
      for (int i = 0; i < cnt[0]; ++i) {
        long ii = g.axis_index(0, base[0] + i, st[0]);
        if (ii < 0) continue;
        s += w[0][i] * w[1][j] * w[2][k] * F[g.idx(ii, jj, kk)];
      }
    }
  }
  return s;
}

template <class R>
void gather_one(const Grid& g, const R* E, const R* B, const R X[3], R Ep[3],
                R Bp[3]) {
  const long nc = g.ncell();
  for (int c = 0; c < 3; ++c) {
    int se[3] = {stag_e(c, 0), stag_e(c, 1), stag_e(c, 2)};
    int sb[3] = {stag_b(c, 0), stag_b(c, 1), stag_b(c, 2)};
    Ep[c] = interp(g, E + c * nc, se, X);
    Bp[c] = interp(g, B + c * nc, sb, X);
  }
}

// ---------------------------------------------------------------- push
// Relativistic Boris step u^{n-1/2} -> u^{n+1/2} (the paper asks only for the
// fully relativistic equations of motion, Sec. 2; Boris is the reading):
// half electric kick, magnetic rotation with gamma from the half-kicked
// momentum, half electric kick.
template <class R>
void boris_one(const Grid& g, R u[3], const R Ep[3], const R Bp[3]) {
  const double h = 0.5 * g.qm * g.dt;
  R um[3], t[3], s[3], up[3], uq[3];
  for (int c = 0; c < 3; ++c) um[c] = u[c] + h * Ep[c];
  R gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  for (int c = 0; c < 3; ++c) t[c] = h * Bp[c] / gm;
  R tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  for (int c = 0; c < 3; ++c) s[c] = 2.0 * t[c] / (1.0 + tt);
  // u' = u- + u- x t
  up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
  up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
  up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
  // u+ = u- + u' x s
  uq[0] = um[0] + (up[1] * s[2] - up[2] * s[1]);
  uq[1] = um[1] + (up[2] * s[0] - up[0] * s[2]);
  uq[2] = um[2] + (up[0] * s[1] - up[1] * s[0]);
  for (int c = 0; c < 3; ++c) u[c] = uq[c] + h * Ep[c];
}

// ---------------------------------------------------------------- deposit
// Charge-conserving current of one straight path X0 -> X1 (Sec. 5.2, steps
// iv-v): the path is split into virtual segments at the planes where the
// node stencil of the shape switches (at most one crossing per axis, so at
// most dims+1 segments); each segment then deposits with the Esirkepov
// density decomposition on its own fixed (n+1)^D stencil, the stencil being
// chosen from the segment's midpoint.  J_d at (i+1/2) is the running sum
// along d of -q dx_d/dt W_d, starting from zero below the stencil.  In 2D
// the out-of-plane current is q v_z times the segment's time fraction times
// the time-averaged 2D weight.
template <class R>
void deposit_path(const Grid& g, R* J, const R X0[3], const R X1[3], double q,
                  R vz) {
  const int D = g.dims, ord = g.order, m = ord + 1;
  const long nc = g.ncell();
  // crossing fractions along the path, one per axis at most
  R fr[3];
  int fax[3];
  double fplane[3];
  int nf = 0;
  for (int d = 0; d < D; ++d) {
    long k0 = piece_index(ord, val(X0[d])), k1 = piece_index(ord, val(X1[d]));
    if (k0 == k1) continue;
    double P = (double)std::max(k0, k1) - ((ord % 2 == 0) ? 0.5 : 0.0);
    R f = (P - X0[d]) / (X1[d] - X0[d]);
    if (!(val(f) > 0.0 && val(f) < 1.0)) continue;  // crossing at an end: none
    fr[nf] = f;
    fax[nf] = d;
    fplane[nf] = P;
    ++nf;
  }
  // ascending order of the fractions (insertion sort, at most 3 entries)
  for (int a = 1; a < nf; ++a)
    for (int b = a; b > 0 && val(fr[b]) < val(fr[b - 1]); --b) {
      std::swap(fr[b], fr[b - 1]);
      std::swap(fax[b], fax[b - 1]);
      std::swap(fplane[b], fplane[b - 1]);
    }
  // segment end points: X0, crossing points, X1
  R pts[5][3];  // X0, up to three crossing points, X1
  R tpar[5];
  for (int d = 0; d < 3; ++d) pts[0][d] = X0[d];
  tpar[0] = R(0.0);
  for (int s = 0; s < nf; ++s) {
    for (int d = 0; d < 3; ++d)
      pts[s + 1][d] = (d == fax[s]) ? R(fplane[s]) : X0[d] + fr[s] * (X1[d] - X0[d]);
    tpar[s + 1] = fr[s];
  }
  for (int d = 0; d < 3; ++d) pts[nf + 1][d] = X1[d];
  tpar[nf + 1] = R(1.0);

  for (int s = 0; s <= nf; ++s) {
    const R* Xa = pts[s];
    const R* Xb = pts[s + 1];
    R ftime = tpar[s + 1] - tpar[s];
    if (!(val(ftime) > 0.0)) continue;  // equal crossings: zero-length segment
    long base[3];
    R S0[3][5], dS[3][5];
    for (int d = 0; d < D; ++d) {
      double mid = 0.5 * (val(Xa[d]) + val(Xb[d]));
      base[d] = stencil_base(ord, mid);
      R S1[5];
      shape_on_base(ord, Xa[d], base[d], S0[d]);
      shape_on_base(ord, Xb[d], base[d], S1);
      for (int i = 0; i < m; ++i) dS[d][i] = S1[i] - S0[d][i];
    }
    if (D == 3) {
      for (int c = 0; c < 3; ++c) {
        // W_c on the stencil, then the prefix sum along c
        const int a = (c + 1) % 3, b = (c + 2) % 3;
        const double fac = -q * g.dx[c] / g.dt;
        for (int ib = 0; ib < m; ++ib)
          for (int ia = 0; ia < m; ++ia) {
            R acc(0.0);
            for (int ic = 0; ic < m - 1; ++ic) {
              R W = dS[c][ic] * (S0[a][ia] * S0[b][ib] + 0.5 * dS[a][ia] * S0[b][ib] +
                                 0.5 * S0[a][ia] * dS[b][ib] +
                                 dS[a][ia] * dS[b][ib] / 3.0);
              acc += fac * W;
              long L[3];
              L[c] = base[c] + ic;
              L[a] = base[a] + ia;
              L[b] = base[b] + ib;
              long ii = g.axis_index(0, L[0], stag_e(c, 0));
              long jj = g.axis_index(1, L[1], stag_e(c, 1));
              long kk = g.axis_index(2, L[2], stag_e(c, 2));
              if (ii < 0 || jj < 0 || kk < 0) continue;
              J[c * nc + g.idx(ii, jj, kk)] += acc;
            }
          }
      }
    } else {
      // in-plane components: prefix sums along x and along y
      for (int c = 0; c < 2; ++c) {
        const int a = 1 - c;
        const double fac = -q * g.dx[c] / g.dt;
        for (int ia = 0; ia < m; ++ia) {
          R acc(0.0);
          for (int ic = 0; ic < m - 1; ++ic) {
            R W = dS[c][ic] * (S0[a][ia] + 0.5 * dS[a][ia]);
            acc += fac * W;
            long L[2];
            L[c] = base[c] + ic;
            L[a] = base[a] + ia;
            long ii = g.axis_index(0, L[0], stag_e(c, 0));
            long jj = g.axis_index(1, L[1], stag_e(c, 1));
            if (ii < 0 || jj < 0) continue;
            J[c * nc + g.idx(ii, jj, 0)] += acc;
          }
        }
      }
      // out-of-plane component, node-located in the plane
      for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
          R W = S0[0][i] * S0[1][j] + 0.5 * dS[0][i] * S0[1][j] +
                0.5 * S0[0][i] * dS[1][j] + dS[0][i] * dS[1][j] / 3.0;
          long ii = g.axis_index(0, base[0] + i, 0);
          long jj = g.axis_index(1, base[1] + j, 0);
          if (ii < 0 || jj < 0) continue;
          J[2 * nc + g.idx(ii, jj, 0)] += q * vz * ftime * W;
        }
    }
  }
}

// ---------------------------------------------------------------- particle pass
// One particle: gather at X^n, push u^{n-1/2} -> u^{n+1/2}, move to X^{n+1},
// deposit J^{n+1/2} along X^n -> X^{n+1}, then wrap (periodic) or absorb
// (open: outside [0, n-1)).
template <class R>
void advance_particle(const Grid& g, R* X, R* u, double q, int8_t* alive,
                      const R* E, const R* B, R* J) {
  R Ep[3], Bp[3];
  gather_one(g, E, B, X, Ep, Bp);
  boris_one(g, u, Ep, Bp);
  R gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  R X1[3];
  for (int d = 0; d < 3; ++d)
    X1[d] = (d < g.dims) ? X[d] + g.dt * u[d] / (gam * g.dx[d]) : X[d];
  deposit_path(g, J, X, X1, q, u[2] / gam);
  bool dead = false;
  for (int d = 0; d < g.dims; ++d) {
    const double nd = (double)g.n[d];
    if (g.bc[d] == ORACLE_PERIODIC) {
      if (val(X1[d]) >= nd) X1[d] = X1[d] - nd;
      else if (val(X1[d]) < 0.0) X1[d] = X1[d] + nd;
      if (val(X1[d]) >= nd) X1[d] = X1[d] - nd;  // -tiny + n rounded up to n
    } else if (val(X1[d]) < 0.0 || val(X1[d]) >= nd - 1.0) {
      dead = true;
    }
  }
  for (int d = 0; d < 3; ++d) X[d] = X1[d];
  if (dead) *alive = 0;
}

template <class R>
void push_deposit_impl(const Grid& g, long np, R* X, R* u, const double* q,
                       int8_t* alive, const R* E, const R* B, R* J, bool add = false) {
  if (!add) std::fill(J, J + 3 * g.ncell(), R(0.0));
  for (long p = 0; p < np; ++p) {
    if (!alive[p]) continue;
    advance_particle(g, X + 3 * p, u + 3 * p, q[p], alive + p, E, B, J);
  }
}

// Shared-memory variant (Sec. 3.1): particles split evenly over nthreads,
// each thread deposits into its own copy of the current grid, then the
// copies are reduced into J, the reduction also split over the threads.
void push_deposit_threads(const Grid& g, long np, double* X, double* u,
                          const double* q, int8_t* alive, const double* E,
                          const double* B, double* J, int nthreads, bool add = false) {
  const long len = 3 * g.ncell();
  std::vector<double> copies((size_t)nthreads * len, 0.0);
#ifdef _OPENMP
#pragma omp parallel num_threads(nthreads)
#endif
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    long lo = np * t / nthreads, hi = np * (t + 1) / nthreads;
    double* Jt = copies.data() + (size_t)t * len;
    for (long p = lo; p < hi; ++p) {
      if (!alive[p]) continue;
      advance_particle(g, X + 3 * p, u + 3 * p, q[p], alive + p, E, B, Jt);
    }
#ifdef _OPENMP
#pragma omp barrier
#pragma omp for
#endif
    for (long i = 0; i < len; ++i) {
      double s = 0.0;
      for (int c = 0; c < nthreads; ++c) s += copies[(size_t)c * len + i];
      J[i] = add ? J[i] + s : s;
    }
  }
}

// ---------------------------------------------------------------- FDTD
// Forward-difference curl of E at the B positions: (C E)_c = d_a E_b - d_b E_a
// with (c, a, b) cyclic; derivatives along axes absent in 2D are zero.
template <class R>
R curl_e_at(const Grid& g, const R* E, int c, long i, long j, long k) {
  const long nc = g.ncell();
  const int a = (c + 1) % 3, b = (c + 2) % 3;
  long L[3] = {i, j, k};
  auto fwd = [&](int comp, int axis) -> R {  // d_axis E_comp, forward
    if (axis >= g.dims) return R(0.0);
    long M[3] = {L[0], L[1], L[2]};
    M[axis] += 1;
    long ii = g.axis_index(0, M[0], stag_e(comp, 0));
    long jj = g.axis_index(1, M[1], stag_e(comp, 1));
    long kk = g.axis_index(2, M[2], stag_e(comp, 2));
    R up = (ii < 0 || jj < 0 || kk < 0) ? R(0.0) : E[comp * nc + g.idx(ii, jj, kk)];
    R here = E[comp * nc + g.idx(L[0], L[1], L[2])];
    return (up - here) / g.dx[axis];
  };
  return fwd(b, a) - fwd(a, b);
}

// Backward-difference curl of B at the E positions, the transpose of C:
// (C^T B)_c = d_a B_b - d_b B_a, backward differences.
template <class R>
R curl_b_at(const Grid& g, const R* B, int c, long i, long j, long k) {
  const long nc = g.ncell();
  const int a = (c + 1) % 3, b = (c + 2) % 3;
  long L[3] = {i, j, k};
  auto bwd = [&](int comp, int axis) -> R {  // d_axis B_comp, backward
    if (axis >= g.dims) return R(0.0);
    long M[3] = {L[0], L[1], L[2]};
    M[axis] -= 1;
    long ii = g.axis_index(0, M[0], stag_b(comp, 0));
    long jj = g.axis_index(1, M[1], stag_b(comp, 1));
    long kk = g.axis_index(2, M[2], stag_b(comp, 2));
    R dn = (ii < 0 || jj < 0 || kk < 0) ? R(0.0) : B[comp * nc + g.idx(ii, jj, kk)];
    R here = B[comp * nc + g.idx(L[0], L[1], L[2])];
    return (here - dn) / g.dx[axis];
  };
  return bwd(b, a) - bwd(a, b);
}

// The field loops below update every sample from values that no other
// iteration of the same loop writes, so their z planes run in parallel
// (OpenMP) with results identical to the serial loops.

// Is the storage slot (i,j,k) of a component with staggering st inside the
// domain?
inline bool slot_inside(const Grid& g, const int st[3], long i, long j, long k) {
  return g.axis_index(0, i, st[0]) >= 0 && g.axis_index(1, j, st[1]) >= 0 &&
         g.axis_index(2, k, st[2]) >= 0;
}

template <class R>
void half_b(const Grid& g, const R* E, R* B, double h) {
  const long nc = g.ncell();
  std::vector<R> cE(3 * nc);
  for (int c = 0; c < 3; ++c) {
    int sb[3] = {stag_b(c, 0), stag_b(c, 1), stag_b(c, 2)};
#ifdef _OPENMP
    #pragma omp parallel for schedule(static)
#endif
    for (long k = 0; k < g.n[2]; ++k)
      for (long j = 0; j < g.n[1]; ++j)
        for (long i = 0; i < g.n[0]; ++i)
          cE[c * nc + g.idx(i, j, k)] =
              slot_inside(g, sb, i, j, k) ? curl_e_at(g, E, c, i, j, k) : R(0.0);
  }
  for (int c = 0; c < 3; ++c) {
    int sb[3] = {stag_b(c, 0), stag_b(c, 1), stag_b(c, 2)};
#ifdef _OPENMP
    #pragma omp parallel for schedule(static)
#endif
    for (long k = 0; k < g.n[2]; ++k)
      for (long j = 0; j < g.n[1]; ++j)
        for (long i = 0; i < g.n[0]; ++i)
          if (slot_inside(g, sb, i, j, k))
            B[c * nc + g.idx(i, j, k)] -= h * cE[c * nc + g.idx(i, j, k)];
  }
}

// Open-face classification of an E_c slot: the open axes d != c on whose
// first or last node plane the (tangential) sample lies.
inline int e_boundary_axes(const Grid& g, int c, const long L[3], int* axes) {
  int cnt = 0;
  for (int d = 0; d < g.dims; ++d) {
    if (d == c || !g.open(d)) continue;
    if (L[d] == 0 || L[d] == g.n[d] - 1) axes[cnt++] = d;
  }
  return cnt;
}

template <class R>
void advance_e(const Grid& g, R* E, const R* B, const R* J) {
  const long nc = g.ncell();
  std::vector<R> Eold(E, E + 3 * nc);
  // Yee update of every interior sample
  for (int c = 0; c < 3; ++c) {
    int se[3] = {stag_e(c, 0), stag_e(c, 1), stag_e(c, 2)};
#ifdef _OPENMP
    #pragma omp parallel for schedule(static)
#endif
    for (long k = 0; k < g.n[2]; ++k)
      for (long j = 0; j < g.n[1]; ++j)
        for (long i = 0; i < g.n[0]; ++i) {
          if (!slot_inside(g, se, i, j, k)) continue;
          long L[3] = {i, j, k};
          int axes[3];
          if (e_boundary_axes(g, c, L, axes) > 0) continue;
          long s = c * nc + g.idx(i, j, k);
          E[s] = Eold[s] + g.dt * (curl_b_at(g, B, c, i, j, k) - J[s]);
        }
  }
  // Mur first order on open faces, F0^{n+1} = F1^n + kappa (F1^{n+1} - F0^n),
  // kappa = (dt - dx)/(dt + dx), F1 the next sample inward along the face
  // normal.  Samples on one face first; samples on two faces (edges) then use
  // the lowest such axis, whose inward neighbour lies on one face only.
  for (int pass = 1; pass <= 2; ++pass)
    for (int c = 0; c < 3; ++c) {
      int se[3] = {stag_e(c, 0), stag_e(c, 1), stag_e(c, 2)};
#ifdef _OPENMP
      #pragma omp parallel for schedule(static)
#endif
      for (long k = 0; k < g.n[2]; ++k)
        for (long j = 0; j < g.n[1]; ++j)
          for (long i = 0; i < g.n[0]; ++i) {
            if (!slot_inside(g, se, i, j, k)) continue;
            long L[3] = {i, j, k};
            int axes[3];
            if (e_boundary_axes(g, c, L, axes) != pass) continue;
            int d = axes[0];
            long M[3] = {i, j, k};
            M[d] += (L[d] == 0) ? 1 : -1;
            long s0 = c * nc + g.idx(i, j, k);
            long s1 = c * nc + g.idx(M[0], M[1], M[2]);
            double kap = (g.dt - g.dx[d]) / (g.dt + g.dx[d]);
            E[s0] = Eold[s1] + kap * (E[s1] - Eold[s0]);
          }
    }
}

template <class R>
void field_advance_impl(const Grid& g, R* E, R* B, const R* J) {
  half_b(g, E, B, 0.5 * g.dt);
  advance_e(g, E, B, J);
  half_b(g, E, B, 0.5 * g.dt);
}

template <class R>
void step_impl(const Grid& g, long np, R* X, R* u, const double* q,
               int8_t* alive, R* E, R* B, R* J, int nsteps) {
  for (int s = 0; s < nsteps; ++s) {
    push_deposit_impl(g, np, X, u, q, alive, E, B, J);
    field_advance_impl(g, E, B, J);
  }
}

std::vector<Dual> to_dual(const double* v, const double* d, size_t n) {
  std::vector<Dual> out(n);
  for (size_t i = 0; i < n; ++i) out[i] = Dual(v[i], d[i]);
  return out;
}
void from_dual(const std::vector<Dual>& a, double* v, double* d) {
  for (size_t i = 0; i < a.size(); ++i) {
    v[i] = a[i].v;
    d[i] = a[i].d;
  }
}

}  // namespace

// ================================================================ C API
extern "C" {

void oracle_shape(int32_t order, double X, int64_t* base, double* w) {
  long b = stencil_base(order, X);
  *base = b;
  shape_on_base(order, X, b, w);
}

void oracle_gather(const oracle_config* cfg, int64_t np, const double* X,
                   const double* E, const double* B, double* Ep, double* Bp) {
  Grid g(*cfg);
  for (long p = 0; p < np; ++p) gather_one(g, E, B, X + 3 * p, Ep + 3 * p, Bp + 3 * p);
}

void oracle_boris(const oracle_config* cfg, int64_t np, double* u,
                  const double* Ep, const double* Bp) {
  Grid g(*cfg);
  for (long p = 0; p < np; ++p) boris_one(g, u + 3 * p, Ep + 3 * p, Bp + 3 * p);
}

void oracle_deposit_paths(const oracle_config* cfg, int64_t np,
                          const double* X0, const double* X1, const double* q,
                          const double* vz, double* J) {
  Grid g(*cfg);
  for (long p = 0; p < np; ++p)
    deposit_path(g, J, X0 + 3 * p, X1 + 3 * p, q[p], vz ? vz[p] : 0.0);
}

void oracle_push_deposit(const oracle_config* cfg, int64_t np, double* X,
                         double* u, const double* q, int8_t* alive,
                         const double* E, const double* B, double* J,
                         int32_t nthreads) {
  Grid g(*cfg);
  if (nthreads > 1)
    push_deposit_threads(g, np, X, u, q, alive, E, B, J, nthreads);
  else
    push_deposit_impl(g, np, X, u, q, alive, E, B, J);
}

void oracle_push_deposit_add(const oracle_config* cfg, int64_t np, double* X,
                             double* u, const double* q, int8_t* alive,
                             const double* E, const double* B, double* J,
                             int32_t nthreads) {
  Grid g(*cfg);
  if (nthreads > 1)
    push_deposit_threads(g, np, X, u, q, alive, E, B, J, nthreads, true);
  else
    push_deposit_impl(g, np, X, u, q, alive, E, B, J, true);
}

void oracle_field_advance(const oracle_config* cfg, double* E, double* B,
                          const double* J) {
  Grid g(*cfg);
  field_advance_impl(g, E, B, J);
}

void oracle_step(const oracle_config* cfg, int64_t np, double* X, double* u,
                 const double* q, int8_t* alive, double* E, double* B,
                 double* J, int32_t nsteps, int32_t nthreads) {
  Grid g(*cfg);
  for (int s = 0; s < nsteps; ++s) {
    if (nthreads > 1)
      push_deposit_threads(g, np, X, u, q, alive, E, B, J, nthreads);
    else
      push_deposit_impl(g, np, X, u, q, alive, E, B, J);
    field_advance_impl(g, E, B, J);
  }
}

void oracle_step_jvp(const oracle_config* cfg, int64_t np, double* X,
                     double* dX, double* u, double* du, const double* q,
                     int8_t* alive, double* E, double* dE, double* B,
                     double* dB, double* J, double* dJ, int32_t nsteps) {
  Grid g(*cfg);
  const size_t nf = 3 * (size_t)g.ncell(), npart = 3 * (size_t)np;
  std::vector<Dual> Xd = to_dual(X, dX, npart), ud = to_dual(u, du, npart);
  std::vector<Dual> Ed = to_dual(E, dE, nf), Bd = to_dual(B, dB, nf);
  std::vector<Dual> Jd = to_dual(J, dJ, nf);
  step_impl(g, np, Xd.data(), ud.data(), q, alive, Ed.data(), Bd.data(), Jd.data(),
            nsteps);
  from_dual(Xd, X, dX);
  from_dual(ud, u, du);
  from_dual(Ed, E, dE);
  from_dual(Bd, B, dB);
  from_dual(Jd, J, dJ);
}

void oracle_deposit_rho(const oracle_config* cfg, int64_t np, const double* X,
                        const double* q, const int8_t* alive, double* rho) {
  Grid g(*cfg);
  std::fill(rho, rho + g.ncell(), 0.0);
  const int m = g.order + 1;
  for (long p = 0; p < np; ++p) {
    if (!alive[p]) continue;
    long base[3] = {0, 0, 0};
    double w[3][5] = {{1, 0, 0, 0, 0}, {1, 0, 0, 0, 0}, {1, 0, 0, 0, 0}};
    int cnt[3] = {1, 1, 1};
    for (int d = 0; d < g.dims; ++d) {
      base[d] = stencil_base(g.order, X[3 * p + d]);
      shape_on_base(g.order, X[3 * p + d], base[d], w[d]);
      cnt[d] = m;
    }
    for (int k = 0; k < cnt[2]; ++k) {
      long kk = g.axis_index(2, base[2] + k, 0);
      if (kk < 0) continue;
      for (int j = 0; j < cnt[1]; ++j) {
        long jj = g.axis_index(1, base[1] + j, 0);
        if (jj < 0) continue;
        for (int i = 0; i < cnt[0]; ++i) {
          long ii = g.axis_index(0, base[0] + i, 0);
          if (ii < 0) continue;
          rho[g.idx(ii, jj, kk)] += q[p] * w[0][i] * w[1][j] * w[2][k];
        }
      }
    }
  }
}

void oracle_divergence(const oracle_config* cfg, const double* V, double* out) {
  Grid g(*cfg);
  const long nc = g.ncell();
  for (long k = 0; k < g.n[2]; ++k)
    for (long j = 0; j < g.n[1]; ++j)
      for (long i = 0; i < g.n[0]; ++i) {
        long L[3] = {i, j, k};
        bool interior = true;
        for (int d = 0; d < g.dims; ++d)
          if (g.open(d) && (L[d] == 0 || L[d] == g.n[d] - 1)) interior = false;
        double s = 0.0;
        if (interior) {
          for (int d = 0; d < g.dims; ++d) {
            long M[3] = {i, j, k};
            M[d] -= 1;
            long ii = g.axis_index(0, M[0], stag_e(d, 0));
            long jj = g.axis_index(1, M[1], stag_e(d, 1));
            long kk = g.axis_index(2, M[2], stag_e(d, 2));
            s += (V[d * nc + g.idx(i, j, k)] - V[d * nc + g.idx(ii, jj, kk)]) / g.dx[d];
          }
        }
        out[g.idx(i, j, k)] = s;
      }
}

void oracle_energies(const oracle_config* cfg, int64_t np, const double* u,
                     const double* q, const int8_t* alive, const double* E,
                     const double* B, double* w_field, double* w_kin) {
  Grid g(*cfg);
  const long nc = g.ncell();
  const double dV = g.cell_volume();
  double wf = 0.0;
  for (int c = 0; c < 3; ++c) {
    int se[3] = {stag_e(c, 0), stag_e(c, 1), stag_e(c, 2)};
    int sb[3] = {stag_b(c, 0), stag_b(c, 1), stag_b(c, 2)};
    for (long k = 0; k < g.n[2]; ++k)
      for (long j = 0; j < g.n[1]; ++j)
        for (long i = 0; i < g.n[0]; ++i) {
          long s = c * nc + g.idx(i, j, k);
          if (slot_inside(g, se, i, j, k)) wf += E[s] * E[s];
          if (slot_inside(g, sb, i, j, k)) wf += B[s] * B[s];
        }
  }
  double wk = 0.0;
  for (long p = 0; p < np; ++p) {
    if (!alive[p]) continue;
    const double* up = u + 3 * p;
    double gam = std::sqrt(1.0 + up[0] * up[0] + up[1] * up[1] + up[2] * up[2]);
    wk += std::fabs(q[p] / g.qm) * (gam - 1.0);  // macro-particle mass density
  }
  *w_field = 0.5 * wf * dV;
  *w_kin = wk * dV;
}

void oracle_curl_e(const oracle_config* cfg, const double* E, double* out) {
  Grid g(*cfg);
  const long nc = g.ncell();
  for (int c = 0; c < 3; ++c) {
    int sb[3] = {stag_b(c, 0), stag_b(c, 1), stag_b(c, 2)};
    for (long k = 0; k < g.n[2]; ++k)
      for (long j = 0; j < g.n[1]; ++j)
        for (long i = 0; i < g.n[0]; ++i)
          out[c * nc + g.idx(i, j, k)] =
              slot_inside(g, sb, i, j, k) ? curl_e_at(g, E, c, i, j, k) : 0.0;
  }
}

void oracle_curl_b(const oracle_config* cfg, const double* B, double* out) {
  Grid g(*cfg);
  const long nc = g.ncell();
  for (int c = 0; c < 3; ++c) {
    int se[3] = {stag_e(c, 0), stag_e(c, 1), stag_e(c, 2)};
    for (long k = 0; k < g.n[2]; ++k)
      for (long j = 0; j < g.n[1]; ++j)
        for (long i = 0; i < g.n[0]; ++i)
          out[c * nc + g.idx(i, j, k)] =
              slot_inside(g, se, i, j, k) ? curl_b_at(g, B, c, i, j, k) : 0.0;
  }
}

}  // extern "C"
