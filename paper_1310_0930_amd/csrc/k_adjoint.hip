// Hand-written adjoint (vector-Jacobian product) of one gather + Boris push +
// move + split + Esirkepov deposit pass: one thread per particle in global
// memory, or in 2D out of LDS per tile of sorted particles.
//
// Given the adjoints of the step's outputs -- lamX^{n+1} (positions, in cell
// units), lamU^{n+1/2} (momenta) and lamJ^{n+1/2} (the current, produced by
// the transpose of the field advance) -- each thread recomputes its particle's
// forward pass from the state at step n and propagates the adjoints back:
// through the charge-conserving deposit (segment end points as functions of
// the path's ends and of the crossing fractions f = (P - X0)/(X1 - X0)),
// the move X1 = X0 + dt u/(gamma dx), the Boris rotation and the gather,
// whose transpose scatters lamE^n, lamB^n (atomics).  The result
// overwrites lamX, lamU with their values at step n and adds to lamE, lamB.
// The map is differentiated along the branch the forward takes (cell and
// piece choices, crossing structure), where it is smooth.
#include "k_particle.h"

namespace pic {

// d w_i / d xi of the order-n weights of one piece.
template <int ORDER, typename R>
__device__ __forceinline__ void shape_deriv(R xi, R* d) {
  if (ORDER == 1) {
    d[0] = R(-1);
    d[1] = R(1);
  } else if (ORDER == 2) {
    d[0] = xi - R(0.5);
    d[1] = R(-2) * xi;
    d[2] = R(0.5) + xi;
  } else if (ORDER == 3) {
    const R s = R(1) - xi;
    d[0] = R(-0.5) * s * s;
    d[1] = xi * (R(1.5) * xi - R(2));
    d[2] = R(0.5) + xi - R(1.5) * xi * xi;
    d[3] = R(0.5) * xi * xi;
  } else {
    const R a = R(1) - R(2) * xi, b = R(1) + R(2) * xi;
    d[0] = R(-1.0 / 48.0) * a * a * a;
    d[1] = R(1.0 / 96.0) * (R(-44) + xi * (R(48) + xi * (R(48) - R(64) * xi)));
    d[2] = xi * (R(-1.25) + xi * xi);
    d[3] = R(1.0 / 96.0) * (R(44) + xi * (R(48) + xi * (R(-48) - R(64) * xi)));
    d[4] = R(1.0 / 48.0) * b * b * b;
  }
}

// Global sample index of component comp (0..2 E/J-like, 3..5 B-like) at
// lattice (x, y, z); -1 outside the domain of an open axis.
template <typename R>
__device__ __forceinline__ int sample_index(const KParams<R>& P, int dims, bool isb, int c, int x,
                                            int y, int z) {
  const int sx = isb ? (c != 0) : (c == 0);
  const int sy = isb ? (c != 1) : (c == 1);
  const int sz = isb ? (c != 2) : (c == 2);
  const int ix = axis_slot(x, P.n[0], P.bc[0] == PIC_BC_OPEN, sx);
  const int iy = axis_slot(y, P.n[1], P.bc[1] == PIC_BC_OPEN, sy);
  const int iz = dims == 3 ? axis_slot(z, P.n[2], P.bc[2] == PIC_BC_OPEN, sz) : 0;
  if (ix < 0 || iy < 0 || iz < 0) return -1;
  return ix + P.n[0] * (iy + P.n[1] * iz);
}

// Sample access of the adjoint helpers, at lattice coordinates: E^n/B^n
// (read), lamE/lamB (added to) and lamJ (read).  AdjGlobal goes to the
// global arrays with the domain's wrap and open faces; AdjLds to a tile's
// LDS regions (coordinates relative to the tile origin), the lamE/lamB
// region accumulating in double.
template <int DIMS, typename R>
struct AdjGlobal {
  const KParams<R>& P;
  const DFields<R>& F;
  R* const* lamE;
  R* const* lamB;
  R* const* lamJ;
  // adds v to the adjoint of sample (isb, c, x, y, z) and returns the field there
  __device__ __forceinline__ R field_add(bool isb, int c, int x, int y, int z, R v) const {
    const int g = sample_index<R>(P, DIMS, isb, c, x, y, z);
    if (g < 0) return R(0);
    atomicAdd(&(isb ? lamB : lamE)[c][g], v);
    return (isb ? F.B : F.E)[c][g];
  }
  __device__ __forceinline__ R lamj(int c, int x, int y, int z) const {
    const int g = sample_index<R>(P, DIMS, false, c, x, y, z);
    return g < 0 ? R(0) : lamJ[c][g];
  }
};

// Region of one workgroup of the LDS adjoint: the push tile, cut along z
// into S slabs when the three regions (E/B and lamJ in the working
// precision, lamE/lamB in double) of a whole 3D tile exceed a CU's LDS.
// Each slab keeps the tile's drift allowance and stencil reach; x and y are
// the tile's.  `fits` is false where even one-cell slabs do not fit (cubic
// in double precision), and that form keeps the global-memory kernel.
template <int DIMS, int ORDER, typename R>
struct AdjGeo : Geo<DIMS, ORDER, R> {
  using B = Geo<DIMS, ORDER, R>;
  using Rc = typename B::Rc;
  static constexpr size_t bytes(int tz) {
    return (sizeof(R) * 6 + sizeof(double) * 6) * (size_t)(B::ex * B::ex * (tz + 2 * B::AZ + Rc::g_hi - Rc::g_lo)) +
           sizeof(R) * 3 * (size_t)(B::jx * B::jx * (tz + 2 * B::AZ + Rc::d_hi - Rc::d_lo));
  }
  static constexpr size_t LDS_MAX = 160 * 1024;
  // 2D: several workgroups share a CU; 3D: one per CU, 8 wavefronts of up
  // to 256 VGPRs
  static constexpr int NT = DIMS == 2 ? 256 : 512;
  // with several slabs each wavefront queues the particles of its slab:
  // 128 indices per wavefront
  static constexpr int QCAP = 128;
  static constexpr size_t queue_bytes = sizeof(int) * QCAP * (NT / 64);
  static constexpr int pick() {
    if (DIMS == 2) return 1;
    for (int s = 1; s <= B::TZ; s *= 2)
      if (B::TZ % s == 0 && bytes(B::TZ / s) + (s > 1 ? queue_bytes : 0) <= LDS_MAX) return s;
    return 0;
  }
  static constexpr int S = pick();
  static constexpr bool fits = S > 0;
  static constexpr int TZ = fits ? B::TZ / S : 1;
  static constexpr int ez = DIMS == 3 ? TZ + 2 * B::AZ + Rc::g_hi - Rc::g_lo : 1;
  static constexpr int e_vol = B::ex * B::ex * ez;
  static constexpr int jz = DIMS == 3 ? TZ + 2 * B::AZ + Rc::d_hi - Rc::d_lo : 1;
  static constexpr int j_vol = B::jx * B::jx * jz;
};

template <int DIMS, int ORDER, typename R, class G>
struct AdjLds {
  const R* eb;   // E^n (0..2), B^n (3..5) over the field region
  const R* lj;   // lamJ over the current region
  double* leb;   // lamE (0..2), lamB (3..5) over the field region
  __device__ __forceinline__ R field_add(bool isb, int c, int x, int y, int z, R v) const {
    const int i = (DIMS == 3 ? (z - G::e_lo_z) * G::ex : 0) * G::ex + (y - G::e_lo) * G::ex +
                  (x - G::e_lo) + (isb ? 3 + c : c) * G::e_vol;
    atomicAdd(&leb[i], (double)v);
    return eb[i];
  }
  __device__ __forceinline__ R lamj(int c, int x, int y, int z) const {
    return lj[(DIMS == 3 ? (z - G::j_lo_z) * G::jx : 0) * G::jx + (y - G::j_lo) * G::jx +
              (x - G::j_lo) + c * G::j_vol];
  }
};

// Transpose of the gather: lamF[node] += w lamFp for every stencil node and
// lamX += sum (dw/dX) F lamFp.
template <int DIMS, int ORDER, typename R, class Acc>
__device__ __forceinline__ void gather_vjp(const Acc& ac, const int* c3, const R* o, const R* lEp,
                                           const R* lBp, R* lX) {
  constexpr int M = ORDER + 1;
  constexpr int MZ = DIMS == 3 ? M : 1;
  R wn[3][M], ws[3][M], dn[3][M], dsg[3][M];
  int bn[3] = {0, 0, 0}, bs[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int i = 0; i < M; ++i) wn[d][i] = ws[d][i] = dn[d][i] = dsg[d][i] = R(0);
#pragma unroll
  for (int d = 0; d < DIMS; ++d) {
    R xi;
    bn[d] = piece_node<ORDER>(o[d], xi) - ORDER / 2;
    shape<ORDER>(xi, wn[d]);
    shape_deriv<ORDER>(xi, dn[d]);
    bs[d] = piece_stag<ORDER>(o[d], xi) - ORDER / 2;
    shape<ORDER>(xi, ws[d]);
    shape_deriv<ORDER>(xi, dsg[d]);
  }
  if (DIMS == 2) {
    wn[2][0] = ws[2][0] = R(1);
  }
  for (int comp = 0; comp < 6; ++comp) {
    const bool isb = comp >= 3;
    const int c = isb ? comp - 3 : comp;
    const R lam = isb ? lBp[c] : lEp[c];
    const R(*w[3])[M];
    const R(*dw[3])[M];
    int b[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const bool st = isb ? (d != c) : (d == c);
      w[d] = st ? &ws[d] : &wn[d];
      dw[d] = st ? &dsg[d] : &dn[d];
      b[d] = st ? bs[d] : bn[d];
    }
    for (int k = 0; k < MZ; ++k)
      for (int j = 0; j < M; ++j)
        for (int i = 0; i < M; ++i) {
          const R wx = (*w[0])[i], wy = (*w[1])[j], wz = (*w[2])[k];
          const R fl = ac.field_add(isb, c, c3[0] + b[0] + i, c3[1] + b[1] + j, c3[2] + b[2] + k,
                                    wx * wy * wz * lam) *
                       lam;
          lX[0] += (*dw[0])[i] * wy * wz * fl;
          lX[1] += wx * (*dw[1])[j] * wz * fl;
          if (DIMS == 3) lX[2] += wx * wy * (*dw[2])[k] * fl;
        }
  }
}

// Transpose of the Boris step u -> u' under (Ep, Bp), recomputing its
// intermediates: in lamU' ; out lamU, lamEp, lamBp.
template <typename R>
__device__ __forceinline__ void boris_vjp(R hqm, const R* u, const R* E, const R* B, const R* lu1,
                                          R* lu, R* lE, R* lB) {
  R um[3], t[3], s[3], up[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) um[c] = u[c] + hqm * E[c];
  const R gm = sqrt(R(1) + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  const R hg = hqm / gm;
#pragma unroll
  for (int c = 0; c < 3; ++c) t[c] = hg * B[c];
  const R tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  const R f = R(2) / (R(1) + tt);
#pragma unroll
  for (int c = 0; c < 3; ++c) s[c] = f * t[c];
  up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
  up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
  up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
  // u' = uq + hqm E, uq = um + up x s
  R luq[3], lum[3], lup[3], ls[3], lt[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    luq[c] = lu1[c];
    lE[c] = hqm * lu1[c];
    lum[c] = luq[c];
  }
  // c = a x b: lam_a = b x lam_c, lam_b = lam_c x a
  lup[0] = s[1] * luq[2] - s[2] * luq[1];
  lup[1] = s[2] * luq[0] - s[0] * luq[2];
  lup[2] = s[0] * luq[1] - s[1] * luq[0];
  ls[0] = luq[1] * up[2] - luq[2] * up[1];
  ls[1] = luq[2] * up[0] - luq[0] * up[2];
  ls[2] = luq[0] * up[1] - luq[1] * up[0];
  // up = um + um x t
#pragma unroll
  for (int c = 0; c < 3; ++c) lum[c] += lup[c];
  lum[0] += t[1] * lup[2] - t[2] * lup[1];
  lum[1] += t[2] * lup[0] - t[0] * lup[2];
  lum[2] += t[0] * lup[1] - t[1] * lup[0];
  lt[0] = lup[1] * um[2] - lup[2] * um[1];
  lt[1] = lup[2] * um[0] - lup[0] * um[2];
  lt[2] = lup[0] * um[1] - lup[1] * um[0];
  // s = f t, f = 2/(1 + t.t)
  const R lf = ls[0] * t[0] + ls[1] * t[1] + ls[2] * t[2];
  const R ltt = R(-0.5) * f * f * lf;
#pragma unroll
  for (int c = 0; c < 3; ++c) lt[c] += f * ls[c] + R(2) * t[c] * ltt;
  // t = (hqm/gm) B
  R bl = R(0);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    lB[c] = hg * lt[c];
    bl += B[c] * lt[c];
  }
  const R lgm = -hg / gm * bl;
  // gm = sqrt(1 + um.um); um = u + hqm E
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    lum[c] += um[c] / gm * lgm;
    lu[c] = lum[c];
    lE[c] += hqm * lum[c];
  }
}

// Transpose of the Esirkepov deposit of one segment: gathers lamJ over the
// segment's stencil and returns lam(xa), lam(xb) per axis and lam(fz).
template <int DIMS, int ORDER, typename R, class Acc>
__device__ __forceinline__ void deposit_segment_vjp(const KParams<R>& P, const Acc& ac,
                                                    const int* c3, const int* base, const R* xa,
                                                    const R* xb, R q, R fz, R* lxa, R* lxb,
                                                    R& lfz) {
  constexpr int M = ORDER + 1;
  constexpr int MZ = DIMS == 3 ? M : 1;
  R S0[3][M], dS[3][M], Sm[3][M], d12[3][M];
  R lS0[3][M], ldS[3][M], lSm[3][M], ld12[3][M];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int i = 0; i < M; ++i) {
      S0[d][i] = dS[d][i] = Sm[d][i] = d12[d][i] = R(0);
      lS0[d][i] = ldS[d][i] = lSm[d][i] = ld12[d][i] = R(0);
    }
#pragma unroll
  for (int d = 0; d < DIMS; ++d) {
    shape<ORDER>(xa[d], S0[d]);
    dshape<ORDER>(xa[d], xb[d], dS[d]);
#pragma unroll
    for (int i = 0; i < M; ++i) {
      Sm[d][i] = S0[d][i] + R(0.5) * dS[d][i];
      d12[d][i] = R(1.0 / 12.0) * dS[d][i];
    }
  }
  lfz = R(0);
  auto lam_at = [&](int comp, int i, int j, int k) -> R {
    return ac.lamj(comp, c3[0] + base[0] + i, c3[1] + base[1] + j, c3[2] + base[2] + k);
  };
  (void)MZ;
  if (DIMS == 3) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int a = (c + 1) % 3, b = (c + 2) % 3;
      const R qj = q * P.jfac[c];
      R Pc[ORDER], lP[ORDER];
      R run = R(0);
#pragma unroll
      for (int i = 0; i < ORDER; ++i) {
        run += dS[c][i];
        Pc[i] = qj * run;
        lP[i] = R(0);
      }
#pragma unroll
      for (int ib = 0; ib < M; ++ib)
#pragma unroll
        for (int ia = 0; ia < M; ++ia) {
          const R A = Sm[a][ia] * Sm[b][ib] + d12[a][ia] * dS[b][ib];
          R lA = R(0);
#pragma unroll
          for (int ic = 0; ic < ORDER; ++ic) {
            int L[3];
            L[c] = ic;
            L[a] = ia;
            L[b] = ib;
            const R g = lam_at(c, L[0], L[1], L[2]);
            lA += g * Pc[ic];
            lP[ic] += g * A;
          }
          lSm[a][ia] += lA * Sm[b][ib];
          lSm[b][ib] += lA * Sm[a][ia];
          ld12[a][ia] += lA * dS[b][ib];
          ldS[b][ib] += lA * d12[a][ia];
        }
      // P_c[ic] = qj * sum_{i <= ic} dS_c[i]
      R acc = R(0);
#pragma unroll
      for (int i = ORDER - 1; i >= 0; --i) {
        acc += lP[i];
        ldS[c][i] += qj * acc;
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int a = 1 - c;
      const R qj = q * P.jfac[c];
      R Pc[ORDER], lP[ORDER];
      R run = R(0);
#pragma unroll
      for (int i = 0; i < ORDER; ++i) {
        run += dS[c][i];
        Pc[i] = qj * run;
        lP[i] = R(0);
      }
#pragma unroll
      for (int ia = 0; ia < M; ++ia)
#pragma unroll
        for (int ic = 0; ic < ORDER; ++ic) {
          int L[2];
          L[c] = ic;
          L[a] = ia;
          const R g = lam_at(c, L[0], L[1], 0);
          lSm[a][ia] += g * Pc[ic];
          lP[ic] += g * Sm[a][ia];
        }
      R acc = R(0);
#pragma unroll
      for (int i = ORDER - 1; i >= 0; --i) {
        acc += lP[i];
        ldS[c][i] += qj * acc;
      }
    }
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
      for (int i = 0; i < M; ++i) {
        const R g = lam_at(2, i, j, 0);
        const R W = Sm[0][i] * Sm[1][j] + d12[0][i] * dS[1][j];
        lfz += g * W;
        lSm[0][i] += g * fz * Sm[1][j];
        lSm[1][j] += g * fz * Sm[0][i];
        ld12[0][i] += g * fz * dS[1][j];
        ldS[1][j] += g * fz * d12[0][i];
      }
  }
  // Sm = S0 + dS/2, d12 = dS/12, S0 = S(xa), dS = S(xb) - S(xa)
#pragma unroll
  for (int d = 0; d < DIMS; ++d) {
    R da[M], db[M];
    shape_deriv<ORDER>(xa[d], da);
    shape_deriv<ORDER>(xb[d], db);
    R la = R(0), lb = R(0);
#pragma unroll
    for (int i = 0; i < M; ++i) {
      lS0[d][i] += lSm[d][i];
      ldS[d][i] += R(0.5) * lSm[d][i] + R(1.0 / 12.0) * ld12[d][i];
      la += (lS0[d][i] - ldS[d][i]) * da[i];
      lb += ldS[d][i] * db[i];
    }
    lxa[d] = la;
    lxb[d] = lb;
  }
}

// Transpose of the whole split deposit: lamX0, lamX1 (cell units, relative
// to the old cell) and lam(vz) for the 2D out-of-plane current.
template <int DIMS, int ORDER, typename R, class Acc>
__device__ __forceinline__ void deposit_vjp(const KParams<R>& P, const Acc& ac, const int* c3,
                                            const R* o0, const int* sh, const R* o1, R q, R vz,
                                            R* lX0, R* lX1, R& lvz) {
  Split<DIMS, R> S;
  split_path<DIMS, ORDER, R>(S, o0, sh, o1);
  R lt[DIMS + 2];
#pragma unroll
  for (int j = 0; j < DIMS + 2; ++j) lt[j] = R(0);
  lvz = R(0);
  for (int s = 0; s <= S.m; ++s) {
    R xa[3], xb[3], ft, lxa[3], lxb[3], lfz;
    int base[3];
    segment_ends<DIMS, ORDER, R>(S, s, xa, xb, base, ft);
    deposit_segment_vjp<DIMS, ORDER, R>(P, ac, c3, base, xa, xb, q, q * vz * ft, lxa, lxb, lfz);
    R ta = R(0), tbb = R(1);
#pragma unroll
    for (int j = 0; j < DIMS + 2; ++j) {
      if (j == s) ta = S.tb[j];
      if (j == s + 1) tbb = S.tb[j];
    }
    // xa = X0 + ta (X1 - X0), xb = X0 + tb (X1 - X0) (up to the piece shift)
    R la = R(0), lb = R(0);
#pragma unroll
    for (int d = 0; d < DIMS; ++d) {
      lX0[d] += lxa[d] * (R(1) - ta) + lxb[d] * (R(1) - tbb);
      lX1[d] += lxa[d] * ta + lxb[d] * tbb;
      la += lxa[d] * S.dl[d];
      lb += lxb[d] * S.dl[d];
    }
    // fz = q vz (tb - ta)
    lvz += lfz * q * (tbb - ta);
    la -= lfz * q * vz;
    lb += lfz * q * vz;
#pragma unroll
    for (int j = 0; j < DIMS + 2; ++j) {
      if (j == s) lt[j] += la;
      if (j == s + 1) lt[j] += lb;
    }
  }
  // crossing fractions f_d = (P_d - X0_d)/(X1_d - X0_d)
#pragma unroll
  for (int d = 0; d < DIMS; ++d) {
    if (!S.cr[d]) continue;
    R l = R(0), f = R(0);
#pragma unroll
    for (int j = 1; j <= DIMS; ++j)
      if (j == S.jd[d]) {
        l = lt[j];
        f = S.tb[j];
      }
    lX0[d] += l * (f - R(1)) / S.dl[d];
    lX1[d] += l * (-f) / S.dl[d];
  }
}

// Forward pass of one particle kept for its adjoint: the gather, the Boris
// push and the move (state s becomes step n+1's, u0 keeps u^{n-1/2}).
template <typename R>
struct FwdPart {
  R Ep[3], Bp[3], u0[3], o1[3], vz;
  int sh[3];
  bool small;
};

template <int DIMS, int ORDER, typename R, class FAcc>
__device__ __forceinline__ bool forward_part(const KParams<R>& P, const FAcc& acc, PState<R>& s,
                                             FwdPart<R>& f, DevFlags* flg) {
  gather<DIMS, ORDER, R>(acc, s.o, f.Ep, f.Bp);
#pragma unroll
  for (int c = 0; c < 3; ++c) f.u0[c] = s.u[c];
  return push_move<DIMS, R>(P, s, f.Ep, f.Bp, f.sh, f.o1, f.vz, f.small, flg);
}

// Adjoint of one particle's step from its forward pass; c3 are the cell's
// coordinates in the accessor's frame.  Reads lam at slot p (adjoints of
// x^{n+1}, u^{n+1/2}) and overwrites it with those of x^n, u^{n-1/2}.
template <int DIMS, int ORDER, typename R, class Acc>
__device__ __forceinline__ void adjoint_part(const KParams<R>& P, const Acc& ac, const int* c3,
                                             const PState<R>& s0, const PState<R>& s1,
                                             const FwdPart<R>& f, const DParts<R>& lam, int p) {
  const R u1[3] = {s1.u[0], s1.u[1], s1.u[2]};
  const R gam = sqrt(R(1) + u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
  // adjoints arriving from step n+1
  R lX1[3] = {R(0), R(0), R(0)}, lX0[3] = {R(0), R(0), R(0)}, lu1[3];
#pragma unroll
  for (int d = 0; d < DIMS; ++d) lX1[d] = lam.off[d][p];
#pragma unroll
  for (int c = 0; c < 3; ++c) lu1[c] = lam.u[c][p];
  // deposit
  R lvz;
  deposit_vjp<DIMS, ORDER, R>(P, ac, c3, s0.o, f.sh, f.o1, s0.q, f.vz, lX0, lX1, lvz);
  // move: X1 = X0 + dt/dx u/gamma, vz = u_z/gamma
  R ld[3] = {R(0), R(0), R(0)};
  R dot = R(0);
#pragma unroll
  for (int d = 0; d < DIMS; ++d) {
    lX0[d] += lX1[d];
    ld[d] = lX1[d] * P.dtdx[d];
    dot += ld[d] * u1[d];
  }
  dot += lvz * u1[2];
  const R ig = R(1) / gam, ig3 = ig * ig * ig;
#pragma unroll
  for (int c = 0; c < 3; ++c) lu1[c] += (ld[c] + (c == 2 ? lvz : R(0))) * ig - u1[c] * ig3 * dot;
  // Boris
  R lu0[3], lEp[3], lBp[3];
  boris_vjp<R>(P.hqm, f.u0, f.Ep, f.Bp, lu1, lu0, lEp, lBp);
  // gather
  gather_vjp<DIMS, ORDER, R>(ac, c3, s0.o, lEp, lBp, lX0);
#pragma unroll
  for (int d = 0; d < DIMS; ++d) lam.off[d][p] = lX0[d];
#pragma unroll
  for (int c = 0; c < 3; ++c) lam.u[c][p] = lu0[c];
}

// One thread per particle, everything in global memory: all particles, or
// (list != NULL) the flg->ndefer particles of the list followed by those
// from *tail on (the particles no tile covers).
template <int DIMS, int ORDER, typename R>
__global__ void __launch_bounds__(256) k_push_deposit_adjoint(KParams<R> P, DParts<R> pa,
                                                              DFields<R> F, DFields<R> L,
                                                              DParts<R> lam, DevFlags* flg,
                                                              int np, const int* list,
                                                              const int* tail) {
  const int open0 = P.bc[0] == PIC_BC_OPEN, open1 = P.bc[1] == PIC_BC_OPEN;
  const int open2 = DIMS == 3 && P.bc[2] == PIC_BC_OPEN;
  const int nl = list ? (int)flg->ndefer : 0;
  const int t0 = list ? *tail : 0;
  const int n = nl + (np - t0);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int p = t < nl ? list[t] : t0 + (t - nl);
    PState<R> s = load_particle<DIMS, R>(pa, p, P.q_const);
    if (s.cl < 0) continue;
    int c3[3];
    if (!decode<DIMS, R>(P, s, c3, flg)) continue;
    GlobalFields<R> acc{F.E, F.B, c3[0], c3[1], c3[2], P.n[0], P.n[1], P.n[2],
                        open0, open1, open2, DIMS};
    const PState<R> s0 = s;
    FwdPart<R> f;
    if (!forward_part<DIMS, ORDER, R>(P, acc, s, f, flg)) continue;
    AdjGlobal<DIMS, R> ac{P, F, L.E, L.B, L.J};
    adjoint_part<DIMS, ORDER, R>(P, ac, c3, s0, s, f, lam, p);
  }
}

// The same out of LDS, one workgroup per tile of sorted particles, or per z
// slab of one in 3D (AdjGeo): E^n, B^n and lamJ of the region are staged,
// lamE/lamB accumulate in double in LDS and are added to the global arrays
// once.  Every slab reads all of its tile's particles and takes those whose
// cell is in the slab, the first and last slabs also the allowance below
// and above the tile.  Particles outside the tile's drift allowance, or
// moving half a cell or more, go to the list for the global-memory kernel
// (entered by the first slab alone).
template <int DIMS, int ORDER, typename R>
__global__ void __launch_bounds__((AdjGeo<DIMS, ORDER, R>::NT)) k_pda_tile(
    KParams<R> P, DParts<R> pa, DFields<R> F, DFields<R> L, DParts<R> lam,
    const int* __restrict__ starts, int* __restrict__ deferred, DevFlags* flg) {
  using G = AdjGeo<DIMS, ORDER, R>;
  constexpr int S = G::S;
  __shared__ R s_eb[6 * G::e_vol];
  __shared__ R s_lj[3 * G::j_vol];
  __shared__ double s_leb[6 * G::e_vol];
  const int grp = blockIdx.x >> 3;
  const int tile = (blockIdx.x & 7) * P.per_xcd + grp / S;
  const int slab = grp % S;
  if (tile >= P.ntiles) return;
  const int pbeg = starts[tile], pend = starts[tile + 1];
  if (pbeg == pend) return;
  int org[3];
  tile_origin<DIMS, ORDER, R>(P, tile, org);
  const int torg2 = org[2];
  org[2] += slab * G::TZ;
  const int open0 = P.bc[0] == PIC_BC_OPEN, open1 = P.bc[1] == PIC_BC_OPEN;
  const int open2 = DIMS == 3 && P.bc[2] == PIC_BC_OPEN;
  const int str1 = P.n[0], str2 = P.n[0] * P.n[1];
  {
    constexpr int NR = (G::e_vol + G::NT - 1) / G::NT;
    R stage[NR][6];
    stage_load<DIMS, ORDER, R, NR, G>(P, F, org, stage);
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int r = threadIdx.x + k * G::NT;
      if (r < G::e_vol) {
#pragma unroll
        for (int c = 0; c < 6; ++c) s_eb[c * G::e_vol + r] = stage[k][c];
      }
    }
  }
  for (int r = threadIdx.x; r < G::j_vol; r += G::NT) {  // lamJ_c, staggered along c
    const int lx = r % G::jx, ly = (r / G::jx) % G::jx, lz = r / (G::jx * G::jx);
    int sx[2], sy[2], sz[2] = {0, 0};
    axis_slots(org[0] + G::j_lo + lx, P.n[0], open0, 1, sx);
    axis_slots(org[1] + G::j_lo + ly, P.n[1], open1, str1, sy);
    if (DIMS == 3) axis_slots(org[2] + G::j_lo_z + lz, P.n[2], open2, str2, sz);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int ix = sx[c == 0], iy = sy[c == 1], iz = sz[c == 2];
      s_lj[c * G::j_vol + r] = (ix >= 0 && iy >= 0 && iz >= 0) ? L.J[c][ix + iy + iz] : R(0);
    }
  }
  for (int i = threadIdx.x; i < 6 * G::e_vol; i += G::NT) s_leb[i] = 0.0;
  __syncthreads();
  const AdjLds<DIMS, ORDER, R, G> ac{s_eb, s_lj, s_leb};
  if constexpr (S == 1) {
    for (int p = pbeg + threadIdx.x; p < pend; p += G::NT) {
      PState<R> s = load_particle<DIMS, R>(pa, p, P.q_const);
      if (s.cl < 0) continue;
      int c3[3] = {0, 0, 0};
      if (!decode<DIMS, R>(P, s, c3, flg)) continue;
      const int tor[3] = {org[0], org[1], torg2};
      int l[3] = {0, 0, 0};
      bool fast = true;
#pragma unroll
      for (int d = 0; d < DIMS; ++d) {
        const int Td = d == 2 ? G::B::TZ : G::T;
        const int Ad = d == 2 ? G::AZ : G::A;
        int v = c3[d] - tor[d];
        if (P.bc[d] == PIC_BC_PERIODIC) {
          v = v < 0 ? v + P.n[d] : v;
          if (v >= Td + Ad) v -= P.n[d];
        }
        l[d] = v;
        fast = fast && v >= -Ad && v < Td + Ad;
      }
      if (!fast) {
        if (slab == 0) deferred[atomicAdd(&flg->ndefer, 1u)] = p;
        continue;
      }
      LdsFields<DIMS, ORDER, R, G> acc{
          (lds_ptr<const R>)s_eb, ((l[2] - G::e_lo_z) * G::ex + (l[1] - G::e_lo)) * G::ex + (l[0] - G::e_lo)};
      const PState<R> s0 = s;
      FwdPart<R> f;
      if (!forward_part<DIMS, ORDER, R>(P, acc, s, f, flg)) continue;
      if (!f.small) {
        deferred[atomicAdd(&flg->ndefer, 1u)] = p;
        continue;
      }
      adjoint_part<DIMS, ORDER, R>(P, ac, l, s0, s, f, lam, p);
    }
  } else {
    const int tor[3] = {org[0], org[1], torg2};
    // the cell relative to the tile (periodic fold); false outside the
    // tile's drift allowance
    auto locate = [&](const int* c3, int* l) {
      bool fast = true;
#pragma unroll
      for (int d = 0; d < DIMS; ++d) {
        const int Td = d == 2 ? G::B::TZ : G::T;
        const int Ad = d == 2 ? G::AZ : G::A;
        int v = c3[d] - tor[d];
        if (P.bc[d] == PIC_BC_PERIODIC) {
          v = v < 0 ? v + P.n[d] : v;
          if (v >= Td + Ad) v -= P.n[d];
        }
        l[d] = v;
        fast = fast && v >= -Ad && v < Td + Ad;
      }
      return fast;
    };
    // Every slab scans all of the tile's particles, a slab's share is about
    // 1/S of them: each wavefront queues the indices of its slab's particles
    // (allowance cells below and above the tile go to the end slabs) and
    // runs whole 64-lane batches from the queue's end (at most 63 wait when
    // 64 more arrive, so 128 entries suffice).
    __shared__ int s_own[G::NT / 64][G::QCAP];
    const int lane = threadIdx.x & 63;
    int* q = s_own[threadIdx.x >> 6];
    int qn = 0;  // uniform over the wavefront
    for (int b = pbeg + (threadIdx.x & ~63);; b += G::NT) {
      const bool more = b < pend;
      if (more) {
        const int p = b + lane;
        bool own = false;
        if (p < pend) {
          const PState<R> s = load_particle<DIMS, R>(pa, p, P.q_const);
          int c3[3] = {0, 0, 0};
          if (s.cl >= 0 && decode<DIMS, R>(P, s, c3, flg)) {
            int l[3] = {0, 0, 0};
            if (!locate(c3, l)) {
              if (slab == 0) deferred[atomicAdd(&flg->ndefer, 1u)] = p;
            } else {
              own = (l[2] < 0 ? 0 : (l[2] / G::TZ < S ? l[2] / G::TZ : S - 1)) == slab;
            }
          }
        }
        const unsigned long long m = __ballot(own);
        if (own) q[qn + (int)__popcll(m & ((1ull << lane) - 1ull))] = p;
        qn += (int)__popcll(m);
      }
      if (qn >= 64 || (!more && qn > 0)) {
        __builtin_amdgcn_wave_barrier();
        const int cnt = qn < 64 ? qn : 64;
        const int p = lane < cnt ? q[qn - cnt + lane] : -1;
        __builtin_amdgcn_wave_barrier();
        qn -= cnt;
        if (p >= 0) {
          PState<R> s = load_particle<DIMS, R>(pa, p, P.q_const);
          int c3[3] = {0, 0, 0};
          decode<DIMS, R>(P, s, c3, flg);
          int l[3] = {0, 0, 0};
          locate(c3, l);
          l[2] -= slab * G::TZ;
          LdsFields<DIMS, ORDER, R, G> acc{(lds_ptr<const R>)s_eb,
                                           ((l[2] - G::e_lo_z) * G::ex + (l[1] - G::e_lo)) * G::ex +
                                               (l[0] - G::e_lo)};
          const PState<R> s0 = s;
          FwdPart<R> f;
          if (forward_part<DIMS, ORDER, R>(P, acc, s, f, flg)) {
            if (!f.small)
              deferred[atomicAdd(&flg->ndefer, 1u)] = p;
            else
              adjoint_part<DIMS, ORDER, R>(P, ac, l, s0, s, f, lam, p);
          }
        }
      }
      if (!more) break;
    }
  }
  __syncthreads();
  // lamE, lamB of the region (its halo overlaps the neighbouring regions')
  for (int r = threadIdx.x; r < G::e_vol; r += G::NT) {
    const int lx = r % G::ex, ly = (r / G::ex) % G::ex, lz = r / (G::ex * G::ex);
    int sx[2], sy[2], sz[2] = {0, 0};
    axis_slots(org[0] + G::e_lo + lx, P.n[0], open0, 1, sx);
    axis_slots(org[1] + G::e_lo + ly, P.n[1], open1, str1, sy);
    if (DIMS == 3) axis_slots(org[2] + G::e_lo_z + lz, P.n[2], open2, str2, sz);
#pragma unroll
    for (int c = 0; c < 6; ++c) {  // E_c staggered along c, B_c along the two others
      const int e = c < 3 ? c : c - 3;
      const bool isb = c >= 3;
      const int ix = sx[isb ? (e != 0) : (e == 0)];
      const int iy = sy[isb ? (e != 1) : (e == 1)];
      const int iz = sz[isb ? (e != 2) : (e == 2)];
      const double v = s_leb[c * G::e_vol + r];
      if (v != 0.0 && ix >= 0 && iy >= 0 && iz >= 0) atomicAdd(&(isb ? L.B : L.E)[e][ix + iy + iz], (R)v);
    }
  }
}

__global__ void k_adj_reset(DevFlags* flg) { flg->ndefer = 0u; }

template <int DIMS, int ORDER, typename R>
static int launch_pda(const pic_ctx* ctx, const pic_particles* p, const pic_fields* f,
                      const pic_fields* lf, pic_particles* lp, void* ws, hipStream_t s) {
  KParams<R> P = make_params<R>(ctx);
  WsLayout Lw = ws_layout(ctx, p->np);
  DParts<R> pa, la;
  pa.cell = p->cell;
  la.cell = nullptr;
  for (int d = 0; d < 3; ++d) {
    pa.off[d] = (R*)p->off[d];
    pa.u[d] = (R*)p->u[d];
    la.off[d] = (R*)lp->off[d];
    la.u[d] = (R*)lp->u[d];
  }
  pa.q = (R*)p->q;
  pa.id = nullptr;
  la.q = nullptr;
  la.id = nullptr;
  DFields<R> F, L;
  for (int c = 0; c < 3; ++c) {
    F.E[c] = (R*)f->E[c];
    F.B[c] = (R*)f->B[c];
    F.J[c] = nullptr;
    L.E[c] = (R*)lf->E[c];
    L.B[c] = (R*)lf->B[c];
    L.J[c] = (R*)lf->J[c];
  }
  if (p->np == 0) return 0;
  DevFlags* flg = (DevFlags*)((char*)ws + Lw.flags);
  const long blocks = (p->np + 255) / 256;
  const unsigned gblocks = (unsigned)(blocks < 8192 ? blocks : 8192);
  // the LDS tile path needs tile bins for these np particles in this
  // workspace (any particle order is then handled correctly: a particle
  // outside the allowance of the tile whose range holds it takes the
  // global-memory kernel)
  if constexpr (AdjGeo<DIMS, ORDER, R>::fits) {
    if (ctx->sorted_np == p->np && ctx->sorted_ws == ws) {
      using G = AdjGeo<DIMS, ORDER, R>;
      const int* starts = (const int*)((char*)ws + Lw.starts);
      int* deferred = (int*)((char*)ws + Lw.tmp_cell);
      k_adj_reset<<<dim3(1), dim3(1), 0, s>>>(flg);
      k_pda_tile<DIMS, ORDER, R><<<dim3(8 * P.per_xcd * G::S), dim3(G::NT), 0, s>>>(P, pa, F, L, la,
                                                                            starts, deferred, flg);
      k_push_deposit_adjoint<DIMS, ORDER, R><<<dim3(gblocks), dim3(256), 0, s>>>(
          P, pa, F, L, la, flg, (int)p->np, deferred, starts + P.ntiles);
      return (int)hipGetLastError();
    }
  }
  k_push_deposit_adjoint<DIMS, ORDER, R><<<dim3(gblocks), dim3(256), 0, s>>>(
      P, pa, F, L, la, flg, (int)p->np, nullptr, nullptr);
  return (int)hipGetLastError();
}

int launch_push_deposit_adjoint(const pic_ctx* ctx, const pic_particles* p, const pic_fields* f,
                                const pic_fields* lam_f, pic_particles* lam_p, void* ws,
                                hipStream_t s) {
  const int D = ctx->cfg.dims, O = ctx->cfg.order;
  const bool dbl = ctx->cfg.real_bytes == 8;
#define PIC_PDA(DD, OO)                                                          \
  if (D == DD && O == OO)                                                        \
    return dbl ? launch_pda<DD, OO, double>(ctx, p, f, lam_f, lam_p, ws, s)     \
               : launch_pda<DD, OO, float>(ctx, p, f, lam_f, lam_p, ws, s);
  PIC_PDA(2, 1) PIC_PDA(2, 2) PIC_PDA(2, 3) PIC_PDA(2, 4)
  PIC_PDA(3, 1) PIC_PDA(3, 2) PIC_PDA(3, 3) PIC_PDA(3, 4)
#undef PIC_PDA
  return (int)hipErrorInvalidValue;
}

}  // namespace pic
