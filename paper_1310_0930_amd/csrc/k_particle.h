// Per-particle device routines shared by the push/deposit kernels and their
// adjoint: B-spline pieces and weights, LDS/global accessors, gather, Boris,
// move, trajectory split and the Esirkepov segment deposit.
#pragma once
#include <type_traits>

#include "k_common.h"

namespace pic {

// ------------------------------------------------------------------ shapes
// Piece of the order-n B-spline that holds a node-centred position c + o
// (o in [0,1)), relative to c, and the coordinate xi inside that piece
// (xi in [0,1) for odd orders, [-1/2,1/2) for even orders).  Exact.
template <int ORDER, typename R>
__device__ __forceinline__ int piece_node(R o, R& xi) {
  if (ORDER & 1) {
    xi = o;
    return 0;
  }
  const int k = o >= R(0.5);
  xi = k ? o - R(1) : o;
  return k;
}

// The same for a position half a cell lower (a component staggered along
// the axis): P = o - 1/2.
template <int ORDER, typename R>
__device__ __forceinline__ int piece_stag(R o, R& xi) {
  if (ORDER & 1) {
    const int k = o >= R(0.5) ? 0 : -1;
    xi = k ? o + R(0.5) : o - R(0.5);
    return k;
  }
  xi = o - R(0.5);
  return 0;
}

// B-spline weights of the piece at coordinate xi, on nodes base..base+ORDER
// where base = piece - ORDER/2.
template <int ORDER, typename R>
__device__ __forceinline__ void shape(R xi, R* w) {
  if (ORDER == 1) {
    w[0] = R(1) - xi;
    w[1] = xi;
  } else if (ORDER == 2) {
    const R a = R(0.5) - xi, b = R(0.5) + xi;
    w[0] = R(0.5) * a * a;
    w[1] = R(0.75) - xi * xi;
    w[2] = R(0.5) * b * b;
  } else if (ORDER == 3) {
    const R s = R(1) - xi, t2 = xi * xi, t3 = t2 * xi;
    const R sixth = R(1.0 / 6.0);
    w[0] = sixth * s * s * s;
    w[1] = sixth * (R(4) - R(6) * t2 + R(3) * t3);
    w[2] = sixth * (R(1) + R(3) * xi + R(3) * t2 - R(3) * t3);
    w[3] = sixth * t3;
  } else {  // quartic: xi is the distance to the centre node of the piece
    const R a = R(1) - R(2) * xi, b = R(1) + R(2) * xi;
    const R a2 = a * a, b2 = b * b, t2 = xi * xi;
    w[0] = R(1.0 / 384.0) * a2 * a2;
    w[1] = R(1.0 / 96.0) * (R(19) + xi * (R(-44) + xi * (R(24) + xi * (R(16) - R(16) * xi))));
    w[2] = R(1.0 / 192.0) * (R(115) + t2 * (R(-120) + R(48) * t2));
    w[3] = R(1.0 / 96.0) * (R(19) + xi * (R(44) + xi * (R(24) + xi * (R(-16) - R(16) * xi))));
    w[4] = R(1.0 / 384.0) * b2 * b2;
  }
}

// Shape differences S(xb) - S(xa) on one piece, in factored form
// (xb - xa) * g(xa, xb): the difference of the end points is formed once,
// so a short move does not lose its digits to cancellation.
template <int ORDER, typename R>
__device__ __forceinline__ void dshape(R xa, R xb, R* d) {
  const R dl = xb - xa;
  if (ORDER == 1) {
    d[0] = -dl;
    d[1] = dl;
  } else if (ORDER == 2) {
    const R s = xa + xb;
    d[0] = R(-0.5) * dl * (R(1) - s);
    d[1] = -dl * s;
    d[2] = R(0.5) * dl * (R(1) + s);
  } else if (ORDER == 3) {
    const R sixth = R(1.0 / 6.0);
    const R s = xa + xb;
    const R Q = xa * xa + xa * xb + xb * xb;
    const R aa = R(1) - xa, ab = R(1) - xb;
    d[0] = -sixth * dl * (aa * aa + aa * ab + ab * ab);
    d[1] = sixth * dl * (R(-6) * s + R(3) * Q);
    d[2] = sixth * dl * (R(3) + R(3) * s - R(3) * Q);
    d[3] = sixth * dl * Q;
  } else {  // quartic: divided differences of the five polynomials
    const R s1 = xa + xb, sq = xa * xa + xb * xb;
    const R s2 = sq + xa * xb, s3 = s1 * sq;
    const R A = R(1) - R(2) * xa, B = R(1) - R(2) * xb;
    const R C = R(1) + R(2) * xa, D = R(1) + R(2) * xb;
    d[0] = R(-1.0 / 192.0) * dl * ((A + B) * (A * A + B * B));
    d[1] = R(1.0 / 96.0) * dl * (R(-44) + R(24) * s1 + R(16) * s2 - R(16) * s3);
    d[2] = R(0.125) * dl * s1 * (R(-5) + R(2) * sq);
    d[3] = R(1.0 / 96.0) * dl * (R(44) + R(24) * s1 - R(16) * s2 - R(16) * s3);
    d[4] = R(1.0 / 192.0) * dl * ((C + D) * (C * C + D * D));
  }
}

// ------------------------------------------------------------------ accessors
// E/B samples staged in LDS: comp 0..2 = E, 3..5 = B.  `base` is the
// particle's cell in region coordinates; ref() folds a component's first
// stencil node into one index so that every stencil offset below is a
// compile-time immediate of the LDS read.
template <typename T>
using lds_ptr = __attribute__((address_space(3))) T*;

template <int DIMS, int ORDER, typename R, class G = Geo<DIMS, ORDER, R>>
struct LdsFields {
  lds_ptr<const R> s;
  int base;
  __device__ __forceinline__ lds_ptr<const R> ref(int comp, const int* b) const {
    // the component's first stencil node as one register, so that every
    // stencil read is a small immediate from it (paired LDS reads reach 255
    // elements; left to itself the compiler folds the array and component
    // offsets into the immediates and then needs an address add per pair)
    return pin(s + comp * G::e_vol + base + (b[2] * G::ex + b[1]) * G::ex + b[0]);
  }
  // planes 0 and 1 of the stencil are within reach of the first node's
  // register; planes 2 and 3 get a second register (far)
  __device__ __forceinline__ lds_ptr<const R> far(lds_ptr<const R> r) const {
    return DIMS == 3 && ORDER >= 2 ? pin(r + 2 * G::ex * G::ex) : r;
  }
  __device__ __forceinline__ lds_ptr<const R> plane(lds_ptr<const R> r, lds_ptr<const R> r2,
                                                    int k) const {
    return k < 2 ? r + k * G::ex * G::ex : r2 + (k - 2) * G::ex * G::ex;
  }
  // One LDS read per value: paired reads (ds_read2) of neighbouring samples
  // cost gfx950's LDS about twice the cycles of two single reads for the
  // lane layouts the sort produces (measured with the LDS probe's
  // push-pattern replay), so the reads go through a volatile pointer, which
  // keeps their compile-time offsets but stops the compiler from pairing
  // them.
  __device__ __forceinline__ R at(lds_ptr<const R> rk, int /*comp*/, int i, int j, int /*k*/) const {
    using vptr = __attribute__((address_space(3))) const volatile R*;
    return ((vptr)rk)[j * G::ex + i];
  }
  static __device__ __forceinline__ lds_ptr<const R> pin(lds_ptr<const R> p) {
    uint32_t a = (uint32_t)(uintptr_t)p;
    asm volatile("" : "+v"(a));
    return (lds_ptr<const R>)(uintptr_t)a;
  }
};

// E/B straight from global memory, with periodic wrap and zero outside the
// domain of open axes (the path of particles that drifted off their tile).
template <typename R>
struct GlobalFields {
  const R* const* E;
  const R* const* B;
  int cx, cy, cz;
  int n0, n1, n2;
  int o0, o1, o2;  // open flags
  int dims;
  struct Ref {
    int x, y, z;
  };
  __device__ __forceinline__ Ref ref(int /*comp*/, const int* b) const {
    return {cx + b[0], cy + b[1], cz + b[2]};
  }
  __device__ __forceinline__ Ref far(const Ref& r) const { return r; }
  __device__ __forceinline__ Ref plane(const Ref& r, const Ref&, int) const { return r; }
  __device__ __forceinline__ R at(const Ref& r, int comp, int i, int j, int k) const {
    const int c = comp < 3 ? comp : comp - 3;
    const bool isb = comp >= 3;
    const int sx = isb ? (c != 0) : (c == 0);
    const int sy = isb ? (c != 1) : (c == 1);
    const int sz = isb ? (c != 2) : (c == 2);
    const int ix = axis_slot(r.x + i, n0, o0, sx);
    const int iy = axis_slot(r.y + j, n1, o1, sy);
    const int iz = dims == 3 ? axis_slot(r.z + k, n2, o2, sz) : 0;
    if (ix < 0 || iy < 0 || iz < 0) return R(0);
    const R* f = isb ? B[c] : E[c];
    return f[ix + n0 * (iy + n1 * iz)];
  }
};

// Current sinks.  segment() fixes the first stencil node of a virtual
// segment; add() then takes compile-time offsets from it.  The LDS tile
// accumulates in double, or (single form) in 64-bit integers of values the
// caller has already scaled (see Geo); the global sink is the path of
// particles off their tile.
template <int DIMS, int ORDER, typename R>
struct LdsCurrent {
  using G = Geo<DIMS, ORDER, R>;
  double* s;
  int base;  // the particle's old cell in the J region
  double* seg;
  __device__ __forceinline__ void segment(const int* b) {
    seg = s + base + (b[2] * G::jx + b[1]) * G::jx + b[0];
  }
  // arithmetic type of the contributions: double for the fixed-point tile
  using C = typename std::conditional<G::fixed, double, R>::type;
  // add the contribution f * a
  __device__ __forceinline__ void put(int comp, int i, int j, int k, C f, C a) const {
    double* t = &seg[comp * G::j_vol + (k * G::jx + j) * G::jx + i];
    if constexpr (G::fixed) {
      // |f a| < 2^51: adding 1.5 * 2^52 rounds the product to an integer n
      // held in the low mantissa bits (one rounding, fused); the bit pattern
      // is then 0x4338 << 48 plus n in two's complement.  The tile adds the
      // patterns as 64-bit integers: the constant parts only touch bits
      // 48..63, so bits 0..47 hold the sum of the n modulo 2^48, which is
      // the exact sum as long as it stays below 2^47 in magnitude (the
      // scales guarantee it; the flush sign-extends bit 47).
      const double y = fma(f, a, 6755399441055744.0);
      atomicAdd((unsigned long long*)t, (unsigned long long)__double_as_longlong(y));
    } else {
      atomicAdd(t, (double)(f * a));
    }
  }
};

template <typename R>
struct GlobalCurrent {
  R* const* J;
  int cx, cy, cz;
  int n0, n1, n2;
  int o0, o1, o2;
  int dims;
  int sx, sy, sz;
  __device__ __forceinline__ void segment(const int* b) {
    sx = cx + b[0];
    sy = cy + b[1];
    sz = cz + b[2];
  }
  using C = R;
  __device__ __forceinline__ void put(int comp, int i, int j, int k, R f, R a) const {
    const R v = f * a;
    const int ix = axis_slot(sx + i, n0, o0, comp == 0);
    const int iy = axis_slot(sy + j, n1, o1, comp == 1);
    const int iz = dims == 3 ? axis_slot(sz + k, n2, o2, comp == 2) : 0;
    if (ix < 0 || iy < 0 || iz < 0) return;  // dropped beyond an open face
    atomic_add(&J[comp][ix + n0 * (iy + n1 * iz)], v);
  }
};

// ------------------------------------------------------------------ gather
// Order-n interpolation of one component: weights per axis `w`, first node
// offsets `b` relative to the particle's cell.
template <int DIMS, int ORDER, typename R, class Acc>
__device__ __forceinline__ R interp(const Acc& acc, int comp, const R (*w)[ORDER + 1],
                                    const int* b) {
  constexpr int M = ORDER + 1;
  constexpr int MZ = DIMS == 3 ? M : 1;
  const auto r = acc.ref(comp, b);
  const auto r2 = acc.far(r);
  R s = R(0);
#pragma unroll
  for (int k = 0; k < MZ; ++k) {
    const auto rk = acc.plane(r, r2, k);
    R sy = R(0);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      R sx = R(0);
#pragma unroll
      for (int i = 0; i < M; ++i) sx += w[0][i] * acc.at(rk, comp, i, j, k);
      sy += w[1][j] * sx;
    }
    s += (DIMS == 3 ? w[2][k] : R(1)) * sy;
  }
  return s;
}

// E and B at the particle (Sec. 5.2 steps i-ii): each component with the
// weights of its own Yee position, staggered along its axis (E_c) or along
// the two other axes (B_c).
template <int DIMS, int ORDER, typename R, class Acc>
__device__ __forceinline__ void gather(const Acc& acc, const R* o, R* Ep, R* Bp) {
  constexpr int M = ORDER + 1;
  R wn[3][M], ws[3][M];
  int bn[3] = {0, 0, 0}, bs[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < DIMS; ++d) {
    R xi;
    bn[d] = piece_node<ORDER>(o[d], xi) - ORDER / 2;
    shape<ORDER>(xi, wn[d]);
    bs[d] = piece_stag<ORDER>(o[d], xi) - ORDER / 2;
    shape<ORDER>(xi, ws[d]);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    R we[3][M], wb[3][M];
    int be[3], bb[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const bool se = (d == c), sb = (d != c);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        we[d][i] = se ? ws[d][i] : wn[d][i];
        wb[d][i] = sb ? ws[d][i] : wn[d][i];
      }
      be[d] = se ? bs[d] : bn[d];
      bb[d] = sb ? bs[d] : bn[d];
    }
    Ep[c] = interp<DIMS, ORDER, R>(acc, c, we, be);
    Bp[c] = interp<DIMS, ORDER, R>(acc, 3 + c, wb, bb);
  }
}

// ------------------------------------------------------------------ push
// 1/sqrt(x) and 1/x.  Single precision takes the hardware approximations
// (v_rsq_f32, v_rcp_f32: about 1 ulp, far below the 1e-5 that the single
// form is held to) instead of the correctly rounded sequences, which cost
// about ten instructions each; double precision keeps the exact forms.
__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_r(double x) { return 1.0 / x; }

// Relativistic Boris step (Sec. 5.2 step iii; Boris is this build's reading
// of "fully relativistic equations of motion"): half electric kick, magnetic
// rotation with gamma of the half-kicked momentum, half electric kick.
template <typename R>
__device__ __forceinline__ void boris(R hqm, R* u, const R* E, const R* B) {
  R um[3], t[3], s[3], up[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) um[c] = u[c] + hqm * E[c];
  const R hg = hqm * rsqrt_r(R(1) + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
#pragma unroll
  for (int c = 0; c < 3; ++c) t[c] = hg * B[c];
  const R f = R(2) * rcp_r(R(1) + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
#pragma unroll
  for (int c = 0; c < 3; ++c) s[c] = f * t[c];
  up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
  up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
  up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
  u[0] = um[0] + (up[1] * s[2] - up[2] * s[1]) + hqm * E[0];
  u[1] = um[1] + (up[2] * s[0] - up[0] * s[2]) + hqm * E[1];
  u[2] = um[2] + (up[0] * s[1] - up[1] * s[0]) + hqm * E[2];
}

// ------------------------------------------------------------------ deposit
// Charge-conserving current of the straight path from offset o0 in the old
// cell to offset o1 in the cell shifted by sh (Sec. 5.2 steps iv-v): split
// at the planes where the node stencil switches (one per axis at most; at
// most DIMS+1 virtual segments), then the Esirkepov density decomposition
// on each segment's own (n+1)^D stencil.  J_c at the slots base_c + i
// (i < n) is fac_c * P_c[i] * A_c(j,k), where P_c is the running sum of the
// shape differences along c and A_c the time-averaged transverse weight.
// Every segment end is expressed in the piece frame of its stencil: crossing
// points exactly on their plane, other coordinates once per point.
template <int DIMS, typename R>
struct Split {
  int k0[3], k1[3];
  R xi0[3], xi1[3], dl[3], pk0[3], pk1[3];
  bool cr[3];
  int jd[3];
  R tb[DIMS + 2];
  int m;  // crossings: the path has m + 1 segments
};

template <int DIMS, int ORDER, typename R>
__device__ __forceinline__ void split_path(Split<DIMS, R>& S, const R* o0, const int* sh,
                                           const R* o1) {
  constexpr bool odd = ORDER & 1;
  R fr[3];
#pragma unroll
  for (int d = 0; d < DIMS; ++d) {
    S.k0[d] = piece_node<ORDER>(o0[d], S.xi0[d]);
    S.k1[d] = sh[d] + piece_node<ORDER>(o1[d], S.xi1[d]);
    S.dl[d] = R(S.k1[d] - S.k0[d]) + (S.xi1[d] - S.xi0[d]);
    S.cr[d] = false;
    fr[d] = R(2);
    S.pk0[d] = S.pk1[d] = R(0);
    if (S.k1[d] != S.k0[d]) {
      const bool up = S.k1[d] > S.k0[d];
      S.pk0[d] = odd ? (up ? R(1) : R(0)) : (up ? R(0.5) : R(-0.5));
      S.pk1[d] = odd ? (up ? R(0) : R(1)) : (up ? R(-0.5) : R(0.5));
      // crossing fraction; charge conservation does not depend on its last
      // bits (neighbouring segments share their end points exactly), so
      // single precision takes a reciprocal instead of a correctly rounded
      // division
      R f;
      if constexpr (sizeof(R) == 4)
        f = (S.pk0[d] - S.xi0[d]) * __builtin_amdgcn_rcpf(S.dl[d]);
      else
        f = (S.pk0[d] - S.xi0[d]) / S.dl[d];
      if (f > R(0) && f < R(1)) {
        S.cr[d] = true;
        fr[d] = f;
      } else if (!(f > R(0))) {  // starts on the plane: the path is in piece k1
        S.k0[d] = S.k1[d];
        S.xi0[d] = S.pk1[d];
      } else {  // ends on the plane: the path is in piece k0
        S.k1[d] = S.k0[d];
        S.xi1[d] = S.pk0[d];
      }
    }
  }
  // ascending crossing fractions; jd[d] = index of axis d's crossing point
  S.jd[0] = S.jd[1] = S.jd[2] = DIMS + 2;
  S.m = 0;
  S.tb[0] = R(0);
#pragma unroll
  for (int d = 0; d < DIMS; ++d) {
    if (!S.cr[d]) continue;
    int rank = 1;
#pragma unroll
    for (int e = 0; e < DIMS; ++e)
      if (e != d && S.cr[e] && (fr[e] < fr[d] || (fr[e] == fr[d] && e < d))) ++rank;
    S.jd[d] = rank;
    ++S.m;
  }
  // tb[j] = the j-th crossing fraction, 1 from tb[m+1] on (selects, so that
  // the struct stays in registers)
#pragma unroll
  for (int j = 1; j < DIMS + 2; ++j) {
    R v = R(1);
#pragma unroll
    for (int d = 0; d < DIMS; ++d)
      if (S.cr[d] && S.jd[d] == j) v = fr[d];
    S.tb[j] = v;
  }
}

// End points of segment s in its piece frame, its first stencil node and
// its fraction of the time step.
template <int DIMS, int ORDER, typename R>
__device__ __forceinline__ void segment_ends(const Split<DIMS, R>& S, int s, R* xa, R* xb,
                                             int* base, R& ft) {
  R ta = R(0), tbb = R(1);
#pragma unroll
  for (int j = 0; j < DIMS + 2; ++j) {
    if (j == s) ta = S.tb[j];
    if (j == s + 1) tbb = S.tb[j];
  }
  ft = tbb - ta;
  base[0] = base[1] = base[2] = 0;
  xa[2] = xb[2] = R(0);
#pragma unroll
  for (int d = 0; d < DIMS; ++d) {
    const bool f1 = S.cr[d] && s >= S.jd[d];
    R a, b;
    if (s == 0)
      a = S.xi0[d];
    else if (S.cr[d] && s == S.jd[d])
      a = S.pk1[d];
    else
      a = f1 ? S.xi1[d] - (R(1) - ta) * S.dl[d] : S.xi0[d] + ta * S.dl[d];
    if (s == S.m)
      b = S.xi1[d];
    else if (S.cr[d] && s + 1 == S.jd[d])
      b = S.pk0[d];
    else
      b = f1 ? S.xi1[d] - (R(1) - tbb) * S.dl[d] : S.xi0[d] + tbb * S.dl[d];
    base[d] = (f1 ? S.k1[d] : S.k0[d]) - ORDER / 2;
    xa[d] = a;
    xb[d] = b;
  }
}

// Esirkepov current of one segment whose first stencil node the sink holds.
// fz (2D only) = q v_z times the segment's time fraction.  Weights and
// transverse factors are formed in R; the final products run in the sink's
// arithmetic type.
template <int DIMS, int ORDER, typename R, class Sink>
__device__ __forceinline__ void deposit_segment(const Sink& sk, const R* jfac, const R* xa,
                                                const R* xb, R q, R fz) {
  constexpr int M = ORDER + 1;
  using C = typename Sink::C;
  // mean weight Sm = S0 + dS/2 and dS/12: the Esirkepov transverse factor
  // S0a S0b + (dSa S0b + S0a dSb)/2 + dSa dSb/3 equals Sma Smb + dSa dSb/12
  R Sm[3][M], dS[3][M], d12[3][M];
#pragma unroll
  for (int d = 0; d < DIMS; ++d) {
    R S0[M];
    shape<ORDER>(xa[d], S0);
    dshape<ORDER>(xa[d], xb[d], dS[d]);
#pragma unroll
    for (int i = 0; i < M; ++i) {
      Sm[d][i] = S0[i] + R(0.5) * dS[d][i];
      d12[d][i] = R(1.0 / 12.0) * dS[d][i];
    }
  }
  if (DIMS == 3) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int a = (c + 1) % 3, b = (c + 2) % 3;
      C P[ORDER];
      R run = R(0);
#pragma unroll
      for (int i = 0; i < ORDER; ++i) {
        run += dS[c][i];
        P[i] = (C)(q * jfac[c] * run);
      }
#pragma unroll
      for (int ib = 0; ib < M; ++ib)
#pragma unroll
        for (int ia = 0; ia < M; ++ia) {
          const C A = (C)(Sm[a][ia] * Sm[b][ib] + d12[a][ia] * dS[b][ib]);
#pragma unroll
          for (int ic = 0; ic < ORDER; ++ic) {
            int L[3];
            L[c] = ic;
            L[a] = ia;
            L[b] = ib;
            sk.put(c, L[0], L[1], L[2], P[ic], A);
          }
        }
    }
  } else {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int a = 1 - c;
      C P[ORDER];
      R run = R(0);
#pragma unroll
      for (int i = 0; i < ORDER; ++i) {
        run += dS[c][i];
        P[i] = (C)(q * jfac[c] * run);
      }
#pragma unroll
      for (int ia = 0; ia < M; ++ia) {
        const C A = (C)Sm[a][ia];
#pragma unroll
        for (int ic = 0; ic < ORDER; ++ic) {
          int L[2];
          L[c] = ic;
          L[a] = ia;
          sk.put(c, L[0], L[1], 0, P[ic], A);
        }
      }
    }
    const C fzc = (C)fz;
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
      for (int i = 0; i < M; ++i)
        sk.put(2, i, j, 0, fzc, (C)(Sm[0][i] * Sm[1][j] + d12[0][i] * dS[1][j]));
  }
}

// The whole path, segment after segment (global-memory path).
template <int DIMS, int ORDER, typename R, class Sink>
__device__ __forceinline__ void deposit(Sink sink, const R* jfac, const R* o0,
                                        const int* sh, const R* o1, R q, R vz) {
  Split<DIMS, R> S;
  split_path<DIMS, ORDER, R>(S, o0, sh, o1);
  for (int s = 0; s <= S.m; ++s) {
    R xa[3], xb[3], ft;
    int base[3];
    segment_ends<DIMS, ORDER, R>(S, s, xa, xb, base, ft);
    sink.segment(base);
    deposit_segment<DIMS, ORDER, R>(sink, jfac, xa, xb, q, q * vz * ft);
  }
}

// ------------------------------------------------------------------ particle
// Particle state in registers.
template <typename R>
struct PState {
  int cl;
  R o[3];
  R u[3];
  R q;
};

template <int DIMS, typename R>
__device__ __forceinline__ PState<R> load_particle(const DParts<R>& pa, int p, R q_const) {
  PState<R> s;
  s.cl = pa.cell[p];
  s.o[0] = s.o[1] = s.o[2] = R(0);
#pragma unroll
  for (int d = 0; d < DIMS; ++d) s.o[d] = pa.off[d][p];
#pragma unroll
  for (int c = 0; c < 3; ++c) s.u[c] = pa.u[c][p];
  s.q = pa.q ? pa.q[p] : q_const;
  return s;
}

// Cell index -> (ix, iy, iz); false (and a raised flag) for a state the
// kernels must not index with.
template <int DIMS, typename R>
__device__ __forceinline__ bool decode(const KParams<R>& P, const PState<R>& s, int* c3,
                                       DevFlags* flg) {
  const int ncell = P.n[0] * P.n[1] * P.n[2];
  bool bad = s.cl >= ncell;
#pragma unroll
  for (int d = 0; d < DIMS; ++d) bad |= !(s.o[d] >= R(0) && s.o[d] < R(1));
  if (bad) {
    raise_flag(flg, s.cl >= ncell ? PIC_FLAG_CELL : PIC_FLAG_OFFSET);
    return false;
  }
  const uint32_t rest = P.dn0.div((uint32_t)s.cl);
  c3[0] = s.cl - (int)rest * P.n[0];
  c3[1] = DIMS == 3 ? (int)(rest - P.dn1.div(rest) * P.n[1]) : (int)rest;
  c3[2] = DIMS == 3 ? (int)P.dn1.div(rest) : 0;
  return true;
}

// Boris push and move of one particle: u^{n-1/2} -> u^{n+1/2}, then the new
// offsets o1 and cell shifts sh (the deposit uses exactly these stored
// values).  Returns false for a non-finite momentum.
template <int DIMS, typename R>
__device__ __forceinline__ bool push_move(const KParams<R>& P, PState<R>& s, const R* Ep,
                                          const R* Bp, int* sh, R* o1, R& vz, bool& small,
                                          DevFlags* flg) {
  boris<R>(P.hqm, s.u, Ep, Bp);
  const R g2 = R(1) + s.u[0] * s.u[0] + s.u[1] * s.u[1] + s.u[2] * s.u[2];
  if (!isfinite(g2)) {
    raise_flag(flg, PIC_FLAG_NONFINITE);
    return false;
  }
  const R ig = rsqrt_r(g2);  // 1/gamma
  small = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    sh[d] = 0;
    o1[d] = R(0);
  }
#pragma unroll
  for (int d = 0; d < DIMS; ++d) {
    const R dlt = s.u[d] * ig * P.dtdx[d];
    // |move| < 0.49 keeps every segment stencil inside the LDS current
    // region even after rounding of o + dlt (a bound of exactly 1/2 could
    // round to x1 = 3/2 and shift a quadratic stencil one node further)
    small = small && dlt < R(0.49) && dlt > R(-0.49);
    R x1 = s.o[d] + dlt;
    if (x1 < R(-1) || x1 >= R(2)) {  // cannot happen below the Courant limit
      raise_flag(flg, PIC_FLAG_OVERSPEED);
      x1 = x1 < R(-1) ? R(-1) : R(1.5);
    }
    int k = x1 >= R(1) ? 1 : (x1 < R(0) ? -1 : 0);
    R on = x1 - R(k);
    if (on >= R(1)) {  // -tiny + 1 rounded up to 1
      on = R(0);
      k += 1;
    }
    sh[d] = k;
    o1[d] = on;
  }
  vz = s.u[2] * ig;
  return true;
}

// New cell after the shifts (periodic wrap; -1 when absorbed at an open face).
template <int DIMS, typename R>
__device__ __forceinline__ int new_cell(const KParams<R>& P, const int* c3, const int* sh) {
  int c1[3] = {c3[0], c3[1], c3[2]};
  bool absorbed = false;
#pragma unroll
  for (int d = 0; d < DIMS; ++d) {
    int cn = c3[d] + sh[d];
    if (P.bc[d] == PIC_BC_PERIODIC)
      cn = wrap1(cn, P.n[d]);
    else if (cn < 0 || cn > P.n[d] - 2)
      absorbed = true;
    c1[d] = cn;
  }
  return absorbed ? -1 : c1[0] + P.n[0] * (c1[1] + P.n[1] * c1[2]);
}

template <int DIMS, typename R>
__device__ __forceinline__ void store_particle(const DParts<R>& pa, int p, const PState<R>& s,
                                               const R* o1, int cell) {
#pragma unroll
  for (int c = 0; c < 3; ++c) pa.u[c][p] = s.u[c];
#pragma unroll
  for (int d = 0; d < DIMS; ++d) pa.off[d][p] = o1[d];
  pa.cell[p] = cell;
}

// ------------------------------------------------------------------ tiles
// threadIdx.x behind an opaque copy: index arithmetic on it inside the
// persistent tile loop stays there instead of being hoisted out of the loop
// and held in registers across the particle loop.
__device__ __forceinline__ int opaque_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// E and B of a tile + halo (zero outside open faces) into registers (G: the
// region's geometry, the push tile's by default).  Each
// thread takes region samples and loads the six components there, with the
// storage offsets along each axis formed once per sample; all loads are in
// flight together.
template <int DIMS, int ORDER, typename R, int NR, class G = Geo<DIMS, ORDER, R>>
__device__ inline void stage_load(const KParams<R>& P, const DFields<R>& F, const int org[3],
                                  R (&stage)[NR][6]) {
  const int open0 = P.bc[0] == PIC_BC_OPEN, open1 = P.bc[1] == PIC_BC_OPEN;
  const int open2 = DIMS == 3 && P.bc[2] == PIC_BC_OPEN;
  const int str1 = P.n[0], str2 = P.n[0] * P.n[1];
  const int tid = opaque_tid();
  const int bx = org[0] + G::e_lo, by = org[1] + G::e_lo, bz = org[2] + G::e_lo_z;
  if (axis_inside(bx, G::ex, P.n[0], open0) && axis_inside(by, G::ex, P.n[1], open1) &&
      (DIMS == 2 || axis_inside(bz, G::ez, P.n[2], open2))) {
    // no wrap, no boundary: one storage offset per sample for all components
    const int base = (DIMS == 3 ? bz * str2 : 0) + by * str1 + bx;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int r = tid + k * G::NT;
#pragma unroll
      for (int c = 0; c < 6; ++c) stage[k][c] = R(0);
      if (r < G::e_vol) {
        const int lx = r % G::ex, ly = (r / G::ex) % G::ex, lz = r / (G::ex * G::ex);
        const int o = base + (DIMS == 3 ? lz * str2 : 0) + ly * str1 + lx;
#pragma unroll
        for (int c = 0; c < 6; ++c) stage[k][c] = (c >= 3 ? F.B[c - 3] : F.E[c])[o];
      }
    }
    return;
  }
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const int r = tid + k * G::NT;
#pragma unroll
    for (int c = 0; c < 6; ++c) stage[k][c] = R(0);
    if (r < G::e_vol) {
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
        if (ix >= 0 && iy >= 0 && iz >= 0) stage[k][c] = (isb ? F.B[e] : F.E[e])[ix + iy + iz];
      }
    }
  }
}

template <int DIMS, int ORDER, typename R>
__device__ inline void tile_origin(const KParams<R>& P, int tile, int org[3]) {
  using G = Geo<DIMS, ORDER, R>;
  org[0] = (tile % P.ntile[0]) * G::T;
  org[1] = ((tile / P.ntile[0]) % P.ntile[1]) * G::T;
  org[2] = (tile / (P.ntile[0] * P.ntile[1])) * G::TZ;
}

}  // namespace pic
