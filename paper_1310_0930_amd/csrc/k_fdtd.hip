// FDTD (Yee) field advance: B -= dt/2 C E; E += dt (C^T B - J); B -= dt/2 C E.
//
// The paper advances the fields with the finite-difference time-domain method
// (Sec. 2), a local, nearest-neighbour solver chosen for its small
// communication volume (Sec. 3).  C is the forward-difference curl of E at
// the B positions and C^T (its transpose) the backward-difference curl of B
// at the E positions.  One thread per cell updates the three components;
// reads of the neighbours along x are coalesced and the rest hit L2.  On 3D
// grids periodic along every axis one thread takes a short z column instead
// (k_half_b_col, k_advance_e_col).
//
// Open faces: the tangential E samples on the first and last node planes of
// an open axis are advanced with the first-order Mur condition
// F0^{n+1} = F1^n + (dt - dx)/(dt + dx) (F1^{n+1} - F0^n), F1 the next sample
// inward.  Samples on two open faces (edges) are done in a second pass along
// the lower such axis.  Samples beyond the last node (half-integer positions)
// are outside the domain, are never written and are read as zero.
#include <mutex>

#include "k_common.h"

namespace pic {

struct FdParams {
  int n[3];
  int open[3];
  int dims;
  FastDiv dn0, dn1;
};

__device__ __forceinline__ void decompose(const FdParams& P, int idx, int& i, int& j, int& k) {
  const uint32_t rest = P.dn0.div((uint32_t)idx);
  i = idx - (int)rest * P.n[0];
  if (P.dims == 3) {
    const uint32_t r2 = P.dn1.div(rest);
    j = (int)(rest - r2 * P.n[1]);
    k = (int)r2;
  } else {
    j = (int)rest;
    k = 0;
  }
}

// Is the slot (i,j,k) of a component with staggering (sx,sy,sz) inside?
__device__ __forceinline__ bool inside(const FdParams& P, int i, int j, int k, int sx, int sy, int sz) {
  if (P.open[0] && i > P.n[0] - 1 - sx) return false;
  if (P.open[1] && j > P.n[1] - 1 - sy) return false;
  if (P.dims == 3 && P.open[2] && k > P.n[2] - 1 - sz) return false;
  return true;
}

// Neighbour index along axis d (+1 or -1); -1 if it falls outside an open axis.
__device__ __forceinline__ int nb(const FdParams& P, int i, int j, int k, int d, int step) {
  int L[3] = {i, j, k};
  L[d] += step;
  if (L[d] < 0 || L[d] >= P.n[d]) {
    if (P.open[d]) return -1;
    L[d] = L[d] < 0 ? L[d] + P.n[d] : L[d] - P.n[d];
  }
  return L[0] + P.n[0] * (L[1] + P.n[1] * L[2]);
}

// Block index with the 8 XCDs each taking a contiguous range of blocks
// (consecutive block ids are dealt round-robin to the XCDs): the neighbour
// rows and planes a stencil reads then sit in the same XCD's L2.  The grid
// must be a multiple of 8 blocks; the mapping is a permutation of it.
__device__ __forceinline__ int xcd_block() {
  const int per = gridDim.x >> 3;
  return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

__host__ inline unsigned xcd_grid(long ncell) {
  const long g = (ncell + 255) / 256;
  return (unsigned)((g + 7) / 8 * 8);
}

template <typename R>
__device__ __forceinline__ R ld_or0(const R* a, int idx) {
  return idx < 0 ? R(0) : a[idx];
}

// B -= h C E
template <typename R>
__global__ void k_half_b(FdParams P, const R* __restrict__ E0, const R* __restrict__ E1,
                         const R* __restrict__ E2, R* __restrict__ B0, R* __restrict__ B1,
                         R* __restrict__ B2, R hx, R hy, R hz, int ncell) {
  const int idx = xcd_block() * blockDim.x + threadIdx.x;
  if (idx >= ncell) return;
  int i, j, k;
  decompose(P, idx, i, j, k);
  const R* E[3] = {E0, E1, E2};
  R* B[3] = {B0, B1, B2};
  const R h[3] = {hx, hy, hz};  // dt/2 / dx_d
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (!inside(P, i, j, k, c != 0, c != 1, c != 2)) continue;
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    R acc = R(0);
    // + d_a E_b - d_b E_a, forward differences
    if (a < P.dims) acc += h[a] * (ld_or0(E[b], nb(P, i, j, k, a, 1)) - E[b][idx]);
    if (b < P.dims) acc -= h[b] * (ld_or0(E[a], nb(P, i, j, k, b, 1)) - E[a][idx]);
    B[c][idx] -= acc;
  }
}

// Tangential E on the boundary plane of an open axis d != c?  Returns the
// number of such axes and the lowest one.
__device__ __forceinline__ int mur_axes(const FdParams& P, int c, int i, int j, int k, int& lowest) {
  const int L[3] = {i, j, k};
  int cnt = 0;
  lowest = -1;
  for (int d = 0; d < P.dims; ++d) {
    if (d == c || !P.open[d]) continue;
    if (L[d] == 0 || L[d] == P.n[d] - 1) {
      if (cnt == 0) lowest = d;
      ++cnt;
    }
  }
  return cnt;
}

// Offset of the saved plane (axis d, side s, component c) in the Mur buffer
// and the index of (i,j,k) inside it.
struct MurPlanes {
  long off[3][2][3];
  int na[3], nbb[3];  // the two other axes per d (a < b)
};

// E += dt (C^T B - J) on interior samples; saves E^n next to open faces.
template <typename R>
__global__ void k_advance_e(FdParams P, MurPlanes M, R* __restrict__ E0, R* __restrict__ E1,
                            R* __restrict__ E2, const R* __restrict__ B0, const R* __restrict__ B1,
                            const R* __restrict__ B2, const R* __restrict__ J0,
                            const R* __restrict__ J1, const R* __restrict__ J2, R gx, R gy, R gz,
                            R dt, int ncell, R* __restrict__ save) {
  const int idx = xcd_block() * blockDim.x + threadIdx.x;
  if (idx >= ncell) return;
  int i, j, k;
  decompose(P, idx, i, j, k);
  R* E[3] = {E0, E1, E2};
  const R* B[3] = {B0, B1, B2};
  const R* J[3] = {J0, J1, J2};
  const R g[3] = {gx, gy, gz};  // dt / dx_d
  const int L[3] = {i, j, k};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (!inside(P, i, j, k, c == 0, c == 1, c == 2)) continue;
    // keep E^n of samples next to an open face for the Mur update
    for (int d = 0; d < P.dims; ++d) {
      if (d == c || !P.open[d]) continue;
      const int side = L[d] == 1 ? 0 : (L[d] == P.n[d] - 2 ? 1 : -1);
      if (side < 0) continue;
      const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
      const long pos = M.off[d][side][c] + L[a] + (long)M.na[d] * (b < 3 ? L[b] : 0);
      save[pos] = E[c][idx];
    }
    int lowest;
    if (mur_axes(P, c, i, j, k, lowest) > 0) continue;
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    R curl = R(0);
    // + d_a B_b - d_b B_a, backward differences
    if (a < P.dims) curl += g[a] * (B[b][idx] - ld_or0(B[b], nb(P, i, j, k, a, -1)));
    if (b < P.dims) curl -= g[b] * (B[a][idx] - ld_or0(B[a], nb(P, i, j, k, b, -1)));
    E[c][idx] += curl - dt * J[c][idx];
  }
}

// The same two updates on a 3D grid with every axis periodic, one thread
// per (i, j) column of FD_KC consecutive z planes: the column's index
// arithmetic and wraps are formed once, and the z neighbour of one plane is
// the next plane's centre sample, kept in registers.  Consecutive threads
// take consecutive x, so every load and store stays coalesced, and the x
// neighbour is the adjacent lane's own sample, passed across the wavefront;
// only a lane at the wavefront's or the row's end loads it.
constexpr int FD_KC = 4;

__device__ __forceinline__ int column_start(const FdParams& P, int t, int& i, int& j, int& k0) {
  const uint32_t q0 = P.dn0.div((uint32_t)t);  // t / n0
  i = t - (int)q0 * P.n[0];
  const uint32_t q1 = P.dn1.div(q0);  // column block along z
  j = (int)(q0 - q1 * P.n[1]);
  k0 = (int)q1 * FD_KC;
  return i + P.n[0] * (j + P.n[1] * k0);
}

// B -= h C E (forward differences)
template <typename R>
__global__ void k_half_b_col(FdParams P, const R* __restrict__ E0, const R* __restrict__ E1,
                             const R* __restrict__ E2, R* __restrict__ B0, R* __restrict__ B1,
                             R* __restrict__ B2, R hx, R hy, R hz, int ncol) {
  const int t = xcd_block() * blockDim.x + threadIdx.x;
  if (t >= ncol) return;
  int i, j, k0;
  int idx = column_start(P, t, i, j, k0);
  const int plane = P.n[0] * P.n[1];
  const int ip = i + 1 < P.n[0] ? 1 : 1 - P.n[0];
  const int jp = j + 1 < P.n[1] ? P.n[0] : P.n[0] - plane;
  R exk = E0[idx], eyk = E1[idx];  // E_x, E_y at plane k
  const int lane = threadIdx.x & 63;
  const bool own = lane < 63 && i + 1 < P.n[0];  // the x neighbour is the next lane's sample
#pragma unroll
  for (int kk = 0; kk < FD_KC; ++kk, idx += plane) {
    const int kp = k0 + kk + 1 < P.n[2] ? plane : plane - P.n[2] * plane;
    const R ex1 = E0[idx + kp], ey1 = E1[idx + kp], ez = E2[idx];
    R ezx = __shfl_down(ez, 1, 64), eyx = __shfl_down(eyk, 1, 64);
    if (!own) {
      ezx = E2[idx + ip];
      eyx = E1[idx + ip];
    }
    B0[idx] -= hy * (E2[idx + jp] - ez) - hz * (ey1 - eyk);
    B1[idx] -= hz * (ex1 - exk) - hx * (ezx - ez);
    B2[idx] -= hx * (eyx - eyk) - hy * (E0[idx + jp] - exk);
    exk = ex1;
    eyk = ey1;
  }
}

// E += g C^T B - dt J (backward differences)
template <typename R>
__global__ void k_advance_e_col(FdParams P, R* __restrict__ E0, R* __restrict__ E1,
                                R* __restrict__ E2, const R* __restrict__ B0,
                                const R* __restrict__ B1, const R* __restrict__ B2,
                                const R* __restrict__ J0, const R* __restrict__ J1,
                                const R* __restrict__ J2, R gx, R gy, R gz, R dt, int ncol) {
  const int t = xcd_block() * blockDim.x + threadIdx.x;
  if (t >= ncol) return;
  int i, j, k0;
  int idx = column_start(P, t, i, j, k0);
  const int plane = P.n[0] * P.n[1];
  const int im = i > 0 ? -1 : P.n[0] - 1;
  const int jm = j > 0 ? -P.n[0] : plane - P.n[0];
  const int km = k0 > 0 ? -plane : (P.n[2] - 1) * plane;
  R bxm = B0[idx + km], bym = B1[idx + km];  // B_x, B_y at plane k - 1
  const int lane = threadIdx.x & 63;
  const bool own = lane > 0 && i > 0;  // the -x neighbour is the previous lane's sample
#pragma unroll
  for (int kk = 0; kk < FD_KC; ++kk, idx += plane) {
    const R bx = B0[idx], by = B1[idx], bz = B2[idx];
    R bzx = __shfl_up(bz, 1, 64), byx = __shfl_up(by, 1, 64);
    if (!own) {
      bzx = B2[idx + im];
      byx = B1[idx + im];
    }
    E0[idx] += (gy * (bz - B2[idx + jm]) - gz * (by - bym)) - dt * J0[idx];
    E1[idx] += (gz * (bx - bxm) - gx * (bz - bzx)) - dt * J1[idx];
    E2[idx] += (gx * (by - byx) - gy * (bx - B0[idx + jm])) - dt * J2[idx];
    bxm = bx;
    bym = by;
  }
}

// Mur update of the samples on the face (d, side) with exactly `pass` open
// boundary axes, along their lowest such axis.
template <typename R>
__global__ void k_mur(FdParams P, MurPlanes M, R* __restrict__ E0, R* __restrict__ E1,
                      R* __restrict__ E2, int d, int side, int pass, R kappa,
                      const R* __restrict__ save) {
  const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
  const int na = P.n[a], nbv = b < P.dims ? P.n[b] : 1;
  const long plane = (long)na * nbv;
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= 2 * plane) return;
  const int which = (int)(t / plane);
  const long r = t - which * plane;
  const int c = (d + 1 + which) % 3;  // the two components tangential to the face
  int L[3];
  L[d] = side ? P.n[d] - 1 : 0;
  L[a] = (int)(r % na);
  L[b] = (int)(r / na);
  if (P.dims == 2 && b == 2 && L[b] != 0) return;
  if (!inside(P, L[0], L[1], L[2], c == 0, c == 1, c == 2)) return;
  int lowest;
  if (mur_axes(P, c, L[0], L[1], L[2], lowest) != pass || lowest != d) return;
  R* E[3] = {E0, E1, E2};
  const int i0 = L[0] + P.n[0] * (L[1] + P.n[1] * L[2]);
  int N[3] = {L[0], L[1], L[2]};
  N[d] += side ? -1 : 1;
  const int i1 = N[0] + P.n[0] * (N[1] + P.n[1] * N[2]);
  const R f1_old = save[M.off[d][side][c] + L[a] + (long)M.na[d] * L[b]];
  E[c][i0] = f1_old + kappa * (E[c][i1] - E[c][i0]);
}

template <typename R>
__global__ void k_fill3_zero(R* a, R* b, R* c, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    a[i] = R(0);
    b[i] = R(0);
    c[i] = R(0);
  }
}

// `save` holds the E samples next to open faces between the Yee update and
// the Mur updates (mur_len(cfg) reals); every call writes them before it
// reads them.
template <typename R>
static int launch_fa(const pic_ctx* ctx, const pic_fields* f, R* save, hipStream_t s) {
  const pic_config& cf = ctx->cfg;
  FdParams P;
  P.dims = cf.dims;
  for (int d = 0; d < 3; ++d) {
    P.n[d] = d < cf.dims ? cf.n[d] : 1;
    P.open[d] = d < cf.dims && cf.bc[d] == PIC_BC_OPEN;
  }
  P.dn0.init((uint32_t)P.n[0]);
  P.dn1.init((uint32_t)P.n[1]);
  const int ncell = P.n[0] * P.n[1] * P.n[2];
  const R dt = (R)cf.dt;
  R h[3], g[3];
  for (int d = 0; d < 3; ++d) {
    h[d] = (R)(0.5 * cf.dt / cf.dx[d]);
    g[d] = (R)(cf.dt / cf.dx[d]);
  }
  R* E[3];
  R* B[3];
  R* J[3];
  for (int c = 0; c < 3; ++c) {
    E[c] = (R*)f->E[c];
    B[c] = (R*)f->B[c];
    J[c] = (R*)f->J[c];
  }
  MurPlanes M;
  long off = 0;
  for (int d = 0; d < 3; ++d) {
    const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
    M.na[d] = P.n[a];
    M.nbb[d] = P.n[b];
    for (int sd = 0; sd < 2; ++sd)
      for (int c = 0; c < 3; ++c) {
        M.off[d][sd][c] = off;
        if (P.open[d] && c != d) off += (long)P.n[a] * P.n[b];
      }
  }
  if (P.dims == 3 && !P.open[0] && !P.open[1] && !P.open[2] && P.n[2] % FD_KC == 0) {
    const int ncol = ncell / FD_KC;
    const unsigned cgrid = xcd_grid(ncol);  // a multiple of 8 blocks (xcd_block)
    k_half_b_col<R><<<dim3(cgrid), dim3(256), 0, s>>>(P, E[0], E[1], E[2], B[0], B[1], B[2], h[0],
                                                       h[1], h[2], ncol);
    k_advance_e_col<R><<<dim3(cgrid), dim3(256), 0, s>>>(P, E[0], E[1], E[2], B[0], B[1], B[2],
                                                          J[0], J[1], J[2], g[0], g[1], g[2], dt,
                                                          ncol);
    k_half_b_col<R><<<dim3(cgrid), dim3(256), 0, s>>>(P, E[0], E[1], E[2], B[0], B[1], B[2], h[0],
                                                       h[1], h[2], ncol);
    return (int)hipGetLastError();
  }
  const unsigned grid = xcd_grid(ncell);  // a multiple of 8 blocks (xcd_block)
  k_half_b<R><<<dim3(grid), dim3(256), 0, s>>>(P, E[0], E[1], E[2], B[0], B[1], B[2], h[0], h[1],
                                              h[2], ncell);
  k_advance_e<R><<<dim3(grid), dim3(256), 0, s>>>(P, M, E[0], E[1], E[2], B[0], B[1], B[2], J[0],
                                                 J[1], J[2], g[0], g[1], g[2], dt, ncell, save);
  for (int pass = 1; pass <= 2; ++pass)
    for (int d = 0; d < cf.dims; ++d) {
      if (!P.open[d]) continue;
      const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
      const long plane = (long)P.n[a] * P.n[b];
      const R kappa = (R)((cf.dt - cf.dx[d]) / (cf.dt + cf.dx[d]));
      for (int sd = 0; sd < 2; ++sd)
        k_mur<R><<<dim3((unsigned)((2 * plane + 255) / 256)), dim3(256), 0, s>>>(
            P, M, E[0], E[1], E[2], d, sd, pass, kappa, save);
    }
  k_half_b<R><<<dim3(grid), dim3(256), 0, s>>>(P, E[0], E[1], E[2], B[0], B[1], B[2], h[0], h[1],
                                              h[2], ncell);
  return (int)hipGetLastError();
}

int launch_field_advance(const pic_ctx* ctx, const pic_fields* f, void* ws, hipStream_t s) {
  char* save = (char*)ws + ws_layout(ctx, 0).mur;
  return ctx->cfg.real_bytes == 8 ? launch_fa<double>(ctx, f, (double*)save, s)
                                  : launch_fa<float>(ctx, f, (float*)save, s);
}

// Scratch of pic_field_advance_static: the saved E planes next to open
// faces, in a file-scope device array instead of the caller's workspace
// (one copy per GPU the library runs on, held until the process ends).  In
// host code `scratch` is only a host-side stand-in for the symbol; its
// device address on each GPU comes from hipGetSymbolAddress, taken once per
// device with that device current and kept in static_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];
static void* static_scratch_ptr[MAX_DEVICES];
static std::mutex static_scratch_mu;

int static_scratch_init(int device) {
  if (device < 0 || device >= MAX_DEVICES) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(static_scratch_mu);
  if (static_scratch_ptr[device]) return 0;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return e != hipSuccess ? (int)e : (int)hipErrorInvalidSymbol;
  static_scratch_ptr[device] = ptr;
  return 0;
}

int launch_field_advance_static(const pic_ctx* ctx, const pic_fields* f, hipStream_t s) {
  void* save = nullptr;
  {
    std::lock_guard<std::mutex> lock(static_scratch_mu);
    if (ctx->device >= 0 && ctx->device < MAX_DEVICES) save = static_scratch_ptr[ctx->device];
  }
  if (!save) return (int)hipErrorNotInitialized;
  return ctx->cfg.real_bytes == 8 ? launch_fa<double>(ctx, f, (double*)save, s)
                                  : launch_fa<float>(ctx, f, (float*)save, s);
}

// ------------------------------------------------------------------ adjoint
// Transpose of the field advance (for the hand-written adjoint of the step).
// The advance is linear in (E, B, J); with mu the adjoint of E^{n+1} after
// the last half step, its transpose is, in reverse order:
//   lamE -= h C^T mask(lamB)                      (the last half step)
//   Mur updates transposed, edge pass then face pass
//   lamB += dt C mu_interior;  lamJ = -dt mu_interior
//   lamE = mu (+ the direct F1^n terms of Mur);   lamE -= h C^T mask(lamB)
// where mask() keeps the B samples inside the domain (the only ones the
// forward updates or reads) and mu_interior keeps the E samples advanced by
// the Yee update.

// lamE -= h C^T lamB over every E sample, lamB read only inside the domain.
template <typename R>
__global__ void k_adj_curl_b(FdParams P, R* __restrict__ L0, R* __restrict__ L1, R* __restrict__ L2,
                             const R* __restrict__ B0, const R* __restrict__ B1,
                             const R* __restrict__ B2, R gx, R gy, R gz, int ncell) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ncell) return;
  int i, j, k;
  decompose(P, idx, i, j, k);
  R* Lm[3] = {L0, L1, L2};
  const R* B[3] = {B0, B1, B2};
  const R g[3] = {gx, gy, gz};  // h / dx_d
  auto bval = [&](int comp, int ii, int jj, int kk, int d, int step) -> R {
    int Lc[3] = {ii, jj, kk};
    Lc[d] += step;
    if (Lc[d] < 0 || Lc[d] >= P.n[d]) {
      if (P.open[d]) return R(0);
      Lc[d] = Lc[d] < 0 ? Lc[d] + P.n[d] : Lc[d] - P.n[d];
    }
    if (!inside(P, Lc[0], Lc[1], Lc[2], comp != 0, comp != 1, comp != 2)) return R(0);
    return B[comp][Lc[0] + P.n[0] * (Lc[1] + P.n[1] * Lc[2])];
  };
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    R curl = R(0);
    if (a < P.dims) curl += g[a] * (bval(b, i, j, k, a, 0) - bval(b, i, j, k, a, -1));
    if (b < P.dims) curl -= g[b] * (bval(a, i, j, k, b, 0) - bval(a, i, j, k, b, -1));
    Lm[c][idx] -= curl;
  }
}

// Mur transpose for the samples of face (d, side) with `pass` open
// boundary axes: mu[s1] += kappa mu[s0]; extra[s1] += mu[s0]; the sample's
// own adjoint becomes -kappa mu[s0] (+ what it received as a neighbour,
// kept in extra).  Runs for pass 2, then pass 1.
template <typename R>
__global__ void k_adj_mur(FdParams P, R* __restrict__ M0, R* __restrict__ M1, R* __restrict__ M2,
                          R* __restrict__ X0, R* __restrict__ X1, R* __restrict__ X2, int d,
                          int side, int pass, R kappa) {
  const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
  const int na = P.n[a], nbv = b < P.dims ? P.n[b] : 1;
  const long plane = (long)na * nbv;
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= 2 * plane) return;
  const int which = (int)(t / plane);
  const long r = t - which * plane;
  const int c = (d + 1 + which) % 3;
  int L[3];
  L[d] = side ? P.n[d] - 1 : 0;
  L[a] = (int)(r % na);
  L[b] = (int)(r / na);
  if (!inside(P, L[0], L[1], L[2], c == 0, c == 1, c == 2)) return;
  int lowest;
  if (mur_axes(P, c, L[0], L[1], L[2], lowest) != pass || lowest != d) return;
  R* M[3] = {M0, M1, M2};
  R* X[3] = {X0, X1, X2};
  const int i0 = L[0] + P.n[0] * (L[1] + P.n[1] * L[2]);
  int N[3] = {L[0], L[1], L[2]};
  N[d] += side ? -1 : 1;
  const int i1 = N[0] + P.n[0] * (N[1] + P.n[1] * N[2]);
  const R mu0 = M[c][i0];
  M[c][i1] += kappa * mu0;
  X[c][i1] += mu0;
  M[c][i0] = -kappa * mu0 + X[c][i0];
  X[c][i0] = R(0);
}

// lamB += dt C mu over the inside B samples, mu read on the E samples the
// Yee update advances (interior ones).
template <typename R>
__global__ void k_adj_curl_e(FdParams P, const R* __restrict__ M0, const R* __restrict__ M1,
                             const R* __restrict__ M2, R* __restrict__ B0, R* __restrict__ B1,
                             R* __restrict__ B2, R gx, R gy, R gz, int ncell) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ncell) return;
  int i, j, k;
  decompose(P, idx, i, j, k);
  const R* M[3] = {M0, M1, M2};
  R* B[3] = {B0, B1, B2};
  const R g[3] = {gx, gy, gz};  // dt / dx_d
  auto muval = [&](int comp, int ii, int jj, int kk, int d, int step) -> R {
    int Lc[3] = {ii, jj, kk};
    Lc[d] += step;
    if (Lc[d] < 0 || Lc[d] >= P.n[d]) {
      if (P.open[d]) return R(0);
      Lc[d] = Lc[d] < 0 ? Lc[d] + P.n[d] : Lc[d] - P.n[d];
    }
    if (!inside(P, Lc[0], Lc[1], Lc[2], comp == 0, comp == 1, comp == 2)) return R(0);
    int lowest;
    if (mur_axes(P, comp, Lc[0], Lc[1], Lc[2], lowest) > 0) return R(0);
    return M[comp][Lc[0] + P.n[0] * (Lc[1] + P.n[1] * Lc[2])];
  };
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (!inside(P, i, j, k, c != 0, c != 1, c != 2)) continue;
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    R acc = R(0);
    if (a < P.dims) acc += g[a] * (muval(b, i, j, k, a, 1) - muval(b, i, j, k, a, 0));
    if (b < P.dims) acc -= g[b] * (muval(a, i, j, k, b, 1) - muval(a, i, j, k, b, 0));
    B[c][idx] += acc;
  }
}

// lamJ = -dt mu on interior E samples (0 elsewhere); lamE = mu + extra there.
template <typename R>
__global__ void k_adj_e_out(FdParams P, R* __restrict__ M0, R* __restrict__ M1, R* __restrict__ M2,
                            R* __restrict__ J0, R* __restrict__ J1, R* __restrict__ J2,
                            R* __restrict__ X0, R* __restrict__ X1, R* __restrict__ X2, R dt,
                            int ncell, int has_extra) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ncell) return;
  int i, j, k;
  decompose(P, idx, i, j, k);
  R* M[3] = {M0, M1, M2};
  R* J[3] = {J0, J1, J2};
  R* X[3] = {X0, X1, X2};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    int lowest;
    const bool yee = inside(P, i, j, k, c == 0, c == 1, c == 2) && mur_axes(P, c, i, j, k, lowest) == 0;
    if (yee) {
      J[c][idx] = -dt * M[c][idx];
      if (has_extra) {
        M[c][idx] += X[c][idx];
        X[c][idx] = R(0);
      }
    } else {
      J[c][idx] = R(0);
    }
  }
}

template <typename R>
static int launch_fa_adj(const pic_ctx* ctx, const pic_fields* lam, void* ws, hipStream_t s) {
  const pic_config& cf = ctx->cfg;
  FdParams P;
  P.dims = cf.dims;
  bool any_open = false;
  for (int d = 0; d < 3; ++d) {
    P.n[d] = d < cf.dims ? cf.n[d] : 1;
    P.open[d] = d < cf.dims && cf.bc[d] == PIC_BC_OPEN;
    any_open = any_open || P.open[d];
  }
  P.dn0.init((uint32_t)P.n[0]);
  P.dn1.init((uint32_t)P.n[1]);
  const int ncell = P.n[0] * P.n[1] * P.n[2];
  R h[3], g[3];
  for (int d = 0; d < 3; ++d) {
    h[d] = (R)(0.5 * cf.dt / cf.dx[d]);
    g[d] = (R)(cf.dt / cf.dx[d]);
  }
  R* E[3];
  R* B[3];
  R* J[3];
  for (int c = 0; c < 3; ++c) {
    E[c] = (R*)lam->E[c];
    B[c] = (R*)lam->B[c];
    J[c] = (R*)lam->J[c];
  }
  WsLayout L = ws_layout(ctx, 0);
  R* extra = (R*)((char*)ws + L.adj);
  R* X[3] = {extra, extra + ncell, extra + 2 * (long)ncell};
  const unsigned grid = (unsigned)((ncell + 255) / 256);
  k_adj_curl_b<R><<<dim3(grid), dim3(256), 0, s>>>(P, E[0], E[1], E[2], B[0], B[1], B[2], h[0],
                                                  h[1], h[2], ncell);
  if (any_open) {
    k_fill3_zero<R><<<dim3(grid < 4096 ? grid : 4096), dim3(256), 0, s>>>(X[0], X[1], X[2], ncell);
    for (int pass = 2; pass >= 1; --pass)
      for (int d = 0; d < cf.dims; ++d) {
        if (!P.open[d]) continue;
        const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
        const long plane = (long)P.n[a] * P.n[b];
        const R kappa = (R)((cf.dt - cf.dx[d]) / (cf.dt + cf.dx[d]));
        for (int sd = 0; sd < 2; ++sd)
          k_adj_mur<R><<<dim3((unsigned)((2 * plane + 255) / 256)), dim3(256), 0, s>>>(
              P, E[0], E[1], E[2], X[0], X[1], X[2], d, sd, pass, kappa);
      }
  }
  k_adj_curl_e<R><<<dim3(grid), dim3(256), 0, s>>>(P, E[0], E[1], E[2], B[0], B[1], B[2], g[0],
                                                  g[1], g[2], ncell);
  k_adj_e_out<R><<<dim3(grid), dim3(256), 0, s>>>(P, E[0], E[1], E[2], J[0], J[1], J[2], X[0],
                                                 X[1], X[2], (R)cf.dt, ncell, any_open ? 1 : 0);
  k_adj_curl_b<R><<<dim3(grid), dim3(256), 0, s>>>(P, E[0], E[1], E[2], B[0], B[1], B[2], h[0],
                                                  h[1], h[2], ncell);
  return (int)hipGetLastError();
}

int launch_field_advance_adjoint(const pic_ctx* ctx, const pic_fields* lam, void* ws, hipStream_t s) {
  return ctx->cfg.real_bytes == 8 ? launch_fa_adj<double>(ctx, lam, ws, s)
                                  : launch_fa_adj<float>(ctx, lam, ws, s);
}

// Size (in reals) of the adjoint's scratch (open axes only).
long adj_len(const pic_config& cf) {
  bool open = false;
  long ncell = 1;
  for (int d = 0; d < cf.dims; ++d) {
    open = open || cf.bc[d] == PIC_BC_OPEN;
    ncell *= cf.n[d];
  }
  return open ? 3 * ncell : 0;
}

// Size (in reals) of the Mur save buffer.
long mur_len(const pic_config& cf) {
  long len = 0;
  int n[3];
  for (int d = 0; d < 3; ++d) n[d] = d < cf.dims ? cf.n[d] : 1;
  for (int d = 0; d < cf.dims; ++d) {
    if (cf.bc[d] != PIC_BC_OPEN) continue;
    const int a = d == 0 ? 1 : 0, b = d == 2 ? 1 : 2;
    len += 2L * 2L * n[a] * n[b];
  }
  return len;
}

}  // namespace pic
