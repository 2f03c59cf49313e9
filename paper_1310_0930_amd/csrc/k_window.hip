// Moving window and laser antenna.
//
// The paper's LWFA runs follow the laser with a window that moves through
// the plasma (Sec. 2).  Here the window moves in whole cells along x: the
// fields shift one cell toward -x (the plane entering at the front is
// empty), particles keep their offsets and move one cell down (those leaving
// at the back are absorbed), and new plasma particles are appended in the
// front column from caller-provided draws.  The laser enters as the field of
// a current sheet on one plane of E samples (a sheet current K radiates
// E = -K/2 on both sides).
#include "k_common.h"

namespace pic {

// Shift by one cell toward -x, row by row: a workgroup owns whole x-rows and
// walks each in chunks; every chunk reads F[x+1] before the barrier and
// writes F[x] after it, and the next chunk reads only beyond what this one
// wrote, so the in-place shift is race-free.  The last sample of a row gets
// zero.  Rows of the three J components are zeroed.
template <typename R>
__global__ void __launch_bounds__(256) k_shift_rows(DFields<R> F, int n0, long nrows) {
  const long task = blockIdx.x;  // component * nrows + row
  const int comp = (int)(task / nrows);
  const long row = task - (long)comp * nrows;
  R* f = comp < 3 ? F.E[comp] : comp < 6 ? F.B[comp - 3] : F.J[comp - 6];
  R* r = f + row * (long)n0;
  for (int c0 = 0; c0 < n0; c0 += blockDim.x) {
    const int x = c0 + (int)threadIdx.x;
    R v = R(0);
    if (comp < 6 && x + 1 < n0) v = r[x + 1];
    __syncthreads();
    if (x < n0) r[x] = v;
    __syncthreads();
  }
}

// Cells move one cell down in x; x = 0 leaves the window (absorbed).
__global__ void k_shift_cells(int* __restrict__ cell, long np, FastDiv dn0) {
  for (long p = blockIdx.x * (long)blockDim.x + threadIdx.x; p < np; p += (long)gridDim.x * blockDim.x) {
    const int c = cell[p];
    if (c < 0) continue;
    const uint32_t rest = dn0.div((uint32_t)c);
    const int x = c - (int)(rest * dn0.d);
    cell[p] = x == 0 ? -1 : c - 1;
  }
}

// Append the front column's particles after the np existing ones (ids
// id_first, id_first + 1, ...).
template <typename R>
__global__ void k_inject(DParts<R> pa, long np, int dims, int n0, int n1, int ncy, int xcol,
                         const R* __restrict__ o0, const R* __restrict__ o1,
                         const R* __restrict__ o2, const R* __restrict__ u0,
                         const R* __restrict__ u1, const R* __restrict__ u2,
                         const R* __restrict__ qin, long n, int ppc, long id_first) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const long col = i / ppc;
    const int cy = (int)(col % ncy);
    const int cz = dims == 3 ? (int)(col / ncy) : 0;
    const long dst = np + i;
    pa.cell[dst] = xcol + n0 * (cy + n1 * cz);
    pa.off[0][dst] = o0[i];
    pa.off[1][dst] = o1[i];
    if (dims == 3) pa.off[2][dst] = o2[i];
    pa.u[0][dst] = u0[i];
    pa.u[1][dst] = u1[i];
    pa.u[2][dst] = u2[i];
    if (pa.q) pa.q[dst] = qin[i];
    if (pa.id) pa.id[dst] = (int32_t)(id_first + i);
  }
}

// Antenna current on the plane x = xi (one thread per (y, z) sample),
// computed in double and added in the working precision.
struct AntParams {
  int xi, pol, dims;
  int n[3], open[3];
  double dx[3];
  double amp;  // -2 a0 omega0 / dx_0 * env(t) * cos(omega0 (t - t_center))
  double yc, zc, inv_w2;
};

template <typename R>
__global__ void k_antenna(AntParams A, R* __restrict__ J) {
  const long m = (long)A.n[1] * (A.dims == 3 ? A.n[2] : 1);
  for (long s = blockIdx.x * (long)blockDim.x + threadIdx.x; s < m; s += (long)gridDim.x * blockDim.x) {
    const int j = (int)(s % A.n[1]);
    const int k = A.dims == 3 ? (int)(s / A.n[1]) : 0;
    // J_y sits half a cell up in y, J_z half a cell up in z
    const int sy = A.pol == 1, sz = A.pol == 2;
    if (A.open[1] && j > A.n[1] - 1 - sy) continue;
    if (A.dims == 3 && A.open[2] && k > A.n[2] - 1 - sz) continue;
    const double y = (j + 0.5 * sy) * A.dx[1] - A.yc;
    const double z = A.dims == 3 ? (k + 0.5 * sz) * A.dx[2] - A.zc : 0.0;
    const double v = A.amp * exp(-(y * y + z * z) * A.inv_w2);
    const long idx = A.xi + (long)A.n[0] * (j + (long)A.n[1] * k);
    J[idx] = (R)((double)J[idx] + v);
  }
}

template <typename R>
static int window_t(const pic_ctx* ctx, pic_particles* p, const pic_fields* f,
                    const pic_inject* in, hipStream_t s) {
  const pic_config& c = ctx->cfg;
  const int n0 = c.n[0], n1 = c.n[1], n2 = c.dims == 3 ? c.n[2] : 1;
  if (f) {  // NULL: a further species, the fields have moved already
    DFields<R> F;
    for (int k = 0; k < 3; ++k) {
      F.E[k] = (R*)f->E[k];
      F.B[k] = (R*)f->B[k];
      F.J[k] = (R*)f->J[k];
    }
    const long nrows = (long)n1 * n2;
    k_shift_rows<R><<<dim3((unsigned)(9 * nrows)), dim3(256), 0, s>>>(F, n0, nrows);
  }
  const long np = p->np;
  if (np > 0) {
    FastDiv dn0;
    dn0.init((uint32_t)n0);
    const long g = (np + 255) / 256;
    k_shift_cells<<<dim3((unsigned)(g < 8192 ? g : 8192)), dim3(256), 0, s>>>(p->cell, np, dn0);
  }
  if (in && in->n > 0) {
    DParts<R> pa;
    pa.cell = p->cell;
    for (int d = 0; d < 3; ++d) {
      pa.off[d] = (R*)p->off[d];
      pa.u[d] = (R*)p->u[d];
    }
    pa.q = (R*)p->q;
    pa.id = p->id;
    const int ncy = n1 - (c.bc[1] == PIC_BC_OPEN ? 1 : 0);
    const long g = (in->n + 255) / 256;
    k_inject<R><<<dim3((unsigned)(g < 8192 ? g : 8192)), dim3(256), 0, s>>>(
        pa, np, c.dims, n0, n1, ncy, n0 - 2, (const R*)in->off[0], (const R*)in->off[1],
        (const R*)in->off[2], (const R*)in->u[0], (const R*)in->u[1], (const R*)in->u[2],
        (const R*)in->q, in->n, in->ppc, (long)in->id_first);
  }
  return (int)hipGetLastError();
}

int launch_window_shift(const pic_ctx* ctx, pic_particles* p, const pic_fields* f,
                        const pic_inject* in, hipStream_t s) {
  return ctx->cfg.real_bytes == 8 ? window_t<double>(ctx, p, f, in, s)
                                  : window_t<float>(ctx, p, f, in, s);
}

int launch_antenna(const pic_ctx* ctx, const pic_fields* f, const pic_antenna* a, double t,
                   hipStream_t s) {
  const pic_config& c = ctx->cfg;
  const double tr = t - a->t_center;
  if (fabs(tr) > 3.0 * a->tau) return 0;  // the pulse is cut beyond 3 tau
  AntParams A;
  A.xi = a->x_index;
  A.pol = a->polarization;
  A.dims = c.dims;
  for (int d = 0; d < 3; ++d) {
    A.n[d] = d < c.dims ? c.n[d] : 1;
    A.open[d] = d < c.dims && c.bc[d] == PIC_BC_OPEN;
    A.dx[d] = c.dx[d];
  }
  A.amp = -2.0 * a->a0 * a->omega0 / c.dx[0] * exp(-tr * tr / (a->tau * a->tau)) *
          cos(a->omega0 * tr);
  A.yc = a->y_center;
  A.zc = a->z_center;
  A.inv_w2 = 1.0 / (a->waist * a->waist);
  const long m = (long)A.n[1] * A.n[2];
  const unsigned g = (unsigned)((m + 255) / 256 < 4096 ? (m + 255) / 256 : 4096);
  if (c.real_bytes == 8)
    k_antenna<double><<<dim3(g), dim3(256), 0, s>>>(A, (double*)f->J[a->polarization]);
  else
    k_antenna<float><<<dim3(g), dim3(256), 0, s>>>(A, (float*)f->J[a->polarization]);
  return (int)hipGetLastError();
}

}  // namespace pic
