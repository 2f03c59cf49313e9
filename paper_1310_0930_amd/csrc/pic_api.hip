// C ABI of libpic: argument validation, workspace layout and dispatch.
// Validation happens on the host before any HIP call, so configuration
// errors are reported the same way with or without a device.
#include <cstddef>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>

#include "pic_internal.h"

namespace pic {
long mur_len(const pic_config& cf);
long diag_len(const pic_config& cf);
long adj_len(const pic_config& cf);

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

WsLayout ws_layout(const pic_ctx* ctx, int64_t np) {
  const size_t R = (size_t)ctx->cfg.real_bytes;
  WsLayout L;
  size_t off = 0;
  L.flags = off;
  off = align256(off + sizeof(DevFlags));
  const size_t nbins = (size_t)ctx->ntiles + 1;
  L.starts = off;
  off = align256(off + sizeof(int) * ((size_t)ctx->ntiles + 2));
  L.counts = off;
  off = align256(off + sizeof(int) * nbins);
  L.bstart = off;
  off = align256(off + sizeof(int) * (nbins + 1));
  L.bsum = off;
  off = align256(off + sizeof(int) * (nbins / 1024 + 1));
  L.rb_tv = off;
  off = align256(off + sizeof(int) * (size_t)ctx->ntiles);
  L.rb_nl = off;
  off = align256(off + sizeof(int) * (size_t)ctx->ntiles);
  L.mur_len = (size_t)mur_len(ctx->cfg);
  L.mur = off;
  off = align256(off + R * L.mur_len);
  L.diag_len = (size_t)diag_len(ctx->cfg);
  L.diag = off;
  off = align256(off + sizeof(double) * L.diag_len);
  L.adj_len = (size_t)adj_len(ctx->cfg);
  L.adj = off;
  off = align256(off + R * L.adj_len);
  const size_t n = np > 0 ? (size_t)np : 0;
  L.tmp_cell = off;
  off = align256(off + sizeof(int) * n);
  L.tmp_id = off;
  off = align256(off + sizeof(int) * n);
  L.keys = off;
  off = align256(off + sizeof(int) * n);
  L.pkey = off;
  off = align256(off + sizeof(int) * n);
  L.order = off;
  off = align256(off + sizeof(int) * 1024);
  L.tmp_real = off;
  off = align256(off + R * 7 * n);
  L.total = off;
  return L;
}

template <typename R>
KParams<R> make_params(const pic_ctx* ctx) {
  const pic_config& c = ctx->cfg;
  KParams<R> P;
  P.dims = c.dims;
  P.order = c.order;
  for (int d = 0; d < 3; ++d) {
    P.n[d] = d < c.dims ? c.n[d] : 1;
    P.bc[d] = d < c.dims ? c.bc[d] : PIC_BC_PERIODIC;
    P.tile[d] = ctx->tile[d];
    P.ntile[d] = ctx->ntile[d];
    P.dtdx[d] = (R)(d < c.dims ? c.dt / c.dx[d] : 0.0);
    P.jfac[d] = (R)(d < c.dims ? -c.dx[d] / c.dt : 0.0);
  }
  P.ntiles = ctx->ntiles;
  P.per_xcd = (ctx->ntiles + 7) / 8;
  P.dn0.init((uint32_t)P.n[0]);
  P.dn1.init((uint32_t)P.n[1]);
  P.hqm = (R)(0.5 * c.q_over_m * c.dt);
  P.dt = (R)c.dt;
  P.q_const = (R)c.q_const;
  return P;
}
template KParams<float> make_params<float>(const pic_ctx*);
template KParams<double> make_params<double>(const pic_ctx*);

// Compile-time tile shape and LDS need of the selected kernel.
template <int DIMS, int ORDER, typename R>
static void geo_of(int* T, int* A, size_t* lds) {
  using G = Geo<DIMS, ORDER, R>;
  T[0] = T[1] = G::T;
  T[2] = G::TZ;
  *A = G::A;
  *lds = G::lds_bytes;
}

static int kernel_geometry(const pic_config* c, int* T, int* A, size_t* lds) {
  const bool dbl = c->real_bytes == 8;
#define PIC_GEO(DD, OO)                                                 \
  if (c->dims == DD && c->order == OO) {                                \
    if (dbl)                                                            \
      geo_of<DD, OO, double>(T, A, lds);                                \
    else                                                                \
      geo_of<DD, OO, float>(T, A, lds);                                 \
    return 0;                                                           \
  }
  PIC_GEO(2, 1) PIC_GEO(2, 2) PIC_GEO(2, 3) PIC_GEO(2, 4)
  PIC_GEO(3, 1) PIC_GEO(3, 2) PIC_GEO(3, 3) PIC_GEO(3, 4)
#undef PIC_GEO
  return -1;
}

}  // namespace pic

using namespace pic;

static bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

static int validate_config(const pic_config* c) {
  if (!c) return PIC_EINVAL;
  if (c->dims != 2 && c->dims != 3) return PIC_EINVAL;
  if (c->order < 1 || c->order > 4) return PIC_EINVAL;
  if (c->real_bytes != 4 && c->real_bytes != 8) return PIC_EINVAL;
  if (c->sort_every < 1) return PIC_EINVAL;
  if (!isfinite(c->q_over_m) || !isfinite(c->q_const)) return PIC_EINVAL;
  double ncell = 1.0;
  for (int d = 0; d < c->dims; ++d) {
    if (c->bc[d] != PIC_BC_PERIODIC && c->bc[d] != PIC_BC_OPEN) return PIC_EINVAL;
    if (c->n[d] < (c->bc[d] == PIC_BC_OPEN ? 4 : 2)) return PIC_EINVAL;
    if (!finite_pos(c->dx[d])) return PIC_EINVAL;
    ncell *= (double)c->n[d];
  }
  if (c->dims == 2 && c->n[2] != 1) return PIC_EINVAL;
  if (ncell >= 2147483647.0) return PIC_EINVAL;
  if (!finite_pos(c->dt)) return PIC_EINVAL;
  double s = 0.0;
  for (int d = 0; d < c->dims; ++d) s += 1.0 / (c->dx[d] * c->dx[d]);
  if (c->dt > (1.0 + 1e-12) / sqrt(s)) return PIC_ECOURANT;
  int T[3], A;
  size_t lds;
  if (kernel_geometry(c, T, &A, &lds) != 0) return PIC_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (c->tile[d] != 0 && c->tile[d] != T[d]) return PIC_EINVAL;
  if (c->drift >= 0 && c->drift != A) return PIC_EINVAL;
  if (lds > 160 * 1024) return PIC_ELDS;
  return PIC_OK;
}

extern "C" {

int pic_create(const pic_config* cfg, pic_ctx** out) {
  if (!out) return PIC_EINVAL;
  *out = nullptr;
  const int v = validate_config(cfg);
  if (v != PIC_OK) return v;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PIC_EHIP;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return PIC_EHIP;
  if (static_scratch_init(dev) != 0) return PIC_EHIP;  // pic_field_advance_static's scratch
  pic_ctx* ctx = new (std::nothrow) pic_ctx();
  if (!ctx) return PIC_EHIP;
  ctx->cfg = *cfg;
  if (cfg->dims == 2) {
    ctx->cfg.n[2] = 1;
    ctx->cfg.dx[2] = 1.0;
    ctx->cfg.bc[2] = PIC_BC_PERIODIC;
  }
  ctx->device = dev;
  ctx->cu_count = cus;
  int T[3], A;
  size_t lds;
  kernel_geometry(cfg, T, &A, &lds);
  ctx->ntiles = 1;
  for (int d = 0; d < 3; ++d) {
    ctx->tile[d] = T[d];
    const int n = d < cfg->dims ? cfg->n[d] : 1;
    ctx->ntile[d] = (n + T[d] - 1) / T[d];
    ctx->ntiles *= ctx->ntile[d];
  }
  ctx->cfg.tile[0] = T[0];
  ctx->cfg.tile[1] = T[1];
  ctx->cfg.tile[2] = T[2];
  ctx->cfg.drift = A;
  ctx->steps_done = 0;
  ctx->rebin = true;
  ctx->pushes_since_sort = 0;
  ctx->sorted_cell = nullptr;
  ctx->sorted_ws = nullptr;
  ctx->sorted_np = -1;
  ctx->antenna_on = false;
  memset(&ctx->antenna, 0, sizeof(ctx->antenna));
  *out = ctx;
  return PIC_OK;
}

int pic_destroy(pic_ctx* ctx) {
  delete ctx;
  return PIC_OK;
}

int pic_workspace_bytes(const pic_ctx* ctx, int64_t np, size_t* bytes) {
  if (!ctx || !bytes || np < 0 || np >= 2147483647LL) return PIC_EINVAL;
  *bytes = ws_layout(ctx, np).total;
  return PIC_OK;
}

static int check_particles(const pic_ctx* ctx, const pic_particles* p) {
  if (!p || p->np < 0 || p->np >= 2147483647LL) return PIC_EINVAL;
  if (p->np == 0) return PIC_OK;
  if (!p->cell) return PIC_EINVAL;
  for (int d = 0; d < ctx->cfg.dims; ++d)
    if (!p->off[d]) return PIC_EINVAL;
  for (int c = 0; c < 3; ++c)
    if (!p->u[c]) return PIC_EINVAL;
  return PIC_OK;
}

static int check_fields(const pic_fields* f, bool need_j) {
  if (!f) return PIC_EINVAL;
  for (int c = 0; c < 3; ++c) {
    if (!f->E[c] || !f->B[c]) return PIC_EINVAL;
    if (need_j && !f->J[c]) return PIC_EINVAL;
  }
  return PIC_OK;
}

static int hip_status(int err) { return err == 0 ? PIC_OK : PIC_EHIP; }

static int ensure_device(const pic_ctx* ctx) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return PIC_EHIP;
  if (dev != ctx->device && hipSetDevice(ctx->device) != hipSuccess) return PIC_EHIP;
  return PIC_OK;
}

int pic_sort(pic_ctx* ctx, pic_particles* p, void* ws, void* stream) {
  if (!ctx || !ws) return PIC_EINVAL;
  int v = check_particles(ctx, p);
  if (v) return v;
  if ((v = ensure_device(ctx))) return v;
  // Whether the pushes since the previous sort (in this workspace) left any
  // particle outside the sorted tile pass: read before the sort clears the
  // count, alongside the live count's read-back below.
  const bool judge = ctx->pushes_since_sort > 0 && ctx->sorted_ws == ws && p->np > 0;
  DevFlags fh;
  hipStream_t s = (hipStream_t)stream;
  if (judge && hipMemcpyAsync(&fh, ws, sizeof(fh), hipMemcpyDeviceToHost, s) != hipSuccess)
    return PIC_EHIP;
  ctx->sorted_cell = nullptr;  // bins are valid only once the sort has completed
  v = hip_status(launch_sort(ctx, p, ws, s));
  if (v != PIC_OK) return v;
  if (p->np > 0) {
    // compaction: the dead bin starts at the live count, which becomes np
    int32_t live = 0;
    const WsLayout L = ws_layout(ctx, p->np);
    if (hipMemcpyAsync(&live, (const char*)ws + L.starts + sizeof(int32_t) * (size_t)ctx->ntiles,
                       sizeof(live), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return PIC_EHIP;
    if (live < 0 || live > p->np) return PIC_EHIP;
    p->np = live;
  }
  if (judge) ctx->rebin = fh.since_sort + fh.ndefer > 0;
  ctx->pushes_since_sort = 0;
  ctx->sorted_cell = p->cell;
  ctx->sorted_ws = ws;
  ctx->sorted_np = p->np;
  return PIC_OK;
}

int pic_push_deposit(pic_ctx* ctx, pic_particles* p, const pic_fields* f, void* ws, void* stream) {
  if (!ctx || !ws) return PIC_EINVAL;
  int v = check_particles(ctx, p);
  if (v) return v;
  if ((v = check_fields(f, true))) return v;
  if (ctx->sorted_cell != p->cell || ctx->sorted_ws != ws || ctx->sorted_np != p->np)
    return PIC_ESTATE;
  if ((v = ensure_device(ctx))) return v;
  ctx->pushes_since_sort += 1;
  return hip_status(launch_push_deposit(ctx, p, f, ws, (hipStream_t)stream, false));
}

int pic_push_deposit_add(pic_ctx* ctx, pic_particles* p, const pic_fields* f, void* ws,
                         void* stream) {
  if (!ctx || !ws) return PIC_EINVAL;
  int v = check_particles(ctx, p);
  if (v) return v;
  if ((v = check_fields(f, true))) return v;
  if (ctx->sorted_cell != p->cell || ctx->sorted_ws != ws || ctx->sorted_np != p->np)
    return PIC_ESTATE;
  if ((v = ensure_device(ctx))) return v;
  ctx->pushes_since_sort += 1;
  return hip_status(launch_push_deposit(ctx, p, f, ws, (hipStream_t)stream, true));
}

int pic_field_advance(pic_ctx* ctx, pic_fields* f, void* ws, void* stream) {
  if (!ctx || !ws) return PIC_EINVAL;
  int v = check_fields(f, true);
  if (v) return v;
  if ((v = ensure_device(ctx))) return v;
  return hip_status(launch_field_advance(ctx, f, ws, (hipStream_t)stream));
}

int pic_field_advance_static(pic_ctx* ctx, pic_fields* f, void* stream) {
  if (!ctx) return PIC_EINVAL;
  int v = check_fields(f, true);
  if (v) return v;
  if ((size_t)mur_len(ctx->cfg) * (size_t)ctx->cfg.real_bytes > STATIC_SCRATCH_BYTES)
    return PIC_ESCRATCH;
  if ((v = ensure_device(ctx))) return v;
  return hip_status(launch_field_advance_static(ctx, f, (hipStream_t)stream));
}

int pic_step(pic_ctx* ctx, pic_particles* p, pic_fields* f, int32_t nsteps, void* ws, void* stream) {
  if (!ctx || !ws || nsteps < 0) return PIC_EINVAL;
  int v = check_particles(ctx, p);
  if (v) return v;
  if ((v = check_fields(f, true))) return v;
  for (int32_t s = 0; s < nsteps; ++s) {
    const bool sorted = ctx->sorted_cell == p->cell && ctx->sorted_ws == ws && ctx->sorted_np == p->np;
    if (!sorted || ctx->steps_done % ctx->cfg.sort_every == 0) {
      if ((v = pic_sort(ctx, p, ws, stream))) return v;
    }
    if ((v = pic_push_deposit(ctx, p, f, ws, stream))) return v;
    if (ctx->antenna_on &&
        (v = pic_antenna_add(ctx, f, &ctx->antenna, (ctx->steps_done + 0.5) * ctx->cfg.dt, stream)))
      return v;
    if ((v = pic_field_advance(ctx, f, ws, stream))) return v;
    ctx->steps_done += 1;
  }
  return PIC_OK;
}

static int check_antenna(const pic_ctx* ctx, const pic_antenna* a) {
  if (!a) return PIC_EINVAL;
  const pic_config& c = ctx->cfg;
  if (a->polarization != 1 && a->polarization != 2) return PIC_EINVAL;
  if (a->x_index < 0 || a->x_index >= c.n[0]) return PIC_EINVAL;
  if (!(a->tau > 0.0) || !(a->waist > 0.0) || !isfinite(a->tau) || !isfinite(a->waist))
    return PIC_EINVAL;
  if (!isfinite(a->a0) || !isfinite(a->omega0) || !isfinite(a->t_center) ||
      !isfinite(a->y_center) || !isfinite(a->z_center))
    return PIC_EINVAL;
  return PIC_OK;
}

int pic_antenna_add(pic_ctx* ctx, pic_fields* f, const pic_antenna* a, double t, void* stream) {
  if (!ctx || !f || !f->J[0] || !f->J[1] || !f->J[2] || !isfinite(t)) return PIC_EINVAL;
  int v = check_antenna(ctx, a);
  if (v) return v;
  if ((v = ensure_device(ctx))) return v;
  return hip_status(launch_antenna(ctx, f, a, t, (hipStream_t)stream));
}

int pic_set_antenna(pic_ctx* ctx, const pic_antenna* a) {
  if (!ctx) return PIC_EINVAL;
  if (!a) {
    ctx->antenna_on = false;
    return PIC_OK;
  }
  int v = check_antenna(ctx, a);
  if (v) return v;
  ctx->antenna = *a;
  ctx->antenna_on = true;
  return PIC_OK;
}

int pic_window_shift(pic_ctx* ctx, pic_particles* p, int64_t capacity, pic_fields* f,
                     const pic_inject* in, void* ws, void* stream) {
  if (!ctx || !ws) return PIC_EINVAL;
  int v = check_particles(ctx, p);
  if (v) return v;
  if (f && (v = check_fields(f, true))) return v;
  const pic_config& c = ctx->cfg;
  if (c.bc[0] != PIC_BC_OPEN) return PIC_EINVAL;  // the window moves along an open x axis
  const int64_t n = in ? in->n : 0;
  if (n < 0 || capacity < p->np + n || capacity >= 2147483647LL) return PIC_EINVAL;
  if (n > 0) {
    const int64_t ncy = c.n[1] - (c.bc[1] == PIC_BC_OPEN ? 1 : 0);
    const int64_t ncz = c.dims == 3 ? c.n[2] - (c.bc[2] == PIC_BC_OPEN ? 1 : 0) : 1;
    if (in->ppc < 1 || n != (int64_t)in->ppc * ncy * ncz) return PIC_EINVAL;
    for (int d = 0; d < c.dims; ++d)
      if (!in->off[d]) return PIC_EINVAL;
    for (int k = 0; k < 3; ++k)
      if (!in->u[k]) return PIC_EINVAL;
    if ((p->q != nullptr) != (in->q != nullptr)) return PIC_EINVAL;
    // appending needs the arrays even at np = 0
    if (!p->cell) return PIC_EINVAL;
    for (int d = 0; d < c.dims; ++d)
      if (!p->off[d]) return PIC_EINVAL;
    for (int k = 0; k < 3; ++k)
      if (!p->u[k]) return PIC_EINVAL;
  }
  if ((v = ensure_device(ctx))) return v;
  v = hip_status(launch_window_shift(ctx, p, f, in, (hipStream_t)stream));
  if (v) return v;
  p->np += n;
  ctx->sorted_np = -1;  // cells moved and particles were appended: sort again
  ctx->sorted_cell = nullptr;
  return PIC_OK;
}

// Species that share fields must share the grid, the time step, the shape
// order, the precision and the boundaries.
static bool same_grid(const pic_ctx* a, const pic_ctx* b) {
  const pic_config &x = a->cfg, &y = b->cfg;
  if (x.dims != y.dims || x.order != y.order || x.real_bytes != y.real_bytes || x.dt != y.dt)
    return false;
  for (int d = 0; d < x.dims; ++d)
    if (x.n[d] != y.n[d] || x.dx[d] != y.dx[d] || x.bc[d] != y.bc[d]) return false;
  return a->device == b->device;
}

static int check_species(int32_t ns, pic_ctx* const* ctx, const pic_particles* const* p,
                         void* const* ws) {
  if (ns < 1 || !ctx || !p || !ws) return PIC_EINVAL;
  for (int32_t k = 0; k < ns; ++k) {
    if (!ctx[k] || !ws[k]) return PIC_EINVAL;
    int v = check_particles(ctx[k], p[k]);
    if (v) return v;
    if (!same_grid(ctx[0], ctx[k])) return PIC_EINVAL;
    for (int32_t j = 0; j < k; ++j)
      if (ctx[j] == ctx[k] || ws[j] == ws[k]) return PIC_EINVAL;
  }
  return PIC_OK;
}

int pic_step_species(int32_t nspecies, pic_ctx* const* ctx, pic_particles* const* p,
                     void* const* ws, pic_fields* f, int32_t nsteps, void* stream) {
  if (nsteps < 0) return PIC_EINVAL;
  int v = check_species(nspecies, ctx, p, ws);
  if (v) return v;
  if ((v = check_fields(f, true))) return v;
  for (int32_t s = 0; s < nsteps; ++s) {
    for (int32_t k = 0; k < nspecies; ++k) {
      pic_ctx* c = ctx[k];
      const bool sorted = c->sorted_cell == p[k]->cell && c->sorted_ws == ws[k] &&
                          c->sorted_np == p[k]->np;
      if (!sorted || c->steps_done % c->cfg.sort_every == 0) {
        if ((v = pic_sort(c, p[k], ws[k], stream))) return v;
      }
      v = k == 0 ? pic_push_deposit(c, p[k], f, ws[k], stream)
                 : pic_push_deposit_add(c, p[k], f, ws[k], stream);
      if (v) return v;
    }
    if (ctx[0]->antenna_on &&
        (v = pic_antenna_add(ctx[0], f, &ctx[0]->antenna,
                             (ctx[0]->steps_done + 0.5) * ctx[0]->cfg.dt, stream)))
      return v;
    if ((v = pic_field_advance(ctx[0], f, ws[0], stream))) return v;
    for (int32_t k = 0; k < nspecies; ++k) ctx[k]->steps_done += 1;
  }
  return PIC_OK;
}

int pic_field_advance_adjoint(pic_ctx* ctx, pic_fields* lam, void* ws, void* stream) {
  if (!ctx || !ws) return PIC_EINVAL;
  int v = check_fields(lam, true);
  if (v) return v;
  if ((v = ensure_device(ctx))) return v;
  return hip_status(launch_field_advance_adjoint(ctx, lam, ws, (hipStream_t)stream));
}

int pic_push_deposit_adjoint(pic_ctx* ctx, const pic_particles* state_n, const pic_fields* EB_n,
                             pic_fields* lam_f, pic_particles* lam_p, void* ws, void* stream) {
  if (!ctx || !ws || !lam_p) return PIC_EINVAL;
  int v = check_particles(ctx, state_n);
  if (v) return v;
  if ((v = check_fields(EB_n, false))) return v;
  if ((v = check_fields(lam_f, true))) return v;
  if (state_n->np > 0) {
    for (int d = 0; d < ctx->cfg.dims; ++d)
      if (!lam_p->off[d]) return PIC_EINVAL;
    for (int c = 0; c < 3; ++c)
      if (!lam_p->u[c]) return PIC_EINVAL;
  }
  if ((v = ensure_device(ctx))) return v;
  return hip_status(
      launch_push_deposit_adjoint(ctx, state_n, EB_n, lam_f, lam_p, ws, (hipStream_t)stream));
}

int pic_deposit_rho(pic_ctx* ctx, const pic_particles* p, double* rho, void* ws, void* stream) {
  if (!ctx || !rho) return PIC_EINVAL;
  int v = check_particles(ctx, p);
  if (v) return v;
  if ((v = ensure_device(ctx))) return v;
  return hip_status(launch_deposit_rho(ctx, p, rho, ws, (hipStream_t)stream, false));
}

int pic_deposit_rho_add(pic_ctx* ctx, const pic_particles* p, double* rho, void* ws, void* stream) {
  if (!ctx || !rho) return PIC_EINVAL;
  int v = check_particles(ctx, p);
  if (v) return v;
  if ((v = ensure_device(ctx))) return v;
  return hip_status(launch_deposit_rho(ctx, p, rho, ws, (hipStream_t)stream, true));
}

int pic_diagnostics_species(int32_t nspecies, pic_ctx* const* ctx, const pic_particles* const* p,
                            void* const* ws, const pic_fields* f, const double* rho_prev,
                            const double* gauss_ref, double* rho_out, double* gauss_out,
                            pic_diag* out, void* stream) {
  if (!rho_out || !out) return PIC_EINVAL;
  int v = check_species(nspecies, ctx, p, ws);
  if (v) return v;
  if ((v = check_fields(f, true))) return v;
  if ((v = ensure_device(ctx[0]))) return v;
  memset(out, 0, sizeof(*out));
  v = hip_status(launch_diagnostics(nspecies, ctx, p, ws, f, rho_prev, gauss_ref, rho_out,
                                    gauss_out, out, (hipStream_t)stream));
  if (v) return v;
  for (int32_t k = 0; k < nspecies; ++k) {
    uint32_t flags = 0;
    int64_t slow = 0;
    v = pic_read_flags(ctx[k], ws[k], 0, &flags, &slow, stream);
    if (v != PIC_OK && v != PIC_EDEVICE) return v;
    out->flags |= flags;
    out->n_slowpath += slow;
  }
  return PIC_OK;
}

int pic_diagnostics(pic_ctx* ctx, const pic_particles* p, const pic_fields* f,
                    const double* rho_prev, const double* gauss_ref, double* rho_out,
                    double* gauss_out, pic_diag* out, void* ws, void* stream) {
  if (!ctx || !ws || !p) return PIC_EINVAL;
  return pic_diagnostics_species(1, &ctx, &p, &ws, f, rho_prev, gauss_ref, rho_out, gauss_out,
                                 out, stream);
}

int pic_read_flags(pic_ctx* ctx, void* ws, int clear, uint32_t* flags, int64_t* n_slowpath,
                   void* stream) {
  if (!ctx || !ws) return PIC_EINVAL;
  int v = ensure_device(ctx);
  if (v) return v;
  DevFlags h;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return PIC_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return PIC_EHIP;
  if (clear) {
    DevFlags z;
    memset(&z, 0, sizeof(z));
    if (hipMemcpyAsync(ws, &z, offsetof(DevFlags, qmax), hipMemcpyHostToDevice, s) != hipSuccess)
      return PIC_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return PIC_EHIP;
  }
  if (flags) *flags = h.flags;
  if (n_slowpath) *n_slowpath = (int64_t)h.slowpath;
  return h.flags ? PIC_EDEVICE : PIC_OK;
}

int pic_read_push_counts(pic_ctx* ctx, void* ws, int64_t* n_rebinned, int64_t* n_slowpath,
                         void* stream) {
  if (!ctx || !ws) return PIC_EINVAL;
  int v = ensure_device(ctx);
  if (v) return v;
  DevFlags h;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(&h, ws, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess) return PIC_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return PIC_EHIP;
  if (n_rebinned) *n_rebinned = (int64_t)h.rebinned;
  if (n_slowpath) *n_slowpath = (int64_t)h.slowpath;
  return PIC_OK;
}

const char* pic_strerror(int status) {
  switch (status) {
    case PIC_OK: return "ok";
    case PIC_EINVAL: return "invalid argument";
    case PIC_ECOURANT: return "time step above the Courant limit";
    case PIC_EHIP: return "HIP runtime error";
    case PIC_ESTATE: return "call order violated (sort the particles first)";
    case PIC_EDEVICE: return "device flags raised";
    case PIC_ELDS: return "tile geometry exceeds the LDS of a compute unit";
    case PIC_ESCRATCH: return "grid needs more scratch than the static no-allocation buffer holds";
    default: return "unknown status";
  }
}

}  // extern "C"
