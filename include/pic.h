/*
 * libpic: MI355X (gfx950) hot path of one explicit, fully relativistic
 * electromagnetic particle-in-cell step.
 *
 * The step follows the PIC loop of Fonseca et al., "Exploiting multi-scale
 * parallelism for large scale numerical modelling of laser wakefield
 * accelerators", Sec. 2 (deposit the current of the moving particles,
 * advance E and B with the FDTD method, interpolate the fields at the
 * particles, advance the fully relativistic equations of motion; time step
 * under the Courant limit), in the per-particle order of its vector
 * algorithm, Sec. 5.2 steps i-v (interpolation weights and field gather,
 * equations of motion, virtual-particle trajectory splitting, charge-
 * conserving deposit).  Positions are kept as an integer cell plus an
 * offset normalised to the cell (Sec. 5.1), which makes single precision
 * sufficient.
 *
 * Units: c = omega_p = 1; lengths in c/omega_p, time in 1/omega_p, momenta
 * u = gamma*beta, fields in m c omega_p / e.  Maxwell: dB/dt = -curl E,
 * dE/dt = curl B - J.  Macro-particle charges q_p are densities (q_p = -n/ppc
 * for electrons at density n), so rho = sum q_p S and J = sum q_p v S.
 *
 * Conventions shared by every entry point:
 *  - All array arguments are DEVICE pointers owned by the caller; the library
 *    never allocates or frees caller memory.  Scratch lives in a caller-owned
 *    device workspace of pic_workspace_bytes() bytes, zero-filled before its
 *    first use, that must persist, and not be used by anything else, between
 *    the calls on one context.
 *  - "real" arrays hold float (real_bytes = 4) or double (real_bytes = 8).
 *  - Grid arrays hold n0*n1*n2 reals per component, x fastest:
 *    index = i + n0*(j + n1*k).  E_c and J_c sit at (i,j,k) + e_c/2, B_c at
 *    (i,j,k) + (1,1,1)/2 - e_c/2 (the Yee layout; Sec. 5.1 notes that the
 *    components sit at different positions), rho at the nodes (i,j,k).  In
 *    2D (2D3V, d/dz = 0) n2 = 1 and all six components are kept.
 *  - On an open axis of n nodes the domain is [0, n-1]: samples at
 *    half-integer positions beyond node n-1 are outside and stay zero;
 *    particles live in [0, n-1) and are absorbed when they leave it.
 *  - Calls validate their arguments on the host and return a status code
 *    synchronously; device work is only enqueued on `stream` (a hipStream_t,
 *    NULL for the null stream).  Device-side anomalies (non-finite values,
 *    offsets out of range) raise sticky flags read by pic_read_flags().
 *  - A context must not be used from two host threads or two streams at once.
 *    No C++ exception crosses this interface.
 */
#ifndef PIC_H
#define PIC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum pic_status {
  PIC_OK = 0,
  PIC_EINVAL = -1,   /* invalid argument (null pointer, size, order, dims) */
  PIC_ECOURANT = -2, /* dt above the Courant limit 1/sqrt(sum 1/dx_d^2) */
  PIC_EHIP = -3,     /* a HIP runtime call failed (no device, launch error) */
  PIC_ESTATE = -4,   /* call order violated (e.g. push before any sort) */
  PIC_EDEVICE = -5,  /* sticky device flags were raised (see pic_read_flags) */
  PIC_ELDS = -6,     /* tile geometry does not fit the 160 KB LDS of a CU */
  PIC_ESCRATCH = -7  /* the static scratch of pic_field_advance_static is too small */
};

enum pic_bc { PIC_BC_PERIODIC = 0, PIC_BC_OPEN = 1 };

/* Sticky device flag bits. */
enum pic_flag {
  PIC_FLAG_NONFINITE = 1u << 0,  /* a momentum or gamma became NaN/Inf */
  PIC_FLAG_OFFSET = 1u << 1,     /* an input offset was outside [0,1) */
  PIC_FLAG_CELL = 1u << 2,       /* an input cell index was out of range */
  PIC_FLAG_OVERSPEED = 1u << 3   /* a move exceeded one cell on some axis */
};

typedef struct pic_ctx pic_ctx; /* opaque, owned by the library */

typedef struct {
  int32_t dims;       /* 2 (2D3V) or 3 */
  int32_t n[3];       /* nodes (= cells) per axis, n[2] = 1 in 2D; each >= 2 (>= 4 if open) */
  double dx[3];       /* cell sizes, > 0 */
  double dt;          /* time step, 0 < dt <= Courant limit */
  int32_t order;      /* B-spline interpolation/deposit order, 1..4 (Table 3) */
  int32_t real_bytes; /* 4 (FP32 offsets, momenta, fields) or 8 (FP64) */
  int32_t bc[3];      /* pic_bc per axis (ignored for z in 2D) */
  int32_t tile[3];    /* cells per tile per axis; 0 selects the default */
  int32_t sort_every; /* pic_step re-sorts every this many steps (>= 1) */
  int32_t drift;      /* cells a particle may drift out of its tile before the
                         push re-bins it; < 0 selects the default */
  double q_over_m;    /* charge-to-mass ratio of the species, in e/m_e (-1 for
                         electrons, Z m_e/m_i for ions); one context per species */
  double q_const;     /* charge of every particle when pic_particles.q is NULL */
} pic_config;

typedef struct {
  int64_t np;     /* particle slots in use; absorbed particles keep their slot until
                     pic_sort compacts them away (np then drops to the live count) */
  int32_t* cell;  /* linear index i+n0*(j+n1*k) of the cell's lower node; -1 = absorbed */
  void* off[3];   /* real offsets in [0,1) from that node, in cell units (off[2] unused in 2D) */
  void* u[3];     /* real momenta gamma*beta */
  void* q;        /* real per-particle charge, or NULL to use q_const */
  int32_t* id;    /* optional payload permuted with the particles by pic_sort, or NULL */
} pic_particles;

typedef struct {
  void* E[3];
  void* B[3];
  void* J[3];
} pic_fields;

typedef struct {
  double gauss_max;     /* max |(D.E - rho) - G_ref| over interior nodes */
  double gauss_rel;     /* gauss_max / max |rho| */
  double cont_max;      /* max |(rho - rho_prev)/dt + D.J| over interior nodes */
  double cont_rel_l2;   /* ||C||_2 / ||(rho - rho_prev)/dt||_2 */
  double cont_rel_inf;  /* cont_max / (max|rho| / dt) */
  double w_field;       /* 1/2 sum (E^2 + B^2) dV over samples inside the domain */
  double w_kin;         /* sum over live particles of m_p dV (gamma - 1), with the
                           mass density m_p = |q_p| / |q_over_m| (all species) */
  double rho_max;       /* max |rho| */
  int64_t n_alive;      /* particles with cell >= 0 */
  uint32_t flags;       /* sticky pic_flag bits */
  int64_t n_slowpath;   /* particle pushes that took the global-memory path */
} pic_diag;

/* Particles entering the front column of a moving window (see
 * pic_window_shift): n = ppc per particle cell of the column, the column's
 * cells in storage order (y fastest, then z), ppc consecutive particles per
 * cell.  Device arrays of the working precision, caller-owned; the random
 * draws of a plasma injection are inputs, not drawn by the library. */
typedef struct {
  int64_t n;         /* particles to append (0: vacuum ahead) */
  int32_t ppc;       /* particles per column cell (n = ppc * column cells) */
  const void* off[3];  /* offsets in [0,1) (all dims, x included) */
  const void* u[3];    /* momenta */
  const void* q;       /* charges, required when the particles carry q, else NULL */
  int64_t id_first;    /* id of the first appended particle (the others follow it),
                          written when the particles carry ids */
} pic_inject;

/* Laser antenna: a sheet of current on the plane of E-samples x = x_index
 * (node index along x) that radiates a pulse of peak field a0*omega0 both
 * ways (a current sheet K radiates E = -K/2): J_pol += -2 a0 omega0 env(t)
 * g(y, z) cos(omega0 (t - t_center)) / dx, with env = exp(-(t-t_center)^2 /
 * tau^2) cut beyond 3 tau and g = exp(-r^2/waist^2) about (y_center,
 * z_center) (cell units times dx).  polarization: 1 = y, 2 = z. */
typedef struct {
  int32_t x_index;
  int32_t polarization;
  double a0, omega0, waist, tau, t_center, y_center, z_center;
} pic_antenna;

/* Validate `cfg` and create a context bound to the current HIP device.
 * Returns PIC_EINVAL / PIC_ECOURANT / PIC_ELDS for a bad configuration
 * (checked before any HIP call), PIC_EHIP if no device is usable.
 * *out receives the context on success, NULL otherwise. */
int pic_create(const pic_config* cfg, pic_ctx** out);

/* Release the context (NULL is accepted). */
int pic_destroy(pic_ctx* ctx);

/* Bytes of device workspace needed for up to `np` particles. */
int pic_workspace_bytes(const pic_ctx* ctx, int64_t np, size_t* bytes);

/* Group the particles by tile (counting sort on the tile of `cell`),
 * permuting every SoA array (and id) in place, and record the tile bins in
 * `ws`.  Absorbed particles (cell = -1, or a cell index out of range) are
 * compacted away: p->np is lowered to the number of live particles, which
 * fill slots 0 .. np-1; the contents of the slots from the new np up to the
 * old one are unspecified.  Reading the live count back synchronises
 * `stream`.  Must precede pic_push_deposit.  Inside a tile the particles are
 * ordered by half-cell class and LDS bank residue of the position a straight
 * line gives (sort_every - 1) / 2 steps ahead (the middle of the interval to
 * the next sort).  This is the data layout change that makes the deposit
 * local; it does not change physics. */
int pic_sort(pic_ctx* ctx, pic_particles* p, void* ws, void* stream);

/* One gather + Boris push + move + split + charge-conserving deposit pass
 * over all live particles (Sec. 2 loop; Sec. 5.2 steps i-v): reads E^n, B^n
 * at the particles, advances u^{n-1/2} -> u^{n+1/2} and x^n -> x^{n+1} in
 * place, and overwrites f->J with J^{n+1/2}.  Requires a prior pic_sort with
 * the same particle arrays and workspace (PIC_ESTATE otherwise).  Particles
 * within `drift` cells of the tile the sort put them in are pushed tile by
 * tile out of LDS; those that have drifted further are re-binned by the tile
 * of their current cell and pushed out of LDS in a second tile pass (the
 * arrays keep their order; only the next pic_sort moves them); a particle
 * that moves half a cell or more in one step, or whose |q| exceeds the bound
 * the sort recorded, is pushed in global memory.  The result does not depend
 * on the path beyond the rounding of the current's accumulation. */
int pic_push_deposit(pic_ctx* ctx, pic_particles* p, const pic_fields* f, void* ws,
                     void* stream);

/* FDTD (Yee) advance with J^{n+1/2}, in place: B -= dt/2 C E; E += dt (C^T B - J)
 * with Mur first-order absorbing updates of the tangential E on open faces;
 * B -= dt/2 C E (Sec. 2: FDTD method, local solver, Sec. 3). */
int pic_field_advance(pic_ctx* ctx, pic_fields* f, void* ws, void* stream);

/* pic_field_advance without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): same arguments and result as
 * pic_field_advance.  Its scratch -- the E samples next to open faces,
 * saved between the Yee and the Mur updates, 4 n_a n_b reals per open axis
 * (n_a, n_b the grid sizes across that axis) -- lives in a static device
 * array of 16 MiB per GPU (each GPU the library runs on holds it until the
 * process ends); a grid that needs more returns PIC_ESCRATCH before any
 * launch.  Nothing in it has to start at zero: every call writes the saved
 * planes before reading them.  All calls on one GPU share that array, so
 * calls that overlap on one GPU (two streams, two host threads) race.  It
 * allocates nothing: no hipMalloc, hipFree or allocating library call. */
int pic_field_advance_static(pic_ctx* ctx, pic_fields* f, void* stream);

/* `nsteps` full steps: pic_sort when due (every sort_every steps, counted
 * per context, and before the first push; p->np drops to the live count at
 * every sort), pic_push_deposit, pic_field_advance. */
int pic_step(pic_ctx* ctx, pic_particles* p, pic_fields* f, int32_t nsteps, void* ws,
             void* stream);

/* Mobile ions and other extra species (the LWFA-1 run of Sec. 6 keeps the
 * ions mobile; each species is pushed in the same E, B and the current of the
 * loop of Sec. 2 is the sum of the species' currents).  One context per
 * species (its q_over_m and q_const), with its own particle arrays and
 * workspace, all contexts on the same grid, time step, order, precision and
 * boundaries (PIC_EINVAL otherwise).
 *
 * pic_push_deposit_add: as pic_push_deposit but ADDS J^{n+1/2} of this
 * species to f->J instead of overwriting it (same sort requirement). */
int pic_push_deposit_add(pic_ctx* ctx, pic_particles* p, const pic_fields* f, void* ws,
                         void* stream);

/* `nsteps` full steps of `nspecies` species (arrays of that length): per step,
 * every species is sorted when due (per context) and pushed (the first
 * overwrites J, the others add to it), then the fields advance once (with
 * ctx[0]'s workspace). */
int pic_step_species(int32_t nspecies, pic_ctx* const* ctx, pic_particles* const* p,
                     void* const* ws, pic_fields* f, int32_t nsteps, void* stream);

/* FP64 charge density at the nodes from the stored cells and offsets with
 * order-n node shapes; `rho` holds n0*n1*n2 doubles and is overwritten. */
int pic_deposit_rho(pic_ctx* ctx, const pic_particles* p, double* rho, void* ws, void* stream);

/* Same, but adds this species' charge density to `rho` (several species). */
int pic_deposit_rho_add(pic_ctx* ctx, const pic_particles* p, double* rho, void* ws,
                        void* stream);

/* FP64 diagnostics (synchronises `stream`): deposits rho^n into `rho_out`,
 * forms the Gauss residual D.E - rho^n (minus `gauss_ref` if not NULL; the
 * residual field is written to `gauss_out` if not NULL) and, if `rho_prev`
 * is not NULL, the continuity residual (rho^n - rho_prev)/dt + D.J with the
 * J currently in `f`; reduces them with the energies into *out.  Interior
 * nodes exclude 1 + order/2 node planes next to each open face. */
int pic_diagnostics(pic_ctx* ctx, const pic_particles* p, const pic_fields* f,
                    const double* rho_prev, const double* gauss_ref, double* rho_out,
                    double* gauss_out, pic_diag* out, void* ws, void* stream);

/* pic_diagnostics over several species sharing `f` (same conventions as
 * pic_step_species): rho is the sum over species, w_kin and n_alive are
 * summed, flags are or-ed and slow-path counts summed over the workspaces. */
int pic_diagnostics_species(int32_t nspecies, pic_ctx* const* ctx, const pic_particles* const* p,
                            void* const* ws, const pic_fields* f, const double* rho_prev,
                            const double* gauss_ref, double* rho_out, double* gauss_out,
                            pic_diag* out, void* stream);

/* Moving window (Sec. 2: the simulation box follows the laser through the
 * plasma): shift the state one cell toward -x.  E and B move one cell
 * (F[i] <- F[i+1], the front plane zeroed), J is zeroed, every particle's
 * cell moves one cell down in x (those leaving at x < 0 are absorbed), and
 * `in->n` particles are appended in the front particle column (x = n0-2) from
 * `in` (ids in->id_first, in->id_first + 1, ... when p->id is not NULL).
 * Requires an open x axis; `capacity` is the length of the particle arrays
 * (PIC_EINVAL if p->np + in->n exceeds it).  Updates p->np; the particles
 * must be sorted again before the next push, and that sort reclaims the
 * slots of the particles absorbed at the back, so a window that keeps
 * moving needs a capacity of about the live count plus one entering column
 * per shift between sorts.  f = NULL shifts only the particles (further
 * species of a multi-species run, after the first species moved the fields). */
int pic_window_shift(pic_ctx* ctx, pic_particles* p, int64_t capacity, pic_fields* f,
                     const pic_inject* in, void* ws, void* stream);

/* Add the antenna's current at time t to f->J (after the deposit, before
 * the field advance: t is the time of J, (n + 1/2) dt). */
int pic_antenna_add(pic_ctx* ctx, pic_fields* f, const pic_antenna* a, double t, void* stream);

/* Attach an antenna to the context (copied; NULL detaches): pic_step and
 * pic_step_species then add its current every step at t = (n + 1/2) dt, with
 * n the context's step count. */
int pic_set_antenna(pic_ctx* ctx, const pic_antenna* a);

/* Transpose of pic_field_advance (hand-written adjoint; the advance is linear
 * in E, B, J).  In: lam->E, lam->B = adjoints of E^{n+1}, B^{n+1}.  Out, in
 * place: lam->E, lam->B = adjoints of E^n, B^n through the field advance alone,
 * and lam->J (overwritten) = adjoint of J^{n+1/2}.  The Mur updates on open
 * faces are transposed with the rest. */
int pic_field_advance_adjoint(pic_ctx* ctx, pic_fields* lam, void* ws, void* stream);

/* Transpose (vector-Jacobian product) of pic_push_deposit for one step, along
 * the branch the forward takes.  state_n: the particles at step n (cell, off,
 * u^{n-1/2}, q; any order, no sort needed); EB_n: E^n and B^n (J unused).
 * lam_f->J: in, adjoint of J^{n+1/2}; lam_f->E, lam_f->B: the gather's
 * contribution is ADDED (atomics).  lam_p->off[d] (cell units) and
 * lam_p->u[c]: in, adjoints of x^{n+1} and u^{n+1/2}; out, adjoints of x^n and
 * u^{n-1/2}, slot by slot with state_n (lam_p->cell, q, id are unused).
 * Absorbed particles (cell = -1) are skipped.  When the context's last
 * pic_sort was of state_n->np particles in this `ws`, particles inside the
 * drift allowance of the tile whose bin range holds them are done out of
 * LDS, per tile in 2D and per z slab of a tile in 3D (the rest, and every
 * particle of the cubic FP64 form, in global memory); the result does not
 * depend on that beyond the order of floating-point atomic additions. */
int pic_push_deposit_adjoint(pic_ctx* ctx, const pic_particles* state_n, const pic_fields* EB_n,
                             pic_fields* lam_f, pic_particles* lam_p, void* ws, void* stream);

/* Read (and optionally clear) the sticky device flags and the slow-path
 * counter (synchronises `stream`).  Returns PIC_EDEVICE if any flag is set.
 * Clearing also clears the re-binned count of pic_read_push_counts. */
int pic_read_flags(pic_ctx* ctx, void* ws, int clear, uint32_t* flags, int64_t* n_slowpath,
                   void* stream);

/* Pushes since the last clear of the flags in `ws` that left the sorted tile
 * pass of pic_push_deposit: *n_rebinned handed to the re-binned tile pass,
 * *n_slowpath done in global memory (either pointer may be NULL).  Host
 * outputs; synchronises `stream`; PIC_EINVAL for a NULL ctx or ws. */
int pic_read_push_counts(pic_ctx* ctx, void* ws, int64_t* n_rebinned, int64_t* n_slowpath,
                         void* stream);

/* Human-readable name of a status code. */
const char* pic_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif
