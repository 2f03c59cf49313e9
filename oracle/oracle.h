/*
 * FP64 CPU oracle for one explicit, fully relativistic electromagnetic
 * particle-in-cell step (Fonseca et al., "Exploiting multi-scale parallelism
 * for large scale numerical modelling of laser wakefield accelerators").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link
 * or call this library: it is used by tests/, by the smoke check in
 * __graft_entry__.py and by the CPU-baseline leg of bench.py.  It shares no
 * code, header or constant with the HIP library under paper_1310_0930_amd/.
 *
 * The method follows the paper's prose description of the PIC loop (Sec. 2:
 * deposit current, advance fields with FDTD, interpolate fields at the
 * particles, advance the relativistic equations of motion; Courant-limited
 * time step) and of its vector form (Sec. 5.2, steps i-v: weights and field
 * interpolation, equations of motion, virtual-particle trajectory splitting,
 * charge-conserving current deposition).  The paper prints no equations; the
 * concrete readings (normalised units, Boris pusher, Yee layout, B-spline
 * shapes, split-then-Esirkepov deposition, Mur-1 open faces) are stated
 * beside each function below.
 *
 * Layout: positions are global, in cell units (X_d = x_d / dx_d), FP64, three
 * per particle (the z entry is ignored in 2D).  Field arrays are
 * n0*n1*n2 doubles per component, x fastest; component c of E and J sits at
 * (i,j,k) + e_c/2, component c of B at (i,j,k) + (1,1,1)/2 - e_c/2.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORACLE_PERIODIC = 0, ORACLE_OPEN = 1 };

typedef struct {
  int32_t dims;     /* 2 (2D3V, d/dz = 0) or 3 */
  int32_t n[3];     /* cells (= nodes) per axis; n[2] = 1 in 2D */
  double dx[3];     /* cell size per axis, in c/omega_p */
  double dt;        /* time step, in 1/omega_p */
  int32_t order;    /* B-spline order 1..4 */
  int32_t bc[3];    /* ORACLE_PERIODIC or ORACLE_OPEN per axis */
  double q_over_m;  /* charge-to-mass ratio of the species (-1 for electrons) */
} oracle_config;

/* Shape weights of order `order` at position X (cell units): writes the
 * first node index to *base and order+1 weights to w. */
void oracle_shape(int32_t order, double X, int64_t* base, double* w);

/* Field interpolation at np positions: Ep, Bp are np*3. */
void oracle_gather(const oracle_config* cfg, int64_t np, const double* X,
                   const double* E, const double* B, double* Ep, double* Bp);

/* Relativistic Boris rotation of np momenta u (np*3, in place) under the
 * given particle fields Ep, Bp (np*3). */
void oracle_boris(const oracle_config* cfg, int64_t np, double* u,
                  const double* Ep, const double* Bp);

/* Charge-conserving deposit of straight paths X0 -> X1 (unwrapped, cell
 * units) with charges q and out-of-plane velocities vz (2D only) into J,
 * which is accumulated (not zeroed). */
void oracle_deposit_paths(const oracle_config* cfg, int64_t np,
                          const double* X0, const double* X1, const double* q,
                          const double* vz, double* J);

/* One gather + push + move + deposit pass over all live particles.  J is
 * zeroed first and receives J^{n+1/2}.  Particles leaving an open face are
 * deposited, then marked dead (alive = 0).  nthreads > 1 splits the
 * particles over threads with one private current grid per thread followed
 * by a reduction (the shared-memory scheme of Sec. 3.1). */
void oracle_push_deposit(const oracle_config* cfg, int64_t np, double* X,
                         double* u, const double* q, int8_t* alive,
                         const double* E, const double* B, double* J,
                         int32_t nthreads);

/* Same as oracle_push_deposit for one species (charge-to-mass ratio
 * cfg->q_over_m) but J is accumulated, not zeroed.  With mobile ions (the
 * LWFA-1 run of Sec. 6) each species is pushed in the same fields and the
 * current of the loop of Sec. 2 is the sum of the species' currents. */
void oracle_push_deposit_add(const oracle_config* cfg, int64_t np, double* X,
                             double* u, const double* q, int8_t* alive,
                             const double* E, const double* B, double* J,
                             int32_t nthreads);

/* FDTD (Yee) advance E^n,B^n -> E^{n+1},B^{n+1} with J^{n+1/2}:
 * B -= dt/2 curl E; E += dt (curl B - J) (Mur-1 on open faces); B -= dt/2 curl E. */
void oracle_field_advance(const oracle_config* cfg, double* E, double* B,
                          const double* J);

/* nsteps full steps: push_deposit then field_advance. */
void oracle_step(const oracle_config* cfg, int64_t np, double* X, double* u,
                 const double* q, int8_t* alive, double* E, double* B,
                 double* J, int32_t nsteps, int32_t nthreads);

/* Same as oracle_step, carrying a forward-mode tangent (dX, du, dE, dB, dJ)
 * alongside every value: the tangents on return are the directional
 * derivatives of the final state along the input tangents. */
void oracle_step_jvp(const oracle_config* cfg, int64_t np, double* X,
                     double* dX, double* u, double* du, const double* q,
                     int8_t* alive, double* E, double* dE, double* B,
                     double* dB, double* J, double* dJ, int32_t nsteps);

/* Charge density at the nodes from order-n node shapes (FP64). */
void oracle_deposit_rho(const oracle_config* cfg, int64_t np, const double* X,
                        const double* q, const int8_t* alive, double* rho);

/* Node-centred Yee divergence of a staggered vector field V (3*cells):
 * out[node] = sum_d (V_d[node] - V_d[node - e_d]) / dx_d.  On open axes the
 * first and last node planes are set to 0 (they are not interior). */
void oracle_divergence(const oracle_config* cfg, const double* V, double* out);

/* Field energy 1/2 sum (E^2 + B^2) dV over the samples inside the domain and
 * kinetic energy sum (q / (q/m)) dV (gamma - 1) over live particles (the
 * macro-particle's mass density times gamma - 1). */
void oracle_energies(const oracle_config* cfg, int64_t np, const double* u,
                     const double* q, const int8_t* alive, const double* E,
                     const double* B, double* w_field, double* w_kin);

/* Curl operators on the Yee grid (used to pin the discrete identities):
 * out = C E (at B positions) and out = C^T B (at E positions). */
void oracle_curl_e(const oracle_config* cfg, const double* E, double* out);
void oracle_curl_b(const oracle_config* cfg, const double* B, double* out);

#ifdef __cplusplus
}
#endif
#endif
