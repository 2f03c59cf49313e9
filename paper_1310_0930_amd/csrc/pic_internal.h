// Internal declarations of libpic (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pic.h"

namespace pic {

// ------------------------------------------------------------------ geometry
// Node offsets, relative to a particle's cell, that the order-n stencils can
// touch.  Gather: union over the six Yee components of the nodes of the
// (order+1)^D stencil at the component's own position.  Deposit: union over
// the virtual segments of a path that moves at most half a cell per axis
// (larger moves take the global-memory path).
template <int ORDER>
struct Reach {
  static constexpr int g_lo = ORDER >= 3 ? -2 : -1;
  static constexpr int g_hi = ORDER == 1 ? 1 : ORDER == 4 ? 3 : 2;
  static constexpr int d_lo = ORDER >= 3 ? -2 : -1;
  static constexpr int d_hi = ORDER >= 3 ? 3 : 2;
};

// Tile shape (cells per axis) and drift allowance A: one workgroup owns the
// particles binned to a tile at the last sort; those whose cell is still
// within A cells of the tile run entirely out of LDS.  The LDS regions cover
// the tile, A cells on each side and the stencil reach.  Sizes are
// compile-time so that every stencil offset is an immediate of the LDS
// instruction.
template <int DIMS, int ORDER, typename R>
struct Geo {
  // 3D tiles are 8^3 cells with one cell of drift allowance; the largest
  // stencils halve the tile along z (quartic, and cubic in double
  // precision), and along every axis for quartic in double precision, so
  // that the allowance stays and the LDS regions still fit a CU
  static constexpr bool wide = ORDER == 4 || (sizeof(R) == 8 && ORDER == 3);
  static constexpr int T = DIMS == 3 ? ((ORDER == 4 && sizeof(R) == 8) ? 4 : 8) : 16;
  static constexpr int TZ = DIMS == 3 ? (wide ? 4 : T) : 1;
  static constexpr int A = DIMS == 3 ? 1 : 2;
  static constexpr int AZ = DIMS == 3 ? A : 0;
  using Rc = Reach<ORDER>;
  // E/B region
  static constexpr int ex = T + 2 * A + Rc::g_hi - Rc::g_lo;
  static constexpr int ez = DIMS == 3 ? TZ + 2 * AZ + Rc::g_hi - Rc::g_lo : 1;
  static constexpr int e_lo = -A + Rc::g_lo;  // region origin relative to the tile origin
  static constexpr int e_lo_z = DIMS == 3 ? e_lo : 0;
  static constexpr int e_vol = ex * ex * ez;
  // J region
  static constexpr int jx = T + 2 * A + Rc::d_hi - Rc::d_lo;
  static constexpr int jz = DIMS == 3 ? TZ + 2 * AZ + Rc::d_hi - Rc::d_lo : 1;
  static constexpr int j_lo = -A + Rc::d_lo;
  static constexpr int j_lo_z = DIMS == 3 ? j_lo : 0;
  static constexpr int j_vol = jx * jx * jz;
  // E/B staged in the working precision.  The current tile has 8-byte
  // cells: in the double form it accumulates with LDS double atomic adds;
  // in the single form each contribution is rounded to a 32-bit integer on
  // a power-of-two scale and summed exactly with LDS 64-bit integer atomic
  // adds (on gfx950 these issue ~1.7x faster than double adds at scattered
  // addresses, and single-precision LDS atomic adds ~17x slower)
  static constexpr bool fixed = sizeof(R) == 4;
  static constexpr size_t lds_bytes = sizeof(R) * 6 * (size_t)e_vol + sizeof(double) * 3 * (size_t)j_vol;
  // threads per workgroup: in 3D one workgroup fills a CU's LDS, so it
  // brings all the wavefronts: 16 (4 per SIMD, <= 128 VGPRs) in FP32 up to
  // cubic order; 12 (<= 168 VGPRs) for FP64 up to quadratic order and FP32
  // quartic, whose gather and deposit need more registers (FP64 quadratic
  // 15 % faster than with 8); 8 for cubic and quartic FP64, which would
  // spill at 168; 2D tiles are small and several workgroups share a CU,
  // with 8 wavefronts each so that a workgroup's batches drain its tile
  // sooner (a 512 x 256 mesh has only 512 tiles of 16 x 16 for 256 CUs)
  static constexpr int NT = DIMS == 2 ? 512
                            : sizeof(R) == 4 ? (ORDER <= 3 ? 1024 : 768)
                                             : (ORDER <= 2 ? 768 : 512);
};

// Unsigned division by a runtime divisor through a precomputed multiplier
// (round-up method of Granlund and Montgomery, "Division by invariant
// integers using multiplication", 1994): q = (mulhi(m, a) + a) >> l, exact
// for every 32-bit a.
struct FastDiv {
  uint32_t d, m, l;
  __host__ void init(uint32_t div) {
    d = div;
    l = 0;
    while ((1ull << l) < div) ++l;
    m = (uint32_t)((((1ull << l) - div) << 32) / div + 1);
  }
  __device__ __forceinline__ uint32_t div(uint32_t a) const {
    uint64_t t = (uint64_t)__umulhi(m, a) + a;
    return (uint32_t)(t >> l);
  }
};

// ------------------------------------------------------------------ params
template <typename R>
struct KParams {
  int dims, order;
  int n[3];
  int bc[3];       // PIC_BC_*
  int tile[3];     // cells per tile
  int ntile[3];    // tiles per axis
  int ntiles;      // product of ntile
  int per_xcd;     // tiles per XCD slice (XCD-aware block remap)
  FastDiv dn0, dn1;  // division by n0 and n1 (cell index decomposition)
  R hqm;           // (q/m) dt / 2
  R dtdx[3];       // dt / dx_d
  R jfac[3];       // -dx_d / dt
  R dt;
  R q_const;
};

// Device-side particle and field pointers.
template <typename R>
struct DParts {
  int32_t* cell;
  R* off[3];
  R* u[3];
  R* q;  // may be null
  int32_t* id;  // may be null
};

template <typename R>
struct DFields {
  R* E[3];
  R* B[3];
  R* J[3];
};

// Sticky flags and counters at the head of the workspace.
struct DevFlags {
  unsigned int flags;
  unsigned int ndefer;          // particles the sorted tile pass left this push (deferred list)
  unsigned long long slowpath;  // total global-memory pushes since the last clear
  unsigned long long rebinned;  // total pushes handed to the re-binned pass since the last clear
  // Written by the sort (not cleared with the flags): bit pattern of the
  // largest |q| (as float) over the per-particle charges it moved.
  unsigned int qmax;
  unsigned int ndefer2;         // particles the re-binned pass left to the global-memory kernel
  // Work counters of the persistent push: tiles taken so far from each
  // XCD's tile range (cleared before every push).
  unsigned int tile_next[8];
  // Re-binned pass (cleared before every push): destination tiles holding
  // re-binned particles, claims of them, and workgroups of the sorted pass
  // that have finished.
  unsigned int rb_m;
  unsigned int rb_next;
  unsigned int rb_done;
  unsigned int pad0;
  // particles the sorted pass left, summed over the pushes since the last
  // sort (each push's prologue adds the previous push's ndefer; the sort's
  // count kernel clears both)
  unsigned long long since_sort;
  unsigned int pad[10];
};
static_assert(sizeof(DevFlags) == 128, "DevFlags layout");

// Particles that drifted beyond the allowance of the tile they were sorted
// into, re-binned by the tile of their current cell for a second tile pass
// (device pointers into the workspace; the sort's scratch is free during a
// push).
struct Rebin {
  int* cnt;     // int32[ntiles]  re-binned particles per destination tile (zeroed per push)
  int* tv;      // int32[ntiles]  slot of a destination tile in nl
  int* nl;      // int32[ntiles]  destination tiles in order of their first particle
  int* base;    // int32[ntiles]  first list position of each slot
  int* rank;    // int32[np]      rank of each deferred entry within its destination tile
  int* list;    // int32[np]      the deferred particles grouped by destination tile
  int* defer2;  // int32[np]      particles left to the global-memory kernel
};

// ------------------------------------------------------------------ workspace
struct WsLayout {
  size_t flags;      // DevFlags
  size_t starts;     // int32[ntiles + 2]   tile starts (entry ntiles = dead bin start, then np)
  size_t counts;     // int32[nbins]        bin counts / scatter cursors
  size_t bstart;     // int32[nbins + 1]    bin starts
  size_t bsum;       // int32[nbins / 1024 + 1]  scan block sums
  size_t rb_tv;      // int32[ntiles]       re-binned pass: slot of each destination tile
  size_t rb_nl;      // int32[ntiles]       re-binned pass: destination tiles
  size_t keys;       // int32[np]           tile of each particle (count, scatter)
  size_t pkey;       // int32[np]           in-tile placement key of each copied particle, then its rank
  size_t order;      // int32[1024]         a tile's cells listed by bank residue
  size_t tmp_cell;   // int32[np]
  size_t tmp_real;   // R[np * 7]  off[3], u[3], q
  size_t tmp_id;     // int32[np]
  size_t mur;        // R[mur_len]  saved E planes next to open faces
  size_t diag;       // double[diag_len]  reduction partials
  size_t adj;        // R[adj_len]  adjoint scratch (open axes)
  size_t total;
  size_t mur_len;
  size_t diag_len;
  size_t adj_len;
};

}  // namespace pic

struct pic_ctx {
  pic_config cfg;
  int device;
  int ntile[3];
  int ntiles;
  int tile[3];
  int64_t steps_done;      // steps taken through pic_step (drives sort_every)
  // Re-binned push pass on or off: decided at each sort from whether the
  // pushes since the previous sort left any particle outside the sorted
  // tile pass (on for a new context).
  bool rebin;
  int64_t pushes_since_sort;
  // sorted-state tracking: pic_push_deposit needs bins that match the arrays
  const void* sorted_cell;
  const void* sorted_ws;
  int64_t sorted_np;
  int64_t sorted_cap;
  int cu_count;
  bool antenna_on;         // pic_set_antenna: added by pic_step every step
  pic_antenna antenna;
};

namespace pic {
WsLayout ws_layout(const pic_ctx* ctx, int64_t np);

// launchers (return hipError_t as int)
int launch_sort(const pic_ctx* ctx, const pic_particles* p, void* ws, hipStream_t s);
int launch_push_deposit(const pic_ctx* ctx, const pic_particles* p, const pic_fields* f,
                        void* ws, hipStream_t s, bool accumulate);
int launch_field_advance(const pic_ctx* ctx, const pic_fields* f, void* ws, hipStream_t s);
// The no-allocation field advance: its scratch is a static device array of
// STATIC_SCRATCH_BYTES per GPU, whose address static_scratch_init takes (once
// per device, with that device current) at context creation.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)16 << 20;
constexpr int MAX_DEVICES = 64;
int static_scratch_init(int device);
int launch_field_advance_static(const pic_ctx* ctx, const pic_fields* f, hipStream_t s);
int launch_field_advance_adjoint(const pic_ctx* ctx, const pic_fields* lam, void* ws, hipStream_t s);
int launch_push_deposit_adjoint(const pic_ctx* ctx, const pic_particles* p, const pic_fields* f,
                                const pic_fields* lam_f, pic_particles* lam_p, void* ws,
                                hipStream_t s);
int launch_deposit_rho(const pic_ctx* ctx, const pic_particles* p, double* rho, void* ws,
                       hipStream_t s, bool accumulate);
int launch_window_shift(const pic_ctx* ctx, pic_particles* p, const pic_fields* f,
                        const pic_inject* in, hipStream_t s);
int launch_antenna(const pic_ctx* ctx, const pic_fields* f, const pic_antenna* a, double t,
                   hipStream_t s);
int launch_diagnostics(int ns, const pic_ctx* const* ctx, const pic_particles* const* p,
                       void* const* ws, const pic_fields* f, const double* rho_prev,
                       const double* gauss_ref, double* rho_out, double* gauss_out, pic_diag* out,
                       hipStream_t s);

template <typename R>
KParams<R> make_params(const pic_ctx* ctx);
}  // namespace pic
