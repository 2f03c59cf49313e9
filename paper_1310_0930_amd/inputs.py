"""Seeded synthetic inputs for the EM-PIC hot path.

This module draws initial particle and field states only; it holds none of
the method's arithmetic and imports neither the HIP binding nor the oracle,
so both sides can start from bit-identical data.

Recipes (the paper's benchmark is a uniform warm plasma, Sec. 6 and Sec. 7,
with a generalised thermal spread u_th = gamma*beta_th; its laser-wakefield
states are not reproducible here, so the laser workloads start from a cold
plasma with a Gaussian pulse placed in the box):

* positions: ``ppc`` i.i.d. offsets U[0,1)^D in every cell of the particle
  domain, drawn in FP64 and rounded to FP32 (an offset that rounds to 1.0 is
  folded to 0 of the same cell, i.e. the largest float below 1 is used);
* momenta: u_i ~ N(0, u_th^2) per component, rounded to FP32;
* charge: q_p = -n(x_p)/ppc with n = 1 (uniform) or n = min(x/L_ramp, 1)
  (linear ramp along x), rounded to FP32;
* ions (optional, ``Workload.ions``): drawn the same way from child seeds
  of their own, charge +n(x)/ppc, charge-to-mass ratio Z/M;
* laser: E_y = a0 w0/wp exp(-r^2/W^2) exp(-(x-xc)^2/tau^2) cos(k0 (x-xc)),
  cut to zero for |x - xc| > 3 tau, B_z = the same profile at B_z's position
  (a forward-moving pulse), rounded to FP32.

Particle domain: [0, n) on periodic axes, [0, n-1) on open axes (the last
node plane is the open face).  Particles are generated cell by cell in
storage order (x fastest), ``ppc`` consecutive particles per cell.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

PERIODIC, OPEN = 0, 1
SEED_BASE = 13100930


def courant_dt(dx, dims):
    return 1.0 / math.sqrt(sum(1.0 / (dx[d] ** 2) for d in range(dims)))


@dataclass(frozen=True)
class Laser:
    a0: float = 4.0
    omega0: float = 10.0   # omega0 / omega_p; k0 = omega0 in units of omega_p/c
    waist: float = 8.0     # c/omega_p
    tau: float = 2.0       # 1/omega_p
    x_center: float = 6.0  # 3 tau: the pulse tail starts at x = 0


@dataclass(frozen=True)
class Ions:
    """A mobile ion species (the paper's LWFA-1 run keeps the ions mobile,
    Sec. 6): charge state Z, mass ratio M = m_i/m_e, thermal spread u_th.
    Drawn like the electrons (ppc per cell, own seeds), charge +n(x)/ppc per
    macro-ion (neutralising), charge-to-mass ratio Z/M in units of e/m_e."""
    mass_ratio: float = 1836.15
    charge: float = 1.0
    u_th: float = 0.0

    @property
    def q_over_m(self) -> float:
        return self.charge / self.mass_ratio


@dataclass(frozen=True)
class Workload:
    name: str
    dims: int
    n: tuple
    dx: tuple
    order: int
    ppc: int
    u_th: float
    steps: int
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)
    courant_fraction: float = 0.5
    ramp_cells: float = 0.0
    laser: Laser | None = None
    sort_every: int = 20
    seed: int = SEED_BASE
    ions: Ions | None = None

    @property
    def dt(self) -> float:
        return self.courant_fraction * courant_dt(self.dx, self.dims)

    @property
    def n3(self):
        return tuple(list(self.n) + [1] * (3 - len(self.n)))

    @property
    def dx3(self):
        return tuple(list(self.dx) + [1.0] * (3 - len(self.dx)))

    @property
    def bc3(self):
        return tuple(list(self.bc) + [PERIODIC] * (3 - len(self.bc)))

    @property
    def ncell(self) -> int:
        a, b, c = self.n3
        return a * b * c

    def particle_cells(self):
        """Cells that hold particles per axis: n on periodic, n-1 on open axes."""
        return tuple((self.n3[d] - (1 if (d < self.dims and self.bc3[d] == OPEN) else 0))
                     if d < self.dims else 1 for d in range(3))

    @property
    def num_particles(self) -> int:
        a, b, c = self.particle_cells()
        return a * b * c * self.ppc

    @property
    def q_const(self) -> float:
        """Charge of one macro-electron at density n0 = 1, rounded to FP32."""
        return float(np.float32(-1.0 / self.ppc))

    @property
    def q_const_ions(self) -> float:
        """Charge of one macro-ion at n0 = 1 (neutralising), rounded to FP32."""
        return float(np.float32(1.0 / self.ppc))

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# The five workloads of this build, smallest first.
WORKLOADS = {
    # 2D3V 64x64, linear shapes, thermal 0.01, periodic, 100 steps (FP64 parity)
    "w2d_64_linear": Workload("w2d_64_linear", 2, (64, 64), (0.2, 0.2), 1, 4, 0.01, 100,
                              seed=SEED_BASE + 1),
    # 3D 128^3, quadratic, thermal 0.05, periodic, 50 steps (primary bandwidth point);
    # sorted every 10 steps: the warm plasma drifts out of the sorted lane
    # layout, and re-sorting every 10 steps gives the shortest whole step
    "w3d_128_quadratic": Workload("w3d_128_quadratic", 3, (128, 128, 128), (0.2, 0.2, 0.2), 2, 8,
                                  0.05, 50, sort_every=10, seed=SEED_BASE + 2),
    # 3D 256x128x128 cubic, cold plasma with a 20-cell ramp, a0=4 laser, open y,z
    # (sorted every 12 steps: electrons in the a0 = 4 pulse move 0.4 cells per
    # step along x and leave their tile's one-cell drift allowance within a few
    # steps; the re-binned tile pass keeps them out of global memory, and 12
    # gave the shortest step)
    "w3d_256_cubic_laser": Workload("w3d_256_cubic_laser", 3, (256, 128, 128), (0.1, 0.2, 0.2), 3,
                                    8, 0.0, 200, bc=(PERIODIC, OPEN, OPEN), ramp_cells=20.0,
                                    laser=Laser(), sort_every=12, seed=SEED_BASE + 3),
    # 2D3V 512x256 quadratic, 16 ppc, ramp + laser, open y (adjoint workload)
    "w2d_512_quadratic_laser": Workload("w2d_512_quadratic_laser", 2, (512, 256), (0.1, 0.2), 2, 16,
                                        0.0, 50, bc=(PERIODIC, OPEN), ramp_cells=20.0,
                                        laser=Laser(), seed=SEED_BASE + 4),
    # 3D 512x256x256 quadratic, cold uniform plasma + laser, periodic, sort every 20
    "w3d_512_quadratic_laser": Workload("w3d_512_quadratic_laser", 3, (512, 256, 256),
                                        (0.1, 0.2, 0.2), 2, 8, 0.0, 100, laser=Laser(),
                                        sort_every=20, seed=SEED_BASE + 5),
}
# The 128^3 warm-plasma recipe at the other orders of Table 3 (linear, cubic,
# quartic), and with a mobile ion species (hydrogen mass ratio, thermal
# spread 0.05 / sqrt(1836) for equal temperatures).
for _o, _name in ((1, "linear"), (3, "cubic"), (4, "quartic")):
    WORKLOADS[f"w3d_128_{_name}"] = WORKLOADS["w3d_128_quadratic"].with_(
        name=f"w3d_128_{_name}", order=_o, seed=SEED_BASE + 10 + _o)
WORKLOADS["w3d_128_quadratic_ions"] = WORKLOADS["w3d_128_quadratic"].with_(
    name="w3d_128_quadratic_ions", ions=Ions(mass_ratio=1836.15, u_th=0.05 / math.sqrt(1836.15)),
    seed=SEED_BASE + 6)


def _round32(a):
    return np.asarray(a, dtype=np.float32)


@dataclass
class Plasma:
    """SoA particle state: linear cell index, FP32-representable offsets and
    momenta (kept in float32), optional per-particle charge."""
    cell: np.ndarray           # int32 (np,)
    off: np.ndarray            # float32 (3, np); rows >= dims are zero
    u: np.ndarray              # float32 (3, np)
    q: np.ndarray | None       # float32 (np,) or None for a uniform charge
    q_const: float
    extra: dict = field(default_factory=dict)

    @property
    def np(self) -> int:
        return int(self.cell.shape[0])

    def global_positions(self, w: Workload) -> np.ndarray:
        """Positions in cell units, (np, 3) float64 (exact: cell + FP32 offset)."""
        n0, n1, _ = w.n3
        c = self.cell.astype(np.int64)
        ix = c % n0
        iy = (c // n0) % n1
        iz = c // (n0 * n1)
        X = np.zeros((self.np, 3), dtype=np.float64)
        X[:, 0] = ix + self.off[0].astype(np.float64)
        X[:, 1] = iy + self.off[1].astype(np.float64)
        if w.dims == 3:
            X[:, 2] = iz + self.off[2].astype(np.float64)
        return X

    def charges(self) -> np.ndarray:
        if self.q is None:
            return np.full(self.np, self.q_const, dtype=np.float64)
        return self.q.astype(np.float64)


def _uniform_offsets(rng, count, dims):
    off = np.zeros((3, count), dtype=np.float32)
    for d in range(dims):
        v = _round32(rng.random(count))
        # rounding to FP32 can turn a draw just below 1 into 1.0: keep it in [0,1)
        v[v >= 1.0] = np.nextafter(np.float32(1.0), np.float32(0.0))
        off[d] = v
    return off


def make_plasma(w: Workload, slabs: range | None = None, quiet: bool = False) -> Plasma:
    """Draw the particles of workload ``w``.

    Generation is per z-slab (per y-row in 2D), each from its own child seed,
    so any slab can be regenerated alone.  ``slabs`` restricts the output to
    those slabs.  ``quiet`` places the particles on a regular sub-lattice
    (for cold-plasma tests) instead of drawing the offsets.
    """
    return _draw(w, slabs, quiet, stream=(), u_th=w.u_th, sign=-1.0, q_const=w.q_const)


def make_ions(w: Workload, slabs: range | None = None, quiet: bool = False) -> Plasma:
    """Draw the ion species of workload ``w`` (``w.ions``): the same cells and
    ppc as the electrons, offsets and momenta from child seeds of their own,
    charge +n(x)/ppc."""
    if w.ions is None:
        raise ValueError(f"workload {w.name} has no ion species")
    return _draw(w, slabs, quiet, stream=(1,), u_th=w.ions.u_th, sign=1.0, q_const=w.q_const_ions)


def _draw(w, slabs, quiet, stream, u_th, sign, q_const) -> Plasma:
    pc = w.particle_cells()
    n0, n1, _ = w.n3
    if w.dims == 3:
        nslab, cells_per_slab = pc[2], pc[0] * pc[1]
    else:
        nslab, cells_per_slab = pc[1], pc[0]
    slabs = range(nslab) if slabs is None else slabs
    per_slab = cells_per_slab * w.ppc
    total = per_slab * len(slabs)
    cell = np.empty(total, dtype=np.int32)
    off = np.zeros((3, total), dtype=np.float32)
    u = np.zeros((3, total), dtype=np.float32)
    if w.dims == 3:
        ii, jj = np.meshgrid(np.arange(pc[0]), np.arange(pc[1]), indexing="xy")
        base_cells = (ii.ravel() + n0 * jj.ravel()).astype(np.int64)
    else:
        base_cells = np.arange(pc[0], dtype=np.int64)
    for t, s in enumerate(slabs):
        rng = np.random.default_rng([w.seed, int(s), *stream])
        lo, hi = t * per_slab, (t + 1) * per_slab
        slab_cells = base_cells + (n0 * n1 * s if w.dims == 3 else n0 * s)
        cell[lo:hi] = np.repeat(slab_cells, w.ppc).astype(np.int32)
        if quiet:
            side = int(round(w.ppc ** (1.0 / w.dims)))
            assert side ** w.dims == w.ppc, "quiet start needs ppc = k^dims"
            g = (np.arange(side) + 0.5) / side
            grids = np.meshgrid(*([g] * w.dims), indexing="ij")
            sub = np.stack([a.ravel() for a in grids])  # (dims, ppc)
            for d in range(w.dims):
                off[d, lo:hi] = np.tile(sub[d], cells_per_slab).astype(np.float32)
        else:
            off[:, lo:hi] = _uniform_offsets(rng, per_slab, w.dims)
        if u_th > 0.0:
            u[:, lo:hi] = _round32(rng.normal(0.0, u_th, size=(3, per_slab)))
    q = None
    if w.ramp_cells > 0.0:
        X = Plasma(cell, off, u, None, q_const).global_positions(w)[:, 0]
        dens = np.clip(X / w.ramp_cells, 0.0, 1.0)
        q = _round32(sign * dens / w.ppc)
    return Plasma(cell, off, u, q, q_const)


def inject_column(w: Workload, shift: int, ions: bool = False) -> Plasma:
    """Plasma entering the front particle column (x = n0 - 2) of a moving
    window at its ``shift``-th move (1, 2, ...): ``ppc`` particles per cell of
    the column, cells in storage order (y fastest, then z), drawn like the
    initial plasma from a child seed of their own (offsets U[0,1)^D, momenta
    N(0, u_th^2), FP32); the charge follows the density at the particle's lab
    position x + shift (the window has moved ``shift`` cells)."""
    pc = w.particle_cells()
    n0, n1, _ = w.n3
    ncol = pc[1] * (pc[2] if w.dims == 3 else 1)
    count = ncol * w.ppc
    rng = np.random.default_rng([w.seed, 7_000_000 + int(shift), 1 if ions else 0])
    cy = np.arange(ncol) % pc[1]
    cz = np.arange(ncol) // pc[1] if w.dims == 3 else np.zeros(ncol, dtype=np.int64)
    cell = np.repeat((n0 - 2) + n0 * (cy + n1 * cz), w.ppc).astype(np.int32)
    off = _uniform_offsets(rng, count, w.dims)
    u = np.zeros((3, count), dtype=np.float32)
    u_th = (w.ions.u_th if ions else w.u_th)
    if u_th > 0.0:
        u[:] = _round32(rng.normal(0.0, u_th, size=(3, count)))
    sign = 1.0 if ions else -1.0
    q_const = w.q_const_ions if ions else w.q_const
    q = None
    if w.ramp_cells > 0.0:
        x_lab = (n0 - 2) + off[0].astype(np.float64) + shift
        q = _round32(sign * np.clip(x_lab / w.ramp_cells, 0.0, 1.0) / w.ppc)
    return Plasma(cell, off, u, q, q_const, extra={"ppc": w.ppc})


def laser_fields(w: Workload, a0: float | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Initial E, B of shape (3, n2, n1, n0), FP32-representable float64.

    Zero when the workload has no laser.  Samples outside the domain of an
    open axis (half-integer positions beyond the last node) are zero.
    """
    n0, n1, n2 = w.n3
    E = np.zeros((3, n2, n1, n0), dtype=np.float64)
    B = np.zeros_like(E)
    if w.laser is None:
        return E, B
    L = w.laser
    a0 = L.a0 if a0 is None else a0
    dx, dy, dz = w.dx3
    lengths = [(w.n3[d] - (1 if w.bc3[d] == OPEN else 0)) * w.dx3[d] for d in range(3)]
    yc, zc = 0.5 * lengths[1], 0.5 * lengths[2]

    def profile(x, y, z):
        r2 = (y - yc) ** 2 + ((z - zc) ** 2 if w.dims == 3 else 0.0)
        xi = x - L.x_center
        env = np.exp(-r2 / L.waist ** 2) * np.exp(-(xi ** 2) / L.tau ** 2)
        val = a0 * L.omega0 * env * np.cos(L.omega0 * xi)
        return np.where(np.abs(xi) > 3.0 * L.tau, 0.0, val)

    k, j, i = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    zpos = k * dz if w.dims == 3 else 0.0
    # E_y at (i, j+1/2, k); B_z at (i+1/2, j+1/2, k)
    E[1] = profile(i * dx, (j + 0.5) * dy, zpos)
    B[2] = profile((i + 0.5) * dx, (j + 0.5) * dy, zpos)
    # half-integer samples beyond the last node of an open axis are outside
    if w.bc3[1] == OPEN:
        E[1][:, n1 - 1, :] = 0.0
        B[2][:, n1 - 1, :] = 0.0
    if w.bc3[0] == OPEN:
        B[2][:, :, n0 - 1] = 0.0
    E = _round32(E).astype(np.float64)
    B = _round32(B).astype(np.float64)
    return E, B
