"""FP64 CPU oracle of the fully relativistic EM-PIC step (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (plain C++
loops, see ``pic_oracle.cpp``) with numpy arrays and shares no code with the
HIP library.

Conventions: positions ``X`` are global, in cell units, shape (np, 3) FP64
(the z column is ignored in 2D); momenta ``u`` = gamma*beta, shape (np, 3);
charges ``q`` shape (np,); ``alive`` int8 (np,); fields ``E, B, J`` shape
(3, n2, n1, n0) FP64 (x fastest).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

PERIODIC, OPEN = 0, 1


class _Cfg(C.Structure):
    _fields_ = [("dims", C.c_int32), ("n", C.c_int32 * 3), ("dx", C.c_double * 3),
                ("dt", C.c_double), ("order", C.c_int32), ("bc", C.c_int32 * 3),
                ("q_over_m", C.c_double)]


@dataclass
class Config:
    dims: int
    n: tuple
    dx: tuple
    dt: float
    order: int
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)
    q_over_m: float = -1.0

    def c(self) -> _Cfg:
        n = list(self.n) + [1] * (3 - len(self.n))
        dx = list(self.dx) + [1.0] * (3 - len(self.dx))
        bc = list(self.bc) + [PERIODIC] * (3 - len(self.bc))
        return _Cfg(self.dims, (C.c_int32 * 3)(*n), (C.c_double * 3)(*dx), self.dt,
                    self.order, (C.c_int32 * 3)(*bc), self.q_over_m)

    @property
    def shape(self):
        n = list(self.n) + [1] * (3 - len(self.n))
        return (n[2], n[1], n[0])

    @property
    def ncell(self) -> int:
        s = self.shape
        return s[0] * s[1] * s[2]

    def zeros_field(self):
        return np.zeros((3,) + self.shape, dtype=np.float64)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        P = C.c_void_p
        i64, i32 = C.c_int64, C.c_int32
        cfgp = C.POINTER(_Cfg)
        sig = {
            "oracle_shape": [i32, C.c_double, P, P],
            "oracle_gather": [cfgp, i64, P, P, P, P, P],
            "oracle_boris": [cfgp, i64, P, P, P],
            "oracle_deposit_paths": [cfgp, i64, P, P, P, P, P],
            "oracle_push_deposit": [cfgp, i64, P, P, P, P, P, P, P, i32],
            "oracle_push_deposit_add": [cfgp, i64, P, P, P, P, P, P, P, i32],
            "oracle_field_advance": [cfgp, P, P, P],
            "oracle_step": [cfgp, i64, P, P, P, P, P, P, P, i32, i32],
            "oracle_step_jvp": [cfgp, i64, P, P, P, P, P, P, P, P, P, P, P, P, i32],
            "oracle_deposit_rho": [cfgp, i64, P, P, P, P],
            "oracle_divergence": [cfgp, P, P],
            "oracle_energies": [cfgp, i64, P, P, P, P, P, P, P],
            "oracle_curl_e": [cfgp, P, P],
            "oracle_curl_b": [cfgp, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = None
        _LIB = L
    return _LIB


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def shape(order: int, X: float):
    """Order-n B-spline weights at X: (first node index, weights)."""
    base = np.zeros(1, dtype=np.int64)
    w = np.zeros(5, dtype=np.float64)  # up to order 4
    lib().oracle_shape(order, float(X), _ptr(base), _ptr(w))
    return int(base[0]), w[: order + 1].copy()


def gather(cfg: Config, X, E, B):
    X = _f64(X, (-1, 3))
    E, B = _f64(E), _f64(B)
    Ep = np.zeros_like(X)
    Bp = np.zeros_like(X)
    lib().oracle_gather(C.byref(cfg.c()), X.shape[0], _ptr(X), _ptr(E), _ptr(B), _ptr(Ep), _ptr(Bp))
    return Ep, Bp


def boris(cfg: Config, u, Ep, Bp):
    u = _f64(u, (-1, 3)).copy()
    Ep, Bp = _f64(Ep, (-1, 3)), _f64(Bp, (-1, 3))
    lib().oracle_boris(C.byref(cfg.c()), u.shape[0], _ptr(u), _ptr(Ep), _ptr(Bp))
    return u


def deposit_paths(cfg: Config, X0, X1, q, vz=None, J=None):
    X0, X1 = _f64(X0, (-1, 3)), _f64(X1, (-1, 3))
    q = _f64(np.broadcast_to(q, (X0.shape[0],)))
    vz = None if vz is None else _f64(np.broadcast_to(vz, (X0.shape[0],)))
    if J is None:
        J = cfg.zeros_field()
    lib().oracle_deposit_paths(C.byref(cfg.c()), X0.shape[0], _ptr(X0), _ptr(X1), _ptr(q),
                               _ptr(vz), _ptr(J))
    return J


@dataclass
class State:
    """Particles and fields advanced in place by the oracle."""
    cfg: Config
    X: np.ndarray
    u: np.ndarray
    q: np.ndarray
    E: np.ndarray
    B: np.ndarray
    alive: np.ndarray = None
    J: np.ndarray = None
    extra: dict = field(default_factory=dict)

    def __post_init__(self):
        self.X = _f64(self.X, (-1, 3)).copy()
        self.u = _f64(self.u, (-1, 3)).copy()
        self.q = _f64(np.broadcast_to(self.q, (self.X.shape[0],))).copy()
        self.E = _f64(self.E).reshape((3,) + self.cfg.shape).copy()
        self.B = _f64(self.B).reshape((3,) + self.cfg.shape).copy()
        if self.alive is None:
            self.alive = np.ones(self.X.shape[0], dtype=np.int8)
        self.alive = np.ascontiguousarray(self.alive, dtype=np.int8).copy()
        if self.J is None:
            self.J = self.cfg.zeros_field()
        self.nstep = 0          # steps taken (time of J: (nstep + 1/2) dt)
        self.antenna = None     # Antenna, or None

    @property
    def np(self) -> int:
        return self.X.shape[0]

    def copy(self) -> "State":
        return State(self.cfg, self.X, self.u, self.q, self.E, self.B, self.alive, self.J.copy())

    def push_deposit(self, nthreads: int = 1):
        lib().oracle_push_deposit(C.byref(self.cfg.c()), self.np, _ptr(self.X), _ptr(self.u),
                                  _ptr(self.q), _ptr(self.alive), _ptr(self.E), _ptr(self.B),
                                  _ptr(self.J), int(nthreads))

    def field_advance(self):
        lib().oracle_field_advance(C.byref(self.cfg.c()), _ptr(self.E), _ptr(self.B), _ptr(self.J))

    def step(self, nsteps: int = 1, nthreads: int = 1):
        if self.antenna is None:
            lib().oracle_step(C.byref(self.cfg.c()), self.np, _ptr(self.X), _ptr(self.u),
                              _ptr(self.q), _ptr(self.alive), _ptr(self.E), _ptr(self.B),
                              _ptr(self.J), int(nsteps), int(nthreads))
            self.nstep += nsteps
            return
        for _ in range(nsteps):  # push, add the antenna's current, advance
            self.push_deposit(nthreads)
            self.J += antenna_current(self.cfg, self.antenna, (self.nstep + 0.5) * self.cfg.dt)
            self.field_advance()
            self.nstep += 1

    def step_jvp(self, nsteps, dX, du, dE, dB, dJ=None):
        """Advance in place and return the tangents (dX, du, dE, dB, dJ)."""
        dX = _f64(dX, (-1, 3)).copy()
        du = _f64(du, (-1, 3)).copy()
        dE = _f64(dE).reshape(self.E.shape).copy()
        dB = _f64(dB).reshape(self.B.shape).copy()
        dJ = np.zeros_like(self.J) if dJ is None else _f64(dJ).reshape(self.J.shape).copy()
        lib().oracle_step_jvp(C.byref(self.cfg.c()), self.np, _ptr(self.X), _ptr(dX), _ptr(self.u),
                              _ptr(du), _ptr(self.q), _ptr(self.alive), _ptr(self.E), _ptr(dE),
                              _ptr(self.B), _ptr(dB), _ptr(self.J), _ptr(dJ), int(nsteps))
        return dX, du, dE, dB, dJ

    def rho(self):
        out = np.zeros(self.cfg.shape, dtype=np.float64)
        lib().oracle_deposit_rho(C.byref(self.cfg.c()), self.np, _ptr(self.X), _ptr(self.q),
                                 _ptr(self.alive), _ptr(out))
        return out

    def energies(self):
        wf = C.c_double()
        wk = C.c_double()
        lib().oracle_energies(C.byref(self.cfg.c()), self.np, _ptr(self.u), _ptr(self.q),
                              _ptr(self.alive), _ptr(self.E), _ptr(self.B), C.byref(wf),
                              C.byref(wk))
        return wf.value, wk.value


@dataclass
class Species:
    """One particle species of a multi-species state: its charge-to-mass
    ratio, positions, momenta, charges and live flags (same conventions as
    State)."""
    q_over_m: float
    X: np.ndarray
    u: np.ndarray
    q: np.ndarray
    alive: np.ndarray = None

    def __post_init__(self):
        self.X = _f64(self.X, (-1, 3)).copy()
        self.u = _f64(self.u, (-1, 3)).copy()
        self.q = _f64(np.broadcast_to(self.q, (self.X.shape[0],))).copy()
        if self.alive is None:
            self.alive = np.ones(self.X.shape[0], dtype=np.int8)
        self.alive = np.ascontiguousarray(self.alive, dtype=np.int8).copy()

    @property
    def np(self) -> int:
        return self.X.shape[0]


class MultiState:
    """Several species in one set of fields (mobile ions, the LWFA-1 run of
    Sec. 6).  A step zeroes J, pushes every species in E^n, B^n and adds its
    current (each with its own q/m), then advances the fields once."""

    def __init__(self, cfg: Config, species, E, B):
        self.cfg = cfg
        self.species = list(species)
        self.E = _f64(E).reshape((3,) + cfg.shape).copy()
        self.B = _f64(B).reshape((3,) + cfg.shape).copy()
        self.J = cfg.zeros_field()
        self.nstep = 0
        self.antenna = None

    def _cfg(self, sp: Species) -> _Cfg:
        c = self.cfg.c()
        c.q_over_m = sp.q_over_m
        return c

    def push_deposit(self, nthreads: int = 1):
        self.J[:] = 0.0
        for sp in self.species:
            lib().oracle_push_deposit_add(C.byref(self._cfg(sp)), sp.np, _ptr(sp.X), _ptr(sp.u),
                                          _ptr(sp.q), _ptr(sp.alive), _ptr(self.E), _ptr(self.B),
                                          _ptr(self.J), int(nthreads))

    def field_advance(self):
        lib().oracle_field_advance(C.byref(self.cfg.c()), _ptr(self.E), _ptr(self.B), _ptr(self.J))

    def step(self, nsteps: int = 1, nthreads: int = 1):
        for _ in range(nsteps):
            self.push_deposit(nthreads)
            if self.antenna is not None:
                self.J += antenna_current(self.cfg, self.antenna, (self.nstep + 0.5) * self.cfg.dt)
            self.field_advance()
            self.nstep += 1

    def rho(self):
        """Total charge density (sum over species)."""
        out = np.zeros(self.cfg.shape, dtype=np.float64)
        part = np.zeros_like(out)
        for sp in self.species:
            lib().oracle_deposit_rho(C.byref(self._cfg(sp)), sp.np, _ptr(sp.X), _ptr(sp.q),
                                     _ptr(sp.alive), _ptr(part))
            out += part
        return out

    def energies(self):
        """Field energy and the kinetic energy of every species, summed."""
        wf = C.c_double()
        wk = C.c_double()
        total_k = 0.0
        for k, sp in enumerate(self.species):
            lib().oracle_energies(C.byref(self._cfg(sp)), sp.np, _ptr(sp.u), _ptr(sp.q),
                                  _ptr(sp.alive), _ptr(self.E), _ptr(self.B), C.byref(wf),
                                  C.byref(wk))
            total_k += wk.value
        return wf.value, total_k


# ---------------------------------------------------------------- window, antenna
@dataclass
class Antenna:
    """A current sheet on the plane of E samples x = x_index that radiates a
    laser pulse of peak field a0 omega0 both ways (polarization 1: y, 2: z)."""
    x_index: int
    polarization: int
    a0: float
    omega0: float
    waist: float
    tau: float
    t_center: float
    y_center: float
    z_center: float = 0.0


def antenna_current(cfg: Config, a: Antenna, t: float):
    """Current of the antenna at time t, shape (3, n2, n1, n0).  In the
    normalised Maxwell equations a sheet current K (per unit area) radiates
    E = -K/2 on both sides, so K = -2 a0 omega0 env(t) g(y, z) cos(omega0 (t -
    t_center)); on the grid the sheet occupies one cell along x: J = K/dx.
    env = exp(-(t - t_center)^2/tau^2) (zero beyond 3 tau), g = exp(-r^2/w^2)
    about (y_center, z_center), each sample at its own Yee position."""
    J = cfg.zeros_field()
    tr = t - a.t_center
    if abs(tr) > 3.0 * a.tau:
        return J
    nz, ny, nx = cfg.shape
    pol = a.polarization
    y = (np.arange(ny) + (0.5 if pol == 1 else 0.0)) * cfg.dx[1] - a.y_center
    if cfg.dims == 3:
        z = (np.arange(nz) + (0.5 if pol == 2 else 0.0)) * cfg.dx[2] - a.z_center
    else:
        z = np.zeros(1)
    r2 = z[:, None] ** 2 + y[None, :] ** 2
    K = -2.0 * a.a0 * a.omega0 * np.exp(-tr * tr / a.tau ** 2) * np.cos(a.omega0 * tr)
    sheet = K / cfg.dx[0] * np.exp(-r2 / a.waist ** 2)
    # samples half-way beyond the last node of an open axis are outside
    if cfg.bc[1] == OPEN and pol == 1:
        sheet[:, ny - 1] = 0.0
    if cfg.dims == 3 and cfg.bc[2] == OPEN and pol == 2:
        sheet[nz - 1, :] = 0.0
    J[pol, :, :, a.x_index] = sheet
    return J


def window_shift(state, injects=()):
    """Move the window one cell along x (the window follows the laser, Sec. 2):
    E and B shift one cell toward -x with an empty front plane, J is zeroed,
    particles move one cell down (those leaving at x < 0 die) and each
    species appends the particles of its entry in ``injects``: (X, u, q) in
    window coordinates (cell units), or None."""
    for F in (state.E, state.B):
        F[..., :-1] = F[..., 1:].copy()
        F[..., -1] = 0.0
    state.J[:] = 0.0
    target = state.species if isinstance(state, MultiState) else [state]
    for k, sp in enumerate(target):
        live = sp.alive > 0
        sp.X[live, 0] -= 1.0
        sp.alive[live & (sp.X[:, 0] < 0.0)] = 0
        inj = injects[k] if k < len(injects) else None
        if inj is None:
            continue
        Xn, un, qn = (_f64(inj[0], (-1, 3)), _f64(inj[1], (-1, 3)), _f64(inj[2]))
        sp.X = np.concatenate([sp.X, Xn])
        sp.u = np.concatenate([sp.u, un])
        sp.q = np.concatenate([sp.q, qn])
        sp.alive = np.concatenate([sp.alive, np.ones(Xn.shape[0], dtype=np.int8)])


def divergence(cfg: Config, V):
    V = _f64(V).reshape((3,) + cfg.shape)
    out = np.zeros(cfg.shape, dtype=np.float64)
    lib().oracle_divergence(C.byref(cfg.c()), _ptr(V), _ptr(out))
    return out


def curl_e(cfg: Config, E):
    E = _f64(E).reshape((3,) + cfg.shape)
    out = np.zeros_like(E)
    lib().oracle_curl_e(C.byref(cfg.c()), _ptr(E), _ptr(out))
    return out


def curl_b(cfg: Config, B):
    B = _f64(B).reshape((3,) + cfg.shape)
    out = np.zeros_like(B)
    lib().oracle_curl_b(C.byref(cfg.c()), _ptr(B), _ptr(out))
    return out


def interior_margin(order: int) -> int:
    """Node planes next to an open face excluded from the conservation checks:
    a particle absorbed just beyond the face (X outside [0, n-1)) still
    reaches order//2 node planes inside with its shape, and the face plane
    itself loses the currents dropped outside."""
    return 1 + order // 2


def interior_mask(cfg: Config):
    """Nodes away from open faces (where continuity and Gauss are exact)."""
    m = np.ones(cfg.shape, dtype=bool)
    n = list(cfg.n) + [1] * (3 - len(cfg.n))
    r = interior_margin(cfg.order)
    for d in range(cfg.dims):
        if cfg.bc[d] == OPEN:
            sl = [slice(None)] * 3
            ax = 2 - d
            sl[ax] = slice(0, r)
            m[tuple(sl)] = False
            sl[ax] = slice(n[d] - r, n[d])
            m[tuple(sl)] = False
    return m


def continuity_residual(cfg: Config, rho0, rho1, J):
    """(rho^{n+1} - rho^n)/dt + D.J at the nodes (zero off the interior)."""
    r = (rho1 - rho0) / cfg.dt + divergence(cfg, J)
    return np.where(interior_mask(cfg), r, 0.0)
