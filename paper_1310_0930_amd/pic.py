"""Thin ctypes binding of libpic (``include/pic.h``).

The module-level functions carry the C names (``pic_create``, ``pic_sort``,
``pic_push_deposit``, ``pic_push_deposit_add``, ``pic_field_advance``,
``pic_step``, ``pic_step_species``, ``pic_deposit_rho``,
``pic_deposit_rho_add``, ``pic_diagnostics``, ``pic_diagnostics_species``,
``pic_read_flags``, the adjoints) and only
marshal arguments: every step of the method runs in the HIP kernels of
``libpic.so``.  PyTorch provides device memory and the stream.  There is no
fallback: a missing library raises.

``Simulation`` bundles one context with its particle, field and workspace
tensors (SoA, FP32 or FP64); ``add_species`` attaches further species
(mobile ions) that share its fields.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")
_LIB = None

PIC_OK, PIC_EINVAL, PIC_ECOURANT, PIC_EHIP, PIC_ESTATE, PIC_EDEVICE, PIC_ELDS = 0, -1, -2, -3, -4, -5, -6
PIC_ESCRATCH = -7
PIC_BC_PERIODIC, PIC_BC_OPEN = 0, 1
FLAG_NAMES = {1: "nonfinite", 2: "offset", 4: "cell", 8: "overspeed"}


class PicConfig(C.Structure):
    _fields_ = [("dims", C.c_int32), ("n", C.c_int32 * 3), ("dx", C.c_double * 3),
                ("dt", C.c_double), ("order", C.c_int32), ("real_bytes", C.c_int32),
                ("bc", C.c_int32 * 3), ("tile", C.c_int32 * 3), ("sort_every", C.c_int32),
                ("drift", C.c_int32), ("q_over_m", C.c_double), ("q_const", C.c_double)]


class PicParticles(C.Structure):
    _fields_ = [("np", C.c_int64), ("cell", C.c_void_p), ("off", C.c_void_p * 3),
                ("u", C.c_void_p * 3), ("q", C.c_void_p), ("id", C.c_void_p)]


class PicFields(C.Structure):
    _fields_ = [("E", C.c_void_p * 3), ("B", C.c_void_p * 3), ("J", C.c_void_p * 3)]


class PicDiag(C.Structure):
    _fields_ = [("gauss_max", C.c_double), ("gauss_rel", C.c_double), ("cont_max", C.c_double),
                ("cont_rel_l2", C.c_double), ("cont_rel_inf", C.c_double),
                ("w_field", C.c_double), ("w_kin", C.c_double), ("rho_max", C.c_double),
                ("n_alive", C.c_int64), ("flags", C.c_uint32), ("n_slowpath", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PicInject(C.Structure):
    _fields_ = [("n", C.c_int64), ("ppc", C.c_int32), ("off", C.c_void_p * 3),
                ("u", C.c_void_p * 3), ("q", C.c_void_p), ("id_first", C.c_int64)]


class PicAntenna(C.Structure):
    _fields_ = [("x_index", C.c_int32), ("polarization", C.c_int32), ("a0", C.c_double),
                ("omega0", C.c_double), ("waist", C.c_double), ("tau", C.c_double),
                ("t_center", C.c_double), ("y_center", C.c_double), ("z_center", C.c_double)]


class PicError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {strerror(status)} ({status})")
        self.status = status


# signatures of every exported entry point (the C ABI of include/pic.h)
_SIGS = {
    "pic_create": ([C.POINTER(PicConfig), C.POINTER(C.c_void_p)], C.c_int),
    "pic_destroy": ([C.c_void_p], C.c_int),
    "pic_workspace_bytes": ([C.c_void_p, C.c_int64, C.POINTER(C.c_size_t)], C.c_int),
    "pic_sort": ([C.c_void_p, C.POINTER(PicParticles), C.c_void_p, C.c_void_p], C.c_int),
    "pic_push_deposit": ([C.c_void_p, C.POINTER(PicParticles), C.POINTER(PicFields), C.c_void_p,
                          C.c_void_p], C.c_int),
    "pic_field_advance": ([C.c_void_p, C.POINTER(PicFields), C.c_void_p, C.c_void_p], C.c_int),
    "pic_field_advance_static": ([C.c_void_p, C.POINTER(PicFields), C.c_void_p], C.c_int),
    "pic_step": ([C.c_void_p, C.POINTER(PicParticles), C.POINTER(PicFields), C.c_int32, C.c_void_p,
                  C.c_void_p], C.c_int),
    "pic_deposit_rho": ([C.c_void_p, C.POINTER(PicParticles), C.c_void_p, C.c_void_p, C.c_void_p],
                        C.c_int),
    "pic_diagnostics": ([C.c_void_p, C.POINTER(PicParticles), C.POINTER(PicFields), C.c_void_p,
                         C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(PicDiag), C.c_void_p,
                         C.c_void_p], C.c_int),
    "pic_push_deposit_add": ([C.c_void_p, C.POINTER(PicParticles), C.POINTER(PicFields),
                              C.c_void_p, C.c_void_p], C.c_int),
    "pic_step_species": ([C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(PicFields),
                          C.c_int32, C.c_void_p], C.c_int),
    "pic_deposit_rho_add": ([C.c_void_p, C.POINTER(PicParticles), C.c_void_p, C.c_void_p,
                             C.c_void_p], C.c_int),
    "pic_diagnostics_species": ([C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.POINTER(PicFields), C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.POINTER(PicDiag), C.c_void_p], C.c_int),
    "pic_window_shift": ([C.c_void_p, C.POINTER(PicParticles), C.c_int64, C.POINTER(PicFields),
                          C.POINTER(PicInject), C.c_void_p, C.c_void_p], C.c_int),
    "pic_antenna_add": ([C.c_void_p, C.POINTER(PicFields), C.POINTER(PicAntenna), C.c_double,
                         C.c_void_p], C.c_int),
    "pic_set_antenna": ([C.c_void_p, C.POINTER(PicAntenna)], C.c_int),
    "pic_field_advance_adjoint": ([C.c_void_p, C.POINTER(PicFields), C.c_void_p, C.c_void_p],
                                  C.c_int),
    "pic_push_deposit_adjoint": ([C.c_void_p, C.POINTER(PicParticles), C.POINTER(PicFields),
                                  C.POINTER(PicFields), C.POINTER(PicParticles), C.c_void_p,
                                  C.c_void_p], C.c_int),
    "pic_read_flags": ([C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_uint32),
                        C.POINTER(C.c_int64), C.c_void_p], C.c_int),
    "pic_read_push_counts": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                              C.c_void_p], C.c_int),
    "pic_strerror": ([C.c_int], C.c_char_p),
}


def lib():
    """Load libpic.so (built in-tree by ``build.py``); raises if it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_1310_0930_amd.build` "
                               "(there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = L
    return _LIB


def strerror(status: int) -> str:
    return lib().pic_strerror(int(status)).decode()


def _check(status, what):
    if status != PIC_OK:
        raise PicError(status, what)


def make_config(dims, n, dx, dt, order, real_bytes=4, bc=(0, 0, 0), sort_every=20,
                q_over_m=-1.0, q_const=-1.0, tile=(0, 0, 0), drift=-1) -> PicConfig:
    n = list(n) + [1] * (3 - len(n))
    dx = list(dx) + [1.0] * (3 - len(dx))
    bc = list(bc) + [0] * (3 - len(bc))
    return PicConfig(dims, (C.c_int32 * 3)(*n), (C.c_double * 3)(*dx), float(dt), int(order),
                     int(real_bytes), (C.c_int32 * 3)(*bc), (C.c_int32 * 3)(*tile), int(sort_every),
                     int(drift), float(q_over_m), float(q_const))


# ---------------------------------------------------------------- C-named wrappers
def pic_create(cfg: PicConfig):
    h = C.c_void_p()
    _check(lib().pic_create(C.byref(cfg), C.byref(h)), "pic_create")
    return h


def pic_destroy(ctx):
    return lib().pic_destroy(ctx)


def pic_workspace_bytes(ctx, np_):
    b = C.c_size_t()
    _check(lib().pic_workspace_bytes(ctx, int(np_), C.byref(b)), "pic_workspace_bytes")
    return b.value


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def pic_sort(ctx, parts: PicParticles, ws, stream=None):
    _check(lib().pic_sort(ctx, C.byref(parts), C.c_void_p(ws), _stream(stream)), "pic_sort")


def pic_push_deposit(ctx, parts: PicParticles, fields: PicFields, ws, stream=None):
    _check(lib().pic_push_deposit(ctx, C.byref(parts), C.byref(fields), C.c_void_p(ws),
                                  _stream(stream)), "pic_push_deposit")


def pic_field_advance(ctx, fields: PicFields, ws, stream=None):
    _check(lib().pic_field_advance(ctx, C.byref(fields), C.c_void_p(ws), _stream(stream)),
           "pic_field_advance")


def pic_field_advance_static(ctx, fields: PicFields, stream=None):
    _check(lib().pic_field_advance_static(ctx, C.byref(fields), _stream(stream)),
           "pic_field_advance_static")


def pic_step(ctx, parts: PicParticles, fields: PicFields, nsteps, ws, stream=None):
    _check(lib().pic_step(ctx, C.byref(parts), C.byref(fields), int(nsteps), C.c_void_p(ws),
                          _stream(stream)), "pic_step")


def pic_deposit_rho(ctx, parts: PicParticles, rho_ptr, ws, stream=None):
    _check(lib().pic_deposit_rho(ctx, C.byref(parts), C.c_void_p(rho_ptr), C.c_void_p(ws),
                                 _stream(stream)), "pic_deposit_rho")


def pic_diagnostics(ctx, parts, fields, rho_prev, gauss_ref, rho_out, gauss_out, ws, stream=None):
    d = PicDiag()
    _check(lib().pic_diagnostics(ctx, C.byref(parts), C.byref(fields), C.c_void_p(rho_prev or 0),
                                 C.c_void_p(gauss_ref or 0), C.c_void_p(rho_out),
                                 C.c_void_p(gauss_out or 0), C.byref(d), C.c_void_p(ws),
                                 _stream(stream)), "pic_diagnostics")
    return d


def _species_arrays(ctxs, parts, wss):
    n = len(ctxs)
    if not (len(parts) == n and len(wss) == n):
        raise ValueError("one context, particle set and workspace per species")
    pa = (C.POINTER(PicParticles) * n)(*[C.pointer(p) for p in parts])
    return (C.c_void_p * n)(*[C.cast(c, C.c_void_p) for c in ctxs]), pa, (C.c_void_p * n)(*wss)


def pic_push_deposit_add(ctx, parts: PicParticles, fields: PicFields, ws, stream=None):
    _check(lib().pic_push_deposit_add(ctx, C.byref(parts), C.byref(fields), C.c_void_p(ws),
                                      _stream(stream)), "pic_push_deposit_add")


def pic_step_species(ctxs, parts, wss, fields: PicFields, nsteps, stream=None):
    c, p, w = _species_arrays(ctxs, parts, wss)
    _check(lib().pic_step_species(len(ctxs), c, p, w, C.byref(fields), int(nsteps), _stream(stream)),
           "pic_step_species")


def pic_deposit_rho_add(ctx, parts: PicParticles, rho_ptr, ws, stream=None):
    _check(lib().pic_deposit_rho_add(ctx, C.byref(parts), C.c_void_p(rho_ptr), C.c_void_p(ws),
                                     _stream(stream)), "pic_deposit_rho_add")


def pic_diagnostics_species(ctxs, parts, wss, fields, rho_prev, gauss_ref, rho_out, gauss_out,
                            stream=None):
    c, p, w = _species_arrays(ctxs, parts, wss)
    d = PicDiag()
    _check(lib().pic_diagnostics_species(len(ctxs), c, p, w, C.byref(fields),
                                         C.c_void_p(rho_prev or 0), C.c_void_p(gauss_ref or 0),
                                         C.c_void_p(rho_out), C.c_void_p(gauss_out or 0),
                                         C.byref(d), _stream(stream)), "pic_diagnostics_species")
    return d


def pic_window_shift(ctx, parts: PicParticles, capacity, fields, inject, ws, stream=None):
    _check(lib().pic_window_shift(ctx, C.byref(parts), int(capacity),
                                  C.byref(fields) if fields is not None else None,
                                  C.byref(inject) if inject is not None else None,
                                  C.c_void_p(ws), _stream(stream)), "pic_window_shift")


def pic_antenna_add(ctx, fields: PicFields, antenna: PicAntenna, t, stream=None):
    _check(lib().pic_antenna_add(ctx, C.byref(fields), C.byref(antenna), float(t), _stream(stream)),
           "pic_antenna_add")


def pic_set_antenna(ctx, antenna):
    _check(lib().pic_set_antenna(ctx, C.byref(antenna) if antenna is not None else None),
           "pic_set_antenna")


def antenna_struct(x_index, polarization, a0, omega0, waist, tau, t_center, y_center,
                   z_center=0.0) -> PicAntenna:
    return PicAntenna(int(x_index), int(polarization), float(a0), float(omega0), float(waist),
                      float(tau), float(t_center), float(y_center), float(z_center))


def pic_field_advance_adjoint(ctx, lam_fields: PicFields, ws, stream=None):
    _check(lib().pic_field_advance_adjoint(ctx, C.byref(lam_fields), C.c_void_p(ws), _stream(stream)),
           "pic_field_advance_adjoint")


def pic_push_deposit_adjoint(ctx, parts: PicParticles, fields: PicFields, lam_fields: PicFields,
                             lam_parts: PicParticles, ws, stream=None):
    _check(lib().pic_push_deposit_adjoint(ctx, C.byref(parts), C.byref(fields), C.byref(lam_fields),
                                          C.byref(lam_parts), C.c_void_p(ws), _stream(stream)),
           "pic_push_deposit_adjoint")


def fields_struct(E, B, J=None) -> PicFields:
    """PicFields over (3, ncell) device tensors."""
    nul = (C.c_void_p * 3)(None, None, None)
    return PicFields((C.c_void_p * 3)(*[E[c].data_ptr() for c in range(3)]),
                     (C.c_void_p * 3)(*[B[c].data_ptr() for c in range(3)]),
                     nul if J is None else (C.c_void_p * 3)(*[J[c].data_ptr() for c in range(3)]))


def particles_struct(np_, cell, off, u, q=None, id_=None) -> PicParticles:
    """PicParticles over SoA device tensors (off and u are (3, np))."""
    return PicParticles(
        int(np_), None if cell is None else cell.data_ptr(),
        (C.c_void_p * 3)(*[off[d].data_ptr() for d in range(3)]),
        (C.c_void_p * 3)(*[u[c].data_ptr() for c in range(3)]),
        None if q is None else q.data_ptr(), None if id_ is None else id_.data_ptr())


def pic_read_flags(ctx, ws, clear=False, stream=None):
    f = C.c_uint32()
    s = C.c_int64()
    st = lib().pic_read_flags(ctx, C.c_void_p(ws), int(bool(clear)), C.byref(f), C.byref(s),
                              _stream(stream))
    if st not in (PIC_OK, PIC_EDEVICE):
        _check(st, "pic_read_flags")
    return f.value, s.value


def pic_read_push_counts(ctx, ws, stream=None):
    r = C.c_int64()
    s = C.c_int64()
    _check(lib().pic_read_push_counts(ctx, C.c_void_p(ws), C.byref(r), C.byref(s), _stream(stream)),
           "pic_read_push_counts")
    return r.value, s.value


# ---------------------------------------------------------------- simulation
@dataclass
class Diag:
    raw: dict
    rho: object  # torch tensor (FP64, ncell)


class Simulation:
    """One context plus its device tensors (torch, on ``device``)."""

    def __init__(self, dims, n, dx, dt, order, real_bytes=4, bc=(0, 0, 0), sort_every=20,
                 q_over_m=-1.0, q_const=-1.0, device="cuda"):
        import torch
        self.torch = torch
        self.dims = dims
        self.n = tuple(list(n) + [1] * (3 - len(n)))
        self.cfg = make_config(dims, n, dx, dt, order, real_bytes, bc, sort_every, q_over_m, q_const)
        self.ctx = pic_create(self.cfg)
        self.device = torch.device(device)
        self.real = torch.float64 if real_bytes == 8 else torch.float32
        self.ncell = self.n[0] * self.n[1] * self.n[2]
        self.np = 0
        self.ws = None
        self.E = torch.zeros((3, self.ncell), dtype=self.real, device=self.device)
        self.B = torch.zeros_like(self.E)
        self.J = torch.zeros_like(self.E)
        self._fields = PicFields((C.c_void_p * 3)(*[self.E[c].data_ptr() for c in range(3)]),
                                 (C.c_void_p * 3)(*[self.B[c].data_ptr() for c in range(3)]),
                                 (C.c_void_p * 3)(*[self.J[c].data_ptr() for c in range(3)]))

        self.species = []  # further species sharing these fields (add_species)
        self.q_over_m = q_over_m

    def add_species(self, plasma, q_over_m, q_const, with_id=True, capacity=None):
        """Another species on this grid (mobile ions): its own context (q/m,
        uniform charge), particle arrays and workspace, pushed in and
        depositing into this simulation's E, B, J.  Returns its Simulation."""
        c = self.cfg
        sp = Simulation(self.dims, self.n, tuple(c.dx), c.dt, c.order, c.real_bytes, tuple(c.bc),
                        c.sort_every, q_over_m, q_const, self.device)
        sp.E, sp.B, sp.J = self.E, self.B, self.J
        sp._fields = self._fields
        sp._load_particles(plasma, with_id, capacity)
        self.species.append(sp)
        return sp

    @classmethod
    def from_workload(cls, w, real_bytes=4, device="cuda", **kw):
        return cls(w.dims, w.n3, w.dx3, w.dt, w.order, real_bytes, w.bc3, w.sort_every, -1.0,
                   kw.pop("q_const", w.q_const), device)

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                pic_destroy(self.ctx)
                self.ctx = None
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    # ---- state upload / download
    def load(self, plasma, E=None, B=None, with_id=True, capacity=None):
        """Upload a Plasma (inputs.Plasma) and initial fields (3, n2, n1, n0).
        ``capacity`` (>= plasma.np) sizes the particle arrays for a moving
        window that appends particles."""
        torch = self.torch
        dev = self.device
        if E is not None:
            self.E.copy_(torch.from_numpy(np.asarray(E).reshape(3, -1)).to(dev, self.real))
        if B is not None:
            self.B.copy_(torch.from_numpy(np.asarray(B).reshape(3, -1)).to(dev, self.real))
        self.J.zero_()
        return self._load_particles(plasma, with_id, capacity)

    def _load_particles(self, plasma, with_id, capacity=None):
        torch = self.torch
        dev = self.device
        self.np = plasma.np
        cap = self.np if capacity is None else int(capacity)
        if cap < self.np:
            raise ValueError("capacity below the particle count")
        self.capacity = cap

        def put(a, dtype):
            t = torch.zeros(a.shape[:-1] + (cap,), dtype=dtype, device=dev)
            t[..., : self.np] = torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype)
            return t

        self.cell = put(plasma.cell, torch.int32)
        self.off = put(plasma.off, self.real)
        self.u = put(plasma.u, self.real)
        self.q = None if plasma.q is None else put(plasma.q, self.real)
        self.id = None
        if with_id:
            self.id = torch.arange(cap, dtype=torch.int32, device=dev)
        self.n_ids = self.np  # ids handed out so far (injected particles continue the count)
        nbytes = pic_workspace_bytes(self.ctx, cap)
        self.ws = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        self._parts = PicParticles(
            self.np, self.cell.data_ptr(),
            (C.c_void_p * 3)(*[self.off[d].data_ptr() for d in range(3)]),
            (C.c_void_p * 3)(*[self.u[c].data_ptr() for c in range(3)]),
            self.q.data_ptr() if self.q is not None else None,
            self.id.data_ptr() if self.id is not None else None)
        return self

    def download(self):
        """Host copies: cell, off (3,np), u (3,np), id, E, B, J (3, n2, n1, n0), float64."""
        shp = (3, self.n[2], self.n[1], self.n[0])
        n = self.np
        out = {
            "cell": self.cell[:n].cpu().numpy(),
            "off": self.off[:, :n].double().cpu().numpy(),
            "u": self.u[:, :n].double().cpu().numpy(),
            "id": None if self.id is None else self.id[:n].cpu().numpy(),
            "E": self.E.double().cpu().numpy().reshape(shp),
            "B": self.B.double().cpu().numpy().reshape(shp),
            "J": self.J.double().cpu().numpy().reshape(shp),
        }
        return out

    def positions(self, st=None):
        """Global positions (np, 3) in cell units and alive mask from a download."""
        st = st or self.download()
        c = st["cell"].astype(np.int64)
        alive = c >= 0
        cc = np.where(alive, c, 0)
        n0, n1, _ = self.n
        X = np.zeros((c.shape[0], 3))
        X[:, 0] = cc % n0 + st["off"][0]
        X[:, 1] = (cc // n0) % n1 + st["off"][1]
        if self.dims == 3:
            X[:, 2] = cc // (n0 * n1) + st["off"][2]
        return X, alive

    # ---- the hot path
    @property
    def stream(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def sort(self):
        """Tile sort; absorbed particles are compacted away (np drops to the
        live count)."""
        pic_sort(self.ctx, self._parts, self.ws.data_ptr(), self.stream)
        self.np = self._parts.np

    def push_deposit(self):
        pic_push_deposit(self.ctx, self._parts, self._fields, self.ws.data_ptr(), self.stream)

    def push_deposit_add(self):
        pic_push_deposit_add(self.ctx, self._parts, self._fields, self.ws.data_ptr(), self.stream)

    def field_advance(self):
        pic_field_advance(self.ctx, self._fields, self.ws.data_ptr(), self.stream)

    def step(self, nsteps=1):
        if self.species:
            all_ = [self] + self.species
            pic_step_species([s.ctx for s in all_], [s._parts for s in all_],
                             [s.ws.data_ptr() for s in all_], self._fields, nsteps, self.stream)
        else:
            pic_step(self.ctx, self._parts, self._fields, nsteps, self.ws.data_ptr(), self.stream)
        for s in [self] + self.species:  # sorts inside the steps compact
            s.np = s._parts.np

    def rho(self):
        """Charge density of all species (FP64, ncell)."""
        r = self.torch.zeros(self.ncell, dtype=self.torch.float64, device=self.device)
        pic_deposit_rho(self.ctx, self._parts, r.data_ptr(), self.ws.data_ptr(), self.stream)
        for sp in self.species:
            pic_deposit_rho_add(sp.ctx, sp._parts, r.data_ptr(), sp.ws.data_ptr(), self.stream)
        return r

    def diagnostics(self, rho_prev=None, gauss_ref=None, want_gauss=False):
        torch = self.torch
        rho = torch.zeros(self.ncell, dtype=torch.float64, device=self.device)
        g = torch.zeros_like(rho) if want_gauss else None
        all_ = [self] + self.species
        d = pic_diagnostics_species([s.ctx for s in all_], [s._parts for s in all_],
                                    [s.ws.data_ptr() for s in all_], self._fields,
                                    None if rho_prev is None else rho_prev.data_ptr(),
                                    None if gauss_ref is None else gauss_ref.data_ptr(),
                                    rho.data_ptr(), None if g is None else g.data_ptr(),
                                    self.stream)
        out = d.as_dict()
        out["gauss_field"] = g
        return Diag(out, rho)

    # ---- moving window and antenna
    def window_shift(self, inject=None, species_inject=()):
        """Move the window one cell along x: fields shift, particles move one
        cell down (leaving ones absorbed), and ``inject`` (an inputs.Plasma of
        the front column, or None) is appended; ``species_inject`` gives the
        front-column particles of each further species."""
        pic_window_shift(self.ctx, self._parts, self.capacity, self._fields,
                         self._inject_struct(inject), self.ws.data_ptr(), self.stream)
        self.np = self._parts.np
        for k, sp in enumerate(self.species):
            inj = species_inject[k] if k < len(species_inject) else None
            pic_window_shift(sp.ctx, sp._parts, sp.capacity, None, sp._inject_struct(inj),
                             sp.ws.data_ptr(), self.stream)
            sp.np = sp._parts.np

    def _inject_struct(self, plasma):
        if plasma is None or plasma.np == 0:
            return None
        torch = self.torch
        off = torch.from_numpy(np.ascontiguousarray(plasma.off)).to(self.device, self.real)
        u = torch.from_numpy(np.ascontiguousarray(plasma.u)).to(self.device, self.real)
        q = None if plasma.q is None else torch.from_numpy(plasma.q).to(self.device, self.real)
        self._inj_keep = (off, u, q)  # alive until the stream has consumed them
        ppc = plasma.extra.get("ppc", 1)
        first = self.n_ids
        self.n_ids += plasma.np
        return PicInject(plasma.np, int(ppc), (C.c_void_p * 3)(*[off[d].data_ptr() for d in range(3)]),
                         (C.c_void_p * 3)(*[u[c].data_ptr() for c in range(3)]),
                         q.data_ptr() if q is not None else None, first)

    def set_antenna(self, antenna):
        pic_set_antenna(self.ctx, antenna)

    def antenna_add(self, antenna, t):
        pic_antenna_add(self.ctx, self._fields, antenna, t, self.stream)

    def read_flags(self, clear=False):
        return pic_read_flags(self.ctx, self.ws.data_ptr(), clear, self.stream)

    def read_push_counts(self):
        """(re-binned, global-memory) pushes since the flags were last cleared."""
        return pic_read_push_counts(self.ctx, self.ws.data_ptr(), self.stream)
