"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare particle by particle (matched by id) and
sample by sample."""
import os
import sys

import numpy as np

import oracle as O
from paper_1310_0930_amd import inputs as I

TOL = {8: 1e-12, 4: 1e-5}  # positions (cells) and momenta (relative to rms |u|)


def say(*a):
    print("[parity]", *a, flush=True)
    sys.stdout.flush()


def oracle_threads():
    return max(1, min(16, os.cpu_count() or 1))


def oracle_config(w):
    return O.Config(w.dims, w.n3, w.dx3, w.dt, w.order, w.bc3)


def inputs_for(w, quiet=False):
    pl = I.make_plasma(w, quiet=quiet)
    E, B = I.laser_fields(w)
    return pl, E, B


def oracle_state(w, pl, E, B):
    return O.State(oracle_config(w), pl.global_positions(w), pl.u.T.astype(np.float64),
                   pl.charges(), E, B)


def gpu_sim(w, real_bytes, pl, E, B, sort_every=None):
    from paper_1310_0930_amd.pic import Simulation
    if sort_every is not None:
        w = w.with_(sort_every=sort_every)
    sim = Simulation.from_workload(w, real_bytes=real_bytes)
    sim.load(pl, E, B)
    return sim


def compare(w, sim, ref, st=None):
    """Errors of the GPU state against the oracle state `ref`."""
    st = st or sim.download()
    Xg, alive_g = sim.positions(st)
    ids = st["id"]
    n = np.array(w.n3, dtype=np.float64)
    Xr = ref.X[ids]
    ur = ref.u[ids]
    alive_r = ref.alive[ids].astype(bool)
    # every particle the oracle still has alive is among the GPU's slots (the
    # GPU's sort compacts absorbed particles away)
    out = {"alive_mismatch": int(np.sum(alive_g != alive_r))
           + abs(int(ref.alive.astype(bool).sum()) - int(alive_g.sum()))}
    both = alive_g & alive_r
    dX = Xg - Xr
    for d in range(w.dims):
        if w.bc3[d] == I.PERIODIC:
            dX[:, d] -= n[d] * np.round(dX[:, d] / n[d])
    dX[:, w.dims:] = 0.0
    out["pos"] = float(np.abs(dX[both]).max()) if both.any() else 0.0
    ug = st["u"].T
    rms = float(np.sqrt(np.mean(np.sum(ur[both] ** 2, axis=1)))) if both.any() else 1.0
    out["u"] = float(np.abs(ug[both] - ur[both]).max() / max(rms, 1e-300)) if both.any() else 0.0
    for name in ("E", "B", "J"):
        a, b = st[name], getattr(ref, name)
        scale = np.abs(b).max()
        out[name] = float(np.abs(a - b).max() / scale) if scale > 0 else float(np.abs(a).max())
    return out
