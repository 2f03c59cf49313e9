"""Benchmark of the EM-PIC hot path on one MI355X.

A step is one pass of the whole hot path over the resident particle set:
tile sort when due (every ``sort_every`` steps), the fused
gather/push/deposit kernel and the FDTD field advance.  Prints one JSON line:
``value`` = particle pushes per second of whole steps (FP32 form), plus the
push/deposit kernel rate, its HBM roofline, the FP64 form, and the oracle
timed on the host cores as a CPU baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1310_0930_amd import inputs as I  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "particle pushes/sec (interp+push+deposit) and % HBM roofline, FP32 vs FP64"


def algorithmic_bytes(w, np_, real_bytes):
    """Bytes the push/deposit must move per step: particle state read and
    written once (cell + D offsets + 3 momenta, + q when per-particle), one
    read of E and B and one write of J per cell for every species."""
    per_particle = 2 * (4 + real_bytes * (w.dims + 3))
    if w.ramp_cells > 0:
        per_particle += real_bytes
    per_cell = 9 * real_bytes
    nspecies = 1 if w.ions is None else 2
    return np_ * per_particle + w.ncell * per_cell * nspecies


# LDS probe (liblds_probe.so): lane-operations per second of one LDS access
# kind with the 64 lanes of every wavefront `stride` elements apart.
PROBE_OPS = {"ds_read_b32": 0, "ds_read_b64": 1, "ds_add_u32": 2, "ds_add_u64": 3,
             "ds_add_f32": 4, "ds_add_f64": 5, "ds_read2_b32_adjacent": 6}
_PROBE = None


def lds_rate(op, stride=1, iters=2048, reps=3):
    """Whole-chip rate of LDS op `op` (G lane-ops/s, best of `reps` runs of
    8 workgroups of 1024 threads per compute unit)."""
    import ctypes as C
    import torch
    from paper_1310_0930_amd import build as B
    global _PROBE
    if _PROBE is None:
        _PROBE = (C.CDLL(B.PROBE_LIB), torch.zeros(1, dtype=torch.int64, device="cuda"))
    lib, sink = _PROBE
    blocks = 8 * torch.cuda.get_device_properties(0).multi_processor_count
    ms = C.c_float()
    best = float("inf")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for _ in range(reps):
        st = lib.lds_probe_run(PROBE_OPS[op], int(stride), int(iters), blocks,
                               C.c_void_p(sink.data_ptr()), stream, C.byref(ms))
        if st != 0:
            raise RuntimeError(f"lds_probe_run({op}, {stride}) failed: {st}")
        best = min(best, ms.value)
    return blocks * 1024 * iters / (best * 1e-3) / 1e9


def lds_probe_table(strides=(1, 2, 4, 8, 16, 32, 64, 128)):
    return {op: {str(s): round(lds_rate(op, s), 1) for s in strides} for op in PROBE_OPS}


def lds_replay(w, real_bytes, iters=64):
    """LDS cycles of the push kernel's access patterns (quadratic 3D, 8^3
    tiles) replayed by the LDS probe (lds_probe_pattern) for the lane layouts
    that the tile sort produces from this workload's plasma (its first 16 z
    planes: two layers of tiles, the first 64 tiles), with the particles at
    the positions the sort places them by (half a sort interval ahead on a
    straight line, which is where the layout is meant to be best), and for the ideal
    layout (each 32 consecutive lanes on 32 distinct bank residues, one
    class).  CU cycles per 64-particle batch: the gather (six 27-node
    stencils) and the current deposit (54 adds of one virtual segment)."""
    import ctypes as C
    import torch
    from paper_1310_0930_amd import build as B
    from paper_1310_0930_amd.pic import Simulation
    if w.dims != 3 or w.order != 2 or w.n3[2] < 16:
        return None
    lib = C.CDLL(B.PROBE_LIB)
    RX = 13  # region width: 8-cell tile, one allowance cell and the stencil reach on each side

    def region_cell(lx, ly, lz):
        return (lx + 2) + RX * ((ly + 2) + RX * (lz + 2))

    w2 = w.with_(n=(w.n3[0], w.n3[1], 16))
    sim = Simulation.from_workload(w2, real_bytes=real_bytes)
    sim.load(I.make_plasma(w, slabs=range(16), quiet=False), None, None, with_id=False)
    sim.sort()
    st = sim.download()
    c, o, u = st["cell"], st["off"], st["u"]
    n0, n1 = w.n3[0], w.n3[1]
    cx, cy, cz = c % n0, (c // n0) % n1, c // (n0 * n1)
    key = cx // 8 + (n0 // 8) * (cy // 8 + (n1 // 8) * (cz // 8))
    # the layout the sort aims at: every particle moved on the straight line
    # the sort estimates, half a sort interval ahead, inside its tile
    lc = [cx % 8, cy % 8, cz % 8]
    lp, op, inside = [], [], np.ones(len(c), dtype=bool)
    for d in range(3):
        x = o[d] + np.clip(u[d], -1.0, 1.0) * (0.5 * (w.sort_every - 1) * w.dt / w.dx3[d])
        f = np.floor(x)
        lp.append(lc[d] + f.astype(np.int64))
        op.append(x - f)
        inside &= (lp[d] >= 0) & (lp[d] < 8)
    lp = [np.where(inside, lp[d], lc[d]) for d in range(3)]
    op = [np.where(inside, op[d], o[d]) for d in range(3)]
    cls = (op[0] >= 0.5).astype(np.int64) | ((op[1] >= 0.5).astype(np.int64) << 1) | \
        ((op[2] >= 0.5).astype(np.int64) << 2)
    lane = region_cell(lp[0], lp[1], lp[2]) | (cls << 16)
    starts = np.searchsorted(key, np.arange(key.max() + 2))
    pats = []
    for t in range(min(64, int(key.max()) + 1)):
        v = lane[starts[t]:starts[t + 1]]
        pats.append(v[: len(v) // 64 * 64].reshape(-1, 64))
    rng = np.random.default_rng(1310)
    lc = np.arange(512)
    resid = (region_cell(lc % 8, (lc // 8) % 8, lc // 64)) % 32
    ideal = []
    for p in range(64):
        cells = [rng.choice(np.flatnonzero(resid == q)) for h in range(2) for q in range(32)]
        ideal.append(np.array([region_cell(x % 8, (x // 8) % 8, x // 64) | ((p % 8) << 16) for x in cells]))
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    blocks = 2 * torch.cuda.get_device_properties(0).multi_processor_count
    modes = {"gather": 4 if real_bytes == 4 else 5, "deposit": 2 if real_bytes == 4 else 3}
    out = {}
    for name, pat in (("as_sorted", np.concatenate(pats)), ("ideal", np.stack(ideal))):
        dev = torch.from_numpy(pat.astype(np.int32).reshape(-1)).cuda()
        row = {}
        for what, m in modes.items():
            ms, best = C.c_float(), float("inf")
            for _ in range(3):
                rc = lib.lds_probe_pattern(m, C.c_void_p(dev.data_ptr()), pat.shape[0], iters, blocks,
                                           C.c_void_p(sink.data_ptr()), stream, C.byref(ms))
                if rc != 0:
                    raise RuntimeError(f"lds_probe_pattern({m}) failed: {rc}")
                best = min(best, ms.value)
            waves = blocks * 16  # 1024-thread workgroups
            row[what] = round(best * 1e-3 * CLOCK_HZ / (waves * iters / CUS), 1)
        out[name] = row
    out["unit"] = "CU cycles per 64-particle batch"
    return out


def lds_atomics(w, np_, push_ms, real_bytes):
    """LDS atomic throughput of the push/deposit tile kernel against the
    conflict-free rate of the same instruction, measured in this run by the
    LDS probe: the Esirkepov current of each particle's first virtual
    segment adds 3 n (n+1)^2 samples in 3D and 2 n (n+1) + (n+1)^2 in 2D3V (a
    lower bound: the few particles that cross a stencil plane add more)."""
    n = w.order
    per = 3 * n * (n + 1) ** 2 if w.dims == 3 else 2 * n * (n + 1) + (n + 1) ** 2
    ops = per * np_
    ach = ops / (push_ms * 1e-3) / 1e9
    op = "ds_add_u64" if real_bytes == 4 else "ds_add_f64"
    peak = round(lds_rate(op), 1)
    return {"op": op + (" (exact fixed point)" if real_bytes == 4 else ""),
            "lane_ops_per_launch": int(ops), "achieved": round(ach, 1), "peak": peak,
            "peak_source": "LDS probe in this run: conflict-free, 8 x 1024-thread workgroups per CU",
            "unit": "G lane-ops/s", "frac": round(ach / peak, 4)}


def kernel_hash():
    """Hash of the push kernel's sources without comments and blank space
    (a comment-only edit keeps the committed counter summaries valid)."""
    import re
    h = hashlib.sha256()
    for f in ("k_push.hip", "k_particle.h", "k_common.h", "pic_internal.h"):
        src = open(os.path.join(ROOT, "paper_1310_0930_amd", "csrc", f)).read()
        src = re.sub(r"//[^\n]*|/\*.*?\*/", "", src, flags=re.S)
        h.update("".join(src.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(workload, real):
    """HBM bytes per push/deposit launch from the committed rocprofv3 counter
    summary, or None when it is absent or the kernel changed since."""
    path = os.path.join(ROOT, "profiles", f"push_deposit_{workload}_{real}_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("traffic_bytes")


# gfx950: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz issue 39.3 T lane-instructions
# of VALU per second without packed FP32 (a wave64 instruction occupies a
# SIMD for 4 cycles); the LDS of each CU serves one access stream.
CUS, CLOCK_HZ = 256, 2.4e9
VALU_PEAK = CUS * 4 * 16 * CLOCK_HZ


def ceilings(workload, real, push_ms):
    """VALU issue and LDS activity of the push/deposit launch: instruction and
    cycle counts per launch from the committed rocprofv3 SQ counter summary
    (None when it is absent or the kernel changed since) over the launch's
    time measured in this run."""
    path = os.path.join(ROOT, "profiles", f"push_deposit_{workload}_{real}_sq.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_hash") != kernel_hash():
        return None
    t = push_ms * 1e-3
    valu = rec["valu_insts"] * 64 / t
    return {"valu_issue": {"achieved": round(valu / 1e12, 2), "peak": round(VALU_PEAK / 1e12, 2),
                           "unit": "T lane-instructions/s", "frac": round(valu / VALU_PEAK, 4),
                           "per_64_particles": round(rec["valu_insts"] / rec["batches"], 1)},
            "lds_active": {"frac": round(rec["lds_active_cycles"] / (CUS * CLOCK_HZ * t), 4),
                           "conflict_share": round(rec["lds_conflict_cycles"] / rec["lds_active_cycles"], 4),
                           "cycles_per_64_particles": round(rec["lds_active_cycles"] / rec["batches"], 1)},
            "source": rec["source"]}


_INPUTS = {}


def workload_inputs(w):
    """Seeded particles and fields of workload w (drawn once, kept for the
    FP32 and the FP64 run)."""
    if w.name not in _INPUTS:
        _INPUTS.clear()
        _INPUTS[w.name] = (I.make_plasma(w),) + tuple(I.laser_fields(w))
    return _INPUTS[w.name]


def sorts_in(warmup, steps, every):
    """Sorts inside the timed steps warmup .. warmup + steps - 1 (step k sorts
    first when k is a multiple of the interval)."""
    return sum(1 for k in range(warmup, warmup + steps) if k % every == 0)


def run_gpu(w, real_bytes, steps, warmup, log):
    import torch
    from paper_1310_0930_amd.pic import Simulation
    pl, E, B = workload_inputs(w)
    sim = Simulation.from_workload(w, real_bytes=real_bytes)
    sim.load(pl, E, B, with_id=False)
    del pl
    if w.ions is not None:  # mobile ions: a second species in the same fields
        sim.add_species(I.make_ions(w), w.ions.q_over_m, w.q_const_ions, with_id=False)
    everyone = [sim] + sim.species
    np_total = sum(s.np for s in everyone)
    torch.cuda.synchronize()
    log(f"loaded {w.name} np={np_total} ({len(everyone)} species) real={real_bytes}")

    def one_step(k, ev=None):
        if k % w.sort_every == 0:
            for s in everyone:
                s.sort()
        if ev is not None:
            ev[0].record()
        sim.push_deposit()
        for s in sim.species:
            s.push_deposit_add()
        if ev is not None:
            ev[1].record()
        sim.field_advance()
        if ev is not None:
            ev[2].record()

    for k in range(warmup):
        one_step(k)
    torch.cuda.synchronize()
    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for k in range(steps):
        one_step(warmup + k, evs[k])
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    push_ms = [a.elapsed_time(b) for a, b, _ in evs]
    fdtd_ms = [b.elapsed_time(c) for _, b, c in evs]
    flags, nslow, nreb = 0, 0, 0
    for s in everyone:
        f_, n_ = s.read_flags()
        flags |= f_
        nslow += n_
        nreb += s.read_push_counts()[0]
    diag = sim.diagnostics()
    # FP64 charge density of the resident particles: tiles of the last sort
    # (LDS) and one thread per particle (no bins)
    from paper_1310_0930_amd import pic as P
    rho = torch.zeros(sim.ncell, dtype=torch.float64, device=sim.device)
    rho_ms = {}
    for tag, ws in (("tiles", sim.ws.data_ptr()), ("per_particle", None)):
        P.pic_deposit_rho(sim.ctx, sim._parts, rho.data_ptr(), ws)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            P.pic_deposit_rho(sim.ctx, sim._parts, rho.data_ptr(), ws)
        e1.record()
        torch.cuda.synchronize()
        rho_ms[tag] = e0.elapsed_time(e1) / 3
    log(f"{w.name} real={real_bytes}: {total_ms / steps:.3f} ms/step, push {np.mean(push_ms):.3f} ms, "
        f"fdtd {np.mean(fdtd_ms):.3f} ms, rho {rho_ms['tiles']:.3f} ms (per particle "
        f"{rho_ms['per_particle']:.3f}), rebinned={nreb} slow={nslow} flags={flags}")
    return {
        "np": np_total, "ms_per_step": total_ms / steps, "wall_s": wall,
        "push_ms_mean": float(np.mean(push_ms)), "push_ms_median": float(np.median(push_ms)),
        "fdtd_ms_mean": float(np.mean(fdtd_ms)), "rho_ms": rho_ms,
        "slowpath": int(nslow), "rebinned": int(nreb), "flags": int(flags),
        "n_alive": int(diag.raw["n_alive"]),
    }


def run_window(w, real_bytes, shifts, log):
    """Moving-window shift on workload w's grid (x made open): ms per shift
    and HBM rate against the algorithmic bytes (E, B read and written, J
    zeroed, cells read and written, the front column's particles read and
    written).  The injected columns are uploaded before the timed region."""
    import ctypes as C
    import torch
    from paper_1310_0930_amd import pic as P
    wo = w.with_(bc=(I.OPEN,) + tuple(w.bc3[1:w.dims]))
    pl = I.make_plasma(wo)
    E, B = I.laser_fields(wo)
    pc = wo.particle_cells()
    ncol = pc[1] * (pc[2] if wo.dims == 3 else 1) * wo.ppc
    sim = P.Simulation.from_workload(wo, real_bytes=real_bytes)
    sim.load(pl, E, B, with_id=False, capacity=pl.np + (shifts + 2) * ncol)
    del pl
    keep, injs = [], []
    for k in range(shifts + 1):
        col = I.inject_column(wo, k + 1)
        off = torch.from_numpy(col.off).to(sim.device, sim.real)
        u = torch.from_numpy(col.u).to(sim.device, sim.real)
        q = None if col.q is None else torch.from_numpy(col.q).to(sim.device, sim.real)
        keep.append((off, u, q))
        injs.append(P.PicInject(col.np, wo.ppc, (C.c_void_p * 3)(*[off[d].data_ptr() for d in range(3)]),
                                (C.c_void_p * 3)(*[u[c].data_ptr() for c in range(3)]),
                                q.data_ptr() if q is not None else None))
    P.pic_window_shift(sim.ctx, sim._parts, sim.capacity, sim._fields, injs[0], sim.ws.data_ptr())
    torch.cuda.synchronize()
    np0 = sim._parts.np
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for k in range(1, shifts + 1):
        P.pic_window_shift(sim.ctx, sim._parts, sim.capacity, sim._fields, injs[k], sim.ws.data_ptr())
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / shifts
    np_mean = np0 + ncol * (shifts + 1) / 2
    R = real_bytes
    per_inject = 2 * R * (wo.dims + 3) + 4 + (2 * R if wo.ramp_cells > 0 else 0)
    alg = wo.ncell * R * (6 * 2 + 3) + 8 * np_mean + ncol * per_inject
    log(f"window shift {wo.name} real={R}: {ms:.4f} ms per shift, {alg / ms / 1e6:.1f} GB/s")
    return {"ms_per_shift": round(ms, 5), "alg_bytes_per_shift": int(alg),
            "roofline": {"bound": "hbm", "achieved": round(alg / ms / 1e6, 2), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)},
            "shifts_per_step": round(wo.dt / wo.dx3[0], 4)}


def run_adjoint(w, real_bytes, reps, log):
    """One step's push/deposit adjoint (pic_push_deposit_adjoint) on workload
    w after a sort: with the sort's workspace (LDS kernel per tile in 2D, per
    z slab of a tile in 3D, where the form fits) and with a workspace holding
    no tile bins (one thread per particle in global memory).  Random adjoint
    inputs; ms per call, mean of `reps` calls after one untimed call."""
    import torch
    from paper_1310_0930_amd import pic as P
    pl = I.make_plasma(w)
    E, B = I.laser_fields(w)
    sim = P.Simulation.from_workload(w, real_bytes=real_bytes)
    sim.load(pl, E, B, with_id=False)
    del pl
    sim.sort()
    g = torch.Generator(device=sim.device).manual_seed(1310)
    LJ = torch.randn(sim.J.shape, generator=g, device=sim.device, dtype=sim.real)
    LX = torch.randn(sim.off.shape, generator=g, device=sim.device, dtype=sim.real)
    LU = torch.randn(sim.u.shape, generator=g, device=sim.device, dtype=sim.real)
    LE, LB = torch.zeros_like(sim.E), torch.zeros_like(sim.B)
    lam_f = P.fields_struct(LE, LB, LJ)
    lam_p = P.particles_struct(sim.np, None, LX, LU)
    res = {}
    for tag, ws in (("lds", sim.ws), ("global", torch.zeros_like(sim.ws))):
        P.pic_push_deposit_adjoint(sim.ctx, sim._parts, sim._fields, lam_f, lam_p, ws.data_ptr(),
                                   sim.stream)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            P.pic_push_deposit_adjoint(sim.ctx, sim._parts, sim._fields, lam_f, lam_p,
                                       ws.data_ptr(), sim.stream)
        t1.record()
        torch.cuda.synchronize()
        res[tag] = t0.elapsed_time(t1) / reps
    log(f"adjoint {w.name} real={real_bytes}: {res['lds']:.3f} ms per step adjoint "
        f"(global-memory kernel {res['global']:.3f} ms)")
    return {"ms": round(res["lds"], 4), "pushes_per_s": sim.np / (res["lds"] * 1e-3),
            "global_memory_kernel_ms": round(res["global"], 4), "particles": sim.np}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, log, budget_s=12.0):
    """The FP64 oracle (as it stands) on the host cores: one push/deposit pass
    over a bounded prefix of the workload's particles plus one full-grid FDTD
    advance, scaled to pushes per second; once on one thread and once on
    every thread this process may use (the CPU share of one GPU: the
    affinity mask, capped by OMP_NUM_THREADS when that is set)."""
    import oracle as O
    visible = os.cpu_count() or 1
    allowed = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else visible
    threads = allowed
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = max(1, min(threads, int(os.environ["OMP_NUM_THREADS"])))
    pl, E, B = workload_inputs(w)
    c = O.Config(w.dims, w.n3, w.dx3, w.dt, w.order, w.bc3)
    X = pl.global_positions(w)
    u = pl.u.T.astype(np.float64)
    q = pl.charges()

    def timed(nthreads, budget):
        # grow the sample (a prefix of the workload's particles) until one
        # pass takes about the time budget; the threaded pass has a fixed
        # cost (a private current grid per thread, reduced at the end), so
        # the estimate is refined from each pass
        m = min(pl.np, 20000)
        while True:
            s = O.State(c, X[:m], u[:m], q[:m], E, B)
            t = time.perf_counter()
            s.push_deposit(nthreads=nthreads)
            el = time.perf_counter() - t
            if m >= pl.np or el >= 0.5 * budget:
                return m, el, s
            m = int(min(pl.np, max(2 * m, m * 0.8 * budget / max(el, 1e-9))))

    m1, t1, _ = timed(1, 0.35 * budget_s)
    m, t_push, s = timed(threads, 0.65 * budget_s)
    t = time.perf_counter()
    s.field_advance()
    t_fdtd = time.perf_counter() - t
    # one whole step of the full workload would take N*t_push/m + t_fdtd
    step_s = w.num_particles * t_push / m + t_fdtd
    log(f"cpu oracle ({cpu_model()}, {visible} visible / {allowed} allowed cpus): {m} pushes in "
        f"{t_push:.2f} s on {threads} threads, {m1} in {t1:.2f} s on 1 thread, fdtd {t_fdtd:.2f} s")
    return {"value": w.num_particles / step_s, "unit": "particle pushes/s", "cores": threads,
            "kind": "oracle",
            "sample": f"1 push/deposit pass over {m} particles of {w.name} on {threads} threads "
                      f"(and over {m1} on 1 thread) plus 1 full-grid FDTD advance, FP64; scaled to "
                      f"whole steps of {w.num_particles} particles",
            "push_only_value": m / t_push, "per_core_push_value": m1 / t1,
            "cpu_model": cpu_model(), "cpus_visible": visible, "cpus_allowed": allowed}


# ---------------------------------------------------------------- rocprofv3
# Summaries of the CSV files rocprofv3 writes for runs of this script
# (``--output-format csv``), for the text summaries kept under profiles/:
#
#   python bench.py summarize trace DIR            kernel times per workload
#   python bench.py summarize bytes FETCH_DIR WRITE_DIR LOG   HBM bytes per kernel
#   python bench.py summarize sq DIR LOG           SQ counters of the push/deposit kernel
#   python bench.py summarize probe DIR            LDS counters of the LDS probe kernels
#
# One run covers several workloads; a dispatch is attributed to the workload
# whose field-advance grid (k_half_b*) comes next for the kernels of a step's
# start (sort, push) and last before for every other kernel.  LOG is the run's
# output, whose last line is this script's JSON record (particle counts).
# ``bytes`` also writes profiles/push_deposit_<workload>_<f32|f64>_counters.json,
# which bench runs read for ``roofline.traffic`` while the push kernel's
# sources are unchanged.

_STEP_START = ("k_push", "k_sort", "k_pda", "k_adj_reset", "k_fill_int", "k_scan", "k_tile_starts")


def _rp_rows(d, suffix):
    import csv
    import glob
    f = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not f:
        raise SystemExit(f"no *{suffix} under {d}")
    return list(csv.DictReader(open(f[0])))


def _rp_short(name):
    n = name.replace("void ", "").replace("(anonymous namespace)::", "")
    if n.startswith("pic::"):
        return n.split("(")[0]
    if "at::native" in n:
        return "torch " + n.split("<")[0]
    return n.split("(")[0][:60]


def _rp_field_grids():
    """Grid size (threads) of the field-advance launch -> workload name."""
    out = {}
    for w in I.WORKLOADS.values():
        n = w.n3 if w.dims == 3 else (w.n3[0], w.n3[1], 1)
        ncell = n[0] * n[1] * n[2]
        col = w.dims == 3 and all(b == 0 for b in w.bc3) and n[2] % 4 == 0
        blocks = -(-(ncell // 4 if col else ncell) // 256)
        out.setdefault(str((blocks + 7) // 8 * 8 * 256), w.name)
    return out


def _rp_attribute(disp):
    """disp: [(dispatch id, kernel name, field grid or None)] in dispatch order."""
    grids = _rp_field_grids()
    nxt, last = {}, None
    for did, name, g in reversed(disp):
        if g is not None:
            last = g
        nxt[did] = last
    lab, prev = {}, None
    for did, name, g in disp:
        if g is not None:
            prev = g
        first = nxt[did] if any(t in name for t in _STEP_START) else prev
        pick = first if first is not None else (nxt[did] if prev is None else prev)
        lab[did] = grids.get(pick, f"grid {pick}")
    return lab


def _rp_field(r):
    return (r.get("Grid_Size") or r.get("Grid_Size_X")) if "k_half_b" in r["Kernel_Name"] else None


def _rp_counters(d):
    by, info = {}, {}
    for r in _rp_rows(d, "counter_collection.csv"):
        did = int(r["Dispatch_Id"])
        c = by.setdefault(did, {})
        c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        info[did] = r
    order = sorted(by)
    lab = _rp_attribute([(i, info[i]["Kernel_Name"], _rp_field(info[i])) for i in order])
    return [(i, info[i]["Kernel_Name"], by[i], lab[i]) for i in order]


def _rp_record(log):
    for line in reversed(open(log).read().splitlines()):
        if line.startswith("{"):
            return json.loads(line)
    raise SystemExit(f"no JSON record in {log}")


def _rp_particles(rec):
    out = {rec["config"]["workload"]: rec["config"]["particles"]}
    if "one_gpu_share" in rec:
        out[rec["one_gpu_share"]["workload"]] = rec["one_gpu_share"]["particles"]
    return out


def summarize_trace(d):
    rows = _rp_rows(d, "kernel_trace.csv")
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    lab = _rp_attribute([(int(r["Dispatch_Id"]), r["Kernel_Name"], _rp_field(r)) for r in rows])
    agg = {}
    for r in rows:
        key = (lab[int(r["Dispatch_Id"])], _rp_short(r["Kernel_Name"]))
        agg.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    for w in sorted({k[0] for k in agg}):
        items = sorted(((sum(v), n, v) for (ww, n), v in agg.items() if ww == w), reverse=True)
        tot = sum(t for t, _, _ in items)
        print(f"## {w}: {tot / 1e3:.3f} ms of kernel time")
        print(f"  {'kernel':56s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}")
        for t, n, v in items:
            if t >= 5e-4 * tot:
                print(f"  {n:56s} {len(v):6d} {t / len(v):10.2f} {t / 1e3:10.3f} {100 * t / tot:6.2f}")


def summarize_bytes(dfetch, dwrite, log):
    rec = _rp_record(log)
    nps = _rp_particles(rec)
    per = {}
    for tag, d in (("FETCH_SIZE", dfetch), ("WRITE_SIZE", dwrite)):
        disp = _rp_counters(d)
        # --calibrate-copy: the run's first three copies, 1 GiB each
        cal = [c[tag] for _, n, c, _ in disp if "copyBuffer" in n][:3]
        scale = (1 << 20) / (sum(cal) / len(cal))
        print(f"# {tag}: the three 1 GiB calibration copies read {', '.join('%.1f' % x for x in cal)} KiB "
              f"-> scale {scale:.4f}")
        for _, n, c, w in disp:
            if n.startswith("void pic::") or n.startswith("pic::"):
                per.setdefault((w, _rp_short(n)), {}).setdefault(tag, []).append(c[tag])
        per[("scale", tag)] = scale
    fs, ws_ = per.pop(("scale", "FETCH_SIZE")), per.pop(("scale", "WRITE_SIZE"))
    print(f"# traffic = FETCH_SIZE x {fs:.4f} + WRITE_SIZE x {ws_:.4f} (KiB per dispatch, mean)")
    khash = kernel_hash()
    for (w, n), v in sorted(per.items()):
        f = float(np.mean(v.get("FETCH_SIZE", [0.0])))
        wr = float(np.mean(v.get("WRITE_SIZE", [0.0])))
        t = (f * fs + wr * ws_) * 1024
        line = (f"  {w:26s} {n:44s} FETCH {f:12.1f} WRITE {wr:12.1f} KiB "
                f"({len(v.get('FETCH_SIZE', []))} dispatches)  {t / 1e6:10.1f} MB")
        if "k_push_tile" in n and ", true>" not in n and w in nps:  # the sorted pass
            rb = 8 if "double" in n else 4
            ab = algorithmic_bytes(I.WORKLOADS[w], nps[w], rb)
            line += f"  algorithmic {ab / 1e6:.1f} MB, ratio {t / ab:.3f}"
            real = "f64" if rb == 8 else "f32"
            json.dump({"kernel": "k_push_tile", "workload": w, "real": real, "kernel_hash": khash,
                       "fetch_kib": f, "write_kib": wr, "fetch_scale": fs, "write_scale": ws_,
                       "traffic_bytes": int(t), "algorithmic_bytes": ab,
                       "source": "profiles/hbm_bytes_" + "_".join(sorted(nps)) + ".txt"},
                      open(os.path.join(ROOT, "profiles", f"push_deposit_{w}_{real}_counters.json"), "w"),
                      indent=1)
        print(line)


def summarize_sq(d, log):
    nps = _rp_particles(_rp_record(log))
    agg = {}
    for _, n, c, w in _rp_counters(d):
        if "k_push_tile" in n and ", true>" not in n:  # the sorted pass
            a = agg.setdefault((w, _rp_short(n)), {})
            for k, v in c.items():
                a.setdefault(k, []).append(v)
    for (w, n), a in sorted(agg.items()):
        nb = nps[w] / 64
        print(f"  {w} {n}: per dispatch, and per batch of 64 particles ({nb:.0f} batches)")
        for k, v in sorted(a.items()):
            print(f"    {k:22s} {np.mean(v):16.0f} {np.mean(v) / nb:10.1f}")
        if a.get("SQ_LDS_IDX_ACTIVE"):
            print(f"    bank-conflict cycles / LDS-active cycles {sum(a['SQ_LDS_BANK_CONFLICT']) / sum(a['SQ_LDS_IDX_ACTIVE']):.3f}")
        if w in nps and all(a.get(k) for k in ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_LDS_IDX_ACTIVE")):
            real = "f64" if "double" in n else "f32"
            json.dump({"kernel": "k_push_tile", "workload": w, "real": real, "kernel_hash": kernel_hash(),
                       "batches": int(nb), "valu_insts": float(np.mean(a["SQ_INSTS_VALU"])),
                       "lds_insts": float(np.mean(a["SQ_INSTS_LDS"])),
                       "lds_active_cycles": float(np.mean(a["SQ_LDS_IDX_ACTIVE"])),
                       "lds_conflict_cycles": float(np.mean(a.get("SQ_LDS_BANK_CONFLICT", [0.0]))),
                       "source": "profiles/push_deposit_sq_counters_" + "_".join(sorted(nps)) + ".txt"},
                      open(os.path.join(ROOT, "profiles", f"push_deposit_{w}_{real}_sq.json"), "w"), indent=1)


def summarize_probe(d, strides=(1, 2, 4, 8, 16, 32, 64, 128), reps=3):
    """The --lds-probe run: the first `reps` dispatches are ds_add_u64 at
    stride 1 (the push's LDS peak), then every op of PROBE_OPS at every
    stride, `reps` each, in that order."""
    disp = [x for x in _rp_counters(d) if "k_lds_rate" in x[1]]
    names = {v: k for k, v in PROBE_OPS.items()}
    body = disp[reps:]
    print(f"  {'op':22s} {'stride':>6s} {'LDS instr/op':>12s} {'active cyc/instr':>16s} "
          f"{'conflict cyc/instr':>18s} {'VALU/op':>8s}")
    for i, op in enumerate(sorted(names)):
        for j, st in enumerate(strides):
            grp = body[(i * len(strides) + j) * reps:(i * len(strides) + j + 1) * reps]
            c = grp[0][2]
            ops = c["SQ_WAVES"] * 2048  # iterations per wavefront of the probe (iters=2048)
            print(f"  {names[op]:22s} {st:6d} {c['SQ_INSTS_LDS'] / ops:12.3f} "
                  f"{c['SQ_LDS_IDX_ACTIVE'] / c['SQ_INSTS_LDS']:16.2f} "
                  f"{c['SQ_LDS_BANK_CONFLICT'] / c['SQ_INSTS_LDS']:18.2f} {c['SQ_INSTS_VALU'] / ops:8.3f}")


def summarize(argv):
    kind, rest = argv[0], argv[1:]
    {"trace": summarize_trace, "bytes": summarize_bytes, "sq": summarize_sq,
     "probe": summarize_probe}[kind](*rest)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "summarize":
        summarize(sys.argv[2:])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="w3d_128_quadratic", choices=sorted(I.WORKLOADS))
    ap.add_argument("--sort-every", type=int, default=0, metavar="N",
                    help="sort every N steps instead of the workload's interval")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--window", type=int, default=0, metavar="K",
                    help="also time K moving-window shifts on the workload's grid (x made open)")
    ap.add_argument("--adjoint", type=int, default=0, metavar="K",
                    help="also time K calls of one step's push/deposit adjoint after a sort")
    ap.add_argument("--share-workload", default="w3d_512_quadratic_laser",
                    choices=sorted(I.WORKLOADS) + ["none"],
                    help="second record: the one-GPU share of an LWFA run (FP32 and FP64)")
    ap.add_argument("--share-steps", type=int, default=0,
                    help="timed steps of the share (default: one sort interval of its workload, so "
                         "that the whole-step rate carries exactly one sort)")
    ap.add_argument("--lds-probe", action="store_true",
                    help="also report the LDS probe's rates for every access kind and lane stride")
    ap.add_argument("--lds-replay", action="store_true",
                    help="also replay the push kernel's LDS access patterns for the sorted lane layout")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy (for scaling the "
                         "rocprofv3 FETCH_SIZE/WRITE_SIZE counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus {a.gpus}",
              file=sys.stderr)
        sys.exit(2)

    def log(msg):
        if not a.quiet:
            print(f"[bench] {msg}", file=sys.stderr, flush=True)

    w = I.WORKLOADS[a.workload]
    if a.sort_every > 0:
        w = w.with_(sort_every=a.sort_every)
    if a.calibrate_copy:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {src.numel() * 4} bytes")
        del src, dst
    r32 = run_gpu(w, 4, a.steps, a.warmup, log)
    r64 = None if a.no_fp64 else run_gpu(w, 8, a.steps, a.warmup, log)

    def roof(r, rb, real):
        ab = algorithmic_bytes(w, r["np"], rb)
        ach = ab / (r["push_ms_mean"] * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile(w.name, real),
                "kernel": "k_push_tile (timed with its J-zeroing prologue, the re-binned pass where it is on, and the deferred-list kernel)",
                "alg_bytes_per_launch": ab,
                "avg_launch_ms": round(r["push_ms_mean"], 5)}

    out = {
        "metric": METRIC,
        "value": r32["np"] / (r32["ms_per_step"] * 1e-3),
        "unit": "particle pushes/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(r32["ms_per_step"], 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "dims": w.dims, "grid": list(w.n3), "dx": list(w.dx3),
                   "ppc": w.ppc, "particles": r32["np"], "order": w.order, "u_th": w.u_th,
                   "species": 1 if w.ions is None else 2,
                   "dt": w.dt, "sort_every": w.sort_every,
                   "sorts_timed": sorts_in(a.warmup, a.steps, w.sort_every), "boundaries": list(w.bc3),
                   "parallelism": "single GPU"},
        "push_deposit_pushes_per_s": r32["np"] / (r32["push_ms_mean"] * 1e-3),
        "field_advance_ms": round(r32["fdtd_ms_mean"], 5),
        "rho_deposit_fp64_ms": {k: round(v, 4) for k, v in r32["rho_ms"].items()},
        "roofline": roof(r32, 4, "f32"),
        "lds_atomics": lds_atomics(w, r32["np"], r32["push_ms_mean"], 4),
        "ceilings": ceilings(w.name, "f32", r32["push_ms_mean"]),
        "rebinned_pushes": r32["rebinned"], "slowpath_pushes": r32["slowpath"],
        "device_flags": r32["flags"],
    }
    if r64:
        out["fp64"] = {"value": r64["np"] / (r64["ms_per_step"] * 1e-3),
                       "ms_per_step": round(r64["ms_per_step"], 5),
                       "push_deposit_pushes_per_s": r64["np"] / (r64["push_ms_mean"] * 1e-3),
                       "roofline": roof(r64, 8, "f64"),
                       "lds_atomics": lds_atomics(w, r64["np"], r64["push_ms_mean"], 8),
                       "ceilings": ceilings(w.name, "f64", r64["push_ms_mean"]),
                       "device_flags": r64["flags"]}
    if a.share_workload != "none" and a.share_workload != w.name:
        ws_ = I.WORKLOADS[a.share_workload]
        k5 = a.share_steps if a.share_steps > 0 else ws_.sort_every
        s32 = run_gpu(ws_, 4, k5, 3, log)
        s64 = None if a.no_fp64 else run_gpu(ws_, 8, k5, 3, log)
        rec = {"workload": ws_.name, "grid": list(ws_.n3), "dx": list(ws_.dx3), "ppc": ws_.ppc,
               "order": ws_.order, "particles": s32["np"], "dt": ws_.dt,
               "sort_every": ws_.sort_every, "steps": k5, "warmup": 3,
               "sorts_timed": sorts_in(3, k5, ws_.sort_every)}

        def share(r, rb, real):
            ab = algorithmic_bytes(ws_, r["np"], rb)
            return {"value": r["np"] / (r["ms_per_step"] * 1e-3),
                    "ms_per_step": round(r["ms_per_step"], 5),
                    "push_deposit_pushes_per_s": r["np"] / (r["push_ms_mean"] * 1e-3),
                    "push_ms": round(r["push_ms_mean"], 5),
                    "field_advance_ms": round(r["fdtd_ms_mean"], 5),
                    "rho_deposit_fp64_ms": {k: round(v, 4) for k, v in r["rho_ms"].items()},
                    "roofline": {"bound": "hbm", "achieved": round(ab / (r["push_ms_mean"] * 1e-3) / 1e9, 2),
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": round(ab / (r["push_ms_mean"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "traffic": traffic_from_profile(ws_.name, real),
                                 "alg_bytes_per_launch": ab},
                    "ceilings": ceilings(ws_.name, real, r["push_ms_mean"]),
                    "rebinned_pushes": r["rebinned"], "slowpath_pushes": r["slowpath"],
                    "device_flags": r["flags"]}
        rec["f32"] = share(s32, 4, "f32")
        if s64:
            rec["f64"] = share(s64, 8, "f64")
        out["one_gpu_share"] = rec
    if a.lds_probe:
        out["lds_probe"] = {"unit": "G lane-ops/s", "rates_by_stride": lds_probe_table()}
    if a.lds_replay:
        out["lds_replay"] = {"f32": lds_replay(w, 4), "f64": None if a.no_fp64 else lds_replay(w, 8)}
    if a.window > 0:
        out["window_shift"] = {"f32": run_window(w, 4, a.window, log)}
        if not a.no_fp64:
            out["window_shift"]["f64"] = run_window(w, 8, a.window, log)
    if a.adjoint > 0:
        out["step_adjoint"] = {"f32": run_adjoint(w, 4, a.adjoint, log)}
        if not a.no_fp64:
            out["step_adjoint"]["f64"] = run_adjoint(w, 8, a.adjoint, log)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, log)
    t3 = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_table3.json")))
    out["paper_context"] = {
        "source": t3["citation"],
        "pushes_per_s_cpu_by_order": {str(r[0]): r[4] * 1e6 for r in t3["rows"]}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
