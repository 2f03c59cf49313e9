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
    h = hashlib.sha256()
    for f in ("k_push.hip", "k_particle.h", "k_common.h", "pic_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1310_0930_amd", "csrc", f), "rb").read())
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


_INPUTS = {}


def workload_inputs(w):
    """Seeded particles and fields of workload w (drawn once, kept for the
    FP32 and the FP64 run)."""
    if w.name not in _INPUTS:
        _INPUTS.clear()
        _INPUTS[w.name] = (I.make_plasma(w),) + tuple(I.laser_fields(w))
    return _INPUTS[w.name]


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

    for k in range(warmup):
        one_step(k)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
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
    push_ms = [a.elapsed_time(b) for a, b in evs]
    flags, nslow = 0, 0
    for s in everyone:
        f_, n_ = s.read_flags()
        flags |= f_
        nslow += n_
    diag = sim.diagnostics()
    log(f"{w.name} real={real_bytes}: {total_ms / steps:.3f} ms/step, push {np.mean(push_ms):.3f} ms, "
        f"slow={nslow} flags={flags}")
    return {
        "np": np_total, "ms_per_step": total_ms / steps, "wall_s": wall,
        "push_ms_mean": float(np.mean(push_ms)), "push_ms_median": float(np.median(push_ms)),
        "slowpath": int(nslow), "flags": int(flags), "n_alive": int(diag.raw["n_alive"]),
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


def main():
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
    ap.add_argument("--share-steps", type=int, default=10)
    ap.add_argument("--lds-probe", action="store_true",
                    help="also report the LDS probe's rates for every access kind and lane stride")
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
                "kernel": "k_push_tile (timed with its J-zeroing prologue and deferred-list kernel)",
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
                   "dt": w.dt, "sort_every": w.sort_every, "boundaries": list(w.bc3),
                   "parallelism": "single GPU"},
        "push_deposit_pushes_per_s": r32["np"] / (r32["push_ms_mean"] * 1e-3),
        "roofline": roof(r32, 4, "f32"),
        "lds_atomics": lds_atomics(w, r32["np"], r32["push_ms_mean"], 4),
        "slowpath_pushes": r32["slowpath"], "device_flags": r32["flags"],
    }
    if r64:
        out["fp64"] = {"value": r64["np"] / (r64["ms_per_step"] * 1e-3),
                       "ms_per_step": round(r64["ms_per_step"], 5),
                       "push_deposit_pushes_per_s": r64["np"] / (r64["push_ms_mean"] * 1e-3),
                       "roofline": roof(r64, 8, "f64"),
                       "lds_atomics": lds_atomics(w, r64["np"], r64["push_ms_mean"], 8),
                       "device_flags": r64["flags"]}
    if a.share_workload != "none" and a.share_workload != w.name:
        ws_ = I.WORKLOADS[a.share_workload]
        k5 = max(1, a.share_steps)
        s32 = run_gpu(ws_, 4, k5, 3, log)
        s64 = None if a.no_fp64 else run_gpu(ws_, 8, k5, 3, log)
        rec = {"workload": ws_.name, "grid": list(ws_.n3), "dx": list(ws_.dx3), "ppc": ws_.ppc,
               "order": ws_.order, "particles": s32["np"], "dt": ws_.dt,
               "sort_every": ws_.sort_every, "steps": k5, "warmup": 3}

        def share(r, rb):
            ab = algorithmic_bytes(ws_, r["np"], rb)
            return {"value": r["np"] / (r["ms_per_step"] * 1e-3),
                    "ms_per_step": round(r["ms_per_step"], 5),
                    "push_deposit_pushes_per_s": r["np"] / (r["push_ms_mean"] * 1e-3),
                    "push_ms": round(r["push_ms_mean"], 5),
                    "roofline": {"bound": "hbm", "achieved": round(ab / (r["push_ms_mean"] * 1e-3) / 1e9, 2),
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": round(ab / (r["push_ms_mean"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "alg_bytes_per_launch": ab},
                    "slowpath_pushes": r["slowpath"], "device_flags": r["flags"]}
        rec["f32"] = share(s32, 4)
        if s64:
            rec["f64"] = share(s64, 8)
        out["one_gpu_share"] = rec
    if a.lds_probe:
        out["lds_probe"] = {"unit": "G lane-ops/s", "rates_by_stride": lds_probe_table()}
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
