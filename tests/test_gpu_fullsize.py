"""Full-size workloads on the GPU, in the launch configuration bench.py uses.

* 512x256 2D3V, 16 ppc, quadratic, ramp + a0=4 laser, open y (2.09M
  particles): 12 steps within 1e-12 (FP64), every one of the 50 steps
  against the oracle beside the per-step conditioning floor (FP64, FP32),
  and the FP32 adjoint gradient of the wake-window energy against FP64
  central differences.
* 256x128x128 cubic, ramp + laser, open y,z (33M particles): 20 whole steps
  (five re-sorts) on every particle and field sample; the same recipe on a
  256x24x24 grid for all 200 steps against the conditioning floor.
* 512x256x256 one-GPU share, quadratic, laser (268M particles): one push on
  sampled particles the oracle recomputes one by one, and FP64 continuity and
  Gauss residuals of the whole state; one whole step (sort, push/deposit,
  field advance) on every particle and field sample, and the FP64
  diagnostics (charge density, Gauss residual, field and kinetic energy)
  against the oracle's on the same state.
"""
import numpy as np
import pytest

import oracle as O
from paper_1310_0930_amd import inputs as I

from _parity import TOL, compare, gpu_sim, inputs_for, oracle_state, oracle_threads, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _check(err, rb, field_tol):
    assert err["alive_mismatch"] == 0, err
    assert err["pos"] <= TOL[rb], err
    assert err["u"] <= TOL[rb], err
    for f in ("E", "B", "J"):
        assert err[f] <= field_tol, (f, err)


def test_w2d_512_twelve_steps_fp64():
    w = I.WORKLOADS["w2d_512_quadratic_laser"].with_(steps=12)
    pl, E, B = inputs_for(w)
    say("case", w.name, "np", pl.np, "steps", w.steps, "fp64")
    sim = gpu_sim(w, 8, pl, E, B)
    sim.step(w.steps)
    torch.cuda.synchronize()
    ref = oracle_state(w, pl, E, B)
    ref.step(w.steps, nthreads=oracle_threads())
    err = compare(w, sim, ref)
    say(w.name, "fp64 12 steps", err)
    _check(err, 8, 1e-10)


def _perturb(st, rb, rng):
    """One storage rounding's worth of noise on an oracle state: +-1 ulp of
    each stored value in FP64, +-2^-24 (relative; absolute for the in-cell
    offsets) in FP32."""
    D = st.cfg.dims
    if rb == 8:
        st.X[:, :D] += rng.uniform(-1, 1, size=(st.np, D)) * np.spacing(st.X[:, :D])
        for a in (st.u, st.E, st.B):
            a += rng.uniform(-1, 1, size=a.shape) * np.spacing(a)
    else:
        ulp = 2.0 ** -24
        st.X[:, :D] += rng.uniform(-1, 1, size=(st.np, D)) * ulp
        for a in (st.u, st.E, st.B):
            a *= 1 + rng.uniform(-1, 1, size=a.shape) * ulp


def _floor(ref, pert):
    both = (ref.alive > 0) & (pert.alive > 0)
    D = ref.cfg.dims
    rms = np.sqrt(np.mean(np.sum(ref.u ** 2, axis=1)))
    return (float(np.abs(pert.X - ref.X)[both][:, :D].max()),
            float(np.abs(pert.u - ref.u)[both].max() / rms),
            int(np.sum(ref.alive != pert.alive)))


@pytest.mark.parametrize("rb", [8, 4])
def test_w2d_512_error_growth_per_step(rb):
    """All 50 steps of the 512x256 laser workload, compared with the oracle
    after every step beside the conditioning floor: an oracle run whose
    stored state gets one storage rounding's worth of noise after every step
    (the a0 = 4 pulse drives gamma ~ 20 and the dynamics amplify any
    difference about 1e3-fold over the run).  At every step the GPU is within
    max(bar, 3 x floor), bar = 1e-12 (FP64) or 1e-5 (FP32)."""
    w = I.WORKLOADS["w2d_512_quadratic_laser"]
    pl, E, B = inputs_for(w)
    sim = gpu_sim(w, rb, pl, E, B)
    ref = oracle_state(w, pl, E, B)
    pert = oracle_state(w, pl, E, B)
    rng = np.random.default_rng(1 if rb == 8 else 0)
    say("case", w.name, "np", pl.np, "real", rb, "per-step error and floor")
    say(" step   pos        floor_pos  u          floor_u    alive(gpu/floor)")
    for n in range(1, w.steps + 1):
        sim.step(1)
        ref.step(1, nthreads=oracle_threads())
        pert.step(1, nthreads=oracle_threads())
        _perturb(pert, rb, rng)
        torch.cuda.synchronize()
        err = compare(w, sim, ref)
        fp, fu, fa = _floor(ref, pert)
        say(" %4d  %.3e  %.3e  %.3e  %.3e  %d/%d" % (n, err["pos"], fp, err["u"], fu,
                                                       err["alive_mismatch"], fa))
        assert err["pos"] <= max(TOL[rb], 3 * fp), (n, err, fp)
        assert err["u"] <= max(TOL[rb], 3 * fu), (n, err, fu)
        assert err["alive_mismatch"] <= (0 if rb == 8 else max(2, 3 * fa)), (n, err, fa)
        if rb == 8:
            for f in ("E", "B", "J"):
                assert err[f] <= 1e-10, (n, f, err)


def test_w2d_512_adjoint_fp32_vs_central_differences():
    """Gradient of L = 1/2 sum_window E_x^2 dV after 50 steps (checkpoint
    every 10) with respect to a0 and to the initial momenta along a
    Rademacher direction: FP32 adjoint vs FP64 central differences."""
    import time
    from paper_1310_0930_amd.adjoint import PicRollout, Runner, window_energy
    w = I.WORKLOADS["w2d_512_quadratic_laser"]
    pl, E1, B1 = inputs_for(w)
    a0v = w.laser.a0
    E1, B1 = E1 / a0v, B1 / a0v
    r32 = Runner(w, real_bytes=4, checkpoint_every=10)
    r32.set_inputs(pl, E1, B1)
    a0 = torch.tensor(a0v, dtype=torch.float64, device="cuda", requires_grad=True)
    u0 = torch.from_numpy(pl.u).to("cuda", torch.float32).requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E, _ = PicRollout.apply(a0, u0, r32)
    L, win = window_energy(w, E)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    say("adjoint 512x256: forward %.3f s, backward %.3f s, window" % (t1 - t0, t2 - t1), win)
    r64 = Runner(w, real_bytes=8, checkpoint_every=10)
    r64.set_inputs(pl, E1, B1)
    u_base = torch.from_numpy(pl.u).to("cuda", torch.float64)
    rng = np.random.default_rng(4)
    v = torch.from_numpy(rng.choice([-1.0, 1.0], size=(3, pl.np))).to("cuda", torch.float64)

    def loss(a, u):
        with torch.no_grad():
            E, _ = r64.forward(torch.tensor(a, dtype=torch.float64, device="cuda"), u)
            return float(window_energy(w, E)[0])

    h = 1e-5
    fd_a0 = (loss(a0v + h, u_base) - loss(a0v - h, u_base)) / (2 * h)
    fd_v = (loss(a0v, u_base + h * v) - loss(a0v, u_base - h * v)) / (2 * h)
    g_v = float((u0.grad.double() * v).sum())
    say("adjoint 512x256 grad a0", float(a0.grad), fd_a0, "v", g_v, fd_v)
    assert abs(float(a0.grad) - fd_a0) <= 1e-3 * abs(fd_a0)
    assert abs(g_v - fd_v) <= 1e-3 * max(abs(fd_v), 1e-3 * abs(fd_a0))


_W3D_256_REF = {}


def _w3d_256_reference(w, pl, E, B, checkpoints):
    """Oracle states of the 256x128x128 workload at the given steps, and the
    FP32 conditioning floor there (a second oracle run with one FP32 storage
    rounding's worth of noise after every step); one run each, shared by the
    FP64 and FP32 cases."""
    key = (w.name, w.n3, tuple(checkpoints))
    if key not in _W3D_256_REF:
        _W3D_256_REF.clear()
        ref = oracle_state(w, pl, E, B)
        pert = oracle_state(w, pl, E, B)
        rng = np.random.default_rng(5)
        out, floors, done = {}, {}, 0
        for n in checkpoints:
            ref.step(n - done, nthreads=oracle_threads())
            for _ in range(n - done):
                pert.step(1, nthreads=oracle_threads())
                _perturb(pert, 4, rng)
            done = n
            out[n] = ref.copy()
            out[n].alive = ref.alive.copy()
            floors[n] = _floor(ref, pert)
            say("oracle step", n, "fp32 floor", floors[n])
        _W3D_256_REF[key] = (out, floors)
    return _W3D_256_REF[key]


@pytest.mark.parametrize("rb", [8, 4])
def test_w3d_256_cubic_twenty_steps(rb):
    """256x128x128, cubic, ramp + a0 = 4 laser, open y and z (33.5M
    particles), sorted every 4 steps: 20 steps (five re-sorts) on every
    particle and field sample, checked at each re-sort.  FP64 within 1e-12
    at every check; FP32 within 1e-5 over the first 12 steps and within
    max(1e-5, 3 x its conditioning floor) after that (the a0 = 4 pulse
    amplifies storage rounding as in the 512x256 case)."""
    w = I.WORKLOADS["w3d_256_cubic_laser"].with_(sort_every=4)
    pl, E, B = inputs_for(w)
    checks = list(range(4, 21, 4))
    refs, floors = _w3d_256_reference(w, pl, E, B, checks)
    say("case", w.name, "np", pl.np, "real", rb, "sort every", w.sort_every)
    sim = gpu_sim(w, rb, pl, E, B)
    done = 0
    for n in checks:
        sim.step(n - done)
        done = n
        torch.cuda.synchronize()
        err = compare(w, sim, refs[n])
        say(w.name, rb, "step", n, err, "fp32 floor", floors[n])
        if rb == 8 or n <= 12:
            _check(err, rb, 1e-10 if rb == 8 else 1e-4)
        else:
            fp, fu, fa = floors[n]
            assert err["alive_mismatch"] <= max(2, 3 * fa), (n, err, fa)
            assert err["pos"] <= max(TOL[4], 3 * fp), (n, err, fp)
            assert err["u"] <= max(TOL[4], 3 * fu), (n, err, fu)
            for f in ("E", "B", "J"):
                assert err[f] <= 1e-4, (n, f, err)


def test_w3d_256_cubic_narrow_two_hundred_steps():
    """The same recipe (cubic, ramp, a0 = 4 laser, open y and z, sorted every
    4 steps) on a 256x24x24 grid (1.2M particles) for all 200 steps, FP64
    and FP32 against the oracle at every 40th step, within max(bar, 3 x the
    conditioning floor of each precision)."""
    w = I.WORKLOADS["w3d_256_cubic_laser"].with_(n=(256, 24, 24), seed=I.SEED_BASE + 90,
                                                  sort_every=4)
    pl, E, B = inputs_for(w)
    say("case", w.name, w.n3, "np", pl.np, "steps", w.steps)
    sims = {rb: gpu_sim(w, rb, pl, E, B) for rb in (8, 4)}
    ref = oracle_state(w, pl, E, B)
    perts = {rb: oracle_state(w, pl, E, B) for rb in (8, 4)}
    rngs = {8: np.random.default_rng(2), 4: np.random.default_rng(3)}
    for n in range(1, w.steps + 1):
        ref.step(1, nthreads=oracle_threads())
        for rb in (8, 4):
            perts[rb].step(1, nthreads=oracle_threads())
            _perturb(perts[rb], rb, rngs[rb])
        if n % 40:
            continue
        for rb in (8, 4):
            sims[rb].step(40)
            torch.cuda.synchronize()
            err = compare(w, sims[rb], ref)
            fp, fu, fa = _floor(ref, perts[rb])
            say("narrow", rb, "step", n, err, "floor", fp, fu, fa)
            assert err["pos"] <= max(TOL[rb], 3 * fp), (n, rb, err, fp)
            assert err["u"] <= max(TOL[rb], 3 * fu), (n, rb, err, fu)
            assert err["alive_mismatch"] <= (0 if rb == 8 else max(2, 3 * fa)), (n, rb, err, fa)


def test_w3d_512_sampled_push_and_conservation():
    """268M particles: after one push, 200k sampled particles equal the
    oracle's push of the same particles (FP32 bar), and the FP64 continuity
    residual of the whole stored state is within 1e-6 (L2)."""
    w = I.WORKLOADS["w3d_512_quadratic_laser"]
    pl = I.make_plasma(w)
    E, B = I.laser_fields(w)
    say("case", w.name, "np", pl.np)
    sim = gpu_sim(w, 4, pl, E, B)
    rng = np.random.default_rng(12)
    sample = np.sort(rng.choice(pl.np, size=200_000, replace=False))
    Xs = I.Plasma(pl.cell[sample], pl.off[:, sample], pl.u[:, sample], None, pl.q_const)
    d0 = sim.diagnostics(want_gauss=True)
    sim.sort()
    sim.push_deposit()
    d1 = sim.diagnostics(rho_prev=d0.rho)
    say("continuity", d1.raw["cont_rel_l2"], d1.raw["cont_rel_inf"], "flags", d1.raw["flags"])
    assert d1.raw["cont_rel_l2"] <= 1e-6
    assert d1.raw["flags"] == 0
    cell = sim.cell.cpu().numpy()
    ids = sim.id.cpu().numpy()
    pos = np.empty(pl.np, dtype=np.int64)
    pos[ids] = np.arange(pl.np)
    k = pos[sample]
    off = sim.off[:, torch.from_numpy(k).cuda()].double().cpu().numpy()
    u = sim.u[:, torch.from_numpy(k).cuda()].double().cpu().numpy()
    n0, n1, _ = w.n3
    c = cell[k].astype(np.int64)
    Xg = np.stack([c % n0 + off[0], (c // n0) % n1 + off[1], c // (n0 * n1) + off[2]], axis=1)
    del sim
    torch.cuda.empty_cache()
    ref = O.State(O.Config(w.dims, w.n3, w.dx3, w.dt, w.order, w.bc3), Xs.global_positions(w),
                  Xs.u.T.astype(np.float64), Xs.charges(), E, B)
    ref.push_deposit(nthreads=oracle_threads())
    dX = Xg - ref.X
    n = np.array(w.n3, dtype=float)
    dX -= n * np.round(dX / n)
    rms = np.sqrt(np.mean(np.sum(ref.u ** 2, axis=1)))
    e_pos = np.abs(dX).max()
    e_u = np.abs(u.T - ref.u).max() / rms
    say("sampled push", e_pos, e_u)
    assert e_pos <= TOL[4] and e_u <= TOL[4]


def test_w3d_512_whole_step_and_diagnostics():
    """268M particles, FP32 (the workload's form): one whole step through
    pic_step (sort, push/deposit, field advance) against the oracle's step on
    every particle and field sample.  Then the FP64 diagnostics of the GPU's
    state (pic_diagnostics: charge density, Gauss residual against the
    initial one, continuity, field and kinetic energy) against the oracle's
    charge density, divergence and energies computed from the same state."""
    w = I.WORKLOADS["w3d_512_quadratic_laser"]
    pl, E, B = inputs_for(w)
    say("case", w.name, "np", pl.np, "whole step + diagnostics")
    sim = gpu_sim(w, 4, pl, E, B)
    d0 = sim.diagnostics(want_gauss=True)
    g0 = d0.raw["gauss_field"]
    sim.step(1)
    d1 = sim.diagnostics(rho_prev=d0.rho, gauss_ref=g0)
    torch.cuda.synchronize()
    st = sim.download()
    rho1 = d1.rho.cpu().numpy()
    g0 = g0.cpu().numpy()
    del sim, d0, d1.raw["gauss_field"]
    torch.cuda.empty_cache()
    say("gpu diagnostics", {k: v for k, v in d1.raw.items() if k != "gauss_field"})
    # the oracle's step
    ref = oracle_state(w, pl, E, B)
    ref.step(1, nthreads=oracle_threads())
    from paper_1310_0930_amd.pic import Simulation
    view = Simulation.__new__(Simulation)
    view.n, view.dims, view.np = w.n3, w.dims, pl.np
    err = compare(w, view, ref, st)
    say("whole step", err)
    _check(err, 4, 1e-4)
    del ref
    # the oracle's diagnostics of the GPU's state
    Xg, alive = view.positions(st)
    cfg = O.Config(w.dims, w.n3, w.dx3, w.dt, w.order, w.bc3)
    q = pl.charges()[st["id"]]
    gs = O.State(cfg, Xg, st["u"].T, q, st["E"], st["B"], alive=alive.astype(np.int8))
    rho_o = gs.rho()
    scale = np.abs(rho_o).max()
    e_rho = np.abs(rho1.reshape(rho_o.shape) - rho_o).max() / scale
    gauss_o = O.divergence(cfg, gs.E) - rho_o - g0.reshape(rho_o.shape)
    wf, wk = gs.energies()
    # the same energies summed pairwise (numpy): the oracle adds its 2e8 and
    # 2.7e8 terms one after the other, whose rounding reaches N * 2^-53
    # relative (about 1e-11 here), while pairwise sums stay near 1e-15
    dV = float(np.prod(w.dx3))
    wf_p = 0.5 * dV * (np.sum(st["E"] ** 2) + np.sum(st["B"] ** 2))
    g1 = np.sqrt(1.0 + np.sum(st["u"] ** 2, axis=0))
    wk_p = dV * np.sum(np.abs(q) * (g1 - 1.0))
    say("oracle diagnostics: rho err %.2e, gauss max %.3e (gpu %.3e), w_field %.12e / pairwise "
        "%.12e (gpu %.12e), w_kin %.12e / pairwise %.12e (gpu %.12e)"
        % (e_rho, np.abs(gauss_o).max(), d1.raw["gauss_max"], wf, wf_p, d1.raw["w_field"], wk,
           wk_p, d1.raw["w_kin"]))
    assert e_rho <= 1e-12
    assert abs(d1.raw["gauss_max"] - np.abs(gauss_o).max()) <= 1e-12 * scale
    nf, nk = 6 * st["E"][0].size, pl.np
    assert abs(d1.raw["w_field"] - wf) <= nf * 2.0 ** -53 * wf
    assert abs(d1.raw["w_kin"] - wk) <= nk * 2.0 ** -53 * wk
    assert abs(d1.raw["w_field"] - wf_p) <= 1e-12 * wf_p
    assert abs(d1.raw["w_kin"] - wk_p) <= 1e-12 * wk_p
    # the physics the diagnostics watch: the FP32 step conserves charge to
    # single precision, and Gauss's law keeps its initial residual up to the
    # rounding of the stored E (each sample within 2^-24 of max |E|, and the
    # divergence sums two of them per axis over dx_d)
    assert d1.raw["cont_rel_l2"] <= 1e-6
    emax = max(np.abs(st["E"]).max(), 1e-300)
    bound = 4 * 2.0 ** -24 * emax * sum(2.0 / w.dx3[d] for d in range(3))
    say("gauss change %.3e, FP32 rounding bound %.3e" % (d1.raw["gauss_max"], bound))
    assert d1.raw["gauss_max"] <= bound
    assert d1.raw["flags"] == 0
