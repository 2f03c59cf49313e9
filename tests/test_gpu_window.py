"""GPU parity of the moving window and the laser antenna (the window that
follows the laser through the plasma, Sec. 2) against the oracle: the state
shifts one cell along x whenever light has travelled one more cell, plasma
enters in the front column from the same seeded draws on both sides, and the
antenna's current sheet launches the pulse.  Particles are matched by id
(injected particles continue the count on both sides)."""
import numpy as np
import pytest

import oracle as O
from paper_1310_0930_amd import inputs as I

from _parity import TOL, compare, inputs_for, oracle_config, oracle_state, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELD_TOL = {8: 1e-10, 4: 1e-4}


def _antenna(w, a0=1.0):
    ny = w.n[1] * w.dx[1]
    return dict(x_index=6, polarization=1, a0=a0, omega0=10.0, waist=0.25 * ny, tau=0.6,
                t_center=1.5, y_center=0.5 * ny, z_center=0.5 * w.n3[2] * w.dx3[2] if w.dims == 3 else 0.0)


def _run(w, rb, steps, antenna=None, ions=False, spare_columns=None):
    """Both sides through `steps` steps with the window following light.
    The GPU's particle arrays hold np plus `spare_columns` entering columns
    (default: every column that enters during the run)."""
    from paper_1310_0930_amd import pic as P
    pe, E, B = inputs_for(w)
    pc = w.particle_cells()
    ncol = pc[1] * (pc[2] if w.dims == 3 else 1) * w.ppc
    nshift = int(steps * w.dt / w.dx[0]) + 1 if spare_columns is None else spare_columns
    sim = P.Simulation.from_workload(w, real_bytes=rb)
    sim.load(pe, E, B, capacity=pe.np + nshift * ncol)
    cfg = oracle_config(w)
    if ions:
        pi = I.make_ions(w)
        sim.add_species(pi, w.ions.q_over_m, w.q_const_ions, capacity=pi.np + nshift * ncol)
        ref = O.MultiState(cfg, [O.Species(-1.0, pe.global_positions(w), pe.u.T, pe.charges()),
                                 O.Species(w.ions.q_over_m, pi.global_positions(w), pi.u.T,
                                           pi.charges())], E, B)
    else:
        ref = oracle_state(w, pe, E, B)
    if antenna is not None:
        sim.set_antenna(P.antenna_struct(**antenna))
        ref.antenna = O.Antenna(**antenna)
    shifts = 0
    for n in range(1, steps + 1):
        sim.step(1)
        ref.step(1)
        while (shifts + 1) * w.dx[0] <= n * w.dt:  # the window follows light
            shifts += 1
            inj = [I.inject_column(w, shifts)]
            if ions:
                inj.append(I.inject_column(w, shifts, ions=True))
            sim.window_shift(inj[0], species_inject=inj[1:])
            O.window_shift(ref, [(p.global_positions(w), p.u.T, p.charges()) for p in inj])
    torch.cuda.synchronize()
    say(w.name, "real", rb, "steps", steps, "shifts", shifts, "np", sim.np, "capacity",
        sim.capacity)
    assert shifts >= 2
    return sim, ref


def _check(w, rb, sim, ref, what):
    err = compare(w, sim, ref)
    say(what, err)
    assert err["alive_mismatch"] == 0, err
    assert err["pos"] <= TOL[rb], err
    assert err["u"] <= TOL[rb], err
    for f in ("E", "B", "J"):
        assert err[f] <= FIELD_TOL[rb], (f, err)
    return err


@pytest.mark.parametrize("rb", [8, 4])
def test_window_shift_thermal_2d(rb):
    """Thermal plasma, open x and y, quadratic: several shifts with injected
    thermal plasma."""
    w = I.Workload("win2d", 2, (48, 24), (0.1, 0.2), 2, 4, 0.1, 12, bc=(I.OPEN, I.OPEN),
                   seed=I.SEED_BASE + 120)
    sim, ref = _run(w, rb, w.steps)
    _check(w, rb, sim, ref, "window 2d")


@pytest.mark.parametrize("rb", [8, 4])
@pytest.mark.parametrize("order", [1, 3])
def test_window_shift_thermal_3d(rb, order):
    w = I.Workload("win3d", 3, (32, 12, 10), (0.1, 0.2, 0.2), order, 2, 0.1, 8,
                   bc=(I.OPEN, I.PERIODIC, I.OPEN), seed=I.SEED_BASE + 121 + order)
    sim, ref = _run(w, rb, w.steps)
    _check(w, rb, sim, ref, f"window 3d order {order}")


@pytest.mark.parametrize("rb,steps", [(8, 40), (4, 16)])
def test_moving_window_lwfa_2d(rb, steps):
    """The LWFA set-up: cold plasma behind a 20-cell ramp, the pulse launched
    by the antenna, the window moving at c with plasma entering at the front."""
    w = I.Workload("lwfa2d", 2, (96, 40), (0.1, 0.2), 2, 4, 0.0, steps, bc=(I.OPEN, I.OPEN),
                   ramp_cells=20.0, seed=I.SEED_BASE + 124)
    sim, ref = _run(w, rb, steps, antenna=_antenna(w))
    _check(w, rb, sim, ref, "moving window lwfa 2d")
    assert np.abs(ref.E[1]).max() > 1.0  # the pulse is there


@pytest.mark.parametrize("rb,steps", [(8, 450), (4, 120)])
def test_long_window_run_reuses_absorbed_slots(rb, steps):
    """A window that keeps moving (about 200 shifts in FP64) in particle
    arrays with room for only two entering columns: every sort compacts the
    particles absorbed at the back, so the slots are reused and np stays
    bounded; the state still matches the oracle particle by particle (by
    id: the entering particles continue the id count on both sides)."""
    w = I.Workload("winlong", 2, (64, 24), (0.1, 0.2), 2, 4, 0.02, steps, bc=(I.OPEN, I.OPEN),
                   ramp_cells=10.0, seed=I.SEED_BASE + 128)
    sim, ref = _run(w, rb, steps, spare_columns=2)
    pc = w.particle_cells()
    assert sim.np <= sim.capacity
    assert ref.np > sim.capacity  # the oracle keeps every particle it ever had
    assert int(sim.id[: sim.np].max()) >= ref.np - 2 * pc[1] * w.ppc
    if rb == 8:
        assert int(steps * w.dt / w.dx[0]) >= 200
    _check(w, rb, sim, ref, "long window run")


@pytest.mark.parametrize("rb", [8, 4])
def test_moving_window_with_ions_3d(rb):
    """Electrons and mobile ions (M = 16) both entering at the front, 3D,
    antenna polarised along z."""
    w = I.Workload("lwfa3d", 3, (32, 12, 12), (0.1, 0.2, 0.2), 2, 2, 0.02, 10,
                   bc=(I.OPEN, I.OPEN, I.OPEN), ramp_cells=8.0,
                   ions=I.Ions(mass_ratio=16.0, u_th=0.01), seed=I.SEED_BASE + 125)
    ant = _antenna(w)
    ant["polarization"] = 2
    sim, ref = _run(w, rb, w.steps, antenna=ant, ions=True)
    import types
    for k, s in enumerate([sim] + sim.species):
        sp = ref.species[k]
        view = types.SimpleNamespace(X=sp.X, u=sp.u, alive=sp.alive, E=ref.E, B=ref.B, J=ref.J)
        _check(w, rb, s, view, f"window + ions species {k}")


def test_antenna_add_matches_oracle_current():
    """pic_antenna_add on a zero J equals the oracle's sheet current (FP64)."""
    from paper_1310_0930_amd import pic as P
    w = I.Workload("ant", 3, (20, 16, 12), (0.1, 0.2, 0.25), 2, 1, 0.0, 1,
                   bc=(I.OPEN, I.OPEN, I.PERIODIC), seed=I.SEED_BASE + 126)
    pe, E, B = inputs_for(w)
    sim = P.Simulation.from_workload(w, real_bytes=8)
    sim.load(pe, E, B)
    for pol in (1, 2):
        a = _antenna(w)
        a["polarization"] = pol
        for t in (0.9, 1.5, 2.2):
            sim.J.zero_()
            sim.antenna_add(P.antenna_struct(**a), t)
            Jg = sim.J.double().cpu().numpy().reshape((3,) + oracle_config(w).shape)
            Jr = O.antenna_current(oracle_config(w), O.Antenna(**a), t)
            assert np.abs(Jg - Jr).max() <= 1e-13 * np.abs(Jr).max()


def test_window_shift_argument_checks():
    """Periodic x, a capacity below np + n and a column count that does not
    match are rejected before any launch (PIC_EINVAL)."""
    from paper_1310_0930_amd import pic as P
    w = I.Workload("winbad", 2, (24, 12), (0.1, 0.2), 2, 2, 0.1, 1, bc=(I.OPEN, I.OPEN),
                   seed=I.SEED_BASE + 127)
    pe, E, B = inputs_for(w)
    sim = P.Simulation.from_workload(w, real_bytes=8)
    sim.load(pe, E, B)  # capacity = np
    inj = I.inject_column(w, 1)
    with pytest.raises(P.PicError) as e:
        sim.window_shift(inj)
    assert e.value.status == P.PIC_EINVAL
    wp = w.with_(bc=(I.PERIODIC, I.OPEN))
    sp = P.Simulation.from_workload(wp, real_bytes=8)
    sp.load(I.make_plasma(wp), capacity=10 ** 5)
    with pytest.raises(P.PicError) as e:
        sp.window_shift(None)
    assert e.value.status == P.PIC_EINVAL
    sim2 = P.Simulation.from_workload(w, real_bytes=8)
    sim2.load(pe, E, B, capacity=pe.np + 10 ** 4)
    bad = I.Plasma(inj.cell[:-1], inj.off[:, :-1], inj.u[:, :-1], None, inj.q_const,
                   extra={"ppc": w.ppc})
    with pytest.raises(P.PicError) as e:
        sim2.window_shift(bad)
    assert e.value.status == P.PIC_EINVAL
