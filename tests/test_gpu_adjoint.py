"""GPU checks of the hand-written adjoint (transpose of the field advance,
vector-Jacobian product of push/deposit, checkpointed autograd rollout).

* dot-product tests <lam, F delta> = <F^T lam, delta> for the linear field
  advance, periodic and open (Mur) boundaries;
* one whole step: <lam_out, J delta_in> with J delta_in from the FP64
  oracle's dual-number JVP (itself pinned against finite differences)
  against <J^T lam_out, delta_in> from the GPU adjoint;
* whole rollouts: dL/da0 and dL/du0 . v against the oracle's JVP and
  central finite differences (FP64 within 1e-8, FP32 within 1e-3).
"""
import numpy as np
import pytest

import oracle as O
from paper_1310_0930_amd import inputs as I

from _parity import inputs_for, oracle_state, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _sim(w, rb, sort_every=None):
    from paper_1310_0930_amd.pic import Simulation
    return Simulation(w.dims, w.n3, w.dx3, w.dt, w.order, rb, w.bc3,
                      sort_every=w.sort_every if sort_every is None else sort_every,
                      q_const=w.q_const)


def _t(a, sim):
    return torch.from_numpy(np.ascontiguousarray(a)).to(sim.device, sim.real)


@pytest.mark.parametrize("dims,bc,rb,nz", [(3, (0, 0, 0), 8, 9), (3, (0, 0, 0), 8, 8),
                                           (3, (0, 0, 0), 4, 8), (2, (0, 1), 8, 0),
                                           (3, (0, 1, 1), 8, 9), (2, (1, 1), 8, 0),
                                           (3, (0, 1, 1), 4, 9)])
def test_field_advance_adjoint_dot_product(dims, bc, rb, nz):
    """<lamE, E'> + <lamB, B'> of one field advance equals the adjoint's
    <lamE', dE> + <lamB', dB> + <lamJ', dJ>.  nz = 8 on a periodic 3D grid
    takes the z-column kernels of the forward advance, nz = 9 the
    one-thread-per-cell ones."""
    from paper_1310_0930_amd import pic as P
    n = (12, 10, nz) if dims == 3 else (16, 12)
    dx = (0.2, 0.25, 0.3)[:dims]
    w = I.Workload("fa", dims, n, dx, 2, 1, 0.0, 1, bc=bc)
    sim = _sim(w, rb)
    empty = I.Plasma(np.zeros(0, np.int32), np.zeros((3, 0), np.float32),
                     np.zeros((3, 0), np.float32), None, -1.0)
    sim.load(empty, None, None, with_id=False)
    rng = np.random.default_rng(7 + dims)
    shp = (3, sim.ncell)
    dE, dB, dJ = (rng.normal(size=shp) for _ in range(3))
    lE, lB = rng.normal(size=shp), rng.normal(size=shp)
    sim.E.copy_(_t(dE, sim))
    sim.B.copy_(_t(dB, sim))
    sim.J.copy_(_t(dJ, sim))
    sim.field_advance()
    lhs = float((_t(lE, sim).double() * sim.E.double()).sum() + (_t(lB, sim).double() * sim.B.double()).sum())
    LE, LB, LJ = _t(lE, sim), _t(lB, sim), torch.zeros_like(sim.J)
    P.pic_field_advance_adjoint(sim.ctx, P.fields_struct(LE, LB, LJ), sim.ws.data_ptr(), sim.stream)
    rhs = float((LE.double() * _t(dE, sim).double()).sum() + (LB.double() * _t(dB, sim).double()).sum()
                + (LJ.double() * _t(dJ, sim).double()).sum())
    say("fdtd adjoint", dims, bc, rb, lhs, rhs)
    assert abs(lhs - rhs) <= (1e-12 if rb == 8 else 1e-5) * (abs(lhs) + 1.0) * 10


def _one_step_check(w, rb, seed, tiled=True):
    """<lam_out, JVP(delta)> (oracle, FP64) vs <VJP(lam_out), delta> (GPU);
    tiled=False hands the adjoint a workspace without tile bins (the
    global-memory kernel for every particle)."""
    from paper_1310_0930_amd import pic as P
    pl, E, B = inputs_for(w)
    D = w.dims
    rng = np.random.default_rng(seed)
    npart = pl.np
    # directions in the caller's particle order
    dX = np.zeros((npart, 3))
    dX[:, :D] = rng.normal(size=(npart, D))
    du = rng.normal(size=(npart, 3))
    dE = rng.normal(size=E.shape)
    dB = rng.normal(size=B.shape)
    lX = np.zeros((npart, 3))
    lX[:, :D] = rng.normal(size=(npart, D))
    lu = rng.normal(size=(npart, 3))
    lE = rng.normal(size=E.shape)
    lB = rng.normal(size=B.shape)
    # oracle JVP of one step
    ref = oracle_state(w, pl, E, B)
    tX, tu, tE, tB, _ = ref.step_jvp(1, dX, du, dE, dB)
    lhs = (np.sum(lX[:, :D] * tX[:, :D]) + np.sum(lu * tu) + np.sum(lE * tE) + np.sum(lB * tB))
    # GPU adjoint of one step
    sim = _sim(w, rb)
    sim.load(pl, E, B, with_id=True)
    sim.sort()
    ids = sim.id.long().cpu().numpy()
    state = (sim.cell.clone(), sim.off.clone(), sim.u.clone(), sim.E.clone(), sim.B.clone())
    LX = torch.zeros_like(sim.off)
    LU = torch.zeros_like(sim.u)
    LX[:D] = _t(lX[ids, :D].T, sim)
    LU[:] = _t(lu[ids].T, sim)
    LE = _t(lE.reshape(3, -1), sim)
    LB = _t(lB.reshape(3, -1), sim)
    LJ = torch.zeros_like(LE)
    lf = P.fields_struct(LE, LB, LJ)
    P.pic_field_advance_adjoint(sim.ctx, lf, sim.ws.data_ptr(), sim.stream)
    parts = P.particles_struct(sim.np, state[0], state[1], state[2], sim.q)
    ws = sim.ws if tiled else torch.zeros_like(sim.ws)
    P.pic_push_deposit_adjoint(sim.ctx, parts, P.fields_struct(state[3], state[4]), lf,
                               P.particles_struct(sim.np, None, LX, LU), ws.data_ptr(), sim.stream)
    torch.cuda.synchronize()
    gX = np.zeros((npart, 3))
    gu = np.zeros((npart, 3))
    gX[ids, :D] = LX[:D].double().cpu().numpy().T
    gu[ids] = LU.double().cpu().numpy().T
    rhs = (np.sum(gX[:, :D] * dX[:, :D]) + np.sum(gu * du)
           + np.sum(LE.double().cpu().numpy().reshape(E.shape) * dE)
           + np.sum(LB.double().cpu().numpy().reshape(B.shape) * dB))
    say("step adjoint", w.name, rb, lhs, rhs, abs(lhs - rhs) / abs(lhs))
    return lhs, rhs


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_step_adjoint_matches_oracle_jvp_3d(order):
    w = I.Workload("adj3", 3, (12, 10, 9), (0.2, 0.25, 0.2), order, 4, 0.3, 1,
                   seed=I.SEED_BASE + 90 + order)
    lhs, rhs = _one_step_check(w, 8, 11 + order)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


@pytest.mark.parametrize("tiled", [True, False])
@pytest.mark.parametrize("bc", [(0, 1, 0), (0, 0, 1), (1, 1, 1)])
@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_step_adjoint_matches_oracle_jvp_3d_open_faces(order, bc, tiled):
    """One 3D step's adjoint against the oracle's JVP with an open y face, an
    open z face (the axis the LDS slabs cut), and every face open; z has a
    ragged last tile.  tiled: sorted particles with their tile bins (LDS
    tiles or z slabs, off-allowance particles through the global kernel);
    otherwise every particle in the global-memory kernel."""
    w = I.Workload("adj3o", 3, (12, 10, 9), (0.2, 0.25, 0.2), order, 4, 0.3, 1, bc=bc,
                   ramp_cells=3.0, seed=I.SEED_BASE + 150 + order + 4 * sum(bc))
    lhs, rhs = _one_step_check(w, 8, 61 + order + 7 * bc[2], tiled=tiled)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_step_adjoint_matches_oracle_jvp_2d_open_laser(order):
    lz = I.Laser(a0=2.0, omega0=4.0, waist=1.0, tau=0.4, x_center=1.2)
    w = I.Workload("adj2", 2, (32, 16), (0.1, 0.2), order, 4, 0.2, 1, bc=(0, 1),
                   ramp_cells=8.0, laser=lz, seed=I.SEED_BASE + 95 + order)
    lhs, rhs = _one_step_check(w, 8, 21 + order)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def _rollout_case(steps=12):
    lz = I.Laser(a0=2.0, omega0=6.0, waist=1.5, tau=0.5, x_center=1.5)
    return I.Workload("roll", 2, (64, 24), (0.1, 0.2), 2, 4, 0.0, steps, bc=(0, 1),
                      ramp_cells=10.0, laser=lz, seed=I.SEED_BASE + 97)


def _oracle_directional(w, pl, E1, B1, a0, du, da0):
    """d/de L(a0 + e da0, u0 + e du) at e = 0 from the oracle's JVP."""
    ref = oracle_state(w, pl, a0 * E1, a0 * B1)
    ref.u[:] = pl.u.T.astype(np.float64)
    _, _, tE, _, _ = ref.step_jvp(w.steps, np.zeros_like(ref.X), du, da0 * E1, da0 * B1)
    from paper_1310_0930_amd.adjoint import window_energy
    Ex = torch.from_numpy(ref.E.reshape(3, -1))
    tEx = torch.from_numpy(tE.reshape(3, -1))
    _, (lo, hi) = window_energy(w, Ex)
    dV = float(np.prod(w.dx[: w.dims]))
    shape = (w.n3[2], w.n3[1], w.n3[0])
    return float(dV * np.sum(ref.E[0].reshape(shape)[:, :, lo:hi] * tE[0].reshape(shape)[:, :, lo:hi]))


@pytest.mark.parametrize("rb", [8, 4])
def test_rollout_gradient_matches_oracle_jvp(rb):
    from paper_1310_0930_amd.adjoint import PicRollout, Runner, window_energy
    w = _rollout_case()
    pl, E1, B1 = inputs_for(w)  # fields for a0 = laser.a0
    a0v = w.laser.a0
    E1 = E1 / a0v
    B1 = B1 / a0v
    runner = Runner(w, real_bytes=rb, checkpoint_every=5)
    runner.set_inputs(pl, E1, B1)
    a0 = torch.tensor(a0v, dtype=torch.float64, device="cuda", requires_grad=True)
    u0 = torch.from_numpy(pl.u).to("cuda", runner.real).requires_grad_(True)
    E, B = PicRollout.apply(a0, u0, runner)
    L, _ = window_energy(w, E)
    L.backward()
    g_a0 = float(a0.grad)
    rng = np.random.default_rng(3)
    v = rng.choice([-1.0, 1.0], size=(pl.np, 3))
    g_v = float((u0.grad.double().cpu().numpy().T * v).sum())
    j_a0 = _oracle_directional(w, pl, E1, B1, a0v, np.zeros((pl.np, 3)), 1.0)
    j_v = _oracle_directional(w, pl, E1, B1, a0v, v, 0.0)
    say("rollout grad", rb, "a0", g_a0, j_a0, "v", g_v, j_v)
    tol = 1e-8 if rb == 8 else 1e-3
    assert abs(g_a0 - j_a0) <= tol * abs(j_a0)
    assert abs(g_v - j_v) <= tol * max(abs(j_v), 1e-3 * abs(j_a0))


def test_rollout_gradient_matches_central_differences_fp64():
    """FP64 GPU forward: central differences of L along a0 and along a
    Rademacher direction of u0 against the adjoint."""
    from paper_1310_0930_amd.adjoint import PicRollout, Runner, window_energy
    w = _rollout_case()
    pl, E1, B1 = inputs_for(w)
    a0v = w.laser.a0
    E1, B1 = E1 / a0v, B1 / a0v
    runner = Runner(w, real_bytes=8, checkpoint_every=4)
    runner.set_inputs(pl, E1, B1)
    u_base = torch.from_numpy(pl.u).to("cuda", torch.float64)
    a0 = torch.tensor(a0v, dtype=torch.float64, device="cuda", requires_grad=True)
    u0 = u_base.clone().requires_grad_(True)
    E, _ = PicRollout.apply(a0, u0, runner)
    L, _ = window_energy(w, E)
    L.backward()
    rng = np.random.default_rng(5)
    v = torch.from_numpy(rng.choice([-1.0, 1.0], size=(3, pl.np))).to("cuda", torch.float64)

    def loss(a, u):
        with torch.no_grad():
            E, _ = runner.forward(torch.tensor(a, dtype=torch.float64, device="cuda"), u)
            return float(window_energy(w, E)[0])

    h = 1e-6
    fd_a0 = (loss(a0v + h, u_base) - loss(a0v - h, u_base)) / (2 * h)
    fd_v = (loss(a0v, u_base + h * v) - loss(a0v, u_base - h * v)) / (2 * h)
    g_v = float((u0.grad * v).sum())
    say("fd", fd_a0, float(a0.grad), fd_v, g_v)
    assert abs(float(a0.grad) - fd_a0) <= 1e-6 * abs(fd_a0)
    assert abs(g_v - fd_v) <= 1e-6 * max(abs(fd_v), 1e-3 * abs(fd_a0))


def _tiled_vs_global(w, rb, seed, shuffled_too=True):
    """Step adjoint with the sort's workspace (LDS tiles or slabs) against a
    workspace holding no tile bins (global memory), and, with the tile bins,
    for the particles in another order (most then take the global-memory
    path inside the tiled call): lamE, lamB, lamX, lamU element by element."""
    from paper_1310_0930_amd import pic as P
    pl, E, B = inputs_for(w)
    sim = _sim(w, rb)
    sim.load(pl, E, B, with_id=True)
    sim.sort()
    rng = np.random.default_rng(seed)
    shp = (3, sim.ncell)
    lE0, lB0, lJ0 = (_t(rng.normal(size=shp), sim) for _ in range(3))
    lX0 = _t(rng.normal(size=(3, sim.np)), sim)
    lU0 = _t(rng.normal(size=(3, sim.np)), sim)
    other_ws = torch.zeros_like(sim.ws)

    def run(perm, ws):
        cell, off, u = sim.cell[perm].clone(), sim.off[:, perm].clone(), sim.u[:, perm].clone()
        q = None if sim.q is None else sim.q[perm].clone()
        LE, LB, LJ = lE0.clone(), lB0.clone(), lJ0.clone()
        LX, LU = lX0[:, perm].clone(), lU0[:, perm].clone()
        P.pic_push_deposit_adjoint(sim.ctx, P.particles_struct(sim.np, cell, off, u, q),
                                   P.fields_struct(sim.E, sim.B), P.fields_struct(LE, LB, LJ),
                                   P.particles_struct(sim.np, None, LX, LU), ws.data_ptr(), sim.stream)
        torch.cuda.synchronize()
        inv = torch.empty_like(perm)
        inv[perm] = torch.arange(perm.numel(), device=perm.device)
        return [t.double().cpu().numpy() for t in (LE, LB, LX[:, inv], LU[:, inv])]

    ident = torch.arange(sim.np, device=sim.device)
    tiled = run(ident, sim.ws)            # LDS tiles (sorted order)
    glob = run(ident, other_ws)           # no tile bins in this workspace
    mixed = None
    if shuffled_too:
        shuffled = torch.from_numpy(rng.permutation(sim.np)).to(sim.device)
        mixed = run(shuffled, sim.ws)     # tile bins, particles in another order
    tol = 1e-11 if rb == 8 else 2e-4
    for k, name in enumerate(("lamE", "lamB", "lamX", "lamU")):
        a, b = tiled[k], glob[k]
        scale = np.abs(b).max() + 1e-30
        say("tiled vs global", w.name, w.dims, w.order, rb, name, np.abs(a - b).max() / scale,
            None if mixed is None else np.abs(mixed[k] - b).max() / scale)
        assert np.abs(a - b).max() <= tol * scale, name
        if mixed is not None:
            assert np.abs(mixed[k] - b).max() <= tol * scale, name


@pytest.mark.parametrize("dims,rb,order,bc", [
    (2, 8, 2, (0, 1)), (2, 4, 2, (0, 1)), (2, 8, 3, (0, 1)),
    (3, 8, 1, (0, 1, 0)), (3, 4, 1, (0, 1, 0)), (3, 8, 2, (0, 1, 0)), (3, 4, 2, (0, 1, 0)),
    (3, 4, 3, (0, 1, 0)), (3, 8, 4, (0, 1, 0)), (3, 4, 4, (0, 1, 0)),
    (3, 8, 1, (0, 1, 1)), (3, 4, 1, (0, 1, 1)), (3, 8, 2, (0, 1, 1)), (3, 4, 2, (0, 1, 1)),
    (3, 4, 3, (0, 1, 1)), (3, 8, 4, (0, 1, 1)), (3, 4, 4, (0, 1, 1))])
def test_tiled_step_adjoint_equals_global_memory_adjoint(dims, rb, order, bc):
    """The step adjoint runs out of LDS when the context holds tile bins for
    the particles (same count, same workspace), else one thread per particle
    in global memory.  In 3D a tile is cut into z slabs (one per workgroup)
    where its regions exceed a CU's LDS: 2 slabs for quadratic FP32 and
    linear FP64, 4 for cubic FP32 and quadratic FP64, one-cell slabs for
    quartic FP32 (linear FP32 and quartic FP64 take whole tiles); the 3D
    grid here has a ragged last tile along z and an open y face, or open y
    and z faces (slabs next to the open z face).  Both paths
    must give the same lamX, lamU, lamE, lamB, also for particles in an
    order other than the sort's."""
    if dims == 2:
        lz = I.Laser(a0=2.0, omega0=4.0, waist=1.0, tau=0.4, x_center=1.2)
        w = I.Workload("adjt", 2, (48, 32), (0.1, 0.2), order, 6, 0.2, 1, bc=bc,
                       ramp_cells=6.0, laser=lz, seed=I.SEED_BASE + 120 + order)
    else:
        w = I.Workload("adjt3", 3, (24, 16, 20), (0.2, 0.25, 0.2), order, 4, 0.3, 1,
                       bc=bc, ramp_cells=4.0, seed=I.SEED_BASE + 130 + order)
    _tiled_vs_global(w, rb, 31 + order)


@pytest.mark.parametrize("rb,order", [(8, 2), (4, 2), (4, 3)])
def test_tiled_step_adjoint_equals_global_memory_adjoint_at_64_cubed(rb, order):
    """The same at the bench plasma's density and temperature on a 64^3 grid
    (8 ppc, 2.1M particles, 512 tiles, 2 or 4 slabs each), sorted order."""
    w = I.Workload("adjt64", 3, (64, 64, 64), (0.2, 0.2, 0.2), order, 8, 0.05, 1,
                   seed=I.SEED_BASE + 140 + order)
    _tiled_vs_global(w, rb, 41 + order, shuffled_too=False)
