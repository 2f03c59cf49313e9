"""Pins of the FP64 oracle against closed forms, invariants, library routines
and brute force (no GPU).  Each test names what fixes the expected value.

The paper states the method in prose only (PIC loop of Sec. 2; virtual
particles and charge-conserving deposit of Sec. 5.2; cell-relative positions
of Sec. 5.1), so every expected value here comes from mathematics, not from
printed numbers.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import BSpline

import oracle as O
from oracle import OPEN as OPEN_
from paper_1310_0930_amd import inputs as I

RNG = np.random.default_rng(20131003)


def cfg3(n=(8, 8, 8), dx=(0.2, 0.2, 0.2), order=2, bc=(0, 0, 0), frac=0.5):
    dt = frac * I.courant_dt(dx, 3)
    return O.Config(3, n, dx, dt, order, bc)


def cfg2(n=(16, 16), dx=(0.2, 0.2), order=1, bc=(0, 0), frac=0.5):
    dt = frac * I.courant_dt(dx, 2)
    return O.Config(2, tuple(n) + (1,), tuple(dx) + (1.0,), dt, order, tuple(bc) + (0,))


# ---------------------------------------------------------------- shapes
@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_shape_matches_cardinal_bspline(order):
    """Weights equal the centred cardinal B-spline of degree `order`
    (scipy's basis element on knots -(n+1)/2 .. (n+1)/2)."""
    knots = np.arange(order + 2) - (order + 1) / 2.0
    M = BSpline.basis_element(knots, extrapolate=False)
    for X in RNG.uniform(-3, 40, size=200):
        base, w = O.shape(order, X)
        nodes = base + np.arange(order + 1)
        ref = np.nan_to_num(M(X - nodes))
        np.testing.assert_allclose(w, ref, atol=1e-14)
        # every node outside the stencil has zero weight
        for far in (base - 1, base + order + 1):
            assert abs(np.nan_to_num(M(X - far))) < 1e-14


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_shape_moments(order):
    for X in RNG.uniform(0, 50, size=100):
        base, w = O.shape(order, X)
        assert np.all(w >= -1e-15)
        assert abs(w.sum() - 1.0) < 1e-14
        assert abs(np.dot(base + np.arange(order + 1), w) - X) < 1e-12


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_gather_reproduces_linear_fields(order):
    """B-splines reproduce linear functions, at node-centred and staggered
    component positions alike (each component sampled where it sits)."""
    c = cfg3(n=(12, 10, 9), order=order)
    nz, ny, nx = c.shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    a = np.array([0.3, -0.7, 0.45])
    E = np.zeros((3, nz, ny, nx))
    B = np.zeros_like(E)
    for comp in range(3):
        se = [1 if d == comp else 0 for d in range(3)]
        sb = [0 if d == comp else 1 for d in range(3)]
        E[comp] = (comp + 1) + a[0] * (i + 0.5 * se[0]) + a[1] * (j + 0.5 * se[1]) + a[2] * (k + 0.5 * se[2])
        B[comp] = -(comp + 2) + a[2] * (i + 0.5 * sb[0]) + a[0] * (j + 0.5 * sb[1]) + a[1] * (k + 0.5 * sb[2])
    # stay away from the periodic seam, where the linear field jumps
    X = RNG.uniform(3.0, 6.0, size=(50, 3))
    Ep, Bp = O.gather(c, X, E, B)
    for comp in range(3):
        np.testing.assert_allclose(Ep[:, comp], (comp + 1) + X @ a, atol=1e-12)
        np.testing.assert_allclose(Bp[:, comp], -(comp + 2) + X @ a[[2, 0, 1]], atol=1e-12)


# ---------------------------------------------------------------- Boris
def test_boris_pure_e_exact_kick():
    """B = 0: u^{n+1/2} = u^{n-1/2} + (q/m) E dt exactly."""
    c = cfg3()
    u = RNG.normal(0, 2.0, size=(64, 3))
    E = RNG.normal(0, 3.0, size=(64, 3))
    out = O.boris(c, u, E, np.zeros_like(E))
    np.testing.assert_allclose(out, u + c.q_over_m * c.dt * E, rtol=0, atol=1e-13)


def test_boris_pure_b_rotation_angle():
    """E = 0: |u| is conserved and u rotates about B by 2 atan(|q/m| B dt / (2 gamma))."""
    c = cfg3()
    for _ in range(50):
        u = RNG.normal(0, 3.0, size=3)
        Bv = RNG.normal(0, 5.0, size=3)
        out = O.boris(c, u[None], np.zeros((1, 3)), Bv[None])[0]
        assert abs(np.linalg.norm(out) - np.linalg.norm(u)) < 1e-12 * np.linalg.norm(u)
        bh = Bv / np.linalg.norm(Bv)
        up0 = u - np.dot(u, bh) * bh
        up1 = out - np.dot(out, bh) * bh
        assert abs(np.dot(u, bh) - np.dot(out, bh)) < 1e-12
        gamma = math.sqrt(1 + u @ u)
        theta = 2 * math.atan(abs(c.q_over_m) * np.linalg.norm(Bv) * c.dt / (2 * gamma))
        cosang = np.dot(up0, up1) / (np.linalg.norm(up0) * np.linalg.norm(up1))
        assert abs(math.acos(min(1.0, cosang)) - theta) < 1e-9
        # electrons (q < 0) rotate right-handed about B
        assert np.dot(np.cross(up0, up1), bh) * np.sign(-c.q_over_m) > 0


def _uniform_field_state(c, Evec, Bvec, X0, u0):
    """A zero-charge test particle in uniform grid fields (J stays zero, so a
    uniform field is a steady state of the field solver)."""
    E = c.zeros_field()
    B = c.zeros_field()
    for comp in range(3):
        E[comp] = Evec[comp]
        B[comp] = Bvec[comp]
    return O.State(c, np.array([X0]), np.array([u0]), np.zeros(1), E, B)


def test_uniform_e_acceleration_second_order():
    """From rest in a uniform E_x (electron, q/m = -1), the position converges at
    second order to x(t) = (sqrt(1 + (E t)^2) - 1)/E along -E."""
    Ex, T = 2.0, 0.8
    errs = []
    for steps in (20, 40, 80):
        dx = (1.0, 1.0, 1.0)
        c = O.Config(3, (64, 8, 8), dx, T / steps, 1)
        s = _uniform_field_state(c, (Ex, 0, 0), (0, 0, 0), (40.0, 4.0, 4.0), (0, 0, 0))
        # u is given at -dt/2: start it there so that x(0) has zero velocity
        s.u[0, 0] = c.q_over_m * Ex * (-c.dt / 2)
        s.step(steps)
        exact = (math.sqrt(1 + (Ex * T) ** 2) - 1) / Ex
        errs.append(abs((40.0 - s.X[0, 0]) * dx[0] - exact))
        # momentum is exact: u(T - dt/2) ... after `steps` kicks from -dt/2
        assert abs(s.u[0, 0] - c.q_over_m * Ex * (T - c.dt / 2)) < 1e-12
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_uniform_b_gyration_orbit():
    """In a uniform B_z, the orbit is a polygon inscribed in a circle: every
    position sits at the same distance from the guiding centre, |u| is
    conserved exactly, and successive chords turn by the Boris angle."""
    Bz, steps = 3.0, 60
    c = O.Config(3, (64, 64, 8), (0.5, 0.5, 0.5), 0.05, 2)
    u0 = (0.8, 0.0, 0.3)
    s = _uniform_field_state(c, (0, 0, 0), (0, 0, Bz), (32.0, 32.0, 4.0), u0)
    pts = []
    for _ in range(steps):
        s.step(1)
        pts.append(s.X[0].copy() * 0.5)
        assert abs(np.linalg.norm(s.u[0]) - np.linalg.norm(u0)) < 1e-13
    pts = np.array(pts)[:, :2]
    gamma = math.sqrt(1 + np.dot(u0, u0))
    theta = 2 * math.atan(Bz * c.dt / (2 * gamma))
    chord = c.dt * math.hypot(u0[0], u0[1]) / gamma
    R = chord / (2 * math.sin(theta / 2))
    # centre from three points
    a, b, d = pts[0], pts[1], pts[2]
    A = np.array([b - a, d - a]) * 2
    rhs = np.array([b @ b - a @ a, d @ d - a @ a])
    ctr = np.linalg.solve(A, rhs)
    r = np.linalg.norm(pts - ctr, axis=1)
    np.testing.assert_allclose(r, R, rtol=1e-9)
    # z drifts at the constant v_z
    assert abs(s.X[0, 2] * 0.5 - (2.0 + steps * c.dt * u0[2] / gamma)) < 1e-12


# ---------------------------------------------------------------- Yee / FDTD
def _phase(c, k, comp_pos, t):
    return k[0] * comp_pos[0] + k[1] * comp_pos[1] + k[2] * comp_pos[2] - t


def test_yee_discrete_eigenmode_2d_oblique():
    """E_z = cos(k.x - w t) with the discrete dispersion
    sin(w dt/2)/dt = |(sin(k_d dx_d/2)/dx_d)_d| is an exact solution of the
    leap-frog Yee scheme; B at -dt/2 is set from the mode and B^0 is formed by
    the half step the solver itself uses."""
    nx, ny = 32, 24
    c = cfg2(n=(nx, ny), dx=(0.2, 0.25), frac=0.9)
    dx, dy = 0.2, 0.25
    kx, ky = 2 * np.pi * 3 / (nx * dx), 2 * np.pi * 2 / (ny * dy)
    kt = np.array([2 * np.sin(kx * dx / 2) / dx, 2 * np.sin(ky * dy / 2) / dy])
    wt = np.linalg.norm(kt)
    w = 2 / c.dt * np.arcsin(wt * c.dt / 2)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    x, y = i * dx, j * dy

    def ez(t):
        return np.cos(kx * x + ky * y - w * t)

    def bx(t):  # at (i, j+1/2)
        return (kt[1] / wt) * np.cos(kx * x + ky * (y + dy / 2) - w * t)

    def by(t):  # at (i+1/2, j)
        return -(kt[0] / wt) * np.cos(kx * (x + dx / 2) + ky * y - w * t)

    E = c.zeros_field()
    B = c.zeros_field()
    E[2, 0] = ez(0.0)
    B[0, 0] = bx(-c.dt / 2)
    B[1, 0] = by(-c.dt / 2)
    # B^0 = B^{-1/2} - dt/2 C E^0
    B -= 0.5 * c.dt * O.curl_e(c, E)
    s = O.State(c, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), E, B)
    steps = 100
    for _ in range(steps):
        s.field_advance()
    T = steps * c.dt
    np.testing.assert_allclose(s.E[2, 0], ez(T), atol=1e-11)
    Bhalf = s.B - 0.5 * c.dt * O.curl_e(c, s.E)  # B^{N+1/2}
    np.testing.assert_allclose(Bhalf[0, 0], bx(T + c.dt / 2), atol=1e-11)
    np.testing.assert_allclose(Bhalf[1, 0], by(T + c.dt / 2), atol=1e-11)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_yee_eigenmode_3d_axis(axis):
    """1D-like discrete mode along each axis of a 3D anisotropic grid."""
    n = (16, 12, 10)
    dxs = (0.1, 0.2, 0.15)
    c = cfg3(n=n, dx=dxs, frac=0.8)
    pol = (axis + 1) % 3          # E polarisation
    bcomp = (axis + 2) % 3        # B component
    kk = 2 * np.pi * 2 / (n[axis] * dxs[axis])
    kt = 2 * np.sin(kk * dxs[axis] / 2) / dxs[axis]
    w = 2 / c.dt * np.arcsin(kt * c.dt / 2)
    grids = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    coord = [grids[2], grids[1], grids[0]][axis] * dxs[axis]
    E = c.zeros_field()
    B = c.zeros_field()
    # E_pol is node-located along `axis`; B_bcomp is half-way along `axis`
    E[pol] = np.cos(kk * coord)
    B[bcomp] = np.cos(kk * (coord + dxs[axis] / 2) + w * c.dt / 2)
    B -= 0.5 * c.dt * O.curl_e(c, E)
    s = O.State(c, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), E, B)
    for _ in range(60):
        s.field_advance()
    np.testing.assert_allclose(s.E[pol], np.cos(kk * coord - w * 60 * c.dt), atol=1e-11)


def test_vacuum_discrete_energy_invariant():
    """Periodic, J = 0: sum|E^n|^2 + sum B^{n-1/2}.B^{n+1/2} is conserved exactly
    by the leap-frog scheme, while 1/2 sum(E^2+B^2) only oscillates."""
    c = cfg3(n=(10, 9, 8), dx=(0.2, 0.3, 0.25), frac=0.9)
    E = RNG.normal(size=(3,) + c.shape)
    B = RNG.normal(size=(3,) + c.shape)
    s = O.State(c, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), E, B)

    def inv():
        cE = O.curl_e(c, s.E)
        bm = s.B + 0.5 * c.dt * cE
        bp = s.B - 0.5 * c.dt * cE
        return np.sum(s.E ** 2) + np.sum(bm * bp)

    i0 = inv()
    for _ in range(100):
        s.field_advance()
    assert abs(inv() - i0) < 1e-12 * abs(i0)


def test_curl_identities():
    """D.(C^T B) = 0, C(G phi) = 0 and <C E, B> = <E, C^T B> on the periodic
    Yee grid."""
    c = cfg3(n=(7, 6, 5), dx=(0.2, 0.3, 0.25))
    E = RNG.normal(size=(3,) + c.shape)
    B = RNG.normal(size=(3,) + c.shape)
    np.testing.assert_allclose(O.divergence(c, O.curl_b(c, B)), 0.0, atol=1e-11)
    phi = RNG.normal(size=c.shape)
    G = np.stack([(np.roll(phi, -1, axis=2 - d) - phi) / c.dx[d] for d in range(3)])
    np.testing.assert_allclose(O.curl_e(c, G), 0.0, atol=1e-11)
    lhs = np.sum(O.curl_e(c, E) * B)
    rhs = np.sum(E * O.curl_b(c, B))
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_mur_exact_at_magic_time_step():
    """At c dt = dy the 1D Yee scheme transports exactly and Mur-1 reduces to
    F0^{n+1} = F1^n, so a pulse leaves through the open faces leaving only
    round-off behind (fields uniform along a periodic x)."""
    ny, dy = 80, 0.2
    c = O.Config(2, (4, ny, 1), (1.0e6, dy, 1.0), dy, 1, (0, 1, 0))
    j = np.arange(ny)
    prof = lambda y: np.exp(-((y - 8.0) / 1.2) ** 2)  # noqa: E731
    E = c.zeros_field()
    B = c.zeros_field()
    # E_x (node along y) and B_z (half-way along y) of a pulse moving in -y,
    # B given at -dt/2 and brought to t = 0 with the solver's own half step
    y_e, y_b = j * dy, (j + 0.5) * dy
    E[0, 0] = prof(y_e)[None, :, None].repeat(4, axis=2)[0]
    B[2, 0] = (prof(y_b - c.dt / 2))[None, :, None].repeat(4, axis=2)[0]
    B[2, 0, ny - 1] = 0.0
    B -= 0.5 * c.dt * O.curl_e(c, E)
    s = O.State(c, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), E, B)
    w0 = s.energies()[0]
    for _ in range(2 * ny):
        s.field_advance()
    assert s.energies()[0] < 1e-24 * max(w0, 1.0) + 1e-26


def test_mur_absorbs_at_half_courant():
    """At half the Courant limit Mur-1 still absorbs a well-resolved normally
    incident pulse: less than 1e-3 of its energy stays in the box."""
    ny, dy = 200, 0.2
    c = O.Config(2, (4, ny, 1), (1.0e6, dy, 1.0), 0.5 * dy, 1, (0, 1, 0))
    j = np.arange(ny)
    prof = lambda y: np.exp(-((y - 20.0) / 3.0) ** 2)  # noqa: E731
    E = c.zeros_field()
    B = c.zeros_field()
    E[0, 0] = np.tile(prof(j * dy)[:, None], (1, 4))
    bz = prof((j + 0.5) * dy - c.dt / 2)
    bz[ny - 1] = 0.0
    B[2, 0] = np.tile(bz[:, None], (1, 4))
    B -= 0.5 * c.dt * O.curl_e(c, E)
    s = O.State(c, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), E, B)
    w0 = s.energies()[0]
    for _ in range(int(2.5 * 20.0 / c.dt)):
        s.field_advance()
    assert s.energies()[0] < 1e-3 * w0


def test_mur_absorbs_at_the_edges_of_two_open_faces():
    """3D, y and z open (x periodic): an E_x pulse (uniform in x, so
    divergence free, B = 0 at t = 0) splits into two packets that run along
    the (y+z) diagonal into the two y-z edges of the box, where every E_x
    sample lies on two open faces.  At half the Courant limit first-order
    Mur absorbs them: after both packets have crossed the edges, less than
    2e-3 of the energy is left (without an update of the edge samples they
    stay at zero and reflect about 2e-2)."""
    ny = nz = 48
    d = 0.2
    c = cfg3(n=(4, ny, nz), dx=(d, d, d), order=1, bc=(0, OPEN_, OPEN_))
    k, j, _ = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(4), indexing="ij")
    yc = zc = (ny - 1) * d / 2
    xi = ((j * d - yc) + (k * d - zc)) / math.sqrt(2)
    eta = ((k * d - zc) - (j * d - yc)) / math.sqrt(2)
    E = c.zeros_field()
    E[0] = np.exp(-(xi / 0.6) ** 2 - (eta / 1.0) ** 2)
    s = O.State(c, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), E, c.zeros_field())
    w0 = s.energies()[0]
    for _ in range(int(15.0 / c.dt)):
        s.field_advance()
    assert s.energies()[0] < 2e-3 * w0


# ---------------------------------------------------------------- deposit
def _random_paths(c, m, maxmove=0.45):
    D = c.dims
    X0 = np.zeros((m, 3))
    n = np.array(c.n, dtype=float)
    X0[:, :D] = RNG.uniform(2.0, n[:D] - 3.0, size=(m, D))
    X1 = X0.copy()
    X1[:, :D] += RNG.uniform(-maxmove, maxmove, size=(m, D))
    return X0, X1


def _rho_of(c, X, q):
    s = O.State(c, X, np.zeros_like(X), q, c.zeros_field(), c.zeros_field())
    return s.rho()


@pytest.mark.parametrize("dims", [2, 3])
@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_deposit_discrete_continuity(dims, order):
    """(rho(X1) - rho(X0))/dt + D.J = 0 node by node, for paths that cross
    0, 1, 2 or 3 stencil-switch planes (the reason for the split)."""
    c = cfg3(n=(10, 9, 8), order=order) if dims == 3 else cfg2(n=(10, 9), order=order)
    X0, X1 = _random_paths(c, 200)
    q = RNG.uniform(-1.0, 1.0, size=200)
    J = O.deposit_paths(c, X0, X1, q, vz=RNG.normal(size=200))
    r = O.continuity_residual(c, _rho_of(c, X0, q), _rho_of(c, X1, q), J)
    scale = np.abs(_rho_of(c, X1, q) - _rho_of(c, X0, q)).max() / c.dt
    assert np.abs(r).max() < 1e-12 * scale


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_deposit_total_current_and_antisymmetry(order):
    """Summed over the grid, J_d = q dx_d (X1-X0)_d / dt (the current of a
    point charge); swapping the ends negates J."""
    c = cfg3(n=(10, 9, 8), order=order, dx=(0.1, 0.2, 0.3))
    X0, X1 = _random_paths(c, 1)
    q = -0.37
    J = O.deposit_paths(c, X0, X1, q)
    for d in range(3):
        assert abs(J[d].sum() - q * c.dx[d] * (X1[0, d] - X0[0, d]) / c.dt) < 1e-12
    Jr = O.deposit_paths(c, X1, X0, q)
    np.testing.assert_allclose(J, -Jr, atol=1e-13)


def test_deposit_linear_equals_path_integral():
    """Order 1: the split deposit equals the exact charge flux of the unit
    cloud: J_x(i+1/2, j, k) = q dx/dt * integral over the path of
    dX_x 1[X_x in (i, i+1)] hat(X_y - j) hat(X_z - k) (midpoint quadrature)."""
    c = cfg3(n=(10, 9, 8), order=1)
    hat = lambda t: np.maximum(0.0, 1.0 - np.abs(t))  # noqa: E731
    for _ in range(6):
        X0, X1 = _random_paths(c, 1, maxmove=0.9)
        q = 0.8
        J = O.deposit_paths(c, X0, X1, q)
        M = 200000
        t = (np.arange(M) + 0.5) / M
        P = X0[0] + t[:, None] * (X1[0] - X0[0])
        dP = (X1[0] - X0[0]) / M
        for comp in range(3):
            a, b = (comp + 1) % 3, (comp + 2) % 3
            ref = np.zeros(c.shape)
            cell = np.floor(P[:, comp]).astype(int)
            for ja in range(int(P[:, a].min()) - 1, int(P[:, a].max()) + 3):
                for jb in range(int(P[:, b].min()) - 1, int(P[:, b].max()) + 3):
                    wgt = hat(P[:, a] - ja) * hat(P[:, b] - jb) * dP[comp]
                    for ic in np.unique(cell):
                        val = q * c.dx[comp] / c.dt * wgt[cell == ic].sum()
                        L = [0, 0, 0]
                        L[comp], L[a], L[b] = ic, ja, jb
                        ref[L[2] % 8, L[1] % 9, L[0] % 10] += val
            np.testing.assert_allclose(J[comp], ref, atol=2e-5 * np.abs(ref).max())


def test_deposit_1d_motion_unique_current():
    """Motion along x only: J_x is the unique flux of the 1D shape,
    J_x(i+1/2) = -q dx/dt sum_{i'<=i} (S(X1) - S(X0))_{i'} times the fixed
    transverse weights; J_y = J_z = 0."""
    for order in (1, 2, 3):
        c = cfg3(n=(12, 9, 8), order=order)
        X0 = np.array([[5.3, 4.6, 3.2]])
        for dxm in (0.41, -0.33, 0.05):
            X1 = X0 + np.array([[dxm, 0, 0]])
            J = O.deposit_paths(c, X0, X1, 1.0)
            S = np.zeros(16)
            for X, sgn in ((X1[0, 0], 1), (X0[0, 0], -1)):
                b, w = O.shape(order, X)
                S[b:b + order + 1] += sgn * w
            flux = -c.dx[0] / c.dt * np.cumsum(S)
            by, wy = O.shape(order, 4.6)
            bz, wz = O.shape(order, 3.2)
            ref = np.zeros(c.shape)
            for jy in range(order + 1):
                for kz in range(order + 1):
                    ref[bz + kz, by + jy, :12] = flux[:12] * wy[jy] * wz[kz]
            np.testing.assert_allclose(J[0], ref, atol=1e-12)
            assert np.abs(J[1]).max() < 1e-13 and np.abs(J[2]).max() < 1e-13


def test_deposit_2d_out_of_plane_current():
    """2D3V: a particle at rest in the plane with velocity v_z deposits
    J_z = q v_z S_x S_y (its charge times v_z); in-plane motion keeps the
    total sum J_z = q v_z."""
    c = cfg2(n=(12, 10), order=2)
    X = np.array([[4.3, 5.8, 0.0]])
    J = O.deposit_paths(c, X, X, 0.5, vz=0.7)
    assert abs(J[2].sum() - 0.35) < 1e-14
    np.testing.assert_allclose(J[2], 0.35 * _rho_of(c, X, np.array([1.0])), atol=1e-14)
    X1 = X + np.array([[0.4, -0.3, 0.0]])
    J = O.deposit_paths(c, X, X1, 0.5, vz=0.7)
    assert abs(J[2].sum() - 0.35) < 1e-14


def _hat_integral_2d(X0, X1, i, j):
    """Exact integral over t in [0, 1] of hat(x(t) - i) hat(y(t) - j) along the
    straight path X0 -> X1: between the crossings of integer planes each hat
    is linear in t, so the product is quadratic and Simpson's rule on every
    such piece is exact."""
    cuts = [0.0, 1.0]
    for d in range(2):
        a, b = X0[d], X1[d]
        if b != a:
            for m in range(int(np.floor(min(a, b))) + 1, int(np.ceil(max(a, b)))):
                t = (m - a) / (b - a)
                if 0.0 < t < 1.0:
                    cuts.append(t)
    cuts = np.sort(np.array(cuts))
    hat = lambda v: max(0.0, 1.0 - abs(v))  # noqa: E731

    def f(t):
        return hat(X0[0] + t * (X1[0] - X0[0]) - i) * hat(X0[1] + t * (X1[1] - X0[1]) - j)

    tot = 0.0
    for ta, tb in zip(cuts[:-1], cuts[1:]):
        tot += (tb - ta) / 6.0 * (f(ta) + 4.0 * f(0.5 * (ta + tb)) + f(tb))
    return tot


def test_deposit_2d_out_of_plane_current_is_the_time_integral_at_order_1():
    """2D3V, order 1: the charge-conserving J_z of a path is the exact time
    average of the particle's charge cloud times q v_z,
    J_z(i, j) = q v_z * integral_0^1 hat(x(t) - i) hat(y(t) - j) dt,
    on paths inside one cell and on paths that cross one or two cell faces
    (virtual segments, Sec. 5.2).  Pins the 1/2 S0 dS and 1/3 dS dS cross
    terms of the out-of-plane deposit, which the at-rest case cannot see."""
    c = cfg2(n=(12, 10), order=1)
    ncross = 0
    for trial in range(40):
        X0 = np.zeros((1, 3))
        X0[0, :2] = RNG.uniform(3.0, 7.0, size=2)
        X1 = X0.copy()
        X1[0, :2] += RNG.uniform(-0.45, 0.45, size=2)
        if trial < 6:  # paths inside one cell
            X1[0, :2] = np.floor(X0[0, :2]) + RNG.uniform(0.0, 1.0, size=2)
        ncross += int(np.any(np.floor(X0[0, :2]) != np.floor(X1[0, :2])))
        q, vz = RNG.uniform(-1.0, 1.0), RNG.normal()
        J = O.deposit_paths(c, X0, X1, q, vz=vz)
        ref = np.zeros(c.shape[1:])
        lo = np.floor(np.minimum(X0[0], X1[0])).astype(int)
        for j in range(lo[1], lo[1] + 3):
            for i in range(lo[0], lo[0] + 3):
                ref[j, i] = q * vz * _hat_integral_2d(X0[0], X1[0], i, j)
        np.testing.assert_allclose(J[2, 0], ref, rtol=0, atol=1e-14 * max(1.0, abs(q * vz)))
    assert ncross >= 8


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_deposit_2d_out_of_plane_current_moments(order):
    """2D3V at every order: with the time-linear shape of each virtual
    segment the out-of-plane current carries the path's moments exactly.
    B-spline weights have unit mass and first moment equal to the position,
    so sum J_z = q v_z, sum i J_z = q v_z (x0 + x1)/2 (likewise in y) and
    sum i j J_z = q v_z * integral_0^1 x(t) y(t) dt
    = q v_z (x0 y0 + (dx y0 + x0 dy)/2 + dx dy / 3) for the straight path."""
    c = cfg2(n=(20, 18), order=order)
    ii, jj = np.meshgrid(np.arange(20), np.arange(18), indexing="xy")
    for _ in range(30):
        X0 = np.zeros((1, 3))
        X0[0, :2] = RNG.uniform(6.0, 11.0, size=2)
        X1 = X0.copy()
        X1[0, :2] += RNG.uniform(-0.45, 0.45, size=2)
        q, vz = RNG.uniform(0.2, 1.0), RNG.uniform(0.2, 1.0)
        Jz = O.deposit_paths(c, X0, X1, q, vz=vz)[2, 0]
        (x0, y0), (x1, y1) = X0[0, :2], X1[0, :2]
        dxp, dyp = x1 - x0, y1 - y0
        qv = q * vz
        assert abs(Jz.sum() - qv) < 1e-13
        assert abs((ii * Jz).sum() - qv * 0.5 * (x0 + x1)) < 1e-12
        assert abs((jj * Jz).sum() - qv * 0.5 * (y0 + y1)) < 1e-12
        xy = x0 * y0 + 0.5 * (dxp * y0 + x0 * dyp) + dxp * dyp / 3.0
        assert abs((ii * jj * Jz).sum() - qv * xy) < 1e-11


# ---------------------------------------------------------------- whole step
def _thermal_state(w, quiet=False):
    pl = I.make_plasma(w, quiet=quiet)
    E, B = I.laser_fields(w)
    c = O.Config(w.dims, w.n3, w.dx3, w.dt, w.order, w.bc3)
    return c, O.State(c, pl.global_positions(w), pl.u.T.astype(np.float64), pl.charges(), E, B)


@pytest.mark.parametrize("dims,order,bc", [(2, 1, (0, 0)), (2, 2, (0, 1)), (3, 2, (0, 0, 0)),
                                           (3, 3, (0, 1, 1)), (3, 1, (1, 0, 1)), (2, 4, (0, 1)),
                                           (3, 4, (0, 0, 1))])
def test_step_continuity_and_gauss(dims, order, bc):
    """Whole steps: discrete continuity holds to round-off at every interior
    node, hence Gauss's law D.E - rho keeps its initial value."""
    if dims == 2:
        w = I.Workload("t", 2, (20, 18), (0.2, 0.25), order, 4, 0.3, 1, bc=bc, seed=7)
    else:
        w = I.Workload("t", 3, (10, 9, 8), (0.2, 0.25, 0.3), order, 2, 0.3, 1, bc=bc, seed=8)
    c, s = _thermal_state(w)
    mask = O.interior_mask(c)
    g0 = O.divergence(c, s.E) - s.rho()
    for _ in range(8):
        r0 = s.rho()
        s.step(1)
        r1 = s.rho()
        res = O.continuity_residual(c, r0, r1, s.J)
        assert np.abs(res[mask]).max() < 1e-11 * (np.abs(r1 - r0).max() / c.dt)
    g = O.divergence(c, s.E) - s.rho() - g0
    assert np.abs(g[mask]).max() < 1e-11 * np.abs(s.rho()).max()


def test_cold_plasma_oscillation_frequency():
    """Cold plasma, u_x = d sin(k x) with d = 1e-3, k = 2 pi / L_x: the
    projection of E_x on sin(k x) oscillates at omega_p = 1 (within 0.5 %)
    with amplitude d omega_p (within 1 %) (regular 2x2 start)."""
    w = I.WORKLOADS["w2d_64_linear"].with_(u_th=0.0)
    c, s = _thermal_state(w, quiet=True)
    L = w.n[0] * w.dx[0]
    k = 2 * np.pi / L
    d = 1e-3
    s.u[:, 0] = d * np.sin(k * s.X[:, 0] * w.dx[0])
    x_e = (np.arange(w.n[0]) + 0.5) * w.dx[0]
    basis = np.sin(k * x_e)
    ts, amps = [], []
    for n in range(w.steps):
        s.step(1)
        ts.append((n + 1) * c.dt)
        amps.append(2 * np.mean(s.E[0, 0] * basis[None, :]))
    from scipy.optimize import curve_fit
    ts, amps = np.array(ts), np.array(amps)
    f = lambda t, A, om, ph: A * np.sin(om * t + ph)  # noqa: E731
    (A, om, ph), _ = curve_fit(f, ts, amps, p0=(d, 1.0, 0.0))
    assert abs(om - 1.0) < 5e-3
    assert abs(abs(A) - d) < 1e-2 * d


def test_threads_match_serial():
    """The shared-memory mode (private current grids + reduction) gives the
    serial result up to summation order."""
    w = I.Workload("t", 3, (12, 10, 8), (0.2, 0.2, 0.2), 2, 4, 0.2, 3, seed=11)
    _, a = _thermal_state(w)
    b = a.copy()
    a.step(3, nthreads=1)
    b.step(3, nthreads=4)
    np.testing.assert_allclose(a.X, b.X, rtol=0, atol=1e-12)
    np.testing.assert_allclose(a.E, b.E, rtol=0, atol=1e-12)


def test_jvp_matches_central_differences():
    """The dual-number JVP of several full steps equals central finite
    differences of the FP64 oracle along the same direction."""
    w = I.Workload("t", 2, (16, 12), (0.2, 0.2), 2, 4, 0.3, 4, bc=(0, 1),
                   laser=I.Laser(a0=0.5, omega0=3.0, waist=1.0, tau=0.5, x_center=1.5), seed=5)
    c, s0 = _thermal_state(w)
    dX = np.zeros_like(s0.X)
    du = RNG.choice([-1.0, 1.0], size=s0.u.shape)
    dE = s0.E / 0.5
    dB = s0.B / 0.5
    a = s0.copy()
    _, duo, dEo, dBo, _ = a.step_jvp(w.steps, dX, du, dE, dB)
    h = 1e-6
    p, m = s0.copy(), s0.copy()
    p.u += h * du
    p.E += h * dE
    p.B += h * dB
    m.u -= h * du
    m.E -= h * dE
    m.B -= h * dB
    p.step(w.steps)
    m.step(w.steps)
    fd_E = (p.E - m.E) / (2 * h)
    fd_u = (p.u - m.u) / (2 * h)
    assert np.abs(dEo - fd_E).max() < 1e-6 * np.abs(fd_E).max()
    assert np.abs(duo - fd_u).max() < 1e-6 * np.abs(fd_u).max()


# ---------------------------------------------------------------- mobile ions
def _two_species(w, M, quiet=True):
    """Electrons and ions (q/m = +1/M) of workload w in its fields."""
    wi = w.with_(ions=I.Ions(mass_ratio=M))
    pe, pi = I.make_plasma(w, quiet=quiet), I.make_ions(wi, quiet=quiet)
    E, B = I.laser_fields(w)
    c = O.Config(w.dims, w.n3, w.dx3, w.dt, w.order, w.bc3)
    e = O.Species(-1.0, pe.global_positions(w), pe.u.T.astype(np.float64), pe.charges())
    i = O.Species(1.0 / M, pi.global_positions(wi), pi.u.T.astype(np.float64), pi.charges())
    return c, O.MultiState(c, [e, i], E, B)


def test_two_species_cold_plasma_frequency():
    """Cold electrons and ions of mass ratio M = 4 on the same quiet lattice
    (rho = 0), electrons kicked with u_x = d sin(k x): the longitudinal mode
    of cold two-fluid theory oscillates at omega^2 = omega_pe^2 + omega_pi^2
    = 1 + 1/M (within 0.5 %), and the ions move against the electrons with
    1/M of their momentum change per unit charge."""
    M = 4.0
    w = I.WORKLOADS["w2d_64_linear"].with_(u_th=0.0)
    c, s = _two_species(w, M)
    e, i = s.species
    k = 2 * np.pi / (w.n[0] * w.dx[0])
    d = 1e-3
    e.u[:, 0] = d * np.sin(k * e.X[:, 0] * w.dx[0])
    x_e = (np.arange(w.n[0]) + 0.5) * w.dx[0]
    basis = np.sin(k * x_e)
    ts, amps = [], []
    for n in range(w.steps):
        s.step(1)
        ts.append((n + 1) * c.dt)
        amps.append(2 * np.mean(s.E[0, 0] * basis[None, :]))
    from scipy.optimize import curve_fit
    f = lambda t, A, om, ph: A * np.sin(om * t + ph)  # noqa: E731
    (A, om, ph), _ = curve_fit(f, np.array(ts), np.array(amps), p0=(d, 1.1, 0.0))
    assert abs(om / np.sqrt(1.0 + 1.0 / M) - 1.0) < 5e-3
    # the ion response: du_i/dt = E/M, du_e/dt = -E, so d(u_e + M u_i)/dt = 0
    xs = e.X[:, 0] * w.dx[0]
    pe_ = 2 * np.mean(e.u[:, 0] * np.sin(k * xs))
    pi_ = 2 * np.mean(i.u[:, 0] * np.sin(k * i.X[:, 0] * w.dx[0]))
    assert abs((pe_ + M * pi_) - d) < 2e-2 * d


def test_two_species_energy_uses_the_mass():
    """Kinetic energy sums (q / (q/m)) (gamma - 1): over the two-species
    oscillation field + kinetic energy stays within 1 % of its initial value
    at dt = 0.1 x Courant (the diagnostic pairs u^{n-1/2} with E^n, an
    O(omega dt) offset; weighting the ions by |q| instead of their mass
    would be ~20 % off)."""
    M = 4.0
    w = I.WORKLOADS["w2d_64_linear"].with_(u_th=0.0, courant_fraction=0.1)
    c, s = _two_species(w, M)
    e, _ = s.species
    k = 2 * np.pi / (w.n[0] * w.dx[0])
    e.u[:, 0] = 1e-2 * np.sin(k * e.X[:, 0] * w.dx[0])
    wf0, wk0 = s.energies()
    W0 = wf0 + wk0
    dev = 0.0
    for _ in range(300):
        s.step(1)
        wf, wk = s.energies()
        dev = max(dev, abs(wf + wk - W0))
    assert dev < 1e-2 * W0


def test_ion_kick_in_uniform_field():
    """A zero-weight ion (q = 0, so no self field) of q/m = Z/M in a uniform
    E: one Boris step changes u by exactly (q/m) E dt."""
    c = cfg2(n=(8, 8), order=2)
    E = np.zeros((3,) + c.shape)
    E[0] = 0.3
    E[1] = -0.7
    B = np.zeros_like(E)
    qm = 2.0 / 7.0
    sp = O.Species(qm, np.array([[3.3, 4.6, 0.0]]), np.zeros((1, 3)), np.zeros(1))
    s = O.MultiState(c, [sp], E, B)
    s.step(1)
    np.testing.assert_allclose(sp.u[0], [qm * 0.3 * c.dt, -qm * 0.7 * c.dt, 0.0], rtol=1e-14)


@pytest.mark.parametrize("dims", [2, 3])
def test_two_species_continuity_and_gauss(dims):
    """Thermal electrons and ions: the total current (sum of the species'
    currents) satisfies discrete continuity with the total charge density at
    every interior node, and Gauss's law keeps its initial residual."""
    if dims == 2:
        w = I.Workload("t", 2, (20, 18), (0.2, 0.25), 2, 4, 0.3, 1, bc=(0, 1), seed=17)
    else:
        w = I.Workload("t", 3, (10, 9, 8), (0.2, 0.25, 0.3), 3, 2, 0.3, 1, bc=(0, 0, 1), seed=18)
    w = w.with_(ions=I.Ions(mass_ratio=9.0, u_th=0.1))
    wi = w
    pe, pi = I.make_plasma(w), I.make_ions(wi)
    E, B = I.laser_fields(w)
    c = O.Config(w.dims, w.n3, w.dx3, w.dt, w.order, w.bc3)
    s = O.MultiState(c, [O.Species(-1.0, pe.global_positions(w), pe.u.T, pe.charges()),
                         O.Species(1.0 / 9.0, pi.global_positions(w), pi.u.T, pi.charges())], E, B)
    mask = O.interior_mask(c)
    g0 = O.divergence(c, s.E) - s.rho()
    for _ in range(6):
        r0 = s.rho()
        s.step(1)
        r1 = s.rho()
        res = O.continuity_residual(c, r0, r1, s.J)
        assert np.abs(res[mask]).max() < 1e-11 * (np.abs(r1 - r0).max() / c.dt)
    g = O.divergence(c, s.E) - s.rho() - g0
    assert np.abs(g[mask]).max() < 1e-11 * np.abs(s.rho()).max() + 1e-13



def test_kinetic_energy_limits():
    """W_kin = sum m_p dV (gamma - 1): exactly zero for a cold plasma, and
    for slow particles the series gamma - 1 = u^2/2 - u^4/8 + O(u^6): the
    Newtonian 1/2 sum m_p u^2 dV plus its first relativistic correction
    (u ~ 1e-3: the next term is 1e-12 relative); m_p = |q_p| / |q/m|."""
    c = cfg2(n=(8, 8), order=2)
    m = 500
    X = np.zeros((m, 3))
    X[:, :2] = RNG.uniform(0.0, 8.0, size=(m, 2))
    q = -RNG.uniform(0.1, 1.0, size=m)
    dV = c.dx[0] * c.dx[1]
    s = O.State(c, X, np.zeros((m, 3)), q, c.zeros_field(), c.zeros_field())
    assert s.energies()[1] == 0.0
    u = RNG.normal(0.0, 1e-3, size=(m, 3))
    s = O.State(c, X, u, q, c.zeros_field(), c.zeros_field())
    u2 = np.sum(u ** 2, axis=1)
    newton = dV * np.sum(np.abs(q) * (0.5 * u2 - 0.125 * u2 ** 2))
    assert abs(s.energies()[1] / newton - 1.0) < 1e-8
    # ions (q/m = 1/M) weigh M times their charge
    ci = O.Config(c.dims, c.n, c.dx, c.dt, c.order, c.bc, q_over_m=1.0 / 25.0)
    si = O.State(ci, X, u, -q, c.zeros_field(), c.zeros_field())
    assert abs(si.energies()[1] / (25.0 * newton) - 1.0) < 1e-8


# ---------------------------------------------------------------- moving window, antenna
def test_discrete_poynting_identity_with_antenna():
    """With B kept at integer times by two half steps, W~ = 1/2 (|E|^2 + |B|^2)
    - dt^2/8 |C E|^2 (times dV) changes over a step by exactly
    -dt/2 <J^{n+1/2}, E^n + E^{n+1}> dV (periodic grid): the antenna's current
    enters the E update with the right sign and scale."""
    c = cfg2(n=(40, 24), dx=(0.1, 0.2), order=2)
    a = O.Antenna(x_index=10, polarization=1, a0=0.7, omega0=5.0, waist=1.5, tau=0.6,
                  t_center=1.0, y_center=2.4)
    E = 0.01 * RNG.normal(size=(3,) + c.shape)
    B = 0.01 * RNG.normal(size=(3,) + c.shape)
    s = O.State(c, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), E, B)
    s.antenna = a
    dV = c.dx[0] * c.dx[1]

    def wt(st):
        ce = O.curl_e(c, st.E)
        return 0.5 * dV * (np.sum(st.E ** 2) + np.sum(st.B ** 2)) - c.dt ** 2 / 8 * dV * np.sum(ce ** 2)

    for _ in range(30):
        E0, w0 = s.E.copy(), wt(s)
        s.step(1)
        work = -0.5 * c.dt * dV * np.sum(s.J * (E0 + s.E))
        assert abs(wt(s) - w0 - work) < 1e-12 * (abs(w0) + abs(work) + 1e-30)
    assert np.abs(s.J).max() > 0


def test_antenna_emits_the_requested_field():
    """A uniform current sheet (quasi-1D: periodic y, huge waist) at small
    k dx radiates a0 omega0 env(t - r) cos(omega0 (t - r - t_c)) on both sides
    (a sheet current K gives E = -K/2): the field seen 30 cells from the
    antenna peaks at a0 omega0 within 1 %."""
    n0 = 400
    c = O.Config(2, (n0, 4, 1), (0.05, 0.2, 1.0), 0.5 * 0.05, 2, (OPEN_, 0, 0))
    a = O.Antenna(x_index=200, polarization=1, a0=0.3, omega0=2.0, waist=1e9, tau=2.0,
                  t_center=6.0, y_center=0.0)
    s = O.State(c, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), c.zeros_field(),
                c.zeros_field())
    s.antenna = a
    probe = 230
    trace = []
    for _ in range(int(14.0 / c.dt)):
        s.step(1)
        trace.append(s.E[1, 0, 0, probe])
    peak = np.max(np.abs(trace))
    assert abs(peak / (a.a0 * a.omega0) - 1.0) < 1e-2


def test_antenna_field_sign_and_phase():
    """The signed field of the antenna: at distance r on either side the
    sheet's field is E_y(t) = a0 omega0 env(t - r) cos(omega0 (t - r - t_c))
    (E = -K/2 with K = -2 a0 omega0 env cos), sample by sample within 1 % of
    the peak (a current of the opposite sign would be off by twice the peak)."""
    n0 = 400
    c = O.Config(2, (n0, 4, 1), (0.05, 0.2, 1.0), 0.5 * 0.05, 2, (OPEN_, 0, 0))
    a = O.Antenna(x_index=200, polarization=1, a0=0.3, omega0=2.0, waist=1e9, tau=2.0,
                  t_center=6.0, y_center=0.0)
    s = O.State(c, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), c.zeros_field(),
                c.zeros_field())
    s.antenna = a
    probes = (230, 170)
    traces = {p: [] for p in probes}
    ts = []
    for n in range(int(14.0 / c.dt)):
        s.step(1)
        ts.append((n + 1) * c.dt)
        for p in probes:
            traces[p].append(s.E[1, 0, 0, p])
    ts = np.array(ts)
    amp = a.a0 * a.omega0
    for p in probes:
        tr = ts - abs(p - a.x_index) * c.dx[0] - a.t_center
        ref = amp * np.exp(-tr ** 2 / a.tau ** 2) * np.cos(a.omega0 * tr) * (np.abs(tr) <= 3 * a.tau)
        assert np.abs(np.array(traces[p]) - ref).max() < 1e-2 * amp


@pytest.mark.parametrize("dims", [2, 3])
def test_window_shift_moves_fields_and_particles_together(dims):
    """After one window shift the Gauss residual D.E - rho at node i equals
    its value at node i+1 before (fields and particles moved by exactly one
    cell), and every surviving particle moved by exactly -1 in x."""
    if dims == 2:
        w = I.Workload("t", 2, (24, 12), (0.1, 0.2), 2, 4, 0.2, 1, bc=(1, 0), seed=21)
    else:
        w = I.Workload("t", 3, (16, 8, 6), (0.1, 0.2, 0.2), 3, 2, 0.2, 1, bc=(1, 0, 0), seed=22)
    c, s = _thermal_state(w)
    s.E += 0.01 * RNG.normal(size=s.E.shape)
    s.step(2)
    g0 = O.divergence(c, s.E) - s.rho()
    X0, alive0 = s.X.copy(), s.alive.copy()
    O.window_shift(s)
    g1 = O.divergence(c, s.E) - s.rho()
    # away from the faces (absorbed particles at the back still reached
    # order/2 + 1 node planes; the front plane of E is new)
    m = 2 + w.order // 2
    np.testing.assert_allclose(g1[..., m:-m], g0[..., m + 1:-m + 1], atol=1e-13)
    keep = (alive0 > 0) & (X0[:, 0] >= 1.0)
    np.testing.assert_array_equal(s.X[keep, 0], X0[keep, 0] - 1.0)
    assert np.all(s.alive[(alive0 > 0) & (X0[:, 0] < 1.0)] == 0)


def test_window_keeps_a_pulse_at_the_yee_group_velocity():
    """A quasi-1D laser pulse in vacuum with the window moving one cell per
    dx of light travel: in the lab frame (window position + shifts) the
    pulse centroid moves at the Yee group velocity v_g = cos(k dx/2) /
    cos(omega dt/2) (sin(omega dt/2)/dt = sin(k dx/2)/dx), within 2e-3."""
    n0, dx = 300, 0.1
    lz = I.Laser(a0=0.1, omega0=10.0, waist=1e9, tau=1.5, x_center=15.0)
    w = I.Workload("t", 2, (n0, 4), (dx, 0.2), 2, 1, 0.0, 1, bc=(1, 0), laser=lz)
    E, B = I.laser_fields(w)
    c = O.Config(2, w.n3, w.dx3, w.dt, 2, w.bc3)
    s = O.State(c, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0), E, B)
    x = np.arange(n0) * dx

    def centroid():
        e2 = s.E[1, 0, 0] ** 2
        return np.sum(x * e2) / np.sum(e2)

    shifts, ts, cs = 0, [], []
    steps = int(8.0 / c.dt)
    for n in range(1, steps + 1):
        s.step(1)
        while (shifts + 1) * dx <= n * c.dt:  # the window follows light
            O.window_shift(s)
            shifts += 1
        ts.append(n * c.dt)
        cs.append(centroid() + shifts * dx)
    vg = np.polyfit(ts[len(ts) // 4:], cs[len(cs) // 4:], 1)[0]
    k = lz.omega0
    om = 2 / c.dt * np.arcsin(c.dt / dx * np.sin(k * dx / 2))
    vg_yee = np.cos(k * dx / 2) / np.cos(om * c.dt / 2)
    assert abs(vg - vg_yee) < 2e-3
    assert abs(vg_yee - 1.0) > 1e-2  # the check can tell v_g from c
