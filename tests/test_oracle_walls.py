"""Pins of the oracle's wall layers against closed forms and exact balances.

The paper closes its boxes (section 3) without describing how the walls are
imposed.  The reading taken is an immobile (or tangentially moving) solid slab
treated by the same site rule as a particle: every wall site takes f^eq(rho,
U_wall) with its own post-collision density.  On a closed axis of n sites,
layers 2 .. n-3 are fluid.  These tests pin that reading:
  - plane Poiseuille flow: the fluid profile is exactly parabolic with
    curvature -f/(2 nu), nu = (tau - 1/2)/3 (eq. 4), for every tau, and at
    tau = 1 it equals a closed form derived by hand from the propagation
    rule (below);
  - plane Couette flow: the fluid profile is exactly linear, and at tau = 1
    it passes through the wall velocity at the BS layers;
  - the walls absorb exactly the injected momentum at steady state, and the
    per-step momentum bookkeeping closes with the wall exchange included;
  - particle-wall hard-core contact reverses the normal velocity;
  - no particle ever owns a wall site.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import Oracle

EPS = np.finfo(np.float64).eps


def _channel(q, n, tau, fb=(0, 0, 0), wall_velocity=None):
    """A channel closed along y (D2Q9) or z (D3Q19), 3 sites across the
    other axes, flow along x."""
    axis = 1 if q == 9 else 2
    box = (3, n, 1) if q == 9 else (3, 3, n)
    wu = None
    if wall_velocity is not None:
        wu = np.zeros((3, 2, 3))
        wu[axis, 0, 0], wu[axis, 1, 0] = wall_velocity
    return Oracle(q, *box, tau, body_force=fb, walls=1 << axis, wall_velocity=wu), axis


def _profile(o, axis):
    rho, u, _ = o.fields()
    if axis == 1:
        return rho[0, :, 1], u[0, :, 1, 0]
    return rho[:, 1, 1], u[:, 1, 1, 0]


def _run_to_steady(o, axis, chunk, max_chunks=200, tol=1e-11):
    _, prev = _profile(o, axis)
    for _ in range(max_chunks):
        o.step(chunk)
        _, u = _profile(o, axis)
        if np.abs(u - prev).max() <= tol * max(np.abs(u).max(), 1e-300):
            return u
        prev = u
    raise AssertionError("no steady state")


@pytest.mark.parametrize("q", [9, 19])
def test_poiseuille_closed_form_at_tau_one(q):
    """At tau = 1 the BGK collision returns f^eq(rho, u) plus the forcing, so
    after propagation a fluid site holds sum over the three layers
    y-1, y, y+1 of their equilibria.  For a unidirectional flow this gives
    u(y) = u(y-1)/6 + 2u(y)/3 + u(y+1)/6 + f in the bulk (weights 1/6, 2/3,
    1/6 are 3 sum w c_x^2 per layer, equal for D2Q9 and D3Q19), i.e.
    u'' = -6f.  The first fluid site (y = 2) receives from the wall's BS layer
    f^eq(rho, 0), which carries neither momentum nor the forcing share 1/6 f,
    so 2 u(2) - u(3) = 5 f.  The solution is u(y) = A - 3 f (y - c)^2 with
    c the channel centre and A = 5 f + 3 f [2 (2 - c)^2 - (3 - c)^2]."""
    n, f = 20, 1e-6
    o, axis = _channel(q, n, 1.0, fb=(f, 0, 0))
    u = _run_to_steady(o, axis, 500)
    y = np.arange(n, dtype=np.float64)
    c = (n - 1) / 2.0
    A = 5 * f + 3 * f * (2 * (2 - c) ** 2 - (3 - c) ** 2)
    exact = A - 3 * f * (y - c) ** 2
    fl = slice(2, n - 2)
    assert np.abs(u[fl] - exact[fl]).max() < 1e-10 * exact.max()
    # the no-slip plane of that parabola, c - sqrt((c - 1)^2 - 1/3), lies
    # just beyond the BS layer (y = 1.0196 for n = 20)
    assert 1.0 < c - math.sqrt(A / (3 * f)) < 1.05


@pytest.mark.parametrize("q,tau", [(9, 0.6), (9, 1.5), (19, 0.8)])
def test_poiseuille_curvature_and_force_balance(q, tau):
    """For any tau the fluid profile is a parabola with curvature -f/(2 nu)
    (the Navier-Stokes limit is exact for a parabola) and at steady state the
    walls take exactly the momentum the body force injects into the box."""
    n, f = 20, 1e-6
    nu = (tau - 0.5) / 3.0
    o, axis = _channel(q, n, tau, fb=(f, 0, 0))
    u = _run_to_steady(o, axis, 2000)
    y = np.arange(n, dtype=np.float64)
    fl = slice(2, n - 2)
    cf = np.polyfit(y[fl], u[fl], 2)
    assert abs(cf[0] / (-f / (2 * nu)) - 1) < 1e-8
    resid = u[fl] - np.polyval(cf, y[fl])
    assert np.abs(resid).max() < 1e-9 * u.max()
    assert np.abs(u - u[::-1]).max() < 1e-12 * u.max()  # mirror symmetry
    d = o.diagnostics()
    assert abs(d["wall_momentum"][0] / (-o.N * f) - 1) < 1e-8
    # the fitted no-slip planes lie between the IS layer and the first fluid layer
    r = np.sort(np.roots(cf).real)
    assert 0.0 <= r[0] <= 2.0 and abs(r[0] + r[1] - (n - 1)) < 1e-6


@pytest.mark.parametrize("q,tau", [(9, 1.0), (19, 1.0), (9, 0.6)])
def test_couette_linear_profile(q, tau):
    """Walls sliding at U_lo, U_hi: the steady fluid profile is exactly
    linear.  At tau = 1 the BS layers act as fluid layers with the wall
    velocity (their equilibrium is what the bulk would have sent), so the
    line passes through (1, U_lo) and (n-2, U_hi)."""
    n = 18
    U_lo, U_hi = -0.005, 0.01
    o, axis = _channel(q, n, tau, wall_velocity=(U_lo, U_hi))
    u = _run_to_steady(o, axis, 2000)
    y = np.arange(n, dtype=np.float64)
    fl = slice(2, n - 2)
    cf = np.polyfit(y[fl], u[fl], 1)
    assert np.abs(u[fl] - np.polyval(cf, y[fl])).max() < 1e-12
    if tau == 1.0:
        exact = U_lo + (U_hi - U_lo) * (y - 1) / (n - 3)
        assert np.abs(u[fl] - exact[fl]).max() < 1e-12
    else:
        # the slip of the equilibrium wall keeps the shear below the nominal one
        assert 0 < cf[0] < (U_hi - U_lo) / (n - 4)
    # the two walls exchange equal and opposite momentum with the fluid
    assert abs(o.diagnostics()["wall_momentum"][0]) < 1e-14


def _settling_with_walls(q):
    if q == 9:
        box, axis = (48, 40, 1), 1
        x = [[12.3, 20.2, 0], [30.6, 14.9, 0], [24.1, 29.0, 0]]
        r = [4.5, 5.0, 4.0]
        g = (0.0, -2e-4, 0.0)
        V = np.pi * np.array(r) ** 2
    else:
        box, axis = (20, 20, 24), 2
        x = [[7.3, 8.1, 9.2], [13.4, 12.2, 15.6]]
        r = [3.5, 4.0]
        g = (0.0, 0.0, -2e-4)
        V = 4.0 / 3.0 * np.pi * np.array(r) ** 3
    m = 1.5 * V
    I = (0.5 if q == 9 else 0.4) * m * np.array(r) ** 2
    o = Oracle(q, *box, 0.7, gravity=g, walls=(1 << axis) | 1)
    o.add_particles(x, radius=r, mass=m, inertia=I)
    return o, np.array(m), np.array(g), V, axis


def _fluid_mass_momentum(o):
    c, _ = oracle.lattice(o.q)
    f = o.get_f().reshape(o.q, -1)
    return math.fsum(f.ravel()), np.array([math.fsum((f * c[:, a:a + 1]).ravel()) for a in range(3)])


@pytest.mark.parametrize("q", [9, 19])
def test_bookkeeping_with_walls(q):
    """Every step: fluid + particle momentum changes by the buoyancy-corrected
    weights + the IS leak + the walls' exchange; mass is conserved."""
    o, m, g, V, _ = _settling_with_walls(q)
    Fext = ((m - V)[:, None] * g).sum(axis=0)
    M0, J0 = _fluid_mass_momentum(o)
    J = J0 + (m[:, None] * o.forces()[3]).sum(axis=0)
    for t in range(1, 41):
        o.step(1)
        d = o.diagnostics()
        M, Jf = _fluid_mass_momentum(o)
        Jn = Jf + np.array([math.fsum(m * o.forces()[3][:, a]) for a in range(3)])
        expect = Fext + d["is_leak"] + d["wall_momentum"]
        assert np.abs(Jn - J - expect).max() < 8 * EPS * o.N, (t, Jn - J - expect)
        J = Jn
        assert abs(M - M0) <= 8 * EPS * o.N * t
    assert np.abs(o.diagnostics()["wall_momentum"]).max() > 1e-6


def test_particles_never_own_wall_sites():
    """A particle touching a wall: its template sites on wall layers are left
    to the wall, every other site of its template is owned as usual."""
    o = Oracle(9, 40, 30, 1, 0.8, walls=2)
    o.add_particles([[20.0, 1.0 + 6.0, 0]], radius=6.0, mass=1e30, inertia=1e30)
    own = o.fields()[2][0]
    kind = o.site_kind()[0]
    assert (own[:2] == -1).all() and (own[-2:] == -1).all() and (kind[:2] == 0).all()
    off, kd = o.template(0)
    b0 = np.floor(np.array([20.0, 7.0]) + 0.5).astype(int)
    ys = off[:, 1] + b0[1]
    assert (ys < 2).any()  # the template does reach into the wall
    mine = int((own == 0).sum())
    assert mine == int((ys >= 2).sum())


@pytest.mark.parametrize("uy,expect", [(-0.3, 0.3), (0.2, 0.2)])
def test_particle_wall_contact(uy, expect):
    """Predicted contact with the wall's BS layer while approaching reverses
    the normal velocity (the wall is an infinite mass at rest); a particle
    moving away is left alone; the tangential component is kept."""
    o = Oracle(9, 40, 30, 1, 0.8, walls=2)
    r = 4.0
    o.add_particles([[20.0, 1.0 + r + 0.2, 0]], u=[[0.05, uy, 0]], radius=r, mass=1e30, inertia=1e30)
    o.step(1)
    _, _, x, u, _ = o.forces()
    assert abs(u[0, 1] - expect) < 1e-15 and abs(u[0, 0] - 0.05) < 1e-15
    assert abs(x[0, 1] - (1.0 + r + 0.2 + expect)) < 1e-14


def test_kinematic_particle_ignores_walls():
    o = Oracle(9, 40, 30, 1, 0.8, walls=2)
    o.add_particles([[20.0, 5.2, 0]], u=[[0, -0.3, 0]], radius=4.0, mass=np.inf, inertia=np.inf)
    o.step(1)
    assert abs(o.forces()[3][0, 1] + 0.3) < 1e-15


def test_wall_parameters_rejected():
    with pytest.raises(ValueError):  # normal wall velocity
        Oracle(9, 8, 8, 1, 0.8, walls=2, wall_velocity=np.array([[0] * 6, [0, 0.1, 0, 0, 0, 0], [0] * 6]))
    with pytest.raises(ValueError):  # no fluid layer left
        Oracle(9, 8, 4, 1, 0.8, walls=2)
    with pytest.raises(ValueError):  # z walls in 2D
        Oracle(9, 8, 8, 1, 0.8, walls=4)


def test_particle_separating_from_wall_is_left_alone():
    """Overlapping the wall's BS layer while already moving away: no
    reflection (the approach test of the contact rule)."""
    o = Oracle(9, 40, 30, 1, 0.8, walls=2)
    r = 4.0
    o.add_particles([[20.0, 1.0 + r - 0.3, 0]], u=[[0, 0.1, 0]], radius=r, mass=1e30, inertia=1e30)
    o.step(1)
    assert abs(o.forces()[3][0, 1] - 0.1) < 1e-15


@pytest.mark.parametrize("q", [9, 19])
def test_wall_sites_hold_wall_equilibrium(q):
    """After the substeps every site of the four wall layers of a closed axis
    (and only those) holds f^eq(rho, U_wall) with its own density: zeroth and
    first moments of the post-substep state are (rho, rho U_wall) exactly."""
    o, m, g, V, axis = _settling_with_walls(q)
    o.step(7)
    fs = o.get_fs().reshape(q, -1)
    c, w = oracle.lattice(q)
    rho = fs.sum(axis=0)
    u = (c.T.astype(np.float64) @ fs) / rho
    n = [o.nx, o.ny, o.nz]
    z, y, x = np.meshgrid(np.arange(o.nz), np.arange(o.ny), np.arange(o.nx), indexing="ij")
    coords = [x.ravel(), y.ravel(), z.ravel()]
    wall = np.zeros(o.N, dtype=bool)
    for a in (0, axis):
        wall |= (coords[a] < 2) | (coords[a] >= n[a] - 2)
    assert np.abs(u[:, wall]).max() < 1e-15  # walls at rest
    for s in np.flatnonzero(wall)[:: max(1, wall.sum() // 200)]:
        assert np.abs(fs[:, s] - oracle.feq(q, rho[s], np.zeros(3))).max() < 4 * EPS
    # the fluid next to the walls does move
    assert np.abs(u[:, ~wall]).max() > 1e-6
