"""Stokes drag on periodic arrays of fixed particles at the particle sizes of
the suspension workloads, on the GPU.  The oracle pins this only on small
particles (its cost); here the same property is checked at full size: the
effective hydrodynamic radius a_h that the drag implies through Hasimoto's
closed forms (1959; square array of disks, simple cubic array of spheres)
lies within [r - 1.5, r + 0.5] and does not drift with r.

At steady state the mean fluid momentum is stationary, so the particle's
site conditions remove exactly the momentum the body force injects, N f_b;
with the superficial velocity U this gives F / (mu U)."""
import math

import numpy as np
import pytest

from paper_1105_2904_amd import lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(*a):
    print(*a, flush=True)


def _disk_K(c):
    # square array of disks: F / (mu U) = 4 pi / (-ln(c)/2 - 0.738 + c - 0.887 c^2 + 2.039 c^3)
    return 4 * np.pi / (-0.5 * np.log(c) - 0.738 + c - 0.887 * c * c + 2.039 * c ** 3)


def _sphere_K(c):
    # simple cubic array of spheres: F / (6 pi mu a U) = 1 / (1 - 1.7601 c^(1/3) + c - 1.5593 c^2)
    return 1.0 / (1.0 - 1.7601 * c ** (1.0 / 3.0) + c - 1.5593 * c * c)


def _radius(F_over_muU, L, dim):
    """Bisection for the radius whose array drag F / (mu U) matches."""
    lo, hi = 0.01 * L, 0.3 * L
    for _ in range(200):
        a = 0.5 * (lo + hi)
        if dim == 2:
            v = _disk_K(math.pi * a * a / (L * L))
        else:
            v = 6 * math.pi * a * _sphere_K(4 * math.pi * a ** 3 / (3 * L ** 3))
        if v < F_over_muU:
            lo = a
        else:
            hi = a
    return 0.5 * (lo + hi)


def _effective_radius(dim, L, r, fb, relax):
    """Run to steady state (about 2.5 relaxation times, then three samples
    0.6 relax apart extrapolated to their limit) and return a_h and the
    fraction of N f_b the particle itself reports as its force."""
    tau = 1.5
    nu = (tau - 0.5) / 3.0
    q, nz = (9, 1) if dim == 2 else (19, L)
    sim = lbm.Simulation(q, L, L, nz, tau=tau, body_force=(fb, 0, 0), storage="fp64", max_particles=1,
                         max_radius=r)
    c = [L / 2, L / 2, L / 2 if dim == 3 else 0.0]
    sim.add_particles([c], radius=[r], mass=[np.inf], inertia=[np.inf])
    sim.set_graph(50)
    grid = np.mgrid[0:nz, 0:L, 0:L]
    d2 = (grid[2] - c[0]) ** 2 + (grid[1] - c[1]) ** 2 + ((grid[0] - c[2]) ** 2 if dim == 3 else 0)
    sim.step(int(1.8 * relax) // 50 * 50)
    Us, Fs = [], []
    for _ in range(3):
        sim.step(int(0.6 * relax) // 50 * 50)
        rho, u, _ = sim.fields()
        solid = (d2 <= r * r) & (sim.site_kind() != 1)
        Us.append((rho * u[..., 0])[~solid].sum() / L ** dim)
        Fs.append(sim.forces()[0][0, 0] / (fb * L ** dim))
    sim.close()

    def limit(v):
        e1, e2 = v[1] - v[0], v[2] - v[1]
        assert 0 < e2 / e1 < 0.9, v  # a decaying approach
        return v[2] - e2 * e2 / (e2 - e1)

    U = limit(Us)
    return _radius(fb * L ** dim / (nu * U), L, dim), limit(Fs), U * 2 * r / nu


@pytest.mark.parametrize("dim,cases", [
    (2, ((128, 16.0), (192, 24.0), (256, 32.0))),
    (3, ((48, 6.0), (72, 9.0), (96, 12.0))),
])
def test_array_drag_effective_radius_at_full_size(dim, cases):
    shifts = []
    for L, r in cases:
        # body force scaled so that the particle Reynolds number stays ~0.05
        fb = (2e-6 * (32.0 / L) ** 2) if dim == 2 else (2e-6 * (24.0 / L) ** 2)
        relax = (0.27 if dim == 2 else 1.2) * L * L  # time constant of the mean flow (measured)
        a_h, frac, re = _effective_radius(dim, L, r, fb, relax)
        _say("%dD L %d r %.0f: a_h %.3f (a_h - r %.3f), particle force / injected %.3f, Re %.3f" %
             (dim, L, r, a_h, a_h - r, frac, re))
        assert r - 1.5 <= a_h <= r + 0.5, (L, r, a_h)
        assert 0.5 < frac < 1.0
        assert re < 0.2
        shifts.append(a_h - r)
    assert max(shifts) - min(shifts) < 0.5, shifts
