"""Device-side status paths: bounded conditions the kernels detect, report
through the status word at the next synchronising call, and survive (every
list they fill is clamped to its capacity, so nothing is written out of
bounds).  After the report the status is cleared and the context keeps
working.

  - LBM_ECOLLISION, speed bound: the collision search lists pairs within
    r_i + r_j + 1 at the start of a step, which finds every contact of the
    step while each speed stays below 0.5 lu/step (section 2.3's hard-core
    model needs every contact); a faster particle is reported.
  - LBM_ECOLLISION, crowding: more than 64 particles within r_i + r_j + 1 of
    one particle overflow its candidate list.
  - LBM_ECAPACITY: more than 1024 pairs closer than the closure's gap in one
    step (the closure handles the first 1024).
"""
import numpy as np
import pytest

from paper_1105_2904_amd import lbm
from paper_1105_2904_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    lbm.lib()


def _expect(code, fn):
    with pytest.raises(lbm.LbmError) as e:
        fn()
    assert e.value.code == code, (e.value.code, code)


def test_fast_particle_reports_ecollision():
    """A kinematic sphere moving at 0.55 lu/step (its speed is imposed, so the
    fluid cannot slow it below the bound) next to a free one."""
    box = (48, 40, 36)
    x = np.array([[14.0, 20.0, 18.0], [30.0, 20.2, 17.6]])
    m, inertia = wl.solid_body(3, np.array([4.0, 4.0]), 2.0)
    m[1] = inertia[1] = np.inf

    def make(speed):
        s = lbm.Simulation(19, *box, tau=0.8, storage="fp32", max_particles=2, max_radius=4.0)
        s.add_particles(x, u=[[0.0, 0.0, 0.0], [-speed, 0.0, 0.0]], radius=[4.0, 4.0], mass=m, inertia=inertia)
        return s

    sim = make(0.55)
    sim.step(1)
    _expect(lbm.LBM_ECOLLISION, sim.forces)
    sim.forces()  # reported once, then cleared
    sim.close()
    ok = make(0.45)  # below the bound: no report
    ok.step(3)
    ok.forces()
    ok.close()


def test_crowded_neighbourhood_reports_ecollision():
    """A disk of r = 12 ringed by 70 disks of r = 0.5 (every one within
    r_i + r_j + 1 of it): 70 candidates for one particle, more than the 64
    its list holds."""
    box = (64, 64, 1)
    n = 70
    a = 2 * np.pi * np.arange(n) / n
    ring = np.stack([32.0 + 12.9 * np.cos(a), 32.0 + 12.9 * np.sin(a), np.zeros(n)], axis=1)
    x = np.vstack([[[32.0, 32.0, 0.0]], ring])
    r = np.concatenate([[12.0], np.full(n, 0.5)])
    sim = lbm.Simulation(9, *box, tau=0.8, storage="fp64", max_particles=n + 1, max_radius=12.0)
    sim.add_particles(x, radius=r, mass=np.inf, inertia=np.inf)
    sim.step(1)
    _expect(lbm.LBM_ECOLLISION, sim.forces)
    sim.forces()
    sim.close()
    # 64 in the ring fit the list: no report
    ok = lbm.Simulation(9, *box, tau=0.8, storage="fp64", max_particles=65, max_radius=12.0)
    a = 2 * np.pi * np.arange(64) / 64
    ring = np.stack([32.0 + 12.9 * np.cos(a), 32.0 + 12.9 * np.sin(a), np.zeros(64)], axis=1)
    ok.add_particles(np.vstack([[[32.0, 32.0, 0.0]], ring]), radius=np.concatenate([[12.0], np.full(64, 0.5)]),
                     mass=np.inf, inertia=np.inf)
    ok.step(2)
    ok.forces()
    ok.close()


def test_closure_pair_capacity_reports_ecapacity():
    """A periodic 24 x 24 lattice of disks r = 2, 5 apart (surface gap 1 <
    h_max = 2): 1152 close pairs, more than the 1024 one step handles."""
    import torch
    k, h = 24, 5.0
    g = (np.arange(k) + 0.5) * h
    X, Y = np.meshgrid(g, g, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), np.zeros(k * k)], axis=1)
    params = torch.tensor(wl.mlp_init(3).astype(np.float32), device="cuda")

    def make(n_rows):
        box = (int(k * h), int(n_rows * h), 1)
        keep = x[:, 1] < n_rows * h
        s = lbm.Simulation(9, *box, tau=0.7, storage="fp32", max_particles=int(keep.sum()), max_radius=2.0)
        s.add_particles(x[keep], radius=2.0, mass=np.inf, inertia=np.inf)
        s.set_closure(params, h_max=2.0)
        return s

    sim = make(k)
    sim.step(1)
    _expect(lbm.LBM_ECAPACITY, sim.forces)
    sim.forces()
    sim.close()
    # 20 rows: 20 * 24 * 2 = 960 pairs, within capacity
    ok = make(20)
    ok.step(2)
    ok.forces()
    ok.close()
