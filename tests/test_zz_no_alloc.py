"""lbm_step_noalloc against lbm_step through the C ABI: the same kernels with
their per-step scratch in the library's own device array instead of the
context's workspace, so two identical contexts stepped one way and the other
must agree bit for bit.  Two calls in a row, the second on a smaller input,
then the capacity limit."""
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


def _twins(q, box, tau, storage, p, gravity, closure=None):
    sims = []
    for _ in range(2):
        s = lbm.Simulation(q, *box, tau=tau, gravity=gravity, zero_net_force=True, storage=storage,
                           max_particles=len(p["radius"]), max_radius=float(np.max(p["radius"])))
        s.add_particles(p["x"], u=p["u"], omega=p["omega"], radius=p["radius"], mass=p["mass"],
                        inertia=p["inertia"])
        if closure is not None:
            s.set_closure(closure, h_max=2.0)
        sims.append(s)
    return sims


def _same(a, b, label):
    assert np.array_equal(a.get_distributions(), b.get_distributions()), label
    for x, y in zip(a.forces(), b.forces()):
        assert np.array_equal(x, y), label
    assert np.array_equal(a.shifts(), b.shifts()), label
    assert np.array_equal(a.site_kind(), b.site_kind()), label


def test_noalloc_matches_step_on_two_calls_then_capacity():
    import torch
    # first call: D3Q19 48 x 40 x 36, six moving spheres, FP32, 30 steps
    box = (48, 40, 36)
    p = wl.suspension(19, box, 6, 4.5, 1.2, seed=95)
    p["u"] = wl.seeded_velocities(6, 3, 0.03, seed=96)
    p["omega"][:, 0] = 1e-3
    a, b = _twins(19, box, 0.65, "fp32", p, (0.0, 0.0, -2e-4))
    a.step(30)
    b.step_noalloc(30)
    print("3D fp32: shifts", b.shifts().tolist(), flush=True)
    _same(a, b, "3D fp32, 30 steps")
    a.close()
    b.close()
    # second call, smaller: D2Q9 64 x 48, three disks, FP64, closure on, 20 steps
    box = (64, 48, 1)
    p = wl.suspension(9, box, 3, 5.0, 1.5, seed=97, min_gap=1.0)
    p["u"] = wl.seeded_velocities(3, 2, 0.02, seed=98)
    params = torch.tensor(wl.mlp_init(5).astype(np.float32), device="cuda")
    a, b = _twins(9, box, 0.75, "fp64", p, (0.0, -1e-4, 0.0), closure=params)
    a.step(20)
    b.step_noalloc(20)
    _same(a, b, "2D fp64 with closure, 20 steps")
    # mixed: the workspace path and the no-allocation path continue each other
    a.step(5)
    b.step_noalloc(2)
    b.step(3)
    _same(a, b, "2D fp64, mixed")
    a.close()
    b.close()
    # more particles than the library array holds: refused, nothing enqueued
    k = 66
    g = (np.arange(k) + 0.5) * 5.0
    X, Y = np.meshgrid(g, g, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), np.zeros(k * k)], axis=1)
    s = lbm.Simulation(9, 330, 330, 1, tau=0.8, storage="fp32", max_particles=k * k, max_radius=0.5)
    s.add_particles(x, radius=0.5, mass=np.inf, inertia=np.inf)
    with pytest.raises(lbm.LbmError) as e:
        s.step_noalloc(1)
    assert e.value.code == lbm.LBM_ECAPACITY
    s.step(1)
    s.forces()
    s.close()
