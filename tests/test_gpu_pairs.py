"""Two sites per lane in the 16-bit row sweep, through the C ABI on the GPU.

With FP16/BF16 storage, two population arrays and an even row length, the
row kernel gives each lane two neighbouring sites (x even, x + 1): one
aligned 4-byte load per population, with the pull's shift along x rebuilt
from the neighbouring lane's word and, at the two ends of a 128-site wave,
from one load past the end.  Every site collides as in the one-site sweeps,
so the tile kernel (one site per lane) must give the same bits after any
number of steps.  Checked on rows of one pair, of part of a wave, of whole
and ragged numbers of waves, with balls across the periodic seam along x,
with walls on x and y, with an occupancy cap, with the words past a wave's
ends passed inside the workgroup or loaded (rows of three and eight waves),
and for an odd row length (which keeps one site per lane).  Against the FP64 oracle, LBGK from random
populations stays within the storage rounding, as in the one-site tests.
"""
import numpy as np
import pytest

import oracle
from paper_1105_2904_amd import lbm
from paper_1105_2904_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    lbm.lib()


def _say(*a):
    print(*a, flush=True)


def _particles(q, specs, density_ratio=4.0):
    dim = 2 if q == 9 else 3
    x = np.array([s[0] for s in specs], dtype=np.float64)
    u = np.array([s[1] for s in specs], dtype=np.float64)
    r = np.array([s[2] for s in specs], dtype=np.float64)
    m, inertia = wl.solid_body(dim, r, density_ratio, 1.0)
    return {"x": x, "u": u, "omega": np.zeros_like(x), "radius": r,
            "mass": np.asarray(m, dtype=np.float64), "inertia": np.asarray(inertia, dtype=np.float64)}


# (q, box, walls, particles: (centre, velocity, radius))
CASES = {
    "d2q9 2x24 one pair per row": (9, (2, 24, 1), 0, []),
    "d2q9 130x28 a wave and one pair, disk across the x seam": (
        9, (130, 28, 1), 0, [((0.4, 14.0, 0.0), (-0.04, 0.01, 0.0), 4.5), ((65.3, 6.2, 0.0), (0.04, 0.0, 0.0), 4.0)]),
    "d2q9 128x40 walls on x and y": (9, (128, 40, 1), 3, [((12.5, 20.2, 0.0), (-0.04, 0.0, 0.0), 4.0)]),
    "d2q9 1024x16 rows of eight waves over two workgroups, disk across the x seam": (
        9, (1024, 16, 1), 0, [((1023.7, 8.0, 0.0), (0.04, 0.01, 0.0), 4.0), ((511.6, 3.0, 0.0), (0.04, 0.0, 0.0), 3.0)]),
    "d2q9 300x20 rows of three waves, workgroups across rows": (
        9, (300, 20, 1), 0, [((127.8, 10.0, 0.0), (0.04, 0.0, 0.0), 4.0), ((256.3, 4.0, 0.0), (-0.04, 0.0, 0.0), 3.0)]),
    "d3q19 198x12x12 a wave and 35 pairs, sphere across the x seam": (
        19, (198, 12, 12), 0, [((0.3, 6.0, 5.0), (-0.04, 0.0, 0.01), 3.5)]),
    "d3q19 256x10x10 two whole waves": (
        19, (256, 10, 10), 0, [((255.6, 5.0, 4.0), (0.04, 0.01, 0.0), 3.0), ((128.2, 3.0, 2.5), (-0.04, 0.0, 0.0), 3.0)]),
    "d3q19 77x14x12 odd rows": (19, (77, 14, 12), 0, [((0.2, 7.0, 6.0), (-0.04, 0.0, 0.0), 3.5)]),
}


def _run(q, box, walls, specs, storage, shape, f0, steps=40, chunk=10):
    p = _particles(q, specs) if specs else None
    rmax = max(s[2] for s in specs) if specs else 1.0
    sim = lbm.Simulation(q, *box, tau=0.7, body_force=(2e-6, -1e-6, 0.0), storage=storage,
                         max_particles=max(1, len(specs)), max_radius=rmax, walls=walls)
    sim.set_distributions(f0)
    if p is not None:
        sim.add_particles(p["x"], u=p["u"], omega=p["omega"], radius=p["radius"], mass=p["mass"],
                          inertia=p["inertia"])
    sim.set_sweep_config(*shape)
    out = []
    for _ in range(steps // chunk):
        sim.step(chunk)
        F, T, x, u, om = sim.forces()
        out.append((sim.get_distributions(), F, T, x, u, sim.shifts()))
    sim.close()
    return out


@pytest.mark.parametrize("storage", ["fp16", "bf16"])
@pytest.mark.parametrize("case", list(CASES))
def test_two_sites_per_lane_equal_one_site_per_lane(case, storage):
    q, box, walls, specs = CASES[case]
    _, w = oracle.lattice(q)
    f0 = wl.random_populations(w, box[::-1], seed=17 + box[0], eps=0.02)
    ref = _run(q, box, walls, specs, storage, (128, 0, 0), f0)  # tiles: one site per lane
    for shape in [(0, 0, 0), (0, 0, 4)]:  # the row kernel, without and with an occupancy cap
        got = _run(q, box, walls, specs, storage, shape, f0)
        for k, (a, b) in enumerate(zip(got, ref)):
            for name, x, y in zip(("f", "F", "T", "x", "u", "shifts"), a, b):
                assert np.array_equal(x, y), (case, storage, shape, "after %d steps" % (10 * (k + 1)), name)
    if specs:  # the balls moved to new integer shifts (re-stamped, IS substep at new sites)
        assert np.abs(ref[-1][5]).max() > 0, (case, "no shift changed")
    _say("%s %s: row kernel = tile kernel, 40 steps" % (case, storage))


@pytest.mark.parametrize("q,box", [(9, (2, 24, 1)), (9, (130, 28, 1)), (19, (198, 12, 10))])
@pytest.mark.parametrize("storage,bits", [("fp16", 11), ("bf16", 8)])
def test_two_sites_per_lane_lbgk_against_oracle(q, box, storage, bits):
    """Random populations, 25 steps: within a few storage roundings of the FP64
    oracle (relative 2^-bits of |g/w|), the bound of the one-site tests."""
    _, w = oracle.lattice(q)
    f0 = wl.random_populations(w, box[::-1], seed=71 + box[0], eps=0.05)
    sim = lbm.Simulation(q, *box, tau=0.7, storage=storage, max_particles=0)
    ora = oracle.Oracle(q, *box, 0.7)
    sim.set_distributions(f0)
    ora.set_f(f0)
    assert sim.sweep_config() == (0, 0, 0)
    gw = np.abs(f0 / w.reshape(q, 1, 1, 1) - 1.0).max()
    tol = 4 * 2.0 ** -bits * gw * w.max() / np.abs(f0).max()
    sim.step(25)
    ora.step(25)
    fo = ora.get_f()
    e = np.abs(sim.get_distributions() - fo).max() / np.abs(fo).max()
    _say("pairs lbgk Q%d %s %s: e_f %.2e (bound %.2e)" % (q, box, storage, e, tol))
    assert e <= tol
    sim.close()
