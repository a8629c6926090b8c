"""The AA pattern (one population array updated in place, even steps at a
site's own slots, odd steps at its neighbours') against two arrays: the same
arithmetic on the same numbers, so every step, read-out and particle quantity
must agree bit for bit, whatever the parity of the step count, and the AA
context must follow the oracle like any other."""
import numpy as np
import pytest

import oracle
from paper_1105_2904_amd import lbm
from paper_1105_2904_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(*a):
    print(*a, flush=True)


def _pair(q, box, storage, parts, boxes=None, capacity=None, **kw):
    sims = []
    n = 0 if parts is None else sum(len(p["radius"]) for p in (parts if boxes else [parts]))
    n = capacity or n
    rmax = 1.0 if parts is None else max(float(np.max(p["radius"])) for p in (parts if boxes else [parts]))
    for aa in (False, True):
        s = lbm.Simulation(q, *box, storage=storage, max_particles=n, max_radius=rmax, boxes=boxes, aa=aa, **kw)
        if parts is not None:
            for b, p in enumerate(parts if boxes else [parts]):
                s.add_particles(p["x"], radius=p["radius"], mass=p["mass"], inertia=p["inertia"],
                                **({"box": b} if boxes else {}))
        sims.append(s)
    return sims


def _same(a, b, label, fields=True):
    assert np.array_equal(a.get_distributions(), b.get_distributions()), (label, "f")
    for k, (x, y) in enumerate(zip(a.forces(), b.forces())):
        assert np.array_equal(x, y), (label, "particle record", k)
    if fields:
        for k, (x, y) in enumerate(zip(a.fields(), b.fields())):
            assert np.array_equal(x, y), (label, "field", k)
    assert np.array_equal(a.shifts(), b.shifts()), label


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "bf16"])
def test_aa_equals_two_arrays_3d(storage):
    box = (40, 36, 32)
    p = wl.suspension(19, box, 6, 5.0, 1.3, seed=91)
    ab, aa = _pair(19, box, storage, p, tau=0.7, gravity=(0, 0, -2e-4), zero_net_force=True)
    _say("AA vs two arrays, D3Q19", storage)
    t = 0
    for n in (1, 1, 4, 3, 6):  # odd and even totals, read-outs in both AA halves
        ab.step(n)
        aa.step(n)
        t += n
        _same(ab, aa, "%s after %d steps" % (storage, t))
    ab.close()
    aa.close()


def test_aa_equals_two_arrays_2d_walls_graph_and_mid_run_changes():
    """A closed D2Q9 box with a sliding wall and free disks: step graphs on
    the AA context, a particle added after an odd number of steps, and the
    state replaced mid-run on both contexts."""
    box = (72, 60, 1)
    wu = np.zeros((3, 2, 3))
    wu[1, 1, 0] = 0.02
    m, inertia = wl.solid_body(2, np.full(4, 5.0), 1.5, 1.0)
    p = {"x": np.array([[15.0, 20.0, 0], [40.3, 30.6, 0], [60.0, 15.2, 0], [24.7, 44.1, 0]]),
         "radius": np.full(4, 5.0), "mass": np.asarray(m, dtype=np.float64),
         "inertia": np.asarray(inertia, dtype=np.float64)}
    ab, aa = _pair(9, box, "fp32", {k: v[:3] for k, v in p.items()}, capacity=4, tau=0.8, walls=2,
                   wall_velocity=wu, gravity=(0, -1e-4, 0))
    aa.set_graph(4)
    ab.step(9)
    aa.step(9)
    _same(ab, aa, "after 9 steps")
    for s in (ab, aa):
        s.add_particles(p["x"][3:], radius=p["radius"][3:], mass=p["mass"][3:], inertia=p["inertia"][3:])
    ab.step(7)
    aa.step(7)
    _same(ab, aa, "after a particle added at an odd step")
    f = ab.get_distributions()
    rng = np.random.default_rng(5)
    f = f * (1.0 + 1e-3 * rng.standard_normal(f.shape))
    ab.set_distributions(f)
    aa.set_distributions(f)
    ab.step(5)
    aa.step(5)
    _same(ab, aa, "after the state was replaced")
    ab.close()
    aa.close()


def test_aa_equals_two_arrays_ensemble_tiles():
    dims = [(64, 48, 1), (50, 70, 1), (96, 40, 1)]
    parts = [wl.suspension(9, d, n, 4.0, 1.5, seed=95 + b) for b, (d, n) in enumerate(zip(dims, [2, 3, 1]))]
    ab, aa = _pair(9, (1, 1, 1), "fp32", parts, boxes=dims, tau=0.7, gravity=(0, -2e-4, 0), zero_net_force=True)
    for s in (ab, aa):
        s.set_sweep_config(128, 0, 0)
    ab.step(11)
    aa.step(11)
    _same(ab, aa, "ensemble after 11 steps", fields=False)
    for s in (ab, aa):
        s.set_sweep_config(64, 8, 3)
    ab.step(6)
    aa.step(6)
    _same(ab, aa, "ensemble after 17 steps", fields=False)
    ab.close()
    aa.close()


@pytest.mark.parametrize("q,box,n", [(9, (64, 40, 1), 3), (9, (300, 24, 1), 4), (9, (549, 18, 1), 5),
                                     (19, (261, 14, 12), 3)])
@pytest.mark.parametrize("storage", ["fp64", "fp32", "bf16"])
def test_aa_equals_two_arrays_rows_across_waves_and_workgroups(q, box, n, storage):
    """Rows of one wave, of several, and of a ragged number of 64-site waves
    over two or three row-kernel workgroups, with the periodic seam inside
    the last wave: every odd step's push along x must land at the right
    neighbour."""
    r = 3.0 if q == 19 else 4.0
    p = wl.suspension(q, box, n, r, 1.3, seed=131 + box[0])
    g = (0, -2e-4, 0)
    ab, aa = _pair(q, box, storage, p, tau=0.7, gravity=g, zero_net_force=True)
    rng = np.random.default_rng(box[0])
    f = ab.get_distributions()
    f = f * (1.0 + 2e-3 * rng.standard_normal(f.shape))
    for s in (ab, aa):
        s.set_sweep_config(0, 0, 0)  # the row kernel
        s.set_distributions(f)
    total = 0
    for n_steps in (1, 2, 5):
        for s in (ab, aa):
            s.step(n_steps)
        total += n_steps
        _same(ab, aa, "Q%d %s %s after %d steps" % (q, box, storage, total))
    _say("AA = two arrays, row kernel, box %s %s: %d steps" % (box, storage, total))
    ab.close()
    aa.close()


def test_aa_context_follows_the_oracle():
    box = (30, 28, 26)
    p = wl.suspension(19, box, 3, 4.5, 1.3, seed=97)
    sim = lbm.Simulation(19, *box, tau=0.75, gravity=(0, 0, -3e-4), zero_net_force=True, storage="fp64",
                         max_particles=3, max_radius=4.5, aa=True)
    sim.add_particles(p["x"], radius=p["radius"], mass=p["mass"], inertia=p["inertia"])
    ora = oracle.Oracle(19, *box, 0.75, gravity=(0, 0, -3e-4), zero_net_force=True)
    ora.add_particles(p["x"], radius=p["radius"], mass=p["mass"], inertia=p["inertia"])
    for n in (3, 4):
        sim.step(n)
        ora.step(n)
        fg, fo = sim.get_distributions(), ora.get_f()
        e_f = np.abs(fg - fo).max() / np.abs(fo).max()
        Fg, Fo = sim.forces()[0], ora.forces()[0]
        e_F = np.abs(Fg - Fo).max() / max(np.abs(Fo).max(), 1e-30)
        _say("AA vs oracle: e_f", e_f, "e_F", e_F)
        assert e_f <= 1e-12 and e_F <= 1e-10
    sim.close()


def test_aa_context_refuses_autotune():
    sim = lbm.Simulation(9, 32, 32, 1, tau=0.8, aa=True)
    with pytest.raises(lbm.LbmError):
        sim.autotune(reps=1)
    sim.set_sweep_config(64, 0, 4)  # an explicit launch is fine
    sim.step(3)
    sim.close()
