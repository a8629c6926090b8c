"""The oracle's per-site loops on several OpenMP threads give the same bits as
on one thread (each iteration writes only its own sites; every sum over sites
or particles stays a fixed-order loop on one thread)."""
import numpy as np

import oracle
from paper_1105_2904_amd import workloads as wl


def _run(threads, q, box, p, g, steps, walls=0):
    oracle.set_threads(threads)
    o = oracle.Oracle(q, *box, 0.7, gravity=g, zero_net_force=not walls, walls=walls)
    o.add_particles(p["x"], u=p["u"], omega=p["omega"], radius=p["radius"], mass=p["mass"],
                    inertia=p["inertia"])
    o.step(steps)
    out = (o.get_f(), o.get_fs()) + tuple(o.forces()) + (o.shifts(), o.site_kind())
    out += tuple(o.fields())
    o.close()
    return out


def test_threads_bit_identical_3d():
    box = (40, 36, 32)
    p = wl.suspension(19, box, 4, 4.5, 1.2, seed=91)
    p["u"][:, 0] = np.linspace(-0.03, 0.03, 4)
    p["omega"][:, 2] = 1e-3
    try:
        one = _run(1, 19, box, p, (0, 0, -3e-4), 12)
        many = _run(8, 19, box, p, (0, 0, -3e-4), 12)
    finally:
        oracle.set_threads(0)
    for a, b in zip(one, many):
        assert np.array_equal(a, b)


def test_threads_bit_identical_2d_walls():
    box = (96, 80, 1)
    p = wl.suspension(9, (90, 60, 1), 5, 5.0, 1.5, seed=92)
    p["x"][:, 0] += 3.0
    p["x"][:, 1] += 12.0
    try:
        one = _run(1, 9, box, p, (0, -2e-4, 0), 30, walls=0b011)
        many = _run(7, 9, box, p, (0, -2e-4, 0), 30, walls=0b011)
        assert oracle.threads() == 7
    finally:
        oracle.set_threads(0)
    for a, b in zip(one, many):
        assert np.array_equal(a, b)
