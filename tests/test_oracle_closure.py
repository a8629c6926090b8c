"""Pins of the oracle's near-contact closure (CPU): its FP16 rounding against
numpy's IEEE binary16, its network against oracle/mlp.py, its inputs for a pair
computed by hand, and the way the force enters a step (zero network = no
change; equal and opposite pair forces; F = mu U (a_n n + a_t t))."""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_1105_2904_amd import workloads as wl


def test_half_rounding_matches_ieee_binary16():
    rng = np.random.Generator(np.random.PCG64(1))
    vals = np.concatenate([rng.uniform(-2, 2, 60000), rng.normal(0, 1e-4, 40000),
                           np.exp(rng.uniform(-25, 11.5, 60000)) * rng.choice([-1, 1], 60000),
                           rng.uniform(-1e-7, 1e-7, 40000)]).astype(np.float32)
    # exact ties between neighbouring FP16 values and the overflow edge
    h = np.arange(-2048, 2048, dtype=np.float64) / 1024.0
    ties = (h[:-1] + h[1:]) / 2
    vals = np.concatenate([vals, ties.astype(np.float32), np.float32([65504.0, 65519.99, 65520.0, 6e-8, 3e-8])])
    ours = np.array([oracle.half(float(v)) for v in vals])
    with np.errstate(over="ignore"):  # 65520 and above round to infinity
        ref = vals.astype(np.float16).astype(np.float64)
    assert np.array_equal(ours, ref)


def test_closure_net_matches_numpy_oracle():
    theta = wl.mlp_init(2)
    rng = np.random.Generator(np.random.PCG64(3))
    X = rng.uniform(-1, 1, size=(200, 8)).astype(np.float32).astype(np.float64)
    y_c = oracle.closure_net(theta, X)
    y_n, _ = omlp.forward(theta, X, quantize=True)
    assert np.abs(y_c - y_n).max() <= 1e-3 * np.abs(y_n).max()
    assert np.median(np.abs(y_c - y_n)) <= 1e-12


def _pair(tau=0.7, u=((0.01, 0, 0), (-0.01, 0, 0)), mass=(np.inf, np.inf)):
    o = oracle.Oracle(9, 64, 48, 1, tau)
    o.add_particles([[20.3, 24.0, 0], [32.8, 24.0, 0]], u=np.array(u), radius=[5.5, 6.0],
                    mass=list(mass), inertia=[1e9, 1e9])
    return o


def test_closure_inputs_for_a_pair_by_hand():
    o = _pair()
    x = o.closure_inputs(0, 1)
    # d = 12.5 along +x, h = 12.5 - 11.5 = 1, midpoint x = 20.3 + 5.5 + 0.5 = 26.3
    assert np.allclose(x, [1.0, (5.5 - 9) / 3, (6.0 - 9) / 3, 1.0, 0.0, 26.3 - 26.0, 24.0 - 24.0, 0.0],
                       rtol=0, atol=1e-13)
    # across the periodic boundary the minimum image is used
    o2 = oracle.Oracle(9, 64, 48, 1, 0.8)
    o2.add_particles([[2.0, 10.0, 0], [58.0, 10.0, 0]], radius=[3.0, 3.0], mass=[1e9, 1e9], inertia=[1e9, 1e9])
    x2 = o2.closure_inputs(0, 1)
    assert abs(x2[0] - 2.0) < 1e-13 and abs(x2[3] + 1.0) < 1e-13 and abs(x2[7] - 1.0) < 1e-13


def test_zero_network_changes_nothing():
    a, b = _pair(), _pair()
    b.set_closure(np.zeros(omlp.N_PARAMS), h_max=2.0)
    a.step(12)
    b.step(12)
    assert np.array_equal(a.get_f(), b.get_f())
    assert all(np.array_equal(p, q) for p, q in zip(a.forces(), b.forces()))


def test_closure_force_assembly_and_third_law():
    """With kinematic particles the closure changes only the reported force:
    F_closure - F_plain = mu U (a_n n + a_t t) on particle 0, the opposite on
    particle 1, with a from the network on the pair's inputs."""
    theta = wl.mlp_init(4) * 3.0
    theta[-2:] = [0.7, -0.2]  # non-zero output biases
    a, b = _pair(), _pair()
    b.set_closure(theta, h_max=2.0)
    x = a.closure_inputs(0, 1)
    a.step(1)
    b.step(1)
    assert np.array_equal(a.get_f(), b.get_f())  # the fluid does not see it
    dF = b.forces()[0] - a.forces()[0]
    y = oracle.closure_net(theta, x[None, :])[0]
    mu = (0.7 - 0.5) / 3.0
    U = 0.02  # approach speed (u_0 - u_1).n
    expect = mu * U * np.array([y[0], y[1], 0.0])  # n = +x, t = +y
    assert np.allclose(dF[0], expect, rtol=1e-12, atol=1e-16)
    assert np.allclose(dF[1], -expect, rtol=1e-12, atol=1e-16)
    assert np.abs(expect).max() > 1e-6


def test_closure_moves_free_particles():
    """Free particles: the closure force enters the acceleration (u' - u)
    = F / m, and only below h_max."""
    theta = wl.mlp_init(5) * 2.0
    theta[-2:] = [5.0, 0.0]
    near = [_pair(mass=(200.0, 300.0)) for _ in range(2)]
    near[1].set_closure(theta, h_max=2.0)
    far = [_pair(mass=(200.0, 300.0)) for _ in range(2)]
    far[1].set_closure(theta, h_max=0.5)  # gap 1 is above this h_max
    for o in near + far:
        o.step(1)
    du = near[1].forces()[3] - near[0].forces()[3]
    dF = near[1].forces()[0] - near[0].forces()[0]
    assert np.allclose(du[0], dF[0] / 200.0, rtol=1e-9, atol=1e-18)
    assert np.allclose(du[1], dF[1] / 300.0, rtol=1e-9, atol=1e-18)
    assert np.abs(dF).max() > 0
    assert all(np.array_equal(p, q) for p, q in zip(far[0].forces(), far[1].forces()))


def test_closure_is_2d_only():
    o = oracle.Oracle(19, 16, 16, 16, 0.8)
    with pytest.raises(ValueError):
        o.set_closure(np.zeros(omlp.N_PARAMS))
