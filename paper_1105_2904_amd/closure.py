"""Training data and training of the near-contact closure network.

The data come from the method itself, run twice on the same cases.  A case is
a pair of kinematic disks (radii r_i, r_j in [6, 12]) that approach each other
head-on at a constant relative speed U in a periodic D2Q9 box, from a surface
gap h0 down to h_end, the pair's axis at a random angle and its centre at a
random sub-lattice position.
  - working lattice: the case as stated;
  - refined lattice: every length times 4 (box, radii, positions), the speed
    divided by 4 and the same tau: the same Reynolds number and, in diffusive
    time (16 refined steps per working step), the same history.
For 2D Stokes flow the force per unit depth is mu U times a function of the
geometry alone, so the refined run gives the force the working lattice should
have seen: F* = 4 F_refined at matched gaps (the refined speed is U/4 at the
same mu).  The network learns a = (F* - F_working) / (mu U) in the pair's
normal and tangent directions from the closure inputs of each working step
with gap below h_max.  All lattice work runs in the HIP kernels (ensembles of
boxes, one per case), training on the matrix cores (lbm.mlp_train).
"""
import math

import numpy as np

from . import lbm
from .workloads import SplitMix64, mlp_init

REFINE = 4


def cases(seed, n, r_range=(6.0, 12.0), pad=28):
    """n seeded pair cases: radii, axis angle, box side and pair centre."""
    rng = SplitMix64(seed)
    out = []
    for _ in range(n):
        ri = r_range[0] + (r_range[1] - r_range[0]) * rng.uniform()
        rj = r_range[0] + (r_range[1] - r_range[0]) * rng.uniform()
        th = 2.0 * math.pi * rng.uniform()
        L = int(math.ceil((2.0 * (ri + rj) + pad) / 4.0)) * 4
        c = (L / 2.0 + rng.uniform() - 0.5, L / 2.0 + rng.uniform() - 0.5)
        out.append({"ri": ri, "rj": rj, "theta": th, "L": L, "c": c})
    return out


def _positions(case, h0, scale):
    n = np.array([math.cos(case["theta"]), math.sin(case["theta"])])
    c = np.array(case["c"]) * scale
    xi = c - n * (case["ri"] + 0.5 * h0) * scale
    xj = c + n * (case["rj"] + 0.5 * h0) * scale
    return xi, xj, n


def approach(cs, scale, U, h0, h_end, tau, storage="fp32", closure=None, h_max=2.0, progress=None):
    """Run every case as one box of an ensemble at `scale` (1 or REFINE):
    returns the force on the first disk of each pair after every step,
    [steps, ncases, 2], and the step count per working step."""
    dims = [(c["L"] * scale, c["L"] * scale, 1) for c in cs]
    steps = int(round((h0 - h_end) / U)) * scale * scale
    sim = lbm.Simulation(9, 1, 1, 1, tau=tau, storage=storage, max_particles=2 * len(cs),
                         max_radius=max(max(c["ri"], c["rj"]) for c in cs) * scale, boxes=dims)
    for b, c in enumerate(cs):
        xi, xj, n = _positions(c, h0, scale)
        v = 0.5 * U / scale * n
        sim.add_particles([[xi[0], xi[1], 0], [xj[0], xj[1], 0]], u=[[v[0], v[1], 0], [-v[0], -v[1], 0]],
                          radius=[c["ri"] * scale, c["rj"] * scale], mass=np.inf, inertia=np.inf, box=b)
    if closure is not None:
        sim.set_closure(closure, h_max)
    F = np.zeros((steps, len(cs), 2))
    for k in range(steps):
        sim.step(1)
        F[k] = sim.forces()[0][0::2, :2]
        if progress and k % 2000 == 0:
            progress(scale, k, steps)
    sim.close()
    return F


def dataset(cs, U=0.005, h0=3.0, h_end=0.25, tau=0.7, h_max=2.0, storage="fp32", progress=None,
            working=None, refined=None):
    """Closure inputs X [m, 8] and targets A [m, 2] of every working step with
    gap below h_max, plus the working and matched refined forces (normal and
    tangential components, [m, 2] each) and the case of every row."""
    Fw = approach(cs, 1, U, h0, h_end, tau, storage, progress=progress) if working is None else working
    Fr = approach(cs, REFINE, U, h0, h_end, tau, storage, progress=progress) if refined is None else refined
    mu = (tau - 0.5) / 3.0
    r2 = REFINE * REFINE
    X, A, Fwn, Frn, rows = [], [], [], [], []
    for k in range(1, Fw.shape[0] + 1):
        h = h0 - U * (k - 1)  # gap at the start of working step k
        if not h < h_max:
            continue
        j = r2 * (k - 1) + 1  # refined step with the same gap
        lo, hi = max(1, j - r2 // 2), min(Fr.shape[0], j + r2 // 2)
        fr = REFINE * Fr[lo - 1:hi].mean(axis=0)  # [ncases, 2]
        for b, c in enumerate(cs):
            xi, xj, n = _positions(c, h0, 1)
            t = np.array([-n[1], n[0]])
            x_now = xi + (k - 1) * 0.5 * U * n
            d = (xj - xi) - (k - 1) * U * n
            X.append(lbm.closure_inputs(x_now, d, c["ri"], c["rj"], tau)[0])
            fw = Fw[k - 1, b]
            Fwn.append([fw @ n, fw @ t])
            Frn.append([fr[b] @ n, fr[b] @ t])
            A.append([(fr[b] - fw) @ n / (mu * U), (fr[b] - fw) @ t / (mu * U)])
            rows.append(b)
    return {"X": np.array(X, dtype=np.float32), "A": np.array(A), "F_working": np.array(Fwn),
            "F_refined": np.array(Frn), "case": np.array(rows), "mu": mu, "U": U}


def train(X, A, steps=8000, batch=256, lr=2e-3, seed=1, chunks=16, scale_out=None):
    """Adam on the GPU from Glorot-initialised parameters over the rows in a
    seeded random order, the learning rate following a cosine from lr to
    zero in `chunks` constant pieces.  Targets are divided by scale_out
    (default: their RMS) and the output layer multiplied back, so the returned
    parameters predict A itself.  Returns (params, per-step losses)."""
    import torch
    X = np.asarray(X, dtype=np.float32)
    A = np.asarray(A, dtype=np.float64)
    perm = np.random.Generator(np.random.PCG64(seed)).permutation(len(X))
    s = float(np.sqrt((A * A).mean())) if scale_out is None else float(scale_out)
    p = torch.tensor(mlp_init(seed).astype(np.float32), device="cuda")
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    x = torch.tensor(X[perm], device="cuda")
    t = torch.tensor((A[perm] / s).astype(np.float32), device="cuda")
    losses, done = [], 0
    for c in range(chunks):
        n = steps * (c + 1) // chunks - done
        lr_c = lr * 0.5 * (1.0 + math.cos(math.pi * (done + 0.5 * n) / steps))
        losses.append(lbm.mlp_train(p, m, v, x, t, batch=batch, steps=n, step0=done, lr=lr_c).cpu().numpy())
        done += n
    # y = h2 W3 + b3 predicts A / s: scale the output layer by s
    k3 = 8 * 64 + 64 + 64 * 64 + 64
    p[k3:] *= s
    return p, np.concatenate(losses)


def smooth_steps(a, ncase, W=24):
    """Running mean over W working steps of rows ordered by step, then case."""
    a = np.asarray(a).reshape(-1, ncase)
    out = np.empty_like(a, dtype=np.float64)
    for k in range(a.shape[0]):
        out[k] = a[max(0, k - W // 2):min(a.shape[0], k + (W + 1) // 2)].mean(axis=0)
    return out.ravel()
