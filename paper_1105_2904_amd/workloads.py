"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no lattice Boltzmann arithmetic: it only draws particle
placements and random populations from a counter-free SplitMix64 stream, and
fills in the particle records (mass and moment of inertia of a uniform disk
or sphere of the given density ratio).  Both the GPU path and the oracle are
fed from here; neither is called from here.

Placement is random sequential addition in a periodic box: draw a centre
uniformly, reject it if its surface comes closer than ``min_gap`` lattice
units to an accepted particle (minimum image), up to ``max_tries`` draws per
particle.
"""
import math

import numpy as np

_MASK = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): 64-bit state, golden-gamma
    increment, two xor-shift-multiply finalisation rounds."""

    def __init__(self, seed):
        self.state = seed & _MASK

    def next_u64(self):
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self):
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))

    def uniform_array(self, n):
        return np.array([self.uniform() for _ in range(n)])

    def randint(self, lo, hi):
        """Integer in [lo, hi] (inclusive)."""
        return lo + int(self.uniform() * (hi - lo + 1))


def place_particles(box, radii, seed, min_gap=2.0, max_tries=10**6):
    """Random sequential addition of particles of the given radii.

    box: (nx, ny, nz) with nz == 1 for 2D.  Returns centres [n][3] (z = 0 in
    2D), in [0, L) per axis.
    """
    rng = SplitMix64(seed)
    dim = 2 if box[2] == 1 else 3
    L = np.array(box, dtype=np.float64)
    placed = []
    rad = []
    for r in radii:
        for _ in range(max_tries):
            c = np.zeros(3)
            for a in range(dim):
                c[a] = rng.uniform() * L[a]
            ok = True
            if placed:
                P = np.array(placed)
                d = P[:, :dim] - c[:dim]
                d -= L[:dim] * np.floor(d / L[:dim] + 0.5)
                dist = np.sqrt((d * d).sum(axis=1))
                if np.any(dist < np.array(rad) + r + min_gap):
                    ok = False
            if ok:
                placed.append(c)
                rad.append(r)
                break
        else:
            raise RuntimeError("could not place particle %d" % len(placed))
    return np.array(placed).reshape(-1, 3)


def solid_body(dim, radius, density_ratio, rho0=1.0):
    """Mass and moment of inertia of a uniform disk (2D) or sphere (3D)."""
    r = np.asarray(radius, dtype=np.float64)
    if dim == 2:
        m = density_ratio * rho0 * math.pi * r * r
        inertia = 0.5 * m * r * r
    else:
        m = density_ratio * rho0 * (4.0 / 3.0) * math.pi * r ** 3
        inertia = 0.4 * m * r * r
    return m, inertia


def random_populations(base, shape, seed, eps):
    """Populations base[i] * (1 + eps * xi) with xi uniform in [-1, 1).

    base: per-direction base values [q]; shape: (nz, ny, nx).  Returns
    [q][nz][ny][nx] float64.
    """
    q = len(base)
    n = q * int(np.prod(shape))
    rng = np.random.Generator(np.random.PCG64(seed))
    xi = rng.uniform(-1.0, 1.0, size=n).reshape((q,) + tuple(shape))
    return np.asarray(base, dtype=np.float64).reshape((q, 1, 1, 1)) * (1.0 + eps * xi)


def suspension(q, box, n, radius, density_ratio, seed, min_gap=2.0, rho0=1.0):
    """Particle records for n equal particles at seeded random positions."""
    dim = 2 if q == 9 else 3
    radii = np.full(n, float(radius))
    x = place_particles(box, radii, seed, min_gap=min_gap)
    m, inertia = solid_body(dim, radii, density_ratio, rho0)
    return {"x": x, "u": np.zeros((n, 3)), "omega": np.zeros((n, 3)),
            "radius": radii, "mass": np.asarray(m, dtype=np.float64),
            "inertia": np.asarray(inertia, dtype=np.float64)}


def seeded_velocities(n, dim, vmax, seed):
    """Initial velocities [n][3]: every in-plane component uniform in
    [-vmax, vmax) from a SplitMix64 stream (the z components are 0 in 2D)."""
    rng = SplitMix64(seed)
    u = np.zeros((n, 3))
    for j in range(n):
        for a in range(dim):
            u[j, a] = vmax * (2.0 * rng.uniform() - 1.0)
    return u


def kinematic_disk_config():
    """D2Q9, tau 0.8, 64x64 periodic, one disk of radius 8 at the centre moving
    with imposed velocity (0.01, 0); FP64; 1000 steps."""
    return {"name": "d2q9-64x64-kinematic-disk", "q": 9, "box": (64, 64, 1),
            "tau": 0.8, "rho0": 1.0, "gravity": (0.0, 0.0, 0.0),
            "zero_net_force": False, "storage": "fp64", "steps": 1000,
            "particles": {"x": np.array([[32.0, 32.0, 0.0]]),
                          "u": np.array([[0.01, 0.0, 0.0]]),
                          "omega": np.zeros((1, 3)), "radius": np.array([8.0]),
                          "mass": np.array([np.inf]), "inertia": np.array([np.inf])}}


def disks_2d_config(seed=1):
    """D2Q9, tau 0.7, 1024x1024 periodic, 200 disks of radius 10, density ratio
    1.5, gravity 1e-5; FP32; 10000 steps."""
    return {"name": "d2q9-1024x1024-200-disks", "q": 9, "box": (1024, 1024, 1),
            "tau": 0.7, "rho0": 1.0, "gravity": (0.0, -1e-5, 0.0),
            "zero_net_force": True, "storage": "fp32", "steps": 10000,
            "particles": suspension(9, (1024, 1024, 1), 200, 10.0, 1.5, seed)}


def spheres_3d_config(seed=2, storage="fp32"):
    """D3Q19, tau 0.6, 256^3 periodic, 500 spheres of radius 6, density ratio
    1.2, gravity 1e-6; FP32; 2000 steps."""
    return {"name": "d3q19-256cubed-500-spheres", "q": 19, "box": (256, 256, 256),
            "tau": 0.6, "rho0": 1.0, "gravity": (0.0, 0.0, -1e-6),
            "zero_net_force": True, "storage": storage, "steps": 2000,
            "particles": suspension(19, (256, 256, 256), 500, 6.0, 1.2, seed)}


def ensemble_2d_config(seed=4, nbox=64, phi_max=0.25):
    """An ensemble of independent D2Q9 boxes: side L uniform in 128..512,
    n uniform in 10..80 disks with radii uniform in [6, 12], density ratio
    1.5, gravity 1e-5, tau 0.7, FP32.  The count is clipped (last disks
    dropped) so that the area fraction stays <= phi_max: 80 disks of mean
    area 264 do not fit a 128^2 box."""
    rng = SplitMix64(seed)
    boxes, parts, clipped = [], [], []
    for b in range(nbox):
        L = rng.randint(128, 512)
        n = rng.randint(10, 80)
        radii = np.array([6.0 + 6.0 * rng.uniform() for _ in range(n)])
        keep = n
        while keep > 0 and np.pi * (radii[:keep] ** 2).sum() > phi_max * L * L:
            keep -= 1
        radii = radii[:keep]
        clipped.append(n - keep)
        x = place_particles((L, L, 1), radii, seed * 1000 + b)
        m, inertia = solid_body(2, radii, 1.5)
        boxes.append((L, L, 1))
        parts.append({"x": x, "u": np.zeros((keep, 3)), "omega": np.zeros((keep, 3)), "radius": radii,
                      "mass": np.asarray(m, dtype=np.float64), "inertia": np.asarray(inertia, dtype=np.float64)})
    return {"name": "d2q9-ensemble-%d-boxes" % nbox, "q": 9, "boxes": np.array(boxes, dtype=np.int32),
            "tau": 0.7, "rho0": 1.0, "gravity": (0.0, -1e-5, 0.0), "zero_net_force": True,
            "storage": "fp32", "steps": 10000, "particles": parts, "clipped": clipped}


MLP_SHAPES = [(8, 64), (64,), (64, 64), (64,), (64, 2), (2,)]


# Table 1 of the paper (settling sphere, D = 15 mm, rho_s = 1120 kg/m^3, box
# 100 x 100 x 160 mm): fluid density [kg/m^3], viscosity [1e-3 N s/m^2], tau
# and time step [1e-3 s] of the four cases.
TEN_CATE_TABLE1 = {"E1": (970.0, 373.0, 0.9, 0.347), "E2": (965.0, 212.0, 0.9, 0.607),
                   "E3": (962.0, 113.0, 0.8, 0.851), "E4": (960.0, 58.0, 0.9, 2.207)}
# the Reynolds numbers the paper gives for its lowest and highest case (section 3.3)
TEN_CATE_RE = {"E1": 1.5, "E4": 32.2}


def ten_cate_config(case="E1", z0=120.0):
    """One sphere settling in a closed box at the scale of the paper's Table 1:
    100 x 100 x 160 sites (walls on all three axes, z up) at a lattice spacing
    of 1 mm (the spacing for which every row of Table 1 agrees with the
    paper's viscosity relation; the oracle tests pin it), so D = 15 lattice
    units, gravity 9.81 dt^2 / dx along -z and density ratio 1120 / rho_f.
    The sphere starts at rest on the box's vertical axis with its centre at
    height z0."""
    rho_f, mu, tau, dt_ms = TEN_CATE_TABLE1[case]
    dt, dx = dt_ms * 1e-3, 1e-3
    g = 9.81 * dt * dt / dx
    ratio = 1120.0 / rho_f
    r = 7.5
    m, inertia = solid_body(3, np.array([r]), ratio)
    return {"name": "ten-cate-%s" % case, "box": (100, 100, 160), "tau": tau, "walls": 7,
            "gravity": (0.0, 0.0, -g), "density_ratio": ratio,
            "particles": {"x": np.array([[49.5, 49.5, float(z0)]]), "radius": np.array([r]),
                          "mass": np.asarray(m, dtype=np.float64), "inertia": np.asarray(inertia, dtype=np.float64)},
            "re_paper": TEN_CATE_RE.get(case)}


def mlp_init(seed):
    """Initial parameters of the 8 -> 64 -> 64 -> 2 closure network as one flat
    FP32-representable vector (W1, b1, W2, b2, W3, b3, row-major): Glorot-uniform
    weights (Glorot & Bengio, AISTATS 2010) from numpy's PCG64, zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for shp in MLP_SHAPES:
        if len(shp) == 2:
            lim = math.sqrt(6.0 / (shp[0] + shp[1]))
            parts.append(rng.uniform(-lim, lim, size=shp).ravel())
        else:
            parts.append(np.zeros(shp))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)
