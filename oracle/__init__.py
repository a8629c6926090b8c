"""FP64 CPU oracle of the site-based suspension lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It
shares no code with the GPU library under ``paper_1105_2904_amd/`` and
imports nothing from it.

The arithmetic lives in ``lbm_oracle.c`` (plain C, FP64; its per-site loops
may run on several OpenMP threads with the same results bit for bit); this
module only builds it with gcc and marshals numpy arrays through ctypes.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_bp = ctypes.POINTER(ctypes.c_int8)


def build():
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
           _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.ora_create.restype = ctypes.c_void_p
        L.ora_create.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double] * 2 + [_dp, _dp, ctypes.c_int]
        L.ora_destroy.argtypes = [ctypes.c_void_p]
        L.ora_add_particles.restype = ctypes.c_int
        L.ora_add_particles.argtypes = [ctypes.c_void_p, ctypes.c_int] + [_dp] * 6
        L.ora_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.ora_forces.argtypes = [ctypes.c_void_p] + [_dp] * 5
        L.ora_fields.argtypes = [ctypes.c_void_p, _dp, _dp, _ip]
        L.ora_site_kind.argtypes = [ctypes.c_void_p, _bp]
        L.ora_shifts.argtypes = [ctypes.c_void_p, _ip]
        L.ora_get_f.argtypes = [ctypes.c_void_p, _dp]
        L.ora_set_f.argtypes = [ctypes.c_void_p, _dp]
        L.ora_get_fs.argtypes = [ctypes.c_void_p, _dp]
        L.ora_template.restype = ctypes.c_int
        L.ora_template.argtypes = [ctypes.c_void_p, ctypes.c_int, _ip, _ip, _ip, _bp]
        L.ora_diagnostics.argtypes = [ctypes.c_void_p, _dp]
        L.ora_num_particles.restype = ctypes.c_int
        L.ora_num_particles.argtypes = [ctypes.c_void_p]
        L.ora_lattice.restype = ctypes.c_int
        L.ora_lattice.argtypes = [ctypes.c_int, _ip, _dp]
        L.ora_feq.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.ora_set_walls.restype = ctypes.c_int
        L.ora_set_walls.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
        L.ora_set_closure.restype = ctypes.c_int
        L.ora_set_closure.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double]
        L.ora_closure_inputs.restype = ctypes.c_int
        L.ora_closure_inputs.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _dp]
        L.ora_closure_net.restype = ctypes.c_int
        L.ora_closure_net.argtypes = [_dp, _dp, _dp]
        L.ora_half.restype = ctypes.c_double
        L.ora_half.argtypes = [ctypes.c_double]
        L.ora_set_threads.argtypes = [ctypes.c_int]
        L.ora_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _vec3(a, n):
    a = np.zeros((n, 3)) if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(n, 3)
    return a


def lattice(q):
    """Velocity set c [q][3] (int) and weights w [q] of D2Q9 / D3Q19."""
    c = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    if lib().ora_lattice(q, c.ctypes.data_as(_ip), _d(w)) != 0:
        raise ValueError("unknown lattice q=%d" % q)
    return c, w


def closure_net(params, x):
    """The closure network of the oracle on inputs x [n, 8] -> [n, 2]."""
    p = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 8)
    y = np.zeros((x.shape[0], 2))
    for k in range(x.shape[0]):
        lib().ora_closure_net(_d(p), _d(x[k]), y[k].ctypes.data_as(_dp))
    return y


def default_threads():
    """The host's share of cores: OMP_NUM_THREADS when set, else the CPUs this
    process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


def set_threads(n):
    """Threads of the oracle's per-site loops (0: default_threads())."""
    lib().ora_set_threads(int(n) if int(n) > 0 else default_threads())


def threads():
    return lib().ora_threads()


def half(x):
    return lib().ora_half(float(x))


def feq(q, rho, u):
    """Equilibrium distribution at one site."""
    out = np.zeros(q)
    uu = np.ascontiguousarray(u, dtype=np.float64).reshape(3)
    lib().ora_feq(q, float(rho), _d(uu), _d(out))
    return out


class Oracle:
    """A periodic box stepped by the oracle (same call shape as the C ABI)."""

    def __init__(self, q, nx, ny, nz, tau, rho0=1.0, gravity=(0, 0, 0),
                 body_force=(0, 0, 0), zero_net_force=False, walls=0, wall_velocity=None):
        self.q, self.nx, self.ny, self.nz = q, nx, ny, nz
        self.N = nx * ny * nz
        g = np.ascontiguousarray(gravity, dtype=np.float64)
        fb = np.ascontiguousarray(body_force, dtype=np.float64)
        self._h = lib().ora_create(q, nx, ny, nz, float(tau), float(rho0), _d(g), _d(fb),
                                   int(bool(zero_net_force)))
        if not self._h:
            raise ValueError("invalid oracle parameters")
        if walls:
            wu = np.zeros((3, 2, 3)) if wall_velocity is None else \
                np.ascontiguousarray(wall_velocity, dtype=np.float64).reshape(3, 2, 3)
            if lib().ora_set_walls(self._h, int(walls), _d(wu)) != 0:
                self.close()
                raise ValueError("invalid wall parameters")

    def close(self):
        if self._h:
            lib().ora_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_particles(self):
        return lib().ora_num_particles(self._h)

    def add_particles(self, x, u=None, omega=None, radius=None, mass=None, inertia=None):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        n = x.shape[0]
        u, omega = _vec3(u, n), _vec3(omega, n)
        r = np.ascontiguousarray(np.broadcast_to(radius, (n,)), dtype=np.float64)
        m = np.ascontiguousarray(np.broadcast_to(mass, (n,)), dtype=np.float64)
        I = np.ascontiguousarray(np.broadcast_to(inertia, (n,)), dtype=np.float64)
        first = lib().ora_add_particles(self._h, n, _d(x), _d(u), _d(omega), _d(r), _d(m), _d(I))
        if first < 0:
            raise ValueError("invalid particles")
        return first

    def step(self, n=1):
        lib().ora_step(self._h, int(n))

    def forces(self):
        n = self.n_particles
        F, T, x, u, om = (np.zeros((n, 3)) for _ in range(5))
        lib().ora_forces(self._h, _d(F), _d(T), _d(x), _d(u), _d(om))
        return F, T, x, u, om

    def fields(self):
        rho = np.zeros(self.N)
        u = np.zeros((self.N, 3))
        own = np.zeros(self.N, dtype=np.int32)
        lib().ora_fields(self._h, _d(rho), _d(u), own.ctypes.data_as(_ip))
        shp = (self.nz, self.ny, self.nx)
        return rho.reshape(shp), u.reshape(shp + (3,)), own.reshape(shp)

    def site_kind(self):
        k = np.zeros(self.N, dtype=np.int8)
        lib().ora_site_kind(self._h, k.ctypes.data_as(_bp))
        return k.reshape(self.nz, self.ny, self.nx)

    def shifts(self):
        k = np.zeros((self.n_particles, 3), dtype=np.int32)
        lib().ora_shifts(self._h, k.ctypes.data_as(_ip))
        return k

    def get_f(self):
        f = np.zeros((self.q, self.N))
        lib().ora_get_f(self._h, _d(f))
        return f.reshape(self.q, self.nz, self.ny, self.nx)

    def get_fs(self):
        """Last step's post-collision, post-substep distributions."""
        f = np.zeros((self.q, self.N))
        lib().ora_get_fs(self._h, _d(f))
        return f.reshape(self.q, self.nz, self.ny, self.nx)

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.q, self.N)
        lib().ora_set_f(self._h, _d(f))

    def template(self, p):
        nbs = np.zeros(1, dtype=np.int32)
        nis = np.zeros(1, dtype=np.int32)
        lib().ora_template(self._h, p, nbs.ctypes.data_as(_ip), nis.ctypes.data_as(_ip), None, None)
        n = int(nbs[0] + nis[0])
        off = np.zeros((max(n, 1), 3), dtype=np.int32)
        kind = np.zeros(max(n, 1), dtype=np.int8)
        lib().ora_template(self._h, p, None, None, off.ctypes.data_as(_ip), kind.ctypes.data_as(_bp))
        return off[:n], kind[:n]

    def set_closure(self, params, h_max=2.0):
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        if lib().ora_set_closure(self._h, _d(p), float(h_max)) != 0:
            raise ValueError("invalid closure parameters")

    def closure_inputs(self, i, j):
        x = np.zeros(8)
        if lib().ora_closure_inputs(self._h, int(i), int(j), _d(x)) != 0:
            raise ValueError("invalid pair")
        return x

    def diagnostics(self):
        d = np.zeros(17)
        lib().ora_diagnostics(self._h, _d(d))
        return {"mass": d[0], "momentum": d[1:4].copy(), "is_leak": d[4:7].copy(),
                "conflicts": int(d[7]), "fragility": d[8], "min_gap": d[9],
                "step": int(d[10]), "body_force": d[11:14].copy(), "wall_momentum": d[14:17].copy()}
