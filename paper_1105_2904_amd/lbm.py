"""Thin ctypes binding of the C ABI in include/lbm.h.

Argument marshalling only: every step of the method runs in the HIP kernels
of ``liblbm.so``.  PyTorch provides the device workspace and the stream.
The module-level ``lbm_*`` functions mirror the C entry points one to one;
``Simulation`` bundles a context with its workspace tensor.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_D2Q9, LBM_D3Q19 = 9, 19
LBM_FP64, LBM_FP32, LBM_FP16, LBM_BF16 = 0, 1, 2, 3
STORAGE = {"fp64": LBM_FP64, "fp32": LBM_FP32, "fp16": LBM_FP16, "bf16": LBM_BF16}
LBM_OK = 0
LBM_EINVAL, LBM_EWORKSPACE, LBM_EHIP, LBM_EOVERLAP = -1, -2, -3, -4
LBM_ECAPACITY, LBM_ENONFINITE, LBM_EUNSUPPORTED, LBM_ECOLLISION = -5, -6, -7, -8
LBM_ESTATE = -9


class LbmError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed: %s (%d)" % (what, lbm_strerror(code), code))
        self.code = code


class lbm_params(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
                ("gravity", ctypes.c_double * 3), ("body_force", ctypes.c_double * 3),
                ("zero_net_force", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("max_particles", ctypes.c_int32), ("max_radius", ctypes.c_double),
                ("walls", ctypes.c_int32), ("wall_velocity", ctypes.c_double * 18), ("aa", ctypes.c_int32)]


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lib = None


def lib():
    """Load liblbm.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is not built; run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(lbm_params)
        vp = ctypes.c_void_p
        sig = {
            "lbm_workspace_size": [P, ctypes.POINTER(ctypes.c_size_t)],
            "lbm_create": [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)],
            "lbm_add_particles": [vp, ctypes.c_int32, _dp, _dp, _dp, _dp, _dp, _dp, _ip],
            "lbm_step": [vp, ctypes.c_int32],
            "lbm_forces": [vp, _dp, _dp, _dp, _dp, _dp],
            "lbm_fields": [vp, _dp, _dp, _ip],
            "lbm_destroy": [vp],
            "lbm_get_distributions": [vp, _dp],
            "lbm_set_distributions": [vp, _dp],
            "lbm_site_kind": [vp, ctypes.POINTER(ctypes.c_int8)],
            "lbm_shifts": [vp, _ip],
            "lbm_particle_info": [vp, ctypes.c_int32, _ip, _ip],
            "lbm_set_profiling": [vp, ctypes.c_int32],
            "lbm_profile": [vp, _dp, ctypes.POINTER(ctypes.c_int64)],
            "lbm_bytes_per_site": [P, ctypes.POINTER(ctypes.c_int64)],
            "lbm_device_copy": [vp, vp, ctypes.c_size_t, ctypes.c_int32, vp],
            "lbm_ensemble_workspace_size": [P, ctypes.c_int32, _ip, ctypes.POINTER(ctypes.c_size_t)],
            "lbm_ensemble_create": [P, ctypes.c_int32, _ip, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)],
            "lbm_ensemble_add_particles": [vp, ctypes.c_int32, ctypes.c_int32, _dp, _dp, _dp, _dp, _dp, _dp, _ip],
            "lbm_box_info": [vp, ctypes.c_int32, _ip, ctypes.POINTER(ctypes.c_int64), _ip, _ip],
            "lbm_set_sweep_config": [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
            "lbm_get_sweep_config": [vp, _ip, _ip, _ip],
            "lbm_autotune": [vp, ctypes.c_int32, _ip, _ip, _ip, _dp],
            "lbm_autotune_steps": [vp, ctypes.c_int32, _ip, _ip, _ip, _dp, ctypes.POINTER(ctypes.c_int64)],
            "lbm_set_graph": [vp, ctypes.c_int32],
            "lbm_step_noalloc": [vp, ctypes.c_int32],
            "lbm_set_closure": [vp, vp, ctypes.c_double],
            "lbm_closure_inputs": [ctypes.c_int32, _dp, _dp, _dp, _dp, ctypes.c_double, vp],
            "lbm_mlp_param_count": [_ip],
            "lbm_mlp_forward": [vp, vp, vp, ctypes.c_int64, vp],
            "lbm_mlp_gradient": [vp, vp, vp, ctypes.c_int32, ctypes.c_float, vp, vp, vp],
            "lbm_mlp_train": [vp, vp, vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_float, ctypes.c_float, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.lbm_strerror.argtypes = [ctypes.c_int]
        L.lbm_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def lbm_strerror(code):
    return lib().lbm_strerror(int(code)).decode()


def _check(code, what):
    if code != LBM_OK:
        raise LbmError(code, what)


def _d(a):
    return None if a is None else a.ctypes.data_as(_dp)


def make_params(lattice, nx, ny, nz=1, tau=1.0, rho0=1.0, gravity=(0, 0, 0), body_force=(0, 0, 0),
                zero_net_force=False, storage="fp32", max_particles=0, max_radius=1.0, walls=0,
                wall_velocity=None, aa=False):
    p = lbm_params()
    p.lattice, p.nx, p.ny, p.nz = int(lattice), int(nx), int(ny), int(nz)
    p.tau, p.rho0 = float(tau), float(rho0)
    for a in range(3):
        p.gravity[a] = float(gravity[a])
        p.body_force[a] = float(body_force[a])
    p.zero_net_force = int(bool(zero_net_force))
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.max_particles = int(max_particles)
    p.max_radius = float(max_radius)
    p.walls = int(walls)
    if wall_velocity is not None:
        wu = np.asarray(wall_velocity, dtype=np.float64).reshape(18)
        for k in range(18):
            p.wall_velocity[k] = float(wu[k])
    p.aa = int(bool(aa))
    return p


def lbm_workspace_size(params):
    n = ctypes.c_size_t(0)
    _check(lib().lbm_workspace_size(ctypes.byref(params), ctypes.byref(n)), "lbm_workspace_size")
    return n.value


def lbm_bytes_per_site(params):
    n = ctypes.c_int64(0)
    _check(lib().lbm_bytes_per_site(ctypes.byref(params), ctypes.byref(n)), "lbm_bytes_per_site")
    return n.value


def lbm_create(params, workspace_ptr, workspace_bytes, stream_handle):
    ctx = ctypes.c_void_p()
    _check(lib().lbm_create(ctypes.byref(params), ctypes.c_void_p(workspace_ptr), workspace_bytes,
                            ctypes.c_void_p(stream_handle), ctypes.byref(ctx)), "lbm_create")
    return ctx


def lbm_device_copy(dst_ptr, src_ptr, nbytes, stream_handle, streaming_loads=True):
    _check(lib().lbm_device_copy(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), nbytes,
                                 int(bool(streaming_loads)), ctypes.c_void_p(stream_handle)), "lbm_device_copy")


def _vec3(a, n):
    if a is None:
        return np.zeros((n, 3))
    return np.ascontiguousarray(a, dtype=np.float64).reshape(n, 3)


def _vec1(a, n):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (n,)))


def _dims(dims):
    d = np.ascontiguousarray(dims, dtype=np.int32).reshape(-1, 3)
    return d, d.ctypes.data_as(_ip)


def lbm_ensemble_workspace_size(params, dims):
    d, dp = _dims(dims)
    n = ctypes.c_size_t(0)
    _check(lib().lbm_ensemble_workspace_size(ctypes.byref(params), len(d), dp, ctypes.byref(n)),
           "lbm_ensemble_workspace_size")
    return n.value


class Simulation:
    """A context plus the torch workspace tensor it lives in."""

    def __init__(self, lattice, nx, ny, nz=1, tau=1.0, rho0=1.0, gravity=(0, 0, 0),
                 body_force=(0, 0, 0), zero_net_force=False, storage="fp32", max_particles=0,
                 max_radius=1.0, walls=0, wall_velocity=None, device="cuda", stream=None, boxes=None,
                 aa=False):
        """One box of nx x ny x nz sites, or with boxes = [[nx, ny, nz], ...]
        an ensemble of independent boxes stepped together (nx, ny, nz are then
        ignored).  aa=True keeps one population array updated in place (AA
        pattern) instead of two."""
        import torch
        self.params = make_params(lattice, nx, ny, nz, tau, rho0, gravity, body_force,
                                  zero_net_force, storage, max_particles, max_radius, walls,
                                  wall_velocity, aa)
        self.q = int(lattice)
        if boxes is None:
            self.dims = np.array([[int(nx), int(ny), int(nz)]], dtype=np.int32)
        else:
            self.dims = np.ascontiguousarray(boxes, dtype=np.int32).reshape(-1, 3)
        self.nx, self.ny, self.nz = (int(v) for v in self.dims[0])
        self.box_sites = self.dims.prod(axis=1).astype(np.int64)
        self.box_start = np.concatenate([[0], np.cumsum(self.box_sites)[:-1]])
        self.N = int(self.box_sites.sum())
        stream = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
        self.stream = stream
        if boxes is None:
            self.nbytes = lbm_workspace_size(self.params)
            self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
            self.ctx = lbm_create(self.params, self.workspace.data_ptr(), self.nbytes, stream.cuda_stream)
        else:
            self.nbytes = lbm_ensemble_workspace_size(self.params, self.dims)
            self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
            ctx = ctypes.c_void_p()
            _check(lib().lbm_ensemble_create(ctypes.byref(self.params), len(self.dims), _dims(self.dims)[1],
                                             ctypes.c_void_p(self.workspace.data_ptr()), self.nbytes,
                                             ctypes.c_void_p(stream.cuda_stream), ctypes.byref(ctx)),
                   "lbm_ensemble_create")
            self.ctx = ctx
        self.n_particles = 0

    def close(self):
        if getattr(self, "ctx", None):
            lib().lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_particles(self, x, u=None, omega=None, radius=None, mass=None, inertia=None, box=0):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        n = x.shape[0]
        first = ctypes.c_int32(-1)
        _check(lib().lbm_ensemble_add_particles(self.ctx, int(box), n, _d(x), _d(_vec3(u, n)),
                                                _d(_vec3(omega, n)), _d(_vec1(radius, n)),
                                                _d(_vec1(mass, n)), _d(_vec1(inertia, n)),
                                                ctypes.byref(first)), "lbm_ensemble_add_particles")
        self.n_particles += n
        return first.value

    def box_info(self, box):
        dims = np.zeros(3, dtype=np.int32)
        s0, p0, n = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().lbm_box_info(self.ctx, int(box), dims.ctypes.data_as(_ip), ctypes.byref(s0),
                                  ctypes.byref(p0), ctypes.byref(n)), "lbm_box_info")
        return dims, s0.value, p0.value, n.value

    def set_sweep_config(self, width, grid=0, blocks_per_cu=0):
        _check(lib().lbm_set_sweep_config(self.ctx, int(width), int(grid), int(blocks_per_cu)),
               "lbm_set_sweep_config")

    def sweep_config(self):
        """(width, grid, blocks_per_cu) of the sweep launch."""
        w, g, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().lbm_get_sweep_config(self.ctx, ctypes.byref(w), ctypes.byref(g), ctypes.byref(k)),
               "lbm_get_sweep_config")
        return w.value, g.value, k.value

    def autotune(self, reps=5):
        """Picks and sets the fastest sweep launch; returns (width, grid,
        blocks_per_cu, ms per sweep)."""
        w, g, k, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib().lbm_autotune(self.ctx, int(reps), ctypes.byref(w), ctypes.byref(g), ctypes.byref(k),
                                  ctypes.byref(ms)), "lbm_autotune")
        return w.value, g.value, k.value, ms.value

    def autotune_steps(self, steps=16):
        """Picks and sets the fastest sweep launch timed inside whole steps
        (`steps` per candidate: launches a percent apart need about 16 to rank
        reliably); returns (width, grid, blocks_per_cu, ms per step, steps it
        advanced the simulation by)."""
        w, g, k, ms, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double(), ctypes.c_int64()
        _check(lib().lbm_autotune_steps(self.ctx, int(steps), ctypes.byref(w), ctypes.byref(g), ctypes.byref(k),
                                        ctypes.byref(ms), ctypes.byref(n)), "lbm_autotune_steps")
        return w.value, g.value, k.value, ms.value, n.value

    def set_closure(self, params, h_max=2.0):
        """Near-contact closure with the network parameters `params` (a float32
        CUDA tensor) for gaps below h_max; params None switches it off."""
        p = None if params is None else _ptr(params)
        _check(lib().lbm_set_closure(self.ctx, p, float(h_max)), "lbm_set_closure")

    def set_graph(self, steps_per_graph):
        _check(lib().lbm_set_graph(self.ctx, int(steps_per_graph)), "lbm_set_graph")

    def step(self, n=1):
        _check(lib().lbm_step(self.ctx, int(n)), "lbm_step")

    def step_noalloc(self, n=1):
        _check(lib().lbm_step_noalloc(self.ctx, int(n)), "lbm_step_noalloc")

    def forces(self):
        n = self.n_particles
        F, T, x, u, om = (np.zeros((n, 3)) for _ in range(5))
        _check(lib().lbm_forces(self.ctx, _d(F), _d(T), _d(x), _d(u), _d(om)), "lbm_forces")
        return F, T, x, u, om

    def fields(self):
        rho = np.zeros(self.N)
        u = np.zeros((self.N, 3))
        own = np.zeros(self.N, dtype=np.int32)
        _check(lib().lbm_fields(self.ctx, _d(rho), _d(u), own.ctypes.data_as(_ip)), "lbm_fields")
        if len(self.dims) > 1:
            return rho, u, own  # sites of every box, box after box
        shp = (self.nz, self.ny, self.nx)
        return rho.reshape(shp), u.reshape(shp + (3,)), own.reshape(shp)

    def get_distributions(self):
        f = np.zeros((self.q, self.N))
        _check(lib().lbm_get_distributions(self.ctx, _d(f)), "lbm_get_distributions")
        if len(self.dims) > 1:
            return f
        return f.reshape(self.q, self.nz, self.ny, self.nx)

    def set_distributions(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.q, self.N)
        _check(lib().lbm_set_distributions(self.ctx, _d(f)), "lbm_set_distributions")

    def site_kind(self):
        k = np.zeros(self.N, dtype=np.int8)
        _check(lib().lbm_site_kind(self.ctx, k.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))),
               "lbm_site_kind")
        if len(self.dims) > 1:
            return k
        return k.reshape(self.nz, self.ny, self.nx)

    def shifts(self):
        k = np.zeros((self.n_particles, 3), dtype=np.int32)
        _check(lib().lbm_shifts(self.ctx, k.ctypes.data_as(_ip)), "lbm_shifts")
        return k

    def particle_info(self, p):
        nbs, nis = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().lbm_particle_info(self.ctx, int(p), ctypes.byref(nbs), ctypes.byref(nis)),
               "lbm_particle_info")
        return nbs.value, nis.value

    def set_profiling(self, on):
        _check(lib().lbm_set_profiling(self.ctx, int(bool(on))), "lbm_set_profiling")

    def profile(self):
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().lbm_profile(self.ctx, ctypes.byref(ms), ctypes.byref(n)), "lbm_profile")
        return ms.value, n.value


# ---- closure network: torch CUDA float32 tensors in, kernels of liblbm.so ----
def _ptr(t):
    import torch
    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous(), "float32 contiguous CUDA tensor expected"
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    return ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)


def mlp_param_count():
    n = ctypes.c_int32()
    _check(lib().lbm_mlp_param_count(ctypes.byref(n)), "lbm_mlp_param_count")
    return n.value


def mlp_forward(params, x, stream=None):
    """y [n, 2] of the network with flat parameters `params` on inputs x [n, 8]."""
    import torch
    y = torch.empty((x.shape[0], 2), dtype=torch.float32, device=x.device)
    _check(lib().lbm_mlp_forward(_ptr(params), _ptr(x), _ptr(y), x.shape[0], _stream(stream)), "lbm_mlp_forward")
    return y


def mlp_gradient(params, x, t, loss_scale=1024.0, stream=None):
    """(loss, gradient) over all rows."""
    import torch
    g = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=params.device)
    _check(lib().lbm_mlp_gradient(_ptr(params), _ptr(x), _ptr(t), x.shape[0], float(loss_scale), _ptr(g),
                                  _ptr(loss), _stream(stream)), "lbm_mlp_gradient")
    return loss, g


def mlp_train(params, adam_m, adam_v, x, t, batch, steps, step0=0, lr=1e-3, loss_scale=1024.0, stream=None):
    """Adam steps in place on params; returns the per-step losses."""
    import torch
    losses = torch.empty(max(steps, 1), dtype=torch.float32, device=params.device)
    _check(lib().lbm_mlp_train(_ptr(params), _ptr(adam_m), _ptr(adam_v), _ptr(x), _ptr(t), x.shape[0], int(batch),
                               int(steps), int(step0), float(lr), float(loss_scale), _ptr(losses), _stream(stream)),
           "lbm_mlp_train")
    return losses[:steps]


def closure_inputs(xi, d, ri, rj, tau):
    """Closure inputs [n, 8] (float32) for pairs with centre xi [n, 2] of the
    first particle, separation d [n, 2], radii ri, rj [n]."""
    xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1, 2)
    n = xi.shape[0]
    d = np.ascontiguousarray(d, dtype=np.float64).reshape(n, 2)
    ri = np.ascontiguousarray(np.broadcast_to(np.asarray(ri, dtype=np.float64), (n,)))
    rj = np.ascontiguousarray(np.broadcast_to(np.asarray(rj, dtype=np.float64), (n,)))
    out = np.zeros((n, 8), dtype=np.float32)
    _check(lib().lbm_closure_inputs(n, _d(xi), _d(d), _d(ri), _d(rj), float(tau),
                                    out.ctypes.data_as(ctypes.c_void_p)), "lbm_closure_inputs")
    return out
