"""MI355X (gfx950) incompressible DUGKS with body force (arXiv:1411.6121).

Thin ctypes binding of ``libdugks.so`` (see ``include/dugks.h``).  The names
``dugks_init``, ``dugks_step``, ... mirror the C entry points one to one and
only marshal arguments: every stage of the step runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  There is no CPU
fallback: without the built library every call raises.

Configurations are plain dicts (keys as in ``dugks_config``)::

    lattice 9|19|27, dtype "f32"|"f64", n (3), L (3), mesh (3), k_stretch,
    rho0, RT, tau, dt, G (3), omega, phase, bc (6), uw (6x3), pw (6),
    model (0 incompressible, 1 original DUGKS equilibrium), faces (3 host
    arrays, custom meshes), pw_osc (6: oscillating part of the wall pressures)

Tensors: state ``[Q, nz, ny, nx]``, vector fields ``[D, nz, ny, nx]``,
scalars ``[nz, ny, nx]``, all contiguous on the CUDA (HIP) device, in the
configuration's dtype.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdugks.so")

PERIODIC, NEQ_VELOCITY, NEQ_PRESSURE, BOUNCE_BACK = 0, 1, 2, 3
UNIFORM, TANH = 0, 1
OK, EINVAL, EUNSUPPORTED, EHIP, ENONFINITE, ENOMEM = 0, -1, -2, -3, -4, -5


class DugksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dugks error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int),
        ("dtype", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("L", ctypes.c_double * 3),
        ("mesh", ctypes.c_int * 3),
        ("k_stretch", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("RT", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("G", ctypes.c_double * 3),
        ("omega", ctypes.c_double),
        ("phase", ctypes.c_double),
        ("bc", ctypes.c_int * 6),
        ("uw", (ctypes.c_double * 3) * 6),
        ("pw", ctypes.c_double * 6),
        ("model", ctypes.c_int),
        ("faces", ctypes.POINTER(ctypes.c_double) * 3),
        ("pw_osc", ctypes.c_double * 6),
    ]


_lib = None
_VP = ctypes.c_void_p


def library_path() -> str:
    return LIB_PATH


def load():
    """Load libdugks.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or python -m paper_1411_6121_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    CP = ctypes.POINTER(Config)
    D = ctypes.c_double
    I = ctypes.c_int
    lib.dugks_version.restype = ctypes.c_char_p
    lib.dugks_last_error.restype = ctypes.c_char_p
    lib.dugks_last_error.argtypes = [_VP]
    lib.dugks_dt_from_cfl.restype = D
    lib.dugks_dt_from_cfl.argtypes = [CP, D]
    lib.dugks_init.argtypes = [CP, _VP, _VP, _VP, _VP, _VP, ctypes.POINTER(_VP)]
    lib.dugks_reset.argtypes = [_VP, _VP, _VP, _VP, D, _VP, _VP]
    lib.dugks_step.argtypes = [_VP, _VP, _VP, _VP, D, _VP]
    lib.dugks_run.argtypes = [_VP, _VP, _VP, _VP, D, I, _VP, ctypes.POINTER(I)]
    lib.dugks_moments.argtypes = [_VP, _VP, _VP, D, _VP, _VP, _VP, ctypes.POINTER(D), _VP]
    lib.dugks_totals_async.argtypes = [_VP, _VP, _VP, D, _VP, _VP]
    lib.dugks_velocity_change.argtypes = [_VP, _VP, _VP, _VP, D, D, ctypes.POINTER(D), _VP]
    lib.dugks_step_adjoint.argtypes = [_VP, _VP, _VP, D, _VP, _VP, _VP, _VP]
    lib.dugks_step_adjoint_static.argtypes = [_VP, _VP, _VP, D, _VP, _VP, _VP, _VP]
    lib.dugks_init_vjp.argtypes = [_VP, _VP, _VP, D, _VP, _VP, _VP, _VP]
    lib.dugks_moments_vjp.argtypes = [_VP, _VP, _VP, D, _VP, _VP, _VP]
    lib.dugks_kernel_variant.argtypes = [_VP]
    lib.dugks_destroy.argtypes = [_VP]
    lib.dugks_destroy.restype = None
    lib.dugks_batch_create.argtypes = [CP, I, ctypes.POINTER(ctypes.c_int64), _VP, ctypes.POINTER(_VP)]
    lib.dugks_batch_init.argtypes = [_VP, _VP, _VP]
    lib.dugks_batch_run.argtypes = [_VP, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_int64), I, I, _VP,
                                    ctypes.POINTER(I)]
    lib.dugks_batch_step.argtypes = [_VP, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_int64), I, _VP, ctypes.POINTER(I)]
    lib.dugks_batch_destroy.argtypes = [_VP]
    lib.dugks_batch_destroy.restype = None
    lib.dugks_batch_tune.restype = I
    lib.dugks_batch_tune.argtypes = [_VP, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_int64), I, _VP,
                                     ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.dugks_batch_last_error.restype = ctypes.c_char_p
    lib.dugks_batch_last_error.argtypes = [_VP]
    _lib = lib
    return lib


def config(d: dict) -> Config:
    c = Config()
    c.lattice = int(d["lattice"])
    dt = d.get("dtype", "f64")
    c.dtype = 1 if dt in ("f64", "float64", 1) else 0
    for a in range(3):
        c.n[a] = int(d["n"][a])
        c.L[a] = float(d["L"][a])
        c.mesh[a] = int(d.get("mesh", (0, 0, 0))[a])
        c.G[a] = float(d.get("G", (0.0, 0.0, 0.0))[a])
    c.k_stretch = float(d.get("k_stretch", 0.0))
    c.rho0 = float(d["rho0"])
    c.RT = float(d["RT"])
    c.tau = float(d["tau"])
    c.dt = float(d["dt"])
    c.omega = float(d.get("omega", 0.0))
    c.phase = float(d.get("phase", 0.0))
    c.model = int(d.get("model", 0))
    uw = d.get("uw", [[0.0] * 3] * 6)
    pw = d.get("pw", [0.0] * 6)
    pwo = d.get("pw_osc", [0.0] * 6)
    for s in range(6):
        c.bc[s] = int(d["bc"][s])
        c.pw[s] = float(pw[s])
        c.pw_osc[s] = float(pwo[s])
        for a in range(3):
            c.uw[s][a] = float(uw[s][a])
    # custom face coordinates (mesh kind 2): host float64 arrays, kept alive
    # by the Config object for the duration of the call that reads them
    c._faces = []
    faces = d.get("faces") or (None, None, None)
    for a in range(3):
        X = faces[a] if a < len(faces) else None
        if X is None:
            c.faces[a] = None
        else:
            X = np.ascontiguousarray(X, dtype=np.float64)
            c._faces.append(X)
            c.faces[a] = X.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return c


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(rc, ctx=None):
    if rc != OK:
        msg = load().dugks_last_error(ctx)
        raise DugksError(rc, msg.decode() if msg else "")


def version() -> str:
    return load().dugks_version().decode()


def dugks_dt_from_cfl(cfg: dict, cfl: float) -> float:
    v = load().dugks_dt_from_cfl(ctypes.byref(config(cfg)), float(cfl))
    if v < 0:
        raise DugksError(EINVAL, "invalid configuration")
    return v


def dugks_init(cfg: dict, f_out, rho=None, u=None, force=None, stream=None):
    """returns an opaque context handle (int); writes f~0 into f_out"""
    lib = load()
    h = ctypes.c_void_p()
    rc = lib.dugks_init(ctypes.byref(config(cfg)), _ptr(rho), _ptr(u), _ptr(force), _ptr(f_out), _stream(stream),
                        ctypes.byref(h))
    _check(rc, None)
    return h.value


def dugks_reset(ctx, f_out, rho=None, u=None, force=None, t0=0.0, stream=None):
    _check(load().dugks_reset(_VP(ctx), _ptr(rho), _ptr(u), _ptr(force), float(t0), _ptr(f_out),
                              _stream(stream)), _VP(ctx))


def dugks_step(ctx, f_in, f_out, force=None, t_n=0.0, stream=None):
    _check(load().dugks_step(_VP(ctx), _ptr(f_in), _ptr(f_out), _ptr(force), float(t_n), _stream(stream)),
           _VP(ctx))


def dugks_run(ctx, f_a, f_b, nsteps, force=None, t0=0.0, stream=None) -> int:
    which = ctypes.c_int(0)
    _check(load().dugks_run(_VP(ctx), _ptr(f_a), _ptr(f_b), _ptr(force), float(t0), int(nsteps), _stream(stream),
                            ctypes.byref(which)), _VP(ctx))
    return which.value


def dugks_moments(ctx, f, force=None, t=0.0, rho=None, u=None, p=None, totals=True, stream=None):
    """fills the given output tensors; returns the 6 totals (synchronises) or None"""
    tot = (ctypes.c_double * 6)() if totals else None
    rc = load().dugks_moments(_VP(ctx), _ptr(f), _ptr(force), float(t), _ptr(rho), _ptr(u), _ptr(p),
                              tot, _stream(stream))
    _check(rc, _VP(ctx))
    return list(tot) if totals else None


def dugks_totals_async(ctx, f, out, force=None, t=0.0, stream=None):
    """totals of dugks_moments into the device tensor `out` (6 float64
    values, e.g. a row of a history buffer), in stream order, no sync"""
    _check(load().dugks_totals_async(_VP(ctx), _ptr(f), _ptr(force), float(t), _ptr(out), _stream(stream)),
           _VP(ctx))


def dugks_velocity_change(ctx, f_a, f_b, force=None, t_a=0.0, t_b=0.0, stream=None):
    """(sqrt(sum |u_b - u_a|^2), sqrt(sum |u_b|^2)) over the cells for the
    states f_a at t_a and f_b at t_b; their ratio is the steady/periodic
    convergence criterion of Sec. III (synchronises)"""
    out = (ctypes.c_double * 2)()
    _check(load().dugks_velocity_change(_VP(ctx), _ptr(f_a), _ptr(f_b), _ptr(force), float(t_a), float(t_b), out,
                                        _stream(stream)), _VP(ctx))
    return out[0], out[1]


def dugks_step_adjoint(ctx, f_n, lam_np1, lam_n, force=None, t_n=0.0, grad_force=None, stream=None):
    _check(load().dugks_step_adjoint(_VP(ctx), _ptr(f_n), _ptr(force), float(t_n), _ptr(lam_np1), _ptr(lam_n),
                                     _ptr(grad_force), _stream(stream)), _VP(ctx))


def dugks_step_adjoint_static(ctx, f_n, lam_np1, lam_n, force=None, t_n=0.0, grad_force=None, stream=None):
    """dugks_step_adjoint with its scratch in the library's static device
    area (no device allocation; problems up to 64 MiB of scratch)"""
    _check(load().dugks_step_adjoint_static(_VP(ctx), _ptr(f_n), _ptr(force), float(t_n), _ptr(lam_np1),
                                            _ptr(lam_n), _ptr(grad_force), _stream(stream)), _VP(ctx))


def dugks_init_vjp(ctx, lam0, u=None, force=None, t0=0.0, grad_u=None, grad_force=None, stream=None):
    _check(load().dugks_init_vjp(_VP(ctx), _ptr(u), _ptr(force), float(t0), _ptr(lam0), _ptr(grad_u),
                                 _ptr(grad_force), _stream(stream)), _VP(ctx))


def dugks_moments_vjp(ctx, lam, grad_rho=None, grad_u=None, t=0.0, grad_force=None, stream=None):
    _check(load().dugks_moments_vjp(_VP(ctx), _ptr(grad_rho), _ptr(grad_u), float(t), _ptr(lam), _ptr(grad_force),
                                    _stream(stream)), _VP(ctx))


def dugks_kernel_variant(ctx) -> int:
    return int(load().dugks_kernel_variant(_VP(ctx)))


def dugks_destroy(ctx):
    if ctx:
        load().dugks_destroy(_VP(ctx))


def shape_of(cfg: dict):
    """(Q, D, (nz, ny, nx)) of a configuration dict"""
    Q = int(cfg["lattice"])
    D = 2 if Q == 9 else 3
    n = cfg["n"]
    return Q, D, (int(n[2]), int(n[1]), int(n[0]))


def torch_dtype(cfg: dict):
    import torch

    return torch.float64 if cfg.get("dtype", "f64") in ("f64", "float64", 1) else torch.float32


class Solver:
    """Owns a context and a ping-pong pair of state tensors on one device."""

    def __init__(self, cfg: dict, rho=None, u=None, force=None, device="cuda"):
        import torch

        self.cfg = dict(cfg)
        self.Q, self.D, self.shape = shape_of(cfg)
        self.dtype = torch_dtype(cfg)
        self.device = torch.device(device)
        self.f = torch.empty((self.Q,) + self.shape, dtype=self.dtype, device=self.device)
        self.g = torch.empty_like(self.f)
        self.force = force
        self.t = 0.0
        self.ctx = dugks_init(self.cfg, self.f, rho, u, force)

    def step(self, nsteps: int = 1):
        which = dugks_run(self.ctx, self.f, self.g, nsteps, self.force, self.t)
        if which:
            self.f, self.g = self.g, self.f
        self.t += nsteps * float(self.cfg["dt"])
        return self.f

    def moments(self, totals=True):
        import torch

        rho = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        u = torch.empty((self.D,) + self.shape, dtype=self.dtype, device=self.device)
        p = torch.empty_like(rho)
        tot = dugks_moments(self.ctx, self.f, self.force, self.t, rho, u, p, totals)
        return rho, u, p, tot

    def close(self):
        if self.ctx:
            dugks_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _align(n, a):
    return (n + a - 1) // a * a


class BatchSolver:
    """Many independent instances (same lattice and dtype) advanced together:
    one kernel launch per step for all of them, optionally replayed from a
    captured hipGraph.  State of instance i: ``solver.state(i)``."""

    def __init__(self, cfgs, device="cuda", forces=None):
        import torch

        if not cfgs:
            raise ValueError("need at least one instance")
        self.cfgs = [dict(c) for c in cfgs]
        self.dtype = torch_dtype(self.cfgs[0])
        esize = 8 if self.dtype == torch.float64 else 4
        per = 256 // esize  # 256-byte aligned instance offsets
        self.offsets, self.shapes = [], []
        tot = 0
        for c in self.cfgs:
            Q, D, shp = shape_of(c)
            self.offsets.append(tot)
            self.shapes.append((Q,) + shp)
            tot += _align(Q * shp[0] * shp[1] * shp[2], per)
        self.total = tot
        self.device = torch.device(device)
        self.f = torch.empty(tot, dtype=self.dtype, device=self.device)
        self.g = torch.empty_like(self.f)
        n = len(self.cfgs)
        keep = [config(c) for c in self.cfgs]  # owns any custom face arrays until the create call returns
        arr = (Config * n)(*keep)
        offs = (ctypes.c_int64 * n)(*self.offsets)
        h = ctypes.c_void_p()
        lib = load()
        rc = lib.dugks_batch_create(arr, n, offs, _stream(None), ctypes.byref(h))
        if rc != OK:
            raise DugksError(rc, lib.dugks_batch_last_error(None).decode())
        self.h = h.value
        self.forces, self.force_offsets = None, None
        if forces is not None:
            self.set_forces(forces)
        self._check(lib.dugks_batch_init(_VP(self.h), _ptr(self.f), _stream(None)))
        self.steps = 0
        self._graph_stream = None

    def _check(self, rc):
        if rc != OK:
            raise DugksError(rc, load().dugks_batch_last_error(_VP(self.h)).decode())

    def set_forces(self, forces):
        """forces: list (per instance) of [D, nz, ny, nx] tensors or None"""
        import torch

        esize = 8 if self.dtype == torch.float64 else 4
        per = 256 // esize
        offs, tot = [], 0
        for fr in forces:
            offs.append(tot if fr is not None else -1)
            if fr is not None:
                tot += _align(fr.numel(), per)
        buf = torch.zeros(max(tot, 1), dtype=self.dtype, device=self.device)
        for fr, o in zip(forces, offs):
            if fr is not None:
                buf[o:o + fr.numel()] = fr.reshape(-1)
        self.forces = buf
        self.force_offsets = (ctypes.c_int64 * len(offs))(*offs)

    def state(self, i):
        o = self.offsets[i]
        Q, nz, ny, nx = self.shapes[i]
        return self.f[o:o + Q * nz * ny * nx].view(Q, nz, ny, nx)

    def run(self, nsteps, use_graph=False):
        import torch

        which = ctypes.c_int(0)
        lib = load()
        if use_graph:
            if self._graph_stream is None:
                self._graph_stream = torch.cuda.Stream(device=self.device)
            cur = torch.cuda.current_stream(self.device)
            self._graph_stream.wait_stream(cur)
            with torch.cuda.stream(self._graph_stream):
                self._check(lib.dugks_batch_run(_VP(self.h), _ptr(self.f), _ptr(self.g), _ptr(self.forces),
                                                self.force_offsets, int(nsteps), 1,
                                                ctypes.c_void_p(self._graph_stream.cuda_stream),
                                                ctypes.byref(which)))
            cur.wait_stream(self._graph_stream)
        else:
            self._check(lib.dugks_batch_run(_VP(self.h), _ptr(self.f), _ptr(self.g), _ptr(self.forces),
                                            self.force_offsets, int(nsteps), 0, _stream(None),
                                            ctypes.byref(which)))
        if which.value:
            self.f, self.g = self.g, self.f
        self.steps += int(nsteps)
        return self.f

    def tune(self, nsteps=3):
        """Pick the fastest tile shape and march chunk for this batch
        (dugks_batch_tune) on scratch copies of the current state; the state
        and the batch clock are unchanged.  Returns (tile_variant, chunk)."""
        import torch

        a = self.f.clone()
        b = torch.empty_like(a)
        tile, chunk = ctypes.c_int(0), ctypes.c_int(0)
        self._check(load().dugks_batch_tune(_VP(self.h), _ptr(a), _ptr(b), _ptr(self.forces), self.force_offsets,
                                            int(nsteps), _stream(None), ctypes.byref(tile), ctypes.byref(chunk)))
        del a, b
        return tile.value, chunk.value

    def close(self):
        if self.h:
            load().dugks_batch_destroy(_VP(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
