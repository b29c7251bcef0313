"""FP64 CPU oracle of the incompressible DUGKS step (arXiv:1411.6121).

TEST INFRASTRUCTURE ONLY.  The product package never imports this module; only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It wraps ``liboracle.so`` (plain C, built by
``oracle/build.py``) through ctypes and shares no code with the HIP path.

Configurations are plain dicts with the keys::

    lattice   9 (D2Q9), 19 (D3Q19) or 27 (D3Q27)
    n         (nx, ny, nz)            nz = 1 for D2Q9
    L         (Lx, Ly, Lz)
    mesh      (kx, ky, kz)            0 uniform, 1 tanh-stretched, 2 custom, per axis
    faces     per axis: face coordinates of a custom axis (n+1 values from
              0 to L), else None
    k_stretch tanh constant k
    rho0, RT, tau, dt
    G         uniform acceleration (3)
    omega, phase                      g(t) = cos(omega t + phase)
    bc        6 side codes (-x,+x,-y,+y,-z,+z): 0 periodic, 1 NEQ velocity,
              2 NEQ pressure, 3 bounce-back
    uw        6 x 3 wall velocities, pw  6 wall pressures, pw_osc  6
              oscillating parts of the wall pressures (pw + pw_osc g(t))
    model     0 incompressible (default), 1 original DUGKS equilibrium

Arrays: distributions ``f[q, z, y, x]``, vector fields ``v[d, z, y, x]``,
scalar fields ``s[z, y, x]``; float64, C-contiguous.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

PERIODIC, NEQ_VELOCITY, NEQ_PRESSURE, BOUNCE_BACK = 0, 1, 2, 3


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int),
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


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b

            _b.build()
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(ctypes.c_double)
        C = ctypes.POINTER(_Cfg)
        lib.oracle_lattice.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), P]
        lib.oracle_mesh.argtypes = [C, ctypes.c_int, P, P]
        lib.oracle_feq.argtypes = [C, ctypes.c_double, P, P]
        lib.oracle_force_term.argtypes = [C, ctypes.c_double, P, P, P]
        lib.oracle_init.argtypes = [C, P, P, P, ctypes.c_double, P]
        lib.oracle_step.argtypes = [C, P, P, P, ctypes.c_double]
        lib.oracle_run.argtypes = [C, P, P, P, ctypes.c_double, ctypes.c_int]
        lib.oracle_interface_values.argtypes = [C, ctypes.c_int, P, P]
        lib.oracle_moments.argtypes = [C, P, P, ctypes.c_double, P, P, P, P]
        lib.oracle_step_adjoint.argtypes = [C, P, P, ctypes.c_double, P, P, P]
        lib.oracle_init_adjoint.argtypes = [C, P, P, ctypes.c_double, P, P, P]
        lib.oracle_threads.argtypes = []
        _lib = lib
    return _lib


def _cfg(d: dict) -> _Cfg:
    c = _Cfg()
    c.lattice = int(d["lattice"])
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
    c._faces = []  # keeps custom face arrays alive while the struct is in use
    faces = d.get("faces") or (None, None, None)
    for a in range(3):
        X = faces[a] if a < len(faces) else None
        if X is not None:
            X = np.ascontiguousarray(X, dtype=np.float64)
            c._faces.append(X)
            c.faces[a] = X.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return c


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _arr(a):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected the configuration (rc={rc})")


def dims(d: dict):
    D = 2 if int(d["lattice"]) == 9 else 3
    Q = int(d["lattice"])
    nx, ny, nz = (int(v) for v in d["n"])
    return D, Q, (nz, ny, nx)


def lattice(lat: int):
    lib = _load()
    e = (ctypes.c_int * 81)()
    w = (ctypes.c_double * 27)()
    Q = lib.oracle_lattice(lat, e, w)
    if Q < 0:
        raise ValueError("unknown lattice")
    return np.array(e[: 3 * Q], dtype=np.int64).reshape(Q, 3), np.array(w[:Q])


def mesh(d: dict, axis: int):
    lib = _load()
    N = int(d["n"][axis])
    faces = np.zeros(N + 1)
    centres = np.zeros(N + 2)
    _check(lib.oracle_mesh(ctypes.byref(_cfg(d)), axis, _p(faces), _p(centres)), "mesh")
    return faces, centres


def feq(d: dict, rho: float, u):
    lib = _load()
    _, Q, _ = dims(d)
    uu = np.zeros(3)
    uu[: len(u)] = u
    out = np.zeros(Q)
    _check(lib.oracle_feq(ctypes.byref(_cfg(d)), rho, _p(uu), _p(out)), "feq")
    return out


def force_term(d: dict, rho: float, u, G):
    lib = _load()
    _, Q, _ = dims(d)
    uu = np.zeros(3)
    uu[: len(u)] = u
    gg = np.zeros(3)
    gg[: len(G)] = G
    out = np.zeros(Q)
    _check(lib.oracle_force_term(ctypes.byref(_cfg(d)), rho, _p(uu), _p(gg), _p(out)), "S")
    return out


def init(d: dict, rho=None, u=None, force=None, t0: float = 0.0):
    lib = _load()
    D, Q, shp = dims(d)
    rho, u, force = _arr(rho), _arr(u), _arr(force)
    f = np.zeros((Q,) + shp)
    _check(lib.oracle_init(ctypes.byref(_cfg(d)), _p(rho), _p(u), _p(force), t0, _p(f)), "init")
    return f


def step(d: dict, f, force=None, t: float = 0.0):
    lib = _load()
    f = _arr(f)
    force = _arr(force)
    out = np.empty_like(f)
    _check(lib.oracle_step(ctypes.byref(_cfg(d)), _p(f), _p(out), _p(force), t), "step")
    return out


def run(d: dict, f, nsteps: int, force=None, t0: float = 0.0):
    """nsteps steps from t0; step i starts at t0 + i dt"""
    lib = _load()
    f = _arr(f)
    force = _arr(force)
    out = np.empty_like(f)
    _check(lib.oracle_run(ctypes.byref(_cfg(d)), _p(f), _p(out), _p(force), t0, int(nsteps)), "run")
    return out


def interface_values(d: dict, axis: int, phi):
    """f-bar on every interface of `axis` (Eq. (gradient), before wall rules)
    from f-bar-plus values phi[q, z, y, x] at the centres; returns
    [q, z, y, x] with n+1 entries along `axis`"""
    lib = _load()
    D, Q, shp = dims(d)
    phi = _arr(phi)
    assert phi.shape == (Q,) + shp
    fshp = list(shp)
    fshp[2 - axis] += 1
    out = np.zeros((Q,) + tuple(fshp))
    _check(lib.oracle_interface_values(ctypes.byref(_cfg(d)), int(axis), _p(phi), _p(out)), "interface_values")
    return out


def moments(d: dict, f, force=None, t: float = 0.0):
    """returns rho[z,y,x], u[D,z,y,x], p[z,y,x], totals[6]"""
    lib = _load()
    D, Q, shp = dims(d)
    f = _arr(f)
    force = _arr(force)
    rho = np.zeros(shp)
    u = np.zeros((D,) + shp)
    p = np.zeros(shp)
    tot = np.zeros(6)
    _check(lib.oracle_moments(ctypes.byref(_cfg(d)), _p(f), _p(force), t, _p(rho), _p(u), _p(p), _p(tot)),
           "moments")
    return rho, u, p, tot


def step_adjoint(d: dict, f, lam, force=None, t: float = 0.0, grad_force=None):
    """lam_n = J^T lam; grad_force (array [D,z,y,x]) accumulated in place if given"""
    lib = _load()
    f, lam, force = _arr(f), _arr(lam), _arr(force)
    out = np.empty_like(lam)
    if grad_force is not None:
        assert grad_force.dtype == np.float64 and grad_force.flags["C_CONTIGUOUS"]
    rc = lib.oracle_step_adjoint(ctypes.byref(_cfg(d)), _p(f), _p(force), t, _p(lam), _p(out),
                                 _p(grad_force))
    _check(rc, "step_adjoint")
    return out


def init_adjoint(d: dict, lam0, u=None, force=None, t0: float = 0.0, grad_u=None, grad_force=None):
    lib = _load()
    lam0, u, force = _arr(lam0), _arr(u), _arr(force)
    rc = lib.oracle_init_adjoint(ctypes.byref(_cfg(d)), _p(u), _p(force), t0, _p(lam0), _p(grad_u),
                                 _p(grad_force))
    _check(rc, "init_adjoint")


def threads() -> int:
    return int(_load().oracle_threads())
