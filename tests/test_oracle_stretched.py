"""Pins of the oracle's interface reconstruction and wall rules on walled and
stretched meshes.

Eq. (gradient) on a tanh mesh (Eq. (Nonuniform_mesh)) needs the linear
interpolation weights along the normal, the normal difference over the
centre distance, the tangential difference of the bilinear cross-point
values over the interface width, and the ghost extrapolation next to walls.
Three independent pins:

* exactness on fields linear in x (uniform and stretched, interior and wall
  interfaces): every stencil piece above reproduces a linear field exactly,
  so f-bar(x_b) must equal phi(x_b) - h xi . grad(phi) to rounding;
* a second statement of the whole step in whole-array numpy form
  (tests/brute_step.py: every wall kind, both mesh kinds, all lattices)
  agreeing to rounding on small meshes;
* second-order convergence of manufactured steady flows on meshes stretched
  in every wall-bounded axis (D2Q9, D3Q19 in a plane, D3Q19 fully 3-D).

Mutation check (done on a scratch copy of the oracle, not kept), each
planted mistake failing these tests:
* the two bilinear weights of the cross points swapped (wa <-> wb): the
  linear-field pin and the restatement;
* the tangential width taken from the neighbouring cell: all four groups
  except the 3-D box convergence;
* the normal interpolation weights swapped (w <-> 1-w): the linear-field
  pin and the restatement;
* the ghost value extrapolated from the wrong end of the two-cell pair:
  all four groups;
* the NEQ non-equilibrium part taken at the wall interface itself instead
  of the opposite interface of the wall cell: the restatement.
"""
import numpy as np
import pytest

import oracle as O
from synthetic import field, perturb, rng
from tests import brute_step as B

LID = [[0, 0, 0], [0, 0, 0], [0, 0, 0], [0.1, 0, 0], [0, 0, 0], [0, 0, 0]]


def cfg(lat, n, bc, **kw):
    d = dict(lattice=lat, n=n, L=tuple(float(v) for v in n), rho0=1.0, RT=1 / 3, tau=0.3, dt=0.4, bc=bc,
             k_stretch=1.7)
    d.update(kw)
    return d


def centres(d, a):
    _, xc = O.mesh(d, a)
    return xc[1:-1]


# --------------------------------------------------------------------------
# Eq. (gradient) on linear fields
# --------------------------------------------------------------------------
LINEAR = [
    cfg(9, (6, 7, 1), (1, 1, 1, 1, 0, 0), mesh=(1, 1, 0), k_stretch=2.5),
    cfg(9, (5, 4, 1), (3, 2, 0, 0, 0, 0), mesh=(1, 0, 0)),
    cfg(19, (5, 4, 6), (1,) * 6, mesh=(1, 1, 1), k_stretch=2.0),
    cfg(19, (4, 6, 5), (0, 0, 3, 3, 1, 2), mesh=(0, 1, 1)),
    cfg(19, (2, 3, 2), (1,) * 6, mesh=(1, 1, 1)),
    cfg(27, (4, 5, 3), (1,) * 6, mesh=(1, 1, 1), k_stretch=1.2),
]


@pytest.mark.parametrize("d", LINEAR, ids=[f"q{c['lattice']}-{c['n']}-{c['bc']}-{c['mesh']}" for c in LINEAR])
def test_reconstruction_exact_for_linear_fields(d):
    D, Q, shp = O.dims(d)
    g = rng(41, Q, *d["n"])
    alpha = 1.0 + 0.1 * g.uniform(-1, 1, Q)
    beta = 0.1 * g.uniform(-1, 1, (Q, 3))
    for a in range(D):
        if d["bc"][2 * a] == O.PERIODIC:
            beta[:, a] = 0.0  # a linear field along a periodic axis is not periodic
    xc = [centres(d, a) if a < D else np.zeros(1) for a in range(3)]
    Z, Y, X = np.meshgrid(xc[2], xc[1], xc[0], indexing="ij")
    phi = alpha[:, None, None, None] + beta[:, 0, None, None, None] * X + beta[:, 1, None, None, None] * Y
    if D == 3:
        phi = phi + beta[:, 2, None, None, None] * Z
    e, _ = O.lattice(d["lattice"])
    xi = np.sqrt(3 * d["RT"]) * e
    h = 0.5 * d["dt"]
    for a in range(D):
        got = O.interface_values(d, a, phi)
        Xf, _ = O.mesh(d, a)
        coords = list(xc)
        coords[a] = Xf
        Zf, Yf, Xf3 = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
        want = (alpha[:, None, None, None] + beta[:, 0, None, None, None] * Xf3 +
                beta[:, 1, None, None, None] * Yf)
        if D == 3:
            want = want + beta[:, 2, None, None, None] * Zf
        want = want - h * (xi[:, :D] * beta[:, :D]).sum(1)[:, None, None, None]
        np.testing.assert_allclose(got, want, rtol=0, atol=2e-14)


# --------------------------------------------------------------------------
# whole-step restatement (tests/brute_step.py) on walls and stretched meshes
# --------------------------------------------------------------------------
UW = [[0, 0.02, 0.01], [0, -0.03, 0], [0.01, 0, 0.02], [0.05, 0, 0], [0.02, 0.01, 0], [0, 0, -0.01]]
RESTATE = [
    cfg(9, (3, 3, 1), (1, 1, 1, 1, 0, 0), uw=LID, mesh=(1, 1, 0)),
    cfg(9, (4, 5, 1), (3, 3, 3, 3, 0, 0), uw=UW, mesh=(1, 0, 0), ff=1),
    cfg(9, (4, 5, 1), (2, 2, 1, 3, 0, 0), pw=[2e-3, -1e-3, 0, 0, 0, 0], uw=UW, mesh=(0, 1, 0), G=(1e-3, 0, 0)),
    cfg(9, (3, 3, 1), (0, 0, 2, 2, 0, 0), pw=[0, 0, 1e-3, -2e-3, 0, 0], mesh=(1, 1, 0), ff=1, omega=0.3,
        phase=0.2),
    cfg(9, (4, 5, 1), (3, 3, 1, 1, 0, 0), uw=UW, mesh=(1, 1, 0), model=1, G=(1e-3, 1e-3, 0)),
    cfg(19, (3, 4, 5), (1,) * 6, uw=UW, mesh=(1, 1, 1), ff=1),
    cfg(19, (3, 4, 5), (3, 3, 2, 2, 1, 1), uw=UW, pw=[0, 0, 1e-3, 0, 0, 0], mesh=(1, 0, 1)),
    cfg(19, (3, 4, 5), (0, 0, 3, 1, 2, 3), uw=UW, pw=[0, 0, 0, 0, -1e-3, 0], mesh=(0, 1, 1), ff=1,
        G=(1e-3, 0, 0)),
    cfg(19, (3, 4, 5), (0,) * 6, mesh=(1, 1, 1), ff=1),
    cfg(19, (3, 4, 5), (1,) * 6, uw=UW, mesh=(1, 1, 1), model=1),
    cfg(27, (3, 4, 5), (1, 1, 3, 3, 2, 2), uw=UW, pw=[0, 0, 0, 0, 1e-3, 0], mesh=(1, 1, 1), ff=1),
    # wall pressures following the time factor (pw + pw_osc g(t))
    cfg(9, (4, 3, 1), (2, 2, 3, 3, 0, 0), uw=UW, pw=[1e-3, 0, 0, 0, 0, 0], pw_osc=[-2e-3, 5e-4, 0, 0, 0, 0],
        omega=0.4, phase=0.3, mesh=(1, 0, 0)),
    cfg(19, (3, 4, 5), (0, 0, 3, 3, 2, 2), uw=UW, pw=[0, 0, 0, 0, 1e-3, 0], pw_osc=[0, 0, 0, 0, -1e-3, 2e-3],
        omega=0.5, mesh=(0, 1, 1), G=(1e-3, 0, 0)),
]


@pytest.mark.parametrize("d", RESTATE, ids=[f"q{c['lattice']}-{c['n']}-{c['bc']}-{c['mesh']}-m{c.get('model', 0)}"
                                            for c in RESTATE])
def test_step_matches_whole_array_restatement(d):
    d = dict(d)
    ff = d.pop("ff", 0)
    D, Q, shp = O.dims(d)
    force = field(5, (D,) + shp, 1e-3) if ff else None
    f0 = perturb(3, O.init(d, rho=1 + field(1, shp, 0.01), u=field(2, (D,) + shp, 0.03), force=force), 1e-2)
    a1 = O.step(d, f0, force, 0.7)
    b1 = B.step(d, f0, force, 0.7)
    assert np.abs(a1 - f0).max() > 1e-3  # the step does change the state
    assert np.abs(a1 - b1).max() / np.abs(a1).max() < 2e-15
    a3 = O.run(d, f0, 3, force, 0.7)
    b3 = B.run(d, f0, 3, force, 0.7)
    assert np.abs(a3 - b3).max() / np.abs(a3).max() < 5e-15


def random_faces(seed, n, L):
    """strictly increasing face coordinates from 0 to L with widths varying
    by up to a factor 3 between neighbours"""
    w = rng(seed, n).uniform(0.5, 1.5, n)
    X = np.concatenate([[0.0], np.cumsum(w)])
    X = X * (L / X[-1])
    X[-1] = L
    return X


def test_custom_faces_equal_to_the_tanh_formula_give_the_tanh_step():
    d = cfg(19, (4, 5, 3), (1, 1, 3, 3, 0, 0), uw=UW, mesh=(1, 1, 0), k_stretch=1.3)
    faces = [O.mesh(d, a)[0] for a in range(3)]
    c = dict(d, mesh=(2, 2, 0), faces=(faces[0], faces[1], None))
    D, Q, shp = O.dims(d)
    f0 = perturb(3, O.init(d, rho=1 + field(1, shp, 0.01), u=field(2, (D,) + shp, 0.03)), 1e-2)
    np.testing.assert_array_equal(O.step(c, f0), O.step(d, f0))


@pytest.mark.parametrize("lat", [9, 19])
def test_custom_faces_step_matches_whole_array_restatement(lat):
    n = (5, 4, 1) if lat == 9 else (4, 5, 3)
    L = tuple(float(v) for v in n)
    faces = tuple(random_faces(60 + a, n[a], L[a]) for a in range(3))
    d = cfg(lat, n, (1, 3, 2, 1, 0, 0) if lat == 9 else (1, 3, 2, 1, 1, 1), uw=UW, pw=[0, 0, 1e-3, 0, 0, 0],
            mesh=(2, 2, 2 if lat != 9 else 0), faces=faces)
    D, Q, shp = O.dims(d)
    force = field(5, (D,) + shp, 1e-3)
    f0 = perturb(3, O.init(d, rho=1 + field(1, shp, 0.01), u=field(2, (D,) + shp, 0.03), force=force), 1e-2)
    a3 = O.run(d, f0, 3, force, 0.7)
    b3 = B.run(d, f0, 3, force, 0.7)
    assert np.abs(a3 - b3).max() / np.abs(a3).max() < 5e-15
    # and Eq. (gradient) stays exact on a linear field on this mesh
    xc = [O.mesh(d, a)[1][1:-1] if a < D else np.zeros(1) for a in range(3)]
    Z, Y, X = np.meshgrid(xc[2], xc[1], xc[0], indexing="ij")
    phi = np.broadcast_to(1.0 + 0.1 * X - 0.05 * Y + 0.02 * Z, shp)[None].repeat(Q, 0)
    e, _ = O.lattice(lat)
    h = 0.5 * d["dt"]
    grad = np.array([0.1, -0.05, 0.02])[:D]
    for a in range(D):
        Xf = O.mesh(d, a)[0]
        coords = list(xc)
        coords[a] = Xf
        Zf, Yf, Xf3 = np.meshgrid(coords[2], coords[1], coords[0], indexing="ij")
        want = (1.0 + 0.1 * Xf3 - 0.05 * Yf + (0.02 * Zf if D == 3 else 0))[None] - \
            h * (np.sqrt(3 * d["RT"]) * e[:, :D] @ grad)[:, None, None, None]
        np.testing.assert_allclose(O.interface_values(d, a, phi), want, rtol=0, atol=2e-14)


def test_custom_faces_rejected_unless_increasing_from_zero_to_L():
    d = cfg(9, (4, 3, 1), (1, 1, 1, 1, 0, 0), mesh=(2, 0, 0))
    for bad in ([0.0, 1.0, 1.0, 3.0, 4.0], [0.5, 1.0, 2.0, 3.0, 4.0], [0.0, 1.0, 2.0, 3.0, 4.5]):
        with pytest.raises(ValueError):
            O.step(dict(d, faces=(np.array(bad), None, None)), np.ones((9, 1, 3, 4)))


# --------------------------------------------------------------------------
# manufactured steady flows on stretched meshes: second order
# --------------------------------------------------------------------------
# Divergence-free u = (psi_y, -psi_x) with psi = U sin^2(pi x) sin^2(pi y),
# zero on every wall; the body force G = (u.grad) u - nu lap(u) makes it a
# steady solution of the incompressible equations with uniform pressure.
# Started from it, the computed flow departs from it only by the scheme's
# truncation error, so the error after a fixed time falls as dx^2.  Regime:
# RT = 1000/3, tau = 1e-4 (Knudsen number 3e-3), U = 0.01 (Mach 3e-4), as in
# the paper's wall tests, where O(dx^2) dominates the kinetic terms.
RT_C, NU, U = 1000.0 / 3.0, 1.0 / 30.0, 0.01
PI = np.pi


def _planar(s, t):
    """u, v and the force along the two in-plane coordinates s, t"""
    ss, st = np.sin(PI * s), np.sin(PI * t)
    s2s, s2t, c2s, c2t = np.sin(2 * PI * s), np.sin(2 * PI * t), np.cos(2 * PI * s), np.cos(2 * PI * t)
    u = U * PI * ss ** 2 * s2t
    v = -U * PI * s2s * st ** 2
    us, ut = U * PI * PI * s2s * s2t, 2 * U * PI * PI * ss ** 2 * c2t
    vs, vt = -2 * U * PI * PI * c2s * st ** 2, -U * PI * PI * s2s * s2t
    lu = 2 * U * PI ** 3 * s2t * (2 * c2s - 1)
    lv = -2 * U * PI ** 3 * s2s * (2 * c2t - 1)
    return u, v, u * us + v * ut - NU * lu, u * vs + v * vt - NU * lv, lu, lv


def _mms_error(d, ua, G, T):
    X, _ = O.mesh(d, 1)
    d["dt"] = 0.5 * np.diff(X).min() / np.sqrt(3 * d["RT"])
    nsteps = int(round(T / d["dt"]))
    f = O.run(d, O.init(d, u=ua, force=G), nsteps, force=G)
    _, u, _, _ = O.moments(d, f, force=G, t=nsteps * d["dt"])
    return np.sqrt(((u - ua) ** 2).sum() / (ua ** 2).sum())


def _orders(errs):
    return [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]


def test_manufactured_flow_d2q9_tanh_second_order():
    errs = []
    for N in (16, 32, 64):
        d = dict(lattice=9, n=(N, N, 1), L=(1.0, 1.0, 1.0), mesh=(1, 1, 0), k_stretch=1.5, rho0=1.0, RT=RT_C,
                 tau=NU / RT_C, dt=1.0, bc=(1, 1, 1, 1, 0, 0))
        Y, X = np.meshgrid(centres(d, 1), centres(d, 0), indexing="ij")
        u, v, gx, gy, _, _ = _planar(X, Y)
        errs.append(_mms_error(d, np.stack([u, v])[:, None], np.stack([gx, gy])[:, None], 1.0))
    assert all(r > 3.5 for r in _orders(errs)), errs
    assert errs[-1] < 2e-3


def test_manufactured_flow_d3q19_plane_tanh_second_order():
    # the same flow in the (y, z) plane: walls and tanh meshes on y and z
    # (z is the march axis of the kernels), one periodic cell along x
    errs = []
    for N in (16, 32, 64):
        d = dict(lattice=19, n=(1, N, N), L=(1.0 / N, 1.0, 1.0), mesh=(0, 1, 1), k_stretch=1.5, rho0=1.0,
                 RT=RT_C, tau=NU / RT_C, dt=1.0, bc=(0, 0, 1, 1, 1, 1))
        Z, Y = np.meshgrid(centres(d, 2), centres(d, 1), indexing="ij")
        v, w, gy, gz, _, _ = _planar(Y, Z)
        zero = np.zeros_like(v)
        ua = np.stack([zero, v, w])[:, :, :, None]
        G = np.stack([zero, gy, gz])[:, :, :, None]
        errs.append(_mms_error(d, ua, G, 1.0))
    assert all(r > 3.5 for r in _orders(errs)), errs
    assert errs[-1] < 2e-3


def test_manufactured_flow_d3q19_tanh_box_second_order():
    # fully 3-D: u = sin^2(pi z) (psi_y, -psi_x, 0), walls on all six sides,
    # tanh mesh on every axis; the force carries the z curvature of the
    # profile and the z-modulated convective term
    errs = []
    for N in (8, 16, 32):
        d = dict(lattice=19, n=(N, N, N), L=(1.0, 1.0, 1.0), mesh=(1, 1, 1), k_stretch=1.5, rho0=1.0, RT=RT_C,
                 tau=NU / RT_C, dt=1.0, bc=(1,) * 6)
        x = centres(d, 0)
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        u, v, gx, gy, lu, lv = _planar(X, Y)
        ph, d2ph = np.sin(PI * Z) ** 2, 2 * PI * PI * np.cos(2 * PI * Z)
        conv_x, conv_y = gx + NU * lu, gy + NU * lv  # (u.grad) u of the planar field
        ua = np.stack([ph * u, ph * v, np.zeros_like(u)])
        G = np.stack([ph * ph * conv_x - NU * (ph * lu + d2ph * u),
                      ph * ph * conv_y - NU * (ph * lv + d2ph * v), np.zeros_like(u)])
        errs.append(_mms_error(d, ua, G, 0.5))
    assert all(r > 3.5 for r in _orders(errs)), errs
    assert errs[-1] < 1e-2
