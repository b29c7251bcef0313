"""Pins of the oracle's tape-free reverse mode: <J v, w> from central finite
differences of the forward step against <v, J^T w> from the adjoint.

The step is a polynomial in (f~, G^) (the velocity divides by the constant
rho0), so central differences are accurate to O(eps^2)."""
import numpy as np
import pytest

import oracle as O
from synthetic import field, perturb


def setup(lat, stretch=0):
    if lat == 9:
        d = dict(lattice=9, n=(5, 4, 1), L=(5.0, 4.0, 1.0), mesh=(stretch, stretch, 0), k_stretch=1.5)
    else:
        d = dict(lattice=19, n=(3, 4, 5), L=(3.0, 4.0, 5.0), mesh=(stretch,) * 3, k_stretch=1.5)
    d.update(rho0=1.0, RT=1 / 3, tau=0.45, dt=0.5, bc=(0,) * 6, G=(1e-3, -5e-4, 2e-4), omega=0.7, phase=0.3)
    D, Q, shp = O.dims(d)
    Gf = field(21, (D,) + shp, 2e-3)
    f = perturb(22, O.init(d, rho=1 + field(23, shp, 0.02), u=field(24, (D,) + shp, 0.05), force=Gf), 1e-2)
    return d, f, Gf


@pytest.mark.parametrize("lat,stretch", [(9, 0), (9, 1), (19, 0)])
def test_step_adjoint_dot_product(lat, stretch):
    d, f, Gf = setup(lat, stretch)
    t = 0.4
    v = field(25, f.shape, 1.0)
    w = field(26, f.shape, 1.0)
    vg = field(27, Gf.shape, 1.0)
    eps = 1e-5
    jv = (O.step(d, f + eps * v, Gf, t) - O.step(d, f - eps * v, Gf, t)) / (2 * eps)
    jg = (O.step(d, f, Gf + eps * 1e-2 * vg, t) - O.step(d, f, Gf - eps * 1e-2 * vg, t)) / (2 * eps * 1e-2)
    gG = np.zeros_like(Gf)
    jtw = O.step_adjoint(d, f, w, force=Gf, t=t, grad_force=gG)
    lhs, rhs = np.vdot(jv, w), np.vdot(v, jtw)
    assert rhs == pytest.approx(lhs, rel=5e-9)
    lhs_g, rhs_g = np.vdot(jg, w), np.vdot(vg, gG)
    assert rhs_g == pytest.approx(lhs_g, rel=1e-7)


LID = [[0, 0, 0], [0, 0, 0], [0, 0, 0], [0.05, 0, 0], [0, 0, 0], [0, 0, 0]]
MOVING = [[0, 0.02, 0], [0, -0.01, 0], [0.03, 0, 0], [0.05, 0, 0], [0, 0, 0.01], [0.02, 0, 0]]


def wall_setup(lat, bc, stretch=0, uw=LID, pw=(0,) * 6):
    """small meshes with walls: every wall cell is next to a wall, a corner or
    the opposite wall (n = 2 along some axes)"""
    if lat == 9:
        d = dict(lattice=9, n=(5, 4, 1), L=(5.0, 4.0, 1.0), mesh=(stretch, stretch, 0), k_stretch=1.5)
    else:
        d = dict(lattice=19, n=(3, 4, 2), L=(3.0, 4.0, 2.0), mesh=(stretch,) * 3, k_stretch=1.5)
    d.update(rho0=1.0, RT=1 / 3, tau=0.45, dt=0.5, bc=bc, uw=uw, pw=list(pw), G=(1e-3, -5e-4, 2e-4),
             omega=0.7, phase=0.3)
    D, Q, shp = O.dims(d)
    Gf = field(41, (D,) + shp, 2e-3)
    f = perturb(42, O.init(d, rho=1 + field(43, shp, 0.02), u=field(44, (D,) + shp, 0.05), force=Gf), 1e-2)
    return d, f, Gf


WALL_CASES = [
    (9, (1, 1, 1, 1, 0, 0), 0, LID, (0,) * 6),                       # NEQ velocity cavity
    (9, (3, 3, 3, 3, 0, 0), 1, MOVING, (0,) * 6),                    # bounce-back, moving walls, tanh
    (9, (2, 2, 3, 3, 0, 0), 0, LID, (3e-3, -2e-3, 0, 0, 0, 0)),      # NEQ pressure in x, BB in y
    (9, (1, 3, 2, 1, 0, 0), 1, MOVING, (0, 0, 1e-3, 0, 0, 0)),       # every kind, tanh
    (9, (0, 0, 1, 1, 0, 0), 1, LID, (0,) * 6),                       # periodic x, NEQ walls, tanh
    (19, (1, 1, 1, 1, 1, 1), 0, LID, (0,) * 6),                      # NEQ cube
    (19, (3, 2, 1, 3, 0, 0), 1, MOVING, (0, 2e-3, 0, 0, 0, 0)),      # mixed, periodic z, tanh
]


@pytest.mark.parametrize("lat,bc,stretch,uw,pw", WALL_CASES,
                         ids=["q9-neq", "q9-bb-moving-tanh", "q9-neqp-bb", "q9-mixed-tanh", "q9-channel-tanh",
                              "q19-neq", "q19-mixed-tanh"])
def test_step_adjoint_dot_product_walls(lat, bc, stretch, uw, pw):
    # reverse mode through the wall rules (Eqs. BB, NEQ), the ghost
    # extrapolation and the stretched-mesh metrics, against central FD of
    # the forward step (the step stays a polynomial in (f~, G^))
    d, f, Gf = wall_setup(lat, bc, stretch, uw, pw)
    t = 0.4
    v = field(45, f.shape, 1.0)
    w = field(46, f.shape, 1.0)
    vg = field(47, Gf.shape, 1.0)
    eps = 1e-5
    jv = (O.step(d, f + eps * v, Gf, t) - O.step(d, f - eps * v, Gf, t)) / (2 * eps)
    jg = (O.step(d, f, Gf + eps * 1e-2 * vg, t) - O.step(d, f, Gf - eps * 1e-2 * vg, t)) / (2 * eps * 1e-2)
    gG = np.zeros_like(Gf)
    jtw = O.step_adjoint(d, f, w, force=Gf, t=t, grad_force=gG)
    assert np.vdot(v, jtw) == pytest.approx(np.vdot(jv, w), rel=5e-9)
    assert np.vdot(vg, gG) == pytest.approx(np.vdot(jg, w), rel=1e-7)


@pytest.mark.parametrize("lat,bc", [(9, (2, 2, 3, 3, 0, 0)), (19, (2, 2, 1, 3, 3, 3))], ids=["q9", "q19"])
def test_step_adjoint_dot_product_oscillating_pressure(lat, bc):
    # pressure sides following the time factor (pw + pw_osc g(t)), at two
    # times of the oscillation
    d, f, Gf = wall_setup(lat, bc, 1, MOVING, (1e-3, -1e-3, 0, 0, 0, 0))
    d["pw_osc"] = [3e-3, 1e-3, 0, 0, 0, 0]
    v = field(45, f.shape, 1.0)
    w = field(46, f.shape, 1.0)
    eps = 1e-5
    for t in (0.4, 2.9):
        jv = (O.step(d, f + eps * v, Gf, t) - O.step(d, f - eps * v, Gf, t)) / (2 * eps)
        jtw = O.step_adjoint(d, f, w, force=Gf, t=t)
        assert np.vdot(v, jtw) == pytest.approx(np.vdot(jv, w), rel=5e-9)


DEGENERATE = [
    (9, (1, 5, 1), (0, 0, 1, 1, 0, 0)),       # one-column periodic axis, NEQ walls
    (19, (4, 3, 1), (1, 1, 3, 3, 0, 0)),      # one-plane periodic axis
    (19, (1, 3, 2), (0, 0, 3, 3, 1, 1)),      # one-column periodic axis, BB and NEQ walls
]


@pytest.mark.parametrize("lat,n,bc", DEGENERATE, ids=["q9-one-column", "q19-one-plane", "q19-one-column"])
def test_step_adjoint_dot_product_degenerate_axes(lat, n, bc):
    # periodic axes of one cell: the cell is its own neighbour on both sides,
    # so every interface of that axis couples a cell with itself
    d = dict(lattice=lat, n=n, L=tuple(float(v) for v in n), mesh=(0, 0, 0), k_stretch=1.5, rho0=1.0, RT=1 / 3,
             tau=0.45, dt=0.5, bc=bc, uw=MOVING, pw=[0.0] * 6, G=(1e-3, -5e-4, 2e-4), omega=0.7, phase=0.3)
    D, Q, shp = O.dims(d)
    Gf = field(51, (D,) + shp, 2e-3)
    f = perturb(52, O.init(d, rho=1 + field(53, shp, 0.02), u=field(54, (D,) + shp, 0.05), force=Gf), 1e-2)
    t = 0.4
    v = field(55, f.shape, 1.0)
    w = field(56, f.shape, 1.0)
    vg = field(57, Gf.shape, 1.0)
    eps = 1e-5
    jv = (O.step(d, f + eps * v, Gf, t) - O.step(d, f - eps * v, Gf, t)) / (2 * eps)
    jg = (O.step(d, f, Gf + eps * 1e-2 * vg, t) - O.step(d, f, Gf - eps * 1e-2 * vg, t)) / (2 * eps * 1e-2)
    gG = np.zeros_like(Gf)
    jtw = O.step_adjoint(d, f, w, force=Gf, t=t, grad_force=gG)
    assert np.vdot(v, jtw) == pytest.approx(np.vdot(jv, w), rel=5e-9)
    assert np.vdot(vg, gG) == pytest.approx(np.vdot(jg, w), rel=1e-7)


def test_step_adjoint_wall_columns_by_brute_force():
    # full Jacobian columns of a tiny walled mesh: e_k^T J^T w for a few unit
    # vectors e_k next to walls and corners, each against a central FD
    d, f, Gf = wall_setup(9, (1, 3, 2, 1, 0, 0), 1, MOVING, (0, 0, 1e-3, 0, 0, 0))
    w = field(48, f.shape, 1.0)
    jtw = O.step_adjoint(d, f, w, force=Gf, t=0.4)
    eps = 1e-5
    for idx in [(1, 0, 0, 0), (5, 0, 3, 4), (8, 0, 0, 4), (2, 0, 3, 0), (0, 0, 1, 2)]:
        e = np.zeros_like(f)
        e[idx] = 1.0
        col = (O.step(d, f + eps * e, Gf, 0.4) - O.step(d, f - eps * e, Gf, 0.4)) / (2 * eps)
        assert jtw[idx] == pytest.approx(np.vdot(col, w), rel=1e-8, abs=1e-12)


def test_step_adjoint_rejects_the_original_model():
    d, f, Gf = setup(9)
    d["model"] = 1
    with pytest.raises(ValueError):
        O.step_adjoint(d, f, f)


def test_init_adjoint_matches_fd():
    d, _, Gf = setup(9)
    D, Q, shp = O.dims(d)
    u = field(28, (D,) + shp, 0.05)
    w = field(29, (Q,) + shp, 1.0)
    vu = field(30, u.shape, 1.0)
    vg = field(31, Gf.shape, 1.0)
    gu, gg = np.zeros_like(u), np.zeros_like(Gf)
    O.init_adjoint(d, w, u=u, force=Gf, t0=0.2, grad_u=gu, grad_force=gg)
    eps = 1e-5
    ju = (O.init(d, u=u + eps * vu, force=Gf, t0=0.2) - O.init(d, u=u - eps * vu, force=Gf, t0=0.2)) / (2 * eps)
    jg = (O.init(d, u=u, force=Gf + eps * vg, t0=0.2) - O.init(d, u=u, force=Gf - eps * vg, t0=0.2)) / (2 * eps)
    assert np.vdot(vu, gu) == pytest.approx(np.vdot(ju, w), rel=1e-9)
    assert np.vdot(vg, gg) == pytest.approx(np.vdot(jg, w), rel=1e-8)


def test_rollout_gradient_matches_fd():
    # loss = mean of the squared final velocity after a short rollout; the
    # chained adjoint (init VJP + step VJPs + read-out) against central FD on
    # a few force components
    d, _, Gf = setup(9)
    D, Q, shp = O.dims(d)
    nsteps = 4
    u0 = field(32, (D,) + shp, 0.02)
    target = field(33, (D,) + shp, 0.02)

    def loss(G, u0_):
        f = O.init(d, u=u0_, force=G)
        f = O.run(d, f, nsteps, force=G)
        _, u, _, _ = O.moments(d, f, force=G, t=nsteps * d["dt"])
        return np.mean((u - target) ** 2)

    # reverse
    fs = [O.init(d, u=u0, force=Gf)]
    for k in range(nsteps):
        fs.append(O.step(d, fs[-1], Gf, k * d["dt"]))
    _, u, _, _ = O.moments(d, fs[-1], force=Gf, t=nsteps * d["dt"])
    du = 2 * (u - target) / u.size
    e, _ = O.lattice(9)
    xi = np.sqrt(3 * d["RT"]) * e[:, :D]
    lam = np.tensordot(xi, du, axes=(1, 0)) / d["rho0"]
    gG = np.zeros_like(Gf)
    T = nsteps * d["dt"]
    gG += np.cos(d["omega"] * T + d["phase"]) * d["dt"] / 2 * du  # read-out u carries + dt/2 G
    for k in reversed(range(nsteps)):
        lam = O.step_adjoint(d, fs[k], lam, force=Gf, t=k * d["dt"], grad_force=gG)
    gu = np.zeros_like(u0)
    O.init_adjoint(d, lam, u=u0, force=Gf, t0=0.0, grad_u=gu, grad_force=gG)
    for idx in [(0, 0, 1, 2), (1, 0, 3, 4), (0, 0, 0, 0)]:
        eps = 1e-5
        Gp, Gm = Gf.copy(), Gf.copy()
        Gp[idx] += eps
        Gm[idx] -= eps
        fd = (loss(Gp, u0) - loss(Gm, u0)) / (2 * eps)
        assert gG[idx] == pytest.approx(fd, rel=1e-6, abs=1e-14)
        up, um = u0.copy(), u0.copy()
        up[idx] += eps
        um[idx] -= eps
        fd = (loss(Gf, up) - loss(Gf, um)) / (2 * eps)
        assert gu[idx] == pytest.approx(fd, rel=1e-6, abs=1e-14)
