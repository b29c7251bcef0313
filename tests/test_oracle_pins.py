"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them re-types the oracle's
formulas: they use printed tables, exact moment identities, closed-form
conservation increments, an independent stencil restatement of the step on
periodic meshes, and the D3Q19 / D3Q27 -> D2Q9 projection.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from synthetic import field, perturb
from tests import brute_stencil

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cfg2(n=(5, 4), L=None, bc=(0,) * 6, **kw):
    d = dict(lattice=9, n=(n[0], n[1], 1), L=L or (float(n[0]), float(n[1]), 1.0), rho0=1.0, RT=1 / 3,
             tau=0.6, dt=0.5, bc=bc)
    d.update(kw)
    return d


def cfg3(n=(3, 4, 5), L=None, bc=(0,) * 6, **kw):
    d = dict(lattice=19, n=n, L=L or tuple(float(v) for v in n), rho0=1.0, RT=1 / 3, tau=0.6, dt=0.5, bc=bc)
    d.update(kw)
    return d


# --------------------------------------------------------------------------
# velocity sets (Sec. II.C)
# --------------------------------------------------------------------------
def test_d2q9_matches_printed_table():
    rows = np.loadtxt(os.path.join(GOLDEN, "d2q9_printed.txt"))
    e, w = O.lattice(9)
    assert e.shape == (9, 3)
    for r in rows:
        i = int(r[0]) - 1
        assert tuple(e[i, :2]) == (int(r[1]), int(r[2]))
        assert e[i, 2] == 0
        assert w[i] == pytest.approx(r[3] / r[4], rel=1e-15)


def test_printed_d3q27_weights_fix_the_1d_weights():
    # the 3-D printed weights are cubes/products of the 1-D weights, which
    # must therefore be 2/3 (rest) and 1/6 (+-1), not the printed 1/3
    w0, w1 = Fraction(2, 3), Fraction(1, 6)
    with open(os.path.join(GOLDEN, "d3q27_printed_weights.txt")) as fh:
        rows = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    expect = {"rest": w0 ** 3, "axis": w0 ** 2 * w1, "edge": w0 * w1 ** 2, "corner": w1 ** 3}
    total = Fraction(0)
    for r in rows:
        wt = Fraction(int(r[1]), int(r[2]))
        assert wt == expect[r[0]]
        total += wt * len(r[3:])
    assert total == 1
    # the oracle's D3Q27 carries exactly these weights, class by |e|^2
    e, w = O.lattice(27)
    cls = {0: "rest", 1: "axis", 2: "edge", 3: "corner"}
    for q in range(27):
        assert w[q] == pytest.approx(float(expect[cls[int((e[q] ** 2).sum())]]), rel=1e-15)
    # and the oracle's D2Q9 weights are the 2-D products of the same rule
    e, w = O.lattice(9)
    for q in range(9):
        f = [w0 if v == 0 else w1 for v in e[q, :2]]
        assert w[q] == pytest.approx(float(f[0] * f[1]), rel=1e-15)


@pytest.mark.parametrize("lat", [9, 19, 27])
def test_lattice_isotropy(lat):
    # Gauss-Hermite quadrature requirements for Eq. (icfeq): with c^2 = 3RT,
    # sum W = 1, sum W xi_a xi_b = RT delta_ab, sum W xi_a^4 = 3 RT^2,
    # sum W xi_a^2 xi_b^2 = RT^2 (a != b), odd moments vanish
    e, w = O.lattice(lat)
    D = 2 if lat == 9 else 3
    assert len(w) == lat
    c2 = 3.0  # RT = 1
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    for a in range(D):
        assert (w * e[:, a]).sum() == pytest.approx(0, abs=1e-15)
        assert (w * e[:, a] ** 3).sum() == pytest.approx(0, abs=1e-15)
        assert (w * c2 * e[:, a] ** 2).sum() == pytest.approx(1.0, abs=1e-14)
        assert (w * c2 ** 2 * e[:, a] ** 4).sum() == pytest.approx(3.0, abs=1e-14)
        for b in range(D):
            if b != a:
                assert (w * e[:, a] * e[:, b]).sum() == pytest.approx(0, abs=1e-15)
                assert (w * c2 ** 2 * e[:, a] ** 2 * e[:, b] ** 2).sum() == pytest.approx(1.0, abs=1e-14)
                assert (w * e[:, a] ** 2 * e[:, b]).sum() == pytest.approx(0, abs=1e-15)
    # every velocity has its opposite
    s = {tuple(v) for v in e}
    assert all(tuple(-v) in s for v in e)
    assert len(s) == lat


# --------------------------------------------------------------------------
# equilibrium and force term (Eqs. icfeq, S)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("lat", [9, 19, 27])
def test_feq_moments(lat):
    d = cfg2(rho0=1.3, RT=0.7) if lat == 9 else cfg3(rho0=1.3, RT=0.7, lattice=lat)
    e, _ = O.lattice(lat)
    D = 2 if lat == 9 else 3
    xi = np.sqrt(3 * 0.7) * e[:, :D]
    for s in range(4):
        rho = 1.3 + field(s, (), 0.05)
        u = field(s + 10, (D,), 0.2)
        fe = O.feq(d, float(rho), u)
        assert fe.sum() == pytest.approx(rho, rel=1e-14)
        np.testing.assert_allclose(xi.T @ fe, 1.3 * u, rtol=0, atol=1e-14)
        P = np.einsum("qa,qb,q->ab", xi, xi, fe)
        np.testing.assert_allclose(P, rho * 0.7 * np.eye(D) + 1.3 * np.outer(u, u), rtol=0, atol=1e-13)


@pytest.mark.parametrize("lat", [9, 19, 27])
def test_force_term_moments(lat):
    # with the incompressible equilibrium: sum S = (rho0 - rho) G.u / RT,
    # sum xi S = rho G
    d = cfg2(rho0=0.9, RT=0.4) if lat == 9 else cfg3(rho0=0.9, RT=0.4, lattice=lat)
    e, _ = O.lattice(lat)
    D = 2 if lat == 9 else 3
    xi = np.sqrt(3 * 0.4) * e[:, :D]
    for s in range(4):
        rho = 0.9 + float(field(s, (), 0.05))
        u = field(s + 20, (D,), 0.2)
        G = field(s + 30, (D,), 0.1)
        S = O.force_term(d, rho, u, G)
        assert S.sum() == pytest.approx((0.9 - rho) * (G @ u) / 0.4, abs=1e-14)
        np.testing.assert_allclose(xi.T @ S, rho * G, rtol=0, atol=1e-14)


# --------------------------------------------------------------------------
# mesh (Eq. Nonuniform_mesh)
# --------------------------------------------------------------------------
def test_tanh_mesh_properties():
    d = cfg2(n=(64, 40), L=(2.0, 1.0, 1.0), mesh=(1, 1, 0), k_stretch=2.5, bc=(1,) * 6)
    for axis, N, L in ((0, 64, 2.0), (1, 40, 1.0)):
        X, xc = O.mesh(d, axis)
        assert X[0] == 0.0 and X[-1] == L
        assert np.all(np.diff(X) > 0)
        np.testing.assert_allclose(X + X[::-1], L, atol=1e-14)        # symmetric about L/2
        dx = np.diff(X)
        assert dx[0] < dx[N // 2 - 1]                                  # refined at the walls
        np.testing.assert_allclose(xc[1:-1], 0.5 * (X[:-1] + X[1:]), atol=1e-15)
        assert xc[0] == pytest.approx(-xc[1])                          # mirrored ghosts
        assert xc[-1] == pytest.approx(2 * L - xc[-2])
    # k -> 0 gives the uniform mesh
    d0 = cfg2(n=(16, 16), L=(1.0, 1.0, 1.0), mesh=(1, 1, 0), k_stretch=1e-6, bc=(1,) * 6)
    X, _ = O.mesh(d0, 0)
    np.testing.assert_allclose(X, np.linspace(0, 1, 17), atol=1e-12)


# --------------------------------------------------------------------------
# whole-step invariants
# --------------------------------------------------------------------------
@pytest.mark.parametrize("lat", [9, 19, 27])
@pytest.mark.parametrize("stretch", [0, 1])
def test_uniform_state_fixed_point(lat, stretch):
    # G = 0, periodic: any uniform equilibrium is preserved (coefficients sum
    # to one, gradients vanish, fluxes cancel)
    if lat == 9:
        d = cfg2(n=(6, 5), mesh=(stretch, stretch, 0), k_stretch=1.5)
    else:
        d = cfg3(n=(4, 5, 3), mesh=(stretch,) * 3, k_stretch=1.5, lattice=lat)
    D, Q, shp = O.dims(d)
    u = np.zeros((D,) + shp)
    u[0], u[1] = 0.04, -0.03
    if D == 3:
        u[2] = 0.02
    f0 = O.init(d, rho=np.full(shp, 1.02), u=u)
    f1 = O.run(d, f0, 3)
    np.testing.assert_allclose(f1, f0, rtol=0, atol=2e-15)


@pytest.mark.parametrize("lat", [9, 19, 27])
@pytest.mark.parametrize("tau,dt", [(0.6, 0.5), (0.05, 0.5), (1e-3, 0.2)])
def test_homogeneous_relaxation_closed_form(lat, tau, dt):
    # one periodic cell, no force: the interface fluxes cancel and the step
    # is the collision alone.  Eqs. (f_bar_+) and (f_tilde_+) then give
    # f~(n+1) = f~ + (4/3) B1 (feq - f~), B1 = 3h/(2 tau + dt), h = dt/2, with
    # rho and j unchanged, i.e. the non-equilibrium part decays by the
    # trapezoidal factor (2 tau - dt)/(2 tau + dt) per step (negative and
    # close to -1 for tau << dt) -- a closed form independent of the scheme's
    # transcription.  Planted mistakes each fail it: h for dt in B1's
    # numerator, 2 tau - dt for 2 tau - h in the f~ coefficient, and 3/2, 1/2
    # for 4/3, 1/3 in Eq. (f_tilde_+)
    d = cfg2(n=(1, 1), tau=tau, dt=dt, lattice=lat) if lat == 9 else cfg3(n=(1, 1, 1), tau=tau, dt=dt, lattice=lat)
    D, Q, shp = O.dims(d)
    e, _ = O.lattice(lat)
    xi = np.sqrt(3 * d["RT"]) * e[:, :D]
    f = perturb(4, O.init(d, rho=np.full(shp, 1.01), u=np.full((D,) + shp, 0.02)), 2e-2)
    fv = f.reshape(Q)
    rho, u = fv.sum(), (xi * fv[:, None]).sum(0) / d["rho0"]
    feq = O.feq(d, rho, np.concatenate([u, np.zeros(3 - D)]))[:Q]
    r = (2 * tau - dt) / (2 * tau + dt)
    fn = f
    for n in range(1, 4):
        fn = O.step(d, fn)
        np.testing.assert_allclose(fn.reshape(Q) - feq, r ** n * (fv - feq), rtol=0, atol=5e-16 * n)


@pytest.mark.parametrize("lat", [9, 19, 27])
@pytest.mark.parametrize("stretch", [0, 1])
def test_periodic_conservation_without_force(lat, stretch):
    if lat == 9:
        d = cfg2(n=(7, 6), mesh=(stretch, stretch, 0), k_stretch=1.5)
    else:
        d = cfg3(n=(4, 5, 6), mesh=(stretch,) * 3, k_stretch=1.5, lattice=lat)
    D, Q, shp = O.dims(d)
    f0 = perturb(1, O.init(d, rho=1 + field(2, shp, 0.01), u=field(3, (D,) + shp, 0.05)), 1e-2)
    _, _, _, t0 = O.moments(d, f0)
    _, _, _, t1 = O.moments(d, O.run(d, f0, 4))
    np.testing.assert_allclose(t1[:4], t0[:4], rtol=0, atol=1e-12 * np.prod(shp))


@pytest.mark.parametrize("lat", [9, 19, 27])
def test_periodic_increments_with_force(lat):
    # Eq. (f_j+n) summed over velocities: per step and cell the momentum
    # grows by dt G (rho0 dt + 2 tau rho) / (2 tau + dt) and the mass by
    # 2 tau dt/(2 tau + dt) (rho0 - rho) G.u / RT (fluxes telescope)
    d = cfg2(n=(6, 5), tau=0.3, dt=0.4) if lat == 9 else cfg3(n=(3, 4, 5), tau=0.3, dt=0.4, lattice=lat)
    D, Q, shp = O.dims(d)
    Gf = field(5, (D,) + shp, 1e-3)
    t = 0.7
    d.update(omega=0.9, phase=0.2, G=(2e-4, -1e-4, 3e-4))
    f0 = perturb(6, O.init(d, rho=1 + field(7, shp, 0.02), u=field(8, (D,) + shp, 0.05), force=Gf), 5e-3)
    rho, u, _, t0 = O.moments(d, f0, force=Gf, t=t)
    f1 = O.step(d, f0, force=Gf, t=t)
    _, _, _, t1 = O.moments(d, f1, force=Gf, t=t + d["dt"])
    dt, tau, rho0, RT = d["dt"], d["tau"], d["rho0"], d["RT"]
    g = np.cos(d["omega"] * t + d["phase"])
    G = g * (np.array(d["G"][:D]).reshape((D,) + (1,) * 3) + Gf)
    V = 1.0  # unit cells
    dmom = (V * dt * G * (rho0 * dt + 2 * tau * rho) / (2 * tau + dt)).reshape(D, -1).sum(1)
    dmass = (V * 2 * tau * dt / (2 * tau + dt) * (rho0 - rho) * (G * u).sum(0) / RT).sum()
    np.testing.assert_allclose(t1[1:1 + D] - t0[1:1 + D], dmom, rtol=1e-9, atol=1e-15)
    assert t1[0] - t0[0] == pytest.approx(dmass, rel=1e-6, abs=1e-15)


def test_init_recovers_velocity():
    # f~0 = feq - dt/2 S: at rho = rho0 the macro recovery returns u exactly
    d = cfg2(n=(5, 4), G=(1e-3, 2e-3, 0))
    D, Q, shp = O.dims(d)
    u = field(9, (D,) + shp, 0.05)
    Gf = field(10, (D,) + shp, 1e-3)
    f0 = O.init(d, u=u, force=Gf)
    rho, u1, p, _ = O.moments(d, f0, force=Gf)
    np.testing.assert_allclose(u1, u, rtol=0, atol=1e-15)


# --------------------------------------------------------------------------
# independent restatement on periodic uniform meshes
# --------------------------------------------------------------------------
@pytest.mark.parametrize("lat,n,dx", [(9, (5, 4, 1), (0.5, 0.7)), (19, (3, 4, 5), (0.5, 0.6, 0.8)),
                                      (27, (3, 4, 5), (0.5, 0.6, 0.8))])
def test_oracle_matches_stencil_restatement(lat, n, dx):
    D = 2 if lat == 9 else 3
    L = tuple(n[a] * dx[a] for a in range(D)) + ((1.0,) if D == 2 else ())
    d = dict(lattice=lat, n=n, L=L, rho0=1.1, RT=0.45, tau=0.37, dt=0.3, bc=(0,) * 6,
             G=(2e-3, -1e-3, 5e-4), omega=1.3, phase=0.4)
    _, Q, shp = O.dims(d)
    Gf = field(11, (D,) + shp, 2e-3)
    f0 = perturb(12, O.init(d, rho=1.1 + field(13, shp, 0.03), u=field(14, (D,) + shp, 0.08), force=Gf),
                 2e-2)
    t = 0.25
    ref = brute_stencil.step(lat, f0, 1.1, 0.45, 0.37, 0.3, dx, Gfield=Gf,
                             gt=np.cos(1.3 * t + 0.4), gth=np.cos(1.3 * (t + 0.15) + 0.4), G0=d["G"])
    got = O.step(d, f0, force=Gf, t=t)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-14)


# --------------------------------------------------------------------------
# D3Q19 and D3Q27 project onto D2Q9
# --------------------------------------------------------------------------
@pytest.mark.parametrize("lat3", [19, 27])
@pytest.mark.parametrize("plane", [(0, 1), (0, 2), (1, 2)])
def test_3d_lattice_reduces_to_d2q9(lat3, plane):
    # summing D3Q19 or D3Q27 over the velocity component normal to a plane gives the
    # D2Q9 weights; a flow invariant along that axis (periodic, no normal
    # velocity) therefore evolves exactly like the D2Q9 flow in the plane
    a, b = plane
    c = 3 - a - b
    n2 = (6, 5)
    d2 = dict(lattice=9, n=(n2[0], n2[1], 1), L=(6.0, 5.0, 1.0), rho0=1.0, RT=1 / 3, tau=0.4, dt=0.5,
              bc=(0, 0, 1, 1, 0, 0), uw=[[0, 0, 0], [0, 0, 0], [0, 0, 0], [0.05, 0.01, 0], [0, 0, 0],
                                         [0, 0, 0]], G=(1e-4, 0, 0))
    D, Q, shp2 = O.dims(d2)
    u2 = field(15, (2,) + shp2, 0.03)
    f2 = perturb(16, O.init(d2, rho=1 + field(17, shp2, 0.01), u=u2), 1e-2)
    # 3-D: in-plane axes (a, b) carry (x, y) of the 2-D run, axis c periodic, 3 cells
    n3 = [0, 0, 0]
    n3[a], n3[b], n3[c] = n2[0], n2[1], 3
    L3 = [0.0, 0.0, 0.0]
    L3[a], L3[b], L3[c] = 6.0, 5.0, 3.0
    bc3 = [0] * 6
    bc3[2 * b] = bc3[2 * b + 1] = 1
    uw3 = [[0.0] * 3 for _ in range(6)]
    uw3[2 * b + 1][a], uw3[2 * b + 1][b] = 0.05, 0.01
    G3 = [0.0] * 3
    G3[a] = 1e-4
    d3 = dict(lattice=lat3, n=tuple(n3), L=tuple(L3), rho0=1.0, RT=1 / 3, tau=0.4, dt=0.5, bc=tuple(bc3),
              uw=uw3, G=tuple(G3))
    e2, _ = O.lattice(9)
    e3, _ = O.lattice(lat3)

    def to3(v2):  # 2-D field [.., 1, Y, X] -> 3-D [.., z, y, x], (X, Y) on axes (a, b), constant along c
        v = v2[..., 0, :, :]
        A = np.zeros(v.shape[:-2] + (n3[0], n3[1], n3[2]))
        for k in range(n3[c]):
            idx = [slice(None)] * 3
            idx[c] = k
            A[(Ellipsis,) + tuple(idx)] = np.swapaxes(v, -1, -2) if a < b else v
        return np.swapaxes(A, -1, -3)

    # 3-D initial state: split each 2-D population evenly over its e_c family
    f3 = np.zeros((lat3, n3[2], n3[1], n3[0]))
    fam = {}
    for q3 in range(lat3):
        key = (e3[q3, a], e3[q3, b])
        fam.setdefault(key, []).append(q3)
    _, w3 = O.lattice(lat3)
    _, w2 = O.lattice(9)
    for q2 in range(9):
        key = (e2[q2, 0], e2[q2, 1])
        big = to3(f2[q2])
        for q3 in fam[key]:
            f3[q3] = big * (w3[q3] / w2[q2])
    r2 = O.run(d2, f2, 3)
    r3 = O.run(d3, f3, 3)
    for q2 in range(9):
        key = (e2[q2, 0], e2[q2, 1])
        s = sum(r3[q3] for q3 in fam[key])
        np.testing.assert_allclose(s, to3(r2[q2]), rtol=0, atol=1e-14)
