"""Pins of the oracle's original-DUGKS variant (model = 1): the equilibrium
of Eq. (feq) with rho u = sum xi f + rho G dt/2, against the paper's own
comparison of the two models and the exact identities of Eq. (feq)."""
import os

import numpy as np
import pytest

import oracle as O
from synthetic import field, perturb

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cfg(lat, **kw):
    n = (6, 5, 1) if lat == 9 else (3, 4, 5)
    d = dict(lattice=lat, n=n, L=tuple(float(v) for v in n), rho0=1.0, RT=1 / 3, tau=0.3, dt=0.4,
             bc=(0,) * 6, model=1)
    d.update(kw)
    return d


@pytest.mark.parametrize("lat", [9, 19])
def test_original_feq_moments(lat):
    # Eq. (feq) on an isotropic set: sum = rho, sum xi = rho u,
    # sum xi xi = rho RT I + rho u u (rho multiplies every term)
    d = cfg(lat, rho0=1.3, RT=0.7)
    e, _ = O.lattice(lat)
    D = 2 if lat == 9 else 3
    xi = np.sqrt(3 * 0.7) * e[:, :D]
    for s in range(4):
        rho = 1.3 + float(field(s, (), 0.05))
        u = field(s + 10, (D,), 0.2)
        fe = O.feq(d, rho, u)
        assert fe.sum() == pytest.approx(rho, rel=1e-14)
        np.testing.assert_allclose(xi.T @ fe, rho * u, rtol=0, atol=1e-14)
        P = np.einsum("qa,qb,q->ab", xi, xi, fe)
        np.testing.assert_allclose(P, rho * 0.7 * np.eye(D) + rho * np.outer(u, u), rtol=0, atol=1e-13)
        # at rho = rho0 the two equilibria coincide
        np.testing.assert_allclose(O.feq(d, 1.3, u), O.feq(dict(d, model=0), 1.3, u), rtol=1e-15, atol=1e-16)


@pytest.mark.parametrize("lat", [9, 19])
def test_original_force_term_moments(lat):
    # Eq. (S) with Eq. (feq): sum S = 0, sum xi S = rho G
    d = cfg(lat, rho0=0.9, RT=0.4)
    e, _ = O.lattice(lat)
    D = 2 if lat == 9 else 3
    xi = np.sqrt(3 * 0.4) * e[:, :D]
    for s in range(4):
        rho = 0.9 + float(field(s, (), 0.05))
        u = field(s + 20, (D,), 0.2)
        G = field(s + 30, (D,), 0.1)
        S = O.force_term(d, rho, u, G)
        assert abs(S.sum()) < 1e-15
        np.testing.assert_allclose(xi.T @ S, rho * G, rtol=0, atol=1e-14)


@pytest.mark.parametrize("lat", [9, 19])
def test_original_periodic_increments(lat):
    # summed over velocities and a periodic mesh: mass is conserved exactly
    # with forcing, and the momentum grows by dt rho G per cell and step
    # (sum xi (feq - f~) = rho G dt/2 and sum xi S = rho G in Eq. f_j+n)
    d = cfg(lat, omega=0.9, phase=0.2, G=(2e-4, -1e-4, 3e-4))
    D, Q, shp = O.dims(d)
    Gf = field(5, (D,) + shp, 1e-3)
    t = 0.7
    f0 = perturb(6, O.init(d, rho=1 + field(7, shp, 0.02), u=field(8, (D,) + shp, 0.05), force=Gf), 5e-3)
    rho, u, _, t0 = O.moments(d, f0, force=Gf, t=t)
    f1 = O.step(d, f0, force=Gf, t=t)
    _, _, _, t1 = O.moments(d, f1, force=Gf, t=t + d["dt"])
    g = np.cos(d["omega"] * t + d["phase"])
    G = g * (np.array(d["G"][:D]).reshape((D,) + (1,) * 3) + Gf)
    dmom = (d["dt"] * rho[None] * G).reshape(D, -1).sum(1)
    np.testing.assert_allclose(t1[1:1 + D] - t0[1:1 + D], dmom, rtol=1e-9, atol=1e-15)
    assert t1[0] == pytest.approx(t0[0], rel=1e-14)


@pytest.mark.parametrize("lat", [9, 19])
def test_original_model_recovers_velocity(lat):
    # f~0 = feq - dt/2 S, then rho u = sum xi f~ + rho G dt/2 gives u back
    d = cfg(lat, G=(1e-3, 2e-3, -1e-3))
    D, Q, shp = O.dims(d)
    rho = 1 + field(1, shp, 0.02)
    u = field(2, (D,) + shp, 0.05)
    f = O.init(d, rho=rho, u=u)
    r2, u2, _, _ = O.moments(d, f)
    np.testing.assert_allclose(r2, rho, rtol=1e-14)
    np.testing.assert_allclose(u2, u, rtol=0, atol=1e-15)


def test_original_model_has_no_adjoint():
    d = cfg(9)
    D, Q, shp = O.dims(d)
    f = O.init(d)
    with pytest.raises(Exception):
        O.step_adjoint(d, f, np.ones_like(f))


def periodic_flow_error(model, Ma, N=32, nu=0.01, T=4.0, dt=1e-4, cfl=0.1):
    """L2 velocity error of the force-driven periodic flow, Eq. (PF_AS), at
    t = T from the analytic state (parameters of Sec. III.A)"""
    c = cfl / N / dt
    RT = c * c / 3
    u0 = Ma * c
    d = dict(lattice=9, n=(N, N, 1), L=(1, 1, 1), rho0=1.0, RT=RT, tau=nu / RT, dt=dt, bc=(0,) * 6, model=model)
    _, xc = O.mesh(d, 0)
    X, Y = np.meshgrid(xc[1:-1], xc[1:-1], indexing="xy")
    ua = np.stack([u0 * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y),
                   u0 * np.cos(2 * np.pi * X) * np.cos(2 * np.pi * Y)])[:, None]
    pa = 0.25 * u0 ** 2 * (np.cos(4 * np.pi * X) - np.cos(4 * np.pi * Y))[None]
    F = 8 * np.pi ** 2 * nu * ua
    f = O.init(d, rho=1.0 + pa / RT, u=ua, force=F)
    f = O.run(d, f, int(round(T / dt)), force=F)
    _, u, _, _ = O.moments(d, f, force=F)
    return np.sqrt(((u - ua) ** 2).sum() / (ua ** 2).sum())


def test_compressibility_error_of_the_two_models():
    # Sec. III.A, Fig. ICD_D_Ma: from Ma = 0.0152 to 0.1216 the original
    # model's error grows by about a quarter, the incompressible model's by
    # under one percent, and at Ma = 0.1216 the incompressible error is about
    # a fifth smaller (printed: 24.5 %, 0.8 %, 19.0 %)
    with open(os.path.join(GOLDEN, "compressibility_periodic_flow.txt")) as fh:
        ref = dict(ln.split() for ln in fh if ln.strip() and not ln.startswith("#"))
    lo, hi = 0.0152, 0.1216
    ec = [periodic_flow_error(1, m) for m in (lo, hi)]
    ei = [periodic_flow_error(0, m) for m in (lo, hi)]
    growth_c = ec[1] / ec[0] - 1
    growth_i = ei[1] / ei[0] - 1
    reduction = 1 - ei[1] / ec[1]
    assert growth_c == pytest.approx(float(ref["growth_original"]), abs=0.06)
    assert 0 <= growth_i < 2 * float(ref["growth_incompressible"])
    assert reduction == pytest.approx(float(ref["reduction_at_max"]), abs=0.04)
    # at the lowest Mach number the models agree
    assert ec[0] == pytest.approx(ei[0], rel=1e-3)


def _wom_recipe():
    import importlib.util
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    spec = importlib.util.spec_from_file_location("table_wom_c_ic_recipe", os.path.join(here, "table_wom_c_ic_recipe.py"))
    R = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(R)
    printed = {r[0]: r for r in np.loadtxt(os.path.join(here, "table_wom_c_ic.txt"))}
    recorded = {r[0]: r for r in np.loadtxt(os.path.join(here, "table_wom_c_ic_recipe.txt"))}
    return R, printed, recorded


def test_womersley_model_comparison_table():
    # Table Wom_C_IC (Sec. III.C) at the reading recorded in
    # tests/golden/table_wom_c_ic_recipe.py (the Sec. III.C channel with
    # nu = 0.01 for alpha = 1.253): the printed M_max column is reproduced;
    # at the smallest forcing both models err alike, at the largest the
    # original model errs 3.5x (E_max) and 5.5x (<E>) as much as the
    # incompressible one, as printed; every error is within 25 % of the
    # printed one (the oracle is up to 22 % more accurate at small G, within
    # 7 % at G = 0.15).  One settling period here (three in the recorded
    # table) changes the errors by under 2 %.
    R, printed, recorded = _wom_recipe()
    for G in printed:
        assert R.m_max(G) == pytest.approx(printed[G][1], rel=3e-3)
    got = {}
    for G in (0.005, 0.15):
        orig = R.table_row(G, 1, periods=1)
        pres = R.table_row(G, 0, periods=1)
        got[G] = (orig[0], orig[1], pres[0], pres[1])
        for k in range(4):
            assert 100 * got[G][k] == pytest.approx(recorded[G][2 + k], rel=2e-2)
            assert 100 * got[G][k] == pytest.approx(printed[G][2 + k], rel=0.25)
    assert got[0.005][0] / got[0.005][2] == pytest.approx(1.0, abs=0.1)
    assert got[0.15][0] / got[0.15][2] == pytest.approx(printed[0.15][2] / printed[0.15][4], rel=0.1)
    assert got[0.15][1] / got[0.15][3] == pytest.approx(printed[0.15][3] / printed[0.15][5], rel=0.1)
