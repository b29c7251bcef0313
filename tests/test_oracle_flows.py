"""Whole-flow pins of the CPU oracle: analytic solutions the paper uses
(Sec. III) and special cases with closed forms.

Regime note: the scheme is a kinetic solver with a physical relaxation time;
at finite tau = nu/RT the walls carry a kinetic slip ~ tau and the NEQ rule
(non-equilibrium part taken one interface away, Eq. NEQ) an O(tau dx) term.
The paper's wall tests run with tau ~ 1e-3, where the O(dx^2) error
dominates; the wall pins below use the same regime.
"""
import numpy as np
import pytest

import oracle as O
from tests.test_oracle_pins import cfg2

RT_C = 1000.0 / 3.0  # continuum regime for wall tests (tau = nu/RT = 1e-4)


def channel(N, bc, RT, nu=1 / 30.0, G=2.667e-3, stretch=0, uw_top=None, nx=1, cfl=0.5, **kw):
    uw = [[0.0] * 3 for _ in range(6)]
    if uw_top is not None:
        uw[3] = [uw_top, 0.0, 0.0]
    d = dict(lattice=9, n=(nx, N, 1), L=(nx / N, 1.0, 1.0), mesh=(0, stretch, 0), k_stretch=1.5, rho0=1.0,
             RT=RT, tau=nu / RT, dt=1.0, G=(G, 0, 0), bc=(0, 0, bc, bc, 0, 0), uw=uw)
    d.update(kw)
    X, xc = O.mesh(d, 1)
    d["dt"] = cfl * np.diff(X).min() / np.sqrt(3 * RT)
    return d, xc[1:-1]


def run_to(d, f, T, force=None):
    return O.run(d, f, int(round(T / d["dt"])), force=force)


@pytest.mark.parametrize("bc", [O.BOUNCE_BACK, O.NEQ_VELOCITY])
@pytest.mark.parametrize("stretch", [0, 1])
def test_couette_linear_profile_is_exact(bc, stretch):
    # plane Couette (moving top wall, G = 0): the linear profile is a fixed
    # point of the discrete scheme; the flow relaxes to it to rounding
    U = 0.01
    d, y = channel(8, bc, RT=1 / 3, G=0.0, stretch=stretch, uw_top=U)
    D, Q, shp = O.dims(d)
    u0 = np.zeros((2,) + shp)
    u0[0] = (U * y)[None, :, None]
    f = run_to(d, O.init(d, u=u0), 150.0)
    _, u, p, _ = O.moments(d, f)
    np.testing.assert_allclose(u[0, 0, :, 0], U * y, rtol=0, atol=1e-11 * U * 100)
    np.testing.assert_allclose(u[1], 0.0, atol=1e-13)


@pytest.mark.parametrize("bc", [O.BOUNCE_BACK, O.NEQ_VELOCITY])
def test_poiseuille_converges(bc):
    # Eq. (Poiseuille_AS): u = G/(2 nu) y (1 - y), both wall rules
    # (Sec. III.B: both second order, close to each other)
    errs = []
    for N in (8, 16, 32):
        d, y = channel(N, bc, RT_C)
        G, nu = d["G"][0], d["tau"] * d["RT"]
        ua = G / (2 * nu) * y * (1 - y)
        D, Q, shp = O.dims(d)
        u0 = np.zeros((2,) + shp)
        u0[0] = ua[None, :, None]
        f = run_to(d, O.init(d, u=u0), 30.0)
        _, u, _, _ = O.moments(d, f)
        ux = u[0, 0, :, 0]
        errs.append(np.sqrt(((ux - ua) ** 2).sum() / (ua ** 2).sum()))
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] / errs[2] > 16.0          # at least second order over the range
    assert errs[2] < 2e-3


def test_kinetic_slip_scales_with_tau():
    # at finite Knudsen number the bounce-back wall slips by O(tau); the
    # profile error at fixed mesh falls when tau falls at fixed viscosity
    errs = []
    for RT in (1 / 3, 10 / 3):
        d, y = channel(16, O.BOUNCE_BACK, RT)
        G, nu = d["G"][0], d["tau"] * d["RT"]
        ua = G / (2 * nu) * y * (1 - y)
        f = run_to(d, O.init(d), 60.0)
        _, u, _, _ = O.moments(d, f)
        errs.append(np.abs(u[0, 0, :, 0] - ua).max() / ua.max())
    assert errs[0] > 0.02 and errs[1] < errs[0] / 4


def test_pressure_driven_poiseuille():
    # NEQ pressure inlet/outlet (Eq. NEQ, pressure condition) with bounce-back
    # walls: the steady profile is the parabola with G_eff = dp / (rho0 Lx)
    N = 16
    nu, RT, dp, Lx = 1 / 30.0, RT_C, 2.0e-3, 2.0
    d = dict(lattice=9, n=(2 * N, N, 1), L=(Lx, 1.0, 1.0), rho0=1.0, RT=RT, tau=nu / RT, dt=1.0,
             bc=(O.NEQ_PRESSURE, O.NEQ_PRESSURE, O.BOUNCE_BACK, O.BOUNCE_BACK, 0, 0),
             pw=[dp, 0.0, 0.0, 0.0, 0.0, 0.0])
    d["dt"] = 0.5 / N / np.sqrt(3 * RT)
    _, yc = O.mesh(d, 1)
    _, xc = O.mesh(d, 0)
    y, x = yc[1:-1], xc[1:-1]
    ua = dp / Lx / (2 * nu) * y * (1 - y)
    pa = dp * (1 - x / Lx)
    D, Q, shp = O.dims(d)
    u0 = np.zeros((2,) + shp)
    u0[0] = ua[None, :, None]
    f = run_to(d, O.init(d, rho=1.0 + np.broadcast_to(pa[None, None, :], shp) / RT, u=u0), 30.0)
    _, u, p, _ = O.moments(d, f)
    ux = u[0, 0, :, N]
    assert np.sqrt(((ux - ua) ** 2).sum() / (ua ** 2).sum()) < 2e-2
    pc = p[0, N // 2, :]
    assert np.sqrt(((pc - pa) ** 2).sum() / (pa ** 2).sum()) < 2e-2
    assert np.abs(u[1]).max() < 1e-2 * ua.max()


def womersley_u(y, t, G, omega, nu, Ly=1.0):
    # force-driven plane Womersley flow: du/dt = G cos(omega t) + nu u_yy,
    # u(0) = u(Ly) = 0.  u = Re{ G/(i omega) [1 - cosh(l s)/cosh(l)] e^{i omega t} },
    # s = 2y/Ly - 1, l^2 = i omega Ly^2/(4 nu) (the paper's alpha^2 = Ly^2 omega/(4 nu))
    lam = np.sqrt(1j * omega * Ly * Ly / (4 * nu))
    s = 2 * y / Ly - 1
    return np.real(G / (1j * omega) * (1 - np.cosh(lam * s) / np.cosh(lam)) * np.exp(1j * omega * t))


def test_womersley_number_of_the_paper():
    # printed alpha = 3.963 for Ly = 1, T = 100, nu = 1e-3 (Sec. III.C) is
    # alpha = (Ly/2) sqrt(omega / nu)
    assert 0.5 * np.sqrt(2 * np.pi / 100 / 1e-3) == pytest.approx(3.963, abs=5e-4)


def test_womersley_force_driven():
    # oscillating body force G cos(omega t); compare over a period with the
    # closed form, on two meshes
    nu, alpha, G = 0.01, 4.0, 1e-3
    omega = 4 * alpha ** 2 * nu
    errs = []
    for N in (16, 32):
        d, y = channel(N, O.BOUNCE_BACK, RT_C, nu=nu, G=G)
        d["omega"] = omega
        D, Q, shp = O.dims(d)
        u0 = np.zeros((2,) + shp)
        u0[0] = womersley_u(y, 0.0, G, omega, nu)[None, :, None]
        f = O.init(d, u=u0)
        T = 2 * np.pi / omega
        nper = int(round(T / d["dt"]))
        dtp = T / nper
        d["dt"] = dtp
        t, worst = 0.0, 0.0
        for k in range(16):
            f = O.run(d, f, nper // 8, t0=t)
            t += (nper // 8) * dtp
            if k >= 8:
                _, u, _, _ = O.moments(d, f, t=t)
                ua = womersley_u(y, t, G, omega, nu)
                worst = max(worst, np.abs(u[0, 0, :, 0] - ua).max() / (G / omega))
        errs.append(worst)
    assert errs[1] < errs[0] / 3
    assert errs[1] < 2e-2


def _recipe_rows():
    import os
    rows = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "table_ec_vp_recipe.txt")) as fh:
        for ln in fh:
            if ln.strip() and not ln.startswith("#"):
                v = ln.split()
                rows[int(v[0])] = dict(eu=float(v[3]), ep=float(v[4]), ru=float(v[6]), rp=float(v[7]))
    return rows


def test_periodic_flow_table_recipe():
    # Table EC_VP at the paper's recipe (Sec. III.A): Eq. (PF_AS) with its
    # body force, dt = 1e-4, run to the relative velocity change of 1e-6 per
    # 1000 steps; E(u) and E(p) against Eq. (PF_AS).  Both fall at second
    # order from N = 16 to 32, and their ratios to the printed values stay
    # within 20 % of the ratios recorded at the recipe for N = 16, 32 and 64
    # (tests/golden/table_ec_vp_recipe.txt, written by the oracle through
    # tests/golden/table_ec_vp_recipe.py): about 5.3-6.5 for E(u) and
    # 3.6-6.2 for E(p).  The error is a pure amplitude error of the steady
    # field (+5.2 % at N = 16): with dt << tau the interface term h xi.sigma
    # of Eq. (gradient) vanishes and the interface value is the mean of the
    # two cells, so the viscous operator is the wide central stencil, whose
    # amplitude error (k dx)^2 / 3 = 5.1 % at N = 16 is four times that of
    # the compact stencil the printed magnitudes correspond to.
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    import table_ec_vp_recipe as R
    tab = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "table_ec_vp.txt"))
    rec = _recipe_rows()
    errs = {}
    for N in (16, 32):
        eu, ep, amp, n = R.steady_errors(N, 1e-4)
        errs[N] = (eu, ep)
        printed_u, printed_p = tab[tab[:, 0] == N][0, 1:3]
        assert eu / printed_u == pytest.approx(rec[N]["ru"], rel=0.2)
        assert ep / printed_p == pytest.approx(rec[N]["rp"], rel=0.2)
        assert amp > 1.0  # the steady velocity is larger than the analytic one
    assert 1.8 < np.log2(errs[16][0] / errs[32][0]) < 2.2
    assert 1.6 < np.log2(errs[16][1] / errs[32][1]) < 2.2


def pressure_womersley(N):
    # Sec. III.C: the channel 0 <= x <= 2, 0 <= y <= 1 on a 2N x N mesh,
    # NEQ pressure inlet/outlet, bounce-back walls, rho0 = 1, nu = 1e-3,
    # G = 1e-3, RT = 16/3, CFL 0.5, period T = 100 (alpha = 3.963).  The
    # outlet holds p_out = 0 and the inlet p_out - Lx G cos(omega t), the
    # pressure of Eq. (Wom_AS_Pressure) at x = 0, i.e. dP/dx = G cos(omega t)
    Lx, Ly, nu, G, RT, T = 2.0, 1.0, 1e-3, 1e-3, 16.0 / 3.0, 100.0
    omega = 2 * np.pi / T
    d = dict(lattice=9, n=(2 * N, N, 1), L=(Lx, Ly, 1.0), rho0=1.0, RT=RT, tau=nu / RT,
             dt=0.5 * (Ly / N) / np.sqrt(3 * RT), bc=(O.NEQ_PRESSURE, O.NEQ_PRESSURE, O.BOUNCE_BACK, O.BOUNCE_BACK,
                                                       0, 0),
             pw=[0.0] * 6, pw_osc=[-Lx * G, 0, 0, 0, 0, 0], omega=omega, phase=0.0)
    nper = int(round(T / d["dt"]))
    d["dt"] = T / nper
    x, y = O.mesh(d, 0)[1][1:-1], O.mesh(d, 1)[1][1:-1]

    def p_exact(t):
        return -(Lx - x) * G * np.cos(omega * t)

    def u_exact(t):
        # a pressure gradient +G cos(omega t) drives like a force -G cos(omega t)
        return womersley_u(y, t, -G, omega, nu, Ly)

    return d, nper, p_exact, u_exact


def pressure_womersley_errors(N, periods):
    # start from the analytic pressure and velocity (as the paper does), run
    # `periods` periods, then E(p) and E(u) as L2 relative errors over the
    # eight times nT/8 of one more period (over the whole period: the
    # pressure passes through zero at T/4 and 3T/4)
    d, nper, p_exact, u_exact = pressure_womersley(N)
    D, Q, shp = O.dims(d)
    u0 = np.zeros((2,) + shp)
    u0[0] = u_exact(0.0)[None, :, None]
    f = O.init(d, rho=1.0 + np.broadcast_to(p_exact(0.0)[None, None, :], shp) / d["RT"], u=u0)
    f = O.run(d, f, periods * nper)
    t = periods * nper * d["dt"]
    sums = np.zeros(4)
    for _ in range(8):
        f = O.run(d, f, nper // 8, t0=t)
        t += (nper // 8) * d["dt"]
        _, u, p, _ = O.moments(d, f, t=t)
        pa = np.broadcast_to(p_exact(t)[None, None, :], shp)
        ua = np.broadcast_to(u_exact(t)[None, :, None], shp)
        sums += [((p - pa) ** 2).sum(), (pa ** 2).sum(), ((u[0] - ua) ** 2).sum(), (ua ** 2).sum()]
        assert np.abs(u[1]).max() < 2e-2 * np.abs(ua).max() + 1e-6
    return np.sqrt(sums[0] / sums[1]), np.sqrt(sums[2] / sums[3])


def test_pressure_driven_womersley_of_the_paper():
    # the printed bound: the relative pressure error over the period stays
    # under 0.42 % (Sec. III.C); the velocity follows the closed form and
    # converges under refinement (2.0 % at 40 x 20, 0.57 % at 80 x 40)
    ep20, eu20 = pressure_womersley_errors(20, 1)
    assert ep20 < 0.0042
    assert eu20 < 0.03
    ep40, eu40 = pressure_womersley_errors(40, 1)
    assert ep40 < ep20
    assert eu20 / eu40 > 3.0
