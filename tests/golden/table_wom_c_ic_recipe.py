"""Runs the oracle on the pressure-driven Womersley flow of Table Wom_C_IC
(Sec. III.C) for both equilibrium models and writes
tests/golden/table_wom_c_ic_recipe.txt.

Reading of the unstated parameters: the channel, mesh and fluid of the
Sec. III.C profile run (0 <= x <= 2, 0 <= y <= 1 on 40 x 20 cells, NEQ
pressure inlet and outlet, bounce-back walls, rho0 = 1, RT = 16/3, CFL 0.5,
period T = 100) with the viscosity that gives the table's Womersley number:
alpha = (L_y / 2) sqrt(omega / nu) = 1.253 at omega = 2 pi / 100 means
nu = 0.01.  The outlet holds p = 0 and the inlet -L_x G cos(omega t)
(Eq. Wom_AS_Pressure).  M_max = U_max / C with C = sqrt(3 RT) = 4 and U_max
the largest analytic centre-line speed at the eight sample times; this
reproduces the printed M_max column (0.0129 at G = 0.005).  The equilibrium
is initialised from the analytic pressure and velocity; after PERIODS
periods E(u), the relative L2 error of the velocity field against the
closed form, is taken at t = nT/8 over one more period: E_max its largest
value, <E> its mean.

Usage: python tests/golden/table_wom_c_ic_recipe.py     Calls only the oracle.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle as O  # noqa: E402

LX, LY, RT, T, NU, N = 2.0, 1.0, 16.0 / 3.0, 100.0, 0.01, 20
OMEGA = 2 * np.pi / T
PERIODS = 3


def womersley_u(y, t, G):
    # dP/dx = G cos(omega t) drives like a force -G cos(omega t):
    # u = Re{ -G/(i omega) [1 - cosh(l s)/cosh(l)] e^{i omega t} },
    # s = 2y/L_y - 1, l^2 = i omega L_y^2 / (4 nu)
    lam = np.sqrt(1j * OMEGA * LY * LY / (4 * NU))
    s = 2 * y / LY - 1
    return np.real(-G / (1j * OMEGA) * (1 - np.cosh(lam * s) / np.cosh(lam)) * np.exp(1j * OMEGA * t))


def problem(G, model, n=N):
    d = dict(lattice=9, n=(2 * n, n, 1), L=(LX, LY, 1.0), rho0=1.0, RT=RT, tau=NU / RT,
             dt=0.5 * (LY / n) / np.sqrt(3 * RT), bc=(2, 2, 3, 3, 0, 0), pw=[0.0] * 6,
             pw_osc=[-LX * G, 0, 0, 0, 0, 0], omega=OMEGA, phase=0.0, model=model)
    nper = int(round(T / d["dt"]))
    d["dt"] = T / nper
    x, y = O.mesh(d, 0)[1][1:-1], O.mesh(d, 1)[1][1:-1]
    return d, nper, x, y


def initial_state(d, x, y, G):
    D, Q, shp = O.dims(d)
    u0 = np.zeros((2,) + shp)
    u0[0] = womersley_u(y, 0.0, G)[None, :, None]
    p0 = np.broadcast_to((-(LX - x) * G)[None, None, :], shp)
    return O.init(d, rho=1.0 + p0 / RT, u=u0)


def velocity_error(d, f, y, t, G):
    D, Q, shp = O.dims(d)
    _, u, _, _ = O.moments(d, f, t=t)
    ua = np.broadcast_to(womersley_u(y, t, G)[None, :, None], shp)
    return float(np.sqrt(((u[0] - ua) ** 2 + u[1] ** 2).sum() / (ua ** 2).sum()))


def m_max(G):
    U = max(abs(womersley_u(np.array([0.5 * LY]), n * T / 8, G)[0]) for n in range(8))
    return U / np.sqrt(3 * RT)


def table_row(G, model, periods=PERIODS):
    d, nper, x, y = problem(G, model)
    f = O.run(d, initial_state(d, x, y, G), periods * nper)
    t, E = periods * nper * d["dt"], []
    for _ in range(8):
        f = O.run(d, f, nper // 8, t0=t)
        t += (nper // 8) * d["dt"]
        E.append(velocity_error(d, f, y, t, G))
    return max(E), float(np.mean(E)), E


def main():
    rows = []
    for G in (0.005, 0.01, 0.05, 0.1, 0.15):
        t0 = time.time()
        orig = table_row(G, 1)
        pres = table_row(G, 0)
        rows.append(f"{G} {m_max(G):.4f} {100 * orig[0]:.4f} {100 * orig[1]:.4f} {100 * pres[0]:.4f} "
                    f"{100 * pres[1]:.4f} " + " ".join(f"{v:.8e}" for v in orig[2] + pres[2]))
        print(rows[-1][:80], f"({time.time() - t0:.0f} s)", flush=True)
    with open(os.path.join(HERE, "table_wom_c_ic_recipe.txt"), "w") as fh:
        fh.write("# Oracle at the Table Wom_C_IC reading (Sec. III.C); written by table_wom_c_ic_recipe.py\n")
        fh.write(f"# {PERIODS} periods, then E(u) at t = nT/8 over the next one; errors of the first six\n")
        fh.write("# columns in percent; then the 8 + 8 values of E(u) (original, present) as fractions\n")
        fh.write("# G M_max Emax_original Eavg_original Emax_present Eavg_present E_orig[0..7] E_pres[0..7]\n")
        for r in rows:
            fh.write(r + "\n")


if __name__ == "__main__":
    main()
