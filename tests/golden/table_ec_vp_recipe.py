"""Runs the oracle on the force-driven periodic flow of Sec. III.A at the
paper's own recipe and writes tests/golden/table_ec_vp_recipe.txt.

Recipe (Sec. III.A, Table EC_VP): Eq. (PF_AS) on [0,1]^2, u0 = 0.1, Re = 10
(nu = 0.01), RT = 5, rho0 = 1, dt = 1e-4, N x N uniform cells; the
equilibrium initialised with the analytic velocity and rho = rho0 + p/RT;
run until the relative L2 change of the velocity over 1000 steps is at most
1e-6; E(u) and E(p) are relative L2 errors against Eq. (PF_AS) at the cell
centres (the pressure compared after removing its mean, since the
analytic pressure has zero mean and only its gradient enters the flow).

A second block records E(u) at N = 16 for other time steps (each run to
the same criterion), which shows how the error depends on dt / tau.

Usage: python tests/golden/table_ec_vp_recipe.py [N ...]   (default 16 32 64)
Calls only the oracle.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle as O  # noqa: E402

U0, RT, NU, RHO0 = 0.1, 5.0, 0.01, 1.0


def problem(N, dt):
    d = dict(lattice=9, n=(N, N, 1), L=(1.0, 1.0, 1.0), rho0=RHO0, RT=RT, tau=NU / RT, dt=dt, bc=(0,) * 6)
    _, xc = O.mesh(d, 0)
    X, Y = np.meshgrid(xc[1:-1], xc[1:-1], indexing="xy")
    s2x, s2y, c2x, c2y = (np.sin(2 * np.pi * X), np.sin(2 * np.pi * Y), np.cos(2 * np.pi * X),
                          np.cos(2 * np.pi * Y))
    ua = np.stack([U0 * s2x * s2y, U0 * c2x * c2y])[:, None]
    pa = (0.25 * RHO0 * U0 ** 2 * (np.cos(4 * np.pi * X) - np.cos(4 * np.pi * Y)))[None]
    force = 8 * np.pi ** 2 * NU * ua
    return d, ua, pa, force


def steady_errors(N, dt, crit=1e-6, block=1000, max_steps=3_000_000):
    d, ua, pa, force = problem(N, dt)
    f = O.init(d, rho=RHO0 + pa / RT, u=ua, force=force)
    _, u_prev, _, _ = O.moments(d, f, force=force)
    n = 0
    while n < max_steps:
        f = O.run(d, f, block, force=force, t0=n * dt)
        n += block
        _, u, p, _ = O.moments(d, f, force=force, t=n * dt)
        change = np.sqrt(((u - u_prev) ** 2).sum() / (u ** 2).sum())
        u_prev = u
        if change <= crit:
            break
    eu = np.sqrt(((u - ua) ** 2).sum() / (ua ** 2).sum())
    pm = p - p.mean()
    ep = np.sqrt(((pm - pa) ** 2).sum() / (pa ** 2).sum())
    amp = float((u * ua).sum() / (ua * ua).sum())
    return eu, ep, amp, n


def main():
    Ns = [int(v) for v in sys.argv[1:]] or [16, 32, 64]
    printed = {int(r[0]): (r[1], r[2]) for r in np.loadtxt(os.path.join(HERE, "table_ec_vp.txt"))}
    rows = []
    for N in Ns:
        t0 = time.time()
        eu, ep, amp, n = steady_errors(N, 1e-4)
        pu, pp = printed[N]
        rows.append(f"{N} 1e-4 {n} {eu:.6e} {ep:.6e} {amp:.6f} {eu / pu:.4f} {ep / pp:.4f}")
        print(rows[-1], f"({time.time() - t0:.0f} s)", flush=True)
    scan = []
    for dt in (1e-4, 5e-4, 1e-3, 2e-3, 3e-3, 4e-3, 8.069e-3):
        eu, ep, amp, n = steady_errors(16, dt)
        scan.append(f"{dt:.4e} {dt / (NU / RT):.3f} {n} {eu:.6e} {ep:.6e} {amp:.6f}")
        print(scan[-1], flush=True)
    with open(os.path.join(HERE, "table_ec_vp_recipe.txt"), "w") as fh:
        fh.write("# Oracle at the Table EC_VP recipe (Sec. III.A); written by table_ec_vp_recipe.py\n")
        fh.write("# N dt steps E(u) E(p) amplitude(u.ua/ua.ua) E(u)/printed E(p)/printed\n")
        fh.write("\n".join(rows) + "\n")
        fh.write("# N = 16, other time steps: dt dt/tau steps E(u) E(p) amplitude\n")
        fh.write("\n".join("#scan " + s for s in scan) + "\n")


if __name__ == "__main__":
    main()
