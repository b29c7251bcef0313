"""Independent numpy restatement of one DUGKS step on a fully periodic,
uniform mesh, written in stencil form (np.roll) rather than over explicit
point sets.  It exists only to pin the oracle's bookkeeping (indices, point
sets, signs) on small inputs; it is not used by the product.

On a uniform periodic mesh the face value of f-bar-plus is the mean of the
two cells, the normal gradient the two-cell difference, and each tangential
gradient the mean of the two cells' central differences (the difference of
the bilinear cross-point values over the face width).
"""
import numpy as np


def lattice(lat):
    if lat == 9:
        w1 = {-1: 1 / 6, 0: 2 / 3, 1: 1 / 6}
        es = [(ex, ey, 0) for ex in (-1, 0, 1) for ey in (-1, 0, 1)]
        W = [w1[ex] * w1[ey] for ex, ey, _ in es]
    elif lat == 27:
        w1 = {-1: 1 / 6, 0: 2 / 3, 1: 1 / 6}
        es = [(ex, ey, ez) for ex in (-1, 0, 1) for ey in (-1, 0, 1) for ez in (-1, 0, 1)]
        W = [w1[ex] * w1[ey] * w1[ez] for ex, ey, ez in es]
    else:
        es = [(ex, ey, ez) for ex in (-1, 0, 1) for ey in (-1, 0, 1) for ez in (-1, 0, 1)
              if ex * ex + ey * ey + ez * ez < 3]
        W = [{0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[ex * ex + ey * ey + ez * ez] for ex, ey, ez in es]
    return np.array(es, dtype=float), np.array(W)


def _ax(a):
    # array layout [q or comp, z, y, x]: spatial axis a -> numpy axis 3 - a
    return 3 - a


def step(lat, f, rho0, RT, tau, dt, dx, Gfield=None, gt=1.0, gth=1.0, G0=(0, 0, 0)):
    e, W = lattice(lat)
    D = 2 if lat == 9 else 3
    c = np.sqrt(3 * RT)
    xi = c * e[:, :D]
    h = dt / 2
    Q = len(W)
    shp = f.shape[1:]

    def moments(g):
        return g.sum(0), np.tensordot(xi.T, g, axes=(1, 0))

    def feq_S(rho, u, G):
        xu = np.tensordot(xi, u, axes=(1, 0))
        uu = (u * u).sum(0)
        feq = W[:, None, None, None] * (rho + rho0 * (xu / RT + xu ** 2 / (2 * RT ** 2) - uu / (2 * RT)))
        xg = np.tensordot(xi, G, axes=(1, 0))
        ug = (u * G).sum(0)
        return feq, (xg - ug) / RT * feq

    Gsp = np.zeros((D,) + shp) if Gfield is None else Gfield
    G0a = np.array(G0[:D]).reshape(D, 1, 1, 1)
    Gc = gt * (G0a + Gsp)
    rho, j = moments(f)
    u = j / rho0 + dt / 2 * Gc
    feq, S = feq_S(rho, u, Gc)
    phi = (2 * tau - h) / (2 * tau + dt) * f + 3 * h / (2 * tau + dt) * feq + 3 * tau * h / (2 * tau + dt) * S

    fnew = 4 / 3 * phi - 1 / 3 * f
    for a in range(D):
        na = _ax(a)
        R = np.roll(phi, -1, axis=na)
        fb = 0.5 * (phi + R) - h * xi[:, a].reshape(Q, 1, 1, 1) * (R - phi) / dx[a]
        for b in range(D):
            if b == a:
                continue
            nb = _ax(b)
            dL = (np.roll(phi, -1, axis=nb) - np.roll(phi, 1, axis=nb)) / (2 * dx[b])
            dR = np.roll(dL, -1, axis=na)
            fb = fb - h * xi[:, b].reshape(Q, 1, 1, 1) * 0.5 * (dL + dR)
        Gb = gth * (G0a + 0.5 * (Gsp + np.roll(Gsp, -1, axis=na)))
        rb, jb = moments(fb)
        ub = jb / rho0 + h / 2 * Gb
        feqb, Sb = feq_S(rb, ub, Gb)
        ff = 2 * tau / (2 * tau + h) * fb + h / (2 * tau + h) * feqb + tau * h / (2 * tau + h) * Sb
        # ff is the value on the +a face of each cell
        fnew = fnew - dt / dx[a] * xi[:, a].reshape(Q, 1, 1, 1) * (ff - np.roll(ff, 1, axis=na))
    return fnew
