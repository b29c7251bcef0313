"""Second, independent statement of one DUGKS step for every boundary kind
and both mesh kinds, written in whole-array numpy form.

It pins the C oracle's bookkeeping (point sets, indices, weights, signs,
wall rules) on small meshes.  It shares nothing with the oracle: its own
lattice tables, mesh, ghost layer (built axis by axis in the reverse order),
interface interpolation, cross-point values (interpolate along the normal to
every interface, then along the tangent to the interface's edges), wall
rules, moments and update, with the convex combinations written in
deviation form f + B (g - f).  It is not used by the product.

Sources (Wu, Shi, Chai & Wang): Eq. (icfeq) / Eq. (feq), Eq. (S),
Eq. (macro_values), Eq. (f_bar_+), Eq. (gradient), Eqs. (BB), (NEQ),
Eq. (original_f), Eq. (microflux), Eq. (f_tilde_+), Eq. (evolution_equation);
tanh mesh of Eq. (Nonuniform_mesh).  Readings as in the oracle: ghost
centres mirrored in the wall and filled by linear extrapolation; the NEQ
point x_c is the opposite interface of the wall cell; the wall rules replace
only the velocities entering the domain and act before the interface
moments; the interface acceleration is interpolated like f-bar-plus.
"""
import numpy as np

PERIODIC, NEQ_VELOCITY, NEQ_PRESSURE, BOUNCE_BACK = 0, 1, 2, 3


def lattice(lat):
    """velocity set in the order e_x outer, e_y, e_z inner: D2Q9, D3Q19
    (the |e|^2 = 3 corners dropped) or D3Q27; weights from the 1-D rule
    2/3, 1/6 (D3Q19: 1/3, 1/18, 1/36)"""
    one = {-1: 1 / 6, 0: 2 / 3, 1: 1 / 6}
    if lat == 9:
        es = [(ex, ey, 0) for ex in (-1, 0, 1) for ey in (-1, 0, 1)]
        W = [one[ex] * one[ey] for ex, ey, _ in es]
    elif lat == 27:
        es = [(ex, ey, ez) for ex in (-1, 0, 1) for ey in (-1, 0, 1) for ez in (-1, 0, 1)]
        W = [one[ex] * one[ey] * one[ez] for ex, ey, ez in es]
    else:
        es = [(ex, ey, ez) for ex in (-1, 0, 1) for ey in (-1, 0, 1) for ez in (-1, 0, 1)
              if abs(ex) + abs(ey) + abs(ez) < 3]
        W = [{0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[abs(ex) + abs(ey) + abs(ez)] for ex, ey, ez in es]
    e = np.array(es, dtype=np.int64)
    opp = [es.index((-a, -b, -c)) for a, b, c in es]
    return e, np.array(W), np.array(opp)


def axis_faces(cfg, a):
    """face coordinates X_0..X_N of axis a (uniform, Eq. (Nonuniform_mesh), or
    given)"""
    N, L = int(cfg["n"][a]), float(cfg["L"][a])
    i = np.arange(N + 1) / N
    kind = cfg.get("mesh", (0, 0, 0))[a]
    if kind == 2:  # caller-given coordinates
        return np.array(cfg["faces"][a], dtype=np.float64)
    if kind:
        k = float(cfg["k_stretch"])
        X = L * (0.5 + np.tanh(k * (i - 0.5)) / (2.0 * np.tanh(0.5 * k)))
    else:
        X = L * i
    X[0], X[-1] = 0.0, L
    return X


def _nax(a):
    # numpy axis of spatial axis a in arrays laid out [q or comp, z, y, x]
    return 3 - a


def _take(v, a, idx):
    sl = [slice(None)] * v.ndim
    sl[_nax(a)] = idx
    return v[tuple(sl)]


class _Mesh:
    def __init__(self, cfg, D):
        self.D = D
        self.X, self.xe, self.dl, self.per = [], [], [], []
        for a in range(D):
            X = axis_faces(cfg, a)
            xc = 0.5 * (X[1:] + X[:-1])
            per = cfg["bc"][2 * a] == PERIODIC
            L = X[-1]
            if per:
                lo, hi = xc[-1] - L, xc[0] + L
            else:
                lo, hi = 2 * X[0] - xc[0], 2 * X[-1] - xc[-1]
            self.X.append(X)
            self.xe.append(np.concatenate([[lo], xc, [hi]]))  # centres with ghost/wrapped ends
            self.dl.append(X[1:] - X[:-1])
            self.per.append(per)

    def pad(self, v):
        """one ghost layer on every active axis, built z, then y, then x
        (tensor-product extrapolation on wall axes, wrap on periodic ones)"""
        for a in reversed(range(self.D)):
            if self.per[a]:
                lo, hi = _take(v, a, slice(-1, None)), _take(v, a, slice(0, 1))
            else:
                x = self.xe[a]
                v0, v1 = _take(v, a, slice(0, 1)), _take(v, a, slice(1, 2))
                w0, w1 = _take(v, a, slice(-1, None)), _take(v, a, slice(-2, -1))
                lo = v0 + (x[0] - x[1]) / (x[2] - x[1]) * (v1 - v0)
                hi = w0 + (x[-1] - x[-2]) / (x[-3] - x[-2]) * (w1 - w0)
            v = np.concatenate([lo, v, hi], axis=_nax(a))
        return v

    def to_faces(self, v, a):
        """linear interpolation along a from the (padded) centres to the n+1
        interfaces of axis a; v has n+2 entries along a"""
        x, X = self.xe[a], self.X[a]
        shp = [1, 1, 1, 1]
        shp[_nax(a)] = -1
        w = ((X - x[:-1]) / (x[1:] - x[:-1])).reshape(shp)
        L, R = _take(v, a, slice(0, -1)), _take(v, a, slice(1, None))
        return L + w * (R - L)

    def normal_diff(self, v, a):
        x = self.xe[a]
        shp = [1, 1, 1, 1]
        shp[_nax(a)] = -1
        return (_take(v, a, slice(1, None)) - _take(v, a, slice(0, -1))) / (x[1:] - x[:-1]).reshape(shp)

    def interior(self, v, a):
        """drop the ghost layer along a"""
        return _take(v, a, slice(1, -1))


def _acc(cfg, D, Gsp, gfac):
    G0 = np.array([float(g) for g in cfg.get("G", (0, 0, 0))][:D]).reshape(D, 1, 1, 1)
    return gfac * (G0 + Gsp)


def step(cfg, f, force=None, t=0.0):
    lat = int(cfg["lattice"])
    D = 2 if lat == 9 else 3
    e, W, opp = lattice(lat)
    Q = len(W)
    RT, rho0, tau, dt = (float(cfg[k]) for k in ("RT", "rho0", "tau", "dt"))
    orig = int(cfg.get("model", 0)) == 1
    c = np.sqrt(3.0 * RT)
    xi = c * e[:, :D].astype(float)
    h = 0.5 * dt
    om, ph = float(cfg.get("omega", 0.0)), float(cfg.get("phase", 0.0))
    g_n, g_h = np.cos(om * t + ph), np.cos(om * (t + h) + ph)
    mesh = _Mesh(cfg, D)
    f = np.asarray(f, dtype=np.float64)
    shp = f.shape[1:]
    Wb = W.reshape(Q, 1, 1, 1)

    def macro(g, G, half):
        rho = g.sum(0)
        j = np.tensordot(xi.T, g, axes=(1, 0))
        m = rho if orig else rho0
        return rho, (j + m * G * half) / m

    def equilibrium(rho, u):
        xu = np.tensordot(xi, u, axes=(1, 0))
        uu = (u * u).sum(0)
        poly = xu / RT + xu * xu / (2 * RT * RT) - uu / (2 * RT)
        return Wb * (rho * (1 + poly) if orig else rho + rho0 * poly)

    def source(u, G, feq):
        return (np.tensordot(xi, G, axes=(1, 0)) - (u * G).sum(0)) / RT * feq

    Gsp = np.zeros((D,) + shp) if force is None else np.asarray(force, dtype=np.float64)
    Gpad = mesh.pad(Gsp)

    # Eq. (f_bar_+) in deviation form
    Gc = _acc(cfg, D, Gsp, g_n)
    rho, u = macro(f, Gc, dt / 2)
    feq = equilibrium(rho, u)
    B1, C1 = 3 * h / (2 * tau + dt), 3 * tau * h / (2 * tau + dt)
    phi = f + B1 * (feq - f) + C1 * source(u, Gc, feq)
    P = mesh.pad(phi)

    B7, C7 = h / (2 * tau + h), tau * h / (2 * tau + h)
    out = phi + (phi - f) / 3.0  # Eq. (f_tilde_+)
    for a in range(D):
        # Eq. (gradient) on every interface of axis a
        core = P
        for b in range(D):
            if b != a:
                core = mesh.interior(core, b)
        fb = mesh.to_faces(core, a) - h * xi[:, a].reshape(Q, 1, 1, 1) * mesh.normal_diff(core, a)
        for b in range(D):
            if b == a:
                continue
            Pb = P
            for c2 in range(D):
                if c2 != a and c2 != b:
                    Pb = mesh.interior(Pb, c2)
            edges = mesh.to_faces(mesh.to_faces(Pb, a), b)  # cross points (n_a+1) x (n_b+1)
            shp_b = [1, 1, 1, 1]
            shp_b[_nax(b)] = -1
            sig = (_take(edges, b, slice(1, None)) - _take(edges, b, slice(0, -1))) / mesh.dl[b].reshape(shp_b)
            fb = fb - h * xi[:, b].reshape(Q, 1, 1, 1) * sig
        # acceleration at the interfaces, time t_n + h
        Gcore = Gpad
        for b in range(D):
            if b != a:
                Gcore = mesh.interior(Gcore, b)
        Gb = _acc(cfg, D, mesh.to_faces(Gcore, a), g_h)
        # walls: Eqs. (BB), (NEQ) for the velocities entering the domain
        if not mesh.per[a]:
            n_a = len(mesh.X[a]) - 1
            pre = fb.copy()
            for side, fw, fo, out_n in ((0, 0, 1, -1), (1, n_a, n_a - 1, 1)):
                s = 2 * a + side
                kind = int(cfg["bc"][s])
                inn = np.nonzero(e[:, a] * out_n < 0)[0]
                uw = np.array([float(v) for v in cfg.get("uw", [[0, 0, 0]] * 6)[s]][:D])
                wall = _take(pre, a, slice(fw, fw + 1))
                if kind == BOUNCE_BACK:
                    new = wall[opp[inn]] + (2 * rho0 * W[inn] * (xi[inn] @ uw) / RT).reshape(-1, 1, 1, 1)
                else:
                    other = _take(pre, a, slice(fo, fo + 1))
                    Go = _take(Gb, a, slice(fo, fo + 1))
                    rc, uc = macro(other, Go, h / 2)
                    if kind == NEQ_VELOCITY:
                        ra = rc
                        ua = np.broadcast_to(uw.reshape(D, 1, 1, 1), uc.shape)
                    else:
                        p_w = float(cfg.get("pw", [0.0] * 6)[s]) + float(cfg.get("pw_osc", [0.0] * 6)[s]) * g_h
                        ra = np.full_like(rc, rho0 + p_w / RT)
                        ua = uc
                    new = (equilibrium(ra, ua) + other - equilibrium(rc, uc))[inn]
                sl = [slice(None)] * 4
                sl[0] = inn
                sl[_nax(a)] = slice(fw, fw + 1)
                fb[tuple(sl)] = new
        # interface moments and the original distribution (inverse of Eq. (original_f))
        rb, ub = macro(fb, Gb, h / 2)
        feqb = equilibrium(rb, ub)
        fo_ = fb + B7 * (feqb - fb) + C7 * source(ub, Gb, feqb)
        flux = xi[:, a].reshape(Q, 1, 1, 1) * fo_
        shp_a = [1, 1, 1, 1]
        shp_a[_nax(a)] = -1
        # Eq. (evolution_equation): dt / |V| sum_j (xi.n_j) f s_j = dt sum_a (flux+ - flux-) / Delta_a
        out = out - dt * (_take(flux, a, slice(1, None)) - _take(flux, a, slice(0, -1))) / mesh.dl[a].reshape(shp_a)
    return out


def run(cfg, f, nsteps, force=None, t0=0.0):
    t = t0
    for _ in range(nsteps):
        f = step(cfg, f, force, t)
        t += float(cfg["dt"])
    return f
