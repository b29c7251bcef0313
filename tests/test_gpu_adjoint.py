"""Adjoint on the GPU vs the oracle's tape-free adjoint and vs central finite
differences of the GPU forward (FP64): periodic meshes on the fast reverse
pass, meshes with walls (bounce-back, NEQ velocity and pressure; uniform
and stretched) on the general one."""
import numpy as np
import pytest

import oracle as O
from synthetic import field, gaussian_bumps, perturb

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1411_6121_amd")

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def periodic_cfg(lat, n, mesh=0, **kw):
    D = 2 if lat == 9 else 3
    d = dict(lattice=lat, dtype="f64", n=tuple(n) if D == 3 else (n[0], n[1], 1),
             L=tuple(float(v) for v in n) if D == 3 else (float(n[0]), float(n[1]), 1.0),
             mesh=(mesh,) * 3 if D == 3 else (mesh, mesh, 0), k_stretch=1.5, rho0=1.0, RT=1 / 3, tau=0.45, dt=0.5,
             bc=(0,) * 6, G=(1e-3, -5e-4, 2e-4), omega=0.7, phase=0.3)
    d.update(kw)
    return d


@pytest.mark.parametrize("lat,n,mesh", [(9, (37, 29), 0), (9, (21, 18), 1), (19, (13, 11, 9), 0),
                                        (9, (1, 7), 0), (19, (5, 4, 1), 0), (19, (2, 1, 3), 1)])
def test_step_adjoint_matches_oracle(lat, n, mesh):
    say(f"[adjoint step] lattice={lat} n={n} mesh={mesh}")
    cfg = periodic_cfg(lat, n, mesh)
    Q, D, shp = M.shape_of(cfg)
    Gf = field(21, (D,) + shp, 2e-3)
    f = perturb(22, O.init(cfg, rho=1 + field(23, shp, 0.02), u=field(24, (D,) + shp, 0.05), force=Gf), 1e-2)
    lam = field(25, f.shape, 1.0)
    t = 0.4
    gref = np.zeros_like(Gf)
    ref = O.step_adjoint(cfg, f, lam, force=Gf, t=t, grad_force=gref)
    buf = torch.empty((Q,) + shp, dtype=torch.float64, device="cuda")
    ctx = M.dugks_init(cfg, buf)
    try:
        out = torch.empty_like(buf)
        gG = torch.zeros((D,) + shp, dtype=torch.float64, device="cuda")
        M.dugks_step_adjoint(ctx, dev(f), dev(lam), out, dev(Gf), t, gG)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-12
        gg = gG.cpu().numpy()
        assert np.abs(gg - gref).max() / np.abs(gref).max() < 1e-11
    finally:
        M.dugks_destroy(ctx)


LID = [[0, 0, 0], [0, 0, 0], [0, 0, 0], [0.05, 0, 0], [0, 0, 0], [0, 0, 0]]
MOVING = [[0, 0.02, 0], [0, -0.01, 0], [0.03, 0, 0], [0.05, 0, 0], [0, 0, 0.01], [0.02, 0, 0]]
WALL_CASES = [
    ("q9-neq-cavity", 9, (37, 29), (1, 1, 1, 1, 0, 0), 0, LID, (0,) * 6),
    ("q9-bb-moving-tanh", 9, (33, 26), (3, 3, 3, 3, 0, 0), 1, MOVING, (0,) * 6),
    ("q9-neqp-bb", 9, (40, 17), (2, 2, 3, 3, 0, 0), 0, LID, (3e-3, -2e-3, 0, 0, 0, 0)),
    ("q9-mixed-tanh", 9, (23, 31), (1, 3, 2, 1, 0, 0), 1, MOVING, (0, 0, 1e-3, 0, 0, 0)),
    ("q9-channel-tanh", 9, (6, 32), (0, 0, 1, 1, 0, 0), 1, LID, (0,) * 6),
    ("q9-minimal", 9, (2, 2), (1, 3, 2, 1, 0, 0), 0, MOVING, (0, 0, 1e-3, 0, 0, 0)),
    ("q19-neq-cube", 19, (13, 11, 9), (1,) * 6, 0, LID, (0,) * 6),
    ("q19-mixed-tanh", 19, (9, 12, 7), (3, 2, 1, 3, 0, 0), 1, MOVING, (0, 2e-3, 0, 0, 0, 0)),
    ("q19-minimal", 19, (2, 2, 2), (1, 1, 3, 3, 2, 1), 0, MOVING, (0, 0, 0, 0, 1e-3, 0)),
    ("q19-one-column-periodic-x", 19, (1, 6, 5), (0, 0, 3, 3, 1, 1), 1, MOVING, (0,) * 6),
    ("q19-one-plane-periodic-z", 19, (7, 6, 1), (1, 3, 1, 1, 0, 0), 0, MOVING, (0,) * 6),
]


@pytest.mark.parametrize("name,lat,n,bc,mesh,uw,pw", WALL_CASES, ids=[c[0] for c in WALL_CASES])
def test_step_adjoint_walls_match_oracle(name, lat, n, bc, mesh, uw, pw):
    say(f"[adjoint walls] {name} n={n}")
    cfg = periodic_cfg(lat, n, mesh, bc=bc, uw=uw, pw=list(pw))
    Q, D, shp = M.shape_of(cfg)
    Gf = field(31, (D,) + shp, 2e-3)
    f = perturb(32, O.init(cfg, rho=1 + field(33, shp, 0.02), u=field(34, (D,) + shp, 0.05), force=Gf), 1e-2)
    lam = field(35, f.shape, 1.0)
    t = 0.4
    gref = np.zeros_like(Gf)
    ref = O.step_adjoint(cfg, f, lam, force=Gf, t=t, grad_force=gref)
    buf = torch.empty((Q,) + shp, dtype=torch.float64, device="cuda")
    ctx = M.dugks_init(cfg, buf)
    try:
        out = torch.empty_like(buf)
        gG = torch.zeros((D,) + shp, dtype=torch.float64, device="cuda")
        M.dugks_step_adjoint(ctx, dev(f), dev(lam), out, dev(Gf), t, gG)
        torch.cuda.synchronize()
        assert np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max() < 1e-12
        assert np.abs(gG.cpu().numpy() - gref).max() / np.abs(gref).max() < 1e-11
        # without a force field and without a gradient request
        ref0 = O.step_adjoint(cfg, f, lam, t=t)
        M.dugks_step_adjoint(ctx, dev(f), dev(lam), out, None, t, None)
        torch.cuda.synchronize()
        assert np.abs(out.cpu().numpy() - ref0).max() / np.abs(ref0).max() < 1e-12
    finally:
        M.dugks_destroy(ctx)


@pytest.mark.parametrize("lat,n,bc,mesh", [(9, (40, 17), (2, 2, 3, 3, 0, 0), 0),
                                           (19, (9, 12, 7), (2, 2, 1, 3, 3, 3), 1)], ids=["q9", "q19"])
def test_step_adjoint_oscillating_pressure_matches_oracle(lat, n, bc, mesh):
    # pressure sides whose wall pressure follows the time factor (pw +
    # pw_osc g(t)): the linearisation point of the wall rule moves with t
    say(f"[adjoint walls] oscillating pressure q{lat} n={n}")
    cfg = periodic_cfg(lat, n, mesh, bc=bc, uw=MOVING, pw=[1e-3, -1e-3, 0, 0, 0, 0],
                       pw_osc=[3e-3, 1e-3, 0, 0, 0, 0])
    Q, D, shp = M.shape_of(cfg)
    Gf = field(41, (D,) + shp, 2e-3)
    f = perturb(42, O.init(cfg, rho=1 + field(43, shp, 0.02), u=field(44, (D,) + shp, 0.05), force=Gf), 1e-2)
    lam = field(45, f.shape, 1.0)
    buf = torch.empty((Q,) + shp, dtype=torch.float64, device="cuda")
    ctx = M.dugks_init(cfg, buf)
    try:
        out = torch.empty_like(buf)
        for t in (0.4, 2.9):
            gref = np.zeros_like(Gf)
            ref = O.step_adjoint(cfg, f, lam, force=Gf, t=t, grad_force=gref)
            gG = torch.zeros((D,) + shp, dtype=torch.float64, device="cuda")
            M.dugks_step_adjoint(ctx, dev(f), dev(lam), out, dev(Gf), t, gG)
            torch.cuda.synchronize()
            assert np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max() < 1e-12
            assert np.abs(gG.cpu().numpy() - gref).max() / np.abs(gref).max() < 1e-11
    finally:
        M.dugks_destroy(ctx)


@pytest.mark.parametrize("lat,n,mesh", [(9, (21, 18), 1), (19, (7, 6, 5), 0)])
def test_general_reverse_pass_on_periodic_meshes(lat, n, mesh, monkeypatch):
    # the wall-capable reverse pass, forced on a periodic mesh, against the
    # oracle (there face n of each axis is transposed as a face of its own)
    say(f"[adjoint general pass, periodic] lattice={lat} n={n}")
    monkeypatch.setenv("DUGKS_ADJOINT_GENERAL", "1")
    cfg = periodic_cfg(lat, n, mesh)
    Q, D, shp = M.shape_of(cfg)
    Gf = field(36, (D,) + shp, 2e-3)
    f = perturb(37, O.init(cfg, rho=1 + field(38, shp, 0.02), u=field(39, (D,) + shp, 0.05), force=Gf), 1e-2)
    lam = field(40, f.shape, 1.0)
    gref = np.zeros_like(Gf)
    ref = O.step_adjoint(cfg, f, lam, force=Gf, t=0.4, grad_force=gref)
    buf = torch.empty((Q,) + shp, dtype=torch.float64, device="cuda")
    ctx = M.dugks_init(cfg, buf)
    try:
        out = torch.empty_like(buf)
        gG = torch.zeros((D,) + shp, dtype=torch.float64, device="cuda")
        M.dugks_step_adjoint(ctx, dev(f), dev(lam), out, dev(Gf), 0.4, gG)
        torch.cuda.synchronize()
        assert np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max() < 1e-12
        assert np.abs(gG.cpu().numpy() - gref).max() / np.abs(gref).max() < 1e-11
    finally:
        M.dugks_destroy(ctx)


def test_cavity_force_gradient_matches_fd():
    # a cavity-type control problem: D2Q9 lid-driven cavity on a tanh mesh
    # with NEQ walls, force field to be found; loss = MSE of the velocity
    # after N steps vs a target run; checkpointed adjoint vs central FD of
    # the GPU forward on seeded components (interior, next to walls, corners)
    from paper_1411_6121_amd.autograd import rollout

    n, nsteps = 48, 300
    say(f"[cavity force gradient vs FD] {n}^2 tanh, NEQ walls, {nsteps} steps")
    cfg = periodic_cfg(9, (n, n), 1, bc=(1, 1, 1, 1, 0, 0), uw=LID, tau=0.3, G=(0, 0, 0), omega=0.0, phase=0.0)
    Q, D, shp = M.shape_of(cfg)
    Gtar = dev(field(50, (D,) + shp, 1e-4))
    zero_u = torch.zeros((D,) + shp, dtype=torch.float64, device="cuda")
    with torch.no_grad():
        u_tar = rollout(cfg, Gtar, zero_u, nsteps)

    def loss_of(G):
        return ((rollout(cfg, G, zero_u, nsteps) - u_tar) ** 2).mean()

    G = torch.zeros((D,) + shp, dtype=torch.float64, device="cuda", requires_grad=True)
    L = loss_of(G)
    L.backward()
    grad = G.grad.cpu().numpy()
    idx = [(0, 0, 0, 0), (1, 0, n - 1, n - 1), (0, 0, n - 1, 3), (1, 0, 5, 0), (0, 0, 1, 1), (1, 0, 24, 17),
           (0, 0, 40, n - 2), (1, 0, 12, 33)]
    eps = 1e-5
    for ix in idx:
        with torch.no_grad():
            Gp = torch.zeros_like(G)
            Gp[ix] = eps
            fd = (loss_of(Gp) - loss_of(-Gp)).item() / (2 * eps)
        assert grad[ix] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(grad).max())


def test_walled_d3q19_rollout_gradients_match_fd():
    # D3Q19 cavity with mixed walls on a tanh mesh: gradients of the final
    # velocity MSE with respect to the initial velocity field (through the
    # initial-state VJP) and the body-force field (through every adjoint
    # step), each against central FD of the GPU forward on seeded components
    from paper_1411_6121_amd.autograd import rollout

    n, nsteps = (10, 9, 8), 40
    say(f"[walled d3q19 rollout gradients vs FD] n={n}, {nsteps} steps")
    cfg = periodic_cfg(19, n, 1, bc=(1, 3, 1, 1, 3, 2), uw=MOVING, pw=[0, 0, 0, 0, 0, 1e-3], tau=0.35,
                       G=(0, 0, 0), omega=0.0, phase=0.0)
    Q, D, shp = M.shape_of(cfg)
    u0 = dev(field(60, (D,) + shp, 0.02))
    G0 = dev(field(61, (D,) + shp, 1e-4))
    with torch.no_grad():
        u_tar = rollout(cfg, dev(field(62, (D,) + shp, 1e-4)), dev(field(63, (D,) + shp, 0.02)), nsteps)

    def loss_of(G, u):
        return ((rollout(cfg, G, u, nsteps) - u_tar) ** 2).mean()

    G = G0.clone().requires_grad_(True)
    u = u0.clone().requires_grad_(True)
    loss_of(G, u).backward()
    gG, gu = G.grad.cpu().numpy(), u.grad.cpu().numpy()
    idx = [(0, 0, 0, 0), (1, 7, 8, 9), (2, 3, 0, 5), (0, 7, 4, 0), (1, 4, 4, 4), (2, 0, 8, 9)]
    # steps balance truncation against the rounding floor of the loss
    for name, base, grad, eps in (("u0", u0, gu, 1e-6), ("force", G0, gG, 1e-5)):
        for ix in idx:
            with torch.no_grad():
                p = torch.zeros_like(base)
                p[ix] = eps
                lp = loss_of(G0 + p, u0) if name == "force" else loss_of(G0, u0 + p)
                lm = loss_of(G0 - p, u0) if name == "force" else loss_of(G0, u0 - p)
                fd = (lp - lm).item() / (2 * eps)
            assert grad[ix] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(grad).max()), (name, ix)


def test_init_and_readout_vjp_match_oracle():
    say("[init vjp]")
    cfg = periodic_cfg(9, (16, 12))
    Q, D, shp = M.shape_of(cfg)
    u = field(28, (D,) + shp, 0.05)
    Gf = field(29, (D,) + shp, 1e-3)
    lam0 = field(30, (Q,) + shp, 1.0)
    gu_ref, gg_ref = np.zeros_like(u), np.zeros_like(Gf)
    O.init_adjoint(cfg, lam0, u=u, force=Gf, t0=0.2, grad_u=gu_ref, grad_force=gg_ref)
    buf = torch.empty((Q,) + shp, dtype=torch.float64, device="cuda")
    ctx = M.dugks_init(cfg, buf)
    try:
        gu = torch.zeros((D,) + shp, dtype=torch.float64, device="cuda")
        gg = torch.zeros_like(gu)
        M.dugks_init_vjp(ctx, dev(lam0), dev(u), dev(Gf), 0.2, gu, gg)
        np.testing.assert_allclose(gu.cpu().numpy(), gu_ref, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(gg.cpu().numpy(), gg_ref, rtol=1e-12, atol=1e-15)
        # read-out: lam = xi.grad_u/rho0, grad_force += g(t) dt/2 grad_u
        e, _ = O.lattice(9)
        gu_out = field(31, (D,) + shp, 1.0)
        lam = torch.empty((Q,) + shp, dtype=torch.float64, device="cuda")
        gg2 = torch.zeros_like(gu)
        M.dugks_moments_vjp(ctx, lam, None, dev(gu_out), 0.6, gg2)
        xi = np.sqrt(3 * cfg["RT"]) * e[:, :2]
        np.testing.assert_allclose(lam.cpu().numpy(), np.tensordot(xi, gu_out, axes=(1, 0)), rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(gg2.cpu().numpy(), np.cos(0.7 * 0.6 + 0.3) * 0.25 * gu_out, rtol=1e-14)
    finally:
        M.dugks_destroy(ctx)


def test_rollout_gradient_matches_oracle_chain():
    # autograd rollout (sqrt(N) checkpoints) vs the oracle's chained adjoint
    from paper_1411_6121_amd.autograd import rollout

    say("[rollout vs oracle]")
    cfg = periodic_cfg(9, (12, 10))
    Q, D, shp = M.shape_of(cfg)
    nsteps = 9
    Gf = field(40, (D,) + shp, 1e-3)
    u0 = field(41, (D,) + shp, 0.02)
    target = field(42, (D,) + shp, 0.02)
    # oracle chain
    fs = [O.init(cfg, u=u0, force=Gf)]
    for k in range(nsteps):
        fs.append(O.step(cfg, fs[-1], Gf, k * cfg["dt"]))
    _, u, _, _ = O.moments(cfg, fs[-1], force=Gf, t=nsteps * cfg["dt"])
    du = 2 * (u - target) / u.size
    e, _ = O.lattice(9)
    xi = np.sqrt(3 * cfg["RT"]) * e[:, :2]
    lam = np.tensordot(xi, du, axes=(1, 0)) / cfg["rho0"]
    gG = np.cos(cfg["omega"] * nsteps * cfg["dt"] + cfg["phase"]) * cfg["dt"] / 2 * du
    for k in reversed(range(nsteps)):
        lam = O.step_adjoint(cfg, fs[k], lam, force=Gf, t=k * cfg["dt"], grad_force=gG)
    gu = np.zeros_like(u0)
    O.init_adjoint(cfg, lam, u=u0, force=Gf, t0=0.0, grad_u=gu, grad_force=gG)
    # GPU
    Gt = dev(Gf).requires_grad_(True)
    ut = dev(u0).requires_grad_(True)
    uN = rollout(cfg, Gt, ut, nsteps)
    loss = ((uN - dev(target)) ** 2).mean()
    loss.backward()
    np.testing.assert_allclose(uN.detach().cpu().numpy(), u, rtol=0, atol=1e-14)
    np.testing.assert_allclose(Gt.grad.cpu().numpy(), gG, rtol=1e-10, atol=1e-14 * np.abs(gG).max())
    np.testing.assert_allclose(ut.grad.cpu().numpy(), gu, rtol=1e-10, atol=1e-14 * np.abs(gu).max())


def test_force_field_gradient_matches_fd():
    # the adjoint workload: D2Q9 256^2 periodic, tau = 1 (nu = 1/3), force
    # field target = 8 Gaussian bumps (amplitude 1e-5, width 16 cells),
    # loss = MSE of the final velocity after N steps from rest vs the target
    # run; gradient at zero force by the checkpointed adjoint, checked
    # against central differences of the GPU forward on 16 seeded components
    from paper_1411_6121_amd.autograd import rollout

    n, nsteps = 256, 2000
    say(f"[force gradient vs FD] {n}^2, {nsteps} steps")
    cfg = dict(lattice=9, dtype="f64", n=(n, n, 1), L=(float(n), float(n), 1.0), rho0=1.0, RT=1 / 3, tau=1.0,
               dt=0.5, bc=(0,) * 6)
    Q, D, shp = M.shape_of(cfg)
    Gtar = dev(gaussian_bumps(7, n))
    zero_u = torch.zeros((D,) + shp, dtype=torch.float64, device="cuda")
    with torch.no_grad():
        u_tar = rollout(cfg, Gtar, zero_u, nsteps)

    def loss_of(G):
        return ((rollout(cfg, G, zero_u, nsteps) - u_tar) ** 2).mean()

    G = torch.zeros((D,) + shp, dtype=torch.float64, device="cuda", requires_grad=True)
    L = loss_of(G)
    L.backward()
    grad = G.grad.cpu().numpy()
    rng = np.random.default_rng(11)
    idx = [(int(rng.integers(0, D)), 0, int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(16)]
    eps = 1e-5
    for ix in idx:
        with torch.no_grad():
            Gp = torch.zeros_like(G)
            Gp[ix] = eps
            fd = (loss_of(Gp) - loss_of(-Gp)).item() / (2 * eps)
        assert grad[ix] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(grad).max())


F32_CASES = [("q9-periodic", 9, (37, 29), (0,) * 6, 0, LID, (0,) * 6), WALL_CASES[0], WALL_CASES[3], WALL_CASES[7]]


@pytest.mark.parametrize("name,lat,n,bc,mesh,uw,pw", F32_CASES, ids=[c[0] for c in F32_CASES])
def test_step_adjoint_f32_against_oracle(name, lat, n, bc, mesh, uw, pw):
    # FP32 reverse pass against the FP64 oracle: the adjoint of one step is
    # a sum of O(10) terms of O(1) per entry, so FP32 rounding stays near
    # 1e-6 of the largest entry; 2e-5 is the FP32 gate of the forward path
    say(f"[adjoint f32] {name}")
    cfg = periodic_cfg(lat, n, mesh, bc=bc, uw=uw, pw=list(pw))
    Q, D, shp = M.shape_of(cfg)
    Gf = field(51, (D,) + shp, 2e-3)
    f = perturb(52, O.init(cfg, rho=1 + field(53, shp, 0.02), u=field(54, (D,) + shp, 0.05), force=Gf), 1e-2)
    lam = field(55, f.shape, 1.0)
    gref = np.zeros_like(Gf)
    ref = O.step_adjoint(cfg, f, lam, force=Gf, t=0.4, grad_force=gref)
    c32 = dict(cfg, dtype="f32")
    buf = torch.empty((Q,) + shp, dtype=torch.float32, device="cuda")
    ctx = M.dugks_init(c32, buf)
    try:
        out = torch.empty_like(buf)
        gG = torch.zeros((D,) + shp, dtype=torch.float32, device="cuda")
        M.dugks_step_adjoint(ctx, dev(f).float(), dev(lam).float(), out, dev(Gf).float(), 0.4, gG)
        torch.cuda.synchronize()
        assert np.abs(out.double().cpu().numpy() - ref).max() / np.abs(ref).max() < 2e-5
        assert np.abs(gG.double().cpu().numpy() - gref).max() / np.abs(gref).max() < 2e-5
    finally:
        M.dugks_destroy(ctx)
