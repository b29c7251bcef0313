"""HIP path vs the CPU oracle, through the C ABI, on the same seeded inputs.

Tolerances (accuracy gates): FP64 state 1e-12 relative L-inf per
step and 1e-10 after 10^4 steps; FP32 velocity within 2e-5 of the velocity
scale.  Sizes span several kernel tiles with ragged tails; walls of every
kind, both meshes, both lattices, forcing with a time factor.
"""
import numpy as np
import pytest

import oracle as O
from synthetic import field, perturb

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1411_6121_amd")

pytestmark = pytest.mark.gpu

LID = [[0, 0, 0], [0, 0, 0], [0, 0, 0], [0.1, 0, 0], [0, 0, 0], [0, 0, 0]]
LID3 = [[0, 0, 0], [0, 0, 0], [0, 0, 0], [0.1, 0, 0], [0, 0, 0], [0, 0, 0]]


def say(msg):
    print(msg, flush=True)


def tdt(cfg):
    return torch.float64 if cfg.get("dtype", "f64") == "f64" else torch.float32


def to_dev(a, cfg):
    if a is None:
        return None
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=tdt(cfg))


VARIANTS = {"general": 0, "fused-twice": 1, "fused": 2, "split": 3}


def default_kernel(cfg):
    """the library's default step kernel for a launch without a force field
    (documented in dugks.h); the original-model variant takes the two-lane
    kernel where the incompressible model would, else the general kernels"""
    if cfg["lattice"] == 27:
        return 3
    if cfg["lattice"] == 9 or cfg.get("dtype", "f64") == "f64":
        return 3
    uniform = all(m == 0 for m in cfg.get("mesh", (0, 0, 0)))
    if cfg.get("model", 0) == 1:
        return 3 if uniform else 0
    return 3 if uniform else 2


def make_ctx(cfg, fb, variant=None, **kw):
    """context on the requested step kernel (None: the library default);
    'split' = faces once, velocity set split over two lanes per column;
    'fused' = faces once, one lane per column; 'fused-twice' evaluates every
    face from both cells; 'general' = two-kernel path"""
    import os
    keys = ("DUGKS_FORCE_GENERAL", "DUGKS_FUSED_VARIANT")
    old = {k: os.environ.get(k) for k in keys}
    os.environ["DUGKS_FORCE_GENERAL"] = "1" if variant == "general" else "0"
    os.environ["DUGKS_FUSED_VARIANT"] = {"fused-twice": "1", "fused": "2", "split": "3"}.get(variant, "0")
    try:
        ctx = M.dugks_init(cfg, fb, **kw)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v
    if variant is None:
        assert M.dugks_kernel_variant(ctx) == default_kernel(cfg)
    else:
        assert M.dugks_kernel_variant(ctx) == VARIANTS[variant]
    return ctx


def gpu_run(cfg, f0, nsteps, force=None, t0=0.0, variant=None):
    fa = to_dev(f0, cfg)
    fb = torch.empty_like(fa)
    ctx = make_ctx(cfg, fb, variant)
    try:
        which = M.dugks_run(ctx, fa, fb, nsteps, to_dev(force, cfg), t0)
        torch.cuda.synchronize()
        return (fb if which else fa).double().cpu().numpy()
    finally:
        M.dugks_destroy(ctx)


def rel_linf(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def start_state(cfg, seed, force=None, du=0.03):
    Q, D, shp = M.shape_of(cfg)
    f0 = O.init(cfg, rho=1.0 + field(seed, shp, 0.01), u=field(seed + 1, (D,) + shp, du), force=force)
    return perturb(seed + 2, f0, 1e-3)


def custom_faces(seed, n, L):
    """seeded strictly increasing face coordinates from 0 to L (cell widths
    between 0.5 and 1.5 of the mean, neighbours differing up to 3x)"""
    from synthetic import rng
    w = rng(seed, 7, n).uniform(0.5, 1.5, n)
    X = np.concatenate([[0.0], np.cumsum(w)]) * (L / w.sum())
    X[0], X[-1] = 0.0, L
    return X


def c2(name, n, bc, **kw):
    d = dict(name=name, lattice=9, dtype="f64", n=(n[0], n[1], 1), L=(float(n[0]), float(n[1]), 1.0), rho0=1.0,
             RT=1 / 3, tau=0.3, dt=0.5, bc=bc)
    d.update(kw)
    return d


def c3(name, n, bc, **kw):
    d = dict(name=name, lattice=19, dtype="f64", n=n, L=tuple(float(v) for v in n), rho0=1.0, RT=1 / 3, tau=0.3,
             dt=0.5, bc=bc)
    d.update(kw)
    return d


CASES = [
    c2("d2q9-periodic-force", (37, 29), (0,) * 6, G=(2e-4, -1e-4, 0), omega=0.05, phase=0.3, force_field=True),
    c2("d2q9-channel-bb", (4, 32), (0, 0, 3, 3, 0, 0), G=(2.6e-3, 0, 0), L=(0.125, 1.0, 1.0), dt=1 / 64, tau=0.1),
    c2("d2q9-channel-neq", (4, 32), (0, 0, 1, 1, 0, 0), G=(2.6e-3, 0, 0), L=(0.125, 1.0, 1.0), dt=1 / 64, tau=0.1),
    c2("d2q9-cavity-neq", (41, 35), (1, 1, 1, 1, 0, 0), uw=LID),
    c2("d2q9-cavity-neq-tanh", (33, 40), (1, 1, 1, 1, 0, 0), uw=LID, mesh=(1, 1, 0), k_stretch=2.5, dt=0.2),
    c2("d2q9-cavity-bb-tanh", (30, 27), (3, 3, 3, 3, 0, 0), uw=LID, mesh=(1, 1, 0), k_stretch=1.5, dt=0.25),
    c2("d2q9-pressure-bb", (48, 17), (2, 2, 3, 3, 0, 0), pw=[3e-3, 0, 0, 0, 0, 0]),
    c2("d2q9-mixed-force-walls", (23, 18), (1, 3, 2, 1, 0, 0), uw=[[0, 0.02, 0], [0, -0.01, 0], [0, 0, 0],
                                                                       [0.05, 0, 0], [0, 0, 0], [0, 0, 0]],
       pw=[0, 0, 1e-3, 0, 0, 0], G=(1e-4, 2e-4, 0), force_field=True, mesh=(0, 1, 0), k_stretch=1.0, dt=0.3),
    c2("d2q9-minimal", (1, 2), (0, 0, 1, 1, 0, 0), uw=LID),
    # inlet/outlet pressures following the time factor (pw + pw_osc g(t)),
    # without acceleration (the source-free instances)
    c2("d2q9-pressure-osc-bb", (48, 17), (2, 2, 3, 3, 0, 0), pw=[1e-3, 0, 0, 0, 0, 0],
       pw_osc=[-3e-3, 1e-3, 0, 0, 0, 0], omega=0.05, phase=0.4),
    c2("d2q9-custom-faces", (29, 23), (1, 3, 1, 2, 0, 0), uw=LID, pw=[0, 0, 0, 1e-3, 0, 0], mesh=(2, 2, 0),
       faces=(custom_faces(1, 29, 29.0), custom_faces(2, 23, 23.0), None), dt=0.25, G=(1e-4, 0, 0),
       force_field=True),
    c2("d2q9-wide-tiles", (300, 21), (1, 1, 0, 0, 0, 0), uw=[[0, 0.01, 0], [0, -0.01, 0]] + [[0, 0, 0]] * 4,
       G=(0, 1e-4, 0)),
    c3("d3q19-multi-tile", (40, 30, 20), (3, 3, 1, 1, 0, 0), uw=LID3, G=(0, 0, 1e-4)),
    c3("d3q19-periodic-force", (13, 11, 9), (0,) * 6, G=(1e-4, 0, -2e-4), omega=0.1, force_field=True),
    c3("d3q19-cavity-neq", (17, 15, 13), (1,) * 6, uw=LID3),
    c3("d3q19-cavity-neq-tanh", (16, 19, 14), (1,) * 6, uw=LID3, mesh=(1, 1, 1), k_stretch=1.5, dt=0.25),
    c3("d3q19-duct-bb-force", (6, 12, 10), (0, 0, 3, 3, 3, 3), G=(1e-4, 0, 0), force_field=True),
    c3("d3q19-mixed", (12, 9, 11), (2, 2, 1, 3, 0, 0), pw=[2e-3, 0, 0, 0, 0, 0], uw=LID3, mesh=(0, 1, 0),
       k_stretch=1.2, dt=0.3),
    c3("d3q19-minimal", (2, 2, 2), (1, 1, 3, 3, 1, 1), uw=LID3),
    c3("d3q19-pressure-osc", (12, 9, 11), (2, 2, 3, 3, 1, 1), pw=[0, 1e-3, 0, 0, 0, 0],
       pw_osc=[2e-3, -1e-3, 0, 0, 0, 0], omega=0.1, uw=LID3, mesh=(0, 1, 0), k_stretch=1.2, dt=0.3),
    c3("d3q19-custom-faces", (14, 11, 12), (1,) * 6, uw=LID3, mesh=(2, 2, 2), dt=0.25,
       faces=(custom_faces(3, 14, 14.0), custom_faces(4, 11, 11.0), custom_faces(5, 12, 12.0))),
    # degenerate periodic axes: a march axis of one plane (the plane ring
    # holds the same plane three times), a tile axis of one column (both
    # halo columns are the cell itself), two cells on two periodic axes
    c3("d3q19-one-plane-periodic-z", (9, 7, 1), (1, 1, 1, 1, 0, 0), uw=LID3),
    # x walls whose ghost columns come from neighbouring lanes of the tile
    # row, without acceleration: moving bounce-back walls over two x tiles,
    # and bounce-back / pressure in one tile
    c3("d3q19-xwalls-bb-moving", (18, 9, 7), (3, 3, 1, 1, 0, 0),
       uw=[[0, 0.02, 0], [0, 0, -0.01], [0, 0, 0], [0.1, 0, 0], [0, 0, 0], [0, 0, 0]]),
    c3("d3q19-xwalls-mixed-kinds", (12, 10, 9), (3, 2, 1, 3, 1, 1), pw=[0, 1.5e-3, 0, 0, 0, 0], uw=LID3),
    c3("d3q19-one-column-periodic-x", (1, 6, 5), (0, 0, 3, 3, 1, 1), uw=LID3, G=(1e-4, 0, 0)),
    c3("d3q19-two-cell-periodic-yz", (5, 2, 2), (1, 1, 0, 0, 0, 0),
       uw=[[0, 0.01, 0], [0, 0, 0.01]] + [[0, 0, 0]] * 4),
]


def case_force(cfg, seed):
    if not cfg.get("force_field"):
        return None
    Q, D, shp = M.shape_of(cfg)
    return field(seed, (D,) + shp, 1e-4)


@pytest.mark.parametrize("variant", ["split", "fused", "fused-twice", "general"])
@pytest.mark.parametrize("cfg", CASES, ids=[c["name"] for c in CASES])
def test_step_parity_f64(cfg, variant):
    say(f"[parity f64] {cfg['name']} n={cfg['n']} {variant}")
    force = case_force(cfg, 5)
    f0 = start_state(cfg, 11, force)
    t0 = 0.7
    ref1 = O.step(cfg, f0, force, t0)
    got1 = gpu_run(cfg, f0, 1, force, t0, variant)
    assert rel_linf(got1, ref1) < 1e-12
    ref = O.run(cfg, f0, 30, force, t0)
    got = gpu_run(cfg, f0, 30, force, t0, variant)
    assert rel_linf(got, ref) < 1e-11


@pytest.mark.parametrize("lat", [9, 19])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_init_and_moments_parity(lat, dtype):
    cfg = (c2("init", (21, 17), (1, 1, 1, 1, 0, 0), uw=LID, G=(1e-3, 2e-3, 0), omega=0.3) if lat == 9 else
           c3("init", (9, 7, 8), (0, 0, 1, 1, 3, 3), uw=LID3, G=(1e-3, 0, 2e-3), omega=0.3))
    cfg["dtype"] = dtype
    say(f"[init/moments] lattice={lat} {dtype}")
    Q, D, shp = M.shape_of(cfg)
    rho = 1.0 + field(1, shp, 0.01)
    u = field(2, (D,) + shp, 0.05)
    force = field(3, (D,) + shp, 1e-3)
    ref = O.init(cfg, rho=rho, u=u, force=force, t0=0.0)
    f = torch.empty((Q,) + shp, dtype=tdt(cfg), device="cuda")
    ctx = M.dugks_init(cfg, f, to_dev(rho, cfg), to_dev(u, cfg), to_dev(force, cfg))
    try:
        tol = 1e-14 if dtype == "f64" else 2e-7
        assert rel_linf(f.double().cpu().numpy(), ref) < tol
        # moments of an oracle state at t = 0.4
        fs = perturb(4, ref, 1e-3)
        r_ref, u_ref, p_ref, tot_ref = O.moments(cfg, fs, force, 0.4)
        rho_d = torch.empty(shp, dtype=tdt(cfg), device="cuda")
        u_d = torch.empty((D,) + shp, dtype=tdt(cfg), device="cuda")
        p_d = torch.empty_like(rho_d)
        tot = M.dugks_moments(ctx, to_dev(fs, cfg), to_dev(force, cfg), 0.4, rho_d, u_d, p_d)
        tol = 1e-13 if dtype == "f64" else 2e-6
        assert rel_linf(rho_d.double().cpu().numpy(), r_ref) < tol
        assert np.abs(u_d.double().cpu().numpy() - u_ref).max() < tol
        assert np.abs(p_d.double().cpu().numpy() - p_ref).max() < tol
        np.testing.assert_allclose(tot[:5], tot_ref[:5], rtol=tol, atol=tol * np.prod(shp))
        assert tot[5] == 0
    finally:
        M.dugks_destroy(ctx)


def test_moments_detect_non_finite():
    cfg = c2("nan", (8, 8), (0,) * 6)
    say("[moments nan]")
    Q, D, shp = M.shape_of(cfg)
    f = torch.empty((Q,) + shp, dtype=torch.float64, device="cuda")
    ctx = M.dugks_init(cfg, f)
    try:
        f[3, 0, 2, 5] = float("nan")
        with pytest.raises(M.DugksError) as ei:
            M.dugks_moments(ctx, f)
        assert ei.value.code == M.ENONFINITE
    finally:
        M.dugks_destroy(ctx)


def test_step_rejects_aliasing():
    cfg = c2("alias", (8, 8), (0,) * 6)
    say("[alias]")
    Q, D, shp = M.shape_of(cfg)
    f = torch.empty((Q,) + shp, dtype=torch.float64, device="cuda")
    ctx = M.dugks_init(cfg, f)
    try:
        with pytest.raises(M.DugksError) as ei:
            M.dugks_step(ctx, f, f)
        assert ei.value.code == M.EINVAL
    finally:
        M.dugks_destroy(ctx)


@pytest.mark.parametrize("lat", [9, 19])
def test_long_run_parity_f64(lat):
    # 10^4 steps: relative L-inf within 1e-10
    cfg = (c2("long", (16, 14), (1, 1, 1, 1, 0, 0), uw=LID, tau=0.2) if lat == 9 else
           c3("long", (8, 7, 6), (1, 1, 1, 1, 0, 0), uw=LID3, tau=0.2))
    say(f"[long run] lattice={lat}")
    f0 = O.init(cfg)
    ref = O.run(cfg, f0, 10000)
    got = gpu_run(cfg, f0, 10000)
    assert rel_linf(got, ref) < 1e-10


@pytest.mark.parametrize("lat", [9, 19])
def test_f32_velocity_parity(lat):
    # FP32 state against the FP64 oracle: velocity within 2e-5 of the lid speed
    cfg = (c2("f32", (24, 20), (1, 1, 1, 1, 0, 0), uw=LID, tau=0.2) if lat == 9 else
           c3("f32", (10, 9, 8), (1, 1, 1, 1, 1, 1), uw=LID3, tau=0.2))
    say(f"[f32] lattice={lat}")
    f0 = O.init(cfg)
    ref = O.run(cfg, f0, 500)
    c32 = dict(cfg, dtype="f32")
    got = gpu_run(c32, f0, 500)
    _, u_ref, _, _ = O.moments(cfg, ref)
    _, u_got, _, _ = O.moments(cfg, got)
    assert np.abs(u_got - u_ref).max() / 0.1 < 2e-5



F32_CASES = [
    c3("f32-d3q19-cavity-tanh", (16, 19, 14), (1,) * 6, uw=LID3, mesh=(1, 1, 1), k_stretch=1.5, dt=0.25, tau=0.2),
    c3("f32-d3q19-duct-bb-force", (6, 12, 10), (0, 0, 3, 3, 3, 3), G=(1e-3, 0, 0), force_field=True, tau=0.2),
    c3("f32-d3q19-one-plane-periodic-z", (9, 7, 1), (1, 1, 1, 1, 0, 0), uw=LID3, tau=0.2),
    c3("f32-d3q19-minimal", (2, 2, 2), (1, 1, 3, 3, 1, 1), uw=LID3, tau=0.2),
    c2("f32-d2q9-periodic-force", (37, 29), (0,) * 6, G=(4e-3, -2e-3, 0), omega=0.05, phase=0.3,
       force_field=True, tau=0.2),
    c2("f32-d2q9-cavity-bb-tanh", (30, 27), (3, 3, 3, 3, 0, 0), uw=LID, mesh=(1, 1, 0), k_stretch=1.5, dt=0.25,
       tau=0.2),
]


@pytest.mark.parametrize("cfg", F32_CASES, ids=[c["name"] for c in F32_CASES])
def test_f32_velocity_parity_cases(cfg):
    # every FP32 kernel instance (stretched and uniform meshes, force fields,
    # degenerate axes) against the FP64 oracle over 500 steps: velocity
    # within 2e-5 of the velocity scale U = 0.1 (the lid speed; the forced
    # flows reach 0.006-0.12)
    say(f"[f32] {cfg['name']} n={cfg['n']}")
    force = case_force(cfg, 5)
    f0 = O.init(cfg, force=force)
    ref = O.run(cfg, f0, 500, force, 0.0)
    got = gpu_run(dict(cfg, dtype="f32"), f0, 500, force)
    _, u_ref, _, _ = O.moments(cfg, ref, force=force, t=500 * cfg["dt"])
    _, u_got, _, _ = O.moments(cfg, got, force=force, t=500 * cfg["dt"])
    assert np.abs(u_ref).max() > 0.005
    assert np.abs(u_got - u_ref).max() / 0.1 < 2e-5