"""D3Q27 (the paper's 3-D velocity set) on the GPU against the oracle:
walls of every kind, both meshes, forcing; initial state and moments; FP32
velocity; the paths without D3Q27 refuse it."""
import numpy as np
import pytest

import oracle as O
from synthetic import field, perturb
from tests.test_gpu_parity import LID3, c3, gpu_run, rel_linf, tdt, to_dev

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1411_6121_amd")

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


# tangential velocities of the x walls (and the lid)
XBB = [[0, 0.02, 0], [0, 0, -0.01], [0, 0, 0], [0.1, 0, 0], [0, 0, 0], [0, 0, 0]]


def q27(name, n, bc, **kw):
    d = c3(name, n, bc, **kw)
    d["lattice"] = 27
    return d


CASES = [
    q27("d3q27-periodic-force", (13, 11, 9), (0,) * 6, G=(1e-4, 0, -2e-4), omega=0.1, force_field=True),
    q27("d3q27-cavity-neq", (17, 15, 13), (1,) * 6, uw=LID3),
    q27("d3q27-cavity-neq-tanh", (16, 19, 14), (1,) * 6, uw=LID3, mesh=(1, 1, 1), k_stretch=1.5, dt=0.25),
    q27("d3q27-duct-bb-force", (6, 12, 10), (0, 0, 3, 3, 3, 3), G=(1e-4, 0, 0), force_field=True),
    q27("d3q27-mixed", (12, 9, 11), (2, 2, 1, 3, 0, 0), pw=[2e-3, 0, 0, 0, 0, 0], uw=LID3, mesh=(0, 1, 0),
        k_stretch=1.2, dt=0.3),
    q27("d3q27-original-model", (10, 9, 8), (1,) * 6, uw=LID3, model=1),
    q27("d3q27-minimal", (2, 2, 2), (1, 1, 3, 3, 1, 1), uw=LID3),
    q27("d3q27-one-plane-periodic-z", (7, 6, 1), (1, 1, 1, 1, 0, 0), uw=LID3),
    q27("d3q27-one-column-periodic-x", (1, 5, 4), (0, 0, 3, 3, 1, 1), uw=LID3, G=(1e-4, 0, 0)),
    # x walls of every kind (the x ghost columns and the x wall faces' NEQ
    # values come from neighbouring lanes of the tile row): moving
    # bounce-back walls on two x tiles, bounce-back / pressure in one tile,
    # with acceleration, and a high ghost in the tile's last column (n = 14)
    q27("d3q27-xwalls-bb-moving", (18, 9, 7), (3, 3, 1, 1, 0, 0), uw=XBB),
    q27("d3q27-xwalls-mixed-kinds", (12, 10, 9), (3, 2, 1, 3, 1, 1), pw=[0, 1.5e-3, 0, 0, 0, 0], uw=LID3),
    q27("d3q27-xwalls-accel", (16, 8, 6), (1, 1, 3, 3, 0, 0), uw=XBB, G=(0, 1e-4, 2e-4)),
    q27("d3q27-xwalls-full-tile", (14, 7, 5), (1, 1, 1, 1, 3, 3), uw=LID3),
]


@pytest.mark.parametrize("cfg", CASES, ids=[c["name"] for c in CASES])
def test_d3q27_step_parity(cfg):
    say(f"[d3q27] {cfg['name']} n={cfg['n']}")
    Q, D, shp = M.shape_of(cfg)
    assert Q == 27
    force = field(5, (D,) + shp, 1e-4) if cfg.get("force_field") else None
    f0 = perturb(13, O.init(cfg, rho=1.0 + field(11, shp, 0.01), u=field(12, (D,) + shp, 0.03), force=force), 1e-3)
    t0 = 0.7
    assert rel_linf(gpu_run(cfg, f0, 1, force, t0), O.step(cfg, f0, force, t0)) < 1e-12
    assert rel_linf(gpu_run(cfg, f0, 30, force, t0), O.run(cfg, f0, 30, force, t0)) < 1e-11


def test_d3q27_init_moments_and_refusals():
    cfg = q27("q27init", (9, 7, 8), (0, 0, 1, 1, 3, 3), uw=LID3, G=(1e-3, 0, 2e-3), omega=0.3)
    say("[d3q27 init/moments]")
    Q, D, shp = M.shape_of(cfg)
    rho = 1.0 + field(1, shp, 0.01)
    u = field(2, (D,) + shp, 0.05)
    force = field(3, (D,) + shp, 1e-3)
    ref = O.init(cfg, rho=rho, u=u, force=force, t0=0.0)
    f = torch.empty((Q,) + shp, dtype=tdt(cfg), device="cuda")
    ctx = M.dugks_init(cfg, f, to_dev(rho, cfg), to_dev(u, cfg), to_dev(force, cfg))
    try:
        assert rel_linf(f.cpu().numpy(), ref) < 1e-14
        fs = perturb(4, ref, 1e-3)
        _, u_ref, _, tot_ref = O.moments(cfg, fs, force, 0.4)
        u_d = torch.empty((D,) + shp, dtype=tdt(cfg), device="cuda")
        tot = M.dugks_moments(ctx, to_dev(fs, cfg), to_dev(force, cfg), 0.4, u=u_d)
        assert np.abs(u_d.cpu().numpy() - u_ref).max() < 1e-13
        np.testing.assert_allclose(tot[:5], tot_ref[:5], rtol=1e-13, atol=1e-13 * np.prod(shp))
        with pytest.raises(M.DugksError) as ei:
            M.dugks_step_adjoint(ctx, f, torch.zeros_like(f), torch.empty_like(f))
        assert ei.value.code == M.EUNSUPPORTED
    finally:
        M.dugks_destroy(ctx)
    with pytest.raises(M.DugksError) as ei:
        M.BatchSolver([cfg])
    assert ei.value.code == M.EUNSUPPORTED


def test_d3q27_f32_velocity():
    cfg = q27("q27f32", (10, 9, 8), (1, 1, 1, 1, 1, 1), uw=LID3, tau=0.2)
    say("[d3q27 f32]")
    f0 = O.init(cfg)
    ref = O.run(cfg, f0, 300)
    got = gpu_run(dict(cfg, dtype="f32"), f0, 300)
    _, u_ref, _, _ = O.moments(cfg, ref)
    _, u_got, _, _ = O.moments(cfg, got)
    assert np.abs(u_got - u_ref).max() / 0.1 < 2e-5


F32_XWALLS = [
    q27("q27f32-xwalls-bb-moving", (18, 9, 7), (3, 3, 1, 1, 0, 0), uw=XBB, tau=0.2),
    q27("q27f32-xwalls-mixed-kinds", (12, 10, 9), (3, 2, 1, 3, 1, 1), pw=[0, 1.5e-3, 0, 0, 0, 0], uw=LID3, tau=0.2),
]


@pytest.mark.parametrize("cfg", F32_XWALLS, ids=[c["name"] for c in F32_XWALLS])
def test_d3q27_f32_velocity_x_walls(cfg):
    # the FP32 instance (16 x 8 tiles, two workgroups per CU) with x walls of
    # each kind against the FP64 oracle over 300 steps: velocity within 2e-5
    # of the lid speed U = 0.1
    say(f"[d3q27 f32] {cfg['name']} n={cfg['n']}")
    f0 = O.init(cfg)
    ref = O.run(cfg, f0, 300)
    got = gpu_run(dict(cfg, dtype="f32"), f0, 300)
    _, u_ref, _, _ = O.moments(cfg, ref)
    _, u_got, _, _ = O.moments(cfg, got)
    assert np.abs(u_ref).max() > 0.005
    assert np.abs(u_got - u_ref).max() / 0.1 < 2e-5
