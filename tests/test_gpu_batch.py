"""Batched instances: one launch per step for many uneven problems must give,
per instance, exactly the single-instance result; graph replays must equal
eager runs; small instances are checked against the oracle."""
import numpy as np
import pytest

import oracle as O
from tests.test_gpu_parity import custom_faces
from synthetic import batch_instances, field

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1411_6121_amd")

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def instance_cfg(spec, dtype, scale=1):
    """cfg of one batch instance from a synthetic spec (cavity or periodic-x
    channel, lid U = 0.1 or body force along +x); sizes divided by `scale`"""
    nx, ny = max(spec["nx"] // scale, 4), max(spec["ny"] // scale, 4)
    U, RT = spec["U"], 1.0 / 3.0
    nu = U * ny / spec["Re"]
    if spec["kind"] == "cavity":
        bc = (1, 1, 1, 1, 0, 0)
        uw = [[0, 0, 0], [0, 0, 0], [0, 0, 0], [U, 0, 0], [0, 0, 0], [0, 0, 0]]
    else:
        bc = (0, 0, 1, 1, 0, 0)
        uw = [[0, 0, 0]] * 6
    return dict(lattice=9, dtype=dtype, n=(nx, ny, 1), L=(float(nx), float(ny), 1.0), rho0=1.0, RT=RT,
                tau=nu / RT, dt=0.5, bc=bc, uw=uw, G=(spec["force"], 0.0, 0.0))


def make_set(dtype, count=10, scale=4):
    specs = batch_instances(seed=3, count=count)
    cfgs = [instance_cfg(s, dtype, scale) for s in specs]
    # vary the time factor and give some instances a force field
    for i, c in enumerate(cfgs):
        c["omega"] = 0.01 * i
        c["phase"] = 0.1 * i
    forces = []
    for i, c in enumerate(cfgs):
        Q, D, shp = M.shape_of(c)
        forces.append(None if i % 3 else torch.from_numpy(field(50 + i, (D,) + shp, 1e-5)).to(
            "cuda", dtype=M.torch_dtype(c)))
    return cfgs, forces


def single_run(cfg, f0, nsteps, force):
    fa = f0.clone()
    fb = torch.empty_like(fa)
    ctx = M.dugks_init(cfg, fb)
    try:
        which = M.dugks_run(ctx, fa, fb, nsteps, force, 0.0)
        return (fb if which else fa).clone()
    finally:
        M.dugks_destroy(ctx)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_equals_single_instance_runs(dtype):
    cfgs, forces = make_set(dtype)
    say(f"[batch == single] {dtype} sizes={[c['n'][:2] for c in cfgs]}")
    B = M.BatchSolver(cfgs, forces=forces)
    try:
        f0 = [B.state(i).clone() for i in range(len(cfgs))]
        B.run(7)
        B.run(6)  # the batch clock carries the time across runs
        torch.cuda.synchronize()
        for i, c in enumerate(cfgs):
            ref = single_run(c, f0[i], 13, forces[i])
            assert torch.equal(B.state(i), ref), f"instance {i} differs"
    finally:
        B.close()


def test_graph_replays_equal_eager_runs():
    cfgs, forces = make_set("f64", count=6)
    say("[batch graph replay]")
    Bg = M.BatchSolver(cfgs, forces=forces)
    Be = M.BatchSolver(cfgs, forces=forces)
    try:
        for rep in range(3):
            Bg.run(4, use_graph=True)
            Be.run(4, use_graph=False)
            torch.cuda.synchronize()
            extra = Be.f.sum()  # eager work between replays
            torch.cuda.synchronize()
            assert torch.isfinite(extra)
            for i in range(len(cfgs)):
                assert torch.equal(Bg.state(i), Be.state(i)), f"replay {rep} instance {i}"
    finally:
        Bg.close()
        Be.close()


def test_batch_matches_oracle():
    cfgs, forces = make_set("f64", count=4, scale=8)
    say("[batch vs oracle]")
    B = M.BatchSolver(cfgs, forces=forces)
    try:
        f0 = [B.state(i).cpu().numpy() for i in range(len(cfgs))]
        B.run(10)
        torch.cuda.synchronize()
        for i, c in enumerate(cfgs):
            oc = {k: v for k, v in c.items() if k != "dtype"}
            fr = None if forces[i] is None else forces[i].cpu().numpy()
            ref = O.run(oc, f0[i], 10, force=fr)
            got = B.state(i).cpu().numpy()
            assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-12, i
            # the initial state is the oracle's equilibrium at rest under the
            # uniform acceleration (force fields enter from the first step)
            assert np.abs(f0[i] - O.init(oc)).max() < 1e-14
    finally:
        B.close()


def d3q19_set(with_forces, dtype="f64"):
    """uneven D3Q19 instances, degenerate ones included: a cavity, the
    2x2x2 minimum, a one-column periodic axis, a one-plane periodic march
    axis, a stretched duct, a fully periodic box"""
    lid = [[0, 0, 0], [0, 0, 0], [0, 0, 0], [0.05, 0, 0], [0, 0, 0], [0, 0, 0]]

    def c(n, bc, **kw):
        d = dict(lattice=19, dtype=dtype, n=n, L=tuple(float(v) for v in n), rho0=1.0, RT=1 / 3, tau=0.3,
                 dt=0.5, bc=bc, uw=lid)
        d.update(kw)
        return d

    cfgs = [c((20, 17, 9), (1,) * 6, tau=0.25),
            c((2, 2, 2), (1, 1, 3, 3, 1, 1)),
            c((1, 6, 5), (0, 0, 3, 3, 1, 1), G=(1e-4, 0, 0)),
            c((9, 7, 1), (1, 1, 1, 1, 0, 0), omega=0.2, G=(0, 1e-4, 0)),
            c((8, 12, 10), (0, 0, 3, 3, 3, 3), mesh=(0, 1, 1), k_stretch=1.3, dt=0.3, G=(2e-4, 0, 0)),
            c((13, 11, 9), (0,) * 6, G=(1e-4, 0, -2e-4), omega=0.1, phase=0.4),
            c((7, 6, 8), (1,) * 6, mesh=(2, 2, 2), dt=0.25,
              faces=(custom_faces(8, 7, 7.0), custom_faces(9, 6, 6.0), custom_faces(10, 8, 8.0)))]
    forces = [None] * len(cfgs)
    if with_forces:
        for i in (0, 3, 5):
            Q, D, shp = M.shape_of(cfgs[i])
            forces[i] = torch.from_numpy(field(70 + i, (D,) + shp, 1e-4)).to("cuda", dtype=M.torch_dtype(cfgs[i]))
    return cfgs, forces


@pytest.mark.parametrize("with_forces", [False, True], ids=["no-field", "force-fields"])
def test_batch_d3q19_matches_oracle(with_forces):
    cfgs, forces = d3q19_set(with_forces)
    say(f"[batch d3q19 vs oracle] fields={with_forces} sizes={[c['n'] for c in cfgs]}")
    B = M.BatchSolver(cfgs, forces=forces)
    try:
        f0 = [B.state(i).cpu().numpy() for i in range(len(cfgs))]
        B.run(6)
        B.run(5)
        torch.cuda.synchronize()
        for i, c in enumerate(cfgs):
            oc = {k: v for k, v in c.items() if k != "dtype"}
            fr = None if forces[i] is None else forces[i].cpu().numpy()
            ref = O.run(oc, f0[i], 11, force=fr)
            got = B.state(i).cpu().numpy()
            assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-12, c["n"]
    finally:
        B.close()


@pytest.mark.parametrize("with_forces", [False, True], ids=["no-field", "force-fields"])
def test_batch_d3q19_f32_velocity(with_forces):
    # FP32 batch against the FP64 oracle from the same (rounded) initial
    # states: velocities within 2e-5 of the lid speed after 100 steps
    cfgs, forces = d3q19_set(with_forces, "f32")
    say(f"[batch d3q19 f32 vs oracle] fields={with_forces}")
    B = M.BatchSolver(cfgs, forces=forces)
    try:
        f0 = [B.state(i).double().cpu().numpy() for i in range(len(cfgs))]
        B.run(100)
        torch.cuda.synchronize()
        for i, c in enumerate(cfgs):
            oc = {k: v for k, v in c.items() if k != "dtype"}
            fr = None if forces[i] is None else forces[i].double().cpu().numpy()
            ref = O.run(oc, f0[i], 100, force=fr)
            t = 100 * c["dt"]
            _, u_ref, _, _ = O.moments(oc, ref, force=fr, t=t)
            _, u_got, _, _ = O.moments(oc, B.state(i).double().cpu().numpy(), force=fr, t=t)
            assert np.abs(u_got - u_ref).max() / 0.05 < 2e-5, c["n"]
    finally:
        B.close()


@pytest.mark.parametrize("with_forces", [False, True], ids=["no-field", "force-fields"])
def test_batch_d3q19_graph_replays_equal_eager_runs(with_forces):
    # graph replays of the D3Q19 batch (the time factor comes from the
    # device step counter) against eager launches, with eager work between
    cfgs, forces = d3q19_set(with_forces)
    say(f"[batch d3q19 graph replay] fields={with_forces}")
    Bg = M.BatchSolver(cfgs, forces=forces)
    Be = M.BatchSolver(cfgs, forces=forces)
    try:
        for rep in range(3):
            Bg.run(3, use_graph=True)
            Be.run(3, use_graph=False)
            torch.cuda.synchronize()
            assert torch.isfinite(Be.f.sum())
            torch.cuda.synchronize()
            for i in range(len(cfgs)):
                assert torch.equal(Bg.state(i), Be.state(i)), f"replay {rep} instance {i}"
    finally:
        Bg.close()
        Be.close()


def test_batch_rejects_mixed_lattices():
    say("[batch invalid]")
    a = instance_cfg(batch_instances(1, 1)[0], "f64", 8)
    b = dict(a, lattice=19, n=(4, 4, 4), L=(4.0, 4.0, 4.0), bc=(1,) * 6)
    with pytest.raises(M.DugksError) as ei:
        M.BatchSolver([a, b])
    assert ei.value.code == M.EINVAL


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_tuned_batch_equals_untuned(dtype):
    # the autotuner only changes the tiling and march chunk: the states stay
    # bitwise equal, and the batch clock (time-dependent forcing) is kept
    cfgs, forces = make_set(dtype, count=8)
    say(f"[batch tune] {dtype}")
    Bt = M.BatchSolver(cfgs, forces=forces)
    Bu = M.BatchSolver(cfgs, forces=forces)
    try:
        Bt.run(3)
        Bu.run(3)
        tile, chunk = Bt.tune(nsteps=2)
        say(f"  chose tile variant {tile}, chunk {chunk}")
        assert tile in (0, 1, 2) and chunk in (0, 4, 8, 16, 32, 64)  # 0: a chunk per instance
        Bt.run(4, use_graph=True)
        Bu.run(4, use_graph=True)
        torch.cuda.synchronize()
        for i in range(len(cfgs)):
            assert torch.equal(Bt.state(i), Bu.state(i)), f"instance {i}"
    finally:
        Bt.close()
        Bu.close()
