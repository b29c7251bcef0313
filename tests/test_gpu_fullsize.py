"""Parity at the full workload sizes, in the launch configuration the
benchmark times: the D3Q19 128^3 cavity (uniform and tanh meshes, FP64 and
FP32), the D2Q9 1024^2 cavity, the 2-D Re = 12000 cavity (128^2 tanh
mesh, bounce-back walls), the 4 x 32 channel over 20000 steps, the 32 x 256
Womersley channel, the 64-instance uneven batch, a 640^3 periodic mesh
(5e9 state elements, past 32-bit offsets) checked block by block, the
spanwise mirror symmetry of the GPU's own 128^3 cavity runs, and the
pressure-driven Womersley channel of Sec. III.C at its printed parameters.

Whole-field comparisons: one oracle step at these sizes takes well under a
second on the host cores, so every output value is checked, not a sample.
"""
import numpy as np
import pytest

import bench
import oracle as O
from tests.test_gpu_parity import default_kernel
from synthetic import batch_instances, field, perturb

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1411_6121_amd")

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def rel_linf(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def flow_state(cfg, seed):
    """the oracle's equilibrium of a seeded density/velocity field, perturbed
    off equilibrium (a state with every term of the step active)"""
    Q, D, shp = M.shape_of(cfg)
    f0 = O.init(cfg, rho=1.0 + field(seed, shp, 0.01), u=field(seed + 1, (D,) + shp, 0.03))
    return perturb(seed + 2, f0, 1e-3)


def gpu_steps(cfg, f0, nsteps):
    dt = torch.float64 if cfg["dtype"] == "f64" else torch.float32
    fa = torch.from_numpy(f0).to(device="cuda", dtype=dt)
    fb = torch.empty_like(fa)
    ctx = M.dugks_init(cfg, fb)
    try:
        assert M.dugks_kernel_variant(ctx) == default_kernel(cfg)  # the benchmarked step kernel
        which = M.dugks_run(ctx, fa, fb, nsteps, None, 0.0)
        torch.cuda.synchronize()
        return (fb if which else fa).double().cpu().numpy()
    finally:
        M.dugks_destroy(ctx)


@pytest.mark.parametrize("mesh,re", [("uniform", 100.0), ("tanh", 1000.0)])
def test_cavity_128_f64(mesh, re):
    cfg = bench.cavity_cfg(128, "f64", mesh, re)
    say(f"[full size] D3Q19 128^3 cavity {mesh} Re {re:g} f64")
    oc = {k: v for k, v in cfg.items() if k != "dtype"}
    f0 = flow_state(oc, 61)
    ref = O.run(oc, f0, 2)
    got = gpu_steps(cfg, f0, 2)
    assert rel_linf(got, ref) < 1e-12


def test_cavity_128_f32_velocity():
    cfg = bench.cavity_cfg(128, "f32", "uniform", 100.0)
    say("[full size] D3Q19 128^3 cavity f32")
    oc = {k: v for k, v in cfg.items() if k != "dtype"}
    f0 = flow_state(oc, 62)
    ref = O.run(oc, f0, 2)
    got = gpu_steps(cfg, f0, 2)
    _, u_ref, _, _ = O.moments(oc, ref)
    _, u_got, _, _ = O.moments(oc, got)
    assert np.abs(u_got - u_ref).max() / 0.1 < 2e-5


def test_cavity_1024_d2q9_f64():
    cfg = bench.cavity_cfg(1024, "f64", "uniform", 1000.0, lattice=9)
    say("[full size] D2Q9 1024^2 cavity Re 1000 f64")
    oc = {k: v for k, v in cfg.items() if k != "dtype"}
    f0 = flow_state(oc, 63)
    ref = O.run(oc, f0, 2)
    got = gpu_steps(cfg, f0, 2)
    assert rel_linf(got, ref) < 1e-12


@pytest.mark.parametrize("n", [128, 80])
def test_cavity_re12000_f64(n):
    cfg = bench.cavity12000_cfg(n)
    say(f"[full size] D2Q9 {n}^2 Re 12000 cavity, tanh k=2.5, bounce-back, f64")
    oc = {k: v for k, v in cfg.items() if k != "dtype"}
    # a lid-scale velocity field so that every term (and the walls) is active
    Q, D, shp = M.shape_of(cfg)
    f0 = perturb(66, O.init(oc, rho=1.0 + field(64, shp, 1e-3), u=field(65, (D,) + shp, 0.3)), 1e-3)
    ref = O.run(oc, f0, 3)
    got = gpu_steps(cfg, f0, 3)
    assert rel_linf(got, ref) < 1e-12


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_batch_equals_plain_launches(dtype):
    cfgs = [bench.batch_cfg(s, dtype) for s in batch_instances(seed=3, count=64)]
    say(f"[full size] 64-instance batch {dtype}, {sum(c['n'][0] * c['n'][1] for c in cfgs)} cells")
    B = M.BatchSolver(cfgs)
    try:
        f0 = [B.state(i).clone() for i in range(len(cfgs))]
        B.run(3, use_graph=True)
        torch.cuda.synchronize()
        for i, c in enumerate(cfgs):
            fa = f0[i].clone()
            fb = torch.empty_like(fa)
            ctx = M.dugks_init(c, fb)
            try:
                which = M.dugks_run(ctx, fa, fb, 3, None, 0.0)
                ref = fb if which else fa
                assert torch.equal(B.state(i), ref), f"instance {i}"
            finally:
                M.dugks_destroy(ctx)
    finally:
        B.close()


@pytest.mark.parametrize("bc", [3, 1], ids=["bounce-back", "neq"])
def test_channel_workload_20000_steps(bc):
    # the force-driven periodic channel: 4 x 32 cells, periodic in x, walls
    # in y, rho0 = 1, RT = 1/3, tau = 0.1 (nu = tau RT), dt from CFL 0.5,
    # G for u_max = 0.01, from rest, 20000 steps; GPU vs oracle and both
    # against the parabola (at this tau the walls slip by O(tau): a few %)
    from tests.test_oracle_flows import channel

    nu = 0.1 / 3
    d, y = channel(32, bc, 1 / 3, nu=nu, G=8 * nu * 0.01, nx=4)
    d["dtype"] = "f64"
    say(f"[full size] channel 4x32 bc={bc}, 20000 steps")
    oc = {k: v for k, v in d.items() if k != "dtype"}
    f0 = O.init(oc)
    ref = O.run(oc, f0, 20000)
    got = gpu_steps(d, f0, 20000)
    assert rel_linf(got, ref) < 1e-10
    ua = d["G"][0] / (2 * nu) * y * (1 - y)
    _, u, _, _ = O.moments(oc, got)
    err = np.sqrt(((u[0, 0, :, 0] - ua) ** 2).sum() / (ua ** 2).sum())
    assert err < 0.1


def test_womersley_channel_32x256():
    # Womersley channel, 32 x 256 cells (periodic x), bounce-back walls,
    # oscillating force G cos(omega t) at Womersley number 4 (alpha^2 =
    # Ly^2 omega / (4 nu)), continuum regime (RT = 1000/3): parity with the
    # oracle over 200 steps, then one period on the GPU from the analytic
    # state against the closed form at eight phases of the next period
    from tests.test_oracle_flows import RT_C, channel, womersley_u

    nu, alpha, G = 0.01, 4.0, 1e-3
    omega = 4 * alpha ** 2 * nu
    d, y = channel(256, 3, RT_C, nu=nu, G=G, nx=32)
    T = 2 * np.pi / omega
    nper = int(round(T / d["dt"]))
    nper -= nper % 8
    d["dt"] = T / nper
    d["omega"] = omega
    d["dtype"] = "f64"
    say(f"[full size] Womersley 32x256, alpha 4, {nper} steps per period")
    oc = {k: v for k, v in d.items() if k != "dtype"}
    Q, D, shp = M.shape_of(d)
    u0 = np.zeros((2,) + shp)
    u0[0] = womersley_u(y, 0.0, G, omega, nu)[None, :, None]
    f0 = O.init(oc, u=u0)
    ref = O.run(oc, f0, 200)
    assert rel_linf(gpu_steps(d, f0, 200), ref) < 1e-12
    fa = torch.from_numpy(f0).to("cuda")
    fb = torch.empty_like(fa)
    ctx = M.dugks_init(d, fb)
    try:
        t, worst = 0.0, 0.0
        cur, nxt = fa, fb
        u = torch.empty((2,) + shp, dtype=torch.float64, device="cuda")
        for k in range(16):
            if M.dugks_run(ctx, cur, nxt, nper // 8, None, t):
                cur, nxt = nxt, cur
            t += (nper // 8) * d["dt"]
            if k >= 8:
                M.dugks_moments(ctx, cur, t=t, u=u)
                ux = u[0, 0, :, 0].cpu().numpy()
                worst = max(worst, np.abs(ux - womersley_u(y, t, G, omega, nu)).max() / (G / omega))
    finally:
        M.dugks_destroy(ctx)
    say(f"[full size] Womersley worst error {worst:.2e} of G/omega")
    assert worst < 1e-2


@pytest.mark.parametrize("G", [(0.0, 0.0, 0.0), (2e-5, -1e-5, 1e-5)], ids=["no-acceleration", "forced"])
def test_large_periodic_mesh_64bit_offsets(G):
    # 640^3 D3Q19 FP64 (19 x 640^3 = 5.0e9 state elements, beyond 32-bit
    # offsets): a periodic state that repeats a seeded 10^3 block stays
    # periodic, so after two steps every 10^3 block must equal the oracle's
    # two steps of the 10^3 periodic mesh
    n, p = 640, 10
    small = c3_periodic(p, G)
    big = dict(small, n=(n, n, n), L=(float(n),) * 3)
    say(f"[full size] D3Q19 {n}^3 periodic from a tiled {p}^3 block, G={G}")
    f0 = flow_state(small, 67)
    ref = torch.from_numpy(O.run(small, f0, 2)).to("cuda")
    r = n // p
    fa = torch.from_numpy(f0).to("cuda").repeat(1, r, r, r)
    fb = torch.empty_like(fa)
    ctx = M.dugks_init(big, fb)
    try:
        assert M.dugks_kernel_variant(ctx) == default_kernel(big)
        which = M.dugks_run(ctx, fa, fb, 2, None, 0.0)
        got = fb if which else fa
        worst = 0.0
        scale = ref.abs().max().item()
        for z0 in range(0, n, 80):  # compare slab by slab (bounded temporaries)
            sl = got[:, z0:z0 + 80].reshape(19, 80 // p, p, r, p, r, p)
            d = (sl - ref.reshape(19, 1, p, 1, p, 1, p)).abs().max().item()
            worst = max(worst, d)
        torch.cuda.synchronize()
    finally:
        M.dugks_destroy(ctx)
        del fa, fb
        torch.cuda.empty_cache()
    assert worst / scale < 1e-12


def c3_periodic(p, G):
    return dict(lattice=19, dtype="f64", n=(p, p, p), L=(float(p),) * 3, rho0=1.0, RT=1 / 3, tau=0.3, dt=0.5,
                bc=(0,) * 6, G=G)


@pytest.mark.parametrize("lat,mesh,re,nsteps", [(19, "uniform", 100.0, 400), (19, "tanh", 1000.0, 400),
                                                (27, "uniform", 100.0, 100)])
def test_cavity_128_spanwise_mirror_symmetry(lat, mesh, re, nsteps):
    # a property that holds at any size: the cavity from rest keeps the
    # z -> L - z mirror symmetry (velocity (ex, ey, ez) -> (ex, ey, -ez)) to
    # FP64 rounding over the GPU's own run
    cfg = bench.cavity_cfg(128, "f64", mesh, re, lattice=lat)
    oc = {k: v for k, v in cfg.items() if k != "dtype"}
    say(f"[full size] D{3}Q{lat} 128^3 cavity {mesh} Re {re:g} f64: mirror symmetry after {nsteps} steps")
    f = gpu_steps(cfg, O.init(oc), nsteps)
    e, _ = O.lattice(lat)
    idx = {tuple(v): k for k, v in enumerate(e)}
    kmap = [idx[(v[0], v[1], -v[2])] for v in e]
    err = np.abs(f - f[kmap][:, ::-1]).max() / np.abs(f).max()
    uz = O.moments(oc, f)[1][2]
    say(f"    mirror error {err:.2e}, max |u_z| {np.abs(uz).max():.2e}")
    assert np.abs(uz).max() > 1e-6
    assert err < 1e-12


def test_pressure_driven_womersley_40x20():
    # the pressure-driven channel of Sec. III.C at its printed parameters
    # (inlet pressure oscillating in time): one period against the oracle,
    # then the printed bound on the pressure error over the next period
    from tests.test_oracle_flows import pressure_womersley
    d, nper, p_exact, u_exact = pressure_womersley(20)
    cfg = dict(d, dtype="f64")
    Q, D, shp = M.shape_of(cfg)
    say(f"[full size] pressure-driven Womersley 40x20, {nper} steps per period")
    u0 = np.zeros((2,) + shp)
    u0[0] = u_exact(0.0)[None, :, None]
    f0 = O.init(d, rho=1.0 + np.broadcast_to(p_exact(0.0)[None, None, :], shp) / d["RT"], u=u0)
    fa = torch.from_numpy(f0).to("cuda")
    fb = torch.empty_like(fa)
    ctx = M.dugks_init(cfg, fb)
    try:
        which = M.dugks_run(ctx, fa, fb, nper, None, 0.0)
        if which:
            fa, fb = fb, fa
        torch.cuda.synchronize()
        ref = O.run(d, f0, nper)
        err = rel_linf(fa.cpu().numpy(), ref)
        say(f"    after one period: rel L-inf {err:.2e}")
        assert err < 1e-10
        t, sums = nper * d["dt"], np.zeros(2)
        for _ in range(8):
            which = M.dugks_run(ctx, fa, fb, nper // 8, None, t)
            if which:
                fa, fb = fb, fa
            t += (nper // 8) * d["dt"]
            torch.cuda.synchronize()
            _, u, p, _ = O.moments(d, fa.cpu().numpy(), t=t)
            pa = np.broadcast_to(p_exact(t)[None, None, :], shp)
            sums += [((p - pa) ** 2).sum(), (pa ** 2).sum()]
        ep = np.sqrt(sums[0] / sums[1])
        say(f"    E(p) over the period {100 * ep:.3f} %")
        assert ep < 0.0042
    finally:
        M.dugks_destroy(ctx)
