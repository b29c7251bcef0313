"""Convergence monitor (dugks_velocity_change) through the C ABI.

The monitor's two sums are checked against the velocities the oracle reads
from the same two states (Eq. macro_values), for both models, all three
lattices, a force field with a time factor and FP32.  A whole-flow check
then uses it the way Sec. III does: a force-driven channel started at rest
is advanced in blocks of 1000 steps until the relative velocity change per
block falls below 1e-6, and the converged profile is the Poiseuille
parabola.
"""
import numpy as np
import pytest

import oracle as O
from tests.test_gpu_parity import c2, c3, case_force, say, start_state, to_dev
from tests.test_oracle_flows import RT_C, channel

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1411_6121_amd")

pytestmark = pytest.mark.gpu

CASES = [
    c2("d2q9-periodic-force", (37, 29), (0,) * 6, G=(2e-4, -1e-4, 0), omega=0.05, phase=0.3, force_field=True),
    c2("d2q9-cavity-original", (33, 30), (1, 1, 1, 1, 0, 0), model=1,
       uw=[[0, 0, 0], [0, 0, 0], [0, 0, 0], [0.1, 0, 0], [0, 0, 0], [0, 0, 0]]),
    c3("d3q19-duct-bb-force", (6, 12, 10), (0, 0, 3, 3, 3, 3), G=(1e-4, 0, 0), force_field=True),
    c3("d3q27-cavity", (12, 10, 9), (1,) * 6, lattice=27,
       uw=[[0, 0, 0], [0, 0, 0], [0, 0, 0], [0.1, 0, 0], [0, 0, 0], [0, 0, 0]]),
]


def reference(cfg, fa, fb, force, ta, tb):
    _, ua, _, _ = O.moments(cfg, fa, force=force, t=ta)
    _, ub, _, _ = O.moments(cfg, fb, force=force, t=tb)
    return np.sqrt(((ub - ua) ** 2).sum()), np.sqrt((ub ** 2).sum())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("cfg", CASES, ids=[c["name"] for c in CASES])
def test_monitor_matches_oracle_velocities(cfg, dtype):
    say(f"[monitor] {cfg['name']} {dtype}")
    force = case_force(cfg, 5)
    fa = start_state(cfg, 21, force)
    ta, nsteps = 0.4, 7
    fb = O.run(cfg, fa, nsteps, force, ta)
    tb = ta + nsteps * cfg["dt"]
    d_ref, b_ref = reference(cfg, fa, fb, force, ta, tb)
    c = dict(cfg, dtype=dtype)
    da, db = to_dev(fa, c), to_dev(fb, c)
    ctx = M.dugks_init(c, torch.empty_like(da))
    try:
        d_got, b_got = M.dugks_velocity_change(ctx, da, db, to_dev(force, c), ta, tb)
    finally:
        M.dugks_destroy(ctx)
    if dtype == "f64":
        assert abs(d_got - d_ref) <= 1e-12 * b_ref
        assert abs(b_got - b_ref) <= 1e-12 * b_ref
    else:
        # FP32 velocity gate (2e-5 of the velocity scale 0.1) per cell,
        # summed in quadrature over the cells
        tol = 2e-5 * 0.1 * np.sqrt(np.prod(cfg["n"]))
        assert abs(d_got - d_ref) <= tol
        assert abs(b_got - b_ref) <= tol


def test_monitor_identical_states_and_errors():
    cfg = CASES[0]
    force = case_force(cfg, 5)
    f = to_dev(start_state(cfg, 22, force), cfg)
    fr = to_dev(force, cfg)
    ctx = M.dugks_init(cfg, torch.empty_like(f))
    try:
        d, b = M.dugks_velocity_change(ctx, f, f, fr, 0.3, 0.3)
        assert d == 0.0 and b > 0.0
        bad = f.clone()
        bad[0, 0, 3, 4] = float("nan")
        with pytest.raises(M.DugksError) as ei:
            M.dugks_velocity_change(ctx, f, bad, fr, 0.3, 0.3)
        assert ei.value.code == M.ENONFINITE
    finally:
        M.dugks_destroy(ctx)


def test_channel_converges_to_poiseuille_under_the_steady_criterion():
    d, y = channel(32, O.BOUNCE_BACK, RT_C)
    say(f"[monitor] channel to steady state, dt={d['dt']:.3e}")
    G, nu = d["G"][0], d["tau"] * d["RT"]
    ua = G / (2 * nu) * y * (1 - y)
    fa = torch.empty((9,) + tuple(d["n"][::-1]), dtype=torch.float64, device="cuda")
    fb = torch.empty_like(fa)
    ctx = M.dugks_init(d, fa)  # at rest
    try:
        cur, nxt = fa, fb
        blocks, ratio = 0, 1.0
        while ratio > 1e-6 and blocks < 400:
            prev = cur.clone()
            which = M.dugks_run(ctx, cur, nxt, 1000)
            if which:
                cur, nxt = nxt, cur
            dn, bn = M.dugks_velocity_change(ctx, prev, cur)
            ratio = dn / bn
            blocks += 1
        assert ratio <= 1e-6, f"not steady after {blocks} blocks (ratio {ratio:.2e})"
        u = torch.empty((2,) + tuple(d["n"][::-1]), dtype=torch.float64, device="cuda")
        M.dugks_moments(ctx, cur, u=u)
        ux = u[0, 0, :, 0].cpu().numpy()
    finally:
        M.dugks_destroy(ctx)
    say(f"[monitor] steady after {blocks} blocks")
    err = np.sqrt(((ux - ua) ** 2).sum() / (ua ** 2).sum())
    assert err < 2e-3


def test_totals_async_equals_moments_totals():
    cfg = CASES[0]
    force = case_force(cfg, 5)
    f = to_dev(start_state(cfg, 23, force), cfg)
    fr = to_dev(force, cfg)
    hist = torch.full((3, 6), -1.0, dtype=torch.float64, device="cuda")
    ctx = M.dugks_init(cfg, torch.empty_like(f))
    try:
        M.dugks_totals_async(ctx, f, hist[1], fr, 0.25)
        torch.cuda.synchronize()
        ref = M.dugks_moments(ctx, f, fr, 0.25)
        bad = f.clone()
        bad[2, 0, 1, 1] = float("inf")
        M.dugks_totals_async(ctx, bad, hist[2], fr, 0.25)
        torch.cuda.synchronize()
    finally:
        M.dugks_destroy(ctx)
    h = hist.cpu().numpy()
    assert (h[0] == -1.0).all()                 # untouched neighbour row
    assert np.array_equal(h[1], np.asarray(ref))  # same reduction, bitwise
    assert h[2, 5] == 1.0                       # non-finite count, no error
