"""Step coefficients across the regimes of the cavity workloads.

Without acceleration the FP32 D3Q19 and the D3Q27 kernels can update a cell
without its own state, using f~(n+1) = phi + B1/(3(1 - B1)) (feq - phi)
(Eq. (f_tilde_+) with f~ recovered from Eq. (f_bar_+)).  That coefficient has
a pole at B1 = 1, i.e. dt = 4 tau, so the library uses the form only where
|1 - B1| >= 1/4 and otherwise the update with the own state.  These cases
put dt/tau on both sides of the pole and at it (3.9, 4, 4.1), at 2.5
(B1 < 1) and at the dt/tau of the Re 400 and Re 1000 cavities (about 5 and
13, B1 > 1), against the FP64 oracle: FP64 state within 1e-12 after one step
and 1e-11 after 30, FP32 velocity within 2e-5 of the lid speed after 600
steps.
"""
import numpy as np
import pytest

import oracle as O
from tests.test_gpu_parity import LID3, c3, gpu_run, rel_linf, start_state

torch = pytest.importorskip("torch")
M = pytest.importorskip("paper_1411_6121_amd")

pytestmark = pytest.mark.gpu

RATIOS = [2.5, 3.9, 4.0, 4.1, 5.2, 13.0]


def say(msg):
    print(msg, flush=True)


def cavity(lat, n, ratio, mesh=(0, 0, 0)):
    d = c3(f"q{lat}-dt/tau={ratio}", n, (1,) * 6, uw=LID3, mesh=mesh, k_stretch=1.5, dt=0.5)
    d["lattice"] = lat
    d["tau"] = d["dt"] / ratio
    return d


@pytest.mark.parametrize("ratio", RATIOS)
def test_d3q27_f64_across_the_pole(ratio):
    cfg = cavity(27, (13, 11, 10), ratio)
    say(f"[coefficients] {cfg['name']} f64")
    f0 = start_state(cfg, 21)
    assert rel_linf(gpu_run(cfg, f0, 1), O.step(cfg, f0)) < 1e-12
    assert rel_linf(gpu_run(cfg, f0, 30), O.run(cfg, f0, 30)) < 1e-11


@pytest.mark.parametrize("lat,mesh", [(19, (0, 0, 0)), (27, (0, 0, 0)), (19, (1, 1, 1))])
@pytest.mark.parametrize("ratio", RATIOS)
def test_f32_velocity_across_the_pole(lat, mesh, ratio):
    cfg = cavity(lat, (12, 10, 9), ratio, mesh)
    say(f"[coefficients] {cfg['name']} mesh={mesh} f32")
    f0 = O.init(cfg)
    ref = O.run(cfg, f0, 600)
    got = gpu_run(dict(cfg, dtype="f32"), f0, 600)
    _, u_ref, _, _ = O.moments(cfg, ref)
    _, u_got, _, _ = O.moments(cfg, got)
    assert np.abs(u_ref).max() > 0.02
    assert np.abs(u_got - u_ref).max() / 0.1 < 2e-5
