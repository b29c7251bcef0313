"""Mirror symmetry of the 3-D lid-driven cavity in the oracle (Sec. III.E
geometry: lid on the +y side moving along x, z spanwise).

The problem is symmetric under z -> L_z - z, which maps velocity e =
(ex, ey, ez) to (ex, ey, -ez).  Started from rest (or from any mirror-
symmetric state) the scheme keeps the symmetry exactly in exact arithmetic:
every stencil, ghost extrapolation and wall rule of the -z side is the
mirror image of the +z side.  In floating point only the order of the sums
over velocities differs between mirrored cells, so the two halves agree to
a few FP64 rounding units.  A sign or index slip on one z side (a z-gradient
term, a ghost plane, the NEQ point of one wall, a tanh weight of one half)
breaks the symmetry at O(1) of the flow.

Planted one-sided mistakes in the oracle, each failing every symmetry pin
below except the negative control: the +z ghost extrapolation ratio with
its sign flipped, the +z NEQ point taken one cell further in, and the +z
ghost extrapolated through cells N-1 and N-3.
"""
import numpy as np
import pytest

import oracle as O
from synthetic import field

U = 0.05


def cavity(lat, n, stretch):
    uw = [[0.0] * 3 for _ in range(6)]
    uw[3] = [U, 0.0, 0.0]
    d = dict(lattice=lat, n=n, L=tuple(float(v) for v in n), mesh=(stretch,) * 3, k_stretch=1.5, rho0=1.0,
             RT=1 / 3, tau=0.2, dt=0.5, bc=(1, 1, 1, 1, 1, 1), uw=uw)
    X, _ = O.mesh(d, 0)
    d["dt"] = 0.5 * min(np.diff(O.mesh(d, a)[0]).min() for a in range(3)) / np.sqrt(3 * d["RT"])
    return d


def mirror_z(lat, f):
    e, _ = O.lattice(lat)
    idx = {tuple(v): k for k, v in enumerate(e)}
    kmap = [idx[(v[0], v[1], -v[2])] for v in e]
    return f[kmap][:, ::-1, :, :]


def mirrored_pair_error(lat, f):
    return np.abs(f - mirror_z(lat, f)).max() / np.abs(f).max()


@pytest.mark.parametrize("lat", [19, 27])
@pytest.mark.parametrize("stretch", [0, 1], ids=["uniform", "tanh"])
def test_cavity_keeps_spanwise_mirror_symmetry(lat, stretch):
    d = cavity(lat, (6, 5, 7), stretch)
    f = O.run(d, O.init(d), 60)
    _, u, _, _ = O.moments(d, f)
    assert np.abs(u).max() > 0.1 * U                     # the lid has set the fluid moving
    assert np.abs(u[2]).max() > 1e-4 * U                 # with spanwise velocity (odd in z)
    assert mirrored_pair_error(lat, f) < 1e-13


def test_symmetric_forced_state_stays_symmetric():
    # a perturbed, mirror-symmetric start with a force along x: every term
    # of the step active, still symmetric
    lat = 19
    d = cavity(lat, (5, 6, 8), 1)
    d["G"] = (1e-4, -5e-5, 0.0)
    D, Q, shp = O.dims(d)
    rho = 1.0 + field(3, shp, 0.01)
    u = field(4, (3,) + shp, 0.02)
    rho = 0.5 * (rho + rho[::-1])
    u = 0.5 * (u + u[:, ::-1] * np.array([1, 1, -1])[:, None, None, None])
    f0 = O.init(d, rho=rho, u=u)
    assert mirrored_pair_error(lat, f0) < 1e-15
    f = O.run(d, f0, 30)
    assert mirrored_pair_error(lat, f) < 1e-13


def test_symmetry_detects_a_one_sided_slip():
    # the check has teeth: the same run with the lid given a spanwise
    # component (a one-sided asymmetry) leaves the mirror error at the size
    # of the flow
    d = cavity(19, (6, 5, 7), 1)
    d["uw"][3] = [U, 0.0, 0.2 * U]
    f = O.run(d, O.init(d), 60)
    assert mirrored_pair_error(19, f) > 1e-5
