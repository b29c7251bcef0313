"""Seeded synthetic inputs shared by the oracle tests, the HIP parity tests and
the benchmark.

This module holds no arithmetic of the method: it only draws random numbers
and builds workload descriptions (sizes, parameters, seeds).  Every quantity
of the scheme (equilibria, moments, coefficients) is computed separately by
the oracle and by the HIP library from these inputs.
"""
from __future__ import annotations

import numpy as np


def rng(seed, *stream):
    """numpy Generator for a (seed, stream...) tuple."""
    return np.random.default_rng([int(seed)] + [int(s) for s in stream])


def field(seed, shape, scale=1.0, offset=0.0):
    """uniform(-1, 1) * scale + offset, float64."""
    return offset + scale * rng(seed, 1).uniform(-1.0, 1.0, size=shape)


def perturb(seed, base, rel=1e-3):
    """base * (1 + rel * uniform(-1,1)); used to move a state off equilibrium."""
    r = rng(seed, 2).uniform(-1.0, 1.0, size=np.shape(base))
    return np.asarray(base, dtype=np.float64) * (1.0 + rel * r)


def gaussian_bumps(seed, n, nbumps=8, amp=1e-5, width=16.0):
    """Force field made of `nbumps` periodic Gaussian bumps on an n x n grid,
    each with a random direction; returns [2, 1, n, n] (components, z, y, x).
    Centres ~ U[0,n)^2, directions ~ U[0, 2 pi); minimum-image distance."""
    g = rng(seed, 3)
    cx = g.uniform(0, n, nbumps)
    cy = g.uniform(0, n, nbumps)
    th = g.uniform(0, 2 * np.pi, nbumps)
    x = np.arange(n) + 0.5
    X, Y = np.meshgrid(x, x, indexing="xy")
    out = np.zeros((2, 1, n, n))
    for b in range(nbumps):
        dx = (X - cx[b] + n / 2) % n - n / 2
        dy = (Y - cy[b] + n / 2) % n - n / 2
        env = amp * np.exp(-(dx * dx + dy * dy) / (2 * width * width))
        out[0, 0] += np.cos(th[b]) * env
        out[1, 0] += np.sin(th[b]) * env
    return out


def batch_instances(seed=0, count=64, sides=tuple(range(64, 513, 32)), U=0.1):
    """Uneven D2Q9 instance set: per instance i an independent stream
    (seed, i) draws nx, ny from `sides`, Re ~ U[100,1000] and a body-force
    amplitude ~ U[0, 1e-5]; even i are lid-driven cavities, odd i periodic-x
    channels.  Returns a list of plain dicts."""
    out = []
    for i in range(count):
        g = rng(seed, 100, i)
        nx = int(g.choice(sides))
        ny = int(g.choice(sides))
        Re = float(g.uniform(100.0, 1000.0))
        amp = float(g.uniform(0.0, 1e-5))
        out.append(dict(index=i, nx=nx, ny=ny, Re=Re, force=amp,
                        kind="cavity" if i % 2 == 0 else "channel", U=U))
    return out
