"""Uniform isolated grid and the sampled (Hockney) Coulomb kernel.  TEST INFRASTRUCTURE ONLY.

The paper solves the exchange integral of Eq. (2) as a Poisson problem for the pair
density (Sec. 3.1) with zero boundary conditions on an isolated domain (Sec. 3.4).  It
names interpolating-scaling-function solvers but gives no discrete kernel, so the reading
taken here is:

* points x_k = (k - (N-1)/2) h, k = 0..N-1, on each axis (box centred on the origin);
  orbitals vanish outside the box;
* G(d) = 1 / (h |d|) for an integer displacement d != 0, and G(0) = C0 / h, where C0 is
  the average of 1/|r| over the unit cube centred on the origin:
  C0 = 3 ln(2 + sqrt 3) - pi/2 = 2.380077363979553...
* v(r_i) = dV * sum_j G(r_i - r_j) rho(r_j), dV = h^3.

Pinned by: tests/test_oracle_poisson.py (C0 by numerical cubature, the Gaussian Hartree
energy and two-centre erf closed forms, brute force equality with ``poisson.direct``).
"""

import math

import numpy as np

#: Average of 1/|r| over the unit cube [-1/2, 1/2]^3 (closed form of the cube integral).
C0 = 3.0 * math.log(2.0 + math.sqrt(3.0)) - math.pi / 2.0


def coords(n, h):
    """1-D coordinates x_k = (k - (n-1)/2) h of a box of n points centred on the origin."""
    return (np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * h


def mesh(n, h):
    """Three (n, n, n) coordinate arrays, C order [x][y][z] (z fastest)."""
    x = coords(n, h)
    return np.meshgrid(x, x, x, indexing="ij")


def kernel_value(dx, dy, dz, h):
    """G for an integer displacement (dx, dy, dz): 1/(h|d|), or C0/h at d = 0."""
    r2 = np.asarray(dx, dtype=np.float64) ** 2 + np.asarray(dy, dtype=np.float64) ** 2 \
        + np.asarray(dz, dtype=np.float64) ** 2
    out = np.empty(np.broadcast(r2).shape, dtype=np.float64)
    zero = r2 == 0
    with np.errstate(divide="ignore"):
        out[...] = 1.0 / (h * np.sqrt(r2))
    out[zero] = C0 / h
    return out


def padded_kernel(p, h):
    """G sampled on the periodic P^3 grid with minimum-image displacements.

    Index k on an axis stands for the displacement min(k, P-k) (sign is irrelevant as G is
    even).  With P = 2N every in-box difference lies in [-(N-1), N-1] and is represented
    exactly, so a circular convolution on this grid equals the aperiodic one on the box.
    """
    k = np.arange(p)
    d = np.minimum(k, p - k).astype(np.float64)
    dx = d[:, None, None]
    dy = d[None, :, None]
    dz = d[None, None, :]
    return kernel_value(dx, dy, dz, h)
