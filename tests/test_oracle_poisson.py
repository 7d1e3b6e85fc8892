"""Pins of the oracle's isolated Poisson solver (paper Sec. 3.1) against things other than itself.

* C0 (self term of the sampled kernel) by numerical cubature of the cube average of 1/r.
* The padded-FFT route against the O(N^2) direct sum on tiny grids, incl. odd edges.
* The continuum limit: Gaussian Hartree self-energy and the two-centre erf formula, with the
  O(h^2) discretisation error removed by Richardson extrapolation.
"""

import math

import numpy as np
import pytest
import scipy.integrate
import scipy.special

from oracle import grid, poisson
from golden_values import closed_forms


def test_c0_by_cubature():
    # Average of 1/|r| over [-1/2, 1/2]^3 = 8 * int_{[0,1/2]^2} asinh(0.5/rho) dx dy
    # (the z integral of 1/|r| done in closed form); log singularity at the corner only.
    f = lambda y, x: math.asinh(0.5 / math.hypot(x, y)) if (x or y) else 0.0
    val, err = scipy.integrate.dblquad(f, 0.0, 0.5, 0.0, 0.5, epsabs=1e-13, epsrel=1e-13)
    assert abs(8.0 * val - grid.C0) < 1e-9
    assert abs(closed_forms()["cube_average_inverse_r"] - grid.C0) < 1e-15


def test_kernel_values():
    h = 0.3
    g = grid.padded_kernel(8, h)
    assert g[0, 0, 0] == pytest.approx(grid.C0 / h, rel=1e-15)
    assert g[1, 0, 0] == pytest.approx(1.0 / h, rel=1e-15)
    assert g[7, 0, 0] == pytest.approx(1.0 / h, rel=1e-15)       # minimum image
    assert g[1, 2, 2] == pytest.approx(1.0 / (3.0 * h), rel=1e-15)
    assert g[4, 4, 4] == pytest.approx(1.0 / (h * math.sqrt(48.0)), rel=1e-15)


@pytest.mark.parametrize("n,cplx", [(4, True), (7, True), (10, False), (11, True)])
def test_fft_equals_brute_force(n, cplx):
    rng = np.random.default_rng(7 + n)
    h = 0.37
    rho = rng.normal(size=(n, n, n))
    if cplx:
        rho = rho + 1j * rng.normal(size=(n, n, n))
    v_fft = poisson.fft(rho, h)
    v_dir = poisson.direct(rho, h)
    assert np.max(np.abs(v_fft - v_dir)) <= 1e-13 * np.max(np.abs(v_dir))


def _gauss_density(n, h, alpha, centre=(0.0, 0.0, 0.0)):
    x = grid.coords(n, h)
    r2 = ((x - centre[0])[:, None, None] ** 2 + (x - centre[1])[None, :, None] ** 2
          + (x - centre[2])[None, None, :] ** 2)
    return (alpha / math.pi) ** 1.5 * np.exp(-alpha * r2)


def _hartree_self(n, h, alpha):
    rho = _gauss_density(n, h, alpha)
    v = poisson.fft(rho, h)
    return 0.5 * float(np.sum(rho * v)) * h ** 3


def test_gaussian_hartree_energy_continuum_limit():
    alpha = 1.0
    exact = 0.5 * math.sqrt(2.0 * alpha / math.pi)
    h1, h2 = 0.25, 0.2
    e1 = _hartree_self(48, h1, alpha)
    e2 = _hartree_self(60, h2, alpha)
    # O(h^2) error of a cell-averaged self term: small, negative, shrinking as h^2
    r1, r2 = (e1 - exact) / exact, (e2 - exact) / exact
    assert -0.05 * alpha * h1 ** 2 < r1 < 0.0
    assert r2 / r1 == pytest.approx((h2 / h1) ** 2, rel=0.05)
    ext = (h1 ** 2 * e2 - h2 ** 2 * e1) / (h1 ** 2 - h2 ** 2)
    assert abs(ext - exact) / exact < 1e-4


def test_two_centre_erf():
    a, b, sep = 1.3, 0.8, 1.5
    exact = scipy.special.erf(math.sqrt(a * b / (a + b)) * sep) / sep
    vals = []
    for n, h in ((48, 0.25), (60, 0.2)):
        ra = _gauss_density(n, h, a, (-sep / 2, 0.0, 0.0))
        rb = _gauss_density(n, h, b, (sep / 2, 0.0, 0.0))
        vals.append(float(np.sum(rb * poisson.fft(ra, h))) * h ** 3)
    h1, h2 = 0.25, 0.2
    ext = (h1 ** 2 * vals[1] - h2 ** 2 * vals[0]) / (h1 ** 2 - h2 ** 2)
    assert abs(ext - exact) / exact < 1e-4
    assert abs(vals[1] - exact) / exact < 3e-3


def test_pair_symmetry_and_reality():
    rng = np.random.default_rng(3)
    n, h = 9, 0.4
    a = rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n))
    b = rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n))
    vab = poisson.fft(np.conj(a) * b, h)
    vba = poisson.fft(np.conj(b) * a, h)
    assert np.max(np.abs(vab - np.conj(vba))) < 1e-13 * np.max(np.abs(vab))
    r = poisson.fft(np.abs(a) ** 2, h)
    assert r.dtype == np.float64
