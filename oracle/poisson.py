"""Isolated Poisson solve of a pair density.  TEST INFRASTRUCTURE ONLY.

Sec. 3.1 of the paper turns the integral in Eq. (2) into a Poisson problem for the pair
density and compares the O(N log N) solver route with O(N^2) direct integration.  Both
routes are written out here for the discrete convolution defined in ``oracle.grid``:

* ``fft``    -- zero-pad the N^3 density to P^3 (P = 2N), multiply its DFT by the DFT of
               the minimum-image kernel, inverse DFT, keep the N^3 box.  Exact (up to
               rounding) because the padded circular convolution contains the aperiodic one.
* ``direct`` -- v(r_i) = dV * sum_j G(r_i - r_j) rho(r_j) by brute force (tiny grids only).

Pinned by: brute force vs FFT to 1e-13, and the Gaussian Hartree energy / two-centre
closed forms with their O(h^2) discretisation error (tests/test_oracle_poisson.py).
"""

import os

import numpy as np
import scipy.fft

from . import grid

_WORKERS = os.cpu_count() or 1


def kernel_hat(n, h):
    """DFT of the minimum-image kernel on the padded P = 2N grid (real, even), times dV."""
    p = 2 * n
    g = grid.padded_kernel(p, h)
    gh = scipy.fft.fftn(g, workers=_WORKERS)
    return gh.real * h ** 3


def fft(rho, h, khat=None):
    """v = dV * G (*) rho on an N^3 box by the 2x zero-padded FFT.

    rho: (N, N, N) real or complex array, C order [x][y][z].  Returns an array of the same
    shape (complex if rho is complex, else real).
    """
    rho = np.asarray(rho)
    n = rho.shape[0]
    assert rho.shape == (n, n, n)
    p = 2 * n
    if khat is None:
        khat = kernel_hat(n, h)
    pad = np.zeros((p, p, p), dtype=np.complex128)
    pad[:n, :n, :n] = rho
    spec = scipy.fft.fftn(pad, workers=_WORKERS)
    spec *= khat
    out = scipy.fft.ifftn(spec, workers=_WORKERS)[:n, :n, :n]
    if np.iscomplexobj(rho):
        return np.ascontiguousarray(out)
    return np.ascontiguousarray(out.real)


def direct(rho, h):
    """Brute-force v(r_i) = dV * sum_j G(r_i - r_j) rho(r_j).  O(N^6): use N <= 12."""
    rho = np.asarray(rho)
    n = rho.shape[0]
    idx = np.indices((n, n, n)).reshape(3, -1).T.astype(np.float64)  # (Ng, 3)
    flat = rho.reshape(-1)
    out = np.empty(flat.shape, dtype=np.result_type(flat.dtype, np.float64))
    dv = h ** 3
    for i in range(idx.shape[0]):
        d = idx - idx[i]
        gi = grid.kernel_value(d[:, 0], d[:, 1], d[:, 2], h)
        out[i] = dv * np.dot(gi, flat)
    return out.reshape(rho.shape)
