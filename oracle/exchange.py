"""Exact exchange, direct and through Adaptively Compressed Exchange.  TEST INFRASTRUCTURE ONLY.

Paper: Eq. (2) (action of the exchange operator), Sec. 3.1 Eqs. (11)-(13) (ACE).

Readings of the paper taken here:

* Conjugation.  Eqs. (2), (11)-(13) are printed for real orbitals.  For complex orbitals the
  pair density is conj(phi_j) * psi, W_i = -sum_j phi_j v[conj(phi_j) phi_i],
  M_kl = dV sum_r conj(phi_k) W_l, -M = L L^H, xi = W L^{-H}, K_ACE = -xi xi^H dV.
* Sign.  The sentence introducing ACE writes the operator as zeta zeta^T while Eq. (13)
  carries a minus sign; Eq. (13) is followed (the exchange operator is negative
  semi-definite).
* Hermitisation.  M is replaced by (M + M^H)/2 before the Cholesky factorisation; in exact
  arithmetic M is already Hermitian.
* Energy.  The paper never writes the exchange energy; E_x = 1/2 sum_i <phi_i|K phi_i> dV
  = 1/2 sum_i M_ii, occupation 1 per orbital (one spin channel).

Orbitals are stored orbital-major: an (n, N, N, N) array.

Pinned by (tests/test_oracle_exchange.py): single-Gaussian and hydrogen-1s exchange energy
closed forms, Hermiticity and negativity of K, ACE exactness on the occupied span (the
paper's statement that ACE acts on the orbitals exactly as the full operator), invariance of
E_x under a unitary rotation of the orbitals, rank of K_ACE, and the brute-force Poisson sum.
"""

import numpy as np
import scipy.linalg

from . import poisson


def pair_potential(phi_a, phi_b, h, khat=None):
    """v = dV * G (*) (conj(phi_a) * phi_b): the Poisson solve of one pair density (Sec. 3.1)."""
    return poisson.fft(np.conj(phi_a) * phi_b, h, khat)


def apply_direct(phi, psi, h, khat=None):
    """(K psi)(r) = -sum_j phi_j(r) v[conj(phi_j) psi](r): Eq. (2), one Poisson solve per j."""
    n = phi.shape[0]
    if khat is None:
        khat = poisson.kernel_hat(phi.shape[1], h)
    out = np.zeros(psi.shape, dtype=np.result_type(phi.dtype, psi.dtype, np.float64))
    for j in range(n):
        out -= phi[j] * pair_potential(phi[j], psi, h, khat)
    return out


def build_w(phi, h, khat=None):
    """W_i = K[phi] phi_i for every occupied i: Eq. (11)."""
    if khat is None:
        khat = poisson.kernel_hat(phi.shape[1], h)
    return np.stack([apply_direct(phi, phi[i], h, khat) for i in range(phi.shape[0])])


def ace_build(phi, h, khat=None):
    """ACE construction, Sec. 3.1, in the paper's order.

    1. W_i = K phi_i (Eq. (11));
    2. M_kl = dV sum_r conj(phi_k) W_l;
    3. Cholesky of -M: -M = L L^H, L lower with positive diagonal;
    4. xi_k = sum_i W_i (L^{-H})_{ik} (Eq. (12));
    Returns (xi, M, L, E_x) with xi shaped like phi.
    """
    n = phi.shape[0]
    dv = h ** 3
    w = build_w(phi, h, khat)
    phim = phi.reshape(n, -1)
    wm = w.reshape(n, -1)
    m = dv * (np.conj(phim) @ wm.T)           # M_kl = dV <phi_k | W_l>
    m = 0.5 * (m + np.conj(m.T))
    lower = scipy.linalg.cholesky(-m, lower=True)
    # xi_k = sum_i W_i (L^{-H})_{ik}; rows of wm are the W_i, so row k of the result is
    # sum_i (L^{-H})_{ik} wm[i] = ((L^{-H})^T @ wm)[k].
    linv = scipy.linalg.solve_triangular(lower, np.eye(n), lower=True)
    lih = np.conj(linv.T)                     # L^{-H}
    xim = lih.T @ wm
    ex = 0.5 * float(np.real(np.trace(m)))
    return xim.reshape(phi.shape), m, lower, ex


def ace_build_targets(phi, psi, h, khat=None):
    """ACE of the exchange operator of the occupied orbitals phi compressed on the span of
    the target orbitals psi (Sec. 3.1: the unoccupied-orbital run includes the unoccupied
    orbitals in Eqs. (11)-(13)):

    1. W_t = K[phi] psi_t (Eq. (2));
    2. M_kl = dV sum_r conj(psi_k) W_l;
    3. -M = L L^H;
    4. xi_k = sum_t W_t (L^{-H})_{tk}.
    Returns (xi, M).
    """
    nt = psi.shape[0]
    dv = h ** 3
    if khat is None:
        khat = poisson.kernel_hat(phi.shape[1], h)
    w = np.stack([apply_direct(phi, psi[t], h, khat) for t in range(nt)])
    pm = psi.reshape(nt, -1)
    wm = w.reshape(nt, -1)
    m = dv * (np.conj(pm) @ wm.T)
    m = 0.5 * (m + np.conj(m.T))
    lower = scipy.linalg.cholesky(-m, lower=True)
    linv = scipy.linalg.solve_triangular(lower, np.eye(nt), lower=True)
    xim = np.conj(linv.T).T @ wm
    return xim.reshape(psi.shape), m


def ace_apply(xi, psi, h):
    """K_ACE psi = -sum_k xi_k (dV sum_r conj(xi_k) psi): Eq. (13) applied to psi.

    psi may hold one vector (N, N, N) or many (nv, N, N, N).
    """
    dv = h ** 3
    single = psi.ndim == 3
    ps = psi[None] if single else psi
    n = xi.shape[0]
    xim = xi.reshape(n, -1)
    pm = ps.reshape(ps.shape[0], -1)
    z = dv * (np.conj(xim) @ pm.T)            # (n, nv)
    out = -(z.T @ xim)                        # (nv, Ng)
    out = out.reshape(ps.shape)
    return out[0] if single else out


def exchange_energy(phi, h, khat=None):
    """E_x = 1/2 sum_i <phi_i | K phi_i> dV, from the direct operator (Eq. (2))."""
    w = build_w(phi, h, khat)
    dv = h ** 3
    return 0.5 * float(np.real(np.sum(np.conj(phi) * w)) * dv)
