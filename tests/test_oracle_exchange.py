"""Pins of the oracle's exchange operator (paper Eq. (2)) and ACE (Eqs. (11)-(13)).

Each check is chosen so that a plausible slip in the oracle fails it:
* closed-form exchange energies (kernel scale, factor 1/2, sign of K);
* the O(N_g^2) real-space operator matrix (conjugation placement, which factor is summed);
* Hermiticity / negativity of K (conjugation, sign);
* ACE exactness on the occupied span -- the paper's statement that after self-consistency ACE
  acts on the orbitals exactly as the full operator (transpose vs adjoint of L, sign of M);
* unitary invariance of E_x and of K_ACE (index bookkeeping of pairs);
* rank of K_ACE equal to the number of orbitals.
"""

import math

import numpy as np
import pytest

import synth
from golden_values import closed_forms
from oracle import exchange, grid, poisson


def _gauss_orbital(n, h, alpha):
    x = grid.coords(n, h)
    r2 = x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2
    return ((2.0 * alpha / math.pi) ** 0.75 * np.exp(-alpha * r2))[None]


def test_single_gaussian_exchange_energy():
    alpha = 0.9
    exact = closed_forms()["gaussian_exchange_coefficient"] * math.sqrt(alpha)
    vals = []
    for n, h in ((48, 0.25), (60, 0.2)):
        vals.append(exchange.exchange_energy(_gauss_orbital(n, h, alpha), h))
    h1, h2 = 0.25, 0.2
    ext = (h1 ** 2 * vals[1] - h2 ** 2 * vals[0]) / (h1 ** 2 - h2 ** 2)
    assert abs(ext - exact) / abs(exact) < 1e-4
    # the ACE route returns the same energy
    _, m, _, ex = exchange.ace_build(_gauss_orbital(48, 0.25, alpha), 0.25)
    assert ex == pytest.approx(vals[0], rel=1e-12)


@pytest.mark.slow
def test_hydrogen_1s_exchange_energy():
    n, h, z = 64, 0.2, 1.0
    x = grid.coords(n, h)
    r = np.sqrt(x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2)
    phi = (z ** 1.5 / math.sqrt(math.pi)) * np.exp(-z * r)
    phi = phi / math.sqrt(np.sum(phi ** 2) * h ** 3)
    ex = exchange.exchange_energy(phi[None], h)
    assert abs(ex - closed_forms()["hydrogen_1s_exchange_per_Z"] * z) < 2e-3


def _operator_matrix_brute(phi, h):
    """K(r, r') = -dV sum_j phi_j(r) G(r - r') conj(phi_j(r')) as an explicit matrix (tiny grids)."""
    n = phi.shape[1]
    idx = np.indices((n, n, n)).reshape(3, -1).T.astype(np.float64)
    d = idx[:, None, :] - idx[None, :, :]
    g = grid.kernel_value(d[..., 0], d[..., 1], d[..., 2], h)
    pm = phi.reshape(phi.shape[0], -1)
    k = np.zeros(g.shape, dtype=np.complex128)
    for j in range(pm.shape[0]):
        k -= pm[j][:, None] * g * np.conj(pm[j])[None, :]
    return k * h ** 3


def test_direct_exchange_equals_operator_matrix():
    m = synth.small_complex(11, 6, 0.45, 3)
    kmat = _operator_matrix_brute(m.phi, m.h)
    rng = np.random.default_rng(5)
    psi = rng.normal(size=m.phi.shape[1:]) + 1j * rng.normal(size=m.phi.shape[1:])
    ref = (kmat @ psi.reshape(-1)).reshape(psi.shape)
    got = exchange.apply_direct(m.phi, psi, m.h)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    # the matrix is Hermitian and negative semi-definite
    assert np.max(np.abs(kmat - kmat.conj().T)) < 1e-13 * np.max(np.abs(kmat))
    ev = np.linalg.eigvalsh(kmat)
    assert ev.max() < 1e-12 * abs(ev.min())


@pytest.fixture(scope="module")
def sys16():
    return synth.small_complex(21, 16, 0.35, 4, nvec=3)


def test_hermitian_and_negative(sys16):
    m = sys16
    a, b = m.psi[0], m.psi[1]
    ka = exchange.apply_direct(m.phi, a, m.h)
    kb = exchange.apply_direct(m.phi, b, m.h)
    dv = m.h ** 3
    ab = np.vdot(a, kb) * dv
    ba = np.vdot(b, ka) * dv
    assert abs(ab - np.conj(ba)) < 1e-13 * abs(ab)
    assert np.real(np.vdot(a, ka)) * dv < 0.0
    _, mm, _, ex = exchange.ace_build(m.phi, m.h)
    assert np.all(np.linalg.eigvalsh(mm) < 0.0)
    assert ex < 0.0


def test_ace_exact_on_occupied_span(sys16):
    m = sys16
    xi, mm, lower, ex = exchange.ace_build(m.phi, m.h)
    w = exchange.build_w(m.phi, m.h)
    kace = exchange.ace_apply(xi, m.phi, m.h)
    assert np.max(np.abs(kace - w)) < 1e-12 * np.max(np.abs(w))
    # any vector in the span is reproduced too
    c = np.array([0.3 - 0.2j, 1.1, -0.4j, 0.7 + 0.1j])
    v = np.tensordot(c, m.phi, axes=1)
    assert np.max(np.abs(exchange.ace_apply(xi, v, m.h) - exchange.apply_direct(m.phi, v, m.h))) \
        < 1e-12 * np.max(np.abs(w))
    # -M = L L^H with L lower triangular, positive diagonal
    assert np.allclose(np.triu(lower, 1), 0.0)
    assert np.all(np.real(np.diag(lower)) > 0)
    assert np.max(np.abs(lower @ lower.conj().T + mm)) < 1e-13 * np.max(np.abs(mm))
    # E_x = 1/2 trace M equals 1/2 sum <phi|K phi> from the direct operator
    assert ex == pytest.approx(exchange.exchange_energy(m.phi, m.h), rel=1e-13)


def test_unitary_invariance(sys16):
    m = sys16
    rng = np.random.default_rng(9)
    q, _ = np.linalg.qr(rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)))
    rot = np.tensordot(q.T, m.phi, axes=1)          # phi'_k = sum_i q_ik phi_i
    xi1, _, _, ex1 = exchange.ace_build(m.phi, m.h)
    xi2, _, _, ex2 = exchange.ace_build(rot, m.h)
    assert ex2 == pytest.approx(ex1, rel=1e-12)
    k1 = exchange.ace_apply(xi1, m.psi, m.h)
    k2 = exchange.ace_apply(xi2, m.psi, m.h)
    assert np.max(np.abs(k1 - k2)) < 1e-12 * np.max(np.abs(k1))


def test_ace_rank_and_hermitian():
    m = synth.small_complex(31, 6, 0.5, 3)
    xi, _, _, _ = exchange.ace_build(m.phi, m.h)
    ng = 6 ** 3
    eye = np.eye(ng).reshape(ng, 6, 6, 6).astype(np.complex128)
    cols = exchange.ace_apply(xi, eye, m.h).reshape(ng, ng).T    # column j = K e_j
    s = np.linalg.svd(cols, compute_uv=False)
    assert np.sum(s > 1e-10 * s[0]) == 3
    assert np.max(np.abs(cols - cols.conj().T)) < 1e-13 * np.max(np.abs(cols))


def test_ace_with_targets_exact_on_target_span():
    """ACE built over occupied + extra orbitals reproduces the exchange operator of the
    occupied orbitals on every target and on their combinations, and reduces to the plain
    construction when the targets are the occupied orbitals."""
    import synth
    mol = synth.small_real(31, 12, 0.45, 2, 3)
    phi, virt = mol.phi, mol.phi_virt
    h = 0.45
    khat = poisson.kernel_hat(12, h)
    psi = np.concatenate([phi, virt])
    xi, m = exchange.ace_build_targets(phi, psi, h, khat)
    for t in range(psi.shape[0]):
        ref = exchange.apply_direct(phi, psi[t], h, khat)
        got = exchange.ace_apply(xi, psi[t], h)
        assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    comb = 0.3 * psi[0] - 1.1 * psi[3] + 0.7 * psi[4]
    assert np.allclose(exchange.ace_apply(xi, comb, h), exchange.apply_direct(phi, comb, h, khat),
                       atol=1e-12)
    xi2, m2 = exchange.ace_build_targets(phi, phi, h, khat)
    xi1, m1, _, _ = exchange.ace_build(phi, h, khat)
    assert np.allclose(m1, m2, atol=1e-13) and np.allclose(xi1, xi2, atol=1e-12)
