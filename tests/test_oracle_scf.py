"""Pins of the oracle's SCF pieces (paper Eq. (1), (14), (15)) and of its convolutional-network
reference, against closed forms, library routines and numerical differentiation."""

import math

import numpy as np
import pytest
import scipy.ndimage

from oracle import convnet, grid, poisson, scf


def _gauss(n, h, a):
    x = grid.coords(n, h)
    r2 = x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2
    return np.exp(-a * r2), r2


def test_laplacian_of_gaussian_fourth_order():
    a = 0.5
    errs = []
    for n, h in ((60, 0.2), (120, 0.1)):
        f, r2 = _gauss(n, h, a)
        exact = (4 * a * a * r2 - 6 * a) * f
        errs.append(np.max(np.abs(scf.laplacian(f, h) - exact)))
    assert errs[1] < 1e-4
    assert errs[0] / errs[1] == pytest.approx(16.0, rel=0.1)   # O(h^4)


def test_harmonic_oscillator_levels():
    # T + 1/2 sum_a w_a^2 x_a^2 (anisotropic, no degeneracy): levels sum_a w_a (m_a + 1/2)
    n, h = 36, 0.22
    w = (1.0, 1.3, 1.6)
    x = grid.coords(n, h)
    v = 0.5 * (w[0] ** 2 * x[:, None, None] ** 2 + w[1] ** 2 * x[None, :, None] ** 2
               + w[2] ** 2 * x[None, None, :] ** 2)
    e, vec = scf.lowest_states(lambda f: scf.kinetic(f, h) + v * f, n, 4, h)
    e0 = 0.5 * sum(w)
    assert np.allclose(e, [e0, e0 + w[0], e0 + w[1], e0 + w[2]], atol=1e-3)
    # dV-normalised, orthogonal
    s = np.einsum("ixyz,jxyz->ij", vec, vec) * h ** 3
    assert np.allclose(s, np.eye(4), atol=1e-10)


def test_external_potential_values():
    n, h = 12, 0.5
    v = scf.external_potential(n, h, [(0.0, 0.0, 0.25)], [2.0], 0.7)
    x = grid.coords(n, h)
    r = math.sqrt(x[7] ** 2 + x[7] ** 2 + (x[3] - 0.25) ** 2)
    assert v[7, 7, 3] == pytest.approx(-2.0 * math.erf(r / 0.7) / r, rel=1e-14)


def test_one_orbital_hartree_exchange_ratio():
    # one doubly occupied orbital: exchange = -1/2 Hartree exactly
    n, h = 20, 0.35
    f, _ = _gauss(n, h, 0.8)
    f = f / math.sqrt(np.sum(f * f) * h ** 3)
    e = scf.energies(f[None], np.zeros((n, n, n)), h, poisson.kernel_hat(n, h))
    assert e["exchange"] == pytest.approx(-0.5 * e["hartree"], rel=1e-13)


@pytest.mark.slow
def test_scf_self_consistent():
    n, h = 14, 0.45
    v = scf.external_potential(n, h, [(-0.6, 0.0, 0.0), (0.6, 0.2, 0.0)], [3.0, 3.0], 0.8)
    rng = np.random.default_rng(4)
    x = grid.coords(n, h)
    guess = np.stack([np.exp(-0.7 * ((x[:, None, None] - c[0]) ** 2 + (x[None, :, None] - c[1]) ** 2
                                      + x[None, None, :] ** 2)) for c in ((-0.6, 0), (0.6, 0.2))])
    phi, e, hist = scf.scf(guess + 0.01 * rng.normal(size=guess.shape), v, h, tol=1e-8)
    assert hist[-1]["density_error"] < 1e-8
    khat = poisson.kernel_hat(n, h)
    vloc = v + poisson.fft(scf.density(phi), h, khat)
    fphi = scf.fock_apply(phi, phi, vloc, h, khat)
    lam = np.einsum("ixyz,jxyz->ij", phi, fphi) * h ** 3
    res = fphi - np.tensordot(lam, phi, axes=1)
    assert np.max(np.abs(res)) < 1e-4 * np.max(np.abs(fphi))
    # orbital energies are the eigenvalues of the Lagrange matrix; total energy is variational
    assert np.allclose(np.linalg.eigvalsh(lam), hist[-1]["eigenvalues"], atol=1e-6)
    assert e["exchange"] < 0.0 < e["hartree"]
    # a perturbed (orthonormalised) orbital set has higher energy
    pert = scf.loewdin(phi + 0.02 * rng.normal(size=phi.shape), h)
    assert scf.energies(pert, v, h, khat)["total"] > e["total"]


def test_conv_delta_and_scipy():
    rng = np.random.default_rng(1)
    w = rng.normal(size=(2, 1, 3, 3, 3))
    b = np.array([0.5, -1.0])
    x = np.zeros((1, 7, 7, 7))
    x[0, 3, 3, 3] = 1.0
    y = convnet.conv3d(x, w, b)
    # y[o](p) = b + w[o, 0, c - p + 1]: the flipped kernel around the delta
    for o in range(2):
        patch = y[o, 2:5, 2:5, 2:5] - b[o]
        assert np.allclose(patch, w[o, 0, ::-1, ::-1, ::-1])
    xr = rng.normal(size=(3, 6, 6, 6))
    wr = rng.normal(size=(2, 3, 3, 3, 3))
    y = convnet.conv3d(xr, wr, np.zeros(2))
    ref = sum(scipy.ndimage.correlate(xr[i], wr[0, i], mode="constant") for i in range(3))
    assert np.max(np.abs(y[0] - ref)) < 1e-12


def test_conv_gradients_finite_difference():
    rng = np.random.default_rng(2)
    params = convnet.init_params(rng, scale=1.0)
    params = [(w, rng.normal(scale=0.1, size=b.shape)) for w, b in params]
    x = rng.normal(size=(6, 6, 6))
    t = rng.normal(size=(6, 6, 6))
    y, cache = convnet.forward(params, x)
    grads = convnet.backward(params, cache, y, t)
    eps = 1e-6
    for li, idx in [(0, (3, 0, 1, 2, 0)), (1, (5, 7, 2, 1, 1)), (2, (0, 4, 0, 0, 2))]:
        w, b = params[li]
        wp = w.copy(); wp[idx] += eps
        wm = w.copy(); wm[idx] -= eps
        pp = list(params); pp[li] = (wp, b)
        pm = list(params); pm[li] = (wm, b)
        num = (convnet.loss(convnet.forward(pp, x)[0], t) - convnet.loss(convnet.forward(pm, x)[0], t)) / (2 * eps)
        assert grads[li][0][idx] == pytest.approx(num, rel=1e-5, abs=1e-10)
    bp = params[1][1].copy(); bp[3] += eps
    bm = params[1][1].copy(); bm[3] -= eps
    pp = list(params); pp[1] = (params[1][0], bp)
    pm = list(params); pm[1] = (params[1][0], bm)
    num = (convnet.loss(convnet.forward(pp, x)[0], t) - convnet.loss(convnet.forward(pm, x)[0], t)) / (2 * eps)
    assert grads[1][1][3] == pytest.approx(num, rel=1e-5, abs=1e-10)


def test_kinetic_precondition_converges_to_shifted_solve():
    n, h, shift = 12, 0.5, 1.0
    # the diagonal used by the preconditioner is the operator's own diagonal element
    delta = np.zeros((n, n, n))
    delta[6, 5, 4] = 1.0
    assert scf.kinetic(delta, h)[6, 5, 4] == pytest.approx(scf.kinetic_diagonal(h), rel=1e-14)
    rng = np.random.default_rng(3)
    r = rng.normal(size=(n, n, n))
    z = scf.kinetic_precondition(r, h, shift, 3000, 0.8)
    res = scf.kinetic(z, h) + shift * z - r
    assert np.max(np.abs(res)) < 1e-8 * np.max(np.abs(r))
    # one sweep: the diagonal (Jacobi) scaling alone
    assert np.allclose(scf.kinetic_precondition(r, h, shift, 1, 0.8),
                       r / (scf.kinetic_diagonal(h) + shift), rtol=0, atol=0)


def test_adam_constant_gradient_moves_by_lr_sign():
    # with a constant gradient the bias-corrected moments are g and g^2 exactly, so every
    # step moves each parameter by lr * g / (|g| + eps)
    g = [np.array([2.0, -0.5, 1e-3]), np.array([[-3.0]])]
    p = [np.zeros(3), np.zeros((1, 1))]
    st = {}
    for _ in range(5):
        p = convnet.adam_step(p, g, st, lr=0.01)
    assert np.allclose(p[0], -5 * 0.01 * g[0] / (np.abs(g[0]) + 1e-8), rtol=1e-12)
    assert np.allclose(p[1], [[0.05]], rtol=1e-12)


def test_param_flatten_roundtrip_and_count():
    rng = np.random.default_rng(5)
    params = convnet.init_params(rng)
    vec = convnet.flatten(params)
    assert vec.size == 2177
    back = convnet.unflatten(vec)
    for (w, b), (w2, b2) in zip(params, back):
        assert np.array_equal(w, w2) and np.array_equal(b, b2)
