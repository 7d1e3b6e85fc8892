"""Pins of the oracle's two-electron integrals and RHF TDA coupling block (paper Eq. (7)).

* single integrals against an explicit double sum over grid points (tiny grid);
* the (ii|ii) self-integral of a Gaussian orbital against its closed form;
* symmetries: 8-fold for real orbitals, Hermiticity of the block, singlet - triplet =
  2 (ai|jb) (the delta_M structure of Eq. (7));
* the TDA matrix reduces to the independent-particle excitations when C = 0.
"""

import math

import numpy as np
import pytest

import synth
from golden_values import closed_forms
from oracle import grid, poisson, tda


def _brute_integral(p, q, r, s, h):
    n = p.shape[0]
    idx = np.indices((n, n, n)).reshape(3, -1).T.astype(np.float64)
    d = idx[:, None, :] - idx[None, :, :]
    g = grid.kernel_value(d[..., 0], d[..., 1], d[..., 2], h)
    left = (np.conj(p) * q).reshape(-1)        # at r'
    right = (np.conj(r) * s).reshape(-1)       # at r
    return complex(right @ g @ left) * h ** 6


def test_integral_brute_force():
    rng = np.random.default_rng(2)
    n, h = 6, 0.5
    f = [rng.normal(size=(n, n, n)) + 1j * rng.normal(size=(n, n, n)) for _ in range(4)]
    got = tda.integral(*f, h)
    ref = _brute_integral(*f, h)
    assert abs(got - ref) < 1e-12 * abs(ref)


def test_gaussian_self_integral():
    alpha = 0.7          # density exponent 2*alpha; h^4 terms stay below 1e-4
    exact = -2.0 * closed_forms()["gaussian_exchange_coefficient"] * math.sqrt(alpha)
    vals = []
    for n, h in ((48, 0.25), (60, 0.2)):
        x = grid.coords(n, h)
        r2 = x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2
        g = (2.0 * alpha / math.pi) ** 0.75 * np.exp(-alpha * r2)
        vals.append(tda.integral(g, g, g, g, h).real)
    ext = (0.25 ** 2 * vals[1] - 0.2 ** 2 * vals[0]) / (0.25 ** 2 - 0.2 ** 2)
    assert abs(ext - exact) / exact < 1e-4


@pytest.fixture(scope="module")
def small():
    return synth.small_real(41, 10, 0.5, 3, 4)


def test_real_eightfold_symmetry(small):
    o, v, h = small.phi, small.phi_virt, small.h
    base = tda.integral(o[0], v[1], o[2], v[3], h)
    for perm in [(v[1], o[0], o[2], v[3]), (o[0], v[1], v[3], o[2]),
                 (o[2], v[3], o[0], v[1]), (v[3], o[2], v[1], o[0])]:
        assert abs(tda.integral(*perm, h) - base) < 1e-13 * abs(base)


@pytest.mark.parametrize("delta_m", [2, 0])
def test_block_structure(small, delta_m):
    o, v, h = small.phi, small.phi_virt, small.h
    c = tda.coupling_block(o, v, h, delta_m)
    assert c.shape == (12, 12)
    assert np.max(np.abs(c - c.T)) < 1e-13 * np.max(np.abs(c))
    for (i, a, j, b) in [(0, 0, 0, 0), (1, 2, 0, 3), (2, 3, 1, 1)]:
        e = tda.coupling_element(o, v, h, delta_m, i, a, j, b)
        assert abs(c[i * 4 + a, j * 4 + b] - e.real) < 1e-13 * np.max(np.abs(c))


def test_singlet_minus_triplet(small):
    o, v, h = small.phi, small.phi_virt, small.h
    cs = tda.coupling_block(o, v, h, 2)
    ct = tda.coupling_block(o, v, h, 0)
    for (i, a, j, b) in [(0, 1, 2, 3), (1, 1, 1, 1)]:
        ex = tda.integral(v[a], o[i], o[j], v[b], h).real
        assert cs[i * 4 + a, j * 4 + b] - ct[i * 4 + a, j * 4 + b] == pytest.approx(2 * ex, rel=1e-12)


def test_complex_block_hermitian():
    m = synth.small_complex(43, 8, 0.5, 4)
    o, v = m.phi[:2], m.phi[2:]
    c = tda.coupling_block(o, v, m.h, 2)
    assert np.max(np.abs(c - c.conj().T)) < 1e-13 * np.max(np.abs(c))


def test_tda_reduces_to_ipa(small):
    eo, ev = small.eps_occ, small.eps_virt
    w, _ = tda.excitations(tda.tda_matrix(np.zeros((12, 12)), eo, ev))
    assert np.allclose(w, tda.ipa_excitations(eo, ev), atol=1e-15)


def test_oscillator_two_level():
    # one transition, no coupling: f = 2/3 (eps_a - eps_i) |<i|r|a>|^2
    n, h = 16, 0.4
    x = grid.coords(n, h)
    r2 = x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2
    s = np.exp(-r2)
    p = x[:, None, None] * np.exp(-r2)
    s /= math.sqrt(np.sum(s * s) * h ** 3)
    p /= math.sqrt(np.sum(p * p) * h ** 3)
    mesh = np.meshgrid(x, x, x, indexing="ij")
    dip = tda.dipole_elements(s[None], p[None], h, mesh)
    # <s|x|p> for these two normalised functions: sum x s p dV, evaluated independently
    dx = float(np.sum(mesh[0] * s * p) * h ** 3)
    assert abs(dip[0, 0, 0] - dx) < 1e-14 and abs(dip[1, 0, 0]) < 1e-14
    f = tda.oscillator_strengths(np.array([0.5]), np.ones((1, 1)), dip)
    assert f[0] == pytest.approx(2.0 / 3.0 * 0.5 * dx * dx, rel=1e-13)
    # strength function integrates to the oscillator strength
    wg = np.linspace(-200.0, 200.0, 400001)
    sfun = tda.strength_function(wg, np.array([0.5]), f, 0.01)
    assert np.trapezoid(sfun, wg) == pytest.approx(f[0], rel=1e-4)


def test_rpa_closed_forms():
    # one transition: omega = sqrt(A^2 - B^2); B = 0: the Tamm-Dancoff eigenvalues
    assert tda.rpa_excitations(np.array([[0.7]]), np.array([[0.2]]))[0] == pytest.approx(
        np.sqrt(0.7 ** 2 - 0.2 ** 2), rel=1e-14)
    rng = np.random.default_rng(3)
    a = rng.normal(size=(6, 6))
    a = a @ a.T + 6 * np.eye(6)
    assert np.allclose(tda.rpa_excitations(a, np.zeros((6, 6))), np.linalg.eigvalsh(a))
    b = rng.normal(size=(6, 6)) * 0.3
    b = 0.5 * (b + b.T)
    assert np.allclose(tda.rpa_excitations(a, b), tda.rpa_hermitian(a, b), rtol=1e-12)


def test_b_block_structure(small):
    occ, virt, h = small.phi, small.phi_virt, small.h
    b2 = tda.b_block(occ, virt, h, 2)
    b0 = tda.b_block(occ, virt, h, 0)
    assert np.allclose(b2, b2.T, atol=1e-12)
    no, nv = occ.shape[0], virt.shape[0]
    i, a, j, bb = 1, 2, 0, 1
    ref = 2 * tda.integral(occ[i], virt[a], virt[bb], occ[j], h) - \
        tda.integral(occ[i], virt[bb], virt[a], occ[j], h)
    assert b2[i * nv + a, j * nv + bb] == pytest.approx(ref.real, abs=1e-12)
    # singlet - triplet = 2 (ia|bj), the same matrix as the A block's (ai|jb) for real orbitals
    c2 = tda.coupling_block(occ, virt, h, 2)
    c0 = tda.coupling_block(occ, virt, h, 0)
    assert np.allclose(b2 - b0, c2 - c0, atol=1e-12)


def test_closed_shell_uhf_is_union_of_singlets_and_triplets(small):
    occ, virt, h = small.phi, small.phi_virt, small.h
    no, nv = occ.shape[0], virt.shape[0]
    eo = np.array([-1.3, -1.1, -0.9][:no])
    ev = np.linspace(0.1, 0.5, nv)
    de = (ev[None, :] - eo[:, None]).reshape(-1)
    cu, bu = tda.uhf_blocks(occ, virt, occ, virt, h)
    du = np.concatenate([de, de])
    uhf_tda = np.linalg.eigvalsh(np.diag(du) + cu)
    rhf = [np.linalg.eigvalsh(np.diag(de) + tda.coupling_block(occ, virt, h, dm)) for dm in (2, 0)]
    assert np.allclose(uhf_tda, np.sort(np.concatenate(rhf)), atol=1e-10)
    uhf_rpa = tda.rpa_excitations(np.diag(du) + cu, bu)
    rhf_rpa = [tda.rpa_excitations(np.diag(de) + tda.coupling_block(occ, virt, h, dm),
                                   tda.b_block(occ, virt, h, dm)) for dm in (2, 0)]
    assert np.allclose(uhf_rpa, np.sort(np.concatenate(rhf_rpa)), atol=1e-9)


def _oscillator_states(n, h, w):
    """Eigenfunctions of the anisotropic harmonic oscillator V = 1/2 sum_c w_c c^2, sampled
    on the grid: psi(n_x, n_y, n_z) = prod_c H_{n_c}-type factors times the ground Gaussian,
    normalised analytically (no grid renormalisation).  Returned as a dict keyed by
    (n_x, n_y, n_z) for quanta 0..2 per axis."""
    x = grid.coords(n, h)
    c = np.meshgrid(x, x, x, indexing="ij")
    g = np.ones((n, n, n))
    for k in range(3):
        g = g * (w[k] / math.pi) ** 0.25 * np.exp(-0.5 * w[k] * c[k] ** 2)

    def factor(k, q):
        u = math.sqrt(w[k]) * c[k]
        if q == 0:
            return 1.0
        if q == 1:
            return math.sqrt(2.0) * u
        return (2.0 * u * u - 1.0) / math.sqrt(2.0)

    out = {}
    for q in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (0, 0, 2)]:
        out[q] = g * factor(0, q[0]) * factor(1, q[1]) * factor(2, q[2])
    return out, c


def test_dipoles_and_oscillator_strengths_harmonic_closed_forms():
    """Eqs. (8)-(9) on harmonic-oscillator states, where every matrix element is known:
    <0|x|1_x> = 1/sqrt(2 w_x), <1_z|z|2_z> = 1/sqrt(w_z), and the ground-state strengths
    f = 2/3 w |d|^2 are 1/3 per axis, summing to 1 (the Thomas-Reiche-Kuhn sum rule for one
    electron).  Two occupied orbitals and four virtual ones make the ia = i * n_virt + a
    index layout matter; the dipole operator uses the grid coordinates of the oracle."""
    w = (0.8, 1.1, 1.4)
    n, h = 56, 0.25   # box +-6.9 bohr: Gaussian tails below 1e-15
    st, coords = _oscillator_states(n, h, w)
    occ = np.stack([st[(0, 0, 0)], st[(0, 0, 1)]])
    virt = np.stack([st[(1, 0, 0)], st[(0, 1, 0)], st[(0, 0, 2)], st[(2, 0, 0)]])
    dip = tda.dipole_elements(occ, virt, h, coords)
    nv = 4
    expect = np.zeros((3, 2, nv))
    expect[0, 0, 0] = 1.0 / math.sqrt(2.0 * w[0])     # <0|x|1x>
    expect[1, 0, 1] = 1.0 / math.sqrt(2.0 * w[1])     # <0|y|1y>
    expect[2, 1, 2] = 1.0 / math.sqrt(w[2])           # <1z|z|2z>
    assert np.max(np.abs(dip - expect)) < 1e-12
    # pure transitions (unit TDA vectors) and their energies
    omega = np.array([w[0], w[1], w[2], 2.0 * w[0]])
    x = np.zeros((2 * nv, 4))
    for k, ia in enumerate([0 * nv + 0, 0 * nv + 1, 1 * nv + 2, 0 * nv + 3]):
        x[ia, k] = 1.0
    f = tda.oscillator_strengths(omega, x, dip)
    assert np.allclose(f, [1.0 / 3.0, 1.0 / 3.0, 2.0 / 3.0, 0.0], atol=1e-12)
    # the ground state alone against every excited state of the set: the strengths sum to 1
    virt0 = np.stack([st[q] for q in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (0, 0, 2)]])
    dip0 = tda.dipole_elements(occ[:1], virt0, h, coords)
    om0 = np.array([w[0], w[1], w[2], 2.0 * w[0], 2.0 * w[2]])
    f0 = tda.oscillator_strengths(om0, np.eye(5), dip0)
    assert np.sum(f0) == pytest.approx(1.0, abs=1e-12)
    # a mixed state: d = (d_x, d_y, 0) / sqrt(2), f = 2/3 w (1/(2 w_x) + 1/(2 w_y)) / 2
    xm = np.zeros((2 * nv, 1))
    xm[0 * nv + 0, 0] = xm[0 * nv + 1, 0] = 1.0 / math.sqrt(2.0)
    fm = tda.oscillator_strengths(np.array([0.9]), xm, dip)
    ref = 2.0 / 3.0 * 0.9 * 0.5 * (1.0 / (2.0 * w[0]) + 1.0 / (2.0 * w[1]))
    assert fm[0] == pytest.approx(ref, rel=1e-12)
