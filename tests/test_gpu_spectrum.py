"""GPU parity of the Tamm-Dancoff eigen-solution and spectrum (paper Sec. 2, Eqs. (7)-(10)) and of
the small dense helpers they use, against the FP64 oracle and numpy's LAPACK routines."""

import numpy as np
import pytest
import torch

import synth
from oracle import grid, tda

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _ace():
    import paper_2405_01522_amd as ace
    return ace


@pytest.mark.parametrize("n", [1, 2, 7, 33, 64])
def test_sym_eig_small(n):
    ace = _ace()
    rng = np.random.default_rng(n)
    a = rng.normal(size=(n, n))
    a = a + a.T
    w, v = ace.sym_eig_small(torch.from_numpy(a).to(DEV))
    w, v = w.cpu().numpy(), v.cpu().numpy()
    wr = np.linalg.eigvalsh(a)
    assert np.max(np.abs(w - wr)) < 1e-12 * max(1.0, np.max(np.abs(wr)))
    assert np.max(np.abs(a @ v - v * w[None, :])) < 1e-11 * max(1.0, np.max(np.abs(wr)))
    assert np.max(np.abs(v.T @ v - np.eye(n))) < 1e-12


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_dense_gemm(ta, tb):
    ace = _ace()
    rng = np.random.default_rng(3 + 2 * ta + tb)
    m, n, k = 70, 45, 130
    a = rng.normal(size=(k, m) if ta else (m, k))
    b = rng.normal(size=(n, k) if tb else (k, n))
    c0 = rng.normal(size=(m, n))
    ref = 0.7 * ((a.T if ta else a) @ (b.T if tb else b)) - 0.3 * c0
    out = torch.from_numpy(c0.copy()).to(DEV)
    got = ace.dense_gemm(torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV), ta, tb, 0.7, -0.3, out)
    assert np.max(np.abs(got.cpu().numpy() - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.fixture(scope="module")
def mid():
    m = synth.small_real(23, 24, 0.3, 4, 8)
    return m, tda.coupling_block(m.phi, m.phi_virt, m.h, 2)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tda_states_and_spectrum(mid, prec):
    """Lowest TDA states (Davidson), oscillator strengths and the broadened spectrum vs the
    oracle's dense eigendecomposition: 1e-9 eV (FP64 storage) / 1e-4 eV (FP32 storage)."""
    ace = _ace()
    m, cref = mid
    dt = torch.float64 if prec == "fp64" else torch.float32
    single = prec == "fp32"
    ctx = ace.AceContext(m.n, m.h, dt)
    occ = torch.from_numpy(synth.to_precision(m.phi, single)).to(DEV)
    virt = torch.from_numpy(synth.to_precision(m.phi_virt, single)).to(DEV)
    c = ctx.tda_coupling(occ, virt, 2)
    k = 6
    omega, x, it = ctx.tda_excitations(c, m.eps_occ, m.eps_virt, k, tol=1e-9)
    assert it > 0
    w_ref, x_ref = tda.excitations(tda.tda_matrix(cref, m.eps_occ, m.eps_virt))
    ev = 27.211386245988
    tol_ev = 1e-9 if prec == "fp64" else 1e-4
    assert np.max(np.abs(omega.cpu().numpy() - w_ref[:k])) * ev < tol_ev
    # oscillator strengths (vectors unique up to sign for these non-degenerate states)
    f, d = ctx.tda_oscillator_strengths(occ, virt, x, omega)
    mesh = np.meshgrid(grid.coords(m.n, m.h), grid.coords(m.n, m.h), grid.coords(m.n, m.h), indexing="ij")
    dip = tda.dipole_elements(m.phi, m.phi_virt, m.h, mesh)
    f_ref = tda.oscillator_strengths(w_ref[:k], x_ref[:, :k], dip)
    ftol = 1e-8 if prec == "fp64" else 2e-4
    assert np.max(np.abs(f.cpu().numpy() - f_ref)) < ftol * max(1e-3, np.max(np.abs(f_ref)))
    s = ace.strength_function(omega, f, 0.0, 0.01, 400, 0.0005)
    s_ref = tda.strength_function(np.arange(400) * 0.01, w_ref[:k], f_ref, 0.0005)
    assert np.max(np.abs(s.cpu().numpy() - s_ref)) < max(1e-6, ftol) * max(1.0, np.max(np.abs(s_ref))) * 50


def test_tda_states_config3():
    """Full 64^3 / 16 + 32 block: the Davidson states equal the dense eigendecomposition of the
    same GPU block (numpy LAPACK), and the lowest excitation is positive."""
    ace = _ace()
    m = synth.config3()
    ctx = ace.AceContext(m.n, m.h, torch.float32)
    occ = torch.from_numpy(synth.to_precision(m.phi, True)).to(DEV)
    virt = torch.from_numpy(synth.to_precision(m.phi_virt, True)).to(DEV)
    c = ctx.tda_coupling(occ, virt, 2)
    omega, x, it = ctx.tda_excitations(c, m.eps_occ, m.eps_virt, 8, tol=1e-8)
    assert it > 0
    a = tda.tda_matrix(c.cpu().numpy(), m.eps_occ, m.eps_virt)
    w_ref = np.linalg.eigvalsh(a)[:8]
    assert np.max(np.abs(omega.cpu().numpy() - w_ref)) < 1e-10
    assert w_ref[0] > 0.0


# ---- full TDHF (B block), UHF, RHF = UHF ---------------------------------------------------

def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("delta_m", [2, 0])
def test_tdhf_blocks_match_oracle(prec, delta_m):
    import paper_2405_01522_amd as ace
    from oracle import tda
    mol = synth.small_real(51, 12, 0.45, 3, 4)
    dt = torch.float64 if prec == "fp64" else torch.float32
    ctx = ace.AceContext(12, 0.45, dt)
    c, b = ctx.tdhf_coupling(_dev(mol.phi).to(dt), _dev(mol.phi_virt).to(dt), delta_m)
    cr = tda.coupling_block(mol.phi, mol.phi_virt, 0.45, delta_m)
    br = tda.b_block(mol.phi, mol.phi_virt, 0.45, delta_m)
    tol = 1e-10 if prec == "fp64" else 3e-6
    sc = max(np.max(np.abs(cr)), np.max(np.abs(br)))
    assert np.max(np.abs(c.cpu().numpy() - cr)) < tol * sc
    assert np.max(np.abs(b.cpu().numpy() - br)) < tol * sc
    assert np.array_equal(b.cpu().numpy(), b.cpu().numpy().T)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_uhf_blocks_match_oracle_open_shell(prec):
    import paper_2405_01522_amd as ace
    from oracle import tda
    a = synth.small_real(61, 12, 0.45, 3, 4)
    b = synth.small_real(62, 12, 0.45, 2, 3)
    dt = torch.float64 if prec == "fp64" else torch.float32
    ctx = ace.AceContext(12, 0.45, dt)
    t = lambda x: _dev(x).to(dt)
    c, bb = ctx.uhf_coupling(t(a.phi), t(a.phi_virt), t(b.phi), t(b.phi_virt))
    cr, br = tda.uhf_blocks(a.phi, a.phi_virt, b.phi, b.phi_virt, 0.45)
    tol = 1e-10 if prec == "fp64" else 3e-6
    sc = max(np.max(np.abs(cr)), np.max(np.abs(br)))
    assert np.max(np.abs(c.cpu().numpy() - cr)) < tol * sc
    assert np.max(np.abs(bb.cpu().numpy() - br)) < tol * sc


def test_tdhf_excitations_match_oracle_and_rhf_equals_uhf():
    import paper_2405_01522_amd as ace
    from oracle import tda
    mol = synth.small_real(71, 12, 0.45, 3, 5)
    no, nv = 3, 5
    ctx = ace.AceContext(12, 0.45, torch.float64)
    occ, virt = _dev(mol.phi), _dev(mol.phi_virt)
    de = (mol.eps_virt[None, :] - mol.eps_occ[:, None]).reshape(-1)
    k = 6
    res = {}
    for dm in (2, 0):
        c, b = ctx.tdhf_coupling(occ, virt, dm)
        om, xpy, it = ctx.tdhf_excitations(c, b, de, k, tol=1e-9)
        ref = tda.rpa_excitations(np.diag(de) + c.cpu().numpy(), b.cpu().numpy())
        assert np.allclose(om.cpu().numpy(), ref[:k], atol=1e-9), (om, ref[:k])
        # X+Y solves the first Casida equation pair: (A-B)(A+B)(X+Y) = omega^2 (X+Y)
        am = np.diag(de) + c.cpu().numpy()
        bm = b.cpu().numpy()
        v = xpy.cpu().numpy()
        lhs = (am - bm) @ (am + bm) @ v.T
        assert np.max(np.abs(lhs - v.T * om.cpu().numpy() ** 2)) < 1e-7 * np.max(np.abs(lhs))
        # B = 0 in the same solver gives the Tamm-Dancoff eigenvalues
        tda_om, _, _ = ctx.tda_excitations_diag(c, de, k, tol=1e-9)
        zom, _, _ = ctx.tdhf_excitations(c, torch.zeros_like(b), de, k, tol=1e-9)
        assert np.allclose(zom.cpu().numpy(), tda_om.cpu().numpy(), atol=1e-9)
        res[dm] = np.linalg.eigvalsh(am)[:], ref
    # closed-shell UHF: union of singlet and triplet spectra (TDA and full TDHF)
    cu, bu = ctx.uhf_coupling(occ, virt, occ, virt)
    du = np.concatenate([de, de])
    om_u, _, _ = ctx.tda_excitations_diag(cu, du, 8, tol=1e-9)
    union_tda = np.sort(np.concatenate([res[2][0], res[0][0]]))[:8]
    assert np.allclose(om_u.cpu().numpy(), union_tda, atol=1e-8)
    om_r, _, _ = ctx.tdhf_excitations(cu, bu, du, 8, tol=1e-9)
    union_rpa = np.sort(np.concatenate([res[2][1], res[0][1]]))[:8]
    assert np.allclose(om_r.cpu().numpy(), union_rpa, atol=1e-8)
