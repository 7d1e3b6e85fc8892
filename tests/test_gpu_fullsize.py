"""GPU parity at the full sizes of the benchmark workloads, against the FP64 oracle.

* Box edges 32, 40 and 56 (P = 64, 80, 112: radices 2, 5 and 7, and the 512-thread z-forward
  pass of edge 56) for single pair solves and an ACE build.
* The whole 512 x 512 singlet coupling block of the 64^3 workload (16 occupied + 32 virtual
  real orbitals) element by element, and every eigenvalue of A = diag(eps_a - eps_i) + C, against
  values the oracle wrote (tests/golden/make_c3_golden.py).
* Every one of the 64 systems of the uneven batch (edges 32-64, 2-16 complex orbitals) against
  the oracle's E_x, M and sampled xi (tests/golden/make_c4_golden.py).
* FP64 storage at edges 56 and 64 (the rows-and-strips XY pass) and the energy terms of the
  64^3 SCF workload.

Bars: FP32 storage -- E_x within 1e-6 Ha, TDA eigenvalues within 1e-4 eV (the targets of the
mixed-precision path), single results 2e-5 relative (an FP32 FFT convolution of length-P
transforms carries about 1e-6); FP64 storage -- 1e-10 relative.
"""

import json
import os

import numpy as np
import pytest
import torch

import synth
from oracle import exchange, poisson, tda

pytestmark = pytest.mark.gpu

DEV = "cuda"
HA_TO_EV = 27.211386
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _ace():
    import paper_2405_01522_amd as ace
    return ace


def _t(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("n", [32, 40, 56])
def test_pair_poisson_fp32_large_edges(n):
    ace = _ace()
    rng = np.random.default_rng(300 + n)
    h = 0.25
    a = rng.normal(size=(2, n, n, n)) + 1j * rng.normal(size=(2, n, n, n))
    ctx = ace.AceContext(n, h, torch.complex64)
    pairs = [[0, 1], [1, 1], [1, 0]]
    v = ctx.pair_poisson_batched(_t(a, torch.complex64), _t(a, torch.complex64),
                                 pairs).cpu().numpy()
    for p, (j, i) in enumerate(pairs):
        ref = poisson.fft(np.conj(a[j]) * a[i], 0.25)
        assert _rel(v[p], ref) < 2e-5, (n, p, _rel(v[p], ref))
    ctx.close()


@pytest.mark.parametrize("n", [56, 64])
def test_pair_poisson_fp64_strip_edges(n):
    """FP64 at edges 56 and 64, whose P x P plane exceeds the LDS: the XY pass keeps the N
    y-transformed rows and runs the x transforms over column strips."""
    ace = _ace()
    rng = np.random.default_rng(400 + n)
    a = rng.normal(size=(2, n, n, n)) + 1j * rng.normal(size=(2, n, n, n))
    ctx = ace.AceContext(n, 0.25, torch.complex128)
    pairs = [[0, 1], [1, 1]]
    v = ctx.pair_poisson_batched(_t(a, torch.complex128), _t(a, torch.complex128),
                                 pairs).cpu().numpy()
    for p, (j, i) in enumerate(pairs):
        ref = poisson.fft(np.conj(a[j]) * a[i], 0.25)
        assert _rel(v[p], ref) < 1e-12, (n, p, _rel(v[p], ref))
    ctx.close()


@pytest.mark.parametrize("n", [56, 64])
def test_ace_build_fp64_strip_edges(n):
    ace = _ace()
    m = synth.small_complex(600 + n, n, 0.25, 3, nvec=2)
    ctx = ace.AceContext(m.n, m.h, torch.complex128)
    xi, mm, ex = ctx.ace_build(_t(m.phi, torch.complex128))
    kpsi = ctx.ace_apply(xi, _t(m.psi, torch.complex128)).cpu().numpy()
    assert ctx.status()[0] == 0
    xi_o, m_o, _, ex_o = exchange.ace_build(m.phi, m.h)
    assert abs(float(ex.cpu()) - ex_o) < 1e-10 * abs(ex_o)
    assert _rel(mm.cpu().numpy(), m_o) < 1e-10
    assert _rel(xi.cpu().numpy(), xi_o) < 1e-10
    assert _rel(kpsi, exchange.ace_apply(xi_o, m.psi, m.h)) < 1e-10
    ctx.close()


@pytest.mark.parametrize("n", [40, 56])
def test_ace_build_and_apply_fp32_large_edges(n):
    """ACE build + apply with FP32 storage at edges whose padded FFTs use radices 5 and 7."""
    ace = _ace()
    m = synth.small_complex(500 + n, n, 0.25, 3, nvec=2)
    ctx = ace.AceContext(m.n, m.h, torch.complex64)
    phi = _t(synth.to_precision(m.phi, True), torch.complex64)
    psi = _t(synth.to_precision(m.psi, True), torch.complex64)
    xi, mm, ex = ctx.ace_build(phi)
    kpsi = ctx.ace_apply(xi, psi).cpu().numpy()
    st, info = ctx.status()
    assert st == 0, (st, info)
    xi_o, m_o, _, ex_o = exchange.ace_build(m.phi, m.h)
    assert abs(float(ex.cpu()) - ex_o) < 1e-6
    assert _rel(mm.cpu().numpy(), m_o) < 2e-6
    assert _rel(xi.cpu().numpy(), xi_o) < 2e-5
    assert _rel(kpsi, exchange.ace_apply(xi_o, m.psi, m.h)) < 2e-5
    ctx.close()


@pytest.fixture(scope="module")
def c3_golden():
    c = np.load(os.path.join(GOLDEN, "c3_coupling_singlet.npy"), allow_pickle=False)
    with open(os.path.join(GOLDEN, "c3_eigen.json")) as f:
        meta = json.load(f)
    return c, meta


def test_config3_full_coupling_block_and_eigenvalues(c3_golden):
    """The singlet coupling block of the 64^3 workload from the GPU (FP32 storage, split-BF16
    MFMA contractions with FP64 split-K sums) against the oracle's block, every element, and
    every TDA eigenvalue within 1e-4 eV."""
    ref, meta = c3_golden
    ace = _ace()
    c3 = synth.config3()
    assert (meta["n"], meta["n_occ"], meta["n_virt"]) == (c3.n, 16, 32)
    ctx = ace.AceContext(c3.n, c3.h, torch.float32)
    occ = _t(synth.to_precision(c3.phi, True), torch.float32)
    virt = _t(synth.to_precision(c3.phi_virt, True), torch.float32)
    c = ctx.tda_coupling(occ, virt, 2).cpu().numpy()
    ctx.close()
    scale = float(np.max(np.abs(ref)))
    err = float(np.max(np.abs(c - ref)))
    assert err < 2e-6 * scale, (err, scale)
    w, _ = tda.excitations(tda.tda_matrix(c, c3.eps_occ, c3.eps_virt))
    w_ref = np.asarray(meta["eigenvalues_ha"])
    err_ev = float(np.max(np.abs(w - w_ref))) * HA_TO_EV
    assert err_ev < 1e-4, err_ev


@pytest.fixture(scope="module")
def c4_golden():
    with open(os.path.join(GOLDEN, "c4_ace.json")) as f:
        return json.load(f)["systems"]


def _check_c4_system(g, sysd, tol_ex, tol_rel):
    ex = float(sysd["ex"].cpu())
    assert abs(ex - g["ex"]) < tol_ex, (g["index"], ex, g["ex"])
    m_ref = np.asarray(g["m_re"]) + 1j * np.asarray(g["m_im"])
    assert _rel(sysd["M"].cpu().numpy(), m_ref) < tol_rel, g["index"]
    xi = sysd["xi"].cpu().numpy().reshape(g["norb"], -1)
    xs_ref = np.asarray(g["xi_re"]) + 1j * np.asarray(g["xi_im"])
    xs = xi[:, g["points"]]
    scale = np.max(np.abs(xi), axis=1)[:, None]
    assert np.max(np.abs(xs - xs_ref) / scale) < tol_rel, g["index"]


def test_config4_every_system_vs_oracle(c4_golden):
    """The uneven 64-system batch (FP32 storage) in one call: every system's E_x within 1e-6 Ha
    of the oracle, M and sampled xi within 2e-5 relative; every box edge 32-64 is covered."""
    ace = _ace()
    c4 = synth.config4()
    assert len(c4_golden) == len(c4)
    dt = torch.complex64
    systems = [{"h": m.h, "phi": _t(synth.to_precision(m.phi, True), dt)} for m in c4]
    b = ace.AceBatch(dt)
    b.build(systems)
    st, mol, info = b.status()
    assert st == 0, (st, mol, info)
    edges = set()
    for m, g, sysd in zip(c4, c4_golden, systems):
        assert (g["n"], g["norb"]) == (m.n, m.phi.shape[0])
        _check_c4_system(g, sysd, 1e-6, 2e-5)
        edges.add(m.n)
    assert edges == set(synth.C4_EDGES)
    b.close()


def test_config4_every_system_fp64_vs_oracle(c4_golden):
    """The same 64-system batch with FP64 storage (every edge, 56 and 64 through the column-strip
    XY pass): every system's E_x, M and sampled xi within 1e-10 relative of the oracle."""
    ace = _ace()
    c4 = synth.config4()
    dt = torch.complex128
    systems = [{"h": m.h, "phi": _t(m.phi, dt)} for m in c4]
    b = ace.AceBatch(dt)
    b.build(systems)
    st, mol, info = b.status()
    assert st == 0, (st, mol, info)
    for g, sysd in zip(c4_golden, systems):
        _check_c4_system(g, sysd, 1e-10 * abs(g["ex"]), 1e-10)
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config5_energy_terms_vs_oracle(prec):
    """The SCF energy terms of the 64^3 workload (16 doubly occupied orbitals, 8 soft nuclei):
    kinetic (fourth-order differences), external, Hartree (the Poisson solve of the density)
    and exchange (ACE over the 16 orbitals, 136 pair solves at P = 128), each against the
    oracle's on the same orbitals -- FP64 storage to 1e-10 relative; FP32 storage to the unit
    roundoff of FP32 relative to the term (each term is an FP64 sum of products of FP32 grid
    values, each rounded once) plus 1e-7 Ha."""
    ace = _ace()
    from oracle import scf as oscf
    s = synth.config5()
    single = prec == "fp32"
    dt = torch.float32 if single else torch.float64
    phi = synth.to_precision(s.guess, single)
    ctx = ace.AceContext(s.n, s.h, dt)
    got = ctx.scf_energies(_t(synth.to_precision(s.v_ext[None], single), dt), _t(phi, dt))
    ref = oscf.energies(phi.astype(np.float64), synth.to_precision(s.v_ext, single).astype(np.float64),
                        s.h, poisson.kernel_hat(s.n, s.h))
    for term in ("kinetic", "external", "hartree", "exchange", "total"):
        if single:
            tol = 2.0 ** -24 * abs(ref[term]) + 1e-7
            assert abs(got[term] - ref[term]) < tol, (term, got[term], ref[term])
        else:
            assert abs(got[term] - ref[term]) < 1e-10 * abs(ref[term]), (term, got[term], ref[term])
