"""Two-electron integrals and the RHF Tamm-Dancoff matrix.  TEST INFRASTRUCTURE ONLY.

Paper: Sec. 2 -- the two-electron integral (pq|rs) (definition after Eq. (5)), the RHF
matrix A of Eq. (7) with delta_M = 2 (singlet) / 0 (triplet), the Tamm-Dancoff problem
A X = omega X, the independent-particle excitations eps_a - eps_i, transition dipoles
Eq. (8), oscillator strengths Eq. (9) and the strength function Eq. (10).

Readings:

* On the grid, (pq|rs) = dV sum_r conj(phi_r) phi_s (r) * v[conj(phi_p) phi_q](r) with v the
  isolated Poisson solve of ``oracle.poisson``.
* The coupling block C = A - diag(eps_a - eps_i) is C_{ia,jb} = delta_M (ai|jb) - (ab|ji);
  row / column index ia = i * n_virt + a.
* Oscillator strength in atomic units (m_e = hbar = 1): f = 2/3 omega |d|^2, with d taken
  from the TDA eigenvector as printed in Eq. (8) (no extra spin factor; the paper does not
  state one).
* Strength function: each delta of Eq. (10) broadened by a normalised Lorentzian of
  half-width gamma.

Full TDHF (Eq. (3)): the RHF B block (spin-adapted from Eq. (5): singlet
B = 2 (ia|bj) - (ib|aj), triplet B = -(ib|aj), i.e. B_{ia,jb} = delta_M (ia|bj) - (ib|aj)),
the UHF blocks of Eqs. (4)-(5) with (pq||rs) = (pq|rs) - (pr|qs) over spin orbitals, and the
positive eigenvalues of the non-Hermitian problem of Eq. (3).

Pinned by (tests/test_oracle_tda.py): brute-force double sums for single integrals on tiny
grids, the 8-fold symmetry of real integrals, Hermiticity of C, singlet - triplet =
2 (ai|jb), diagonal integrals against the Gaussian closed form; the one-transition closed
form omega = sqrt(A^2 - B^2), B = 0 giving the Tamm-Dancoff eigenvalues, agreement with the
Hermitian half-size form (A-B)^{1/2} (A+B) (A-B)^{1/2} for real orbitals, and the closed-shell
UHF spectrum being the union of the RHF singlet and triplet spectra (TDA and full TDHF).
Transition dipoles and oscillator strengths (Eqs. (8)-(9)): harmonic-oscillator eigenstates
sampled on the grid, whose matrix elements <0|x|1> = 1/sqrt(2 w) and <1|x|2> = 1/sqrt(w) are
closed forms, give f = 1/3 per axis from the ground state (summing to 1, the Thomas-Reiche-
Kuhn rule for one electron), with two occupied orbitals so that the ia layout matters.
"""

import scipy.linalg

import numpy as np

from . import poisson


def integral(phi_p, phi_q, phi_r, phi_s, h, khat=None):
    """(pq|rs) on the grid."""
    v = poisson.fft(np.conj(phi_p) * phi_q, h, khat)
    return complex(np.sum(np.conj(phi_r) * phi_s * v) * h ** 3)


def coupling_block(phi_occ, phi_virt, h, delta_m, khat=None):
    """C_{ia,jb} = delta_M (ai|jb) - (ab|ji) for all i, j occupied and a, b virtual (Eq. (7)).

    Computed from one Poisson solve per (a, i) and per (a, b) pair.
    """
    no, nv = phi_occ.shape[0], phi_virt.shape[0]
    n = phi_occ.shape[1]
    if khat is None:
        khat = poisson.kernel_hat(n, h)
    dv = h ** 3
    po = phi_occ.reshape(no, -1)
    pv = phi_virt.reshape(nv, -1)
    # (ai|jb) = dV sum_r conj(phi_j) phi_b v_ai ;  v_ai = G (*) conj(phi_a) phi_i
    ex = np.zeros((no, nv, no, nv), dtype=np.complex128)
    for a in range(nv):
        for i in range(no):
            v = poisson.fft(np.conj(phi_virt[a]) * phi_occ[i], h, khat).reshape(-1)
            # rows j, cols b: sum_r conj(phi_j(r)) phi_b(r) v(r)
            ex[i, a] = dv * ((np.conj(po) * v[None, :]) @ pv.T)
    # (ab|ji) = dV sum_r conj(phi_j) phi_i v_ab ;  v_ab = G (*) conj(phi_a) phi_b
    co = np.zeros((no, nv, no, nv), dtype=np.complex128)
    for a in range(nv):
        for b in range(nv):
            v = poisson.fft(np.conj(phi_virt[a]) * phi_virt[b], h, khat).reshape(-1)
            co[:, a, :, b] = (dv * ((np.conj(po) * v[None, :]) @ po.T)).T   # [i, j]
    c = delta_m * ex - co
    c = c.reshape(no * nv, no * nv)
    if not (np.iscomplexobj(phi_occ) or np.iscomplexobj(phi_virt)):
        c = c.real
    return c


def _pair_potentials(left, right, h, khat):
    """v[p][q] = G (*) conj(left_p) right_q for every pair, flattened volumes."""
    return np.stack([np.stack([poisson.fft(np.conj(lp) * rq, h, khat).reshape(-1)
                               for rq in right]) for lp in left])


def b_block(phi_occ, phi_virt, h, delta_m, khat=None):
    """RHF B_{ia,jb} = delta_M (ia|bj) - (ib|aj) (Eq. (3), spin-adapted Eq. (5))."""
    no, nv = phi_occ.shape[0], phi_virt.shape[0]
    if khat is None:
        khat = poisson.kernel_hat(phi_occ.shape[1], h)
    dv = h ** 3
    po = phi_occ.reshape(no, -1)
    pv = phi_virt.reshape(nv, -1)
    v_ia = _pair_potentials(phi_occ, phi_virt, h, khat)          # G (*) conj(phi_i) phi_a
    # (ia|bj) = dV sum_r conj(phi_b) phi_j v_ia ; (ib|aj) = dV sum_r conj(phi_a) phi_j v_ib
    t1 = dv * np.einsum("iar,br,jr->iajb", v_ia, np.conj(pv), po)
    t2 = dv * np.einsum("ibr,ar,jr->iajb", v_ia, np.conj(pv), po)
    b = (delta_m * t1 - t2).reshape(no * nv, no * nv)
    if not (np.iscomplexobj(phi_occ) or np.iscomplexobj(phi_virt)):
        b = b.real
    return b


def uhf_blocks(occ_a, virt_a, occ_b, virt_b, h, khat=None):
    """UHF A - diag(eps_a - eps_i) and B over spin orbitals (Eqs. (4), (5)):
    (ia||jb) = (ia|jb) - (ij|ab), (ia||bj) = (ia|bj) - (ib|aj), the second terms only between
    transitions of the same spin.  Index: alpha transitions i*nv_a + a first, then beta."""
    if khat is None:
        khat = poisson.kernel_hat(occ_a.shape[1], h)
    dv = h ** 3
    spins = [(occ_a, virt_a), (occ_b, virt_b)]
    sizes = [o.shape[0] * v.shape[0] for o, v in spins]
    off = [0, sizes[0]]
    n = sum(sizes)
    cplx = any(np.iscomplexobj(x) for x in (occ_a, virt_a, occ_b, virt_b))
    a_m = np.zeros((n, n), dtype=np.complex128)
    b_m = np.zeros((n, n), dtype=np.complex128)
    for s, (os_, vs) in enumerate(spins):
        v_ia = _pair_potentials(os_, vs, h, khat)                     # [i][a] G (*) conj(i) a
        v_ij = _pair_potentials(os_, os_, h, khat)                    # [i][j] G (*) conj(i) j
        for t, (ot, vt) in enumerate(spins):
            po_t = ot.reshape(ot.shape[0], -1)
            pv_t = vt.reshape(vt.shape[0], -1)
            coul = dv * np.einsum("iar,jr,br->iajb", v_ia, np.conj(po_t), pv_t)  # (ia|jb)
            bcou = dv * np.einsum("iar,br,jr->iajb", v_ia, np.conj(pv_t), po_t)  # (ia|bj)
            blk_a, blk_b = coul, bcou
            if s == t:
                pv_s = vs.reshape(vs.shape[0], -1)
                po_s = os_.reshape(os_.shape[0], -1)
                exa = dv * np.einsum("ijr,ar,br->iajb", v_ij, np.conj(pv_s), pv_s)  # (ij|ab)
                v_ib = v_ia
                exb = dv * np.einsum("ibr,ar,jr->iajb", v_ib, np.conj(pv_s), po_s)  # (ib|aj)
                blk_a = coul - exa
                blk_b = bcou - exb
            ns, nt = sizes[s], sizes[t]
            a_m[off[s]:off[s] + ns, off[t]:off[t] + nt] = blk_a.reshape(ns, nt)
            b_m[off[s]:off[s] + ns, off[t]:off[t] + nt] = blk_b.reshape(ns, nt)
    if not cplx:
        a_m, b_m = a_m.real, b_m.real
    return a_m, b_m


def rpa_excitations(a_matrix, b_matrix):
    """Positive eigenvalues omega of Eq. (3): [[A, B], [B*, A*]] z = omega diag(1, -1) z,
    i.e. of [[A, B], [-B*, -A*]]; ascending."""
    n = a_matrix.shape[0]
    big = np.block([[a_matrix, b_matrix], [-np.conj(b_matrix), -np.conj(a_matrix)]])
    w = np.linalg.eigvals(big)
    w = np.sort(w.real[w.real > 0])
    return w[:n]


def rpa_hermitian(a_matrix, b_matrix):
    """For real A, B with A - B positive definite: omega^2 are the eigenvalues of
    (A - B)^{1/2} (A + B) (A - B)^{1/2} (the half-size Hermitian form of Sec. 2)."""
    s = scipy.linalg.sqrtm(a_matrix - b_matrix).real
    return np.sqrt(np.linalg.eigvalsh(s @ (a_matrix + b_matrix) @ s))


def coupling_element(phi_occ, phi_virt, h, delta_m, i, a, j, b, khat=None):
    """One entry C_{ia,jb} = delta_M (ai|jb) - (ab|ji), from two Poisson solves."""
    ex = integral(phi_virt[a], phi_occ[i], phi_occ[j], phi_virt[b], h, khat)
    co = integral(phi_virt[a], phi_virt[b], phi_occ[j], phi_occ[i], h, khat)
    return delta_m * ex - co


def tda_matrix(coupling, eps_occ, eps_virt):
    """A = diag(eps_a - eps_i) + C (Eq. (7)); index ia = i * n_virt + a."""
    de = (np.asarray(eps_virt)[None, :] - np.asarray(eps_occ)[:, None]).reshape(-1)
    return np.diag(de) + coupling


def excitations(a_matrix):
    """Tamm-Dancoff A X = omega X (Hermitian): eigenvalues ascending and eigenvectors."""
    return np.linalg.eigh(a_matrix)


def ipa_excitations(eps_occ, eps_virt):
    """Independent-particle excitations eps_a - eps_i, sorted."""
    return np.sort((np.asarray(eps_virt)[None, :] - np.asarray(eps_occ)[:, None]).reshape(-1))


def dipole_elements(phi_occ, phi_virt, h, coords):
    """<i| r |a> for each Cartesian direction: array (3, n_occ, n_virt)."""
    no, nv = phi_occ.shape[0], phi_virt.shape[0]
    po = phi_occ.reshape(no, -1)
    pv = phi_virt.reshape(nv, -1)
    out = []
    for c in coords:
        out.append(h ** 3 * ((np.conj(po) * c.reshape(-1)[None, :]) @ pv.T))
    return np.stack(out)


def oscillator_strengths(omega, x, dip):
    """d_k = sum_ia <i|r|a> x_{k,ia} (Eq. (8)); f_k = 2/3 omega_k |d_k|^2 (Eq. (9))."""
    d = dip.reshape(3, -1) @ x          # (3, n_states): column k is d_k
    return 2.0 / 3.0 * omega * np.sum(np.abs(d) ** 2, axis=0)


def strength_function(omega_grid, omega, f, gamma):
    """S(w) = sum_k f_k L(w - omega_k), L a normalised Lorentzian of half-width gamma (Eq. (10))."""
    w = np.asarray(omega_grid)[:, None]
    lor = (gamma / np.pi) / ((w - omega[None, :]) ** 2 + gamma ** 2)
    return lor @ f
