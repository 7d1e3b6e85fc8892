"""Closed-shell Hartree-Fock SCF on the isolated grid.  TEST INFRASTRUCTURE ONLY.

Paper: the HF-Roothaan eigenproblem, Eq. (1); the exchange operator, Eq. (2); linear mixing,
Eq. (14) (applied to the states, the scheme the paper finds most robust); the relative density
error stop test, Eq. (15).  The paper's pseudopotentials and molecules are not available, so the
Hamiltonian uses these readings (the same ones the GPU driver uses):

* kinetic energy -1/2 Laplacian by fourth-order central differences on each axis,
  (-f(x-2h) + 16 f(x-h) - 30 f(x) + 16 f(x+h) - f(x+2h)) / (12 h^2), orbitals zero outside the box;
* a synthetic local potential V_ext(r) = -sum_A Z_A erf(|r - R_A| / sigma) / |r - R_A| (finite at
  the nuclei, -2 Z_A / (sigma sqrt(pi)) there);
* closed shell: n doubly occupied spatial orbitals, rho = 2 sum_i |phi_i|^2, Hartree potential
  v_H = dV G (*) rho (``oracle.poisson``), exchange K as in ``oracle.exchange`` (same-spin
  exchange between spatial orbitals);
* E = 2 sum_i <phi_i| T + V_ext |phi_i> + 1/2 int rho v_H + sum_i <phi_i|K|phi_i>.

The solver: each iteration diagonalises the Fock operator built from the current orbitals
(Lanczos, scipy ``eigsh``, from a fixed random start vector), rotates the new occupied set to the old one (orthogonal Procrustes,
so that states can be mixed), mixes q_{N+1} = alpha q_{N-1} + (1 - alpha) q_N, re-orthonormalises
(Loewdin) and stops when the relative density error (Eq. (15)) falls below ``tol``.

Pinned by tests/test_oracle_scf.py: the Laplacian of a Gaussian (analytic, O(h^4)), harmonic-
oscillator eigenvalues (closed form), the 2:1 Hartree / exchange ratio of one doubly occupied
orbital, and the self-consistency of the converged orbitals.
"""

import math

import numpy as np
import scipy.linalg
import scipy.sparse.linalg
import scipy.special

from . import exchange, grid, poisson

_FD = (-1.0 / 12.0, 4.0 / 3.0, -5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0)


def laplacian(f, h):
    """Fourth-order finite-difference Laplacian over the last three axes, zero outside the box."""
    out = np.zeros_like(f)
    n = f.shape[-1]
    lead = f.ndim - 3
    for ax in range(lead, f.ndim):
        shape = list(f.shape)
        shape[ax] = n + 4
        fp = np.zeros(shape, dtype=f.dtype)
        sl = [slice(None)] * f.ndim
        sl[ax] = slice(2, n + 2)
        fp[tuple(sl)] = f
        for k, c in enumerate(_FD):
            sk = [slice(None)] * f.ndim
            sk[ax] = slice(k, k + n)
            out += c * fp[tuple(sk)]
    return out / (h * h)


def kinetic(f, h):
    return -0.5 * laplacian(f, h)


def kinetic_diagonal(h):
    """Diagonal element of T: 1/2 * 3 axes * 5/2 / h^2."""
    return 0.5 * 3.0 * 2.5 / (h * h)


def kinetic_precondition(r, h, shift, sweeps, omega):
    """Approximate (T + shift)^{-1} r: z = r / (d + shift), then sweeps - 1 damped-Jacobi steps
    z <- z + omega (r - (T + shift) z) / (d + shift) (d = diagonal of T).  Not from the paper:
    the plain preconditioner the learned one is compared with."""
    d = kinetic_diagonal(h) + shift
    z = r / d
    for _ in range(sweeps - 1):
        z = z + omega * (r - (kinetic(z, h) + shift * z)) / d
    return z


def external_potential(n, h, centres, charges, sigma):
    x = grid.coords(n, h)
    v = np.zeros((n, n, n))
    for c, z in zip(centres, charges):
        r = np.sqrt((x - c[0])[:, None, None] ** 2 + (x - c[1])[None, :, None] ** 2
                    + (x - c[2])[None, None, :] ** 2)
        with np.errstate(invalid="ignore", divide="ignore"):
            val = scipy.special.erf(r / sigma) / r
        val[r == 0] = 2.0 / (sigma * math.sqrt(math.pi))
        v -= z * val
    return v


def density(phi):
    return 2.0 * np.sum(phi * phi, axis=0)


def fock_apply(psi, phi, v_local, h, khat, exchange_on=True):
    """F psi = T psi + v_local psi + K[phi] psi (v_local = V_ext + v_H)."""
    out = kinetic(psi, h) + v_local * psi
    if exchange_on and phi is not None and phi.shape[0]:
        if psi.ndim == 4:
            out = out + np.stack([exchange.apply_direct(phi, p, h, khat) for p in psi])
        else:
            out = out + exchange.apply_direct(phi, psi, h, khat)
    return out


def energies(phi, v_ext, h, khat):
    dv = h ** 3
    rho = density(phi)
    vh = poisson.fft(rho, h, khat)
    ekin = 2.0 * float(np.sum(phi * kinetic(phi, h)) * dv)
    eext = float(np.sum(rho * v_ext) * dv)
    eh = 0.5 * float(np.sum(rho * vh) * dv)
    ex = float(np.sum(phi * exchange.build_w(phi, h, khat)) * dv)
    return {"total": ekin + eext + eh + ex, "kinetic": ekin, "external": eext,
            "hartree": eh, "exchange": ex}


def lowest_states(apply, n, k, h, v0=None, tol=1e-12):
    """k lowest eigenpairs of a symmetric grid operator (dV-normalised vectors).

    Lanczos (ARPACK) for k + 3 values, the lowest k kept; a single-vector Krylov method can miss
    copies of an exactly degenerate eigenvalue, so the systems it is used on are asymmetric."""
    ng = n ** 3
    op = scipy.sparse.linalg.LinearOperator(
        (ng, ng), matvec=lambda v: apply(v.reshape(n, n, n)).reshape(-1), dtype=np.float64)
    w, vec = scipy.sparse.linalg.eigsh(op, k=k + 3, which="SA", tol=tol, v0=v0)
    order = np.argsort(w)[:k]
    vec = vec[:, order].T.reshape(k, n, n, n) / math.sqrt(h ** 3)
    return w[order], vec


def loewdin(phi, h):
    m = phi.reshape(phi.shape[0], -1)
    s = (m @ m.T) * h ** 3
    w, u = np.linalg.eigh(s)
    return ((u @ np.diag(w ** -0.5) @ u.T) @ m).reshape(phi.shape)


def scf(phi0, v_ext, h, alpha=0.3, tol=1e-9, max_iter=200):
    """Closed-shell HF SCF from orbitals phi0; returns (phi, energy dict, history)."""
    n = phi0.shape[1]
    k = phi0.shape[0]
    khat = poisson.kernel_hat(n, h)
    dv = h ** 3
    ne = 2.0 * k
    phi = loewdin(phi0, h)
    # Krylov start with no spatial symmetry (a symmetric start would confine Lanczos to one
    # symmetry sector of the Fock operator and could miss lower states of another)
    v0 = np.random.default_rng(12345).normal(size=n ** 3)
    hist = []
    for it in range(max_iter):
        rho_in = density(phi)
        vloc = v_ext + poisson.fft(rho_in, h, khat)
        w, new = lowest_states(lambda f: fock_apply(f, phi, vloc, h, khat), n, k, h, v0=v0)
        # rotate the new occupied set onto the old one (orthogonal Procrustes), then mix
        ov = (new.reshape(k, -1) @ phi.reshape(k, -1).T) * dv
        u, _, vt = np.linalg.svd(ov)
        rot = (u @ vt).T
        new = np.tensordot(rot, new, axes=1)
        rho_out = density(new)
        err = float(np.sum(np.abs(rho_out - rho_in)) * dv / ne)
        hist.append({"iter": it, "density_error": err, "eigenvalues": w})
        if err < tol:
            phi = new
            break
        phi = loewdin(alpha * phi + (1.0 - alpha) * new, h)
    return phi, energies(phi, v_ext, h, khat), hist
