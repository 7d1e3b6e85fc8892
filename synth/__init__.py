"""Seeded synthetic inputs shared by the oracle checks, the GPU parity tests and the benchmark.

This module holds no arithmetic of the exchange / ACE / TDA method: it only builds orbitals
and test vectors on the grid.  The paper's molecules (pseudopotential calculations, Sec. 3.3
and 4) are not available, so synthetic Gaussian-orbital "molecules" stand in for them:

* every orbital is (c_s + c_p . (r - R)) exp(-alpha |r - R|^2) with its type drawn per
  orbital (s, or one of p_x, p_y, p_z), the coefficient drawn normal (complex normal for
  complex workloads), alpha uniform in a range and R an atom centre;
* the set is orthonormalised by modified Gram-Schmidt in float64, in index order, with the
  dV inner product; virtual orbitals are orthonormalised after, and against, the occupied;
* test vectors are i.i.d. complex normal per point, normalised in the dV inner product;
* lower precisions receive round-to-nearest-even copies of the same float64 arrays.

Workload presets follow the five configurations the benchmark and tests use (``C1`` ..
``C5``), with fixed seeds 101..105.
"""

from dataclasses import dataclass, field

import numpy as np


def coords(n, h):
    """Grid coordinates x_k = (k - (n-1)/2) h (box centred on the origin)."""
    return (np.arange(n, dtype=np.float64) - (n - 1) / 2.0) * h


def _gaussian(n, h, centre, alpha, kind, coef):
    x = coords(n, h)
    dx = (x - centre[0])[:, None, None]
    dy = (x - centre[1])[None, :, None]
    dz = (x - centre[2])[None, None, :]
    env = np.exp(-alpha * (dx * dx + dy * dy + dz * dz))
    if kind == 0:
        poly = 1.0
    else:
        poly = (dx, dy, dz)[kind - 1]
    return coef * poly * env


def mgs(vectors, dv, against=None):
    """Modified Gram-Schmidt in float64, in index order, with the dV inner product."""
    out = []
    basis = [] if against is None else [np.asarray(a) for a in against]
    for v in vectors:
        w = np.array(v, dtype=np.result_type(v.dtype, np.float64), copy=True)
        for q in basis + out:
            w = w - q * (np.vdot(q, w) * dv)
        nrm = np.sqrt(np.real(np.vdot(w, w)) * dv)
        out.append(w / nrm)
    return np.stack(out) if out else np.zeros((0,) + tuple(vectors.shape[1:]))


def gaussian_orbitals(rng, n_grid, h, count, alpha_range, centres, complex_valued,
                      centre_of=None, against=None):
    """``count`` orthonormalised s/p Gaussian orbitals on an n_grid^3 box (float64/complex128)."""
    raw = []
    for k in range(count):
        kind = int(rng.integers(0, 4))
        alpha = float(rng.uniform(*alpha_range))
        c = centres[k % len(centres)] if centre_of is None else centre_of(k)
        if complex_valued:
            coef = complex(rng.normal(), rng.normal())
        else:
            coef = float(rng.normal())
        raw.append(_gaussian(n_grid, h, c, alpha, kind, coef))
    raw = np.stack(raw)
    return mgs(raw, h ** 3, against=against)


def random_vectors(rng, n_grid, h, count):
    """i.i.d. complex normal vectors per point, normalised in the dV inner product."""
    shape = (count, n_grid, n_grid, n_grid)
    v = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    nrm = np.sqrt(np.sum(np.abs(v) ** 2, axis=(1, 2, 3)) * h ** 3)
    return v / nrm[:, None, None, None]


@dataclass
class Molecule:
    n: int                     # box edge in points (padded edge is 2n)
    h: float                   # spacing, bohr
    phi: np.ndarray            # (n_occ, n, n, n) float64 or complex128
    psi: np.ndarray = None     # (n_vec, n, n, n) complex128 test vectors, or None
    phi_virt: np.ndarray = None
    eps_occ: np.ndarray = None
    eps_virt: np.ndarray = None
    meta: dict = field(default_factory=dict)


def config1(seed=101):
    """Box 32^3, h 0.3, 2 complex s/p orbitals (alpha 0.5-2.0, centres within +-1.5), 4 vectors."""
    rng = np.random.default_rng(seed)
    n, h = 32, 0.3
    centres = [rng.uniform(-1.5, 1.5, size=3) for _ in range(2)]
    phi = gaussian_orbitals(rng, n, h, 2, (0.5, 2.0), centres, True)
    psi = random_vectors(rng, n, h, 4)
    return Molecule(n, h, phi, psi, meta={"name": "C1"})


def config2(seed=102):
    """Box 48^3, h 0.25, 8 complex orbitals on 4 atoms within 2 bohr (alpha 0.3-3.0), 32 vectors."""
    rng = np.random.default_rng(seed)
    n, h = 48, 0.25
    atoms = [rng.uniform(-2.0, 2.0, size=3) for _ in range(4)]
    phi = gaussian_orbitals(rng, n, h, 8, (0.3, 3.0), atoms, True)
    psi = random_vectors(rng, n, h, 32)
    return Molecule(n, h, phi, psi, meta={"name": "C2"})


def config3(seed=103, n=64, h=0.2, n_occ=16, n_virt=32):
    """Box 64^3, h 0.2, 16 occupied + 32 more diffuse virtual real orbitals, orbital energies."""
    rng = np.random.default_rng(seed)
    atoms = [rng.uniform(-2.0, 2.0, size=3) for _ in range(4)]
    occ = gaussian_orbitals(rng, n, h, n_occ, (0.5, 4.0), atoms, False)
    virt = gaussian_orbitals(rng, n, h, n_virt, (0.1, 0.5), atoms, False, against=list(occ))
    eps_occ = np.sort(rng.uniform(-1.5, -1.0, size=n_occ))
    eps_virt = np.sort(rng.uniform(0.0, 0.5, size=n_virt))
    return Molecule(n, h, occ, None, virt, eps_occ, eps_virt, meta={"name": "C3"})


C4_EDGES = (32, 40, 48, 56, 64)


def config4(seed=104, count=64, edges=C4_EDGES, h=0.25, n_range=(2, 16)):
    """64 independent molecules: edge uniform over ``edges``, occupied count uniform 2-16."""
    rng = np.random.default_rng(seed)
    mols = []
    for m in range(count):
        n = int(rng.choice(edges))
        k = int(rng.integers(n_range[0], n_range[1] + 1))
        atoms = [rng.uniform(-2.0, 2.0, size=3) for _ in range(4)]
        phi = gaussian_orbitals(rng, n, h, k, (0.3, 3.0), atoms, True)
        mols.append(Molecule(n, h, phi, meta={"name": "C4[%d]" % m}))
    return mols


def to_precision(a, single):
    """Round-to-nearest-even copy in float32 / complex64 when ``single``, else float64 copy."""
    if not single:
        return np.ascontiguousarray(a)
    if np.iscomplexobj(a):
        return np.ascontiguousarray(a.astype(np.complex64))
    return np.ascontiguousarray(a.astype(np.float32))


def small_complex(seed, n, h, count, nvec=0):
    """A small complex system for parity tests at sizes the oracle finishes quickly."""
    rng = np.random.default_rng(seed)
    span = 0.25 * n * h
    atoms = [rng.uniform(-span, span, size=3) for _ in range(3)]
    phi = gaussian_orbitals(rng, n, h, count, (0.5, 2.5), atoms, True)
    psi = random_vectors(rng, n, h, nvec) if nvec else None
    return Molecule(n, h, phi, psi)


def small_real(seed, n, h, n_occ, n_virt):
    """A small real occupied + virtual system (TDA parity at oracle-friendly sizes)."""
    rng = np.random.default_rng(seed)
    span = 0.25 * n * h
    atoms = [rng.uniform(-span, span, size=3) for _ in range(3)]
    occ = gaussian_orbitals(rng, n, h, n_occ, (0.6, 3.0), atoms, False)
    virt = gaussian_orbitals(rng, n, h, n_virt, (0.2, 0.8), atoms, False, against=list(occ))
    eps_occ = np.sort(rng.uniform(-1.5, -1.0, size=n_occ))
    eps_virt = np.sort(rng.uniform(0.0, 0.5, size=n_virt))
    return Molecule(n, h, occ, None, virt, eps_occ, eps_virt)


# ---- synthetic closed-shell systems for the SCF (no pseudopotentials are available) ----------

@dataclass
class ScfSystem:
    n: int
    h: float
    centres: np.ndarray        # (atoms, 3) bohr
    charges: np.ndarray        # (atoms,)
    sigma: float               # smearing length of the soft nuclei, bohr
    v_ext: np.ndarray          # (n, n, n) float64 local potential
    guess: np.ndarray          # (k, n, n, n) float64 orthonormal starting orbitals
    meta: dict = field(default_factory=dict)


def soft_coulomb(n, h, centres, charges, sigma):
    """V(r) = -sum_A Z_A erf(|r - R_A| / sigma) / |r - R_A|, the value -2 Z_A / (sigma sqrt pi)
    at r = R_A: the synthetic nuclei of the SCF inputs."""
    from scipy.special import erf
    x = coords(n, h)
    v = np.zeros((n, n, n))
    for c, z in zip(centres, charges):
        r = np.sqrt((x - c[0])[:, None, None] ** 2 + (x - c[1])[None, :, None] ** 2
                    + (x - c[2])[None, None, :] ** 2)
        with np.errstate(invalid="ignore", divide="ignore"):
            val = erf(r / sigma) / r
        val[r == 0] = 2.0 / (sigma * np.sqrt(np.pi))
        v -= z * val
    return v


def scf_system(seed, n, h, k, centres=None, charges=None, n_atoms=4, sigma=0.6, span=None,
               min_sep=1.2):
    """A neutral closed-shell system with k doubly occupied orbitals: soft nuclei (charges
    summing to 2k) and a Gaussian s/p starting guess centred on them (orthonormalised)."""
    rng = np.random.default_rng(seed)
    if centres is None:
        span = 0.18 * n * h if span is None else span
        pts = []
        while len(pts) < n_atoms:
            p = rng.uniform(-span, span, size=3)
            if all(np.linalg.norm(p - q) >= min_sep for q in pts):
                pts.append(p)
        centres = np.array(pts)
        base = np.full(n_atoms, (2 * k) // n_atoms, dtype=float)
        base[: (2 * k) % n_atoms] += 1.0
        charges = base
    centres = np.asarray(centres, dtype=float)
    charges = np.asarray(charges, dtype=float)
    v = soft_coulomb(n, h, centres, charges, sigma)
    guess = gaussian_orbitals(rng, n, h, k, (0.6, 1.5), list(centres), False)
    return ScfSystem(n, h, centres, charges, sigma, v, guess)


def scf_small(seed=201):
    """16^3, h 0.4: two soft nuclei of charge 3 (4 electrons, 2 orbitals)."""
    return scf_system(seed, 16, 0.4, 2, centres=[(-0.6, 0.0, 0.0), (0.6, 0.2, 0.0)],
                      charges=[3.0, 3.0], sigma=0.8)


def config5(seed=105, n=64, h=0.2, k=16, n_atoms=8):
    """64^3, h 0.2, 16 doubly occupied orbitals on 8 soft nuclei of charge 4 (C5)."""
    s = scf_system(seed, n, h, k, n_atoms=n_atoms, sigma=0.5, span=2.6, min_sep=1.6)
    s.meta["name"] = "C5"
    return s
