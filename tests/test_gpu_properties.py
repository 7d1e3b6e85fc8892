"""Property tests over random shapes: the HIP path against the FP64 oracle for box edges,
orbital counts, spacings, storage types and pair lists drawn by hypothesis (derandomised, so
every run draws the same cases).  The bars are those of the fixed-case parity tests: 1e-10
relative for FP64 storage; for FP32 storage 2e-5 on a pair potential (one FFT convolution)
and 3e-6 on M and K psi (an FP64 Gram of FP32 volumes); E_x within 1e-6 Ha.
"""

import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, given, settings, strategies as st

import synth
from oracle import exchange, poisson

pytestmark = pytest.mark.gpu

DEV = "cuda"
EDGES = [8, 9, 10, 12, 15, 16, 20, 24]
DTYPES = {"c128": torch.complex128, "c64": torch.complex64,
          "r64": torch.float64, "r32": torch.float32}
SETTINGS = dict(deadline=None, derandomize=True, database=None,
                suppress_health_check=[HealthCheck.too_slow])


def _ace():
    import paper_2405_01522_amd as ace
    return ace


def _t(a, dtype):
    single = dtype in (torch.complex64, torch.float32)
    return torch.from_numpy(synth.to_precision(a, single)).to(DEV, dtype)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _orbitals(seed, n, h, count, cplx):
    rng = np.random.default_rng(seed)
    span = 0.2 * n * h
    atoms = [rng.uniform(-span, span, size=3) for _ in range(2)]
    return synth.gaussian_orbitals(rng, n, h, count, (0.6, 2.0), atoms, cplx)


@settings(max_examples=16, **SETTINGS)
@given(n=st.sampled_from(EDGES), count=st.integers(1, 7), kind=st.sampled_from(sorted(DTYPES)),
       h=st.floats(0.2, 0.5), seed=st.integers(0, 10 ** 6))
def test_ace_build_and_apply_random_shapes(n, count, kind, h, seed):
    ace = _ace()
    dt = DTYPES[kind]
    cplx = dt.is_complex
    phi = _orbitals(seed, n, h, count, cplx)
    ctx = ace.AceContext(n, h, dt)
    xi, m, ex = ctx.ace_build(_t(phi, dt))
    assert ctx.status() == (0, 0)
    phi_used = synth.to_precision(phi, dt in (torch.complex64, torch.float32)).astype(
        np.complex128 if cplx else np.float64)
    xr, mr, _, exr = exchange.ace_build(phi_used, h)
    fp64 = dt in (torch.complex128, torch.float64)
    tol = 1e-10 if fp64 else 3e-6
    assert _rel(m.cpu().numpy(), mr) < tol
    assert abs(ex.item() - exr) < (1e-10 * abs(exr) if fp64 else 1e-6)
    rng = np.random.default_rng(seed + 1)
    v = rng.normal(size=(2, n, n, n))
    if cplx:
        v = v + 1j * rng.normal(size=(2, n, n, n))
    got = ctx.ace_apply(xi, _t(v, dt)).cpu().numpy()
    v_used = synth.to_precision(v, not fp64).astype(np.complex128 if cplx else np.float64)
    ref = exchange.ace_apply(xr, v_used, h)
    assert _rel(got, ref) < tol


@settings(max_examples=16, **SETTINGS)
@given(n=st.sampled_from(EDGES), count=st.integers(1, 9), nv=st.integers(1, 9),
       kind=st.sampled_from(sorted(DTYPES)), h=st.floats(0.2, 0.5), seed=st.integers(0, 10 ** 6))
def test_ace_build_apply_random_shapes(n, count, nv, kind, h, seed):
    """The one-call build + update (merged launches for complex storage and up to 8 orbitals,
    the steps one after another otherwise): xi, M and E_x bit for bit as ace_build, K psi at
    the apply bar against the oracle."""
    ace = _ace()
    dt = DTYPES[kind]
    cplx = dt.is_complex
    phi = _orbitals(seed, n, h, count, cplx)
    rng = np.random.default_rng(seed + 2)
    v = rng.normal(size=(nv, n, n, n))
    if cplx:
        v = v + 1j * rng.normal(size=(nv, n, n, n))
    ctx = ace.AceContext(n, h, dt)
    tphi, tv = _t(phi, dt), _t(v, dt)
    xb, mb, eb = ctx.ace_build(tphi)
    xi, m, ex, kp = ctx.ace_build_apply(tphi, tv)
    assert ctx.status() == (0, 0)
    assert torch.equal(xi, xb) and torch.equal(m, mb) and torch.equal(ex, eb)
    fp64 = dt in (torch.complex128, torch.float64)
    phi_used = synth.to_precision(phi, not fp64).astype(np.complex128 if cplx else np.float64)
    v_used = synth.to_precision(v, not fp64).astype(np.complex128 if cplx else np.float64)
    xr, _, _, _ = exchange.ace_build(phi_used, h)
    ref = exchange.ace_apply(xr, v_used, h)
    assert _rel(kp.cpu().numpy(), ref) < (1e-10 if fp64 else 3e-6)


@settings(max_examples=12, **SETTINGS)
@given(n=st.sampled_from(EDGES), na=st.integers(1, 4), nb=st.integers(1, 4),
       npairs=st.integers(1, 7), kind=st.sampled_from(sorted(DTYPES)),
       on_device=st.booleans(), seed=st.integers(0, 10 ** 6))
def test_pair_poisson_random_lists(n, na, nb, npairs, kind, on_device, seed):
    ace = _ace()
    dt = DTYPES[kind]
    cplx = dt.is_complex
    rng = np.random.default_rng(seed)
    h = 0.3
    a = rng.normal(size=(na, n, n, n))
    b = rng.normal(size=(nb, n, n, n))
    if cplx:
        a = a + 1j * rng.normal(size=a.shape)
        b = b + 1j * rng.normal(size=b.shape)
    pairs = np.stack([rng.integers(0, na, npairs), rng.integers(0, nb, npairs)], 1).astype(np.int32)
    ctx = ace.AceContext(n, h, dt)
    plist = torch.from_numpy(pairs).to(DEV) if on_device else pairs
    v = ctx.pair_poisson_batched(_t(a, dt), _t(b, dt), plist).cpu().numpy()
    assert ctx.status() == (0, 0)
    fp64 = dt in (torch.complex128, torch.float64)
    au = synth.to_precision(a, not fp64)
    bu = synth.to_precision(b, not fp64)
    for p, (j, i) in enumerate(pairs):
        ref = poisson.fft(np.conj(au[j].astype(np.complex128)) * bu[i], h)
        if not cplx:
            ref = ref.real
        assert _rel(v[p], ref) < (1e-12 if fp64 else 2e-5), (p, j, i)


@settings(max_examples=6, **SETTINGS)
@given(edges=st.lists(st.sampled_from([8, 10, 12, 16, 20]), min_size=2, max_size=6),
       counts=st.lists(st.integers(1, 9), min_size=6, max_size=6),
       kind=st.sampled_from(["c64", "r64"]), seed=st.integers(0, 10 ** 6))
def test_batch_random_mix_equals_single_builds(edges, counts, kind, seed):
    """A random mix of box edges and orbital counts in one batched call gives the bits of the
    one-system builds, and the oracle's exchange energies."""
    ace = _ace()
    dt = DTYPES[kind]
    cplx = dt.is_complex
    batch = ace.AceBatch(dt)
    systems, single, refs = [], [], []
    for s, n in enumerate(edges):
        h = 0.3 + 0.02 * s
        phi = _orbitals(seed + s, n, h, counts[s], cplx)
        tphi = _t(phi, dt)
        systems.append({"h": h, "phi": tphi})
        ctx = ace.AceContext(n, h, dt)
        single.append(ctx.ace_build(tphi))
        phi_used = synth.to_precision(phi, kind == "c64").astype(np.complex128 if cplx else np.float64)
        refs.append(exchange.ace_build(phi_used, h)[3])
    batch.build(systems)
    assert batch.status()[0] == 0
    for s, sysd in enumerate(systems):
        xi, m, ex = single[s]
        assert torch.equal(sysd["xi"], xi) and torch.equal(sysd["M"], m)
        assert sysd["ex"].item() == ex.item()
        assert abs(ex.item() - refs[s]) < (1e-6 if kind == "c64" else 1e-10 * abs(refs[s]))
