"""The no-allocation form of the ACE application (ace_apply_noalloc): called through the C ABI,
its K psi equals ace_apply's bit for bit (same kernels and passes, its sums kept in the
library's static device scratch), on two calls in a row with the second smaller -- the
scratch keeps the first call's contents, which must not leak into the second."""

import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _t(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


@pytest.mark.parametrize("dt", [torch.complex128, torch.complex64, torch.float32])
def test_noalloc_apply_equals_apply(dt):
    import paper_2405_01522_amd as ace
    from paper_2405_01522_amd._lib import lib
    single = dt in (torch.complex64, torch.float32)
    m = synth.config2() if dt.is_complex else synth.small_real(19, 24, 0.3, 6, 1)
    if not dt.is_complex:
        m.psi = synth.random_vectors(np.random.default_rng(5), m.n, m.h, 40).real.copy()
    ctx = ace.AceContext(m.n, m.h, dt)
    phi = _t(synth.to_precision(m.phi, single), dt)
    psi = _t(synth.to_precision(m.psi, single), dt)
    xi, _, _ = ctx.ace_build(phi)
    torch.cuda.synchronize()
    # first call: every vector with every orbital; second call: fewer orbitals and vectors
    for n_orb, n_vec in ((phi.shape[0], psi.shape[0]), (max(1, phi.shape[0] // 2 - 1), 5)):
        x = xi[:n_orb].contiguous()
        p = psi[:n_vec].contiguous()
        ref = ctx.ace_apply(x, p)
        out = torch.full_like(p, float("nan"))
        ctx._sync_stream()
        rc = lib().ace_apply_noalloc(ctx._h, ctypes.c_void_p(x.data_ptr()), n_orb,
                                     ctypes.c_void_p(p.data_ptr()), n_vec,
                                     ctypes.c_void_p(out.data_ptr()))
        assert rc == 0, rc
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (dt, n_orb, n_vec)
        assert torch.isfinite(out).all()
    assert ctx.status()[0] == 0
    ctx.close()


def test_noalloc_rejects_bad_arguments():
    import paper_2405_01522_amd as ace
    from paper_2405_01522_amd._lib import lib
    ctx = ace.AceContext(12, 0.4, torch.complex64)
    assert lib().ace_apply_noalloc(ctx._h, None, 1, None, 1, None) == -1
    assert lib().ace_apply_noalloc(None, None, 1, None, 1, None) == -1
    ctx.close()
