"""Python binding of the libace C ABI (include/ace.h).

Argument marshalling only: tensors are checked (device, dtype, shape, contiguity), their data
pointers and the current HIP stream are passed to the library, and every step of the
computation runs in the library's kernels.  Function names follow the C entry points.

Orbital arrays are torch tensors on the GPU shaped (count, N, N, N), C-contiguous, of one of
complex128, complex64, float64, float32 (the context's storage type).
"""

import ctypes

import torch

from ._lib import (AceEigOpts, AceMol, AceScfOpts, AceScfResult, NET_PARAMS, PRECOND_KINETIC,
                   PRECOND_NET, PRECOND_NONE, TRAIN_RANDOM, check, lib)

ACE_C128, ACE_C64, ACE_R64, ACE_R32 = 0, 1, 2, 3
_DTYPES = {torch.complex128: ACE_C128, torch.complex64: ACE_C64,
           torch.float64: ACE_R64, torch.float32: ACE_R32}
_TORCH = {v: k for k, v in _DTYPES.items()}
MAX_ORBITALS = 64           # real orbitals
MAX_ORBITALS_COMPLEX = 32   # complex orbitals


def _device(device):
    """torch.device with an explicit GPU index (the current device when none is given)."""
    d = torch.device(device) if device is not None else torch.device("cuda")
    if d.type != "cuda":
        raise ValueError("device must be a GPU, got %s" % d)
    return d if d.index is not None else torch.device("cuda", torch.cuda.current_device())


def dtype_code(dtype):
    if dtype not in _DTYPES:
        raise TypeError("unsupported orbital dtype %s" % dtype)
    return _DTYPES[dtype]


def _stream_handle():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def check_out(t, name, shape, dtype, device):
    """Validate a caller-supplied result tensor before its pointer goes to the library (the C
    side cannot see its size or type): exact dtype and shape, contiguous, on the given GPU."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s has dtype %s, expected %s" % (name, t.dtype, dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.device != device:
        raise ValueError("%s is on %s, expected %s" % (name, t.device, device))
    return ctypes.c_void_p(t.data_ptr())


def size_supported(n, dtype):
    return bool(lib().ace_size_supported(int(n), dtype_code(dtype)))


class AceContext:
    """One box (N^3 points, spacing h) and one orbital storage type; owns the kernel spectrum
    and the library workspaces.  Calls run on torch's current stream."""

    def __init__(self, n, h, dtype, device=None):
        self.n = int(n)
        self.h = float(h)
        self.dtype = dtype
        self.code = dtype_code(dtype)
        self.device = _device(device)
        with torch.cuda.device(self.device):
            handle = ctypes.c_void_p()
            check(lib().ace_ctx_create(self.n, self.h, self.code, _stream_handle(),
                                       ctypes.byref(handle)), "ace_ctx_create")
        self._h = handle
        self._stream = torch.cuda.current_stream(self.device).cuda_stream

    # -- plumbing -----------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().ace_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        """Point the context at torch's current stream (a no-op when it is unchanged)."""
        cur = torch.cuda.current_stream(self.device).cuda_stream
        if cur != self._stream:
            check(lib().ace_ctx_set_stream(self._h, ctypes.c_void_p(cur)), "ace_ctx_set_stream")
            self._stream = cur

    def _vol(self, t, name, count=None):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("%s must be a CUDA/HIP tensor" % name)
        if t.device != self.device:
            raise ValueError("%s is on %s, the context on %s" % (name, t.device, self.device))
        if t.dtype != self.dtype:
            raise TypeError("%s has dtype %s, context expects %s" % (name, t.dtype, self.dtype))
        if t.dim() != 4 or tuple(t.shape[1:]) != (self.n,) * 3:
            raise ValueError("%s must be shaped (count, %d, %d, %d), got %s"
                             % (name, self.n, self.n, self.n, tuple(t.shape)))
        if count is not None and t.shape[0] != count:
            raise ValueError("%s must hold %d volumes" % (name, count))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        return ctypes.c_void_p(t.data_ptr())

    def _empty(self, count, dtype=None):
        return torch.empty((count, self.n, self.n, self.n), dtype=dtype or self.dtype,
                           device=self.device)

    # -- entry points ---------------------------------------------------------------------
    def pair_poisson_batched(self, phi_a, phi_b, pairs, out=None):
        """v[p] = G (*) (conj(phi_a[j]) phi_b[i]) for the pairs (j, i).  A pair list already on
        the context's device (int32, contiguous, shape (np, 2)) goes to
        pair_poisson_batched_dev and is not copied to the host."""
        if isinstance(pairs, torch.Tensor) and pairs.is_cuda:
            return self.pair_poisson_batched_dev(phi_a, phi_b, pairs, out)
        pr = torch.as_tensor(pairs, dtype=torch.int32).reshape(-1, 2).contiguous().cpu()
        np_ = pr.shape[0]
        if out is None:
            out = self._empty(np_)
        pa = self._vol(phi_a, "phi_a")
        pb = self._vol(phi_b, "phi_b")
        po = self._vol(out, "v_out", np_)
        self._sync_stream()
        ptr = ctypes.cast(pr.data_ptr(), ctypes.POINTER(ctypes.c_int32))
        check(lib().pair_poisson_batched(self._h, pa, phi_a.shape[0], pb, phi_b.shape[0], ptr,
                                         np_, po), "pair_poisson_batched")
        return out

    def pair_poisson_batched_dev(self, phi_a, phi_b, pairs, out=None):
        if not isinstance(pairs, torch.Tensor) or pairs.dtype != torch.int32 or \
                pairs.device != self.device or pairs.dim() != 2 or pairs.shape[1] != 2 or \
                not pairs.is_contiguous():
            raise ValueError("pairs must be a contiguous int32 (np, 2) tensor on %s" % self.device)
        np_ = pairs.shape[0]
        if out is None:
            out = self._empty(np_)
        pa = self._vol(phi_a, "phi_a")
        pb = self._vol(phi_b, "phi_b")
        po = self._vol(out, "v_out", np_)
        self._sync_stream()
        check(lib().pair_poisson_batched_dev(self._h, pa, phi_a.shape[0], pb, phi_b.shape[0],
                                             ctypes.c_void_p(pairs.data_ptr()), np_, po),
              "pair_poisson_batched_dev")
        return out

    def ace_build(self, phi, xi_out=None, m_out=None, ex_out=None):
        n = phi.shape[0]
        if xi_out is None:
            xi_out = self._empty(n)
        cplx = self.dtype.is_complex
        if m_out is None:
            m_out = torch.empty((n, n), dtype=torch.complex128 if cplx else torch.float64,
                                device=self.device)
        if ex_out is None:
            ex_out = torch.empty((), dtype=torch.float64, device=self.device)
        mp = check_out(m_out, "m_out", (n, n), torch.complex128 if cplx else torch.float64,
                       self.device)
        ep = check_out(ex_out, "ex_out", (), torch.float64, self.device)
        p = self._vol(phi, "phi")
        x = self._vol(xi_out, "xi_out", n)
        self._sync_stream()
        check(lib().ace_build(self._h, p, n, x, mp, ep), "ace_build")
        return xi_out, m_out, ex_out

    def ace_apply(self, xi, psi, out=None):
        if out is None:
            out = self._empty(psi.shape[0])
        x = self._vol(xi, "xi")
        p = self._vol(psi, "psi")
        o = self._vol(out, "kpsi_out", psi.shape[0])
        self._sync_stream()
        check(lib().ace_apply(self._h, x, xi.shape[0], p, psi.shape[0], o), "ace_apply")
        return out

    def ace_build_apply(self, phi, psi, xi_out=None, m_out=None, ex_out=None, kpsi_out=None):
        """ace_build and ace_apply in one call (the K psi Gram overlaps the factorisation);
        returns (xi, M, E_x, K psi)."""
        n = phi.shape[0]
        if xi_out is None:
            xi_out = self._empty(n)
        if kpsi_out is None:
            kpsi_out = self._empty(psi.shape[0])
        cplx = self.dtype.is_complex
        if m_out is None:
            m_out = torch.empty((n, n), dtype=torch.complex128 if cplx else torch.float64,
                                device=self.device)
        if ex_out is None:
            ex_out = torch.empty((), dtype=torch.float64, device=self.device)
        mp = check_out(m_out, "m_out", (n, n), torch.complex128 if cplx else torch.float64,
                       self.device)
        ep = check_out(ex_out, "ex_out", (), torch.float64, self.device)
        p = self._vol(phi, "phi")
        ps = self._vol(psi, "psi")
        x = self._vol(xi_out, "xi_out", n)
        o = self._vol(kpsi_out, "kpsi_out", psi.shape[0])
        self._sync_stream()
        check(lib().ace_build_apply(self._h, p, n, ps, psi.shape[0], x, mp, ep, o),
              "ace_build_apply")
        return xi_out, m_out, ex_out, kpsi_out

    def ace_apply_noalloc(self, xi, psi, out):
        """ace_apply through the entry point that allocates nothing (static device scratch);
        the caller provides ``out``."""
        x = self._vol(xi, "xi")
        p = self._vol(psi, "psi")
        o = self._vol(out, "kpsi_out", psi.shape[0])
        self._sync_stream()
        check(lib().ace_apply_noalloc(self._h, x, xi.shape[0], p, psi.shape[0], o),
              "ace_apply_noalloc")
        return out

    def exchange_apply_direct(self, phi, psi, out=None):
        if out is None:
            out = self._empty(psi.shape[0])
        p = self._vol(phi, "phi")
        s = self._vol(psi, "psi")
        o = self._vol(out, "kpsi_out", psi.shape[0])
        self._sync_stream()
        check(lib().exchange_apply_direct(self._h, p, phi.shape[0], s, psi.shape[0], o),
              "exchange_apply_direct")
        return out

    def tda_coupling(self, phi_occ, phi_virt, delta_m, out=None):
        no, nv = phi_occ.shape[0], phi_virt.shape[0]
        if out is None:
            out = torch.empty((no * nv, no * nv), dtype=torch.float64, device=self.device)
        op = check_out(out, "out", (no * nv, no * nv), torch.float64, self.device)
        po = self._vol(phi_occ, "phi_occ")
        pv = self._vol(phi_virt, "phi_virt")
        self._sync_stream()
        check(lib().tda_coupling(self._h, po, no, pv, nv, int(delta_m), op), "tda_coupling")
        return out

    def tda_excitations(self, c, eps_occ, eps_virt, nstates, tol=1e-8, max_iter=200):
        """Lowest nstates TDA eigenpairs of diag(eps_a - eps_i) + C (C from tda_coupling).
        Returns (omega, X, iterations) with omega (nstates,), X (nstates, no*nv) FP64 tensors."""
        import numpy as np
        eo = np.ascontiguousarray(eps_occ, dtype=np.float64)
        ev = np.ascontiguousarray(eps_virt, dtype=np.float64)
        nov = eo.size * ev.size
        if not (c.is_cuda and c.device == self.device and c.dtype == torch.float64 and
                c.shape == (nov, nov) and c.is_contiguous()):
            raise ValueError("c must be the (no*nv, no*nv) FP64 GPU coupling block")
        omega = torch.empty(nstates, dtype=torch.float64, device=self.device)
        x = torch.empty((nstates, nov), dtype=torch.float64, device=self.device)
        it = ctypes.c_int()
        self._sync_stream()
        check(lib().tda_excitations(self._h, ctypes.c_void_p(c.data_ptr()),
                                    eo.ctypes.data_as(ctypes.c_void_p), eo.size,
                                    ev.ctypes.data_as(ctypes.c_void_p), ev.size, int(nstates),
                                    float(tol), int(max_iter), ctypes.c_void_p(omega.data_ptr()),
                                    ctypes.c_void_p(x.data_ptr()), ctypes.byref(it)),
              "tda_excitations")
        return omega, x, it.value

    def tdhf_coupling(self, phi_occ, phi_virt, delta_m, c_out=None, b_out=None):
        """(C, B) of full TDHF for real RHF orbitals (Eq. (3)); FP64 GPU matrices."""
        no, nv = phi_occ.shape[0], phi_virt.shape[0]
        n = no * nv
        if c_out is None:
            c_out = torch.empty((n, n), dtype=torch.float64, device=self.device)
        if b_out is None:
            b_out = torch.empty((n, n), dtype=torch.float64, device=self.device)
        cp = check_out(c_out, "c_out", (n, n), torch.float64, self.device)
        bp = check_out(b_out, "b_out", (n, n), torch.float64, self.device)
        po = self._vol(phi_occ, "phi_occ")
        pv = self._vol(phi_virt, "phi_virt")
        self._sync_stream()
        check(lib().tdhf_coupling(self._h, po, no, pv, nv, int(delta_m), cp, bp), "tdhf_coupling")
        return c_out, b_out

    def uhf_coupling(self, occ_a, virt_a, occ_b, virt_b, with_b=True):
        """(C, B) UHF blocks (Eqs. (4), (5)); alpha transitions first.  B is None unless with_b."""
        n = occ_a.shape[0] * virt_a.shape[0] + occ_b.shape[0] * virt_b.shape[0]
        c_out = torch.empty((n, n), dtype=torch.float64, device=self.device)
        b_out = torch.empty((n, n), dtype=torch.float64, device=self.device) if with_b else None
        self._sync_stream()
        check(lib().uhf_coupling(self._h, self._vol(occ_a, "occ_a"), occ_a.shape[0],
                                 self._vol(virt_a, "virt_a"), virt_a.shape[0],
                                 self._vol(occ_b, "occ_b"), occ_b.shape[0],
                                 self._vol(virt_b, "virt_b"), virt_b.shape[0],
                                 ctypes.c_void_p(c_out.data_ptr()),
                                 ctypes.c_void_p(b_out.data_ptr()) if with_b else None),
              "uhf_coupling")
        return c_out, b_out

    def tda_excitations_diag(self, c, d, nstates, tol=1e-8, max_iter=200):
        """Lowest eigenpairs of C + diag(d) (d host array); (omega, X, iterations)."""
        import numpy as np
        dd = np.ascontiguousarray(d, dtype=np.float64)
        n = dd.size
        check_out(c, "c", (n, n), torch.float64, self.device)
        omega = torch.empty(nstates, dtype=torch.float64, device=self.device)
        x = torch.empty((nstates, n), dtype=torch.float64, device=self.device)
        it = ctypes.c_int()
        self._sync_stream()
        check(lib().tda_excitations_diag(self._h, ctypes.c_void_p(c.data_ptr()),
                                         dd.ctypes.data_as(ctypes.c_void_p), n, int(nstates),
                                         float(tol), int(max_iter), ctypes.c_void_p(omega.data_ptr()),
                                         ctypes.c_void_p(x.data_ptr()), ctypes.byref(it)),
              "tda_excitations_diag")
        return omega, x, it.value

    def tdhf_excitations(self, c, b, d, nstates, tol=1e-8, max_iter=200):
        """Full TDHF excitation energies; (omega, X+Y, iterations)."""
        import numpy as np
        dd = np.ascontiguousarray(d, dtype=np.float64)
        n = dd.size
        check_out(c, "c", (n, n), torch.float64, self.device)
        check_out(b, "b", (n, n), torch.float64, self.device)
        omega = torch.empty(nstates, dtype=torch.float64, device=self.device)
        xpy = torch.empty((nstates, n), dtype=torch.float64, device=self.device)
        it = ctypes.c_int()
        self._sync_stream()
        check(lib().tdhf_excitations(self._h, ctypes.c_void_p(c.data_ptr()),
                                     ctypes.c_void_p(b.data_ptr()),
                                     dd.ctypes.data_as(ctypes.c_void_p), n, int(nstates),
                                     float(tol), int(max_iter), ctypes.c_void_p(omega.data_ptr()),
                                     ctypes.c_void_p(xpy.data_ptr()), ctypes.byref(it)),
              "tdhf_excitations")
        return omega, xpy, it.value

    def tda_oscillator_strengths(self, phi_occ, phi_virt, x, omega):
        """(f, d): oscillator strengths (k,) and transition dipoles (k, 3) of TDA states."""
        k = omega.shape[0]
        check_out(omega, "omega", (k,), torch.float64, self.device)
        check_out(x, "x", (k, phi_occ.shape[0] * phi_virt.shape[0]), torch.float64, self.device)
        f = torch.empty(k, dtype=torch.float64, device=self.device)
        d = torch.empty((k, 3), dtype=torch.float64, device=self.device)
        po = self._vol(phi_occ, "phi_occ")
        pv = self._vol(phi_virt, "phi_virt")
        self._sync_stream()
        check(lib().tda_oscillator_strengths(self._h, po, phi_occ.shape[0], pv, phi_virt.shape[0],
                                             ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(omega.data_ptr()), k,
                                             ctypes.c_void_p(f.data_ptr()),
                                             ctypes.c_void_p(d.data_ptr())),
              "tda_oscillator_strengths")
        return f, d

    # -- closed-shell SCF pieces (real contexts) ----------------------------------------------
    def _ptr(self, t):
        return ctypes.c_void_p(t.data_ptr()) if t is not None else None

    def fock_local_apply(self, v_local, psi, out=None, accumulate=False):
        """out = [out +] T psi + v_local psi (v_local: (1, N, N, N) or None)."""
        if out is None:
            out = self._empty(psi.shape[0])
        p = self._vol(psi, "psi")
        v = self._vol(v_local, "v_local", 1) if v_local is not None else None
        o = self._vol(out, "out", psi.shape[0])
        self._sync_stream()
        check(lib().fock_local_apply(self._h, v, p, psi.shape[0], int(bool(accumulate)), o),
              "fock_local_apply")
        return out

    def scf_density(self, phi, out=None):
        if out is None:
            out = self._empty(1)
        check(lib().scf_density(self._h, self._vol(phi, "phi"), phi.shape[0],
                                self._vol(out, "rho", 1)), "scf_density")
        return out

    def hartree_potential(self, rho, out=None):
        if out is None:
            out = self._empty(1)
        self._sync_stream()
        check(lib().hartree_potential(self._h, self._vol(rho, "rho", 1), self._vol(out, "v_h", 1)),
              "hartree_potential")
        return out

    def kinetic_precondition(self, r, shift=1.0, sweeps=4, omega=0.8, out=None):
        if out is None:
            out = self._empty(r.shape[0])
        self._sync_stream()
        check(lib().kinetic_precondition(self._h, self._vol(r, "r"), r.shape[0], float(shift),
                                         int(sweeps), float(omega), self._vol(out, "z", r.shape[0])),
              "kinetic_precondition")
        return out

    def fock_lowest_states(self, v_local, phi, xi=None, opts=None):
        """LOBPCG for the lowest phi.shape[0] states of T + v_local (+ K_ACE[xi]); phi is
        overwritten by the Ritz vectors.  Returns (eigenvalues, residual norms, steps)."""
        import numpy as np
        k = phi.shape[0]
        o = opts if opts is not None else eig_opts()
        ev = np.zeros(k)
        rn = np.zeros(k)
        st = ctypes.c_int()
        self._sync_stream()
        check(lib().fock_lowest_states(self._h, self._vol(v_local, "v_local", 1),
                                       self._vol(xi, "xi") if xi is not None else None,
                                       xi.shape[0] if xi is not None else 0,
                                       self._vol(phi, "phi"), k, ctypes.byref(o),
                                       ev.ctypes.data_as(ctypes.c_void_p),
                                       rn.ctypes.data_as(ctypes.c_void_p), ctypes.byref(st)),
              "fock_lowest_states")
        return ev, rn, st.value

    def ace_build_targets(self, phi_occ, psi, xi_out=None, m_out=None):
        """ACE of K[phi_occ] compressed on span(psi) (the unoccupied-run construction)."""
        nt = psi.shape[0]
        if xi_out is None:
            xi_out = self._empty(nt)
        if m_out is None:
            m_out = torch.empty((nt, nt), dtype=torch.complex128 if self.dtype.is_complex
                                else torch.float64, device=self.device)
        mp = check_out(m_out, "m_out", (nt, nt),
                       torch.complex128 if self.dtype.is_complex else torch.float64, self.device)
        po = self._vol(phi_occ, "phi_occ")
        ps = self._vol(psi, "psi")
        xo = self._vol(xi_out, "xi_out", nt)
        self._sync_stream()
        check(lib().ace_build_targets(self._h, po, phi_occ.shape[0], ps, nt, xo, mp),
              "ace_build_targets")
        return xi_out, m_out

    def unocc_states(self, v_local, phi_occ, psi, opts=None, max_outer=50, nconv=0):
        """Unoccupied orbitals of the fixed Hamiltonian (psi overwritten); the lowest nconv
        (0: all) must converge, the rest are buffer states.  Returns (eigenvalues, residual
        norms, outer rebuilds, eigensolver steps)."""
        import numpy as np
        nv = psi.shape[0]
        o = opts if opts is not None else eig_opts(max_steps=10)
        ev, rn = np.zeros(nv), np.zeros(nv)
        outer, steps = ctypes.c_int(), ctypes.c_int()
        self._sync_stream()
        check(lib().unocc_states(self._h, self._vol(v_local, "v_local", 1),
                                 self._vol(phi_occ, "phi_occ"), phi_occ.shape[0],
                                 self._vol(psi, "psi"), nv, int(nconv), ctypes.byref(o),
                                 int(max_outer),
                                 ev.ctypes.data_as(ctypes.c_void_p),
                                 rn.ctypes.data_as(ctypes.c_void_p), ctypes.byref(outer),
                                 ctypes.byref(steps)), "unocc_states")
        return ev, rn, outer.value, steps.value

    def scf_energies(self, v_ext, phi):
        """dict(total, kinetic, external, hartree, exchange) of doubly occupied orbitals."""
        import numpy as np
        e = np.zeros(5)
        self._sync_stream()
        check(lib().scf_energies(self._h, self._vol(v_ext, "v_ext", 1), self._vol(phi, "phi"),
                                 phi.shape[0], e.ctypes.data_as(ctypes.c_void_p)), "scf_energies")
        return dict(zip(ENERGY_TERMS, e.tolist()))

    def scf_run(self, v_ext, phi, opts=None, record=None, record_stride=1):
        """Closed-shell HF SCF from phi (overwritten).  record: optional pair of FP32 GPU
        tensors (cap, N, N, N) receiving (normalised residual, normalised vector) pairs.
        Returns a dict with energies, eigenvalues, iterations, density-error history, ..."""
        import numpy as np
        k = phi.shape[0]
        o = opts if opts is not None else scf_opts()
        if record is not None:
            rin, rtg = record
            for t in (rin, rtg):
                if t.dtype != torch.float32 or not t.is_cuda or t.device != self.device or \
                        not t.is_contiguous() or tuple(t.shape[1:]) != (self.n,) * 3:
                    raise ValueError("record tensors must be contiguous FP32 (cap, N, N, N)")
            o.rec_in, o.rec_tgt, o.rec_cap = rin.data_ptr(), rtg.data_ptr(), min(rin.shape[0], rtg.shape[0])
            o.rec_stride = int(record_stride)
        else:
            o.rec_in, o.rec_tgt, o.rec_cap, o.rec_stride = None, None, 0, 1
        res = AceScfResult()
        ev = np.zeros(k)
        hist = np.zeros(o.max_iter)
        self._sync_stream()
        check(lib().scf_run(self._h, self._vol(v_ext, "v_ext", 1), self._vol(phi, "phi"), k,
                            ctypes.byref(o), ctypes.byref(res), ev.ctypes.data_as(ctypes.c_void_p),
                            hist.ctypes.data_as(ctypes.c_void_p)), "scf_run")
        out = dict(zip(ENERGY_TERMS, list(res.energy)))
        out.update(eigenvalues=ev, iterations=res.iterations, eig_steps=res.eig_steps,
                   converged=bool(res.converged), density_error=res.density_error,
                   max_residual=res.max_residual, rec_count=res.rec_count,
                   history=hist[:res.iterations].copy())
        return out

    def precond_targets(self, phi, tgt, count=None):
        """tgt[v] <- Phi (Phi^T tgt[v] dV) - tgt[v] for the first `count` FP32 volumes."""
        count = tgt.shape[0] if count is None else int(count)
        if tgt.dtype != torch.float32 or not tgt.is_contiguous():
            raise ValueError("tgt must be contiguous FP32")
        self._sync_stream()
        check(lib().precond_targets(self._h, self._vol(phi, "phi"), phi.shape[0],
                                    ctypes.c_void_p(tgt.data_ptr()), count), "precond_targets")
        return tgt

    def trace(self, on=True):
        """Enable / disable event timing of the library's kernel classes."""
        check(lib().ace_trace_enable(self._h, 1 if on else 0), "ace_trace_enable")

    def trace_reset(self):
        check(lib().ace_trace_reset(self._h), "ace_trace_reset")

    def trace_read(self):
        """{class name: (total ms, groups)} for every class recorded so far (synchronises)."""
        out = {}
        for i in range(lib().ace_trace_count()):
            ms, cnt = ctypes.c_double(), ctypes.c_longlong()
            check(lib().ace_trace_read(self._h, i, ctypes.byref(ms), ctypes.byref(cnt)),
                  "ace_trace_read")
            if cnt.value:
                out[lib().ace_trace_name(i).decode()] = (ms.value, cnt.value)
        return out

    def status(self):
        st, info = ctypes.c_int(), ctypes.c_int()
        check(lib().ace_ctx_status(self._h, ctypes.byref(st), ctypes.byref(info)), "ace_ctx_status")
        return st.value, info.value


class AceBatch:
    """Uneven batch of independent systems (each its own box edge, spacing and orbital count)
    built by one call: one launch per pass over every system."""

    def __init__(self, dtype, device=None):
        self.dtype = dtype
        self.code = dtype_code(dtype)
        self.device = _device(device)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            self._stream = torch.cuda.current_stream(self.device).cuda_stream
            check(lib().ace_batch_create(self.code, ctypes.c_void_p(self._stream),
                                         ctypes.byref(handle)), "ace_batch_create")
        self._h = handle

    def close(self):
        if getattr(self, "_h", None):
            lib().ace_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        cur = torch.cuda.current_stream(self.device).cuda_stream
        if cur != self._stream:
            check(lib().ace_batch_set_stream(self._h, ctypes.c_void_p(cur)), "ace_batch_set_stream")
            self._stream = cur

    def build(self, systems):
        """systems: list of dicts with keys h, phi (norb, n, n, n) and optional xi, M, ex
        tensors (allocated when absent).  Returns the list with xi, M, ex filled in."""
        arr = (AceMol * len(systems))()
        for k, sysd in enumerate(systems):
            phi = sysd["phi"]
            if phi.dtype != self.dtype or not phi.is_cuda or phi.device != self.device or \
                    not phi.is_contiguous() or phi.dim() != 4:
                raise ValueError("system %d: phi must be a contiguous (norb, n, n, n) %s GPU tensor"
                                 % (k, self.dtype))
            norb, n = phi.shape[0], phi.shape[1]
            if tuple(phi.shape[1:]) != (n, n, n):
                raise ValueError("system %d: cubic boxes only" % k)
            if sysd.get("xi") is None:
                sysd["xi"] = torch.empty_like(phi)
            if sysd.get("M") is None:
                sysd["M"] = torch.empty((norb, norb), device=phi.device,
                                        dtype=torch.complex128 if self.dtype.is_complex else torch.float64)
            if sysd.get("ex") is None:
                sysd["ex"] = torch.empty((), dtype=torch.float64, device=phi.device)
            xi = sysd["xi"]
            check_out(xi, "system %d: xi" % k, tuple(phi.shape), phi.dtype, self.device)
            check_out(sysd["M"], "system %d: M" % k, (norb, norb),
                      torch.complex128 if self.dtype.is_complex else torch.float64, self.device)
            check_out(sysd["ex"], "system %d: ex" % k, (), torch.float64, self.device)
            arr[k] = AceMol(n, float(sysd["h"]), norb, phi.data_ptr(), xi.data_ptr(),
                            sysd["M"].data_ptr(), sysd["ex"].data_ptr())
        self._sync_stream()
        check(lib().ace_build_batched(self._h, arr, len(systems)), "ace_build_batched")
        return systems

    def tuning(self):
        """The launch shape of the last build (text, see ace_batch_tuning)."""
        buf = ctypes.create_string_buffer(512)
        check(lib().ace_batch_tuning(self._h, buf, 512), "ace_batch_tuning")
        return buf.value.decode()

    def status(self):
        st, mol, info = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().ace_batch_status(self._h, ctypes.byref(st), ctypes.byref(mol), ctypes.byref(info)),
              "ace_batch_status")
        return st.value, mol.value, info.value

    def trace(self, on=True):
        check(lib().ace_batch_trace_enable(self._h, 1 if on else 0), "ace_batch_trace_enable")

    def trace_read(self):
        out = {}
        for i in range(lib().ace_trace_count()):
            ms, cnt = ctypes.c_double(), ctypes.c_longlong()
            check(lib().ace_batch_trace_read(self._h, i, ctypes.byref(ms), ctypes.byref(cnt)),
                  "ace_batch_trace_read")
            if cnt.value:
                out[lib().ace_trace_name(i).decode()] = (ms.value, cnt.value)
        return out


ENERGY_TERMS = ("total", "kinetic", "external", "hartree", "exchange")


def eig_opts(max_steps=50, tol=1e-6, precond="kinetic", shift=1.0, sweeps=4, omega=0.8, net=None):
    """ace_eig_opts; precond is "none", "kinetic" or "net" (then pass a ConvNet)."""
    code = {"none": PRECOND_NONE, "kinetic": PRECOND_KINETIC, "net": PRECOND_NET}[precond]
    return AceEigOpts(int(max_steps), float(tol), code, float(shift), int(sweeps), float(omega),
                      net._h if net is not None else None)


def scf_opts(alpha=0.3, tol=1e-6, max_iter=100, eig=None):
    """ace_scf_opts (states mixing alpha, Eq. (14); density error stop tol, Eq. (15))."""
    return AceScfOpts(eig if eig is not None else eig_opts(max_steps=3),
                      float(alpha), float(tol), int(max_iter), None, None, 0, 1)


class ConvNet:
    """The learned preconditioner network (three 3x3x3 convolutions, BF16 weights); its
    parameters live on the device.  Calls run on the stream current at creation."""

    def __init__(self, params=None, device=None):
        self.device = _device(device)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().convnet_create(_stream_handle(), ctypes.byref(handle)), "convnet_create")
        self._h = handle
        if params is not None:
            self.set_params(params)

    def close(self):
        if getattr(self, "_h", None):
            lib().convnet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        import numpy as np
        a = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        if a.size != NET_PARAMS:
            raise ValueError("expected %d parameters" % NET_PARAMS)
        check(lib().convnet_set_params(self._h, a.ctypes.data_as(ctypes.c_void_p)), "convnet_set_params")

    def get_params(self, rounded=False):
        import numpy as np
        a = np.zeros(NET_PARAMS, dtype=np.float32)
        check(lib().convnet_get_params(self._h, a.ctypes.data_as(ctypes.c_void_p), int(bool(rounded))),
              "convnet_get_params")
        return a

    @staticmethod
    def _vols(t, name):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 4 or \
                not (t.shape[1] == t.shape[2] == t.shape[3]):
            raise ValueError("%s must be a contiguous FP32 GPU tensor (count, N, N, N)" % name)
        return ctypes.c_void_p(t.data_ptr())

    def forward(self, x, out=None):
        if out is None:
            out = torch.empty_like(x)
        check(lib().convnet_forward(self._h, x.shape[1], self._vols(x, "x"), x.shape[0],
                                    self._vols(out, "y")), "convnet_forward")
        return out

    def gradient(self, x, t):
        """(loss, gradient (NET_PARAMS,) numpy FP32) of 1/2 mean (net(x) - t)^2."""
        import numpy as np
        g = np.zeros(NET_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        check(lib().convnet_gradient(self._h, x.shape[1], self._vols(x, "x"), self._vols(t, "t"),
                                     x.shape[0], ctypes.byref(loss), g.ctypes.data_as(ctypes.c_void_p)),
              "convnet_gradient")
        return loss.value, g

    def train(self, inputs, targets, steps, batch, lr, seed=0, random=True, count=None):
        """Adam steps on (inputs, targets) pairs; returns the per-step losses (numpy)."""
        import numpy as np
        count = inputs.shape[0] if count is None else int(count)
        hist = np.zeros(int(steps))
        check(lib().convnet_train(self._h, inputs.shape[1], self._vols(inputs, "inputs"),
                                  self._vols(targets, "targets"), count, int(steps), int(batch),
                                  float(lr), int(seed) & ((1 << 64) - 1), TRAIN_RANDOM if random else 0,
                                  hist.ctypes.data_as(ctypes.c_void_p)), "convnet_train")
        return hist


def strength_function(omega, f, w0, dw, nw, gamma):
    """S(w) on w = w0 + i dw (i < nw), Lorentzian half-width gamma (Eq. (10)); GPU tensors."""
    out = torch.empty(nw, dtype=torch.float64, device=omega.device)
    check(lib().strength_function(ctypes.c_void_p(omega.data_ptr()), ctypes.c_void_p(f.data_ptr()),
                                  omega.shape[0], float(w0), float(dw), int(nw), float(gamma),
                                  ctypes.c_void_p(out.data_ptr()), _stream_handle()),
          "strength_function")
    return out


def dense_gemm(a, b, ta=False, tb=False, alpha=1.0, beta=0.0, out=None):
    """C = alpha op(a) op(b) + beta C on FP64 GPU matrices (row-major, contiguous)."""
    m = a.shape[1] if ta else a.shape[0]
    k = a.shape[0] if ta else a.shape[1]
    n = b.shape[0] if tb else b.shape[1]
    kb = b.shape[1] if tb else b.shape[0]
    if kb != k:
        raise ValueError("inner dimensions differ: %d and %d" % (k, kb))
    for t, nm in ((a, "a"), (b, "b")):
        check_out(t, nm, tuple(t.shape), torch.float64, a.device)
    if out is None:
        out = torch.zeros((m, n), dtype=torch.float64, device=a.device)
    check_out(out, "out", (m, n), torch.float64, a.device)
    check(lib().dense_gemm(int(ta), int(tb), m, n, k, float(alpha), ctypes.c_void_p(a.data_ptr()),
                           a.shape[1], ctypes.c_void_p(b.data_ptr()), b.shape[1], float(beta),
                           ctypes.c_void_p(out.data_ptr()), n, _stream_handle()), "dense_gemm")
    return out


def sym_eig_small(a):
    """(w, V) of a symmetric FP64 GPU matrix of order <= 64 (Jacobi, one workgroup)."""
    n = a.shape[0]
    w = torch.empty(n, dtype=torch.float64, device=a.device)
    v = torch.empty((n, n), dtype=torch.float64, device=a.device)
    check(lib().sym_eig_small(n, ctypes.c_void_p(a.data_ptr()), a.shape[1],
                              ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(v.data_ptr()), n,
                              _stream_handle()), "sym_eig_small")
    return w, v


# Module-level functions with the C entry-point names.
def ace_ctx_create(n, h, dtype, device=None):
    return AceContext(n, h, dtype, device)


def pair_poisson_batched(ctx, phi_a, phi_b, pairs, out=None):
    return ctx.pair_poisson_batched(phi_a, phi_b, pairs, out)


def pair_poisson_batched_dev(ctx, phi_a, phi_b, pairs, out=None):
    return ctx.pair_poisson_batched_dev(phi_a, phi_b, pairs, out)


def ace_build(ctx, phi, xi_out=None, m_out=None, ex_out=None):
    return ctx.ace_build(phi, xi_out, m_out, ex_out)


def ace_apply(ctx, xi, psi, out=None):
    return ctx.ace_apply(xi, psi, out)


def ace_build_apply(ctx, phi, psi, xi_out=None, m_out=None, ex_out=None, kpsi_out=None):
    return ctx.ace_build_apply(phi, psi, xi_out, m_out, ex_out, kpsi_out)


def exchange_apply_direct(ctx, phi, psi, out=None):
    return ctx.exchange_apply_direct(phi, psi, out)


def tda_coupling(ctx, phi_occ, phi_virt, delta_m, out=None):
    return ctx.tda_coupling(phi_occ, phi_virt, delta_m, out)


def ace_ctx_status(ctx):
    return ctx.status()


def ace_build_batched(batch, systems):
    return batch.build(systems)
