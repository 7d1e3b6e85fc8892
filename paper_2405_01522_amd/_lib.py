"""ctypes loader for libace.so (the HIP library built from csrc/).

The library must be built (``python -m paper_2405_01522_amd.build``); there is no fallback of
any kind: a missing library raises immediately.  torch is imported first so that libace binds
to the HIP runtime torch already loaded (same SONAME), keeping one runtime per process.
"""

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime libace links against)

# ACE_LIBRARY may name another build of the same sources (e.g. one compiled with different
# tuning macros); by default the in-tree library is used.
LIB_PATH = os.environ.get("ACE_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                          "libace.so")

_lib = None

# entry points declared in include/ace.h: name -> (restype, argtypes)
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
SIGNATURES = {
    "ace_ctx_create": (_I, [_I, _D, _I, _P, ctypes.POINTER(_P)]),
    "ace_ctx_destroy": (_I, [_P]),
    "ace_ctx_set_stream": (_I, [_P, _P]),
    "ace_size_supported": (_I, [_I, _I]),
    "pair_poisson_batched": (_I, [_P, _P, _I, _P, _I, ctypes.POINTER(ctypes.c_int32), _I, _P]),
    "pair_poisson_batched_dev": (_I, [_P, _P, _I, _P, _I, _P, _I, _P]),
    "ace_build": (_I, [_P, _P, _I, _P, _P, _P]),
    "ace_apply": (_I, [_P, _P, _I, _P, _I, _P]),
    "ace_build_apply": (_I, [_P, _P, _I, _P, _I, _P, _P, _P, _P]),
    "ace_apply_noalloc": (_I, [_P, _P, _I, _P, _I, _P]),
    "exchange_apply_direct": (_I, [_P, _P, _I, _P, _I, _P]),
    "tda_coupling": (_I, [_P, _P, _I, _P, _I, _I, _P]),
    "ace_ctx_status": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "ace_strerror": (ctypes.c_char_p, [_I]),
    "ace_batch_create": (_I, [_I, _P, ctypes.POINTER(_P)]),
    "ace_batch_destroy": (_I, [_P]),
    "ace_batch_set_stream": (_I, [_P, _P]),
    "ace_build_batched": (_I, [_P, _P, _I]),
    "ace_batch_status": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "ace_batch_tuning": (_I, [_P, ctypes.c_char_p, _I]),
    "ace_batch_trace_enable": (_I, [_P, _I]),
    "ace_batch_trace_read": (_I, [_P, _I, ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_longlong)]),
    "tda_excitations": (_I, [_P, _P, _P, _I, _P, _I, _I, _D, _I, _P, _P, ctypes.POINTER(_I)]),
    "tda_oscillator_strengths": (_I, [_P, _P, _I, _P, _I, _P, _P, _I, _P, _P]),
    "strength_function": (_I, [_P, _P, _I, _D, _D, _I, _D, _P, _P]),
    "dense_gemm": (_I, [_I, _I, _I, _I, _I, _D, _P, _I, _P, _I, _D, _P, _I, _P]),
    "sym_eig_small": (_I, [_I, _P, _I, _P, _P, _I, _P]),
    "ace_trace_enable": (_I, [_P, _I]),
    "ace_trace_read": (_I, [_P, _I, ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_longlong)]),
    "ace_trace_reset": (_I, [_P]),
    "ace_trace_count": (_I, []),
    "ace_trace_name": (ctypes.c_char_p, [_I]),
    "fock_local_apply": (_I, [_P, _P, _P, _I, _I, _P]),
    "scf_density": (_I, [_P, _P, _I, _P]),
    "hartree_potential": (_I, [_P, _P, _P]),
    "kinetic_precondition": (_I, [_P, _P, _I, _D, _I, _D, _P]),
    "fock_lowest_states": (_I, [_P, _P, _P, _I, _P, _I, _P, _P, _P, ctypes.POINTER(_I)]),
    "scf_energies": (_I, [_P, _P, _P, _I, _P]),
    "ace_build_targets": (_I, [_P, _P, _I, _P, _I, _P, _P]),
    "tdhf_coupling": (_I, [_P, _P, _I, _P, _I, _I, _P, _P]),
    "uhf_coupling": (_I, [_P, _P, _I, _P, _I, _P, _I, _P, _I, _P, _P]),
    "tda_excitations_diag": (_I, [_P, _P, _P, _I, _I, _D, _I, _P, _P, ctypes.POINTER(_I)]),
    "tdhf_excitations": (_I, [_P, _P, _P, _P, _I, _I, _D, _I, _P, _P, ctypes.POINTER(_I)]),
    "unocc_states": (_I, [_P, _P, _P, _I, _P, _I, _I, _P, _I, _P, _P, ctypes.POINTER(_I),
                          ctypes.POINTER(_I)]),
    "scf_run": (_I, [_P, _P, _P, _I, _P, _P, _P, _P]),
    "precond_targets": (_I, [_P, _P, _I, _P, _I]),
    "convnet_create": (_I, [_P, ctypes.POINTER(_P)]),
    "convnet_destroy": (_I, [_P]),
    "convnet_set_params": (_I, [_P, _P]),
    "convnet_get_params": (_I, [_P, _P, _I]),
    "convnet_forward": (_I, [_P, _I, _P, _I, _P]),
    "convnet_gradient": (_I, [_P, _I, _P, _P, _I, _P, _P]),
    "convnet_train": (_I, [_P, _I, _P, _P, _I, _I, _I, _D, ctypes.c_ulonglong, _I, _P]),
}

NET_PARAMS = 2177
PRECOND_NONE, PRECOND_KINETIC, PRECOND_NET = 0, 1, 2
TRAIN_RANDOM = 1


class AceMol(ctypes.Structure):
    """Mirror of ace_mol in include/ace.h."""
    _fields_ = [("n", ctypes.c_int), ("h", ctypes.c_double), ("norb", ctypes.c_int),
                ("phi", ctypes.c_void_p), ("xi", ctypes.c_void_p),
                ("M", ctypes.c_void_p), ("ex", ctypes.c_void_p)]


class AceEigOpts(ctypes.Structure):
    """Mirror of ace_eig_opts."""
    _fields_ = [("max_steps", ctypes.c_int), ("tol", ctypes.c_double), ("precond", ctypes.c_int),
                ("shift", ctypes.c_double), ("sweeps", ctypes.c_int), ("omega", ctypes.c_double),
                ("net", ctypes.c_void_p)]


class AceScfOpts(ctypes.Structure):
    """Mirror of ace_scf_opts."""
    _fields_ = [("eig", AceEigOpts), ("alpha", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("rec_in", ctypes.c_void_p),
                ("rec_tgt", ctypes.c_void_p), ("rec_cap", ctypes.c_int),
                ("rec_stride", ctypes.c_int)]


class AceScfResult(ctypes.Structure):
    """Mirror of ace_scf_result."""
    _fields_ = [("energy", ctypes.c_double * 5), ("density_error", ctypes.c_double),
                ("max_residual", ctypes.c_double), ("iterations", ctypes.c_int),
                ("eig_steps", ctypes.c_int), ("converged", ctypes.c_int),
                ("rec_count", ctypes.c_int)]


class AceError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib().ace_strerror(code).decode() if _lib is not None else str(code)
        super().__init__("%s failed: %s (%d)" % (where, msg, code))


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libace.so is not built (%s); run "
                              "`python -m paper_2405_01522_amd.build`" % LIB_PATH)
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(code, where):
    if code != 0:
        raise AceError(code, where)
