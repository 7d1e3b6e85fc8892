"""MI355X-native exact exchange through ACE and the Tamm-Dancoff coupling block.

The computation lives in libace.so (HIP kernels for gfx950, C ABI in include/ace.h); this
package only marshals torch tensors into it.  Build with
``python -m paper_2405_01522_amd.build``.
"""

from .api import (  # noqa: F401
    AceContext, AceBatch, ace_ctx_create, ace_build_batched, pair_poisson_batched,
    pair_poisson_batched_dev, ace_build, ace_apply, ace_build_apply,
    exchange_apply_direct, tda_coupling, ace_ctx_status, size_supported, MAX_ORBITALS,
    strength_function, dense_gemm, sym_eig_small, ConvNet, eig_opts, scf_opts, ENERGY_TERMS,
)
