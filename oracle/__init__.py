"""Plain FP64 CPU oracle for real-space exact exchange through ACE and the TDA coupling block.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or link this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the HIP library (no kernels, headers,
tables or pre/post-processing) and imports nothing from ``paper_2405_01522_amd``.

Everything here is written for a reader holding the paper (Panta & Strubbe,
"Implementation of time-dependent Hartree-Fock in real space", arXiv 2405.01522):

* ``grid``     -- uniform isolated grid and the sampled Coulomb kernel (Sec. 3.1: the
                  exchange integral solved as a Poisson problem).
* ``poisson``  -- the discrete aperiodic convolution v = dV * G (*) rho, once by a 2x
                  zero-padded FFT and once by the O(N_g^2) direct sum (Sec. 3.1 compares
                  both routes by cost).
* ``exchange`` -- direct exact exchange, Eq. (2); the ACE construction, Eqs. (11)-(13);
                  the exchange energy.
* ``tda``      -- two-electron integrals and the RHF Tamm-Dancoff A matrix, Eq. (7) and
                  the TDA paragraph of Sec. 2; eigenvalues, dipoles, oscillator strengths
                  (Eqs. (8)-(10)).
* ``scf``      -- closed-shell HF ground state on the grid: Eq. (1) with linear mixing of
                  states (Eq. (14)) and the relative density error stop (Eq. (15)).
* ``convnet``  -- a three-layer 3-D convolutional network (forward, exact gradients) used
                  as a learned eigensolver preconditioner; not from the paper.

All arithmetic is float64 / complex128.  Library primitives used as steps: numpy/scipy
FFT, matmul, Cholesky, triangular solve, Hermitian eigensolver.

Parity status per function is stated in each module docstring.
"""

from . import grid, poisson, exchange, tda, scf, convnet  # noqa: F401
