/*
 * ace.h -- C ABI of libace: real-space exact exchange through Adaptively Compressed
 * Exchange (ACE) and the Tamm-Dancoff coupling block, on one AMD Instinct MI355X (gfx950).
 *
 * Paper: U. Panta and D. A. Strubbe, "Implementation of time-dependent Hartree-Fock in real
 * space", arXiv:2405.01522.  Each entry point cites the passage that defines what it computes.
 *
 * Grid.  A cubic box of N^3 points with spacing h (bohr), isolated (orbitals vanish outside
 * the box, the zero-boundary domain of Sec. 3.4).  Point (x, y, z) is stored at
 * ((x * N) + y) * N + z (z fastest).  An "orbital array" holds `count` such volumes back to
 * back: element [k][x][y][z].  Complex values are interleaved (re, im).
 *
 * Poisson kernel.  v(r) = dV sum_{r'} G(r - r') rho(r') with G(d) = 1/(h |d|) for integer
 * displacements d != 0 and G(0) = C0 / h, C0 = 3 ln(2 + sqrt 3) - pi/2 (cube average of
 * 1/|r|), dV = h^3.  Evaluated exactly (up to rounding) by a 2x zero-padded FFT.
 *
 * Precision.  The orbital storage type fixes the arithmetic:
 *   ACE_C128, ACE_R64 : every step in FP64;
 *   ACE_C64,  ACE_R32 : pair densities, FFTs, W, xi and K psi in FP32; the Coulomb kernel
 *                       spectrum, Gram cross-tile sums, M, the Cholesky factor and E_x in FP64.
 *
 * Memory and streams.  All array arguments are DEVICE pointers unless marked (host).  The
 * caller owns every input and output; the context owns its workspaces, the kernel spectrum
 * and a device status word.  Every call enqueues work on the context's HIP stream and returns
 * without synchronising (except ace_ctx_create, ace_ctx_status and calls that must grow a
 * workspace, which synchronise the stream first).  A context is not thread-safe; use one per
 * stream.
 *
 * Errors.  Functions return 0 on success or a negative ACE_ERR_* code; nothing is enqueued
 * when argument checking fails.  Numerical failures found on the device (non positive
 * definite -M, non-finite M) are recorded in the status word and reported by ace_ctx_status.
 */
#ifndef ACE_H
#define ACE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ace_ctx ace_ctx;

typedef enum { ACE_C128 = 0, ACE_C64 = 1, ACE_R64 = 2, ACE_R32 = 3 } ace_dtype;

enum {
  ACE_OK = 0,
  ACE_ERR_INVALID = -1,     /* null pointer, count < 1, bad index, bad flag */
  ACE_ERR_UNSUPPORTED = -2, /* box edge not compiled for the dtype */
  ACE_ERR_HIP = -3,         /* a HIP runtime call failed */
  ACE_ERR_OOM = -4,         /* device allocation failed */
  ACE_ERR_NOT_POSDEF = -5,  /* -M not positive definite (device status; info = pivot) */
  ACE_ERR_NONFINITE = -6,   /* M not finite (device status) */
  ACE_ERR_SCRATCH = -7      /* ace_apply_noalloc: one vector's sums exceed the static scratch */
};

/* Largest orbital count accepted by ace_build / ace_apply: real orbitals, complex orbitals. */
#define ACE_MAX_ORBITALS 64
#define ACE_MAX_ORBITALS_COMPLEX 32

/*
 * Create a context for an N^3 box of spacing h holding orbitals of storage type `dtype`.
 * Computes the spectrum of the isolated Coulomb kernel on the padded (2N)^3 grid in FP64 on
 * the device (kept as its real-even octant) -- the Poisson problem of Sec. 3.1.
 * n: box edge (see ace_size_supported); h > 0 in bohr; hip_stream: a hipStream_t, or NULL
 * for the null stream.  *out receives the context.  Synchronises the stream once.
 */
int ace_ctx_create(int n, double h, int dtype, void* hip_stream, ace_ctx** out);

/* Destroy a context (synchronises its stream, frees its device memory).  NULL is allowed. */
int ace_ctx_destroy(ace_ctx* ctx);

/* Change the stream later calls enqueue on (NULL = null stream). */
int ace_ctx_set_stream(ace_ctx* ctx, void* hip_stream);

/* 1 if a box edge n is compiled for the given dtype, else 0.  Edges 8, 9, 10, 12, 15, 16, 20,
 * 24, 32, 40, 48, 56 and 64 (padded edges with radices 2, 3, 5, 7) in every dtype; where the
 * padded P x P plane of the XY pass does not fit in LDS (FP64 at 56 and 64) the pass keeps the
 * N y-transformed rows and runs the x transforms over strips of columns. */
int ace_size_supported(int n, int dtype);

/*
 * Batched isolated Poisson solves of pair densities (Sec. 3.1: the integral of Eq. (2) posed
 * as a Poisson problem for rho = phi_j phi_i):
 *   v_out[p] = dV * G (*) ( conj(phi_a[pairs[2p]]) * phi_b[pairs[2p+1]] ),  p = 0..np-1.
 * phi_a: [na][N^3], phi_b: [nb][N^3] orbital arrays of the context dtype;
 * pairs (host): np index pairs (j, i) with 0 <= j < na, 0 <= i < nb;
 * v_out: [np][N^3] of the context dtype (real dtypes give real v; pairs are then solved two
 * per complex FFT).  v_out must not overlap the inputs.
 */
int pair_poisson_batched(ace_ctx* ctx, const void* phi_a, int na, const void* phi_b, int nb,
                         const int32_t* pairs, int np, void* v_out);

/*
 * pair_poisson_batched with the pair list in device memory (int32 [np][2], (j, i) as above),
 * for a caller that builds or keeps its list on the GPU.  Nothing is copied or read on the
 * host, so the call can be captured into a HIP graph.  The host cannot check the indices:
 * the kernels clamp each to [0, na) / [0, nb), so no access leaves phi_a or phi_b, and record
 * the first index out of range in the device status word (ace_ctx_status then returns
 * ACE_ERR_INVALID with info = the offending pair); the outputs of such pairs are undefined.
 */
int pair_poisson_batched_dev(ace_ctx* ctx, const void* phi_a, int na, const void* phi_b, int nb,
                             const int32_t* pairs_dev, int np, void* v_out);

/*
 * Build the ACE operator from n orbitals phi (Sec. 3.1, Eqs. (11)-(12)):
 *   W_i  = -sum_j phi_j v_ji,  v_ji = dV G (*) (conj(phi_j) phi_i)      (Eq. (11), Eq. (2))
 *   M    = dV Phi^H W  (Hermitised),  -M = L L^H  (L lower, positive diagonal)
 *   xi   = W L^{-H}                                                    (Eq. (12))
 *   E_x  = 1/2 sum_i M_ii   (occupation 1 per orbital; multiply by 2 for a closed-shell RHF
 *                            determinant built from spatial orbitals)
 * phi: [n][N^3], 1 <= n <= ACE_MAX_ORBITALS (ACE_MAX_ORBITALS_COMPLEX for complex dtypes);
 * xi_out: [n][N^3] (context dtype);
 * M_out: n*n FP64, complex interleaved for complex dtypes, row-major M[k][l], or NULL;
 * ex_out: one double, or NULL.  n(n+1)/2 pair solves are made.  If -M is not positive
 * definite the status word records ACE_ERR_NOT_POSDEF with the pivot and xi is zero.
 */
int ace_build(ace_ctx* ctx, const void* phi, int n, void* xi_out, double* M_out,
              double* ex_out);

/*
 * ACE with extra orbitals (Sec. 3.1: the non-self-consistent run for unoccupied orbitals
 * includes them in Eqs. (11)-(13)): the exchange operator K of the no occupied orbitals
 * phi_occ (Eq. (2)) compressed on the span of nt target orbitals psi (typically the occupied
 * followed by the current unoccupied ones):
 *   W_t = K psi_t (no * nt pair solves), M = Psi^H W dV, -M = L L^H, xi = W L^{-H};
 * K_ACE = -xi xi^H dV then equals K on span(psi).  nt <= ACE_MAX_ORBITALS (complex:
 * ACE_MAX_ORBITALS_COMPLEX).  M_out (device, nt*nt, may be NULL).  Failures of the
 * factorisation go to the device status word (ace_ctx_status).
 */
int ace_build_targets(ace_ctx* ctx, const void* phi_occ, int no, const void* psi, int nt,
                      void* xi_out, double* M_out);

/*
 * Apply the ACE operator (Eq. (13)): kpsi_out[v] = -sum_k xi_k dV <xi_k | psi_v>.
 * xi: [n][N^3] from ace_build; psi: [nv][N^3]; kpsi_out: [nv][N^3] (may not alias psi).
 */
int ace_apply(ace_ctx* ctx, const void* xi, int n, const void* psi, int nv, void* kpsi_out);

/*
 * ace_build followed by ace_apply in one call (Eqs. (11)-(13)): the same xi_out, M_out and
 * ex_out as ace_build (the same arithmetic, so the same bits) and
 *   kpsi_out[v] = -sum_k xi_k dV <xi_k | psi_v>,
 * with dV <xi_k | psi_v> taken as (L^{-1} Y)_kv, Y = dV W^H psi (FP64 sums, as ace_apply's):
 * Y needs only W, so for complex storage and n <= 8 its Gram shares a launch with the
 * reduction of M, and its reduction and L^{-1} Y one with the Cholesky factorisation and xi
 * (two fewer launches on the path than ace_build + ace_apply).  K psi agrees with ace_build + ace_apply
 * to rounding.  Arguments as in ace_build and ace_apply; psi: [nv][N^3], kpsi_out:
 * [nv][N^3]; kpsi_out may not alias psi, phi or xi_out.  Everything runs on the context
 * stream; the call can be captured into a HIP graph once its workspace exists (make one
 * uncaptured call of the same sizes first).
 */
int ace_build_apply(ace_ctx* ctx, const void* phi, int n, const void* psi, int nv, void* xi_out,
                    double* M_out, double* ex_out, void* kpsi_out);

/*
 * ace_apply without any allocation, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments and results as ace_apply (the same kernels and passes, so the same bits); its
 * Gram partial sums and the reduced xi^H psi block live in a static device array of
 * ACE_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends) instead of a context
 * workspace, and the call makes no hipMalloc / hipFree.  The array's address on each device
 * is looked up when a context is created there.  Needs 8 * (1 + complex) * n * (ceil(N^3 /
 * 256) + 1) bytes per vector (every supported edge and orbital count fits; vectors are taken
 * in passes of as many as fit, at most 64); ACE_ERR_SCRATCH otherwise.  All calls on one GPU
 * share its array: calls that overlap in time on one GPU (other streams, other contexts, other
 * threads) race and must be serialised by the caller.  Nothing in the array needs clearing.
 */
#define ACE_NOALLOC_SCRATCH_BYTES (8u << 20)
int ace_apply_noalloc(ace_ctx* ctx, const void* xi, int n, const void* psi, int nv,
                      void* kpsi_out);

/*
 * Direct exact exchange (Eq. (2)), the operator ACE compresses:
 *   kpsi_out[v] = -sum_j phi_j * dV G (*) (conj(phi_j) psi_v).
 * phi: [n][N^3]; psi: [nv][N^3]; kpsi_out: [nv][N^3].  n*nv pair solves.
 */
int exchange_apply_direct(ace_ctx* ctx, const void* phi, int n, const void* psi, int nv,
                          void* kpsi_out);

/*
 * Coupling block of the RHF Tamm-Dancoff matrix for real orbitals (Sec. 2, Eq. (7), without
 * the diagonal (eps_a - eps_i) term, which the caller adds):
 *   C[ia][jb] = delta_M (ai|jb) - (ab|ji),  row/col index ia = i * n_virt + a,
 * with (pq|rs) = dV sum_r phi_r phi_s (r) v_pq(r).  Needs a real dtype (ACE_R64 / ACE_R32).
 * phi_occ: [no][N^3], phi_virt: [nv][N^3]; delta_M: 2 (singlet) or 0 (triplet);
 * C_out: (no*nv)^2 doubles, row-major.  Makes no*nv + no(no+1)/2 pair solves.
 */
int tda_coupling(ace_ctx* ctx, const void* phi_occ, int no, const void* phi_virt, int nv,
                 int delta_M, double* C_out);

/*
 * Full TDHF blocks for real RHF orbitals (Eq. (3)): C as tda_coupling (A without its diagonal
 * eps_a - eps_i) and the B block spin-adapted from Eq. (5),
 *   B[ia][jb] = delta_M (ia|bj) - (ib|aj)   (delta_M = 2 singlet, 0 triplet),
 * from the same pair solves and contraction (for real orbitals (ib|aj) is an entry of the
 * same (ia|jb) matrix).  B_out: (no*nv)^2 FP64 device, or NULL (then this is tda_coupling).
 */
int tdhf_coupling(ace_ctx* ctx, const void* phi_occ, int no, const void* phi_virt, int nv,
                  int delta_M, double* C_out, double* B_out);

/*
 * UHF blocks (Eqs. (4), (5)) for real orbitals of two spin channels, alpha (occ_a, virt_a) and
 * beta (occ_b, virt_b), with (pq||rs) = (pq|rs) - (pr|qs) over spin orbitals:
 *   C[x][y] = (ia|jb) - delta_st (ij|ab),  B[x][y] = (ia|bj) - delta_st (ib|aj),
 * x = transition (i, a) of spin s, y = (j, b) of spin t; alpha transitions i*nv_a + a come
 * first, then beta ones.  C_out, B_out: n x n FP64 device, n = no_a nv_a + no_b nv_b (B_out
 * may be NULL).  A = diag(eps_a - eps_i) + C.  For a closed shell (the same orbitals in both
 * channels) the spectrum is the union of the RHF singlet and triplet spectra.
 */
int uhf_coupling(ace_ctx* ctx, const void* occ_a, int no_a, const void* virt_a, int nv_a,
                 const void* occ_b, int no_b, const void* virt_b, int nv_b, double* C_out,
                 double* B_out);

/*
 * Uneven batches of independent systems (the ACE rebuild of Sec. 3.1, Eqs. (11)-(12), for many
 * molecules at once).  A batch owns one kernel spectrum per distinct (n, h).  Each pass of a
 * build is one launch over every system of every box edge: the three pair-Poisson passes are
 * persistent launches over a device list of transform planes (largest edge first), and W / M /
 * Cholesky / xi one launch each over all systems.  All work is enqueued on the batch stream, so
 * a call can be captured into a HIP graph once an earlier eager call has sized the workspaces.
 * Launch shapes (XY-pass planes per workgroup for each edge, threads of the z passes) are tuned
 * by timing the candidates on the first eager call for each (dtype, set of box edges); the
 * choices are kept for the process and, when the environment variable ACE_TUNE_CACHE names a
 * file, appended to that file and read from it by later processes.  Every shape gives the same
 * bits.
 */
typedef struct ace_batch ace_batch;

typedef struct {
  int n;              /* box edge of this system */
  double h;           /* spacing (bohr) */
  int norb;           /* orbitals, 1..ACE_MAX_ORBITALS (complex: ACE_MAX_ORBITALS_COMPLEX) */
  const void* phi;    /* [norb][n^3] orbitals (batch dtype), device */
  void* xi;           /* [norb][n^3] ACE projectors, device, output */
  double* M;          /* [norb*norb] M (complex interleaved for complex dtypes), device, or NULL */
  double* ex;         /* E_x, device scalar, or NULL */
} ace_mol;

int ace_batch_create(int dtype, void* hip_stream, ace_batch** out);
int ace_batch_destroy(ace_batch* batch);
int ace_batch_set_stream(ace_batch* batch, void* hip_stream);

/*
 * Build the ACE operator of every system in mols (host array of nmol entries): the same
 * results as ace_build on each system.  Returns ACE_ERR_UNSUPPORTED if an edge is not
 * compiled for the dtype.  Device-side failures are reported per system by ace_batch_status.
 */
int ace_build_batched(ace_batch* batch, const ace_mol* mols, int nmol);

/* The launch shape used by the last ace_build_batched call, as text (host buffer of len
 * bytes): "dtype=<d>,edges=<n>-<n>... xy=<edge>:<planes>,... zf=<threads> zi=<threads>
 * source=tuned|cache|default". */
int ace_batch_tuning(ace_batch* batch, char* buf, int len);

/*
 * Synchronise and report the first device-side failure since the last call: *status, the
 * system index *mol (host, may be NULL, -1 if none) and *info (host, may be NULL).  Clears.
 */
int ace_batch_status(ace_batch* batch, int* status, int* mol, int* info);

/* Event tracing of a batch's launches (same classes as ace_trace_*). */
int ace_batch_trace_enable(ace_batch* batch, int on);
int ace_batch_trace_read(ace_batch* batch, int id, double* total_ms, long long* count);

/*
 * Tamm-Dancoff excitations (Sec. 2: A X = omega X, A = diag(eps_a - eps_i) + C, Eq. (7)): the
 * nstates (1..16) lowest eigenpairs by a block Davidson iteration on the device.
 * C: (no*nv)^2 FP64 device (from tda_coupling); eps_occ[no], eps_virt[nv]: host;
 * tol: residual norm |A x - omega x| for convergence; max_iter: iteration cap;
 * omega_out[nstates] device; X_out [nstates][no*nv] device (unit eigenvectors) or NULL;
 * *iterations (host, may be NULL): iterations used, negative if not converged.
 * Synchronises the context stream.
 */
int tda_excitations(ace_ctx* ctx, const double* C, const double* eps_occ, int no,
                    const double* eps_virt, int nv, int nstates, double tol, int max_iter,
                    double* omega_out, double* X_out, int* iterations);

/*
 * Lowest eigenpairs of A = C + diag(d) for any dense symmetric C (n x n FP64 device) and
 * diagonal d (host, n): the general form of tda_excitations (e.g. the UHF transitions of
 * uhf_coupling with d = eps_a - eps_i per spin).  Same outputs and limits as tda_excitations.
 */
int tda_excitations_diag(ace_ctx* ctx, const double* C, const double* d, int n, int nstates,
                         double tol, int max_iter, double* omega_out, double* X_out,
                         int* iterations);

/*
 * Full TDHF (Eq. (3)) for real orbitals, A = C + diag(d), B from tdhf_coupling or
 * uhf_coupling: with A - B = L L^T (blocked Cholesky on the device), the Hermitian half-size
 * problem L^T (A + B) L z = omega^2 z (Sec. 2) is solved by the same Davidson iteration.
 * omega_out (device, nstates) ascending excitation energies; XpY_out (device, nstates x n, may
 * be NULL) the vectors X + Y = L z / sqrt(omega), normalised by (X+Y)^T (X-Y) = 1, for
 * transition dipoles as in Eq. (8).  Returns ACE_ERR_NOT_POSDEF if A - B is not positive
 * definite (an unstable reference).  1 <= nstates <= 16.  Synchronises.
 */
int tdhf_excitations(ace_ctx* ctx, const double* C, const double* B, const double* d, int n,
                     int nstates, double tol, int max_iter, double* omega_out, double* XpY_out,
                     int* iterations);

/*
 * Transition dipoles and oscillator strengths of TDA states (Eqs. (8)-(9), atomic units):
 * d_k = sum_ia <i| r |a> X_k,ia on the context grid, f_k = 2/3 omega_k |d_k|^2.  Real dtypes.
 * phi_occ [no][N^3], phi_virt [nv][N^3]; X [nstates][no*nv] and omega [nstates] FP64 device;
 * f_out [nstates] device; d_out [nstates][3] device or NULL.  Synchronises the stream.
 */
int tda_oscillator_strengths(ace_ctx* ctx, const void* phi_occ, int no, const void* phi_virt,
                             int nv, const double* X, const double* omega, int nstates,
                             double* f_out, double* d_out);

/*
 * Strength function (Eq. (10)) with each delta broadened to a normalised Lorentzian of
 * half-width gamma: S_out[i] = sum_k f_k gamma / (pi ((w_i - omega_k)^2 + gamma^2)),
 * w_i = w0 + i dw, i < nw.  All arrays FP64 device; hip_stream may be NULL.
 */
int strength_function(const double* omega, const double* f, int nstates, double w0, double dw,
                      int nw, double gamma, double* S_out, void* hip_stream);

/*
 * Small dense FP64 helpers used by the eigensolver drivers (device arrays, row-major):
 *   dense_gemm: C = alpha op(A) op(B) + beta C, op(X) = X (t = 0) or X^T (t = 1), C is M x N;
 *   sym_eig_small: eigenvalues (ascending, w[n]) and eigenvectors (columns of V) of the
 *   symmetric part of A, n <= 64, by parallel-order Jacobi rotations in one workgroup.
 */
int dense_gemm(int ta, int tb, int M, int N, int K, double alpha, const double* A, int lda,
               const double* B, int ldb, double beta, double* C, int ldc, void* hip_stream);
int sym_eig_small(int n, const double* A, int lda, double* w, double* V, int ldv,
                  void* hip_stream);

/*
 * Synchronise the context stream and report the device status word: *status (host) receives
 * ACE_OK or the first device-side error recorded since the last call, *info (host, may be
 * NULL) the failing pivot for ACE_ERR_NOT_POSDEF, the pair for ACE_ERR_INVALID (an index out
 * of range in a device pair list).  The word is then cleared.
 */
int ace_ctx_status(ace_ctx* ctx, int* status, int* info);

/*
 * Event tracing of the library's own launches (a measurement aid, not part of the method).
 * When enabled, every group of launches of one kernel class on the context stream is
 * bracketed by a pair of HIP events; totals are accumulated when read.
 *   ace_trace_enable(ctx, on)             start / stop recording (pending records are kept);
 *   ace_trace_read(ctx, id, &ms, &count)  synchronise, return total milliseconds and the
 *                                         number of recorded groups of class id;
 *   ace_trace_reset(ctx)                  zero the totals;
 *   ace_trace_count(), ace_trace_name(id) the classes (e.g. "poisson_xy").
 */
int ace_trace_enable(ace_ctx* ctx, int on);
int ace_trace_read(ace_ctx* ctx, int id, double* total_ms, long long* count);
int ace_trace_reset(ace_ctx* ctx);
int ace_trace_count(void);
const char* ace_trace_name(int id);

/* ---------------------------------------------------------------------------------------
 * Closed-shell Hartree-Fock ground state (Eq. (1)) on the isolated grid, real orbitals
 * (contexts of dtype ACE_R64 or ACE_R32; others return ACE_ERR_UNSUPPORTED).
 *
 * The paper's Hamiltonian needs pseudopotentials that are not part of this library; these
 * pieces are fixed here:
 *   T       = -1/2 Laplacian by fourth-order central differences on each axis,
 *             (-f(x-2h) + 16 f(x-h) - 30 f(x) + 16 f(x+h) - f(x+2h)) / (12 h^2), orbitals
 *             zero outside the box;
 *   V_ext   = any local potential the caller passes (one grid volume);
 *   rho     = 2 sum_i phi_i^2 (n doubly occupied orbitals, normalised sum phi^2 dV = 1);
 *   v_H     = dV G (*) rho with the Poisson kernel above;
 *   K       = the exchange operator of Eq. (2) over the occupied spatial orbitals, applied
 *             through ACE (Eqs. (11)-(13)) rebuilt every SCF iteration (Sec. 3.1);
 *   E       = 2 sum_i <phi_i|T + V_ext|phi_i> + 1/2 int rho v_H + sum_i <phi_i|K phi_i>.
 * ------------------------------------------------------------------------------------- */

/* out_v = (accumulate ? out_v : 0) + T psi_v + v_local psi_v, v < nv (v_local may be NULL). */
int fock_local_apply(ace_ctx* ctx, const void* v_local, const void* psi, int nv, int accumulate,
                     void* out);

/* rho = 2 sum_{i<k} phi_i^2 (Eq. (1)'s closed-shell density). */
int scf_density(ace_ctx* ctx, const void* phi, int k, void* rho);

/* Hartree potential v_H = dV G (*) rho (one isolated Poisson solve, Sec. 3.1).  Allocates a
 * scratch volume and synchronises the stream. */
int hartree_potential(ace_ctx* ctx, const void* rho, void* v_h);

/* Kinetic preconditioner z ~ (T + shift)^{-1} r for nv vectors: z_0 = r / (d + shift) with
 * d = 15 / (4 h^2) the diagonal of T, then sweeps - 1 damped-Jacobi steps
 * z <- z + omega (r - (T + shift) z) / (d + shift).  sweeps >= 1, 0 < omega < 2.
 * Synchronises the stream. */
int kinetic_precondition(ace_ctx* ctx, const void* r, int nv, double shift, int sweeps,
                         double omega, void* z);

/* ---- learned preconditioner: a 3-D convolutional network (not from the paper) ----------
 * x (1 channel) -> conv 3x3x3 (8) -> ReLU -> conv 3x3x3 (8) -> ReLU -> conv 3x3x3 (1), zero
 * padding.  Weights BF16 (rounded from FP32 masters), activations and sums FP32.
 * Parameters (FP32, ACE_NET_PARAMS values): [w0 8x1x27][b0 8][w1 8x8x27][b1 8][w2 1x8x27][b2 1],
 * w[out][in][t] acting on the input at offset (t/9 - 1, (t/3)%3 - 1, t%3 - 1). */
#define ACE_NET_PARAMS 2177
typedef struct ace_convnet ace_convnet;

int convnet_create(void* hip_stream, ace_convnet** out);  /* parameters zero */
int convnet_destroy(ace_convnet* net);
/* params (host, ACE_NET_PARAMS FP32): set the masters, round the compute copy to BF16, reset
 * Adam.  Synchronises. */
int convnet_set_params(ace_convnet* net, const float* params);
/* params (host): the masters (rounded = 0) or the BF16-rounded compute copy (rounded = 1). */
int convnet_get_params(ace_convnet* net, float* params, int rounded);
/* y[b] = net(x[b]) for nb FP32 volumes of edge n (device). */
int convnet_forward(ace_convnet* net, int n, const float* x, int nb, float* y);
/* Loss L = 1/2 sum (net(x) - t)^2 / (nb n^3) and its gradient with respect to the BF16
 * compute weights; *loss and grad[ACE_NET_PARAMS] are host (either may be NULL). */
int convnet_gradient(ace_convnet* net, int n, const float* x, const float* t, int nb,
                     double* loss, float* grad);
/* `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on the loss above
 * over `count` (input, target) volume pairs (device).  flags & ACE_TRAIN_RANDOM: each step
 * draws `batch` pairs (SplitMix64 of seed, step and slot) with random sign; otherwise batch
 * must equal count and every step uses all pairs in order.  loss_hist (host, steps, may be
 * NULL) receives the loss of each step before its update.  Synchronises. */
#define ACE_TRAIN_RANDOM 1
int convnet_train(ace_convnet* net, int n, const float* inputs, const float* targets, int count,
                  int steps, int batch, double lr, unsigned long long seed, int flags,
                  double* loss_hist);

/* ---- block eigensolver and SCF -------------------------------------------------------- */
/* Preconditioners: NONE (residuals as they are), KINETIC (see kinetic_precondition; the
 * recommended default), NET (the network's output on the RMS-normalised residuals as a block of
 * its own beside the kinetic block, so the kinetic directions remain available as the
 * fallback; needs 3k <= 64).  NET saves iterations but, with its larger Rayleigh-Ritz order and
 * the network's own cost, has not saved time on the systems measured. */
enum { ACE_PRECOND_NONE = 0, ACE_PRECOND_KINETIC = 1, ACE_PRECOND_NET = 2 };

typedef struct ace_eig_opts {
  int max_steps;     /* eigensolver steps (per SCF iteration in scf_run) */
  double tol;        /* stop when every residual |F x - lambda x| (dV norm) < tol (0: off) */
  int precond;       /* ACE_PRECOND_* */
  double shift;      /* kinetic preconditioner shift (hartree) */
  int sweeps;        /* kinetic preconditioner Jacobi sweeps (>= 1) */
  double omega;      /* kinetic preconditioner damping (0 < omega < 2) */
  ace_convnet* net;  /* learned preconditioner (ACE_PRECOND_NET) */
} ace_eig_opts;

/*
 * k lowest eigenpairs of F = T + v_local (+ K_ACE with nxi vectors xi, Eq. (13), if nxi > 0)
 * by LOBPCG: Rayleigh-Ritz over [X, M R, P] (current vectors, preconditioned residuals --
 * two blocks with ACE_PRECOND_NET --, previous directions; P is left out when the order would
 * pass 64), orthonormalisation in FP64 (Cholesky when the overlap is provably well conditioned,
 * else canonical with small directions dropped); in FP32 storage F x is recomputed every 10
 * steps.
 * The non-self-consistent run with a fixed Hamiltonian of Sec. 3.1.
 * phi: k start vectors, overwritten by the Ritz vectors (dV-orthonormal); eigval, resnorm
 * (host, k, may be NULL); *steps (host, may be NULL) = steps taken.  Synchronises.
 */
int fock_lowest_states(ace_ctx* ctx, const void* v_local, const void* xi, int nxi, void* phi,
                       int k, const ace_eig_opts* opts, double* eigval, double* resnorm,
                       int* steps);

/*
 * Unoccupied orbitals by the non-self-consistent run of Sec. 3.1: the Hamiltonian
 * F = T + v_local + K[phi_occ] is fixed; each outer iteration rebuilds ACE over the occupied
 * and the current unoccupied orbitals (ace_build_targets) and takes up to opts->max_steps
 * LOBPCG steps for the nv lowest states orthogonal to the occupied ones (phi_occ must be
 * converged, dV-orthonormal eigenvectors of F).  Stops when the residuals of the lowest nconv
 * states (0: all nv; the others are buffer states) measured right after a rebuild -- where
 * K_ACE equals K on the current vectors -- are below opts->tol, or after max_outer rebuilds.
 * psi: nv start vectors (device), overwritten by the unoccupied orbitals; eigval, resnorm
 * (host, nv), *outer, *steps (host) may be NULL.  no + nv <= ACE_MAX_ORBITALS.  Synchronises.
 */
int unocc_states(ace_ctx* ctx, const void* v_local, const void* phi_occ, int no, void* psi,
                 int nv, int nconv, const ace_eig_opts* opts, int max_outer, double* eigval,
                 double* resnorm, int* outer, int* steps);

/* Energy terms of k doubly occupied orbitals: energy[5] (host) = total, kinetic, external,
 * Hartree, exchange (see above).  Synchronises. */
int scf_energies(ace_ctx* ctx, const void* v_ext, const void* phi, int k, double* energy);

typedef struct ace_scf_opts {
  ace_eig_opts eig;  /* eigensolver per iteration; eig.tol also enters the stop test.  When
                        the residuals after eig.max_steps steps exceed eig.tol and ten times
                        the previous density error, up to 3 * max_steps more follow */
  double alpha;      /* states mixing q_{N+1} = alpha q_{N-1} + (1 - alpha) q_N, Eq. (14) */
  double tol;        /* relative density error stop, Eq. (15) */
  int max_iter;
  float* rec_in;     /* optional (device, rec_cap volumes, ACE_R32 only): residuals / RMS */
  float* rec_tgt;    /* optional: the current vectors / RMS of their residuals */
  int rec_cap;
  int rec_stride;    /* record the residual block of every rec_stride-th evaluation (>= 1) */
} ace_scf_opts;

typedef struct ace_scf_result {
  double energy[5];      /* as scf_energies, of the returned orbitals */
  double density_error;  /* Eq. (15) of the last iteration */
  double max_residual;   /* largest eigensolver residual of the last iteration */
  int iterations;
  int eig_steps;         /* eigensolver steps over all iterations */
  int converged;
  int rec_count;         /* recorded (residual, vector) pairs */
} ace_scf_result;

/*
 * Closed-shell HF SCF from the k orbitals phi (device, overwritten).  Each iteration:
 * rho_in and v_H from phi, ACE rebuilt from phi, eig.max_steps eigensolver steps from phi,
 * the new set rotated onto the old (orthogonal Procrustes), the density error of Eq. (15)
 * between the two densities, then the states mixed by Eq. (14) and re-orthonormalised
 * (Loewdin).  Stops when the error is below tol and every residual below eig.tol; phi then
 * holds the rotated new set, else the last mixed set.  res (host) and eigval (host, k) /
 * err_hist (host, max_iter), which may be NULL, receive the results.  Synchronises.
 */
int scf_run(ace_ctx* ctx, const void* v_ext, void* phi, int k, const ace_scf_opts* opts,
            ace_scf_result* res, double* eigval, double* err_hist);

/* Training targets of the learned preconditioner from converged orbitals phi (k):
 * tgt_v <- Phi (Phi^T tgt_v dV) - tgt_v for count FP32 volumes (ACE_R32 contexts), i.e.
 * the correction that takes a recorded vector onto the converged occupied space, then
 * scaled to unit RMS (the eigensolver uses only its direction).  Synchronises. */
int precond_targets(ace_ctx* ctx, const void* phi, int k, float* tgt, int count);

/* Static message for a return code. */
const char* ace_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* ACE_H */
