// Launchers of the grid kernels of the SCF driver (scf.hip): the local part of the Fock
// operator (Eq. (1)), densities, the kinetic preconditioner, block combinations of grid
// vectors and the small dense steps of the block eigensolver.  Grid vectors are real, stored
// [vector][x][y][z] in float or double (fp64 selects); small matrices are FP64 row-major.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace ace {

constexpr int kCombineMax = 64;  // largest number of input vectors of one combination

// y_v = (acc ? y_v : 0) + T x_v + vloc x_v for v < nv (vloc may be null: kinetic only).
// T = -1/2 times the fourth-order central-difference Laplacian, orbitals zero outside the box.
void launch_fock_local(bool fp64, const void* x, int nv, int n, double h, const void* vloc,
                       int acc, void* y, hipStream_t s);

// Kinetic preconditioner: z = (T + shift)^{-1} r approximated by `sweeps` damped-Jacobi steps
// from z = r / (d + shift) (d = diagonal of T).  tmp: nv grid vectors of scratch.
void launch_precond_kinetic(bool fp64, const void* r, int nv, int n, double h, double shift,
                            int sweeps, double omega, void* z, void* tmp, hipStream_t s);

// rho = 2 sum_i x_i^2 (closed shell)
void launch_density(bool fp64, const void* x, int k, size_t ng, void* rho, hipStream_t s);

// out = alpha a + beta b over count elements (b may be null: out = alpha a)
void launch_axpby(bool fp64, const void* a, const void* b, double alpha, double beta,
                  size_t count, void* out, hipStream_t s);

// out[0] = scale * sum |a - b| (FP64 partial sums, fixed order); part: kAbsParts doubles
constexpr int kAbsParts = 512;
void launch_abs_diff_sum(bool fp64, const void* a, const void* b, size_t count, double scale,
                         double* part, double* out, hipStream_t s);

// out_j = sum_{i < mb} C[i * ldc + j] V_i for j < kout (mb <= kCombineMax, kout <= 32);
// out must not overlap V.
void launch_combine(bool fp64, const void* V, int mb, size_t ng, const double* C, int ldc,
                    int kout, void* out, hipStream_t s);

// R_j = HX_j - lam_j X_j
void launch_residual_grid(bool fp64, const void* X, const void* HX, const double* lam, int k,
                          size_t ng, void* R, hipStream_t s);

// inout_v = sum_k Phi_k z[k * nv + v] - inout_v  (complement projection; z FP64, scaled),
// k <= 64
void launch_project_complement(bool fp64, const void* phi, int k, const double* z, int nv,
                               size_t ng, void* inout, hipStream_t s);
// inout_v -= sum_k Phi_k z[k * nv + v]  (removal of the span of Phi), k <= 64
void launch_project_out(bool fp64, const void* phi, int k, const double* z, int nv, size_t ng,
                        void* inout, hipStream_t s);

// dst_v = scale_v * src_v, converted to float (dst is always float); scale: nv doubles
void launch_scale_to_f32(bool fp64, const void* src, const double* scale, int nv, size_t ng,
                         float* dst, hipStream_t s);
// x_v *= scale_v in place (nv vectors of ng points)
void launch_scale_inplace(bool fp64, void* x, const double* scale, int nv, size_t ng,
                          hipStream_t s);
// dst[e] = value for e < count
void launch_fill(bool fp64, double value, size_t count, void* dst, hipStream_t s);
// dst_v = src_v (float) converted to the grid precision
void launch_from_f32(bool fp64, const float* src, size_t count, void* dst, hipStream_t s);

// scale_v = 1 / sqrt(max(G[v * ld + v] / ng, tiny)) (inverse RMS from a Gram diagonal)
void launch_inv_rms(const double* G, int ld, int nv, double ng, double* scale, hipStream_t s);

// ---- small dense steps (one workgroup each) ----
// D_i = S_ii^{-1/2} (0 if S_ii <= 0); Ss = D S D, Gs = D sym(G) D   (m x m)
void launch_sym_scale(const double* S, const double* G, int m, double* Ss, double* Gs,
                      double* D, hipStream_t s);
// T[:, j] = U[:, j] / sqrt(w_j) if w_j > rel * max(w) else 0   (w ascending)
void launch_canon(const double* w, const double* U, int m, double rel, double* T, hipStream_t s,
                  const int* skip = nullptr);
// for every dropped j (w_j <= rel * max(w)): A[j][j] = 1 + max_i sum_l |A[i][l]|, above the
// spectrum of the kept block
void launch_drop_diag(double* A, int m, const double* w, double rel, hipStream_t s);
// out = U diag(f(w)) U^T, f(w) = w^{-1/2} (w > 0; else 0)
void launch_inv_sqrt_from_eig(const double* w, const double* U, int m, double* out,
                              hipStream_t s);
// C[i][j] *= D[i] for i < m, j < k (rows of a coefficient matrix, ld ldc)
void launch_scale_coeff_rows(double* C, int ldc, const double* D, int m, int k, hipStream_t s);
// zero rows [0, r) of C (m x k, ld ldc)
void launch_zero_rows(double* C, int ldc, int r, int k, hipStream_t s);
// out[j] = A[j * ld + j]
void launch_diag(const double* A, int ld, int m, double* out, hipStream_t s);

}  // namespace ace
