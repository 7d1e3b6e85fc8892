// Small dense FP64 linear algebra (linalg.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace ace {

constexpr int kJacobiMax = 64;  // largest order of the one-workgroup Jacobi eigensolver

// C = alpha op(A) op(B) + beta C (row-major; ta / tb select the transpose)
void launch_dgemm(int ta, int tb, int M, int N, int K, double alpha, const double* A, int lda,
                  const double* B, int ldb, double beta, double* C, int ldc, hipStream_t s);

// eigenvalues ascending in w[n], eigenvectors in the columns of V (ld ldv); n <= kJacobiMax
// (a non-null skip pointing at a nonzero device int makes the launch a no-op)
void launch_jacobi(int n, const double* A, int lda, double* w, double* V, int ldv,
                   int max_sweeps, double tol, hipStream_t s, const int* skip = nullptr);
// Cholesky orthonormalisation from a Gram matrix S (n <= kJacobiMax): T = L^{-T} with
// S = L L^T, accepted (*ok = 1, w[0:n] = 1, T written) only when the smallest eigenvalue of S
// is provably above thr; otherwise *ok = 0 and T, w untouched.  ok is device memory.
void launch_chol_orth(int n, const double* S, double thr, double* T, double* w, int* ok,
                      hipStream_t s);

// Davidson helpers (rows of length n are vectors)
void launch_add_diag(const double* C, const double* d, int n, double* A, hipStream_t s);
void launch_residual(const double* X, const double* AX, const double* theta, int n, int k,
                     double* R, double* norm2, hipStream_t s);
void launch_dav_precond(const double* R, const double* d, const double* theta, int n, int k,
                        double* T, hipStream_t s);
void launch_scale_rows(double* Y, const double* sc, int n, int k, hipStream_t s);

// full TDHF helpers: P = C + B + diag(d), M = C - B + diag(d)
void launch_pm(const double* C, const double* B, const double* d, int n, double* P, double* M,
               hipStream_t s);
// blocked Cholesky A = L L^T in place (lower; upper set to zero); info[0] (device, zeroed by
// the caller) = first non-positive pivot + 1
void launch_potrf(double* A, int n, int lda, int* info, hipStream_t s);
// v <- sqrt(max(v, 0)), sinv <- 1 / sqrt(v) of the new v (k values)
void launch_sqrt_and_inv(double* v, double* sinv, int k, hipStream_t s);

}  // namespace ace
