// Small dense FP64 linear algebra used by the eigensolver drivers built on top of the ACE
// engine (subspace Rayleigh-Ritz of the SCF eigensolver, Davidson for the Tamm-Dancoff
// problem): a tiled GEMM with transpose flags and a one-workgroup parallel-order Jacobi
// eigensolver for symmetric matrices of order <= 64.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "linalg.hpp"

namespace ace {

namespace {

// C = alpha op(A) op(B) + beta C, row-major; op(X) = X or X^T.  64 x 64 tiles, 256 threads,
// 4 x 4 outputs per thread, K staged 16 at a time through LDS.
constexpr int GT = 64, GK = 16;

__global__ __launch_bounds__(256) void k_dgemm(int ta, int tb, int M, int N, int K, double alpha,
                                               const double* __restrict__ A, int lda,
                                               const double* __restrict__ B, int ldb,
                                               double beta, double* __restrict__ C, int ldc) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += GK) {
    for (int e = threadIdx.x; e < GT * GK; e += 256) {
      const int r = e / GK, kk = e % GK;  // tile row r, depth kk
      const int m = m0 + r, n = n0 + r, k = k0 + kk;
      double av = 0.0, bv = 0.0;
      if (m < M && k < K) av = ta ? A[(size_t)k * lda + m] : A[(size_t)m * lda + k];
      if (n < N && k < K) bv = tb ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n];
      As[kk][r] = av;
      Bs[kk][r] = bv;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + ty + 16 * i, n = n0 + tx + 16 * j;
      if (m < M && n < N) {
        double* c = C + (size_t)m * ldc + n;
        *c = alpha * acc[i][j] + (beta == 0.0 ? 0.0 : beta * *c);
      }
    }
}

// Symmetric eigendecomposition by the cyclic Jacobi method in round-robin (tournament)
// order: each round rotates n/2 disjoint index pairs at once.  The rotations of a round are
// computed once (one thread per pair); the two-sided update is then one pass over 2x2 blocks:
// the block (rows of pair k, columns of pair l) becomes R_k B R_l^T with R = [[c, -s], [s, c]],
// and the eigenvector columns of each pair rotate.  One workgroup; matrix and eigenvectors in
// LDS.  Output: w ascending, V[i][k] = component i of eigenvector k (row-major, leading
// dimension ldv).
constexpr int JMAX = 64;
constexpr int JT = 1024;

// 1 / x and 1 / sqrt(x) in FP64 from the hardware estimates plus two Newton steps
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * fma(-x, r, 2.0);
  r = r * fma(-x, r, 2.0);
  return r;
}
__device__ __forceinline__ double rsq_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-0.5 * x * r, r, 1.5);
  r = r * fma(-0.5 * x * r, r, 1.5);
  return r;
}

__global__ __launch_bounds__(JT) void k_jacobi(int n, const double* __restrict__ Ain, int lda,
                                               double* __restrict__ w, double* __restrict__ V,
                                               int ldv, int max_sweeps, double tol,
                                               const int* __restrict__ skip) {
  if (skip != nullptr && *skip) return;  // the caller's result is already in place
  __shared__ double a[JMAX][JMAX + 1];
  __shared__ double v[JMAX][JMAX + 1];
  __shared__ double cs[JMAX / 2], sn[JMAX / 2];
  __shared__ int pp[JMAX / 2], qq[JMAX / 2];
  __shared__ double red[2][JT / 64];
  __shared__ int rank_s[JMAX];
  const int m = n + (n & 1);  // even order; a padding index acts as an isolated zero row
  const int h = m / 2;
  for (int e = threadIdx.x; e < m * m; e += JT) {
    const int i = e / m, j = e % m;
    double x = 0.0;
    if (i < n && j < n) x = 0.5 * (Ain[(size_t)i * lda + j] + Ain[(size_t)j * lda + i]);
    a[i][j] = x;
    v[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = threadIdx.x; e < m * m; e += JT) {
      const int i = e / m, j = e % m;
      const double x = a[i][j] * a[i][j];
      tot += x;
      if (i != j) off += x;
    }
    // wavefront butterflies, then the JT / 64 wavefront sums in order (every thread)
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, 64);
      tot += __shfl_xor(tot, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      red[0][threadIdx.x >> 6] = off;
      red[1][threadIdx.x >> 6] = tot;
    }
    __syncthreads();
    double offn = 0.0, totn = 0.0;
    for (int w = 0; w < JT / 64; ++w) {
      offn += red[0][w];
      totn += red[1][w];
    }
    __syncthreads();
    if (offn <= tol * tol * totn || offn == 0.0) break;
    // tournament pairing: position 0 fixed, the others rotate by one each round.  Every thread
    // keeps the indices at the positions of its work items in registers and advances them
    // (no LDS reads, no divisions); at round 0 the index at position pos is pos.
    constexpr int KI = (JMAX / 2 * JMAX / 2 + JMAX * JMAX / 2 + JT - 1) / JT;  // items per thread
    const int nitem = h * h + m * h;
    int ia[KI][4];  // A items: positions k, m-1-k, l, m-1-l; V items: l, m-1-l
#pragma unroll
    for (int u = 0; u < KI; ++u) {
      const int e = threadIdx.x + u * JT;
      const int k = e < h * h ? e / h : (e - h * h) / m;
      const int l = e < h * h ? e % h : 0;
      ia[u][0] = k;
      ia[u][1] = m - 1 - k;
      ia[u][2] = l;
      ia[u][3] = m - 1 - l;
    }
    int ra = (int)threadIdx.x, rb = m - 1 - (int)threadIdx.x;  // rotation phase (thread < h)
    auto adv = [&](int x) { return x == 0 ? 0 : (x == m - 1 ? 1 : x + 1); };
    for (int round = 0; round < m - 1; ++round) {
      if ((int)threadIdx.x < h) {
        const int k = threadIdx.x;
        const int p = ra < rb ? ra : rb, q = ra < rb ? rb : ra;
        const double apq = a[p][q];
        double c = 1.0, sv = 0.0;
        if (fabs(apq) > 1e-290) {  // below that the rotation is the identity to rounding
          // t = sign(theta) / (|theta| + sqrt(theta^2 + 1)), c = 1 / sqrt(t^2 + 1), s = t c;
          // hardware reciprocal / reciprocal square root refined by two Newton steps each
          // (full FP64 accuracy, much shorter dependency chains than IEEE division)
          const double theta = (a[q][q] - a[p][p]) * rcp_nr(2.0 * apq);
          const double at = fabs(theta);
          double t;
          if (at > 1e150) {
            t = 0.5 / theta;
          } else {
            const double r2 = theta * theta + 1.0;
            t = (theta >= 0.0 ? 1.0 : -1.0) * rcp_nr(at + r2 * rsq_nr(r2));
          }
          c = rsq_nr(t * t + 1.0);
          sv = t * c;
        }
        cs[k] = c;
        sn[k] = sv;
        ra = adv(ra);
        rb = adv(rb);
      }
      __syncthreads();
      // A <- J^T A J by 2x2 blocks; V <- V J by column pairs
#pragma unroll
      for (int u = 0; u < KI; ++u) {
        const int e = threadIdx.x + u * JT;
        if (e < nitem) {
          const int a0 = ia[u][0], b0 = ia[u][1];
          const int p = a0 < b0 ? a0 : b0, q = a0 < b0 ? b0 : a0;
          if (e < h * h) {
            const int k = e / h, l = e % h;
            const int a1 = ia[u][2], b1 = ia[u][3];
            const int r = a1 < b1 ? a1 : b1, t = a1 < b1 ? b1 : a1;
            const double ck = cs[k], sk = sn[k], cl = cs[l], sl = sn[l];
            const double b00 = a[p][r], b01 = a[p][t], b10 = a[q][r], b11 = a[q][t];
            const double r00 = ck * b00 - sk * b10, r01 = ck * b01 - sk * b11;
            const double r10 = sk * b00 + ck * b10, r11 = sk * b01 + ck * b11;
            a[p][r] = cl * r00 - sl * r01;
            a[p][t] = sl * r00 + cl * r01;
            a[q][r] = cl * r10 - sl * r11;
            a[q][t] = sl * r10 + cl * r11;
          } else {
            const int f = e - h * h;
            const int l = f / m, i = f % m;
            const double c = cs[l], sv = sn[l];
            const double vx = v[i][p], vy = v[i][q];
            v[i][p] = c * vx - sv * vy;
            v[i][q] = sv * vx + c * vy;
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) ia[u][j] = adv(ia[u][j]);
      }
      __syncthreads();
    }
  }
  // ascending order: rank of each eigenvalue (ties broken by index)
  for (int i = threadIdx.x; i < n; i += JT) {
    int r = 0;
    for (int j = 0; j < n; ++j)
      if (a[j][j] < a[i][i] || (a[j][j] == a[i][i] && j < i)) ++r;
    rank_s[i] = r;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += JT) {
    const int i = e / n, k = e % n;  // component i of eigenvector k (unsorted)
    V[(size_t)i * ldv + rank_s[k]] = v[i][k];
  }
  for (int k = threadIdx.x; k < n; k += JT) w[rank_s[k]] = a[k][k];
}

// Orthonormalisation of a basis from its Gram matrix S (n <= JMAX, symmetrised on load) by
// Cholesky: S = L L^T, T = L^{-T}, so that T^T S T = I.  Accepted only when the smallest
// eigenvalue of S is provably above thr: lambda_min >= 1 / tr(S^{-1}) = 1 / ||L^{-1}||_F^2.  On
// acceptance T (row-major n x n) is written, w[0:n] = 1 and *ok = 1; otherwise only *ok = 0.
// Right-looking elimination, one barrier per column: step j updates the Schur complement of
// the pivot d_j = l[j][j] and, in the same pass, eliminates column j from the right-hand side
// Y (started at I, lower triangular): y_i -= l_ij y_j / d_j for i > j.  Then
// L^{-1} = diag(d)^{-1/2} Y, and L itself is never formed.
__global__ __launch_bounds__(JT) void k_chol_orth(int n, const double* __restrict__ S, double thr,
                                                  double* __restrict__ T, double* __restrict__ w,
                                                  int* __restrict__ ok) {
  __shared__ double l[JMAX][JMAX + 1];
  __shared__ double y[JMAX][JMAX + 1];
  __shared__ double piv[JMAX];
  __shared__ double red[JT / 64];
  for (int e = threadIdx.x; e < n * n; e += JT) {
    const int i = e / n, j = e % n;
    l[i][j] = 0.5 * (S[(size_t)i * n + j] + S[(size_t)j * n + i]);
    y[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  bool good = true;
  for (int j = 0; j < n; ++j) {
    const double d = l[j][j];  // same value in every thread: uniform control flow
    if (!(d > 0.0) || !isfinite(d)) {
      good = false;
      break;
    }
    const double rd = 1.0 / d;
    const int t = n - j - 1, c1 = j + 1;
    // step j writes rows / columns > j of l and rows > j of y; it reads only column j of l
    // and row j of y, which no thread writes in this step
    for (int e = threadIdx.x; e < t * t + t * c1; e += JT) {
      if (e < t * t) {
        const int i = j + 1 + e / t, k = j + 1 + e % t;
        if (k <= i) l[i][k] -= l[i][j] * l[k][j] * rd;
      } else {
        const int f = e - t * t;
        const int i = j + 1 + f / c1, c = f % c1;
        y[i][c] -= l[i][j] * y[j][c] * rd;
      }
    }
    if (threadIdx.x == 0) piv[j] = d;
    __syncthreads();
  }
  if (!good) {
    if (threadIdx.x == 0) *ok = 0;
    return;
  }
  // ||L^{-1}||_F^2 = sum_i |y_i|^2 / d_i (y lower triangular)
  double fr = 0.0;
  for (int e = threadIdx.x; e < n * n; e += JT) {
    const int i = e / n, c = e % n;
    if (c <= i) fr += y[i][c] * y[i][c] / piv[i];
  }
  for (int o = 32; o > 0; o >>= 1) fr += __shfl_xor(fr, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = fr;
  __syncthreads();
  double tr = 0.0;
  for (int v = 0; v < JT / 64; ++v) tr += red[v];
  const bool accept = isfinite(tr) && tr * thr < 1.0;
  if (accept) {
    // T[i][j] = L^{-1}[j][i] = y[j][i] / sqrt(d_j) (zero above the diagonal of L^{-1})
    for (int e = threadIdx.x; e < n * n; e += JT) {
      const int i = e / n, j = e % n;
      T[e] = i <= j ? y[j][i] / sqrt(piv[j]) : 0.0;
    }
    for (int j = threadIdx.x; j < n; j += JT) w[j] = 1.0;
  }
  if (threadIdx.x == 0) *ok = accept ? 1 : 0;
}

// A = C + diag(d) (copy); n x n row-major
__global__ void k_add_diag(const double* __restrict__ C, const double* __restrict__ d, int n,
                           double* __restrict__ A) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (size_t)n * n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    A[e] = C[e] + (i == j ? d[i] : 0.0);
  }
}

// R_j = AX_j - theta_j X_j and the squared norms |R_j|^2 (one block per row j)
__global__ void k_residual(const double* __restrict__ X, const double* __restrict__ AX,
                           const double* __restrict__ theta, int n, double* __restrict__ R,
                           double* __restrict__ norm2) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double r = AX[(size_t)j * n + i] - theta[j] * X[(size_t)j * n + i];
    R[(size_t)j * n + i] = r;
    s += r * r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) norm2[j] = red[0];
}

// Davidson correction T_j = R_j / (theta_j - d) (denominator kept away from zero)
__global__ void k_dav_precond(const double* __restrict__ R, const double* __restrict__ d,
                              const double* __restrict__ theta, int n, int k,
                              double* __restrict__ T) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (size_t)n * k;
       e += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(e / n), i = (int)(e % n);
    double den = theta[j] - d[i];
    if (fabs(den) < 1e-6) den = den < 0.0 ? -1e-6 : 1e-6;
    T[e] = R[e] / den;
  }
}

// rows of Y scaled: Y_j *= s_j
__global__ void k_scale_rows(double* __restrict__ Y, const double* __restrict__ s, int n, int k) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (size_t)n * k;
       e += (size_t)gridDim.x * blockDim.x)
    Y[e] *= s[e / n];
}

// P = C + B + diag(d), M = C - B + diag(d) (n x n row-major)
__global__ void k_pm(const double* __restrict__ C, const double* __restrict__ B,
                     const double* __restrict__ d, int n, double* __restrict__ P,
                     double* __restrict__ M) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (size_t)n * n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    const double dg = i == j ? d[i] : 0.0;
    P[e] = C[e] + B[e] + dg;
    M[e] = C[e] - B[e] + dg;
  }
}

// Blocked Cholesky A = L L^T (lower, in place), panel width kPanel.
constexpr int kPanel = 64;

// factor the diagonal block A[j0:j0+nb, j0:j0+nb] in LDS; info[0] = first failing column + 1
__global__ __launch_bounds__(256) void k_potrf_panel(double* __restrict__ A, int lda, int j0,
                                                     int nb, int* __restrict__ info) {
  __shared__ double a[kPanel][kPanel + 1];
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int i = e / nb, j = e % nb;
    a[i][j] = A[(size_t)(j0 + i) * lda + j0 + j];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (threadIdx.x == 0) {
      double p = a[j][j];
      if (!(p > 0.0)) {
        if (info && info[0] == 0) info[0] = j0 + j + 1;
        p = 1.0;
      }
      a[j][j] = sqrt(p);
    }
    __syncthreads();
    const double inv = 1.0 / a[j][j];
    for (int i = j + 1 + threadIdx.x; i < nb; i += blockDim.x) a[i][j] *= inv;
    __syncthreads();
    const int m = nb - j - 1;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
      const int i = j + 1 + e / m, k = j + 1 + e % m;
      if (k <= i) a[i][k] -= a[i][j] * a[k][j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int i = e / nb, j = e % nb;
    if (j <= i) A[(size_t)(j0 + i) * lda + j0 + j] = a[i][j];
  }
}

// rows r >= j0 + nb of the panel columns: solve X L11^T = A21 by forward substitution
__global__ __launch_bounds__(256) void k_trsm_rows(double* __restrict__ A, int lda, int j0, int nb,
                                                   int n) {
  __shared__ double l[kPanel][kPanel + 1];
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int i = e / nb, j = e % nb;
    l[i][j] = j <= i ? A[(size_t)(j0 + i) * lda + j0 + j] : 0.0;
  }
  __syncthreads();
  const int r = j0 + nb + blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double* row = A + (size_t)r * lda + j0;
  double x[kPanel];
#pragma unroll
  for (int k = 0; k < kPanel; ++k) {
    if (k < nb) {
      double sv = row[k];
#pragma unroll
      for (int q = 0; q < k; ++q) sv -= x[q] * l[k][q];
      x[k] = sv / l[k][k];
    } else {
      x[k] = 0.0;
    }
  }
#pragma unroll
  for (int k = 0; k < kPanel; ++k)
    if (k < nb) row[k] = x[k];
}

__global__ void k_zero_upper(double* __restrict__ A, int n, int lda) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (size_t)n * n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / n), j = (int)(e % n);
    if (j > i) A[(size_t)i * lda + j] = 0.0;
  }
}

// v[i] = sqrt(max(v[i], 0)); s[i] = 1 / sqrt(v[i]) after the root (0 where v = 0)
__global__ void k_sqrt_and_inv(double* __restrict__ v, double* __restrict__ s, int k) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const double w = sqrt(fmax(v[i], 0.0));
    v[i] = w;
    s[i] = w > 0.0 ? 1.0 / sqrt(w) : 0.0;
  }
}

}  // namespace

void launch_add_diag(const double* C, const double* d, int n, double* A, hipStream_t s) {
  k_add_diag<<<256, 256, 0, s>>>(C, d, n, A);
}

void launch_residual(const double* X, const double* AX, const double* theta, int n, int k,
                     double* R, double* norm2, hipStream_t s) {
  k_residual<<<k, 256, 0, s>>>(X, AX, theta, n, R, norm2);
}

void launch_dav_precond(const double* R, const double* d, const double* theta, int n, int k,
                        double* T, hipStream_t s) {
  k_dav_precond<<<256, 256, 0, s>>>(R, d, theta, n, k, T);
}

void launch_scale_rows(double* Y, const double* sc, int n, int k, hipStream_t s) {
  k_scale_rows<<<256, 256, 0, s>>>(Y, sc, n, k);
}

void launch_dgemm(int ta, int tb, int M, int N, int K, double alpha, const double* A, int lda,
                  const double* B, int ldb, double beta, double* C, int ldc, hipStream_t s) {
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  k_dgemm<<<grid, 256, 0, s>>>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

void launch_jacobi(int n, const double* A, int lda, double* w, double* V, int ldv,
                   int max_sweeps, double tol, hipStream_t s, const int* skip) {
  k_jacobi<<<1, JT, 0, s>>>(n, A, lda, w, V, ldv, max_sweeps, tol, skip);
}

void launch_chol_orth(int n, const double* S, double thr, double* T, double* w, int* ok,
                      hipStream_t s) {
  k_chol_orth<<<1, JT, 0, s>>>(n, S, thr, T, w, ok);
}

}  // namespace ace

namespace ace {

void launch_pm(const double* C, const double* B, const double* d, int n, double* P, double* M,
               hipStream_t s) {
  k_pm<<<512, 256, 0, s>>>(C, B, d, n, P, M);
}

void launch_potrf(double* A, int n, int lda, int* info, hipStream_t s) {
  for (int j0 = 0; j0 < n; j0 += kPanel) {
    const int nb = std::min(kPanel, n - j0);
    k_potrf_panel<<<1, 256, 0, s>>>(A, lda, j0, nb, info);
    const int m = n - j0 - nb;
    if (m > 0) {
      k_trsm_rows<<<(m + 255) / 256, 256, 0, s>>>(A, lda, j0, nb, n);
      const double* l21 = A + (size_t)(j0 + nb) * lda + j0;
      launch_dgemm(0, 1, m, m, nb, -1.0, l21, lda, l21, lda, 1.0,
                   A + (size_t)(j0 + nb) * lda + j0 + nb, lda, s);
    }
  }
  k_zero_upper<<<512, 256, 0, s>>>(A, n, lda);
}

void launch_sqrt_and_inv(double* v, double* sinv, int k, hipStream_t s) {
  k_sqrt_and_inv<<<1, 64, 0, s>>>(v, sinv, k);
}

}  // namespace ace
