// Grid kernels of the closed-shell SCF driver (paper Eq. (1) with the readings stated in
// scf.hpp): the local Fock part (fourth-order finite-difference kinetic energy plus a local
// potential), densities, the damped-Jacobi kinetic preconditioner, block combinations of
// grid vectors, and the one-workgroup FP64 steps of the block eigensolver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <initializer_list>

#include "scf.hpp"

namespace ace {

namespace {

constexpr int kT = 256;

// Fourth-order central second difference on one axis: (-1/12, 4/3, -5/2, 4/3, -1/12) / h^2.
// T = -1/2 Laplacian: centre 3 * 5/4 / h^2, first neighbours -2/3 / h^2, second 1/24 / h^2.
// The weights sum to zero, and the operator is evaluated in that form,
//   T x = c1 (n1 - 6 x) + c2 (n2 - 6 x)   (n1, n2: sums of the first / second neighbours),
// so that rounding c1 and c2 only scales the two differences: with the weights rounded
// separately (c0 x + c1 n1 + c2 n2) they no longer sum to zero in FP32: at h = 0.2 the
// operator gains a constant 3.6e-6 Ha, and each doubly occupied orbital's kinetic energy
// 7.2e-6 Ha.  FP32 also carries c1 and c2 as hi + lo pairs (the products rounded once).
// c0 (the diagonal) is kept for the Jacobi preconditioner.
template <typename T>
struct Fd4 {
  T c0, c1, c2, c1l, c2l;
  explicit Fd4(double h) {
    const double ih2 = 1.0 / (h * h);
    const double d1 = -2.0 / 3.0 * ih2, d2 = 1.0 / 24.0 * ih2;
    c0 = T(3.75 * ih2);
    c1 = T(d1);
    c2 = T(d2);
    c1l = T(d1 - double(c1));
    c2l = T(d2 - double(c2));
  }
};

// c1 * d1 + c2 * d2 with the constants' low parts
__device__ __forceinline__ double fd4_comb(double d1, double d2, const Fd4<double>& f) {
  return f.c1 * d1 + f.c2 * d2;
}
__device__ __forceinline__ float fd4_comb(float d1, float d2, const Fd4<float>& f) {
  return fmaf(d1, f.c1, fmaf(d2, f.c2, fmaf(d1, f.c1l, d2 * f.c2l)));
}

// value of x at (coordinate + off) along an axis of stride `stride`, zero outside the box;
// the load itself is always in bounds (clamped to the centre point)
template <typename T>
__device__ __forceinline__ T nb(const T* __restrict__ xv, size_t r, int coord, int n,
                                long long stride, int off) {
  const int q = coord + off;
  const bool ok = (unsigned)q < (unsigned)n;
  const T v = xv[ok ? (long long)r + off * stride : (long long)r];
  return ok ? v : T(0);
}

template <typename T>
__device__ __forceinline__ T kinetic_at(const T* __restrict__ xv, size_t r, int n,
                                        const Fd4<T>& f) {
  const int iz = (int)(r % n), iy = (int)((r / n) % n), ix = (int)(r / ((size_t)n * n));
  const long long sy = n, sx = (long long)n * n;
  const T n1 = nb(xv, r, iz, n, 1, -1) + nb(xv, r, iz, n, 1, 1) + nb(xv, r, iy, n, sy, -1) +
               nb(xv, r, iy, n, sy, 1) + nb(xv, r, ix, n, sx, -1) + nb(xv, r, ix, n, sx, 1);
  const T n2 = nb(xv, r, iz, n, 1, -2) + nb(xv, r, iz, n, 1, 2) + nb(xv, r, iy, n, sy, -2) +
               nb(xv, r, iy, n, sy, 2) + nb(xv, r, ix, n, sx, -2) + nb(xv, r, ix, n, sx, 2);
  const T x6 = T(6) * xv[r];
  return fd4_comb(n1 - x6, n2 - x6, f);
}

// FP32, n a multiple of 4: the kinetic operator at the 4 consecutive z-points from r0 (a
// multiple of 4) with 16-byte loads: the z row from three aligned runs, each y / x neighbour
// row as one run (11 loads for 4 points instead of 52).  Same sums in the same order as
// kinetic_at.
__device__ __forceinline__ float4 ld4z(const float* __restrict__ p, bool ok) {
  return ok ? *reinterpret_cast<const float4*>(p) : make_float4(0.f, 0.f, 0.f, 0.f);
}
__device__ __forceinline__ float f4(const float4& v, int i) {
  return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}
__device__ __forceinline__ void kinetic_at4(const float* __restrict__ xv, size_t r0, int n,
                                            const Fd4<float>& f, float out[4]) {
  const int iz = (int)(r0 % n), iy = (int)((r0 / n) % n), ix = (int)(r0 / ((size_t)n * n));
  const size_t sy = n, sx = (size_t)n * n;
  const float4 zl = ld4z(xv + r0 - (iz >= 4 ? 4 : 0), iz >= 4);
  const float4 zc = ld4z(xv + r0, true);
  const float4 zh = ld4z(xv + r0 + (iz + 4 < n ? 4 : 0), iz + 4 < n);
  const float4 ym1 = ld4z(xv + (iy >= 1 ? r0 - sy : r0), iy >= 1);
  const float4 yp1 = ld4z(xv + (iy + 1 < n ? r0 + sy : r0), iy + 1 < n);
  const float4 ym2 = ld4z(xv + (iy >= 2 ? r0 - 2 * sy : r0), iy >= 2);
  const float4 yp2 = ld4z(xv + (iy + 2 < n ? r0 + 2 * sy : r0), iy + 2 < n);
  const float4 xm1 = ld4z(xv + (ix >= 1 ? r0 - sx : r0), ix >= 1);
  const float4 xp1 = ld4z(xv + (ix + 1 < n ? r0 + sx : r0), ix + 1 < n);
  const float4 xm2 = ld4z(xv + (ix >= 2 ? r0 - 2 * sx : r0), ix >= 2);
  const float4 xp2 = ld4z(xv + (ix + 2 < n ? r0 + 2 * sx : r0), ix + 2 < n);
  float w[12];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    w[i] = f4(zl, i);
    w[4 + i] = f4(zc, i);
    w[8 + i] = f4(zh, i);
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const float n1 = w[p + 3] + w[p + 5] + f4(ym1, p) + f4(yp1, p) + f4(xm1, p) + f4(xp1, p);
    const float n2 = w[p + 2] + w[p + 6] + f4(ym2, p) + f4(yp2, p) + f4(xm2, p) + f4(xp2, p);
    const float x6 = 6.f * w[p + 4];
    out[p] = fd4_comb(n1 - x6, n2 - x6, f);
  }
}

__global__ __launch_bounds__(kT) void k_fock_local4(const float* __restrict__ x, int n, size_t ng,
                                                    Fd4<float> f,
                                                    const float* __restrict__ vloc, int acc,
                                                    float* __restrict__ y) {
  const size_t r0 = 4 * ((size_t)blockIdx.x * kT + threadIdx.x);
  if (r0 >= ng) return;
  const size_t off = (size_t)blockIdx.y * ng;
  const float* xv = x + off;
  float s[4];
  kinetic_at4(xv, r0, n, f, s);
  if (vloc) {
    const float4 v = *reinterpret_cast<const float4*>(vloc + r0);
    const float4 xc = *reinterpret_cast<const float4*>(xv + r0);
    s[0] += v.x * xc.x;
    s[1] += v.y * xc.y;
    s[2] += v.z * xc.z;
    s[3] += v.w * xc.w;
  }
  if (acc) {
    const float4 a = *reinterpret_cast<const float4*>(y + off + r0);
    s[0] += a.x;
    s[1] += a.y;
    s[2] += a.z;
    s[3] += a.w;
  }
  *reinterpret_cast<float4*>(y + off + r0) = make_float4(s[0], s[1], s[2], s[3]);
}

__global__ __launch_bounds__(kT) void k_jacobi_sweep4(const float* __restrict__ rr,
                                                      const float* __restrict__ zin,
                                                      float* __restrict__ zout, int n, size_t ng,
                                                      Fd4<float> f, float shift,
                                                      float omega, int first) {
  const size_t r0 = 4 * ((size_t)blockIdx.x * kT + threadIdx.x);
  if (r0 >= ng) return;
  const size_t off = (size_t)blockIdx.y * ng;
  const float inv = 1.f / (f.c0 + shift);
  const float4 rv = *reinterpret_cast<const float4*>(rr + off + r0);
  if (first) {
    *reinterpret_cast<float4*>(zout + off + r0) =
        make_float4(rv.x * inv, rv.y * inv, rv.z * inv, rv.w * inv);
    return;
  }
  const float* zv = zin + off;
  float k[4];
  kinetic_at4(zv, r0, n, f, k);
  const float4 zc = *reinterpret_cast<const float4*>(zv + r0);
  float o[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const float az = k[p] + shift * f4(zc, p);
    o[p] = f4(zc, p) + omega * (f4(rv, p) - az) * inv;
  }
  *reinterpret_cast<float4*>(zout + off + r0) = make_float4(o[0], o[1], o[2], o[3]);
}

template <typename T>
__global__ __launch_bounds__(kT) void k_fock_local(const T* __restrict__ x, int n, size_t ng,
                                                   Fd4<T> f, const T* __restrict__ vloc,
                                                   int acc, T* __restrict__ y) {
  const size_t r = (size_t)blockIdx.x * kT + threadIdx.x;
  if (r >= ng) return;
  const size_t off = (size_t)blockIdx.y * ng;
  const T* xv = x + off;
  T s = kinetic_at(xv, r, n, f);
  if (vloc) s += vloc[r] * xv[r];
  if (acc) s += y[off + r];
  y[off + r] = s;
}

// one damped-Jacobi step for (T + shift) z = r; first: z = r / (d + shift)
template <typename T>
__global__ __launch_bounds__(kT) void k_jacobi_sweep(const T* __restrict__ rr, const T* __restrict__ zin,
                                                     T* __restrict__ zout, int n, size_t ng,
                                                     Fd4<T> f, T shift, T omega, int first) {
  const size_t r = (size_t)blockIdx.x * kT + threadIdx.x;
  if (r >= ng) return;
  const size_t off = (size_t)blockIdx.y * ng;
  const T inv = T(1) / (f.c0 + shift);
  if (first) {
    zout[off + r] = rr[off + r] * inv;
    return;
  }
  const T* zv = zin + off;
  const T az = kinetic_at(zv, r, n, f) + shift * zv[r];
  zout[off + r] = zv[r] + omega * (rr[off + r] - az) * inv;
}

template <typename T>
__global__ __launch_bounds__(kT) void k_density(const T* __restrict__ x, int k, size_t ng,
                                                T* __restrict__ rho) {
  const size_t r = (size_t)blockIdx.x * kT + threadIdx.x;
  if (r >= ng) return;
  T s = T(0);
  for (int i = 0; i < k; ++i) {
    const T v = x[(size_t)i * ng + r];
    s += v * v;
  }
  rho[r] = T(2) * s;
}

template <typename T>
__global__ __launch_bounds__(kT) void k_axpby(const T* __restrict__ a, const T* __restrict__ b,
                                              T alpha, T beta, size_t count, T* __restrict__ out) {
  for (size_t e = (size_t)blockIdx.x * kT + threadIdx.x; e < count; e += (size_t)gridDim.x * kT)
    out[e] = b ? alpha * a[e] + beta * b[e] : alpha * a[e];
}

__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

template <typename T>
__global__ __launch_bounds__(kT) void k_abs_part(const T* __restrict__ a, const T* __restrict__ b,
                                                 size_t count, double* __restrict__ part) {
  __shared__ double red[kT];
  double s = 0.0;
  for (size_t e = (size_t)blockIdx.x * kT + threadIdx.x; e < count; e += (size_t)gridDim.x * kT)
    s += fabs((double)a[e] - (double)b[e]);
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kT) void k_sum_parts(const double* __restrict__ part, int np,
                                                  double scale, double* __restrict__ out) {
  __shared__ double red[kT];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += kT) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = scale * s;
}

// out_j(r) = sum_i C[i][j] V_i(r); coefficients staged in LDS in the grid precision
template <typename T, int KO>
__global__ __launch_bounds__(kT) void k_combine(const T* __restrict__ V, int mb, size_t ng,
                                                const double* __restrict__ C, int ldc, int kout,
                                                T* __restrict__ out) {
  __shared__ T cs[kCombineMax * KO];
  for (int t = threadIdx.x; t < mb * KO; t += kT) {
    const int i = t / KO, j = t % KO;
    cs[t] = j < kout ? (T)C[(size_t)i * ldc + j] : T(0);
  }
  __syncthreads();
  const size_t r = (size_t)blockIdx.x * kT + threadIdx.x;
  if (r >= ng) return;
  T acc[KO];
#pragma unroll
  for (int j = 0; j < KO; ++j) acc[j] = T(0);
  int i = 0;
  for (; i + 4 <= mb; i += 4) {
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = V[(size_t)(i + u) * ng + r];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int j = 0; j < KO; ++j) acc[j] += cs[(i + u) * KO + j] * v[u];
  }
  for (; i < mb; ++i) {
    const T v = V[(size_t)i * ng + r];
#pragma unroll
    for (int j = 0; j < KO; ++j) acc[j] += cs[i * KO + j] * v;
  }
#pragma unroll
  for (int j = 0; j < KO; ++j)
    if (j < kout) out[(size_t)j * ng + r] = acc[j];
}

template <typename T>
__global__ __launch_bounds__(kT) void k_residual_grid(const T* __restrict__ X, const T* __restrict__ HX,
                                                      const double* __restrict__ lam, size_t ng,
                                                      T* __restrict__ R) {
  const size_t r = (size_t)blockIdx.x * kT + threadIdx.x;
  if (r >= ng) return;
  const size_t off = (size_t)blockIdx.y * ng + r;
  R[off] = HX[off] - (T)lam[blockIdx.y] * X[off];
}

constexpr int kPVB = 16;  // vectors per block of the complement projection

template <typename T, int KMAX, bool OUT>
__global__ __launch_bounds__(kT) void k_project_complement(const T* __restrict__ phi, int k,
                                                           const double* __restrict__ z, int nv,
                                                           size_t ng, T* __restrict__ io) {
  __shared__ T zs[KMAX * kPVB];
  const int v0 = blockIdx.y * kPVB;
  for (int t = threadIdx.x; t < k * kPVB; t += kT) {
    const int i = t / kPVB, vb = t % kPVB;
    zs[t] = (v0 + vb < nv) ? (T)z[(size_t)i * nv + v0 + vb] : T(0);
  }
  __syncthreads();
  const size_t r = (size_t)blockIdx.x * kT + threadIdx.x;
  if (r >= ng) return;
  T p[KMAX];
#pragma unroll
  for (int i = 0; i < KMAX; ++i) p[i] = phi[(size_t)(i < k ? i : k - 1) * ng + r];
  for (int vb = 0; vb < kPVB && v0 + vb < nv; ++vb) {
    T s = T(0);
#pragma unroll
    for (int i = 0; i < KMAX; ++i)
      if (i < k) s += p[i] * zs[i * kPVB + vb];
    const size_t o = (size_t)(v0 + vb) * ng + r;
    io[o] = OUT ? io[o] - s : s - io[o];
  }
}

template <typename T>
__global__ __launch_bounds__(kT) void k_scale_to_f32(const T* __restrict__ src,
                                                     const double* __restrict__ scale, size_t ng,
                                                     float* __restrict__ dst) {
  const size_t r = (size_t)blockIdx.x * kT + threadIdx.x;
  if (r >= ng) return;
  const size_t o = (size_t)blockIdx.y * ng + r;
  dst[o] = (float)((double)src[o] * scale[blockIdx.y]);
}

template <typename T>
__global__ __launch_bounds__(kT) void k_scale_inplace(T* __restrict__ x,
                                                      const double* __restrict__ scale, size_t ng) {
  const size_t r = (size_t)blockIdx.x * kT + threadIdx.x;
  if (r >= ng) return;
  const size_t o = (size_t)blockIdx.y * ng + r;
  x[o] = (T)((double)x[o] * scale[blockIdx.y]);
}

template <typename T>
__global__ __launch_bounds__(kT) void k_fill(T value, size_t count, T* __restrict__ dst) {
  for (size_t e = (size_t)blockIdx.x * kT + threadIdx.x; e < count; e += (size_t)gridDim.x * kT)
    dst[e] = value;
}

template <typename T>
__global__ __launch_bounds__(kT) void k_from_f32(const float* __restrict__ src, size_t count,
                                                 T* __restrict__ dst) {
  for (size_t e = (size_t)blockIdx.x * kT + threadIdx.x; e < count; e += (size_t)gridDim.x * kT)
    dst[e] = (T)src[e];
}

__global__ void k_inv_rms(const double* __restrict__ G, int ld, int nv, double ng,
                          double* __restrict__ scale) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < nv) scale[v] = 1.0 / sqrt(fmax(G[(size_t)v * ld + v] / ng, 1e-300));
}

// ---- one-workgroup FP64 steps ----

__global__ __launch_bounds__(kT) void k_sym_scale(const double* __restrict__ S,
                                                  const double* __restrict__ G, int m,
                                                  double* __restrict__ Ss, double* __restrict__ Gs,
                                                  double* __restrict__ D) {
  __shared__ double d[kCombineMax];
  for (int i = threadIdx.x; i < m; i += kT) {
    const double sii = S[(size_t)i * m + i];
    d[i] = sii > 0.0 ? 1.0 / sqrt(sii) : 0.0;
    D[i] = d[i];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < m * m; e += kT) {
    const int i = e / m, j = e % m;
    const double f = d[i] * d[j];
    Ss[e] = 0.5 * (S[e] + S[(size_t)j * m + i]) * f;
    Gs[e] = 0.5 * (G[e] + G[(size_t)j * m + i]) * f;
  }
}

__global__ __launch_bounds__(kT) void k_canon(const double* __restrict__ w,
                                              const double* __restrict__ U, int m, double rel,
                                              double* __restrict__ T, const int* __restrict__ skip) {
  if (skip != nullptr && *skip) return;  // T already holds an accepted orthonormalisation
  const double wmax = w[m - 1];
  for (int e = threadIdx.x; e < m * m; e += kT) {
    const int j = e % m;
    const double wj = w[j];
    T[e] = (wj > rel * wmax && wj > 0.0) ? U[e] / sqrt(wj) : 0.0;
  }
}

__global__ __launch_bounds__(kT) void k_drop_diag(double* __restrict__ A, int m,
                                                  const double* __restrict__ w, double rel) {
  __shared__ double red[kT];
  double rowmax = 0.0;
  for (int i = threadIdx.x; i < m; i += kT) {
    double s = 0.0;
    for (int l = 0; l < m; ++l) s += fabs(A[(size_t)i * m + l]);
    rowmax = fmax(rowmax, s);
  }
  red[threadIdx.x] = rowmax;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double bound = 1.0 + red[0];
  const double wmax = w[m - 1];
  for (int j = threadIdx.x; j < m; j += kT)
    if (!(w[j] > rel * wmax && w[j] > 0.0)) A[(size_t)j * m + j] = bound;
}

__global__ __launch_bounds__(kT) void k_inv_sqrt_eig(const double* __restrict__ w,
                                                     const double* __restrict__ U, int m,
                                                     double* __restrict__ out) {
  __shared__ double f[kCombineMax];
  for (int k = threadIdx.x; k < m; k += kT) f[k] = w[k] > 0.0 ? 1.0 / sqrt(w[k]) : 0.0;
  __syncthreads();
  for (int e = threadIdx.x; e < m * m; e += kT) {
    const int i = e / m, j = e % m;
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += U[(size_t)i * m + k] * f[k] * U[(size_t)j * m + k];
    out[e] = s;
  }
}

__global__ void k_scale_coeff_rows(double* __restrict__ C, int ldc, const double* __restrict__ D,
                                   int m, int k) {
  for (int e = threadIdx.x; e < m * k; e += blockDim.x) C[(size_t)(e / k) * ldc + e % k] *= D[e / k];
}

__global__ void k_zero_rows(double* __restrict__ C, int ldc, int r, int k) {
  for (int e = threadIdx.x; e < r * k; e += blockDim.x) C[(size_t)(e / k) * ldc + e % k] = 0.0;
}

__global__ void k_diag(const double* __restrict__ A, int ld, int m, double* __restrict__ out) {
  for (int j = threadIdx.x; j < m; j += blockDim.x) out[j] = A[(size_t)j * ld + j];
}

unsigned grid_blocks(size_t ng) { return (unsigned)((ng + kT - 1) / kT); }

// every non-null pointer 16-byte aligned (the 4-point kernels' vector loads)
bool aligned16(std::initializer_list<const void*> ps) {
  for (const void* p : ps)
    if (p && (reinterpret_cast<uintptr_t>(p) & 15)) return false;
  return true;
}

}  // namespace

void launch_fock_local(bool fp64, const void* x, int nv, int n, double h, const void* vloc,
                       int acc, void* y, hipStream_t s) {
  const size_t ng = (size_t)n * n * n;
  const Fd4<double> fd(h);
  const Fd4<float> ff(h);
  dim3 grid(grid_blocks(ng), nv);
  const bool v4 = !fp64 && n % 4 == 0 && aligned16({x, vloc, y});
  if (fp64)
    k_fock_local<double><<<grid, kT, 0, s>>>((const double*)x, n, ng, fd, (const double*)vloc,
                                             acc, (double*)y);
  else if (v4)
    k_fock_local4<<<dim3(grid_blocks(ng / 4), nv), kT, 0, s>>>((const float*)x, n, ng, ff,
                                                               (const float*)vloc, acc, (float*)y);
  else
    k_fock_local<float><<<grid, kT, 0, s>>>((const float*)x, n, ng, ff, (const float*)vloc, acc,
                                            (float*)y);
}

void launch_precond_kinetic(bool fp64, const void* r, int nv, int n, double h, double shift,
                            int sweeps, double omega, void* z, void* tmp, hipStream_t s) {
  const size_t ng = (size_t)n * n * n;
  const Fd4<double> fd(h);
  const Fd4<float> ff(h);
  dim3 grid(grid_blocks(ng), nv);
  const bool v4 = !fp64 && n % 4 == 0 && aligned16({r, z, tmp});
  // the last sweep must land in z: start in z if the number of later sweeps is even
  void* bufs[2] = {z, tmp};
  int cur = ((sweeps - 1) % 2 == 0) ? 0 : 1;
  for (int t = 0; t < sweeps; ++t) {
    const void* zin = bufs[cur];
    void* zout = t == 0 ? bufs[cur] : bufs[cur ^ 1];
    if (t > 0) cur ^= 1;
    if (fp64)
      k_jacobi_sweep<double><<<grid, kT, 0, s>>>((const double*)r, (const double*)zin,
                                                 (double*)zout, n, ng, fd, shift, omega, t == 0);
    else if (v4)
      k_jacobi_sweep4<<<dim3(grid_blocks(ng / 4), nv), kT, 0, s>>>(
          (const float*)r, (const float*)zin, (float*)zout, n, ng, ff, (float)shift,
          (float)omega, t == 0);
    else
      k_jacobi_sweep<float><<<grid, kT, 0, s>>>((const float*)r, (const float*)zin, (float*)zout,
                                                n, ng, ff,
                                                (float)shift, (float)omega, t == 0);
  }
}

void launch_density(bool fp64, const void* x, int k, size_t ng, void* rho, hipStream_t s) {
  if (fp64)
    k_density<double><<<grid_blocks(ng), kT, 0, s>>>((const double*)x, k, ng, (double*)rho);
  else
    k_density<float><<<grid_blocks(ng), kT, 0, s>>>((const float*)x, k, ng, (float*)rho);
}

void launch_axpby(bool fp64, const void* a, const void* b, double alpha, double beta,
                  size_t count, void* out, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<size_t>(4096, (count + kT - 1) / kT);
  if (fp64)
    k_axpby<double><<<nb, kT, 0, s>>>((const double*)a, (const double*)b, alpha, beta, count,
                                      (double*)out);
  else
    k_axpby<float><<<nb, kT, 0, s>>>((const float*)a, (const float*)b, (float)alpha, (float)beta,
                                     count, (float*)out);
}

void launch_abs_diff_sum(bool fp64, const void* a, const void* b, size_t count, double scale,
                         double* part, double* out, hipStream_t s) {
  if (fp64)
    k_abs_part<double><<<kAbsParts, kT, 0, s>>>((const double*)a, (const double*)b, count, part);
  else
    k_abs_part<float><<<kAbsParts, kT, 0, s>>>((const float*)a, (const float*)b, count, part);
  k_sum_parts<<<1, kT, 0, s>>>(part, kAbsParts, scale, out);
}

template <typename T>
static void combine_impl(const void* V, int mb, size_t ng, const double* C, int ldc, int kout,
                         void* out, hipStream_t s) {
  const unsigned g = grid_blocks(ng);
  if (kout <= 8)
    k_combine<T, 8><<<g, kT, 0, s>>>((const T*)V, mb, ng, C, ldc, kout, (T*)out);
  else if (kout <= 16)
    k_combine<T, 16><<<g, kT, 0, s>>>((const T*)V, mb, ng, C, ldc, kout, (T*)out);
  else
    k_combine<T, 32><<<g, kT, 0, s>>>((const T*)V, mb, ng, C, ldc, kout, (T*)out);
}

void launch_combine(bool fp64, const void* V, int mb, size_t ng, const double* C, int ldc,
                    int kout, void* out, hipStream_t s) {
  if (fp64)
    combine_impl<double>(V, mb, ng, C, ldc, kout, out, s);
  else
    combine_impl<float>(V, mb, ng, C, ldc, kout, out, s);
}

void launch_residual_grid(bool fp64, const void* X, const void* HX, const double* lam, int k,
                          size_t ng, void* R, hipStream_t s) {
  dim3 grid(grid_blocks(ng), k);
  if (fp64)
    k_residual_grid<double><<<grid, kT, 0, s>>>((const double*)X, (const double*)HX, lam, ng,
                                                (double*)R);
  else
    k_residual_grid<float><<<grid, kT, 0, s>>>((const float*)X, (const float*)HX, lam, ng,
                                               (float*)R);
}

template <typename T, bool OUT>
static void project_impl(const void* phi, int k, const double* z, int nv, size_t ng, void* io,
                         hipStream_t s) {
  dim3 grid(grid_blocks(ng), (nv + kPVB - 1) / kPVB);
  if (k <= 16)
    k_project_complement<T, 16, OUT><<<grid, kT, 0, s>>>((const T*)phi, k, z, nv, ng, (T*)io);
  else if (k <= 32)
    k_project_complement<T, 32, OUT><<<grid, kT, 0, s>>>((const T*)phi, k, z, nv, ng, (T*)io);
  else
    k_project_complement<T, 64, OUT><<<grid, kT, 0, s>>>((const T*)phi, k, z, nv, ng, (T*)io);
}

void launch_project_complement(bool fp64, const void* phi, int k, const double* z, int nv,
                               size_t ng, void* inout, hipStream_t s) {
  if (fp64)
    project_impl<double, false>(phi, k, z, nv, ng, inout, s);
  else
    project_impl<float, false>(phi, k, z, nv, ng, inout, s);
}

void launch_project_out(bool fp64, const void* phi, int k, const double* z, int nv, size_t ng,
                        void* inout, hipStream_t s) {
  if (fp64)
    project_impl<double, true>(phi, k, z, nv, ng, inout, s);
  else
    project_impl<float, true>(phi, k, z, nv, ng, inout, s);
}

void launch_scale_to_f32(bool fp64, const void* src, const double* scale, int nv, size_t ng,
                         float* dst, hipStream_t s) {
  dim3 grid(grid_blocks(ng), nv);
  if (fp64)
    k_scale_to_f32<double><<<grid, kT, 0, s>>>((const double*)src, scale, ng, dst);
  else
    k_scale_to_f32<float><<<grid, kT, 0, s>>>((const float*)src, scale, ng, dst);
}

void launch_scale_inplace(bool fp64, void* x, const double* scale, int nv, size_t ng,
                          hipStream_t s) {
  dim3 grid(grid_blocks(ng), nv);
  if (fp64)
    k_scale_inplace<double><<<grid, kT, 0, s>>>((double*)x, scale, ng);
  else
    k_scale_inplace<float><<<grid, kT, 0, s>>>((float*)x, scale, ng);
}

void launch_fill(bool fp64, double value, size_t count, void* dst, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<size_t>(4096, (count + kT - 1) / kT);
  if (fp64)
    k_fill<double><<<nb, kT, 0, s>>>(value, count, (double*)dst);
  else
    k_fill<float><<<nb, kT, 0, s>>>((float)value, count, (float*)dst);
}

void launch_from_f32(bool fp64, const float* src, size_t count, void* dst, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<size_t>(4096, (count + kT - 1) / kT);
  if (fp64)
    k_from_f32<double><<<nb, kT, 0, s>>>(src, count, (double*)dst);
  else
    k_from_f32<float><<<nb, kT, 0, s>>>(src, count, (float*)dst);
}

void launch_inv_rms(const double* G, int ld, int nv, double ng, double* scale, hipStream_t s) {
  k_inv_rms<<<(nv + 63) / 64, 64, 0, s>>>(G, ld, nv, ng, scale);
}

void launch_sym_scale(const double* S, const double* G, int m, double* Ss, double* Gs,
                      double* D, hipStream_t s) {
  k_sym_scale<<<1, kT, 0, s>>>(S, G, m, Ss, Gs, D);
}

void launch_canon(const double* w, const double* U, int m, double rel, double* T, hipStream_t s,
                  const int* skip) {
  k_canon<<<1, kT, 0, s>>>(w, U, m, rel, T, skip);
}

void launch_drop_diag(double* A, int m, const double* w, double rel, hipStream_t s) {
  k_drop_diag<<<1, kT, 0, s>>>(A, m, w, rel);
}

void launch_inv_sqrt_from_eig(const double* w, const double* U, int m, double* out,
                              hipStream_t s) {
  k_inv_sqrt_eig<<<1, kT, 0, s>>>(w, U, m, out);
}

void launch_scale_coeff_rows(double* C, int ldc, const double* D, int m, int k, hipStream_t s) {
  k_scale_coeff_rows<<<1, kT, 0, s>>>(C, ldc, D, m, k);
}

void launch_zero_rows(double* C, int ldc, int r, int k, hipStream_t s) {
  if (r > 0) k_zero_rows<<<1, kT, 0, s>>>(C, ldc, r, k);
}

void launch_diag(const double* A, int ld, int m, double* out, hipStream_t s) {
  k_diag<<<1, 64, 0, s>>>(A, ld, m, out);
}

}  // namespace ace
