// ACE construction and application around the pair-Poisson engine (paper Sec. 3.1,
// Eqs. (11)-(13)):
//   W_i   = -sum_j phi_j v_ji                      (Eq. (11) with Eq. (2))
//   M     = Phi^H W dV                             (Gram kernel, FP64 cross-tile sums)
//   -M    = L L^H, E_x = 1/2 tr M                  (one workgroup, FP64)
//   xi    = W L^{-H}                               (Eq. (12), per-point triangular product)
//   K psi = -xi (xi^H psi dV)                      (Eq. (13), Gram kernel + per-point update)
// Conjugation follows the complex reading of the real-orbital equations: pair densities are
// conj(phi_j) phi_i, so v_ij = conj(v_ji) and only pairs j <= i are solved.
#include "ace_kernels.hpp"
#include "elem.hpp"

namespace ace {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ size_t pair_index(int a, int b) {  // a <= b
  return (size_t)b * (b + 1) / 2 + a;
}

// W_i(r) = -sum_j phi_j(r) v_ji(r); v holds pair (a<=b) volumes G (*) conj(phi_a) phi_b.
template <typename E>
__global__ __launch_bounds__(kThreads) void k_wacc(const E* __restrict__ phi,
                                                   const E* __restrict__ v, int n, size_t ng,
                                                   E* __restrict__ w) {
  const int i = blockIdx.x % n;
  const size_t r = (size_t)(blockIdx.x / n) * kThreads + threadIdx.x;
  if (r >= ng) return;
  E acc = e_zero<E>();
  for (int j = 0; j < n; ++j) {
    E vj;
    if (j <= i)
      vj = v[pair_index(j, i) * ng + r];
    else
      vj = e_conj(v[pair_index(i, j) * ng + r]);
    acc = e_add(acc, e_mul(phi[(size_t)j * ng + r], vj));
  }
  w[(size_t)i * ng + r] = e_neg(acc);
}

// Partial Gram sums G_kl = sum_r conj(A_k(r)) B_l(r) over one chunk of points per block.
// Tiles of kTile points are staged through LDS (rows padded by one element against bank
// conflicts); a thread owns one output (k, l) and a strided subset of the tile's points when
// there are at most 256 outputs, else up to 4 outputs over all points.  Products are summed in
// the storage precision over one tile, then added into FP64 accumulators.
constexpr int kTile = 64;
constexpr int kLS = kTile + 1;

template <typename E>
__global__ __launch_bounds__(kThreads) void k_gram(const E* __restrict__ A, int na,
                                                   const E* __restrict__ B, int nb, size_t ng,
                                                   size_t chunk,
                                                   typename Elem<E>::wide* __restrict__ part) {
  typedef typename Elem<E>::wide W;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  E* sA = reinterpret_cast<E*>(smem_raw);
  E* sB = sA + (size_t)na * kLS;
  const int no = na * nb;
  const bool few = no <= kThreads;
  const int lanes = few ? kThreads / no : 1;
  const int lane = few ? threadIdx.x / no : 0;
  const size_t start = (size_t)blockIdx.x * chunk;
  const size_t end = start + chunk < ng ? start + chunk : ng;
  W acc[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) acc[m] = W{};
  for (size_t t0 = start; t0 < end; t0 += kTile) {
    for (int idx = threadIdx.x; idx < (na + nb) * kTile; idx += kThreads) {
      const int row = idx / kTile, c = idx % kTile;
      const size_t r = t0 + c;
      E val = e_zero<E>();
      if (r < end) val = row < na ? A[(size_t)row * ng + r] : B[(size_t)(row - na) * ng + r];
      sA[row * kLS + c] = val;  // sB rows follow sA rows contiguously
    }
    __syncthreads();
    if (lane < lanes) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int o = few ? (m == 0 ? (int)(threadIdx.x % no) : no) : (int)threadIdx.x + m * kThreads;
        if (o < no) {
          const E* ra = sA + (o / nb) * kLS;
          const E* rb = sB + (o % nb) * kLS;
          E s = e_zero<E>();
          for (int c = lane; c < kTile; c += lanes) s = e_add(s, e_mulc(ra[c], rb[c]));
          acc[m] = e_add(acc[m], e_wide(s));
        }
      }
    }
    __syncthreads();
  }
  W* red = reinterpret_cast<W*>(smem_raw);
  if (few) {
    red[threadIdx.x] = acc[0];
    __syncthreads();
    if ((int)threadIdx.x < no) {
      W s = W{};
      for (int q = 0; q < lanes; ++q) s = e_add(s, red[q * no + threadIdx.x]);
      part[(size_t)blockIdx.x * no + threadIdx.x] = s;
    }
  } else {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int o = (int)threadIdx.x + m * kThreads;
      if (o < no) part[(size_t)blockIdx.x * no + o] = acc[m];
    }
  }
}

template <typename W>
__global__ void k_gram_reduce(const W* __restrict__ part, int nblk, int no, double scale,
                              W* __restrict__ out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= no) return;
  W s = W{};
  for (int b = 0; b < nblk; ++b) s = e_add(s, part[(size_t)b * no + o]);
  out[o] = e_scale(s, scale);
}

// Cholesky of -M (Hermitised), L^{-H}, E_x; one workgroup.  W is double or C2<double>.
template <typename W>
__global__ __launch_bounds__(kThreads) void k_chol(const W* __restrict__ mred, int n,
                                                   W* __restrict__ m_out, double* __restrict__ ex_out,
                                                   W* __restrict__ linvh, int* __restrict__ status) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  W* a = reinterpret_cast<W*>(smem_raw);  // n*n: -M, then L in the lower triangle
  W* x = a + n * n;                       // n*n: L^{-1}
  __shared__ int fail, bad;
  if (threadIdx.x == 0) {
    fail = -1;
    bad = 0;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < n * n; idx += kThreads) {
    const int k = idx / n, l = idx % n;
    const W mkl = mred[k * n + l], mlk = mred[l * n + k];
    if (!e_finite(mkl)) bad = 1;
    const W herm = e_scale(e_add(mkl, e_conj(mlk)), 0.5);
    if (m_out) m_out[idx] = herm;
    a[idx] = e_neg(herm);
  }
  __syncthreads();
  if (threadIdx.x == 0 && ex_out) {
    double e = 0.0;
    for (int k = 0; k < n; ++k) e += -e_re(a[k * n + k]);
    *ex_out = 0.5 * e;
  }
  // left-looking Cholesky, column by column
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double d = e_re(a[j * n + j]);
      for (int k = 0; k < j; ++k) d -= e_abs2(a[j * n + k]);
      if (!(d > 0.0) && fail < 0) fail = j;
      double s = d > 0.0 ? sqrt(d) : 1.0;
      W dj = W{};
      if constexpr (Elem<W>::cplx) dj.r = s; else dj = s;
      a[j * n + j] = dj;
    }
    __syncthreads();
    const double djj = e_re(a[j * n + j]);
    for (int i = j + 1 + threadIdx.x; i < n; i += kThreads) {
      W s = a[i * n + j];
      for (int k = 0; k < j; ++k) s = e_sub(s, e_mulc(a[j * n + k], a[i * n + k]));
      a[i * n + j] = e_scale(s, 1.0 / djj);
    }
    __syncthreads();
  }
  // X = L^{-1}: column c solved by one thread
  for (int c = threadIdx.x; c < n; c += kThreads) {
    for (int i = 0; i < n; ++i) x[i * n + c] = W{};
    {
      W inv = W{};
      if constexpr (Elem<W>::cplx) inv.r = 1.0 / e_re(a[c * n + c]); else inv = 1.0 / a[c * n + c];
      x[c * n + c] = inv;
    }
    for (int i = c + 1; i < n; ++i) {
      W s = W{};
      for (int k = c; k < i; ++k) s = e_add(s, e_mul(a[i * n + k], x[k * n + c]));
      x[i * n + c] = e_scale(s, -1.0 / e_re(a[i * n + i]));
    }
  }
  __syncthreads();
  const bool ok = fail < 0 && !bad;
  // L^{-H}[i][k] = conj(X[k][i])
  for (int idx = threadIdx.x; idx < n * n; idx += kThreads) {
    const int i = idx / n, k = idx % n;
    linvh[idx] = ok ? e_conj(x[k * n + i]) : W{};
  }
  if (threadIdx.x == 0 && !ok && status) {
    if (status[0] == 0) {
      status[0] = bad ? -6 : -5;
      status[1] = bad ? -1 : fail;
    }
  }
}

// xi_k(r) = sum_{i<=k} W_i(r) (L^{-H})_{ik}; in place allowed (xi may alias W).
template <typename E, int NMAX>
__global__ __launch_bounds__(kThreads) void k_trsm(const E* w, int n, size_t ng,
                                                   const typename Elem<E>::wide* __restrict__ linvh,
                                                   E* xi) {
  const size_t r = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= ng) return;
  E wr[NMAX];
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
    if (i < n) wr[i] = w[(size_t)i * ng + r];
#pragma unroll
  for (int k = 0; k < NMAX; ++k) {
    if (k < n) {
      E s = e_zero<E>();
#pragma unroll
      for (int i = 0; i <= k; ++i) s = e_add(s, e_mul(wr[i], e_narrow<E>(linvh[i * n + k])));
      xi[(size_t)k * ng + r] = s;
    }
  }
}

// out_v(r) = -sum_k xi_k(r) Z_kv,  Z = xi^H psi dV (already scaled).  Grid: (point blocks,
// vector groups of kVB): more threads than points so that the GPU is filled.
constexpr int kVB = 4;

template <typename E, int NMAX>
__global__ __launch_bounds__(kThreads) void k_apply_out(const E* __restrict__ xi, int n, size_t ng,
                                                        const typename Elem<E>::wide* __restrict__ z,
                                                        int nv, E* __restrict__ out) {
  const size_t r = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const int v0 = blockIdx.y * kVB;
  if (r >= ng) return;
  E xr[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k)
    if (k < n) xr[k] = xi[(size_t)k * ng + r];
#pragma unroll
  for (int vb = 0; vb < kVB; ++vb) {
    const int v = v0 + vb;
    if (v < nv) {
      E s = e_zero<E>();
#pragma unroll
      for (int k = 0; k < NMAX; ++k)
        if (k < n) s = e_add(s, e_mul(xr[k], e_narrow<E>(z[k * nv + v])));
      out[(size_t)v * ng + r] = e_neg(s);
    }
  }
}

template <typename E>
void gram_impl(const void* A, int na, const void* B, int nb, size_t ng, void* part, int nblk,
               size_t chunk, double scale, void* out, hipStream_t s) {
  typedef typename Elem<E>::wide W;
  const size_t lds_tiles = (size_t)(na + nb) * kLS * sizeof(E);
  const size_t lds_red = (size_t)kThreads * sizeof(W);
  const size_t lds = lds_tiles > lds_red ? lds_tiles : lds_red;
  k_gram<E><<<nblk, kThreads, lds, s>>>((const E*)A, na, (const E*)B, nb, ng, chunk, (W*)part);
  const int no = na * nb;
  k_gram_reduce<W><<<(no + 255) / 256, 256, 0, s>>>((const W*)part, nblk, no, scale, (W*)out);
}

}  // namespace

int gram_blocks(size_t ng, size_t* chunk) {
  // 256 points per block: enough blocks to fill the GPU at the box sizes of interest
  size_t c = 256;
  size_t nblk = (ng + c - 1) / c;
  if (nblk < 1) nblk = 1;
  *chunk = c;
  return (int)nblk;
}

void launch_wacc(int et, const void* phi, const void* v, int n, size_t ng, void* w, hipStream_t s, Trace* tr) {
  TraceScope ts(tr, TR_WACC);
  const unsigned blocks = (unsigned)(((ng + kThreads - 1) / kThreads) * n);
  switch (et) {
    case ET_C128: k_wacc<C2<double>><<<blocks, kThreads, 0, s>>>((const C2<double>*)phi, (const C2<double>*)v, n, ng, (C2<double>*)w); break;
    case ET_C64: k_wacc<C2<float>><<<blocks, kThreads, 0, s>>>((const C2<float>*)phi, (const C2<float>*)v, n, ng, (C2<float>*)w); break;
    case ET_R64: k_wacc<double><<<blocks, kThreads, 0, s>>>((const double*)phi, (const double*)v, n, ng, (double*)w); break;
    case ET_R32: k_wacc<float><<<blocks, kThreads, 0, s>>>((const float*)phi, (const float*)v, n, ng, (float*)w); break;
  }
}

void launch_gram(int et, const void* A, int na, const void* B, int nb, size_t ng, void* part,
                 double scale, void* out, hipStream_t s, Trace* tr) {
  TraceScope ts(tr, TR_GRAM);
  size_t chunk;
  const int nblk = gram_blocks(ng, &chunk);
  switch (et) {
    case ET_C128: gram_impl<C2<double>>(A, na, B, nb, ng, part, nblk, chunk, scale, out, s); break;
    case ET_C64: gram_impl<C2<float>>(A, na, B, nb, ng, part, nblk, chunk, scale, out, s); break;
    case ET_R64: gram_impl<double>(A, na, B, nb, ng, part, nblk, chunk, scale, out, s); break;
    case ET_R32: gram_impl<float>(A, na, B, nb, ng, part, nblk, chunk, scale, out, s); break;
  }
}

void launch_chol(int et, const void* mred, int n, void* m_out, double* ex_out, void* linvh,
                 int* status, hipStream_t s, Trace* tr) {
  TraceScope ts(tr, TR_CHOL);
  if (et == ET_C128 || et == ET_C64) {
    const size_t lds = 2 * (size_t)n * n * sizeof(C2<double>);
    k_chol<C2<double>><<<1, kThreads, lds, s>>>((const C2<double>*)mred, n, (C2<double>*)m_out, ex_out,
                                                (C2<double>*)linvh, status);
  } else {
    const size_t lds = 2 * (size_t)n * n * sizeof(double);
    k_chol<double><<<1, kThreads, lds, s>>>((const double*)mred, n, (double*)m_out, ex_out,
                                            (double*)linvh, status);
  }
}

template <typename E>
static void trsm_impl(const void* w, int n, size_t ng, const void* linvh, void* xi, hipStream_t s) {
  typedef typename Elem<E>::wide W;
  const unsigned blocks = (unsigned)((ng + kThreads - 1) / kThreads);
  if (n <= 8)
    k_trsm<E, 8><<<blocks, kThreads, 0, s>>>((const E*)w, n, ng, (const W*)linvh, (E*)xi);
  else if (n <= 16)
    k_trsm<E, 16><<<blocks, kThreads, 0, s>>>((const E*)w, n, ng, (const W*)linvh, (E*)xi);
  else
    k_trsm<E, 32><<<blocks, kThreads, 0, s>>>((const E*)w, n, ng, (const W*)linvh, (E*)xi);
}

void launch_trsm(int et, const void* w, int n, size_t ng, const void* linvh, void* xi, hipStream_t s, Trace* tr) {
  TraceScope ts(tr, TR_TRSM);
  switch (et) {
    case ET_C128: trsm_impl<C2<double>>(w, n, ng, linvh, xi, s); break;
    case ET_C64: trsm_impl<C2<float>>(w, n, ng, linvh, xi, s); break;
    case ET_R64: trsm_impl<double>(w, n, ng, linvh, xi, s); break;
    case ET_R32: trsm_impl<float>(w, n, ng, linvh, xi, s); break;
  }
}

template <typename E>
static void apply_impl(const void* xi, int n, size_t ng, const void* z, int nv, void* out,
                       hipStream_t s) {
  typedef typename Elem<E>::wide W;
  dim3 blocks((unsigned)((ng + kThreads - 1) / kThreads), (unsigned)((nv + kVB - 1) / kVB));
  if (n <= 8)
    k_apply_out<E, 8><<<blocks, kThreads, 0, s>>>((const E*)xi, n, ng, (const W*)z, nv, (E*)out);
  else if (n <= 16)
    k_apply_out<E, 16><<<blocks, kThreads, 0, s>>>((const E*)xi, n, ng, (const W*)z, nv, (E*)out);
  else
    k_apply_out<E, 32><<<blocks, kThreads, 0, s>>>((const E*)xi, n, ng, (const W*)z, nv, (E*)out);
}

void launch_apply_out(int et, const void* xi, int n, size_t ng, const void* z, int nv, void* out,
                      hipStream_t s, Trace* tr) {
  TraceScope ts(tr, TR_APPLY);
  switch (et) {
    case ET_C128: apply_impl<C2<double>>(xi, n, ng, z, nv, out, s); break;
    case ET_C64: apply_impl<C2<float>>(xi, n, ng, z, nv, out, s); break;
    case ET_R64: apply_impl<double>(xi, n, ng, z, nv, out, s); break;
    case ET_R32: apply_impl<float>(xi, n, ng, z, nv, out, s); break;
  }
}

}  // namespace ace

namespace ace {
namespace {

// Direct exchange accumulation (Eq. (2)): out_v(r) = -sum_j phi_j(r) v[v*n + j](r).
template <typename E>
__global__ __launch_bounds__(256) void k_direct_acc(const E* __restrict__ phi, int n,
                                                     const E* __restrict__ v, int nv, size_t ng,
                                                     E* __restrict__ out) {
  const int vi = blockIdx.x % nv;
  const size_t r = (size_t)(blockIdx.x / nv) * 256 + threadIdx.x;
  if (r >= ng) return;
  E acc = e_zero<E>();
  for (int j = 0; j < n; ++j)
    acc = e_add(acc, e_mul(phi[(size_t)j * ng + r], v[((size_t)vi * n + j) * ng + r]));
  out[(size_t)vi * ng + r] = e_neg(acc);
}

}  // namespace

void launch_direct_acc(int et, const void* phi, int n, const void* v, int nv, size_t ng, void* out,
                       hipStream_t s, Trace* tr) {
  TraceScope ts(tr, TR_DIRECT);
  const unsigned blocks = (unsigned)(((ng + 255) / 256) * nv);
  switch (et) {
    case ET_C128: k_direct_acc<C2<double>><<<blocks, 256, 0, s>>>((const C2<double>*)phi, n, (const C2<double>*)v, nv, ng, (C2<double>*)out); break;
    case ET_C64: k_direct_acc<C2<float>><<<blocks, 256, 0, s>>>((const C2<float>*)phi, n, (const C2<float>*)v, nv, ng, (C2<float>*)out); break;
    case ET_R64: k_direct_acc<double><<<blocks, 256, 0, s>>>((const double*)phi, n, (const double*)v, nv, ng, (double*)out); break;
    case ET_R32: k_direct_acc<float><<<blocks, 256, 0, s>>>((const float*)phi, n, (const float*)v, nv, ng, (float*)out); break;
  }
}

}  // namespace ace
