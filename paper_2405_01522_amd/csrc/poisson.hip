// Isolated Poisson solves of pair densities on an N^3 box: zero-padded (P = 2N) FFT
// convolution with the sampled Coulomb kernel (the exchange integral of Eq. (2) posed as a
// Poisson problem, paper Sec. 3.1).
//
// Three passes per pair, with one volume of N*N*P complex values between them (the z axis
// is the only one ever padded in HBM):
//   Z-forward  (grid: x-plane x pair)   rho = conj(a) b on the box, pruned FFT along z,
//                                       written transposed as work[pair][qz][x][y];
//   XY         (grid: qz-plane x pair)  one N x N slice -> P x P plane in LDS; pruned FFT
//                                       along y then x, multiply by the kernel spectrum,
//                                       inverse along x then y keeping only the N x N box;
//                                       written back in place;
//   Z-inverse  (grid: x-plane x pair)   inverse FFT along z keeping z < N -> v[pair][x][y][z].
// Every 1-D transform is P = P1 * P2 with one LDS exchange; see fftplan.hpp.  The x-axis
// forward second factor, the kernel multiply and the inverse first factor are fused in
// registers.  The kernel spectrum is real and even, so it is stored as the octant
// (P/2+1)^3 and indexed by min(k, P-k) per axis; it already carries dV / P^3.
#include <algorithm>

#include "common.hpp"
#include "fftplan.hpp"
#include "internal.hpp"

namespace ace {

namespace {

// threads of the z passes.  Each pass has a phase of N * P2 items (one per column and
// second-factor index) and one of N * P1 items.  From edge 32 on, the z-forward pass takes one
// thread per item of its N * P2 phase and the z-inverse pass one per item of its N * P1 phase
// (rounded up to whole wavefronts, at most 1024), so neither pass runs a partly filled extra
// round; smaller edges use 256.  (Measured at 48^3 against 256 threads for both: z-forward
// 16.8 -> 14.9 us with 576, z-inverse 17.1 -> 15.9 us with 384.)  The z-forward pass at edge
// 56 keeps 512 threads: 832 (13 wavefronts, two workgroups per CU) was 1.5x slower.
constexpr int z_round(int t) { return ((t + 63) / 64) * 64 > 1024 ? 1024 : ((t + 63) / 64) * 64; }
template <int N>
constexpr int zf_threads() {
  return N == 56 ? 512 : (N >= 32 ? z_round(N * Plan<N>::P2) : 256);
}
template <int N>
constexpr int zi_threads() {
  return N >= 32 ? z_round(N * Plan<N>::P1) : 256;
}
#ifndef ACE_XY_THREADS
#define ACE_XY_THREADS 1024
#endif
constexpr int kXyThreads = ACE_XY_THREADS;  // XY pass (one P x P plane per workgroup)

template <typename T>
__device__ __forceinline__ C2<T>* lds() {
  extern __shared__ __align__(16) unsigned char ace_smem[];
  return reinterpret_cast<C2<T>*>(ace_smem);
}

// LDS bytes of `elems` complex values followed by the P table twiddles (16-byte aligned).
template <typename T>
constexpr size_t tw_offset(size_t elems) {
  return (elems * sizeof(C2<T>) + 15) / 16 * 16;
}
template <typename T, int P>
constexpr size_t lds_with_twiddles(size_t elems) {
  return tw_offset<T>(elems) + (size_t)P * sizeof(TwE<T>);
}

// Copy the P twiddles exp(-2 pi i m / P) into LDS after `elems` complex values.
template <typename T, int P>
__device__ __forceinline__ const TwE<T>* stage_twiddles(C2<T>* base, size_t elems,
                                                        const TwE<T>* __restrict__ tw) {
  TwE<T>* s = reinterpret_cast<TwE<T>*>(reinterpret_cast<unsigned char*>(base) +
                                        tw_offset<T>(elems));
  for (int m = threadIdx.x; m < P; m += blockDim.x) s[m] = tw[m];
  return s;
}

// ---------------------------------------------------------------------------------------
// Where pair q's two orbitals and its output volume live.  PairsByIndex: one pair list of
// (j, i) indices into two orbital arrays and a contiguous output array (one system);
// PairsByPointer: explicit pointers per pair (many systems batched into one launch).
struct PairsByIndex {
  const void* pa;
  const void* pb;
  const int* pairs;
  void* vout;
  int np;
  template <typename E>
  __device__ __forceinline__ const E* a(int q, size_t ng) const {
    return reinterpret_cast<const E*>(pa) + (size_t)pairs[2 * q] * ng;
  }
  template <typename E>
  __device__ __forceinline__ const E* b(int q, size_t ng) const {
    return reinterpret_cast<const E*>(pb) + (size_t)pairs[2 * q + 1] * ng;
  }
  template <typename E>
  __device__ __forceinline__ E* v(int q, size_t ng) const {
    return reinterpret_cast<E*>(vout) + (size_t)q * ng;
  }
  __device__ __forceinline__ int kind(int) const { return 0; }
  template <typename E>
  __device__ __forceinline__ E* v2(int, size_t) const { return nullptr; }
};

// Complex transforms of one system from 4 ints each (a, b, out0, out1); see launch_pair_slots.
struct SlotsByIndex {
  const void* pa;
  const int* slots;
  void* vout;
  int np;
  template <typename E>
  __device__ __forceinline__ const E* a(int q, size_t ng) const {
    return reinterpret_cast<const E*>(pa) + (size_t)slots[4 * q] * ng;
  }
  template <typename E>
  __device__ __forceinline__ const E* b(int q, size_t ng) const {
    return reinterpret_cast<const E*>(pa) + (size_t)slots[4 * q + 1] * ng;
  }
  template <typename E>
  __device__ __forceinline__ E* v(int q, size_t ng) const {
    return reinterpret_cast<E*>(vout) + (size_t)slots[4 * q + 2] * ng;
  }
  __device__ __forceinline__ int kind(int q) const {
    const int o1 = slots[4 * q + 3];
    return o1 == -1 ? 0 : (o1 == -2 ? 2 : 1);
  }
  template <typename E>
  __device__ __forceinline__ E* v2(int q, size_t ng) const {
    return reinterpret_cast<E*>(vout) + (size_t)slots[4 * q + 3] * ng;
  }
};

struct PairsByPointer {
  const PairPtrs* items;
  int np;
  template <typename E>
  __device__ __forceinline__ const E* a(int q, size_t) const {
    return reinterpret_cast<const E*>(items[q].a);
  }
  template <typename E>
  __device__ __forceinline__ const E* b(int q, size_t) const {
    return reinterpret_cast<const E*>(items[q].b);
  }
  template <typename E>
  __device__ __forceinline__ E* v(int q, size_t) const {
    return reinterpret_cast<E*>(items[q].v);
  }
  __device__ __forceinline__ int kind(int q) const { return items[q].kind; }
  template <typename E>
  __device__ __forceinline__ E* v2(int q, size_t) const {
    return reinterpret_cast<E*>(items[q].v2);
  }
};

// ---------------------------------------------------------------------------------------
// Z-forward pass
template <typename T, int N, bool RP, typename R>
__global__ __launch_bounds__(zf_threads<N>()) void k_zfwd(R res, C2<T>* __restrict__ work,
                                                   const TwE<T>* __restrict__ twg) {
  typedef Plan<N> PL;
  constexpr int P = PL::P, P1 = PL::P1, P2 = PL::P2, H1 = PL::H1, RS = P + 1;
  constexpr size_t NG = (size_t)N * N * N;
  C2<T>* buf = lds<T>();
  const TwE<T>* tw = stage_twiddles<T, P>(buf, N * RS, twg);
  __syncthreads();
  const int x = blockIdx.x;
  const int p = blockIdx.y;
  const size_t plane = (size_t)x * N * N;

  const C2<T>* ca = nullptr;
  const C2<T>* cb = nullptr;
  const T *ra0 = nullptr, *rb0 = nullptr, *ra1 = nullptr, *rb1 = nullptr;
  // complex mode: 0 pair density, 1 two real densities |a|^2 + i |b|^2, 2 one real density
  const int kd = RP ? 0 : res.kind(p);
  if constexpr (RP) {
    const int q0 = 2 * p, q1 = 2 * p + 1;
    ra0 = res.template a<T>(q0, NG) + plane;
    rb0 = res.template b<T>(q0, NG) + plane;
    if (q1 < res.np) {
      ra1 = res.template a<T>(q1, NG) + plane;
      rb1 = res.template b<T>(q1, NG) + plane;
    }
  } else {
    ca = res.template a<C2<T>>(p, NG) + plane;
    cb = res.template b<C2<T>>(p, NG) + plane;
  }

  for (int it = threadIdx.x; it < N * P2; it += zf_threads<N>()) {
    const int n2 = it % P2, y = it / P2;
    C2<T> v[P1];
#pragma unroll
    for (int n1 = 0; n1 < H1; ++n1) {
      const int idx = y * N + n1 * P2 + n2;
      if constexpr (RP) {
        v[n1].r = ra0[idx] * rb0[idx];
        v[n1].i = ra1 ? ra1[idx] * rb1[idx] : T(0);
      } else {
        // both orbitals are loaded for every kind (b = a for kind 2) and the kind selects the
        // result, so the loads stay unconditional and issue back to back
        const C2<T> xa = ca[idx], xb = cb[idx];
        const C2<T> pd = cmulc(xa, xb);
        const T da = xa.r * xa.r + xa.i * xa.i, db = xb.r * xb.r + xb.i * xb.i;
        v[n1].r = kd == 0 ? pd.r : da;
        v[n1].i = kd == 0 ? pd.i : (kd == 1 ? db : T(0));
      }
    }
    dft_in_half<T, P1, -1>(v);
    buf[y * RS + n2] = v[0];
#pragma unroll
    for (int k1 = 1; k1 < P1; ++k1) buf[y * RS + k1 * P2 + n2] = tw_mul(v[k1], tw[n2 * k1]);
  }
  __syncthreads();
  C2<T>* dst0 = work + (size_t)p * P * N * N + (size_t)x * N;
  for (int it = threadIdx.x; it < N * P1; it += zf_threads<N>()) {
    const int y = it % N, k1 = it / N;
    C2<T> v[P2];
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = buf[y * RS + k1 * P2 + k2];
    dft<T, P2, -1>(v);
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) dst0[(size_t)(k1 * P2 + k2) * N * N + y] = v[k2];
  }
}

// ---------------------------------------------------------------------------------------
// XY pass: one qz plane per workgroup, the whole P x P plane in LDS.
template <typename T, int N>
__global__ __launch_bounds__(kXyThreads) void k_xy(C2<T>* __restrict__ work,
                                                 const T* __restrict__ gpos,
                                                 const TwE<T>* __restrict__ twg) {
  typedef Plan<N> PL;
  constexpr int P = PL::P, P1 = PL::P1, P2 = PL::P2, H1 = PL::H1, RS = P + 1;
  C2<T>* pl = lds<T>();
  const TwE<T>* tw = stage_twiddles<T, P>(pl, P * RS, twg);
  __syncthreads();
  const int qz = blockIdx.x, p = blockIdx.y;
  C2<T>* g = work + ((size_t)p * P + qz) * N * N;
  const T* gz = gpos + (size_t)qz * P * P;  // kernel spectrum in position order [qz][qx][qy]

  // 1. y forward, first factor (rows x < N, input y < N): global -> LDS
  for (int it = threadIdx.x; it < N * P2; it += kXyThreads) {
    const int n2 = it % P2, x = it / P2;
    C2<T> v[P1];
#pragma unroll
    for (int n1 = 0; n1 < H1; ++n1) v[n1] = g[x * N + n1 * P2 + n2];
    dft_in_half<T, P1, -1>(v);
    pl[x * RS + n2] = v[0];
#pragma unroll
    for (int k1 = 1; k1 < P1; ++k1) pl[x * RS + k1 * P2 + n2] = tw_mul(v[k1], tw[n2 * k1]);
  }
  __syncthreads();
  // 2. y forward, second factor
  for (int it = threadIdx.x; it < N * P1; it += kXyThreads) {
    const int x = it % N, k1 = it / N;
    C2<T> v[P2];
    C2<T>* row = pl + x * RS + k1 * P2;
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = row[k2];
    dft<T, P2, -1>(v);
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) row[k2] = v[k2];
  }
  __syncthreads();
  // 3. x forward, first factor (columns qy, input x < N)
  for (int it = threadIdx.x; it < P * P2; it += kXyThreads) {
    const int qy = it % P, n2 = it / P;
    C2<T> v[P1];
#pragma unroll
    for (int n1 = 0; n1 < H1; ++n1) v[n1] = pl[(n1 * P2 + n2) * RS + qy];
    dft_in_half<T, P1, -1>(v);
    pl[n2 * RS + qy] = v[0];
#pragma unroll
    for (int k1 = 1; k1 < P1; ++k1) pl[(k1 * P2 + n2) * RS + qy] = tw_mul(v[k1], tw[n2 * k1]);
  }
  __syncthreads();
  // 4. x forward second factor, kernel multiply, x inverse first factor (in registers)
  for (int it = threadIdx.x; it < P * P1; it += kXyThreads) {
    const int qy = it % P, k1 = it / P;
    C2<T> v[P2];
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = pl[(k1 * P2 + k2) * RS + qy];
    dft<T, P2, -1>(v);
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = cscale(v[k2], gz[(k1 * P2 + k2) * P + qy]);
    dft<T, P2, 1>(v);
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) pl[(k1 * P2 + k2) * RS + qy] = v[k2];
  }
  __syncthreads();
  // 5. x inverse, second factor, output x < N only
  for (int it = threadIdx.x; it < P * P2; it += kXyThreads) {
    const int qy = it % P, n2 = it / P;
    C2<T> v[P1];
    v[0] = pl[n2 * RS + qy];
#pragma unroll
    for (int k1 = 1; k1 < P1; ++k1) v[k1] = tw_mul_conj(pl[(k1 * P2 + n2) * RS + qy], tw[n2 * k1]);
    dft_out_half<T, P1, 1>(v);
#pragma unroll
    for (int n1 = 0; n1 < H1; ++n1) pl[(n1 * P2 + n2) * RS + qy] = v[n1];
  }
  __syncthreads();
  // 6. y inverse, first factor (rows x < N)
  for (int it = threadIdx.x; it < N * P1; it += kXyThreads) {
    const int x = it % N, k1 = it / N;
    C2<T> v[P2];
    C2<T>* row = pl + x * RS + k1 * P2;
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = row[k2];
    dft<T, P2, 1>(v);
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) row[k2] = v[k2];
  }
  __syncthreads();
  // 7. y inverse, second factor, output y < N: LDS -> global (in place over the input slice)
  for (int it = threadIdx.x; it < N * P2; it += kXyThreads) {
    const int n2 = it % P2, x = it / P2;
    C2<T> v[P1];
    v[0] = pl[x * RS + n2];
#pragma unroll
    for (int k1 = 1; k1 < P1; ++k1) v[k1] = tw_mul_conj(pl[x * RS + k1 * P2 + n2], tw[n2 * k1]);
    dft_out_half<T, P1, 1>(v);
#pragma unroll
    for (int n1 = 0; n1 < H1; ++n1) g[x * N + n1 * P2 + n2] = v[n1];
  }
}

// ---------------------------------------------------------------------------------------
// Z-inverse pass
template <typename T, int N, bool RP, typename R>
__global__ __launch_bounds__(zi_threads<N>()) void k_zinv(const C2<T>* __restrict__ work, R res,
                                                   const TwE<T>* __restrict__ twg) {
  typedef Plan<N> PL;
  constexpr int P = PL::P, P1 = PL::P1, P2 = PL::P2, H1 = PL::H1, RS = P + 1;
  constexpr size_t NG = (size_t)N * N * N;
  C2<T>* buf = lds<T>();
  const TwE<T>* tw = stage_twiddles<T, P>(buf, N * RS, twg);
  const int x = blockIdx.x, p = blockIdx.y;
  const C2<T>* src0 = work + (size_t)p * P * N * N + (size_t)x * N;
  for (int it = threadIdx.x; it < N * P1; it += zi_threads<N>()) {
    const int y = it % N, k1 = it / N;
    C2<T> v[P2];
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = src0[(size_t)(k1 * P2 + k2) * N * N + y];
    dft<T, P2, 1>(v);
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) buf[y * RS + k1 * P2 + k2] = v[k2];
  }
  __syncthreads();
  for (int it = threadIdx.x; it < N * P2; it += zi_threads<N>()) {
    const int n2 = it % P2, y = it / P2;
    C2<T> v[P1];
    v[0] = buf[y * RS + n2];
#pragma unroll
    for (int k1 = 1; k1 < P1; ++k1) v[k1] = tw_mul_conj(buf[y * RS + k1 * P2 + n2], tw[n2 * k1]);
    dft_out_half<T, P1, 1>(v);
    const size_t base = ((size_t)x * N + y) * N + n2;
    if constexpr (RP) {
      T* o0 = res.template v<T>(2 * p, NG) + base;
      const bool has1 = (2 * p + 1) < res.np;
#pragma unroll
      for (int n1 = 0; n1 < H1; ++n1) o0[n1 * P2] = v[n1].r;
      if (has1) {
        T* o1 = res.template v<T>(2 * p + 1, NG) + base;
#pragma unroll
        for (int n1 = 0; n1 < H1; ++n1) o1[n1 * P2] = v[n1].i;
      }
    } else {
      const int kd = res.kind(p);
      C2<T>* o = res.template v<C2<T>>(p, NG) + base;
      if (kd == 0) {
#pragma unroll
        for (int n1 = 0; n1 < H1; ++n1) o[n1 * P2] = v[n1];
      } else {
        // real densities: the two potentials are the real and imaginary parts
#pragma unroll
        for (int n1 = 0; n1 < H1; ++n1) o[n1 * P2] = C2<T>{v[n1].r, T(0)};
        if (kd == 1) {
          C2<T>* o1 = res.template v2<C2<T>>(p, NG) + base;
#pragma unroll
          for (int n1 = 0; n1 < H1; ++n1) o1[n1 * P2] = C2<T>{v[n1].i, T(0)};
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// Kernel spectrum setup (FP64).
__global__ void k_ghat_init(double* __restrict__ g, int ho, double h, double c0) {
  const int total = ho * ho * ho;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int c = i % ho, b = (i / ho) % ho, a = i / (ho * ho);
    const double r2 = double(a) * a + double(b) * b + double(c) * c;
    g[i] = (r2 == 0.0) ? c0 / h : 1.0 / (h * sqrt(r2));
  }
}

// out[..k..] = sum_a cosw[k * ho + a] * in[..a..] along one axis of an ho^3 array.
__global__ void k_axis_cos(const double* __restrict__ in, double* __restrict__ out,
                           const double* __restrict__ cosw, int ho, int axis) {
  const int total = ho * ho * ho;
  const int stride = axis == 0 ? ho * ho : (axis == 1 ? ho : 1);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int k = (i / stride) % ho;
    const int base = i - k * stride;
    double s = 0.0;
    for (int a = 0; a < ho; ++a) s += cosw[k * ho + a] * in[base + a * stride];
    out[i] = s;
  }
}

__global__ void k_ghat_final(const double* __restrict__ in, double* __restrict__ g64,
                             float* __restrict__ g32, double scale, int total) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const double v = in[i] * scale;
    g64[i] = v;
    g32[i] = (float)v;
  }
}

// Kernel spectrum in the position order of the passes: g[qz][qx][qy] = ghat(f(qx), f(qy),
// f(qz)) with f(q) = q / P2 + P1 (q % P2) and the octant folded by min(k, P - k).
template <typename T>
__global__ void k_ghat_positions(const double* __restrict__ oct, T* __restrict__ g, int p,
                                 int p1, int p2) {
  const int ho = p / 2 + 1;
  const size_t total = (size_t)p * p * p;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int qy = (int)(i % p), qx = (int)((i / p) % p), qz = (int)(i / ((size_t)p * p));
    int fx = qx / p2 + p1 * (qx % p2), fy = qy / p2 + p1 * (qy % p2), fz = qz / p2 + p1 * (qz % p2);
    fx = fx <= p - fx ? fx : p - fx;
    fy = fy <= p - fy ? fy : p - fy;
    fz = fz <= p - fz ? fz : p - fz;
    g[i] = (T)oct[((size_t)fx * ho + fy) * ho + fz];
  }
}

// ---------------------------------------------------------------------------------------
template <typename K>
void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)bytes);
}

template <typename T, int N, typename R>
void run_poisson(bool rp, R res, void* work, const void* ghat, const void* tw, hipStream_t s,
                 Trace* tr) {
  typedef Plan<N> PL;
  constexpr int P = PL::P;
  const int np = res.np;
  const int items = rp ? (np + 1) / 2 : np;
  if (items <= 0) return;
  const size_t lds_z = lds_with_twiddles<T, P>((size_t)N * (P + 1));
  const size_t lds_xy = lds_with_twiddles<T, P>((size_t)P * (P + 1));
  C2<T>* w = reinterpret_cast<C2<T>*>(work);
  const TwE<T>* t = reinterpret_cast<const TwE<T>*>(tw);
  const T* gh = reinterpret_cast<const T*>(ghat);
  if (rp) {
    allow_lds(k_zfwd<T, N, true, R>, lds_z);
    allow_lds(k_zinv<T, N, true, R>, lds_z);
  } else {
    allow_lds(k_zfwd<T, N, false, R>, lds_z);
    allow_lds(k_zinv<T, N, false, R>, lds_z);
  }
  allow_lds(k_xy<T, N>, lds_xy);
  dim3 gz(N, items), gxy(P, items);
  {
    TraceScope ts(tr, TR_ZFWD);
    if (rp)
      k_zfwd<T, N, true, R><<<gz, zf_threads<N>(), lds_z, s>>>(res, w, t);
    else
      k_zfwd<T, N, false, R><<<gz, zf_threads<N>(), lds_z, s>>>(res, w, t);
  }
  {
    TraceScope ts(tr, TR_XY);
    k_xy<T, N><<<gxy, kXyThreads, lds_xy, s>>>(w, gh, t);
  }
  {
    TraceScope ts(tr, TR_ZINV);
    if (rp)
      k_zinv<T, N, true, R><<<gz, zi_threads<N>(), lds_z, s>>>(w, res, t);
    else
      k_zinv<T, N, false, R><<<gz, zi_threads<N>(), lds_z, s>>>(w, res, t);
  }
}

constexpr size_t kMaxLds = 160 * 1024;

template <typename T, int N>
constexpr bool fits() {
  return lds_with_twiddles<T, 2 * N>((size_t)(2 * N) * (2 * N + 1)) <= kMaxLds;
}

#define ACE_SIZES(X) X(8) X(9) X(10) X(12) X(15) X(16) X(20) X(24) X(32) X(40) X(48) X(56) X(64)

}  // namespace

bool poisson_size_supported(int n, bool fp64) {
#define ACE_CASE(NN) \
  case NN:           \
    return fp64 ? fits<double, NN>() : fits<float, NN>();
  switch (n) {
    ACE_SIZES(ACE_CASE)
    default:
      return false;
  }
#undef ACE_CASE
}

void launch_kernel_positions(int n, bool fp64, const double* oct, void* gpos, hipStream_t s) {
  const int p = 2 * n, p1 = plan_p1(p), p2 = p / p1;
  const size_t total = (size_t)p * p * p;
  const unsigned blocks = (unsigned)std::min<size_t>(65535, (total + 255) / 256);
  if (fp64)
    k_ghat_positions<double><<<blocks, 256, 0, s>>>(oct, (double*)gpos, p, p1, p2);
  else
    k_ghat_positions<float><<<blocks, 256, 0, s>>>(oct, (float*)gpos, p, p1, p2);
}

size_t poisson_work_bytes_per_item(int n, bool fp64) {
  return (size_t)n * n * (2 * n) * (fp64 ? 16 : 8);
}

void launch_kernel_setup(int n, double h, double c0, const double* cosw, double* tmp0,
                         double* tmp1, double* ghat64, float* ghat32, hipStream_t s) {
  const int p = 2 * n, ho = p / 2 + 1, total = ho * ho * ho;
  const int blocks = (total + 255) / 256;
  k_ghat_init<<<blocks, 256, 0, s>>>(tmp0, ho, h, c0);
  k_axis_cos<<<blocks, 256, 0, s>>>(tmp0, tmp1, cosw, ho, 0);
  k_axis_cos<<<blocks, 256, 0, s>>>(tmp1, tmp0, cosw, ho, 1);
  k_axis_cos<<<blocks, 256, 0, s>>>(tmp0, tmp1, cosw, ho, 2);
  const double scale = h * h * h / ((double)p * p * p);
  k_ghat_final<<<blocks, 256, 0, s>>>(tmp1, ghat64, ghat32, scale, total);
}

template <typename R>
static void dispatch_poisson(int n, bool fp64, bool real_packed, R res, void* work,
                             const void* ghat, const void* tw, hipStream_t s, Trace* tr) {
#define ACE_CASE(NN)                                                                 \
  case NN:                                                                           \
    if constexpr (fits<double, NN>()) {                                              \
      if (fp64) {                                                                    \
        run_poisson<double, NN, R>(real_packed, res, work, ghat, tw, s, tr);         \
        return;                                                                      \
      }                                                                              \
    }                                                                                \
    if (!fp64) run_poisson<float, NN, R>(real_packed, res, work, ghat, tw, s, tr);   \
    return;
  switch (n) {
    ACE_SIZES(ACE_CASE)
    default:
      return;
  }
#undef ACE_CASE
}

void launch_pair_poisson(int n, bool fp64, bool real_packed, const void* phi_a,
                         const void* phi_b, const int* pairs_dev, int np, void* work,
                         void* v_out, const void* ghat, const void* tw, hipStream_t s,
                         Trace* tr) {
  PairsByIndex res{phi_a, phi_b, pairs_dev, v_out, np};
  dispatch_poisson(n, fp64, real_packed, res, work, ghat, tw, s, tr);
}

void launch_pair_slots(int n, bool fp64, const void* phi, const int* slots_dev, int nslots,
                       void* work, void* v_out, const void* ghat, const void* tw, hipStream_t s,
                       Trace* tr) {
  SlotsByIndex res{phi, slots_dev, v_out, nslots};
  dispatch_poisson(n, fp64, false, res, work, ghat, tw, s, tr);
}

void launch_pair_poisson_ptrs(int n, bool fp64, bool real_packed, const PairPtrs* items, int np,
                              void* work, const void* ghat, const void* tw, hipStream_t s,
                              Trace* tr) {
  PairsByPointer res{items, np};
  dispatch_poisson(n, fp64, real_packed, res, work, ghat, tw, s, tr);
}

}  // namespace ace
