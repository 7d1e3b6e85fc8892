// Shared pieces of the pair-Poisson passes (poisson.hip: one launch sequence per system or
// box edge; poisson_queue.hip: persistent passes over many systems of any edges): launch
// geometry, LDS layout, the pair resolvers and the per-plane bodies of the three passes.
// The bodies compute every item the same way whatever the launch shape, so the two files' 
// kernels give the same bits.
#pragma once

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
// threads of the one-system XY pass (one P x P plane per workgroup): 512 where the phases are
// small (FP32 up to edge 40, FP64 up to 32), else 1024 -- measured per edge with the planes of
// a few dozen transforms (edge 32: 28.6 against 34.5 us, edge 40: 59.0 against 62.8 us, edge 48:
// 77.6 against 71.1 us for 512 against 1024 threads); every shape gives the same bits.
#ifndef ACE_XY_THREADS
#define ACE_XY_THREADS 0
#endif
template <typename T, int N>
constexpr int xy_threads() {
  return ACE_XY_THREADS > 0 ? ACE_XY_THREADS : (N <= (sizeof(T) == 4 ? 40 : 32) ? 512 : 1024);
}

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
// The indices are clamped to [0, na) and [0, nb) so that no access leaves the orbital arrays
// (a list that the host did not check); an index out of range is recorded in the status word
// (ACE_ERR_INVALID = -1, info = the pair), once.
struct PairsByIndex {
  const void* pa;
  const void* pb;
  const int* pairs;
  void* vout;
  int np;
  int na, nb;
  int* status;
  __device__ __forceinline__ int clamp_index(int j, int lim, int q) const {
    if (j >= 0 && j < lim) return j;
    if (status && atomicCAS(status, 0, -1) == 0) status[1] = q;
    return j < 0 ? 0 : lim - 1;
  }
  template <typename E>
  __device__ __forceinline__ const E* a(int q, size_t ng) const {
    return reinterpret_cast<const E*>(pa) + (size_t)clamp_index(pairs[2 * q], na, q) * ng;
  }
  template <typename E>
  __device__ __forceinline__ const E* b(int q, size_t ng) const {
    return reinterpret_cast<const E*>(pb) + (size_t)clamp_index(pairs[2 * q + 1], nb, q) * ng;
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
// Z-forward pass body: x-plane x of transform p of the resolver res (its pair density formed
// on the fly), pruned FFT along z, written transposed into this transform's work volume wp
// [qz][x][y].  buf: N (P+1) complex values of LDS; tw: the table twiddles in LDS.
template <typename T, int N, bool RP, typename R>
__device__ __forceinline__ void zfwd_plane(const R& res, int p, int x, C2<T>* __restrict__ wp,
                                           const TwE<T>* __restrict__ tw,
                                           C2<T>* __restrict__ buf, int tid, int nt) {
  typedef Plan<N> PL;
  constexpr int P = PL::P, P1 = PL::P1, P2 = PL::P2, H1 = PL::H1, RS = P + 1;
  constexpr size_t NG = (size_t)N * N * N;
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

  for (int it = tid; it < N * P2; it += nt) {
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
  C2<T>* dst0 = wp + (size_t)x * N;
  for (int it = tid; it < N * P1; it += nt) {
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
// XY pass body: K consecutive qz planes of one transform, each a whole P x P plane in LDS
// (plane j at pl + j P (P+1)), worked by nt threads (tid = this thread).  g: the first
// plane's N x N slice (planes g_stride elements apart), gz: its kernel spectrum in position
// order [qx][qy] (planes P^2 apart), tw: the table twiddles in LDS.  Every item of a phase
// is computed the same way whatever K and nt are, so all launch shapes give the same bits.
template <typename T, int N, int K>
__device__ __forceinline__ void xy_planes(C2<T>* __restrict__ g, size_t g_stride,
                                          const T* __restrict__ gz, C2<T>* __restrict__ pl,
                                          const TwE<T>* __restrict__ tw, int tid, int nt) {
  typedef Plan<N> PL;
  constexpr int P = PL::P, P1 = PL::P1, P2 = PL::P2, H1 = PL::H1, RS = P + 1;
  constexpr int PS = P * RS;  // LDS elements per plane
  // Phases 1 and 7 give each wavefront about 64 / P2 rows of P2 consecutive elements.  With
  // the row stride P + 1, consecutive rows start one bank pair apart and their elements fall
  // on the same LDS banks; so item group q takes row x = (q mod XS) N / XS + q div XS, rows
  // N / XS apart (edge 48: 58.0-58.5 against 58.9-59.4 us).  Only the assignment of items to
  // threads changes, not what an item computes.  (The z passes' LDS phases have the same
  // pattern, but spreading their rows measured no faster.)
  constexpr int XS = N % 4 == 0 ? 4 : 1;
  // 1. y forward, first factor (rows x < N, input y < N): global -> LDS
  for (int it = tid; it < K * N * P2; it += nt) {
    const int j = it / (N * P2), r = it - j * (N * P2);
    const int n2 = r % P2, q = r / P2, x = (q % XS) * (N / XS) + q / XS;
    const C2<T>* gj = g + j * g_stride;
    C2<T>* pj = pl + j * PS;
    C2<T> v[P1];
#pragma unroll
    for (int n1 = 0; n1 < H1; ++n1) v[n1] = gj[x * N + n1 * P2 + n2];
    dft_in_half<T, P1, -1>(v);
    pj[x * RS + n2] = v[0];
#pragma unroll
    for (int k1 = 1; k1 < P1; ++k1) pj[x * RS + k1 * P2 + n2] = tw_mul(v[k1], tw[n2 * k1]);
  }
  __syncthreads();
  // 2. y forward, second factor
  for (int it = tid; it < K * N * P1; it += nt) {
    const int j = it / (N * P1), r = it - j * (N * P1);
    const int x = r % N, k1 = r / N;
    C2<T> v[P2];
    C2<T>* row = pl + j * PS + x * RS + k1 * P2;
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = row[k2];
    dft<T, P2, -1>(v);
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) row[k2] = v[k2];
  }
  __syncthreads();
  // 3. x forward, first factor (columns qy, input x < N)
  for (int it = tid; it < K * P * P2; it += nt) {
    const int j = it / (P * P2), r = it - j * (P * P2);
    const int qy = r % P, n2 = r / P;
    C2<T>* pj = pl + j * PS;
    C2<T> v[P1];
#pragma unroll
    for (int n1 = 0; n1 < H1; ++n1) v[n1] = pj[(n1 * P2 + n2) * RS + qy];
    dft_in_half<T, P1, -1>(v);
    pj[n2 * RS + qy] = v[0];
#pragma unroll
    for (int k1 = 1; k1 < P1; ++k1) pj[(k1 * P2 + n2) * RS + qy] = tw_mul(v[k1], tw[n2 * k1]);
  }
  // the kernel spectrum values of this thread's first phase-4 item are requested before the
  // barrier, so that their latency overlaps the wait and the phase's LDS reads
  T gpre[P2];
  if (tid < K * P * P1) {
    const int j = tid / (P * P1), r = tid - j * (P * P1);
    const int qy = r % P, k1 = r / P;
    const T* gj = gz + (size_t)j * P * P;
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) gpre[k2] = gj[(k1 * P2 + k2) * P + qy];
  }
  __syncthreads();
  // 4. x forward second factor, kernel multiply, x inverse first factor (in registers)
  for (int it = tid; it < K * P * P1; it += nt) {
    const int j = it / (P * P1), r = it - j * (P * P1);
    const int qy = r % P, k1 = r / P;
    C2<T>* pj = pl + j * PS;
    const T* gj = gz + (size_t)j * P * P;
    C2<T> v[P2];
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = pj[(k1 * P2 + k2) * RS + qy];
    if (it != tid) {
#pragma unroll
      for (int k2 = 0; k2 < P2; ++k2) gpre[k2] = gj[(k1 * P2 + k2) * P + qy];
    }
    dft<T, P2, -1>(v);
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = cscale(v[k2], gpre[k2]);
    dft<T, P2, 1>(v);
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) pj[(k1 * P2 + k2) * RS + qy] = v[k2];
  }
  __syncthreads();
  // 5. x inverse, second factor, output x < N only
  for (int it = tid; it < K * P * P2; it += nt) {
    const int j = it / (P * P2), r = it - j * (P * P2);
    const int qy = r % P, n2 = r / P;
    C2<T>* pj = pl + j * PS;
    C2<T> v[P1];
    v[0] = pj[n2 * RS + qy];
#pragma unroll
    for (int k1 = 1; k1 < P1; ++k1) v[k1] = tw_mul_conj(pj[(k1 * P2 + n2) * RS + qy], tw[n2 * k1]);
    dft_out_half<T, P1, 1>(v);
#pragma unroll
    for (int n1 = 0; n1 < H1; ++n1) pj[(n1 * P2 + n2) * RS + qy] = v[n1];
  }
  __syncthreads();
  // 6. y inverse, first factor (rows x < N)
  for (int it = tid; it < K * N * P1; it += nt) {
    const int j = it / (N * P1), r = it - j * (N * P1);
    const int x = r % N, k1 = r / N;
    C2<T> v[P2];
    C2<T>* row = pl + j * PS + x * RS + k1 * P2;
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = row[k2];
    dft<T, P2, 1>(v);
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) row[k2] = v[k2];
  }
  __syncthreads();
  // 7. y inverse, second factor, output y < N: LDS -> global (in place over the input slice)
  for (int it = tid; it < K * N * P2; it += nt) {
    const int j = it / (N * P2), r = it - j * (N * P2);
    const int n2 = r % P2, q = r / P2, x = (q % XS) * (N / XS) + q / XS;
    C2<T>* gj = g + j * g_stride;
    C2<T>* pj = pl + j * PS;
    C2<T> v[P1];
    v[0] = pj[x * RS + n2];
#pragma unroll
    for (int k1 = 1; k1 < P1; ++k1) v[k1] = tw_mul_conj(pj[x * RS + k1 * P2 + n2], tw[n2 * k1]);
    dft_out_half<T, P1, 1>(v);
#pragma unroll
    for (int n1 = 0; n1 < H1; ++n1) gj[x * N + n1 * P2 + n2] = v[n1];
  }
}

// ---------------------------------------------------------------------------------------
// Z-inverse pass body: x-plane x of transform p, read from its work volume wp [qz][x][y],
// inverse FFT along z keeping z < N, written to the resolver's output volume(s).
template <typename T, int N, bool RP, typename R>
__device__ __forceinline__ void zinv_plane(const C2<T>* __restrict__ wp, const R& res, int p,
                                           int x, const TwE<T>* __restrict__ tw,
                                           C2<T>* __restrict__ buf, int tid, int nt) {
  typedef Plan<N> PL;
  constexpr int P = PL::P, P1 = PL::P1, P2 = PL::P2, H1 = PL::H1, RS = P + 1;
  constexpr size_t NG = (size_t)N * N * N;
  const C2<T>* src0 = wp + (size_t)x * N;
  for (int it = tid; it < N * P1; it += nt) {
    const int y = it % N, k1 = it / N;
    C2<T> v[P2];
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = src0[(size_t)(k1 * P2 + k2) * N * N + y];
    dft<T, P2, 1>(v);
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) buf[y * RS + k1 * P2 + k2] = v[k2];
  }
  __syncthreads();
  for (int it = tid; it < N * P2; it += nt) {
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

template <typename K>
void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)bytes);
}

constexpr size_t kMaxLds = 160 * 1024;

// the whole P x P plane of the XY pass fits in LDS
template <typename T, int N>
constexpr bool fits() {
  return lds_with_twiddles<T, 2 * N>((size_t)(2 * N) * (2 * N + 1)) <= kMaxLds;
}

// Otherwise (FP64 at edges 56 and 64) the XY pass keeps only the N y-transformed rows in LDS
// and runs the x transforms over strips of SW columns: the widest divisor SW <= P/2 of P whose
// strip fits beside the rows, or 0.
template <typename T, int N>
constexpr int strip_width() {
  constexpr int P = 2 * N;
  for (int sw = P / 2; sw >= 2; --sw)
    if (P % sw == 0 &&
        lds_with_twiddles<T, P>((size_t)N * (P + 1) + (size_t)P * (sw + 1)) <= kMaxLds)
      return sw;
  return 0;
}
template <typename T, int N>
constexpr size_t strip_lds() {
  constexpr int P = 2 * N;
  return lds_with_twiddles<T, P>((size_t)N * (P + 1) + (size_t)P * (strip_width<T, N>() + 1));
}

// the pair-Poisson passes are compiled for this edge and precision
template <typename T, int N>
constexpr bool supported() {
  return fits<T, N>() || strip_width<T, N>() > 0;
}

// XY pass of one qz plane with the rows-and-strips layout: rows x < N of the y transform in
// LDS R[x][qy] (stride P + 1), then for each strip of SW columns the x transform forward, the
// kernel multiply and the x transform inverse through a strip buffer S[qx][c] (stride SW + 1),
// the N kept rows written back to R, then the y inverse.  Every item is computed as in
// xy_planes, only the x transforms go strip by strip.  g: the plane's N x N slice, gz: its
// kernel spectrum [qx][qy], pl: R followed by S, tw: table twiddles in LDS.
template <typename T, int N, int SW>
__device__ __forceinline__ void xy_strips(C2<T>* __restrict__ g, const T* __restrict__ gz,
                                          C2<T>* __restrict__ pl, const TwE<T>* __restrict__ tw,
                                          int tid, int nt) {
  typedef Plan<N> PL;
  constexpr int P = PL::P, P1 = PL::P1, P2 = PL::P2, H1 = PL::H1, RS = P + 1, SS = SW + 1;
  static_assert(P % SW == 0, "whole strips");
  C2<T>* R = pl;
  C2<T>* S = pl + N * RS;
  // 1. y forward, first factor (rows x < N, input y < N): global -> R
  for (int it = tid; it < N * P2; it += nt) {
    const int n2 = it % P2, x = it / P2;
    C2<T> v[P1];
#pragma unroll
    for (int n1 = 0; n1 < H1; ++n1) v[n1] = g[x * N + n1 * P2 + n2];
    dft_in_half<T, P1, -1>(v);
    R[x * RS + n2] = v[0];
#pragma unroll
    for (int k1 = 1; k1 < P1; ++k1) R[x * RS + k1 * P2 + n2] = tw_mul(v[k1], tw[n2 * k1]);
  }
  __syncthreads();
  // 2. y forward, second factor
  for (int it = tid; it < N * P1; it += nt) {
    const int x = it % N, k1 = it / N;
    C2<T> v[P2];
    C2<T>* row = R + x * RS + k1 * P2;
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = row[k2];
    dft<T, P2, -1>(v);
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) row[k2] = v[k2];
  }
  __syncthreads();
  for (int q0 = 0; q0 < P; q0 += SW) {
    // 3a. x forward, first factor, columns q0 .. q0 + SW - 1: R -> S
    for (int it = tid; it < SW * P2; it += nt) {
      const int c = it % SW, n2 = it / SW, qy = q0 + c;
      C2<T> v[P1];
#pragma unroll
      for (int n1 = 0; n1 < H1; ++n1) v[n1] = R[(n1 * P2 + n2) * RS + qy];
      dft_in_half<T, P1, -1>(v);
      S[n2 * SS + c] = v[0];
#pragma unroll
      for (int k1 = 1; k1 < P1; ++k1) S[(k1 * P2 + n2) * SS + c] = tw_mul(v[k1], tw[n2 * k1]);
    }
    __syncthreads();
    // 3b. x forward second factor, kernel multiply, x inverse first factor
    for (int it = tid; it < SW * P1; it += nt) {
      const int c = it % SW, k1 = it / SW, qy = q0 + c;
      C2<T> v[P2];
#pragma unroll
      for (int k2 = 0; k2 < P2; ++k2) v[k2] = S[(k1 * P2 + k2) * SS + c];
      dft<T, P2, -1>(v);
#pragma unroll
      for (int k2 = 0; k2 < P2; ++k2) v[k2] = cscale(v[k2], gz[(k1 * P2 + k2) * P + qy]);
      dft<T, P2, 1>(v);
#pragma unroll
      for (int k2 = 0; k2 < P2; ++k2) S[(k1 * P2 + k2) * SS + c] = v[k2];
    }
    __syncthreads();
    // 3c. x inverse, second factor, rows x < N: S -> R
    for (int it = tid; it < SW * P2; it += nt) {
      const int c = it % SW, n2 = it / SW, qy = q0 + c;
      C2<T> v[P1];
      v[0] = S[n2 * SS + c];
#pragma unroll
      for (int k1 = 1; k1 < P1; ++k1) v[k1] = tw_mul_conj(S[(k1 * P2 + n2) * SS + c], tw[n2 * k1]);
      dft_out_half<T, P1, 1>(v);
#pragma unroll
      for (int n1 = 0; n1 < H1; ++n1) R[(n1 * P2 + n2) * RS + qy] = v[n1];
    }
    __syncthreads();
  }
  // 4. y inverse, first factor (rows x < N)
  for (int it = tid; it < N * P1; it += nt) {
    const int x = it % N, k1 = it / N;
    C2<T> v[P2];
    C2<T>* row = R + x * RS + k1 * P2;
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) v[k2] = row[k2];
    dft<T, P2, 1>(v);
#pragma unroll
    for (int k2 = 0; k2 < P2; ++k2) row[k2] = v[k2];
  }
  __syncthreads();
  // 5. y inverse, second factor, output y < N: R -> global (in place over the input slice)
  for (int it = tid; it < N * P2; it += nt) {
    const int n2 = it % P2, x = it / P2;
    C2<T> v[P1];
    v[0] = R[x * RS + n2];
#pragma unroll
    for (int k1 = 1; k1 < P1; ++k1) v[k1] = tw_mul_conj(R[x * RS + k1 * P2 + n2], tw[n2 * k1]);
    dft_out_half<T, P1, 1>(v);
#pragma unroll
    for (int n1 = 0; n1 < H1; ++n1) g[x * N + n1 * P2 + n2] = v[n1];
  }
}

#define ACE_SIZES(X) X(8) X(9) X(10) X(12) X(15) X(16) X(20) X(24) X(32) X(40) X(48) X(56) X(64)


}  // namespace

}  // namespace ace
