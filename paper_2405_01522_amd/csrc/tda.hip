// Coupling block of the RHF Tamm-Dancoff matrix for real orbitals (paper Sec. 2, Eq. (7)):
//   C[ia][jb] = delta_M (ai|jb) - (ab|ji)
//             = delta_M * CJ[ia][jb] - CK[ij][ab]
//   CJ[ia][jb] = dV sum_r (phi_i phi_a)(r) v_jb(r)      ("exchange" integrals, Eq. (7))
//   CK[ij][ab] = dV sum_r v_ij(r) (phi_a phi_b)(r)      ("Coulomb" integrals)
// using the symmetry (pq|rs) = (rs|pq) of real orbitals, so only the n_occ*n_virt and
// n_occ(n_occ+1)/2 pair potentials are solved.  The products phi_i phi_a and phi_a phi_b are
// generated while tiles are staged, never stored.  Both contractions are split over the grid
// (split-K) with FP64 partial sums reduced in a fixed order.
#include <algorithm>

#include "common.hpp"
#include "tda.hpp"

namespace ace {

namespace {

constexpr int BM = 64, BN = 64, BK = 16, kThreads = 256;
constexpr int kSub = 256;  // points summed in the storage precision before an FP64 add

template <typename T>
struct Op {
  const T* p;   // rows of length ng, or first factor
  const T* q;   // second factor (product mode) or null
  int div;      // product mode: row -> (row / div, row % div)
  int tri;      // product mode over pairs lo <= hi instead: row t = hi (hi + 1) / 2 + lo
};

// (lo, hi) of triangular pair index t = hi (hi + 1) / 2 + lo, lo <= hi
__device__ __forceinline__ void tri_decode(int t, int* lo, int* hi) {
  int h = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((h + 1) * (h + 2) / 2 <= t) ++h;
  while (h * (h + 1) / 2 > t) --h;
  *hi = h;
  *lo = t - h * (h + 1) / 2;
}

// first- and second-factor rows of operand row `row` (product mode)
template <typename T>
__device__ __forceinline__ void op_rows(const Op<T>& o, int row, int* ip, int* iq) {
  if (o.tri) {
    tri_decode(row, ip, iq);
  } else {
    *ip = row / o.div;
    *iq = row % o.div;
  }
}

template <typename T>
__device__ __forceinline__ T op_load(const Op<T>& o, int row, size_t k, size_t ng) {
  if (o.q) {
    int ip, iq;
    op_rows(o, row, &ip, &iq);
    return o.p[(size_t)ip * ng + k] * o.q[(size_t)iq * ng + k];
  }
  return o.p[(size_t)row * ng + k];
}

// part[z][m][n] = sum_{k in split z} A(m,k) B(n,k)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gemm_nt(Op<T> A, int M, Op<T> B, int N, size_t ng,
                                                      size_t kchunk, double* __restrict__ part) {
  __shared__ T As[BK][BM + 1];
  __shared__ T Bs[BK][BN + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const size_t k0 = (size_t)blockIdx.z * kchunk;
  const size_t k1 = k0 + kchunk < ng ? k0 + kchunk : ng;
  double acc[4][4];
  T sub[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = 0.0;
      sub[i][j] = T(0);
    }
  int steps = 0;
  for (size_t kt = k0; kt < k1; kt += BK) {
    for (int idx = threadIdx.x; idx < BM * BK; idx += kThreads) {
      const int r = idx / BK, kk = idx % BK;
      const size_t k = kt + kk;
      const int m = m0 + r, n = n0 + r;
      As[kk][r] = (m < M && k < k1) ? op_load(A, m, k, ng) : T(0);
      Bs[kk][r] = (n < N && k < k1) ? op_load(B, n, k, ng) : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) sub[i][j] += a[i] * b[j];
    }
    __syncthreads();
    if (++steps == kSub / BK) {
      steps = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j] += (double)sub[i][j];
          sub[i][j] = T(0);
        }
    }
  }
  double* dst = part + (size_t)blockIdx.z * M * N;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + ty + 16 * i, n = n0 + tx + 16 * j;
      if (m < M && n < N) dst[(size_t)m * N + n] = acc[i][j] + (double)sub[i][j];
    }
}

// ---------------------------------------------------------------------------------------
// FP32-input contraction on the matrix cores with split BF16 operands ("bf16x3"):
// part[z][m][n] = sum_{k in split z} A(m,k) B(n,k), each FP32 operand split as x = hi + lo
// (hi = RNE bf16(x), lo = RNE bf16(x - hi)) and A B ~ Ahi Bhi + Ahi Blo + Alo Bhi, accumulated
// in FP32 by v_mfma_f32_16x16x32_bf16 (relative error of one product ~2^-16, the dropped
// Alo Blo term).  Block tile 128 x 128, 4 waves of 64 x 64 (4 x 4 MFMA tiles each); operand
// tiles of 128 rows x 64 points are staged through LDS as hi / lo BF16 rows of stride 72
// (16-byte aligned rows; one 16-byte fragment read per lane), with coalesced row-segment
// loads.  Generated operands (products of two orbitals) are formed in FP32 while staging.  Lane layout of the 16x16x32 instruction:
// A[i][k] in lane i + 16 (k / 8), element k % 8 (B likewise with j); D[i][j] in lane
// j + 16 (i / 4), element i % 4 (output layout checked on gfx950).
constexpr int MT = 128, KB = 64, LB = KB + 8;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Stage one operand tile (128 rows x 64 points from point kt) as hi / lo BF16 rows.  Sixteen
// consecutive lanes read one row (4 consecutive points each, one 16-byte load when VEC), so
// every load instruction covers four 256-byte row segments.  Loads are unconditional (row and
// point clamped); rows >= M and points >= k1 are zeroed.
// rows[r] (r < MT): element offsets of the tile row's first-factor row and second-factor row
// (product mode), computed once per workgroup so that no index arithmetic beyond one add is
// left in the K loop.
__device__ __forceinline__ void tile_rows(const Op<float>& o, int m0, int M, size_t ng, int r,
                                          longlong2* rows) {
  const int m = m0 + r;
  const int mc = m < M ? m : M - 1;
  int ip = mc, iq = 0;
  if (o.q) op_rows(o, mc, &ip, &iq);
  rows[r] = longlong2{(long long)((size_t)ip * ng), (long long)((size_t)iq * ng)};
}

// EDGE: the tile reaches past row M or the step past the chunk end k1, so the rows and points
// outside are zeroed and the loads clamped; interior steps (EDGE false) skip both (the same
// values: the zeroing factor is then 1).
template <bool VEC, bool PROD, bool EDGE>
__device__ __forceinline__ void stage_tile(const Op<float>& o, const longlong2* rows, int m0, int M,
                                           size_t kt, size_t k1, size_t ng, __bf16* H,
                                           __bf16* L) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  const int c4 = (threadIdx.x & 15) * 4;
  const size_t k = kt + c4;
#pragma unroll
  for (int pass = 0; pass < MT / 16; ++pass) {
    const int r = pass * 16 + (threadIdx.x >> 4);
    const bool valid = m0 + r < M;
    const longlong2 rr = rows[r];
    const float* p = o.p + rr.x;
    float x[4], y[4] = {};  // y: the second factor of a product operand
    if constexpr (VEC) {
      const size_t kc = !EDGE || k + 3 < ng ? k : ng - 4;
      const float4 a = *reinterpret_cast<const float4*>(p + kc);
      x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
      if constexpr (PROD) {
        const float4 b = *reinterpret_cast<const float4*>(o.q + rr.y + kc);
        y[0] = b.x; y[1] = b.y; y[2] = b.z; y[3] = b.w;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const size_t kc = !EDGE || k + e < ng ? k + e : ng - 1;
        x[e] = p[kc];
        if constexpr (PROD) y[e] = o.q[rr.y + kc];
      }
    }
    bf16x4 h, l;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      // zeroing by a 0 / 1 factor (all loaded values are finite), not a select the compiler
      // may turn into a branch around the load; exact, so interior and edge steps agree
      const float xe = EDGE ? x[e] * ((valid && k + e < k1) ? 1.f : 0.f) : x[e];
      const float v = PROD ? xe * y[e] : xe;
      const __bf16 vh = (__bf16)v;
      h[e] = vh;
      // the low part of a product from the exact product (one rounding), of a plain value
      // from the exact difference
      l[e] = (__bf16)(PROD ? fmaf(xe, y[e], -(float)vh) : v - (float)vh);
    }
    *reinterpret_cast<bf16x4*>(H + r * LB + c4) = h;
    *reinterpret_cast<bf16x4*>(L + r * LB + c4) = l;
  }
}

// The two halves of stage_tile for a plain (non-product) operand, so that the global loads of
// the next tile can be in flight during the current tile's products: load_rows reads this
// thread's 4-point segments of the tile's rows, store_rows splits and stores them.
template <bool VEC>
__device__ __forceinline__ void load_rows(const Op<float>& o, const longlong2* rows, size_t kt,
                                          size_t ng, float4* x) {
  const int c4 = (threadIdx.x & 15) * 4;
  const size_t k = kt + c4;
#pragma unroll
  for (int pass = 0; pass < MT / 16; ++pass) {
    const int r = pass * 16 + (threadIdx.x >> 4);
    const float* p = o.p + rows[r].x;
    if constexpr (VEC) {
      const size_t kc = k + 3 < ng ? k : ng - 4;
      x[pass] = *reinterpret_cast<const float4*>(p + kc);
    } else {
      float e4[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) e4[e] = p[k + e < ng ? k + e : ng - 1];
      x[pass] = float4{e4[0], e4[1], e4[2], e4[3]};
    }
  }
}

template <bool EDGE>
__device__ __forceinline__ void store_rows(const float4* x, int m0, int M, size_t kt, size_t k1,
                                           __bf16* H, __bf16* L) {
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  const int c4 = (threadIdx.x & 15) * 4;
  const size_t k = kt + c4;
#pragma unroll
  for (int pass = 0; pass < MT / 16; ++pass) {
    const int r = pass * 16 + (threadIdx.x >> 4);
    const bool valid = m0 + r < M;
    const float xv[4] = {x[pass].x, x[pass].y, x[pass].z, x[pass].w};
    bf16x4 h, l;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float v = EDGE ? xv[e] * ((valid && k + e < k1) ? 1.f : 0.f) : xv[e];
      const __bf16 vh = (__bf16)v;
      h[e] = vh;
      l[e] = (__bf16)(v - (float)vh);
    }
    *reinterpret_cast<bf16x4*>(H + r * LB + c4) = h;
    *reinterpret_cast<bf16x4*>(L + r * LB + c4) = l;
  }
}

// tri != 0: M == N and the result is symmetric; blockIdx.x enumerates only the tiles (bx, by)
// with bx <= by (blockIdx.y unused) and the lower tiles are never computed.
// PREF: B is a plain operand whose next tile is prefetched into registers during the products
template <bool VEC, bool PREF>
__global__ __launch_bounds__(256) void k_gemm_nt_mfma(Op<float> A, int M, Op<float> B, int N,
                                                      size_t ng, size_t kchunk,
                                                      float* __restrict__ part, int tri) {
  __shared__ __align__(16) __bf16 Ah[MT * LB];
  __shared__ __align__(16) __bf16 Al[MT * LB];
  __shared__ __align__(16) __bf16 Bh[MT * LB];
  __shared__ __align__(16) __bf16 Bl[MT * LB];
  __shared__ longlong2 rows_a[MT], rows_b[MT];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;  // wave's 64 x 64 quadrant
  int bx = blockIdx.x, by = blockIdx.y;
  if (tri) {
    const int u = blockIdx.x;
    int t = (int)((sqrtf(8.0f * u + 1.0f) - 1.0f) * 0.5f);
    while ((t + 1) * (t + 2) / 2 <= u) ++t;
    while (t * (t + 1) / 2 > u) --t;
    by = t;
    bx = u - t * (t + 1) / 2;
  }
  const int m0 = bx * MT, n0 = by * MT;
  const size_t k0 = (size_t)blockIdx.z * kchunk;
  const size_t k1 = k0 + kchunk < ng ? k0 + kchunk : ng;
  if (threadIdx.x < MT)
    tile_rows(A, m0, M, ng, threadIdx.x, rows_a);
  else if (threadIdx.x < 2 * MT)
    tile_rows(B, n0, N, ng, threadIdx.x - MT, rows_b);
  __syncthreads();
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int li = lane & 15, lg = lane >> 4;
  float4 xb[MT / 16];
  if constexpr (PREF) load_rows<VEC>(B, rows_b, k0, ng, xb);
  for (size_t kt = k0; kt < k1; kt += KB) {
    // uniform per workgroup and step: whether the A / B tile needs its rows or points masked
    const bool step_in = kt + KB <= k1;
    const bool edge_a = !step_in || m0 + MT > M, edge_b = !step_in || n0 + MT > N;
    if constexpr (PREF) {
      if (edge_b)
        store_rows<true>(xb, n0, N, kt, k1, Bh, Bl);
      else
        store_rows<false>(xb, n0, N, kt, k1, Bh, Bl);
      if (kt + KB < k1) load_rows<VEC>(B, rows_b, kt + KB, ng, xb);
    }
    // product (generated) operands load two rows; the choice is uniform per launch
    if (A.q) {
      if (edge_a)
        stage_tile<VEC, true, true>(A, rows_a, m0, M, kt, k1, ng, Ah, Al);
      else
        stage_tile<VEC, true, false>(A, rows_a, m0, M, kt, k1, ng, Ah, Al);
    } else {
      if (edge_a)
        stage_tile<VEC, false, true>(A, rows_a, m0, M, kt, k1, ng, Ah, Al);
      else
        stage_tile<VEC, false, false>(A, rows_a, m0, M, kt, k1, ng, Ah, Al);
    }
    if constexpr (!PREF) {
      if (B.q) {
        if (edge_b)
          stage_tile<VEC, true, true>(B, rows_b, n0, N, kt, k1, ng, Bh, Bl);
        else
          stage_tile<VEC, true, false>(B, rows_b, n0, N, kt, k1, ng, Bh, Bl);
      } else {
        if (edge_b)
          stage_tile<VEC, false, true>(B, rows_b, n0, N, kt, k1, ng, Bh, Bl);
        else
          stage_tile<VEC, false, false>(B, rows_b, n0, N, kt, k1, ng, Bh, Bl);
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KB; ks += 32) {
      bf16x8 bh[4], bl[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int co = (wc * 64 + t * 16 + li) * LB + ks + 8 * lg;
        bh[t] = *reinterpret_cast<const bf16x8*>(Bh + co);
        bl[t] = *reinterpret_cast<const bf16x8*>(Bl + co);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int ro = (wr * 64 + i * 16 + li) * LB + ks + 8 * lg;
        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(Ah + ro);
        const bf16x8 al = *reinterpret_cast<const bf16x8*>(Al + ro);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  float* dst = part + (size_t)blockIdx.z * M * N;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wr * 64 + i * 16 + 4 * lg + r;
        const int n = n0 + wc * 64 + j * 16 + li;
        if (m < M && n < N) dst[(size_t)m * N + n] = acc[i][j][r];
      }
}

__global__ void k_split_reduce_f32(const float* __restrict__ part, int nsplit, size_t count,
                                   double scale, double* __restrict__ out, int ncols) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x) {
    if (ncols > 0 && (int)(i / ncols) / MT > (int)(i % ncols) / MT) continue;
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += (double)part[(size_t)z * count + i];
    out[i] = s * scale;
  }
}

__global__ void k_split_reduce(const double* __restrict__ part, int nsplit, size_t count,
                               double scale, double* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += part[(size_t)z * count + i];
    out[i] = s * scale;
  }
}

// C[ia][jb] = delta_M CJ[ia][jb] - CK[ij][ab], symmetrised: CJ is taken from the computed
// (upper) tile of the pair (ia, jb) / (jb, ia), averaged on diagonal tiles.  CK holds the
// pairs i <= j and a <= b only ((ij|ab) is symmetric in both for real orbitals).
// tile > 0: only tiles with row-tile <= col-tile of CJ hold data.
__global__ void k_tda_assemble(const double* __restrict__ cj, const double* __restrict__ ck,
                               int no, int nv, int delta_m, double* __restrict__ c, int tile) {
  const size_t nov = (size_t)no * nv, nvt = (size_t)nv * (nv + 1) / 2;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < nov * nov;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t row = idx / nov, col = idx % nov;
    const int i = (int)(row / nv), a = (int)(row % nv), j = (int)(col / nv), b = (int)(col % nv);
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    const size_t q = (size_t)hi * (hi + 1) / 2 + lo;
    const int alo = a < b ? a : b, ahi = a < b ? b : a;
    const double k = ck[q * nvt + (size_t)ahi * (ahi + 1) / 2 + alo];
    double jv;
    const int tr = tile > 0 ? (int)row / tile : 0, tc = tile > 0 ? (int)col / tile : 0;
    if (tr < tc)
      jv = cj[idx];
    else if (tr > tc)
      jv = cj[col * nov + row];
    else
      jv = 0.5 * (cj[idx] + cj[col * nov + row]);
    c[idx] = delta_m * jv - k;
  }
}

// CJ[row][col] from the (possibly upper-tile-only) storage, symmetrised as in k_tda_assemble
__device__ __forceinline__ double cj_get(const double* __restrict__ cj, size_t nov, size_t row,
                                        size_t col, int tile) {
  const int tr = tile > 0 ? (int)row / tile : 0, tc = tile > 0 ? (int)col / tile : 0;
  if (tr < tc) return cj[row * nov + col];
  if (tr > tc) return cj[col * nov + row];
  return 0.5 * (cj[row * nov + col] + cj[col * nov + row]);
}

// RHF B block for real orbitals (Eq. (3), spin-adapted Eq. (5)):
//   B[ia][jb] = delta_M (ia|bj) - (ib|aj) = delta_M CJ[ia][jb] - CJ[ib][ja]
__global__ void k_tdhf_b_assemble(const double* __restrict__ cj, int no, int nv, int delta_m,
                                  double* __restrict__ b, int tile) {
  const size_t nov = (size_t)no * nv;
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < nov * nov;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t row = idx / nov, col = idx % nov;
    const int i = (int)(row / nv), a = (int)(row % nv), j = (int)(col / nv), bb = (int)(col % nv);
    const double direct = cj_get(cj, nov, row, col, tile);
    const double swapped = cj_get(cj, nov, (size_t)i * nv + bb, (size_t)j * nv + a, tile);
    b[idx] = delta_m * direct - swapped;
  }
}

template <typename T>
void tda_impl(const void* occ, int no, const void* virt, int nv, const void* v_ov,
              const void* v_oo, size_t ng, double dv, int delta_m, void* ws, const TdaWork& w,
              double* c_out, double* b_out, hipStream_t s, Trace* tr) {
  const int nov = no * nv, noo = no * (no + 1) / 2, nvv = nv * (nv + 1) / 2;
  char* base = (char*)ws;
  double* pj = (double*)(base + w.off_pj);
  double* pk = (double*)(base + w.off_pk);
  double* cj = (double*)(base + w.off_cj);
  double* ck = (double*)(base + w.off_ck);
  Op<T> a_ov{(const T*)occ, (const T*)virt, nv, 0};
  Op<T> b_ov{(const T*)v_ov, nullptr, 1, 0};
  Op<T> a_oo{(const T*)v_oo, nullptr, 1, 0};
  Op<T> b_vv{(const T*)virt, (const T*)virt, nv, 1};  // pairs a <= b
  const size_t cntj = (size_t)nov * nov, cntk = (size_t)noo * nvv;
  const unsigned rbj = (unsigned)std::min<size_t>(4096, (cntj + 255) / 256);
  const unsigned rbk = (unsigned)std::min<size_t>(4096, (cntk + 255) / 256);
  if constexpr (sizeof(T) == 4) {
    const int tj = (nov + MT - 1) / MT;
    {
      TraceScope ts(tr, TR_TDA_GEMM);
      dim3 gj(tj * (tj + 1) / 2, 1, w.nsplit);  // upper tiles only: CJ is symmetric
      if (ng % 4 == 0)
        k_gemm_nt_mfma<true, true><<<gj, 256, 0, s>>>(a_ov, nov, b_ov, nov, ng, w.kchunk, (float*)pj, 1);
      else
        k_gemm_nt_mfma<false, true><<<gj, 256, 0, s>>>(a_ov, nov, b_ov, nov, ng, w.kchunk, (float*)pj, 1);
      dim3 gk((noo + MT - 1) / MT, (nvv + MT - 1) / MT, w.nsplit);
      if (ng % 4 == 0)
        k_gemm_nt_mfma<true, false><<<gk, 256, 0, s>>>(a_oo, noo, b_vv, nvv, ng, w.kchunk, (float*)pk, 0);
      else
        k_gemm_nt_mfma<false, false><<<gk, 256, 0, s>>>(a_oo, noo, b_vv, nvv, ng, w.kchunk, (float*)pk, 0);
    }
    TraceScope ts(tr, TR_TDA_REDUCE);
    k_split_reduce_f32<<<rbj, 256, 0, s>>>((const float*)pj, w.nsplit, cntj, dv, cj, nov);
    k_split_reduce_f32<<<rbk, 256, 0, s>>>((const float*)pk, w.nsplit, cntk, dv, ck, 0);
    k_tda_assemble<<<rbj, 256, 0, s>>>(cj, ck, no, nv, delta_m, c_out, MT);
    if (b_out) k_tdhf_b_assemble<<<rbj, 256, 0, s>>>(cj, no, nv, delta_m, b_out, MT);
    return;
  } else {
    {
      TraceScope ts(tr, TR_TDA_GEMM);
      dim3 gj((nov + BM - 1) / BM, (nov + BN - 1) / BN, w.nsplit);
      k_gemm_nt<T><<<gj, kThreads, 0, s>>>(a_ov, nov, b_ov, nov, ng, w.kchunk, pj);
      dim3 gk((noo + BM - 1) / BM, (nvv + BN - 1) / BN, w.nsplit);
      k_gemm_nt<T><<<gk, kThreads, 0, s>>>(a_oo, noo, b_vv, nvv, ng, w.kchunk, pk);
    }
    TraceScope ts(tr, TR_TDA_REDUCE);
    k_split_reduce<<<rbj, 256, 0, s>>>(pj, w.nsplit, cntj, dv, cj);
    k_split_reduce<<<rbk, 256, 0, s>>>(pk, w.nsplit, cntk, dv, ck);
  }
  k_tda_assemble<<<rbj, 256, 0, s>>>(cj, ck, no, nv, delta_m, c_out, 0);
  if (b_out) k_tdhf_b_assemble<<<rbj, 256, 0, s>>>(cj, no, nv, delta_m, b_out, 0);
}

// D[c][i*nv + a] = dV sum_r phi_i(r) x_c(r) phi_a(r), x_c = (k_c - (n-1)/2) h: one block per
// (i, a), fixed-order tree reduction.
template <typename T>
__global__ __launch_bounds__(256) void k_dipoles(const T* __restrict__ occ, const T* __restrict__ virt,
                                                 int nv, int n, double h, double* __restrict__ D,
                                                 int nov) {
  __shared__ double red[3][256];
  const int i = blockIdx.x / nv, a = blockIdx.x % nv;
  const size_t ng = (size_t)n * n * n;
  const T* pi = occ + (size_t)i * ng;
  const T* pa = virt + (size_t)a * ng;
  const double c0 = 0.5 * (n - 1);
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (size_t r = threadIdx.x; r < ng; r += blockDim.x) {
    const double w = (double)pi[r] * (double)pa[r];
    const int z = (int)(r % n), y = (int)((r / n) % n), x = (int)(r / ((size_t)n * n));
    sx += w * (x - c0);
    sy += w * (y - c0);
    sz += w * (z - c0);
  }
  red[0][threadIdx.x] = sx;
  red[1][threadIdx.x] = sy;
  red[2][threadIdx.x] = sz;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 3) D[(size_t)threadIdx.x * nov + blockIdx.x] = red[threadIdx.x][0] * h * h * h * h;
}

// f_k = 2/3 omega_k |d_k|^2  (d: [k][3])
__global__ void k_oscillator(const double* __restrict__ omega, const double* __restrict__ d, int k,
                             double* __restrict__ f) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k) {
    const double dx = d[3 * j], dy = d[3 * j + 1], dz = d[3 * j + 2];
    f[j] = 2.0 / 3.0 * omega[j] * (dx * dx + dy * dy + dz * dz);
  }
}

// S(w) = sum_k f_k gamma / (pi ((w - omega_k)^2 + gamma^2)),  w = w0 + i dw
__global__ void k_strength(const double* __restrict__ omega, const double* __restrict__ f, int k,
                           double w0, double dw, int nw, double gamma, double* __restrict__ S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nw) return;
  const double w = w0 + i * dw;
  double s = 0.0;
  for (int j = 0; j < k; ++j) {
    const double x = w - omega[j];
    s += f[j] * gamma / (3.14159265358979323846 * (x * x + gamma * gamma));
  }
  S[i] = s;
}

}  // namespace

void launch_dipoles(bool fp64, const void* occ, int no, const void* virt, int nv, int n, double h,
                    double* D, hipStream_t s) {
  const int nov = no * nv;
  if (fp64)
    k_dipoles<double><<<nov, 256, 0, s>>>((const double*)occ, (const double*)virt, nv, n, h, D, nov);
  else
    k_dipoles<float><<<nov, 256, 0, s>>>((const float*)occ, (const float*)virt, nv, n, h, D, nov);
}

void launch_oscillator(const double* omega, const double* d, int k, double* f, hipStream_t s) {
  k_oscillator<<<(k + 63) / 64, 64, 0, s>>>(omega, d, k, f);
}

void launch_strength(const double* omega, const double* f, int k, double w0, double dw, int nw,
                     double gamma, double* S, hipStream_t s) {
  k_strength<<<(nw + 255) / 256, 256, 0, s>>>(omega, f, k, w0, dw, nw, gamma, S);
}

size_t tda_workspace_bytes(int no, int nv, size_t ng, bool fp64, TdaWork* w) {
  const size_t nov = (size_t)no * nv, noo = (size_t)no * (no + 1) / 2,
               nvv = (size_t)nv * (nv + 1) / 2;
  size_t nsplit, kchunk;
  if (fp64) {
    // enough blocks for the GPU: at least ~1024 for the larger contraction
    const size_t tiles = ((nov + BM - 1) / BM) * ((nov + BM - 1) / BM);
    nsplit = (1024 + tiles - 1) / tiles;
    kchunk = (ng + nsplit - 1) / nsplit;
    kchunk = ((kchunk + kSub - 1) / kSub) * kSub;
    if (kchunk < kSub) kchunk = kSub;
  } else {
    // matrix-core contractions: one wave of workgroups (two per CU, as their LDS allows) for
    // the larger launch, so no partly filled second wave; K chunks of whole 64-point tiles
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    const size_t tj = (nov + MT - 1) / MT;
    const size_t tiles = std::max(tj * (tj + 1) / 2, ((noo + MT - 1) / MT) * ((nvv + MT - 1) / MT));
    nsplit = std::max<size_t>(1, (size_t)(2 * cus) / tiles);
    kchunk = (ng + nsplit - 1) / nsplit;
    kchunk = ((kchunk + KB - 1) / KB) * KB;
  }
  nsplit = (ng + kchunk - 1) / kchunk;
  w->nsplit = (int)nsplit;
  w->kchunk = kchunk;
  w->off_pj = 0;
  w->off_pk = w->off_pj + nsplit * nov * nov * sizeof(double);
  w->off_cj = w->off_pk + nsplit * noo * nvv * sizeof(double);
  w->off_ck = w->off_cj + nov * nov * sizeof(double);
  return w->off_ck + noo * nvv * sizeof(double);
}

void launch_tda(bool fp64, const void* occ, int no, const void* virt, int nv, const void* v_ov,
                const void* v_oo, size_t ng, double dv, int delta_m, void* ws, const TdaWork& w,
                double* c_out, double* b_out, hipStream_t s, Trace* tr) {
  if (fp64)
    tda_impl<double>(occ, no, virt, nv, v_ov, v_oo, ng, dv, delta_m, ws, w, c_out, b_out, s, tr);
  else
    tda_impl<float>(occ, no, virt, nv, v_ov, v_oo, ng, dv, delta_m, ws, w, c_out, b_out, s, tr);
}

// ---- UHF blocks (Eqs. (4), (5)) over two spin channels --------------------------------------

namespace {

// split-K contraction out[m][n] = scale * sum_r A(m, r) B(n, r) over the full M x N grid
template <typename T>
void gemm_full(Op<T> A, int M, Op<T> B, int N, size_t ng, const UhfWork& w, void* part,
               double scale, double* out, hipStream_t s) {
  const size_t cnt = (size_t)M * N;
  const unsigned rb = (unsigned)std::min<size_t>(4096, (cnt + 255) / 256);
  if constexpr (sizeof(T) == 4) {
    dim3 g((M + MT - 1) / MT, (N + MT - 1) / MT, w.nsplit);
    const bool pref = B.q == nullptr;
    if (ng % 4 == 0) {
      if (pref)
        k_gemm_nt_mfma<true, true><<<g, 256, 0, s>>>(A, M, B, N, ng, w.kchunk, (float*)part, 0);
      else
        k_gemm_nt_mfma<true, false><<<g, 256, 0, s>>>(A, M, B, N, ng, w.kchunk, (float*)part, 0);
    } else {
      if (pref)
        k_gemm_nt_mfma<false, true><<<g, 256, 0, s>>>(A, M, B, N, ng, w.kchunk, (float*)part, 0);
      else
        k_gemm_nt_mfma<false, false><<<g, 256, 0, s>>>(A, M, B, N, ng, w.kchunk, (float*)part, 0);
    }
    k_split_reduce_f32<<<rb, 256, 0, s>>>((const float*)part, w.nsplit, cnt, scale, out, 0);
  } else {
    dim3 g((M + BM - 1) / BM, (N + BN - 1) / BN, w.nsplit);
    k_gemm_nt<T><<<g, kThreads, 0, s>>>(A, M, B, N, ng, w.kchunk, (double*)part);
    k_split_reduce<<<rb, 256, 0, s>>>((const double*)part, w.nsplit, cnt, scale, out);
  }
}

struct UhfDev {
  const double* g1[2][2];  // G1[s][t][ia][jb] = dV sum_r (phi_i phi_a)_s v^t_jb
  const double* g2[2];     // G2[s][pair(i,j)][a nv + b] = dV sum_r v^s_ij (phi_a phi_b)_s
  int no[2], nv[2], n0;    // n0 = alpha transitions
};

__device__ __forceinline__ double uhf_g1(const UhfDev& u, int s, int t, int x, int y) {
  const int nt = u.no[t] * u.nv[t];
  return 0.5 * (u.g1[s][t][(size_t)x * nt + y] + u.g1[t][s][(size_t)y * (u.no[s] * u.nv[s]) + x]);
}

// C = (ia||jb) - diag part, B = (ia||bj) (real orbitals: (ia|bj) = (ia|jb), (ib|aj) = (ib|ja))
__global__ void k_uhf_assemble(UhfDev u, int n, double* __restrict__ c, double* __restrict__ b) {
  for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < (size_t)n * n;
       idx += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(idx / n), col = (int)(idx % n);
    const int s = row < u.n0 ? 0 : 1, t = col < u.n0 ? 0 : 1;
    const int x = row - (s ? u.n0 : 0), y = col - (t ? u.n0 : 0);
    const double coul = uhf_g1(u, s, t, x, y);
    double cval = coul, bval = coul;
    if (s == t) {
      const int nv = u.nv[s];
      const int i = x / nv, a = x % nv, j = y / nv, bb = y % nv;
      const int lo = i < j ? i : j, hi = i < j ? j : i;
      const double* g2 = u.g2[s] + ((size_t)hi * (hi + 1) / 2 + lo) * (size_t)nv * nv;
      cval -= 0.5 * (g2[(size_t)a * nv + bb] + g2[(size_t)bb * nv + a]);
      bval -= uhf_g1(u, s, s, i * nv + bb, j * nv + a);
    }
    c[idx] = cval;
    if (b) b[idx] = bval;
  }
}

template <typename T>
void uhf_impl(const UhfSpin* sp, size_t ng, double dv, void* ws, const UhfWork& w, double* c_out,
              double* b_out, hipStream_t s, Trace* tr) {
  char* base = (char*)ws;
  void* part = base + w.off_part;
  double* g1[2][2];
  double* g2[2];
  for (int a = 0; a < 2; ++a) {
    for (int b = 0; b < 2; ++b) g1[a][b] = (double*)(base + w.off_g1[a][b]);
    g2[a] = (double*)(base + w.off_g2[a]);
  }
  {
    TraceScope ts(tr, TR_TDA_GEMM);
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        Op<T> rho{(const T*)sp[a].occ, (const T*)sp[a].virt, sp[a].nv, 0};
        Op<T> vt{(const T*)sp[b].v_ov, nullptr, 1, 0};
        gemm_full<T>(rho, sp[a].no * sp[a].nv, vt, sp[b].no * sp[b].nv, ng, w, part, dv, g1[a][b], s);
      }
    for (int a = 0; a < 2; ++a) {
      Op<T> voo{(const T*)sp[a].v_oo, nullptr, 1, 0};
      Op<T> rvv{(const T*)sp[a].virt, (const T*)sp[a].virt, sp[a].nv, 0};  // all nv^2 pairs
      gemm_full<T>(voo, sp[a].no * (sp[a].no + 1) / 2, rvv, sp[a].nv * sp[a].nv, ng, w, part, dv,
                   g2[a], s);
    }
  }
  UhfDev u;
  for (int a = 0; a < 2; ++a) {
    for (int b = 0; b < 2; ++b) u.g1[a][b] = g1[a][b];
    u.g2[a] = g2[a];
    u.no[a] = sp[a].no;
    u.nv[a] = sp[a].nv;
  }
  u.n0 = sp[0].no * sp[0].nv;
  const int n = u.n0 + sp[1].no * sp[1].nv;
  const unsigned rb = (unsigned)std::min<size_t>(4096, ((size_t)n * n + 255) / 256);
  k_uhf_assemble<<<rb, 256, 0, s>>>(u, n, c_out, b_out);
}

}  // namespace

size_t uhf_workspace_bytes(const UhfSpin* sp, size_t ng, bool fp64, UhfWork* w) {
  const size_t tile = fp64 ? BM : MT;
  size_t maxcnt = 0, maxtiles = 0;
  auto consider = [&](size_t m, size_t n) {
    maxcnt = std::max(maxcnt, m * n);
    maxtiles = std::max(maxtiles, ((m + tile - 1) / tile) * ((n + tile - 1) / tile));
  };
  for (int a = 0; a < 2; ++a) {
    for (int b = 0; b < 2; ++b) consider((size_t)sp[a].no * sp[a].nv, (size_t)sp[b].no * sp[b].nv);
    consider((size_t)sp[a].no * (sp[a].no + 1) / 2, (size_t)sp[a].nv * sp[a].nv);
  }
  size_t nsplit = (1024 + maxtiles - 1) / maxtiles;
  size_t kchunk = (ng + nsplit - 1) / nsplit;
  kchunk = ((kchunk + kSub - 1) / kSub) * kSub;
  if (kchunk < kSub) kchunk = kSub;
  nsplit = (ng + kchunk - 1) / kchunk;
  w->nsplit = (int)nsplit;
  w->kchunk = kchunk;
  size_t off = 0;
  w->off_part = off;
  off += nsplit * maxcnt * sizeof(double);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      w->off_g1[a][b] = off;
      off += (size_t)sp[a].no * sp[a].nv * sp[b].no * sp[b].nv * sizeof(double);
    }
  for (int a = 0; a < 2; ++a) {
    w->off_g2[a] = off;
    off += (size_t)sp[a].no * (sp[a].no + 1) / 2 * sp[a].nv * sp[a].nv * sizeof(double);
  }
  return off;
}

void launch_uhf(bool fp64, const UhfSpin* sp, size_t ng, double dv, void* ws, const UhfWork& w,
                double* c_out, double* b_out, hipStream_t s, Trace* tr) {
  if (fp64)
    uhf_impl<double>(sp, ng, dv, ws, w, c_out, b_out, s, tr);
  else
    uhf_impl<float>(sp, ng, dv, ws, w, c_out, b_out, s, tr);
}

}  // namespace ace
