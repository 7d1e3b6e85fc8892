// ACE construction and application around the pair-Poisson engine (paper Sec. 3.1,
// Eqs. (11)-(13)):
//   W_i   = -sum_j phi_j v_ji                      (Eq. (11) with Eq. (2))
//   M     = Phi^H W dV                             (Gram kernel, FP64 cross-tile sums)
//   -M    = L L^H, E_x = 1/2 tr M                  (one workgroup, FP64)
//   xi    = W L^{-H}                               (Eq. (12), per-point triangular product)
//   K psi = -xi (xi^H psi dV)                      (Eq. (13), Gram kernel + per-point update)
// Conjugation follows the complex reading of the real-orbital equations: pair densities are
// conj(phi_j) phi_i, so v_ij = conj(v_ji) and only pairs j <= i are solved.
#include <type_traits>

#include "ace_kernels.hpp"
#include "elem.hpp"

namespace ace {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ size_t pair_index(int a, int b) {  // a <= b
  return (size_t)b * (b + 1) / 2 + a;
}

// Argument sources: one system passed by value, or many systems read from device memory
// (index = the grid coordinate that enumerates systems).
// Arguments of one workgroup: the system's arguments, the workgroup's 256-point block within
// that system, and the system's point count.
template <typename A>
struct Placed {
  A a;
  size_t blk;
  size_t ng;
};
struct OneMol {
  MolArgs m;
  __device__ __forceinline__ MolArgs get(int) const { return m; }
  __device__ __forceinline__ Placed<MolArgs> place(size_t ng) const { return {m, blockIdx.x, ng}; }
};
struct ManyMol {  // systems of one box edge: grid (blocks, systems)
  const MolArgs* ms;
  __device__ __forceinline__ MolArgs get(int i) const { return ms[i]; }
  __device__ __forceinline__ Placed<MolArgs> place(size_t ng) const {
    return {ms[blockIdx.y], blockIdx.x, ng};
  }
};
// systems of any box edges in one flat grid: bsys[blockIdx.x] is the block's system
struct FlatMol {
  const MolArgs* ms;
  const int* bsys;
  __device__ __forceinline__ MolArgs get(int i) const { return ms[i]; }
  __device__ __forceinline__ Placed<MolArgs> place(size_t) const {
    const MolArgs m = ms[bsys[blockIdx.x]];
    return {m, blockIdx.x - (size_t)m.blk0, m.ng};
  }
};
struct GramArgs {
  const void* A;
  int na;
  const void* B;
  int nb;
  void* part;
};
__device__ __forceinline__ GramArgs gram_of(const MolArgs& m) {
  return {m.phi, m.n, m.w, m.n, m.part};
}
struct OneGram {
  GramArgs g;
  __device__ __forceinline__ Placed<GramArgs> place(size_t ng) const {
    return {g, blockIdx.x, ng};
  }
};
struct ManyGram {  // grid (blocks, tiles, systems)
  const MolArgs* ms;
  __device__ __forceinline__ Placed<GramArgs> place(size_t ng) const {
    return {gram_of(ms[blockIdx.z]), blockIdx.x, ng};
  }
};
struct FlatGram {  // grid (blocks of all systems, tiles)
  const MolArgs* ms;
  const int* bsys;
  __device__ __forceinline__ Placed<GramArgs> place(size_t) const {
    const MolArgs m = ms[bsys[blockIdx.x]];
    return {gram_of(m), blockIdx.x - (size_t)m.blk0, m.ng};
  }
};
// a reduction: partial rows, outputs per row, destination, partial rows to add, scale
struct RedArgs {
  const void* part;
  int no;
  void* out;
  int nblk;
  double scale;
};
struct OneRed {
  RedArgs r;
  __device__ __forceinline__ RedArgs get(int) const { return r; }
};
struct ManyRed {
  const MolArgs* ms;
  __device__ __forceinline__ RedArgs get(int i) const {
    const MolArgs m = ms[i];
    return {m.part, m.n * m.n, m.mred, (int)((m.ng + kThreads - 1) / kThreads), m.dv};
  }
};

// W_i(r) = -sum_j phi_j(r) v_ji(r); v holds pair (a<=b) volumes G (*) conj(phi_a) phi_b.
// One thread per point holds every phi_j(r) and W_i(r) in registers, so each pair volume is
// read once: v_ab feeds W_b (with phi_a) and, for a != b, W_a (with phi_b and conj(v_ab)).
// W is accumulated in FP64 for every storage type: a product of two FP32 values is exact in
// FP64, so FP32 storage gets the exact sum rounded once (in place of a compensated FP32 sum);
// the pass stays bound by its HBM traffic.
template <typename E, int NMAX, typename S>
__global__ __launch_bounds__(kThreads) void k_wacc(S src, size_t ng_arg) {
  const Placed<MolArgs> pc = src.place(ng_arg);
  const MolArgs m = pc.a;
  const size_t ng = pc.ng;
  const E* __restrict__ phi = (const E*)m.phi;
  const E* __restrict__ v = (const E*)m.v;
  E* __restrict__ w = (E*)m.w;
  const int n = m.n;
  const size_t r = pc.blk * kThreads + threadIdx.x;
  if (r >= ng) return;
  typedef typename Elem<E>::wide A;
  E ph[NMAX];
  A acc[NMAX];
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    acc[j] = e_zero<A>();
    ph[j] = phi[(size_t)(j < n ? j : n - 1) * ng + r];  // unconditional: loads issue together
  }
#pragma unroll
  for (int b = 0; b < NMAX; ++b) {
    if (b < n) {
#pragma unroll
      for (int a = 0; a <= b; ++a) {
        const A vab = e_wide(v[pair_index(a, b) * ng + r]);
        acc[b] = e_add(acc[b], e_mul(e_wide(ph[a]), vab));
        if (a != b) acc[a] = e_add(acc[a], e_mul(e_wide(ph[b]), e_conj(vab)));
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
    if (i < n) w[(size_t)i * ng + r] = e_narrow<E>(e_neg(acc[i]));
}

// Partial Gram sums G_kl = sum_r conj(A_k(r)) B_l(r) on the matrix cores.  A workgroup of 4
// wavefronts owns 4 consecutive chunks of kGramChunk points and one 16 x 16 output tile
// (k-tile, l-tile).  Each wavefront loads its whole chunk first (lane (i, g) = (lane % 16,
// lane / 16) reads A_{k0+i} and B_{l0+i} at points r0 + 4g + s of every 16-point group), then
// issues v_mfma_f64_16x16x4f64 with the points as the contraction index.  Operands are
// converted to FP64 in registers: products of FP32 inputs are exact in FP64 and the sums
// carry FP64 rounding only, whatever the storage precision.  Complex products take three
// real contractions (Gauss's three-multiplication form of conj(a) b).  The four wavefront tiles
// are summed in LDS in a fixed order; one FP64 partial per workgroup: part[block][o].
// Lane layout of v_mfma_f64_16x16x4f64 (checked on gfx950): A[i][k] in lane i + 16k,
// B[k][j] in lane j + 16k, D[i][j] in lane j + 16 (i % 4), element i / 4.
#ifndef ACE_GRAM_CHUNK
#define ACE_GRAM_CHUNK 64
#endif
constexpr int kGramChunk = ACE_GRAM_CHUNK;      // points per wavefront (multiple of 16)
constexpr int kGramWaves = kThreads / 64;       // wavefronts per workgroup
constexpr int kGramPoints = kGramChunk * kGramWaves;

typedef double gf64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ gf64x4 mma64(double a, double b, gf64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void split_ri(float v, double& r, double& i) { r = v; i = 0.0; }
__device__ __forceinline__ void split_ri(double v, double& r, double& i) { r = v; i = 0.0; }
template <typename T>
__device__ __forceinline__ void split_ri(C2<T> v, double& r, double& i) { r = v.r; i = v.i; }
__device__ __forceinline__ void set_ri(double& x, double r, double) { x = r; }
__device__ __forceinline__ void set_ri(C2<double>& x, double r, double i) { x.r = r; x.i = i; }

// Four consecutive elements r0 .. r0+3 of a row (r0 a multiple of 4).  VEC: the row length
// is a multiple of 4, so the group is 16-byte aligned and wholly inside or outside the row;
// it is loaded with vector instructions (a group past the end reads the last group).
template <typename E, bool VEC>
__device__ __forceinline__ void load4(const E* __restrict__ row, size_t r0, size_t ng, E* out) {
  if constexpr (VEC && sizeof(E) <= 8) {
    const size_t g0 = r0 < ng ? r0 : ng - 4;
    const float4* p = reinterpret_cast<const float4*>(row + g0);
    if constexpr (sizeof(E) == 4) {
      const float4 v = p[0];
      const float t[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int s = 0; s < 4; ++s) out[s] = *reinterpret_cast<const E*>(&t[s]);
    } else {
      const float4 v0 = p[0], v1 = p[1];
      const float t[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
      for (int s = 0; s < 4; ++s) out[s] = *reinterpret_cast<const E*>(&t[2 * s]);
    }
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const size_t r = r0 + s;
      out[s] = row[r < ng ? r : ng - 1];
    }
  }
}

// skip8: complex systems with at most 8 A rows are left to k_gram_c8 (launched beside it)
template <typename E, typename S, int TB, bool VEC>
__global__ __launch_bounds__(kThreads) void k_gram(S src, size_t ng_arg, int skip8) {
  typedef typename Elem<E>::wide W;
  constexpr bool CPLX = Elem<E>::cplx;
  const Placed<GramArgs> pc = src.place(ng_arg);
  const GramArgs ga = pc.a;
  const size_t ng = pc.ng;
  const E* __restrict__ A = (const E*)ga.A;
  const E* __restrict__ B = (const E*)ga.B;
  const int na = ga.na, nb = ga.nb;
  W* __restrict__ part = (W*)ga.part;
  const int tiles_l = (nb + 15) / 16, groups_l = (tiles_l + TB - 1) / TB;
  if ((int)blockIdx.y >= ((na + 15) / 16) * groups_l) return;  // tile beyond this system
  if (CPLX && skip8 && na <= 8) return;
  constexpr int NQ = kGramChunk / 16;
  __shared__ W red[kGramWaves][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k0 = (blockIdx.y / groups_l) * 16, lg0 = (blockIdx.y % groups_l) * 16 * TB;
  const int li = lane & 15, g = lane >> 4;
  const int ka = k0 + li;
  // loads are unconditional (clamped row and point) so they issue back to back; values
  // outside the matrices are zeroed afterwards
  const E* ra = A + (size_t)(ka < na ? ka : na - 1) * ng;
  const size_t start = pc.blk * kGramPoints + (size_t)wave * kGramChunk;
  E av[NQ][4];
#pragma unroll
  for (int q = 0; q < NQ; ++q) load4<E, VEC>(ra, start + 16 * q + 4 * g, ng, av[q]);
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const size_t r = start + 16 * q + 4 * g + s;
      if (!(ka < na && r < ng)) av[q][s] = e_zero<E>();
    }
  // the A tile is reused for TB consecutive B tiles (each A element is read once per block)
#pragma unroll
  for (int t = 0; t < TB; ++t) {
    const int l0 = lg0 + 16 * t;
    if (l0 >= nb) break;  // uniform
    const int lb = l0 + li;
    const E* rb = B + (size_t)(lb < nb ? lb : nb - 1) * ng;
    E bv[NQ][4];
#pragma unroll
    for (int q = 0; q < NQ; ++q) load4<E, VEC>(rb, start + 16 * q + 4 * g, ng, bv[q]);
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const size_t r = start + 16 * q + 4 * g + s;
        if (!(lb < nb && r < ng)) bv[q][s] = e_zero<E>();
      }
    // conj(a) b with c = ar, d = -ai, e = br, f = bi: three real contractions (Gauss)
    //   t1 = e (c + d), t2 = c (f - e), t3 = d (e + f);  re = t1 - t3, im = t1 + t2
    gf64x4 t1 = {}, t2 = {}, t3 = {};
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        double ar, ai, br, bi;
        split_ri(av[q][s], ar, ai);
        split_ri(bv[q][s], br, bi);
        if constexpr (CPLX) {
          t1 = mma64(ar - ai, br, t1);
          t2 = mma64(ar, bi - br, t2);
          t3 = mma64(-ai, br + bi, t3);
        } else {
          t1 = mma64(ar, br, t1);
        }
      }
    if (t > 0) __syncthreads();  // the previous tile's sums have been read
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int tt = (g + 4 * e) * 16 + li;  // tile element (row g + 4e, column li)
      W v;
      if constexpr (CPLX) {
        v.r = t1[e] - t3[e];
        v.i = t1[e] + t2[e];
      } else {
        v = t1[e];
      }
      red[wave][tt] = v;
    }
    __syncthreads();
    const int th = threadIdx.x;  // 256 threads, 256 tile elements
    const int k = k0 + th / 16, l = l0 + th % 16;
    if (k < na && l < nb) {
      W v = red[0][th];
#pragma unroll
      for (int w = 1; w < kGramWaves; ++w) v = e_add(v, red[w][th]);
      part[pc.blk * na * nb + (size_t)k * nb + l] = v;
    }
  }
}

// Complex Gram with at most 8 A rows: the real and imaginary parts of the A rows are stacked
// as the 16 rows of one FP64 MFMA operand, and those of 8 B columns as its 16 columns, so one
// 16x16x4 product per 4 points gives all four real products of the 8 x 8 complex tile
//   D = [Re A; Im A] [Re B, Im B],  Re(A^H B) = D_rr + D_ii,  Im(A^H B) = D_ri - D_ir
// with no padded rows and no third (Gauss) product.  TB tiles of 8 B columns share the A rows.
// (body: partial row blk, tile group grp of the B columns)
template <typename E, int TB, bool VEC, int WAVES>
__device__ __forceinline__ void gram_c8_body(const GramArgs& ga, size_t blk, int grp, size_t ng) {
  typedef typename Elem<E>::wide W;
  static_assert(Elem<E>::cplx, "complex elements");
  const E* __restrict__ A = (const E*)ga.A;
  const E* __restrict__ B = (const E*)ga.B;
  const int na = ga.na, nb = ga.nb;
  W* __restrict__ part = (W*)ga.part;
  const int tiles_l = (nb + 7) / 8;
  if (grp * TB >= tiles_l || na > 8) return;  // beyond this system, or k_gram's
  constexpr int CHUNK = kGramPoints / WAVES;  // points per wavefront
  constexpr int NQ = CHUNK / 16;
  static_assert(NQ >= 2 && NQ % 2 == 0 && CHUNK % 16 == 0, "even number of 16-point steps");
  constexpr int NH = NQ / 2;
  __shared__ double red[WAVES][TB * 256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int ri = li & 7;
  const bool imag = li >= 8;
  const size_t start = blk * kGramPoints + (size_t)wave * CHUNK;
  // Lanes li and li + 8 work on the same row (real and imaginary part).  Each loads half of the
  // wavefront's steps (li < 8 the first NH, li >= 8 the last NH) and gets the other half's
  // component from its partner lane (li ^ 8), so every element is loaded once.
  const int q0 = imag ? NH : 0;
  auto operands = [&](const E (*v)[4], int row, int nrow, double (*op)[4]) {
#pragma unroll
    for (int j = 0; j < NH; ++j)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const size_t r = start + 16 * (q0 + j) + 4 * g + s;
        typedef typename Elem<E>::real Rl;
        const bool ok = row < nrow && r < ng;
        const Rl xr = ok ? v[j][s].r : Rl(0), xi = ok ? v[j][s].i : Rl(0);
        // first half: li < 8 own real part, li >= 8 the partner's imaginary part
        const Rl gi = __shfl_xor(xi, 8, 64);
        // second half: li >= 8 own imaginary part, li < 8 the partner's real part
        const Rl gr = __shfl_xor(xr, 8, 64);
        op[j][s] = imag ? (double)gi : (double)xr;
        op[NH + j][s] = imag ? (double)xi : (double)gr;
      }
  };
  const E* ra = A + (size_t)(ri < na ? ri : na - 1) * ng;
  E av[NH][4];
#pragma unroll
  for (int j = 0; j < NH; ++j) load4<E, VEC>(ra, start + 16 * (q0 + j) + 4 * g, ng, av[j]);
  double ao[NQ][4];
  operands(av, ri, na, ao);
  // every B tile's loads are issued before the first product
  E bv[TB][NH][4];
#pragma unroll
  for (int t = 0; t < TB; ++t) {
    const int l0 = (grp * TB + t) * 8, lb = l0 + ri;
    if (l0 >= nb) break;  // uniform
    const E* rb = B + (size_t)(lb < nb ? lb : nb - 1) * ng;
#pragma unroll
    for (int j = 0; j < NH; ++j) load4<E, VEC>(rb, start + 16 * (q0 + j) + 4 * g, ng, bv[t][j]);
  }
#pragma unroll
  for (int t = 0; t < TB; ++t) {
    const int l0 = (grp * TB + t) * 8, lb = l0 + ri;
    if (l0 >= nb) break;  // uniform; these outputs are not written
    double bo[NQ][4];
    operands(bv[t], lb, nb, bo);
    gf64x4 d = {};
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int s = 0; s < 4; ++s) d = mma64(ao[q][s], bo[q][s], d);
#pragma unroll
    for (int e = 0; e < 4; ++e) red[wave][t * 256 + (g + 4 * e) * 16 + li] = d[e];
  }
  __syncthreads();
  // TB * 64 complex outputs
  for (int th = threadIdx.x; th < TB * 64; th += 64 * WAVES) {
    const int t = th >> 6, k = (th >> 3) & 7, l = th & 7;
    const int l0 = (grp * TB + t) * 8;
    const double* rt = &red[0][t * 256];
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
      re += rt[w * TB * 256 + k * 16 + l] + rt[w * TB * 256 + (k + 8) * 16 + l + 8];
      im += rt[w * TB * 256 + k * 16 + l + 8] - rt[w * TB * 256 + (k + 8) * 16 + l];
    }
    if (k < na && l0 + l < nb) {
      W v;
      v.r = re;
      v.i = im;
      part[blk * na * nb + (size_t)k * nb + l0 + l] = v;
    }
  }
}

template <typename E, typename S, int TB, bool VEC, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_gram_c8(S src, size_t ng_arg) {
  const Placed<GramArgs> pc = src.place(ng_arg);
  gram_c8_body<E, TB, VEC, WAVES>(pc.a, pc.blk, (int)blockIdx.y, pc.ng);
}

template <typename W>
__device__ __forceinline__ W shfl_w(W v, int src);
template <>
__device__ __forceinline__ double shfl_w<double>(double v, int src) { return __shfl(v, src, 64); }
template <>
__device__ __forceinline__ C2<double> shfl_w<C2<double>>(C2<double> v, int src) {
  return {__shfl(v.r, src, 64), __shfl(v.i, src, 64)};
}
__device__ __forceinline__ double w_from_real(double r, double) { return r; }
__device__ __forceinline__ C2<double> w_from_real(double r, C2<double>) { return {r, 0.0}; }

// Cholesky of -M (Hermitised), L^{-H} and E_x for n <= 8 in one wavefront, FP64, with one lane
// per matrix entry (lane 8i + k holds entry (i, k)): every
// elimination step is one pivot broadcast and one rank-1 update across the whole wavefront,
// and L^{-1} is formed the same way, one column step at a time, so the dependent chain is
// O(n) broadcasts instead of O(n^2) serial multiply-adds per lane.
// lds_linvh (optional): L^{-H} also into LDS (same layout); globals: write M, E_x, L^{-H} and
// the status to memory (false in all but one of the workgroups that factorise redundantly).
template <typename W>
__device__ __forceinline__ void chol_lanes_body(const MolArgs& ma, const W* msrc,
                                                W* lds_linvh = nullptr, bool globals = true) {
  const int n = ma.n;
  W* __restrict__ m_out = globals ? (W*)ma.m_out : nullptr;
  double* __restrict__ ex_out = globals ? ma.ex_out : nullptr;
  W* __restrict__ linvh = (W*)ma.linvh;
  int* __restrict__ status = globals ? ma.status : nullptr;
  const int lane = threadIdx.x & 63, i = lane >> 3, k = lane & 7;
  const bool in = i < n && k < n;
  W a = W{};
  bool bad = false;
  double diag = 0.0;
  if (in) {
    const W mik = msrc[i * n + k], mki = msrc[k * n + i];
    bad = !e_finite(mik);
    const W herm = e_scale(e_add(mik, e_conj(mki)), 0.5);
    if (m_out) m_out[i * n + k] = herm;
    if (i == k) diag = e_re(herm);
    a = e_neg(herm);
  }
  // E_x: diagonal i moved to lane i first, so the sum rounds as in k_chol
  const double dl = __shfl(diag, lane < 8 ? 9 * lane : 0, 64);
  double e = lane < n ? dl : 0.0;
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if (lane == 0 && ex_out) *ex_out = 0.5 * e;
  const bool any_bad = __any(bad);
  int fail = -1;
  double dinv = 1.0;  // 1 / L_ii of this lane's row
  for (int j = 0; j < n; ++j) {
    const double piv = __shfl(e_re(a), 9 * j, 64);
    if (!(piv > 0.0) && fail < 0) fail = j;
    const double d = piv > 0.0 ? sqrt(piv) : 1.0;
    const double invd = 1.0 / d;
    if (i == j) dinv = invd;
    if (k == j) a = (i > j) ? e_scale(a, invd) : (i == j ? w_from_real(d, W{}) : W{});
    const W li = shfl_w(a, 8 * i + j), lk = shfl_w(a, 8 * k + j);
    if (i > j && k > j) a = e_sub(a, e_mul(li, e_conj(lk)));
  }
  const W l = (in && k <= i) ? a : W{};
  // X = L^{-1}, right-looking: step m finishes row m of X and removes it from the rows below
  W x = (in && i == k) ? w_from_real(1.0, W{}) : W{};
  for (int m = 0; m < n; ++m) {
    if (i == m) x = e_scale(x, dinv);
    const W xm = shfl_w(x, 8 * m + k), lim = shfl_w(l, 8 * i + m);
    if (i > m) x = e_sub(x, e_mul(lim, xm));
  }
  const bool ok = fail < 0 && !any_bad;
  // L^{-H}[c][r] = conj(X[r][c]); this lane holds X[i][k]
  if (in) {
    const W v = ok ? e_conj(x) : W{};
    if (globals) linvh[k * n + i] = v;
    if (lds_linvh) lds_linvh[k * n + i] = v;
  }
  if (lane == 0 && !ok && status && status[0] == 0) {
    status[0] = any_bad ? -6 : -5;
    status[1] = any_bad ? -1 : fail;
  }
}

// W accumulation fused with the block's partial of M = Phi^H W dV (used when the orbitals and
// W of one workgroup's points fit in LDS): after forming W_i(r) for its 256 points (as k_wacc),
// the workgroup transposes phi and W through LDS and contracts them on the FP64 matrix cores
// (each wavefront 64 points, the four summed in a fixed order), writing the same partial
// layout part[block][o] as k_gram, so M is reduced by k_gram_reduce and W is not read again.
template <typename E, int NMAX, typename S>
__global__ __launch_bounds__(kThreads) void k_wacc_gram(S src, size_t ng_arg) {
  static_assert(NMAX <= 16, "one 16 x 16 tile");
  typedef typename Elem<E>::wide W;
  constexpr bool CPLX = Elem<E>::cplx;
  constexpr int LD = kThreads + 1;
  // phi and W of the workgroup's points; the cross-wavefront sums reuse the same LDS once the
  // products are done (halves the footprint: two workgroups per CU at 16 orbitals)
  constexpr size_t kStage = 2 * (size_t)NMAX * LD * sizeof(E);
  constexpr size_t kRed = (size_t)kGramWaves * 256 * sizeof(W);
  __shared__ __align__(16) unsigned char smem[kStage > kRed ? kStage : kRed];
  E* lp = reinterpret_cast<E*>(smem);
  E* lw = lp + NMAX * LD;
  W(*red)[256] = reinterpret_cast<W(*)[256]>(smem);
  const Placed<MolArgs> pc = src.place(ng_arg);
  const MolArgs m = pc.a;
  const size_t ng = pc.ng;
  const E* __restrict__ phi = (const E*)m.phi;
  const E* __restrict__ v = (const E*)m.v;
  E* __restrict__ w = (E*)m.w;
  W* __restrict__ part = (W*)m.part;
  const int n = m.n;
  const size_t r0 = pc.blk * kThreads;
  const size_t r = r0 + threadIdx.x;
  const bool in = r < ng;
  const size_t rc = in ? r : ng - 1;
  typedef typename Elem<E>::wide A;
  E ph[NMAX];
  A acc[NMAX];
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    acc[j] = e_zero<A>();
    ph[j] = phi[(size_t)(j < n ? j : n - 1) * ng + rc];
  }
#pragma unroll
  for (int b = 0; b < NMAX; ++b) {
    if (b < n) {
#pragma unroll
      for (int a = 0; a <= b; ++a) {
        const A vab = e_wide(v[pair_index(a, b) * ng + rc]);
        acc[b] = e_add(acc[b], e_mul(e_wide(ph[a]), vab));
        if (a != b) acc[a] = e_add(acc[a], e_mul(e_wide(ph[b]), e_conj(vab)));
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NMAX; ++i) {
    const bool use = i < n && in;
    const E wi = e_narrow<E>(e_neg(acc[i]));
    if (use) w[(size_t)i * ng + r] = wi;
    lp[i * LD + threadIdx.x] = use ? ph[i] : e_zero<E>();
    lw[i * LD + threadIdx.x] = use ? wi : e_zero<E>();
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  // products in the same order as k_gram / k_gram_c8 over the same 256 points (wavefront w:
  // points 64w + 16q + 4g + s at step (q, s)), so fused and separate builds agree bit for bit
  if (CPLX && n <= 8) {
    // real and imaginary parts stacked into one 16 x 16 product (as k_gram_c8)
    const int ri = li & 7;
    const bool imag = li >= 8;
    gf64x4 d = {};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int pt = wave * 64 + 16 * q + 4 * g + s;
        double ar, ai, br, bi;
        split_ri(lp[(ri < NMAX ? ri : 0) * LD + pt], ar, ai);
        split_ri(lw[(ri < NMAX ? ri : 0) * LD + pt], br, bi);
        d = mma64(imag ? ai : ar, imag ? bi : br, d);
      }
    double* rd = reinterpret_cast<double*>(smem);
    __syncthreads();  // every wavefront is done with lp / lw
#pragma unroll
    for (int e = 0; e < 4; ++e) rd[wave * 256 + (g + 4 * e) * 16 + li] = d[e];
    __syncthreads();
    const int th = threadIdx.x;
    if (th < 64) {
      const int k = th >> 3, l = th & 7;
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int w = 0; w < kGramWaves; ++w) {
        re += rd[w * 256 + k * 16 + l] + rd[w * 256 + (k + 8) * 16 + l + 8];
        im += rd[w * 256 + k * 16 + l + 8] - rd[w * 256 + (k + 8) * 16 + l];
      }
      if (k < n && l < n) {
        W x = {};
        set_ri(x, re, im);
        part[pc.blk * n * n + (size_t)k * n + l] = x;
      }
    }
  } else {
    gf64x4 t1 = {}, t2 = {}, t3 = {};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int pt = wave * 64 + 16 * q + 4 * g + s;
        double ar = 0, ai = 0, br = 0, bi = 0;
        if (NMAX == 16 || li < NMAX) {
          split_ri(lp[li * LD + pt], ar, ai);
          split_ri(lw[li * LD + pt], br, bi);
        }
        if constexpr (CPLX) {
          t1 = mma64(ar - ai, br, t1);
          t2 = mma64(ar, bi - br, t2);
          t3 = mma64(-ai, br + bi, t3);
        } else {
          t1 = mma64(ar, br, t1);
        }
      }
    __syncthreads();  // every wavefront is done with lp / lw
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int tt = (g + 4 * e) * 16 + li;
      W x;
      if constexpr (CPLX) {
        x.r = t1[e] - t3[e];
        x.i = t1[e] + t2[e];
      } else {
        x = t1[e];
      }
      red[wave][tt] = x;
    }
    __syncthreads();
    const int th = threadIdx.x;
    const int k = th / 16, l = th % 16;
    if (k < n && l < n) {
      W x = red[0][th];
#pragma unroll
      for (int q = 1; q < kGramWaves; ++q) x = e_add(x, red[q][th]);
      part[pc.blk * n * n + (size_t)k * n + l] = x;
    }
  }
}

// Wide real Gram (both sides wider than one 16-row tile, at most 64 rows each): a workgroup
// stages its chunk of kGramPoints points of every A and B row in LDS once, in passes of a
// few dozen points (rows padded by one element against bank conflicts) and its four wavefronts compute all 16 x 16 output tiles
// from there, so each input element is read from HBM once instead of once per tile.  Same
// FP64 MFMA contraction and the same partial layout part[block][o] as k_gram.
constexpr int kWideRows = 64;

// 16-row tile pair (row tile, column tile) of tile index `tile`: all ta x tb pairs, or for a
// symmetric Gram (A = B) the pairs with row <= column only
__device__ __forceinline__ void wide_tile_rc(int tile, int tb, bool sym, int* tr, int* tc) {
  if (!sym) {
    *tr = tile / tb;
    *tc = tile % tb;
    return;
  }
  for (int r = 0; r < tb; ++r) {  // row r holds tiles (r, r .. tb - 1)
    if (tile < tb - r) {
      *tr = r;
      *tc = r + tile;
      return;
    }
    tile -= tb - r;
  }
  *tr = *tc = tb - 1;  // not reached for tile < tb (tb + 1) / 2
}

// NT tiles of one wavefront over one staged pass (unconditional, fully unrolled chains)
template <typename E, int NT, int SC>
__device__ __forceinline__ void wide_tiles(const E* la, const E* lb, int wave, int tb, bool sym,
                                           int ntile, int li, int g, gf64x4* acc) {
  constexpr int LD = SC + 1;
  const E* pa[NT];
  const E* pb[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    int tr, tc;  // a wavefront without a tile of its own works on a valid one, writing nothing
    wide_tile_rc(min(wave + 4 * u, ntile - 1), tb, sym, &tr, &tc);
    pa[u] = la + (tr * 16 + li) * LD + g;
    pb[u] = lb + (tc * 16 + li) * LD + g;
  }
  gf64x4 t[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) t[u] = acc[u];
#pragma unroll 4
  for (int q = 0; q < SC / 4; ++q)
#pragma unroll
    for (int u = 0; u < NT; ++u) t[u] = mma64((double)pa[u][4 * q], (double)pb[u][4 * q], t[u]);
#pragma unroll
  for (int u = 0; u < NT; ++u) acc[u] = t[u];
}

template <typename E, int NT>
__device__ __forceinline__ void k_gram_wide_body(const E* __restrict__ A, int na,
                                                 const E* __restrict__ B, int nb, size_t ng,
                                                 double* __restrict__ part, E* la, E* lb,
                                                 bool sym, int ntile) {
  // points per pass: small enough (about 33 KiB of LDS) for several workgroups per CU
  constexpr int SC = sizeof(E) == 4 ? kGramPoints / 4 : kGramPoints / 8;
  constexpr int LD = SC + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int ta = (na + 15) / 16, tb = (nb + 15) / 16;
  const int ra = ta * 16, rb = tb * 16;
  gf64x4 acc[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) acc[u] = gf64x4{0.0, 0.0, 0.0, 0.0};
  for (int pass = 0; pass < kGramPoints / SC; ++pass) {
    const size_t p0 = (size_t)blockIdx.x * kGramPoints + (size_t)pass * SC;
    // staging: eight unconditional (clamped) loads in flight per thread, then the stores
    constexpr int U = 8;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (side == 1 && sym) break;  // B = A: the staged A rows serve both sides (uniform)
      const E* X = side ? B : A;
      E* lx = side ? lb : la;
      const int nx = side ? nb : na, rx = side ? rb : ra;
      for (int base = 0; base < rx * SC; base += U * kThreads) {
        E v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = base + u * kThreads + threadIdx.x;
          const int row = e / SC, c = e % SC;
          const bool ok = row < nx && p0 + c < ng && e < rx * SC;
          v[u] = X[ok ? (size_t)row * ng + p0 + c : 0];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int e = base + u * kThreads + threadIdx.x;
          const int row = e / SC, c = e % SC;
          const bool ok = row < nx && p0 + c < ng;
          if (e < rx * SC) lx[row * LD + c] = ok ? v[u] : E(0);
        }
      }
    }
    __syncthreads();
    wide_tiles<E, NT, SC>(la, sym ? la : lb, wave, tb, sym, ntile, li, g, acc);
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    if (wave + 4 * u >= ntile) break;  // uniform: no tile of this wavefront
    int tr, tc;
    wide_tile_rc(wave + 4 * u, tb, sym, &tr, &tc);
    const int k0 = tr * 16, l0 = tc * 16;
    double* pw = part + (size_t)blockIdx.x * na * nb;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + g + 4 * e, l = l0 + li;
      if (k < na && l < nb) {
        pw[(size_t)k * nb + l] = acc[u][e];
        if (sym && tr != tc) pw[(size_t)l * nb + k] = acc[u][e];  // the mirrored tile
      }
    }
  }
}

template <typename E>
__global__ __launch_bounds__(kThreads) void k_gram_wide(const E* __restrict__ A, int na,
                                                        const E* __restrict__ B, int nb,
                                                        size_t ng, double* __restrict__ part) {
  constexpr int SC = sizeof(E) == 4 ? kGramPoints / 4 : kGramPoints / 8;
  __shared__ E la[kWideRows * (SC + 1)];
  __shared__ E lb[kWideRows * (SC + 1)];
  const int wave = threadIdx.x >> 6;
  // a Gram of a block with itself is symmetric: its upper tiles are computed and mirrored
  const bool sym = A == B && na == nb;
  const int ta = (na + 15) / 16, tb = (nb + 15) / 16;
  const int ntile = sym ? ta * (ta + 1) / 2 : ta * tb;
  const int nt = (ntile - wave + 3) / 4;  // tiles of this wavefront (uniform), 0..4
  // every wavefront takes part in the staging barriers whatever its tile count (none: the
  // one-tile body, which writes nothing)
  switch (nt) {
    case 4: k_gram_wide_body<E, 4>(A, na, B, nb, ng, part, la, lb, sym, ntile); break;
    case 3: k_gram_wide_body<E, 3>(A, na, B, nb, ng, part, la, lb, sym, ntile); break;
    case 2: k_gram_wide_body<E, 2>(A, na, B, nb, ng, part, la, lb, sym, ntile); break;
    default: k_gram_wide_body<E, 1>(A, na, B, nb, ng, part, la, lb, sym, ntile); break;
  }
}

// out[o] = scale * sum_b part[b][o], one workgroup per output o: thread t adds blocks t,
// t + kThreads, ... in order, each wavefront adds its 64 sums by a butterfly, and the
// wavefront sums are added in order (a fixed summation for every launch).  Many small
// workgroups spread the partial rows over the whole chip; one workgroup reading all of them
// (as a fused reduction + Cholesky would) measured three to four times slower.
template <typename W>
__device__ __forceinline__ W shfl_xor_w(W v, int m);
template <>
__device__ __forceinline__ double shfl_xor_w<double>(double v, int m) {
  return __shfl_xor(v, m, 64);
}
template <>
__device__ __forceinline__ C2<double> shfl_xor_w<C2<double>>(C2<double> v, int m) {
  return {__shfl_xor(v.r, m, 64), __shfl_xor(v.i, m, 64)};
}

// Gram matrices of at least this many entries are reduced by k_gram_reduce_cols, smaller ones
// by k_gram_reduce; the choice is made per system so that a system's sums are the same
// whether it is reduced alone or in a batch (only_cols: -1 any, 0 small ones only, 1 large
// ones only).
constexpr int kColsMin = 1024;

// Output o of a reduction by the first kThreads threads of the workgroup (any further
// wavefronts only take the barrier), so the order of the sums does not depend on the
// workgroup size of the launch it runs in.
template <typename W>
__device__ __forceinline__ void gram_reduce_one(const RedArgs& ra, int o) {
  __shared__ W red[kThreads / 64];
  if (threadIdx.x < kThreads) {
    const W* __restrict__ part = (const W*)ra.part;
    W s = W{};
    for (int b = threadIdx.x; b < ra.nblk; b += kThreads) s = e_add(s, part[(size_t)b * ra.no + o]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s = e_add(s, shfl_xor_w(s, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    W t = red[0];
#pragma unroll
    for (int w = 1; w < kThreads / 64; ++w) t = e_add(t, red[w]);
    ((W*)ra.out)[o] = e_scale(t, ra.scale);
  }
}

template <typename W, typename S>
__global__ __launch_bounds__(kThreads) void k_gram_reduce(S src, int only_cols) {
  const RedArgs ra = src.get(blockIdx.y);
  const int o = blockIdx.x;
  if (o >= ra.no || (only_cols == 0 && ra.no >= kColsMin)) return;
  gram_reduce_one<W>(ra, o);
}

// The same sums for many outputs (large Gram matrices): a workgroup takes 16 consecutive
// outputs, so each partial row is read as one contiguous 16-entry run instead of one entry per
// cache line; thread (block group bg, output ol) adds blocks bg, bg + 16, ... in order and the
// 16 group sums are added in order.
template <typename W, typename S>
__global__ __launch_bounds__(kThreads) void k_gram_reduce_cols(S src, int only_cols) {
  constexpr int NO = 16, NG = kThreads / NO;
  __shared__ W red[NG][NO];
  const RedArgs ra = src.get(blockIdx.y);
  const int nblk = ra.nblk;
  if (only_cols == 1 && ra.no < kColsMin) return;
  const int ol = threadIdx.x % NO, bg = threadIdx.x / NO;
  const int o = blockIdx.x * NO + ol;
  const W* __restrict__ part = (const W*)ra.part;
  W acc = W{};
  if (o < ra.no) {
    // loads batched eight at a time; the additions keep their order
    int b = bg;
    for (; b + 7 * NG < nblk; b += 8 * NG) {
      W v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(b + u * NG) * ra.no + o];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = e_add(acc, v[u]);
    }
    for (; b < nblk; b += NG) acc = e_add(acc, part[(size_t)b * ra.no + o]);
  }
  red[bg][ol] = acc;
  __syncthreads();
  if (threadIdx.x < NO && o < ra.no) {
    W t = red[0][ol];
    for (int g2 = 1; g2 < NG; ++g2) t = e_add(t, red[g2][ol]);
    ((W*)ra.out)[o] = e_scale(t, ra.scale);
  }
}

// nout: the largest output count over the nsys systems.  One system takes the kernel its
// size selects; a batch whose largest system is large runs both kernels, each skipping the
// systems of the other size class.
template <typename W, typename S>
void reduce_launch(S sr, int nout, int nsys, hipStream_t s) {
  if (nout < kColsMin) {
    dim3 rg(nout, nsys);
    k_gram_reduce<W, S><<<rg, kThreads, 0, s>>>(sr, -1);
    return;
  }
  if (nsys > 1) {
    dim3 rg(kColsMin - 1, nsys);
    k_gram_reduce<W, S><<<rg, kThreads, 0, s>>>(sr, 0);
  }
  dim3 rg((nout + 15) / 16, nsys);
  k_gram_reduce_cols<W, S><<<rg, kThreads, 0, s>>>(sr, nsys > 1 ? 1 : -1);
}

// Cholesky of -M (Hermitised), L^{-H} and E_x in one wavefront, FP64.  Lane i holds row i of
// the working matrix in registers (right-looking factorisation, pivots broadcast by
// shuffles); L goes through LDS for the triangular inverse, lane c solving column c.
template <typename W, typename S>
__global__ __launch_bounds__(64) void k_chol_lanes(S src) {
  const MolArgs ma = src.get(blockIdx.x);
  chol_lanes_body<W>(ma, (const W*)ma.mred);
}

template <typename W, int NMAX, typename S>
__global__ __launch_bounds__(64) void k_chol(S src) {
  const MolArgs ma = src.get(blockIdx.x);
  const W* __restrict__ mred = (const W*)ma.mred;
  const int n = ma.n;
  W* __restrict__ m_out = (W*)ma.m_out;
  double* __restrict__ ex_out = ma.ex_out;
  W* __restrict__ linvh = (W*)ma.linvh;
  int* __restrict__ status = ma.status;
  __shared__ W L[NMAX * NMAX];
  const int i = threadIdx.x;
  const bool row = i < n;
  W a[NMAX];
  bool bad = false;
  double diag = 0.0;
#pragma unroll
  for (int k = 0; k < NMAX; ++k) {
    a[k] = W{};
    if (row && k < n) {
      const W mik = mred[i * n + k], mki = mred[k * n + i];
      bad |= !e_finite(mik);
      const W herm = e_scale(e_add(mik, e_conj(mki)), 0.5);
      if (m_out) m_out[i * n + k] = herm;
      if (k == i) diag = e_re(herm);
      a[k] = e_neg(herm);
    }
  }
  // E_x = 1/2 sum_i M_ii
  double e = diag;
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if (i == 0 && ex_out) *ex_out = 0.5 * e;
  const bool any_bad = __any(bad);
  // right-looking factorisation; the pivot and column j are broadcast through LDS (one
  // wavefront, so the barriers are cheap), 1/L_jj is kept for the inverse below
  __shared__ W colj[NMAX];
  __shared__ double piv_s, dinv[NMAX];
  int fail = -1;
#pragma unroll
  for (int j = 0; j < NMAX; ++j) {
    if (j < n) {
      if (i == j) piv_s = e_re(a[j]);
      __syncthreads();
      const double piv = piv_s;
      if (!(piv > 0.0) && fail < 0) fail = j;
      const double d = piv > 0.0 ? sqrt(piv) : 1.0;
      const double invd = 1.0 / d;
      const W lij = (i > j) ? e_scale(a[j], invd) : (i == j ? w_from_real(d, W{}) : W{});
      a[j] = lij;
      if (row) colj[i] = lij;
      if (i == j) dinv[j] = invd;
      __syncthreads();
#pragma unroll
      for (int k = j + 1; k < NMAX; ++k)
        if (k < n) a[k] = e_sub(a[k], e_mul(lij, e_conj(colj[k])));
    }
  }
  if (row) {
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
      if (k < n) L[i * NMAX + k] = k <= i ? a[k] : W{};
  }
  __syncthreads();
  const bool ok = fail < 0 && !any_bad;
  // column c = i of X = L^{-1}: X[r][c] = (delta_rc - sum_{c<=k<r} L[r][k] X[k][c]) / L[r][r]
  if (row) {
    W x[NMAX];
#pragma unroll
    for (int r = 0; r < NMAX; ++r) {
      x[r] = W{};
      if (r < n && r >= i) {
        W s = (r == i) ? w_from_real(1.0, W{}) : W{};
#pragma unroll
        for (int k = 0; k < r; ++k)
          if (k >= i) s = e_sub(s, e_mul(L[r * NMAX + k], x[k]));
        x[r] = e_scale(s, dinv[r]);
      }
    }
    // L^{-H}[c][k] = conj(X[k][c])
#pragma unroll
    for (int k = 0; k < NMAX; ++k)
      if (k < n) linvh[i * n + k] = ok ? e_conj(x[k]) : W{};
  }
  if (i == 0 && !ok && status && status[0] == 0) {
    status[0] = any_bad ? -6 : -5;
    status[1] = any_bad ? -1 : fail;
  }
}

// xi_k(r) = sum_{i<=k} W_i(r) (L^{-H})_{ik}; in place allowed (xi may alias W).  L^{-H} is
// staged in LDS, rounded once to the storage precision.
template <typename E, int NMAX, typename S>
__global__ __launch_bounds__(kThreads) void k_trsm(S src, size_t ng_arg) {
  const Placed<MolArgs> pc = src.place(ng_arg);
  const MolArgs ma = pc.a;
  const size_t ng = pc.ng;
  const E* w = (const E*)ma.w;  // xi may alias w
  E* xi = (E*)ma.xi;
  const int n = ma.n;
  const typename Elem<E>::wide* __restrict__ linvh = (const typename Elem<E>::wide*)ma.linvh;
  __shared__ E lh[NMAX * NMAX];
  // this thread's W values are requested before the staging of L^{-H}, so the two loads
  // overlap (points past the end read the last point and are not stored)
  const size_t r = pc.blk * kThreads + threadIdx.x;
  const size_t rc = r < ng ? r : ng - 1;
  E wr[NMAX];
#pragma unroll
  for (int i = 0; i < NMAX; ++i) wr[i] = w[(size_t)(i < n ? i : n - 1) * ng + rc];
  for (int t = threadIdx.x; t < n * n; t += kThreads)
    lh[(t / n) * NMAX + t % n] = e_narrow<E>(linvh[t]);
  __syncthreads();
  if (r >= ng) return;
#pragma unroll
  for (int k = 0; k < NMAX; ++k) {
    if (k < n) {
      E s = e_zero<E>();
#pragma unroll
      for (int i = 0; i <= k; ++i) s = e_add(s, e_mul(wr[i], lh[i * NMAX + k]));
      xi[(size_t)k * ng + r] = s;
    }
  }
}

// Cholesky (n <= 8) and xi = W L^{-H} in one launch: every workgroup factorises M itself in
// its first wavefront (the same arithmetic as k_chol_lanes, so the same bits) while its W
// values load; workgroup 0 writes M, E_x, L^{-H} and the status.
// (body: point block blk of the system ma)
template <typename E>
__device__ __forceinline__ void chol_trsm_body(const MolArgs& ma, size_t blk, size_t ng) {
  typedef typename Elem<E>::wide W;
  const E* w = (const E*)ma.w;  // xi may alias w
  E* xi = (E*)ma.xi;
  const int n = ma.n;
  __shared__ W lw[64];
  __shared__ E lh[64];
  const size_t r = blk * kThreads + threadIdx.x;
  const size_t rc = r < ng ? r : ng - 1;
  E wr[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) wr[i] = w[(size_t)(i < n ? i : n - 1) * ng + rc];
  if (threadIdx.x < 64) chol_lanes_body<W>(ma, (const W*)ma.mred, lw, blk == 0);
  __syncthreads();
  for (int t = threadIdx.x; t < n * n; t += kThreads) lh[(t / n) * 8 + t % n] = e_narrow<E>(lw[t]);
  __syncthreads();
  if (r >= ng) return;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (k < n) {
      E s = e_zero<E>();
#pragma unroll
      for (int i = 0; i <= k; ++i) s = e_add(s, e_mul(wr[i], lh[i * 8 + k]));
      xi[(size_t)k * ng + r] = s;
    }
  }
}

template <typename E, typename S>
__global__ __launch_bounds__(kThreads) void k_chol_trsm(S src, size_t ng_arg) {
  const Placed<MolArgs> pc = src.place(ng_arg);
  chol_trsm_body<E>(pc.a, pc.blk, pc.ng);
}

// Column v of Z = L^{-1} Y (n <= 8) with Y = scale * (sum of the partial rows in ra; row b
// holds entry (k, v) at k * nv + v): the first wavefront factorises -M into LDS (the same
// arithmetic as every Cholesky workgroup) while the other three reduce the n entries of the
// column, each thread over every G-th row; the G group sums are added in order.
template <typename W>
__device__ __forceinline__ void z_column_body(const MolArgs& ma, const RedArgs& ra, int nv, int v) {
  constexpr int G = (kThreads - 64) / 8;
  __shared__ W lz[64];
  __shared__ W red[G][8];
  __shared__ W ycol[8];
  const int n = ma.n;
  if (threadIdx.x < 64) {
    chol_lanes_body<W>(ma, (const W*)ma.mred, lz, false);
  } else {
    const int t = threadIdx.x - 64, k = t & 7, g = t >> 3;
    W acc{};
    if (k < n) {
      const W* __restrict__ part = (const W*)ra.part + (size_t)k * nv + v;
      const size_t row = (size_t)ra.no;
      int b = g;
      // loads six at a time; the additions keep their order
      for (; b + 5 * G < ra.nblk; b += 6 * G) {
        W x[6];
#pragma unroll
        for (int u = 0; u < 6; ++u) x[u] = part[(size_t)(b + u * G) * row];
#pragma unroll
        for (int u = 0; u < 6; ++u) acc = e_add(acc, x[u]);
      }
      for (; b < ra.nblk; b += G) acc = e_add(acc, part[(size_t)b * row]);
    }
    red[g][k] = acc;
  }
  __syncthreads();
  if (threadIdx.x < 8) {
    W y = red[0][threadIdx.x];
    for (int g = 1; g < G; ++g) y = e_add(y, red[g][threadIdx.x]);
    ycol[threadIdx.x] = e_scale(y, ra.scale);
  }
  __syncthreads();
  if ((int)threadIdx.x < n) {
    const int k = threadIdx.x;
    W z{};
    for (int i = 0; i <= k; ++i) z = e_add(z, e_mul(e_conj(lz[i * n + k]), ycol[i]));
    ((W*)ra.out)[k * nv + v] = z;
  }
}

// Two launches of an ACE build + K psi (complex storage, at most 8 orbitals, one system) that
// each carry a second, independent step in extra workgroups:
//   k_gram_c8_reduce: the partials of Y = W^H psi dV, and in its first nred workgroups (of
//     tile group 0) the reduction of M's partials, one output each -- the code of
//     k_gram_c8 and k_gram_reduce, so the same bits;
//   k_chol_trsm_zcol: the Cholesky factorisation and xi = W L^{-H} (k_chol_trsm's code and
//     bits), and in nv workgroups after them the columns of Z = xi^H psi dV = L^{-1} Y.
template <typename E, int TB, bool VEC, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_gram_c8_reduce(GramArgs ga, size_t ng, RedArgs ra,
                                                               int nred) {
  if ((int)blockIdx.x < nred) {
    if (blockIdx.y == 0) gram_reduce_one<typename Elem<E>::wide>(ra, blockIdx.x);
    return;
  }
  gram_c8_body<E, TB, VEC, WAVES>(ga, blockIdx.x - nred, (int)blockIdx.y, ng);
}

template <typename E>
__global__ __launch_bounds__(kThreads) void k_chol_trsm_zcol(MolArgs ma, size_t ng, RedArgs ra,
                                                             int nv) {
  const size_t nbx = (ng + kThreads - 1) / kThreads;
  if (blockIdx.x < nbx)
    chol_trsm_body<E>(ma, blockIdx.x, ng);
  else
    z_column_body<typename Elem<E>::wide>(ma, ra, nv, (int)(blockIdx.x - nbx));
}

// Streaming (nontemporal) store: the K psi outputs are not read again by this step, and the
// hint keeps them from displacing cached data (measured 11.7 -> 9.8 us at 48^3, 32 vectors).
template <typename E>
__device__ __forceinline__ void store_stream(E* p, E v) {
  if constexpr (Elem<E>::cplx) {
    typedef typename Elem<E>::real R;
    typedef R R2 __attribute__((ext_vector_type(2)));
    R2 x;
    x.x = v.r;
    x.y = v.i;
    __builtin_nontemporal_store(x, reinterpret_cast<R2*>(p));
  } else {
    __builtin_nontemporal_store(v, p);
  }
}

// out_v(r) = -sum_k xi_k(r) Z_kv,  Z = xi^H psi dV (already scaled).  Grid: (point blocks,
// groups of VB vectors); the group's slice of Z is staged in LDS in the storage precision.
// FROM_Y: z holds Y = W^H psi dV instead, and the staging forms Z = L^{-1} Y in FP64 from
// linvh = L^{-H} (xi = W L^{-H}, so xi^H = L^{-1} W^H).
template <typename E, int NMAX, int VB, bool FROM_Y = false>
__global__ __launch_bounds__(kThreads) void k_apply_out(const E* __restrict__ xi, int n, size_t ng,
                                                        const typename Elem<E>::wide* __restrict__ z,
                                                        int nv, E* __restrict__ out,
                                                        const typename Elem<E>::wide* __restrict__ linvh = nullptr) {
  typedef typename Elem<E>::wide W;
  __shared__ E zs[NMAX * VB];
  const int v0 = blockIdx.y * VB;
  // xi is requested before the staging of Z, so the two loads overlap (points past the end
  // read the last point and are not stored)
  const size_t r = (size_t)blockIdx.x * kThreads + threadIdx.x;
  const size_t rc = r < ng ? r : ng - 1;
  E xr[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k) xr[k] = xi[(size_t)(k < n ? k : n - 1) * ng + rc];
  if constexpr (FROM_Y) {
    // Z_kv = sum_{i<=k} conj((L^{-H})_ik) Y_iv: four lanes per entry, lane p adding the terms
    // i = p, p + 4, ..., then the quad's sums (the quads are whole, as 4 n VB is a multiple
    // of 4);
    for (int t = threadIdx.x; t < 4 * n * VB; t += kThreads) {
      const int e = t >> 2, p = t & 3;
      const int k = e / VB, vb = e % VB;
      const int vc = v0 + vb < nv ? v0 + vb : nv - 1;
      W s{};
      if constexpr (NMAX <= 16) {
        // all of the lane's loads are issued before its sums (terms past k read row 0 and are
        // not added)
        constexpr int NT = NMAX / 4;
        W lv[NT], yv[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const int i = p + 4 * j, ic = i <= k ? i : 0;
          lv[j] = linvh[ic * n + k];
          yv[j] = z[ic * nv + vc];
        }
#pragma unroll
        for (int j = 0; j < NT; ++j)
          if (p + 4 * j <= k) s = e_add(s, e_mul(e_conj(lv[j]), yv[j]));
      } else {
        for (int i = p; i <= k; i += 4) s = e_add(s, e_mul(e_conj(linvh[i * n + k]), z[i * nv + vc]));
      }
      s = e_add(s, shfl_xor_w(s, 1));
      s = e_add(s, shfl_xor_w(s, 2));
      if (p == 0) zs[k * VB + vb] = v0 + vb < nv ? e_narrow<E>(s) : e_zero<E>();
    }
  } else {
    for (int t = threadIdx.x; t < n * VB; t += kThreads) {
      const int k = t / VB, vb = t % VB;
      zs[k * VB + vb] = (v0 + vb < nv) ? e_narrow<E>(z[k * nv + v0 + vb]) : e_zero<E>();
    }
  }
  __syncthreads();
  if (r >= ng) return;
#pragma unroll
  for (int vb = 0; vb < VB; ++vb) {
    const int v = v0 + vb;
    if (v < nv) {
      E s = e_zero<E>();
#pragma unroll
      for (int k = 0; k < NMAX; ++k)
        if (k < n) s = e_add(s, e_mul(xr[k], zs[k * VB + vb]));
      store_stream(out + (size_t)v * ng + r, e_neg(s));
    }
  }
}

// ta row tiles; tb column tiles (upper bounds over the systems of a launch); the B tiles of
// a row tile are taken two at a time for single-precision storage
// Launch extent of a pointwise step: bx blocks of 256 points along x (one system's blocks, or
// the blocks of every system of a flat launch), sys systems along the last grid dimension
// (1 for a flat launch), the point count passed to single-edge sources, and whether every
// system's point count is a multiple of 4 (16-byte vector loads in the Gram kernels).
struct Grid {
  unsigned bx;
  unsigned sys;
  size_t ng;
  bool vec;
};
inline Grid grid_one_edge(size_t ng, int nsys) {
  return {(unsigned)((ng + kThreads - 1) / kThreads), (unsigned)nsys, ng, ng % 4 == 0};
}

template <typename E, typename S>
void gram_impl(S src, int ta, int tb, Grid g, int skip8, hipStream_t s) {
  constexpr bool SMALL = sizeof(typename Elem<E>::real) == 4;
  if (SMALL && tb >= 2) {
    dim3 grid(g.bx, ta * ((tb + 1) / 2), g.sys);
    if (g.vec)
      k_gram<E, S, 2, true><<<grid, kThreads, 0, s>>>(src, g.ng, skip8);
    else
      k_gram<E, S, 2, false><<<grid, kThreads, 0, s>>>(src, g.ng, skip8);
  } else {
    dim3 grid(g.bx, ta * tb, g.sys);
    if (g.vec)
      k_gram<E, S, 1, true><<<grid, kThreads, 0, s>>>(src, g.ng, skip8);
    else
      k_gram<E, S, 1, false><<<grid, kThreads, 0, s>>>(src, g.ng, skip8);
  }
}

// dispatch on the storage element type
template <template <typename> class F, typename... Args>
void by_elem(int et, Args... args) {
  switch (et) {
    case ET_C128: F<C2<double>>::run(args...); break;
    case ET_C64: F<C2<float>>::run(args...); break;
    case ET_R64: F<double>::run(args...); break;
    case ET_R32: F<float>::run(args...); break;
  }
}

template <typename E>
struct WaccRun {
  template <typename S>
  static void run(S src, int nmax, Grid g, hipStream_t s) {
    dim3 grid(g.bx, g.sys);
    if (nmax <= 8)
      k_wacc<E, 8, S><<<grid, kThreads, 0, s>>>(src, g.ng);
    else if (nmax <= 16)
      k_wacc<E, 16, S><<<grid, kThreads, 0, s>>>(src, g.ng);
    else if (nmax <= 32 || Elem<E>::cplx)
      k_wacc<E, 32, S><<<grid, kThreads, 0, s>>>(src, g.ng);
    else if constexpr (!Elem<E>::cplx)
      k_wacc<E, 64, S><<<grid, kThreads, 0, s>>>(src, g.ng);
  }
};

// fused W + M partials when one workgroup's phi and W fit in LDS (nmax <= 16, and <= 8 for
// complex FP64); returns false if the separate W and Gram kernels must be used
template <typename E>
struct WaccGramRun {
  template <typename S>
  static void run(S src, int nmax, Grid g, bool* done, hipStream_t s) {
    *done = false;
    const int lim = sizeof(E) > 8 ? 8 : 16;
    if (kGramPoints != kThreads || nmax > lim) return;
    dim3 grid(g.bx, g.sys);
    if (nmax <= 8)
      k_wacc_gram<E, 8, S><<<grid, kThreads, 0, s>>>(src, g.ng);
    else if constexpr (sizeof(E) <= 8)
      k_wacc_gram<E, 16, S><<<grid, kThreads, 0, s>>>(src, g.ng);
    *done = true;
  }
};

template <typename E>
struct TrsmRun {
  template <typename S>
  static void run(S src, int nmax, Grid g, hipStream_t s) {
    dim3 grid(g.bx, g.sys);
    if (nmax <= 8)
      k_trsm<E, 8, S><<<grid, kThreads, 0, s>>>(src, g.ng);
    else if (nmax <= 16)
      k_trsm<E, 16, S><<<grid, kThreads, 0, s>>>(src, g.ng);
    else if (nmax <= 32 || Elem<E>::cplx)
      k_trsm<E, 32, S><<<grid, kThreads, 0, s>>>(src, g.ng);
    else if constexpr (!Elem<E>::cplx)
      k_trsm<E, 64, S><<<grid, kThreads, 0, s>>>(src, g.ng);
  }
};

// c8_waves: wavefronts per workgroup of the stacked kernel (4 gives the fused W + M kernel's
// summation order, for M of a build; 8 is faster for xi^H psi)
template <typename E>
struct GramRun {
  // nred: systems of the reduction (the grid's sys is 1 for a flat launch)
  template <typename SG, typename SR>
  static void run(SG sg, SR sr, int namax, int nbmax, int nout, int nred, Grid g, int c8_waves,
                  hipStream_t s) {
    typedef typename Elem<E>::wide W;
    // complex systems with at most 8 A rows (every one, when namax <= 8) take the stacked
    // kernel; the others the general one
    if constexpr (Elem<E>::cplx) {
      // four 8-column tiles per workgroup (measured best of 2/4 tiles and 4/8/16 wavefronts
      // at 48^3, 8 x 32: eight wavefronts of 32 points)
      const int groups = ((nbmax + 7) / 8 + 3) / 4;
      dim3 grid(g.bx, groups, g.sys);
      if (c8_waves == 8) {
        if (g.vec)
          k_gram_c8<E, SG, 4, true, 8><<<grid, 512, 0, s>>>(sg, g.ng);
        else
          k_gram_c8<E, SG, 4, false, 8><<<grid, 512, 0, s>>>(sg, g.ng);
      } else {
        if (g.vec)
          k_gram_c8<E, SG, 4, true, 4><<<grid, 256, 0, s>>>(sg, g.ng);
        else
          k_gram_c8<E, SG, 4, false, 4><<<grid, 256, 0, s>>>(sg, g.ng);
      }
    }
    if (!Elem<E>::cplx || namax > 8)
      gram_impl<E, SG>(sg, (namax + 15) / 16, (nbmax + 15) / 16, g, 1, s);
    reduce_launch<W, SR>(sr, nout, nred, s);
  }
};

template <bool CPLX>
struct CholRun {
  template <typename S>
  static void run(S src, int nmax, int nsys, hipStream_t s) {
    typedef typename std::conditional<CPLX, C2<double>, double>::type W;
    if (nmax <= 8)
      k_chol_lanes<W, S><<<nsys, 64, 0, s>>>(src);
    else if (nmax <= 16)
      k_chol<W, 16, S><<<nsys, 64, 0, s>>>(src);
    else if (nmax <= 32 || CPLX)
      k_chol<W, 32, S><<<nsys, 64, 0, s>>>(src);
    else if constexpr (!CPLX)
      k_chol<W, 64, S><<<nsys, 64, 0, s>>>(src);
  }
};

template <typename S>
void chol_any(int et, S src, int nmax, int nsys, hipStream_t s) {
  if (et == ET_C128 || et == ET_C64)
    CholRun<true>::run(src, nmax, nsys, s);
  else
    CholRun<false>::run(src, nmax, nsys, s);
}

}  // namespace

int gram_blocks(size_t ng, size_t* chunk) {
  // one partial per workgroup of kGramPoints points
  size_t c = kGramPoints;
  size_t nblk = (ng + c - 1) / c;
  if (nblk < 1) nblk = 1;
  *chunk = c;
  return (int)nblk;
}

static MolArgs single(const void* phi, const void* v, void* w, void* xi, void* mred, void* linvh,
                      void* m_out, double* ex_out, int* status, int n, size_t ng) {
  MolArgs m{};
  m.phi = phi;
  m.v = v;
  m.w = w;
  m.xi = xi;
  m.mred = mred;
  m.linvh = linvh;
  m.m_out = m_out;
  m.ex_out = ex_out;
  m.status = status;
  m.n = n;
  m.blk0 = 0;
  m.ng = ng;
  return m;
}

static int gram_rows(size_t ng) {
  size_t chunk;
  return gram_blocks(ng, &chunk);
}

void launch_wacc(int et, const void* phi, const void* v, int n, size_t ng, void* w, hipStream_t s, Trace* tr) {
  TraceScope ts(tr, TR_WACC);
  OneMol src{single(phi, v, w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, n, ng)};
  by_elem<WaccRun>(et, src, n, grid_one_edge(ng, 1), s);
}

template <typename S>
static void reduce_any(int et, S src, int nout, int nsys, hipStream_t s) {
  if (et == ET_C128 || et == ET_C64)
    reduce_launch<C2<double>, S>(src, nout, nsys, s);
  else
    reduce_launch<double, S>(src, nout, nsys, s);
}

bool launch_wacc_partials(int et, const void* phi, const void* v, int n, size_t ng, void* w,
                          void* part, hipStream_t s, Trace* tr) {
  MolArgs m = single(phi, v, w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, n, ng);
  m.part = part;
  bool done = false;
  {
    TraceScope ts(tr, TR_WACC);
    by_elem<WaccGramRun>(et, OneMol{m}, n, grid_one_edge(ng, 1), &done, s);
  }
  if (!done) launch_wacc(et, phi, v, n, ng, w, s, tr);
  return done;
}

void launch_wacc_finish(int et, bool partials, const void* phi, int n, size_t ng, const void* w,
                        void* part, double scale, void* mred, hipStream_t s, Trace* tr) {
  if (!partials) {
    launch_gram(et, phi, n, w, n, ng, part, scale, mred, s, tr);
  } else {
    TraceScope ts(tr, TR_GRAM);
    reduce_any(et, OneRed{RedArgs{part, n * n, mred, gram_rows(ng), scale}}, n * n, 1, s);
  }
}

void launch_wacc_gram(int et, const void* phi, const void* v, int n, size_t ng, void* w,
                      void* part, double scale, void* mred, hipStream_t s, Trace* tr) {
  const bool partials = launch_wacc_partials(et, phi, v, n, ng, w, part, s, tr);
  launch_wacc_finish(et, partials, phi, n, ng, w, part, scale, mred, s, tr);
}

void launch_chol_trsm(int et, const void* mred, int n, void* m_out, double* ex_out, void* linvh,
                      int* status, const void* w, size_t ng, void* xi, hipStream_t s, Trace* tr) {
  if (n > 8) {
    launch_chol(et, mred, n, m_out, ex_out, linvh, status, s, tr);
    launch_trsm(et, w, n, ng, linvh, xi, s, tr);
    return;
  }
  TraceScope ts(tr, TR_TRSM);
  OneMol src{single(nullptr, nullptr, const_cast<void*>(w), xi, const_cast<void*>(mred), linvh,
                    m_out, ex_out, status, n, ng)};
  dim3 grid((unsigned)((ng + kThreads - 1) / kThreads), 1);
  switch (et) {
    case ET_C128: k_chol_trsm<C2<double>, OneMol><<<grid, kThreads, 0, s>>>(src, ng); break;
    case ET_C64: k_chol_trsm<C2<float>, OneMol><<<grid, kThreads, 0, s>>>(src, ng); break;
    case ET_R64: k_chol_trsm<double, OneMol><<<grid, kThreads, 0, s>>>(src, ng); break;
    case ET_R32: k_chol_trsm<float, OneMol><<<grid, kThreads, 0, s>>>(src, ng); break;
  }
}

void launch_gram(int et, const void* A, int na, const void* B, int nb, size_t ng, void* part,
                 double scale, void* out, hipStream_t s, Trace* tr) {
  TraceScope ts(tr, TR_GRAM);
  const int nch = gram_rows(ng);
  if ((et == ET_R32 || et == ET_R64) && na > 16 && nb > 16 && na <= kWideRows &&
      nb <= kWideRows) {
    if (et == ET_R32)
      k_gram_wide<float><<<nch, kThreads, 0, s>>>((const float*)A, na, (const float*)B, nb, ng,
                                                  (double*)part);
    else
      k_gram_wide<double><<<nch, kThreads, 0, s>>>((const double*)A, na, (const double*)B, nb,
                                                   ng, (double*)part);
    OneRed sr{RedArgs{part, na * nb, out, nch, scale}};
    reduce_launch<double, OneRed>(sr, na * nb, 1, s);
    return;
  }
  OneGram sg{GramArgs{A, na, B, nb, part}};
  OneRed sr{RedArgs{part, na * nb, out, nch, scale}};
  by_elem<GramRun>(et, sg, sr, na, nb, na * nb, 1, grid_one_edge(ng, 1), 8, s);
}

void launch_chol(int et, const void* mred, int n, void* m_out, double* ex_out, void* linvh,
                 int* status, hipStream_t s, Trace* tr) {
  TraceScope ts(tr, TR_CHOL);
  OneMol src{single(nullptr, nullptr, nullptr, nullptr, const_cast<void*>(mred), linvh, m_out,
                    ex_out, status, n, 0)};
  chol_any(et, src, n, 1, s);
}

void launch_trsm(int et, const void* w, int n, size_t ng, const void* linvh, void* xi, hipStream_t s, Trace* tr) {
  TraceScope ts(tr, TR_TRSM);
  OneMol src{single(nullptr, nullptr, const_cast<void*>(w), xi, nullptr, const_cast<void*>(linvh),
                    nullptr, nullptr, nullptr, n, ng)};
  by_elem<TrsmRun>(et, src, n, grid_one_edge(ng, 1), s);
}

void launch_ace_steps_flat(int et, const MolArgs* mols_dev, const int* bsys_dev, int nmol,
                           int nblk, int nmax, hipStream_t s, Trace* tr) {
  // every system's point count is a multiple of 4 exactly when the caller says so through the
  // sign of nblk (negative: some are not)
  const bool vec = nblk > 0;
  const Grid g{(unsigned)(vec ? nblk : -nblk), 1u, 0, vec};
  FlatMol fm{mols_dev, bsys_dev};
  bool fused = false;
  {
    TraceScope ts(tr, TR_WACC);
    by_elem<WaccGramRun>(et, fm, nmax, g, &fused, s);
    if (!fused) by_elem<WaccRun>(et, fm, nmax, g, s);
  }
  {
    TraceScope ts(tr, TR_GRAM);
    if (fused)
      reduce_any(et, ManyRed{mols_dev}, nmax * nmax, nmol, s);
    else
      by_elem<GramRun>(et, FlatGram{mols_dev, bsys_dev}, ManyRed{mols_dev}, nmax, nmax,
                       nmax * nmax, nmol, g, 4, s);
  }
  {
    TraceScope ts(tr, TR_CHOL);
    chol_any(et, ManyMol{mols_dev}, nmax, nmol, s);
  }
  TraceScope ts(tr, TR_TRSM);
  by_elem<TrsmRun>(et, fm, nmax, g, s);
}

template <typename E, int VB, bool FROM_Y>
static void apply_vb(const void* xi, int n, size_t ng, const void* z, int nv, void* out,
                     const void* linvh, hipStream_t s) {
  typedef typename Elem<E>::wide W;
  dim3 blocks((unsigned)((ng + kThreads - 1) / kThreads), (unsigned)((nv + VB - 1) / VB));
  const W* lh = (const W*)linvh;
  if (n <= 8)
    k_apply_out<E, 8, VB, FROM_Y><<<blocks, kThreads, 0, s>>>((const E*)xi, n, ng, (const W*)z, nv, (E*)out, lh);
  else if (n <= 16)
    k_apply_out<E, 16, VB, FROM_Y><<<blocks, kThreads, 0, s>>>((const E*)xi, n, ng, (const W*)z, nv, (E*)out, lh);
  else if (n <= 32 || Elem<E>::cplx)
    k_apply_out<E, 32, VB, FROM_Y><<<blocks, kThreads, 0, s>>>((const E*)xi, n, ng, (const W*)z, nv, (E*)out, lh);
  else if constexpr (!Elem<E>::cplx)
    k_apply_out<E, 64, VB, FROM_Y><<<blocks, kThreads, 0, s>>>((const E*)xi, n, ng, (const W*)z, nv, (E*)out, lh);
}

// 8 vectors per workgroup row (measured against 4, 16 and 32 at 48^3, 8 orbitals, 32 vectors)
template <typename E, bool FROM_Y>
static void apply_impl(const void* xi, int n, size_t ng, const void* z, int nv, void* out,
                       const void* linvh, hipStream_t s) {
  apply_vb<E, 8, FROM_Y>(xi, n, ng, z, nv, out, linvh, s);
}

template <bool FROM_Y>
static void apply_any(int et, const void* xi, int n, size_t ng, const void* z, int nv, void* out,
                      const void* linvh, hipStream_t s) {
  switch (et) {
    case ET_C128: apply_impl<C2<double>, FROM_Y>(xi, n, ng, z, nv, out, linvh, s); break;
    case ET_C64: apply_impl<C2<float>, FROM_Y>(xi, n, ng, z, nv, out, linvh, s); break;
    case ET_R64: apply_impl<double, FROM_Y>(xi, n, ng, z, nv, out, linvh, s); break;
    case ET_R32: apply_impl<float, FROM_Y>(xi, n, ng, z, nv, out, linvh, s); break;
  }
}

void launch_apply_out(int et, const void* xi, int n, size_t ng, const void* z, int nv, void* out,
                      hipStream_t s, Trace* tr) {
  TraceScope ts(tr, TR_APPLY);
  apply_any<false>(et, xi, n, ng, z, nv, out, nullptr, s);
}

void launch_apply_from_y(int et, const void* xi, int n, size_t ng, const void* linvh,
                         const void* y, int nv, void* out, hipStream_t s, Trace* tr) {
  TraceScope ts(tr, TR_APPLY);
  apply_any<true>(et, xi, n, ng, y, nv, out, linvh, s);
}

bool launch_gram_y_reduce_m(int et, const void* w, int n, const void* psi, int nv, size_t ng,
                            void* part_y, const void* part_m, double scale, void* mred,
                            hipStream_t s, Trace* tr) {
  if ((et != ET_C64 && et != ET_C128) || n > 8 || nv < 1) return false;
  TraceScope ts(tr, TR_GRAM);
  const Grid g = grid_one_edge(ng, 1);
  const int nred = n * n;
  // four 8-column tiles per workgroup and eight wavefronts, as launch_gram's Gram of xi^H psi
  const int groups = ((nv + 7) / 8 + 3) / 4;
  dim3 grid(g.bx + nred, groups);
  const GramArgs ga{w, n, psi, nv, part_y};
  const RedArgs ra{part_m, nred, mred, gram_rows(ng), scale};
  if (et == ET_C64) {
    if (g.vec)
      k_gram_c8_reduce<C2<float>, 4, true, 8><<<grid, 512, 0, s>>>(ga, ng, ra, nred);
    else
      k_gram_c8_reduce<C2<float>, 4, false, 8><<<grid, 512, 0, s>>>(ga, ng, ra, nred);
  } else {
    if (g.vec)
      k_gram_c8_reduce<C2<double>, 4, true, 8><<<grid, 512, 0, s>>>(ga, ng, ra, nred);
    else
      k_gram_c8_reduce<C2<double>, 4, false, 8><<<grid, 512, 0, s>>>(ga, ng, ra, nred);
  }
  return true;
}

void launch_chol_trsm_zcol(int et, const void* mred, int n, void* m_out, double* ex_out,
                           void* linvh, int* status, const void* w, size_t ng, void* xi,
                           const void* part_y, int nv, void* z, double scale, hipStream_t s,
                           Trace* tr) {
  TraceScope ts(tr, TR_TRSM);
  const MolArgs ma = single(nullptr, nullptr, const_cast<void*>(w), xi, const_cast<void*>(mred),
                            linvh, m_out, ex_out, status, n, ng);
  const RedArgs ra{part_y, n * nv, z, gram_rows(ng), scale};
  dim3 grid((unsigned)((ng + kThreads - 1) / kThreads) + nv);
  if (et == ET_C64)
    k_chol_trsm_zcol<C2<float>><<<grid, kThreads, 0, s>>>(ma, ng, ra, nv);
  else
    k_chol_trsm_zcol<C2<double>><<<grid, kThreads, 0, s>>>(ma, ng, ra, nv);
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
  typename Elem<E>::wide acc{};
  for (int j = 0; j < n; ++j)
    acc = e_add(acc, e_mul(e_wide(phi[(size_t)j * ng + r]), e_wide(v[((size_t)vi * n + j) * ng + r])));
  out[(size_t)vi * ng + r] = e_narrow<E>(e_neg(acc));
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
