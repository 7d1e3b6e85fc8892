// Learned eigensolver preconditioner: a three-layer 3-D convolutional network
//   x (1 channel) -> conv 3^3 (8) -> ReLU -> conv 3^3 (8) -> ReLU -> conv 3^3 (1)
// with zero padding, BF16 weights (FP32 master copies updated by Adam) and FP32 activations
// and accumulation.  Forward, backward (data and weight gradients), the mean-squared loss and
// Adam are hand-written kernels; the C ABI below drives inference and training on the device.
//
// Activations are [sample][channel][x][y][z] FP32.  Weights of a layer are [out][in][27] with
// tap t = 9 (dx + 1) + 3 (dy + 1) + (dz + 1) acting on the input at offset (dx, dy, dz).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ace.h"
#include "ctx.hpp"

namespace {

using ace::host::Buf;
using ace::host::ensure_on;
using ace::host::hip_check;

constexpr int kT = 256;
// output tile of one workgroup and its halo (each thread computes ZP points along z)
constexpr int TX = 8, TY = 8, TZ = 16, ZP = 4;
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HVOL = HX * HY * HZ;
constexpr int C = 8;  // hidden channels

// parameter layout: [w0 8x1x27][b0 8][w1 8x8x27][b1 8][w2 1x8x27][b2 1]
constexpr int W0 = 0, B0 = W0 + C * 27, W1 = B0 + C, B1 = W1 + C * C * 27, W2 = B1 + C,
              B2 = W2 + C * 27, NPAR = B2 + 1;
static_assert(NPAR == ACE_NET_PARAMS, "parameter count");

struct Tiles {
  int nx, ny, nz;
  explicit Tiles(int n) : nx((n + TX - 1) / TX), ny((n + TY - 1) / TY), nz((n + TZ - 1) / TZ) {}
  int count() const { return nx * ny * nz; }
};

__device__ __forceinline__ void tile_origin(int bt, int tny, int tnz, int* x0, int* y0, int* z0) {
  const int tz = bt % tnz, ty = (bt / tnz) % tny, tx = bt / (tnz * tny);
  *x0 = tx * TX;
  *y0 = ty * TY;
  *z0 = tz * TZ;
}

// stage CI channels of the input tile with a one-point halo (zero outside the box)
template <int CI>
__device__ __forceinline__ void stage_halo(float* tile, const float* __restrict__ inb, int n,
                                           size_t ng, int x0, int y0, int z0) {
  for (int e = threadIdx.x; e < CI * HVOL; e += kT) {
    const int i = e / HVOL, q = e % HVOL;
    const int hz = q % HZ, hy = (q / HZ) % HY, hx = q / (HZ * HY);
    const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
    const bool ok = (unsigned)gx < (unsigned)n && (unsigned)gy < (unsigned)n && (unsigned)gz < (unsigned)n;
    const size_t idx = ok ? (size_t)i * ng + ((size_t)gx * n + gy) * n + gz : 0;
    const float v = inb[idx];
    tile[e] = ok ? v : 0.f;
  }
}

// out[o](p) = act(b[o] + sum_i sum_t w[o][i][t] in[i](p + d_t)) (* (mask[o](p) > 0)).
// The input channels pass through LDS four at a time (a 4-channel halo tile is 28.8 KB, so
// five workgroups fit on a CU instead of two for all eight channels at once).
template <int CI, int CO, bool BIAS, bool RELU, bool MASK>
__global__ __launch_bounds__(kT) void k_conv(const float* __restrict__ in, const float* __restrict__ w,
                                             const float* __restrict__ b,
                                             const float* __restrict__ mask, float* __restrict__ out,
                                             int n, int tny, int tnz) {
  constexpr int CH = CI < 4 ? CI : 4;  // input channels per LDS stage
  static_assert(CI % CH == 0, "whole stages");
  __shared__ float tile[CH * HVOL];
  // weights re-laid out [i][t][o] (o fastest) so a tap's CO weights are one broadcast read
  constexpr int COP = CO < 4 ? 4 : CO;
  __shared__ __align__(16) float wl[CI * 27 * COP];
  const size_t ng = (size_t)n * n * n;
  int x0, y0, z0;
  tile_origin(blockIdx.x, tny, tnz, &x0, &y0, &z0);
  const size_t sb = blockIdx.y;
  for (int e = threadIdx.x; e < CI * 27 * COP; e += kT) {
    const int o = e % COP, it = e / COP;  // it = i * 27 + t
    wl[e] = o < CO ? w[(o * CI + it / 27) * 27 + it % 27] : 0.f;
  }
  const int lz = (threadIdx.x % 4) * ZP, ly = (threadIdx.x / 4) % TY, lx = threadIdx.x / 32;
  float acc[CO][ZP];
#pragma unroll
  for (int o = 0; o < CO; ++o)
#pragma unroll
    for (int p = 0; p < ZP; ++p) acc[o][p] = BIAS ? b[o] : 0.f;
#pragma unroll 1
  for (int c0 = 0; c0 < CI; c0 += CH) {
    if (c0 > 0) __syncthreads();  // every thread is done with the previous stage
    stage_halo<CH>(tile, in + (sb * CI + c0) * ng, n, ng, x0, y0, z0);
    __syncthreads();
#pragma unroll 1
    for (int ii = 0; ii < CH; ++ii) {
      const int i = c0 + ii;
#pragma unroll 1
      for (int dx = 0; dx < 3; ++dx)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
          const float* col = tile + ii * HVOL + ((lx + dx) * HY + (ly + dy)) * HZ + lz;
          float c[ZP + 2];
#pragma unroll
          for (int u = 0; u < ZP + 2; ++u) c[u] = col[u];
#pragma unroll
          for (int dz = 0; dz < 3; ++dz) {
            const float* wt = wl + ((i * 27) + dx * 9 + dy * 3 + dz) * COP;
            float wv[COP];
#pragma unroll
            for (int q = 0; q < COP; q += 4) {
              const float4 v4 = *reinterpret_cast<const float4*>(wt + q);
              wv[q] = v4.x;
              wv[q + 1] = v4.y;
              wv[q + 2] = v4.z;
              wv[q + 3] = v4.w;
            }
#pragma unroll
            for (int o = 0; o < CO; ++o)
#pragma unroll
              for (int p = 0; p < ZP; ++p) acc[o][p] += wv[o] * c[p + dz];
          }
        }
    }
  }
  const int gx = x0 + lx, gy = y0 + ly;
  if (gx >= n || gy >= n) return;
  // with n a multiple of 4 the thread's ZP = 4 points are one aligned 16-byte run (z0 + lz is
  // a multiple of 4): one vector store per channel instead of four scattered ones
  static_assert(ZP == 4 && TZ % 4 == 0, "four z-points per thread");
  const bool vec4 = (n & 3) == 0 && ((reinterpret_cast<uintptr_t>(out) |
                                      (MASK ? reinterpret_cast<uintptr_t>(mask) : 0)) & 15) == 0;
  if (vec4) {
    const int gz = z0 + lz;
    if (gz >= n) return;
    const size_t pt = ((size_t)gx * n + gy) * n + gz;
#pragma unroll
    for (int o = 0; o < CO; ++o) {
      float4 v = make_float4(acc[o][0], acc[o][1], acc[o][2], acc[o][3]);
      if (RELU) v = make_float4(fmaxf(v.x, 0.f), fmaxf(v.y, 0.f), fmaxf(v.z, 0.f), fmaxf(v.w, 0.f));
      const size_t oi = (sb * CO + o) * ng + pt;
      if (MASK) {
        const float4 m = *reinterpret_cast<const float4*>(mask + oi);
        v = make_float4(m.x > 0.f ? v.x : 0.f, m.y > 0.f ? v.y : 0.f, m.z > 0.f ? v.z : 0.f,
                        m.w > 0.f ? v.w : 0.f);
      }
      *reinterpret_cast<float4*>(out + oi) = v;
    }
    return;
  }
#pragma unroll
  for (int p = 0; p < ZP; ++p) {
    const int gz = z0 + lz + p;
    if (gz >= n) continue;
    const size_t pt = ((size_t)gx * n + gy) * n + gz;
#pragma unroll
    for (int o = 0; o < CO; ++o) {
      float v = acc[o][p];
      if (RELU) v = fmaxf(v, 0.f);
      const size_t oi = (sb * CO + o) * ng + pt;
      if (MASK) v = mask[oi] > 0.f ? v : 0.f;
      out[oi] = v;
    }
  }
}

// Weight and bias gradient partials of one tile: gw[o][i][t] = sum_p g[o](p) in[i](p + d_t),
// gb[o] = sum_p g[o](p).  The input tile (with halo) and the tile of g (zero outside the box,
// stored [point][o]) are staged in LDS.  kwg(CI) groups of kT threads split the tile's x-rows;
// in each group thread (i, t[, o-group]) runs over its points reading its input value and the
// (broadcast) g values of the point, and the group partials are added in group order (four
// groups for 8 input channels: 347 against 498 us at 64^3 for 8 -> 8; one group for a single
// input channel, whose threads already carry 8 outputs each).
constexpr int kwg(int ci) { return ci == 1 ? 1 : 4; }
template <int CI, int CO, int KWG = kwg(CI)>
__global__ __launch_bounds__(kT * KWG) void k_wgrad(const float* __restrict__ in, const float* __restrict__ g,
                                                    float* __restrict__ part, int n, int tny, int tnz) {
  __shared__ float tile[CI * HVOL];
  __shared__ __align__(16) float gt[TX * TY * TZ * CO];
  constexpr int OG = (CI == 1) ? CO : 1, OPT = CO / OG, NACT = CI * 27 * OG;
  constexpr int NPL = CO * CI * 27 + CO;
  constexpr int TP = TX * TY * TZ;
  static_assert(NACT + CO <= kT, "threads");
  static_assert(TX % KWG == 0, "x-rows split evenly");
  __shared__ float red[KWG > 1 ? KWG - 1 : 1][kT * OPT];
  const size_t ng = (size_t)n * n * n;
  int x0, y0, z0;
  tile_origin(blockIdx.x, tny, tnz, &x0, &y0, &z0);
  const size_t sb = blockIdx.y;
  {
    const float* inb = in + sb * CI * ng;
    for (int e = threadIdx.x; e < CI * HVOL; e += kT * KWG) {
      const int i = e / HVOL, q = e % HVOL;
      const int hz = q % HZ, hy = (q / HZ) % HY, hx = q / (HZ * HY);
      const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
      const bool ok = (unsigned)gx < (unsigned)n && (unsigned)gy < (unsigned)n && (unsigned)gz < (unsigned)n;
      const size_t idx = ok ? (size_t)i * ng + ((size_t)gx * n + gy) * n + gz : 0;
      const float v = inb[idx];
      tile[e] = ok ? v : 0.f;
    }
  }
  const float* gb = g + sb * CO * ng;
  for (int e = threadIdx.x; e < TP * CO; e += kT * KWG) {
    const int o = e / TP, pt = e % TP;  // consecutive threads: consecutive z (coalesced)
    const int pz = pt % TZ, py = (pt / TZ) % TY, px = pt / (TZ * TY);
    const int gx = x0 + px, gy = y0 + py, gz = z0 + pz;
    const bool ok = gx < n && gy < n && gz < n;
    const size_t idx = ok ? (size_t)o * ng + ((size_t)gx * n + gy) * n + gz : 0;
    const float v = gb[idx];
    gt[pt * CO + o] = ok ? v : 0.f;
  }
  __syncthreads();
  const int grp = threadIdx.x / kT, t = threadIdx.x % kT;
  constexpr int XG = TX / KWG;  // x-rows per group
  float acc[OPT];
#pragma unroll
  for (int q = 0; q < OPT; ++q) acc[q] = 0.f;
  if (t < NACT) {
    const int og = t % OG, id = t / OG;
    const int i = id / 27, tap = id % 27;
    const int dx = tap / 9, dy = (tap / 3) % 3, dz = tap % 3;
    for (int px = grp * XG; px < (grp + 1) * XG; ++px)
      for (int py = 0; py < TY; ++py) {
        const float* trow = tile + i * HVOL + ((px + dx) * HY + (py + dy)) * HZ + dz;
        const float* grow = gt + ((px * TY + py) * TZ) * CO + og * OPT;
#pragma unroll
        for (int pz = 0; pz < TZ; ++pz) {
          const float v = trow[pz];
#pragma unroll
          for (int q = 0; q < OPT; ++q) acc[q] += grow[pz * CO + q] * v;
        }
      }
  } else if (t < NACT + CO) {
    const int o = t - NACT;
    for (int pt = grp * XG * TY * TZ; pt < (grp + 1) * XG * TY * TZ; ++pt) acc[0] += gt[pt * CO + o];
  }
  if (grp > 0) {
#pragma unroll
    for (int q = 0; q < OPT; ++q) red[grp - 1][t * OPT + q] = acc[q];
  }
  __syncthreads();
  if (grp > 0) return;
#pragma unroll
  for (int gq = 0; gq < KWG - 1; ++gq)
#pragma unroll
    for (int q = 0; q < OPT; ++q) acc[q] += red[gq][t * OPT + q];
  float* pb = part + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * NPL;
  if (t < NACT) {
    const int og = t % OG, id = t / OG;
    const int i = id / 27, tap = id % 27;
#pragma unroll
    for (int q = 0; q < OPT; ++q) pb[((og * OPT + q) * CI + i) * 27 + tap] = acc[q];
  } else if (t < NACT + CO) {
    pb[CO * CI * 27 + (t - NACT)] = acc[0];
  }
}

// grad[off + j] = sum over partial rows of part[row][j] (FP64, fixed order), one block per j
__global__ __launch_bounds__(kT) void k_part_reduce(const float* __restrict__ part, int rows, int npl,
                                                    float* __restrict__ grad) {
  __shared__ double red[kT];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int r = threadIdx.x; r < rows; r += kT) s += part[(size_t)r * npl + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[j] = (float)red[0];
}

// wt[i][o][t] = w[o][i][26 - t]: the layer's transposed, flipped kernel (data gradient)
__global__ void k_transpose_flip(const float* __restrict__ w, int co, int ci, float* __restrict__ wt) {
  for (int e = threadIdx.x; e < co * ci * 27; e += blockDim.x) {
    const int t = e % 27, o = (e / 27) % co, i = e / (27 * co);
    wt[e] = w[(o * ci + i) * 27 + 26 - t];
  }
}

// g = (y - t) * inv_count and per-block partial sums of (y - t)^2
constexpr int kLossParts = 256;
__global__ __launch_bounds__(kT) void k_loss(const float* __restrict__ y, const float* __restrict__ t,
                                             size_t count, float inv_count, float* __restrict__ g,
                                             double* __restrict__ part) {
  __shared__ double red[kT];
  double s = 0.0;
  for (size_t e = (size_t)blockIdx.x * kT + threadIdx.x; e < count; e += (size_t)gridDim.x * kT) {
    const float d = y[e] - t[e];
    g[e] = d * inv_count;
    s += (double)d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_loss_final(const double* __restrict__ part, int np, double scale,
                             double* __restrict__ out) {
  __shared__ double red[kT];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += kT) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = scale * red[0];
}

// round to the nearest BF16 value (ties to even), returned as FP32
__device__ __forceinline__ float bf16_round(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

__global__ void k_round_params(const float* __restrict__ w, int np, float* __restrict__ weff) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < np; e += gridDim.x * blockDim.x)
    weff[e] = bf16_round(w[e]);
}

// Adam (bias-corrected moments) on the FP32 masters; refreshes the BF16 compute copy
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int np, float lr, float b1, float b2,
                       float eps, float c1, float c2, float* __restrict__ weff) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < np; e += gridDim.x * blockDim.x) {
    const float ge = g[e];
    const float me = b1 * m[e] + (1.f - b1) * ge;
    const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    const float mh = me / c1, vh = ve / c2;
    const float we = w[e] - lr * mh / (sqrtf(vh) + eps);
    w[e] = we;
    weff[e] = bf16_round(we);
  }
}

// minibatch assembly from a counter-based generator (SplitMix64 of seed and slot)
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(kT) void k_gather(const float* __restrict__ xs, const float* __restrict__ ts,
                                               int count, size_t ng, unsigned long long seed,
                                               long long step, int batch, int random,
                                               float* __restrict__ xb, float* __restrict__ tb) {
  const int s = blockIdx.y;
  int idx = s % count;
  float sg = 1.f;
  if (random) {
    const unsigned long long hsh = splitmix64(seed ^ splitmix64((unsigned long long)step * batch + s));
    idx = (int)((hsh >> 1) % (unsigned long long)count);
    sg = (hsh & 1ull) ? -1.f : 1.f;
  }
  for (size_t e = (size_t)blockIdx.x * kT + threadIdx.x; e < ng; e += (size_t)gridDim.x * kT) {
    xb[(size_t)s * ng + e] = sg * xs[(size_t)idx * ng + e];
    tb[(size_t)s * ng + e] = sg * ts[(size_t)idx * ng + e];
  }
}

}  // namespace

struct ace_convnet {
  hipStream_t stream = nullptr;
  float* w = nullptr;     // FP32 masters [NPAR]
  float* weff = nullptr;  // BF16-rounded compute copy [NPAR]
  float* m = nullptr;
  float* v = nullptr;
  float* grad = nullptr;
  float* wt1 = nullptr;   // transposed-flipped layer-1 and layer-2 kernels
  float* wt2 = nullptr;
  double* loss = nullptr; // device scalar
  long long t = 0;        // Adam step counter
  Buf a1, a2, y, g, g2, g1, part, lpart, xb, tb, lhist;
};

namespace {

int net_alloc(ace_convnet* net) {
  float** bufs[] = {&net->w, &net->weff, &net->m, &net->v, &net->grad};
  for (float** b : bufs)
    if (hipMalloc(b, NPAR * sizeof(float)) != hipSuccess) return ACE_ERR_OOM;
  if (hipMalloc(&net->wt1, C * C * 27 * sizeof(float)) != hipSuccess ||
      hipMalloc(&net->wt2, C * 27 * sizeof(float)) != hipSuccess ||
      hipMalloc(&net->loss, sizeof(double)) != hipSuccess)
    return ACE_ERR_OOM;
  return ACE_OK;
}

// activations of a batch of nb samples of edge n
int net_ensure(ace_convnet* net, int n, int nb, bool train) {
  const size_t ng = (size_t)n * n * n;
  const Tiles tl(n);
  hipStream_t s = net->stream;
  int rc = ensure_on(s, net->a1, sizeof(float) * C * ng * nb);
  if (!rc) rc = ensure_on(s, net->a2, sizeof(float) * C * ng * nb);
  if (!rc && train) {
    const size_t rows = (size_t)tl.count() * nb;
    rc = ensure_on(s, net->y, sizeof(float) * ng * nb);
    if (!rc) rc = ensure_on(s, net->g, sizeof(float) * ng * nb);
    if (!rc) rc = ensure_on(s, net->g2, sizeof(float) * C * ng * nb);
    if (!rc) rc = ensure_on(s, net->g1, sizeof(float) * C * ng * nb);
    if (!rc) rc = ensure_on(s, net->part, sizeof(float) * rows * (C * C * 27 + C));
    if (!rc) rc = ensure_on(s, net->lpart, sizeof(double) * kLossParts);
  }
  return rc;
}

void forward(ace_convnet* net, int n, const float* x, int nb, float* y) {
  const Tiles tl(n);
  dim3 grid(tl.count(), nb);
  hipStream_t s = net->stream;
  float* a1 = (float*)net->a1.p;
  float* a2 = (float*)net->a2.p;
  k_conv<1, C, true, true, false><<<grid, kT, 0, s>>>(x, net->weff + W0, net->weff + B0, nullptr, a1, n, tl.ny, tl.nz);
  k_conv<C, C, true, true, false><<<grid, kT, 0, s>>>(a1, net->weff + W1, net->weff + B1, nullptr, a2, n, tl.ny, tl.nz);
  k_conv<C, 1, true, false, false><<<grid, kT, 0, s>>>(a2, net->weff + W2, net->weff + B2, nullptr, y, n, tl.ny, tl.nz);
}

// loss and gradient into net->grad for targets t; forward must have written net->y
void backward(ace_convnet* net, int n, const float* x, const float* t, int nb) {
  const Tiles tl(n);
  const size_t ng = (size_t)n * n * n, count = ng * nb;
  const int rows = tl.count() * nb;
  dim3 grid(tl.count(), nb);
  hipStream_t s = net->stream;
  float* a1 = (float*)net->a1.p;
  float* a2 = (float*)net->a2.p;
  float* g = (float*)net->g.p;
  float* g2 = (float*)net->g2.p;
  float* g1 = (float*)net->g1.p;
  float* part = (float*)net->part.p;
  k_loss<<<kLossParts, kT, 0, s>>>((const float*)net->y.p, t, count, 1.f / (float)count, g,
                                   (double*)net->lpart.p);
  k_loss_final<<<1, kT, 0, s>>>((const double*)net->lpart.p, kLossParts, 0.5 / (double)count, net->loss);
  k_transpose_flip<<<1, kT, 0, s>>>(net->weff + W1, C, C, net->wt1);
  k_transpose_flip<<<1, kT, 0, s>>>(net->weff + W2, 1, C, net->wt2);
  // layer 2 (8 -> 1)
  k_wgrad<C, 1><<<grid, kT * kwg(C), 0, s>>>(a2, g, part, n, tl.ny, tl.nz);
  k_part_reduce<<<C * 27 + 1, kT, 0, s>>>(part, rows, C * 27 + 1, net->grad + W2);
  k_conv<1, C, false, false, true><<<grid, kT, 0, s>>>(g, net->wt2, nullptr, a2, g2, n, tl.ny, tl.nz);
  // layer 1 (8 -> 8)
  k_wgrad<C, C><<<grid, kT * kwg(C), 0, s>>>(a1, g2, part, n, tl.ny, tl.nz);
  k_part_reduce<<<C * C * 27 + C, kT, 0, s>>>(part, rows, C * C * 27 + C, net->grad + W1);
  k_conv<C, C, false, false, true><<<grid, kT, 0, s>>>(g2, net->wt1, nullptr, a1, g1, n, tl.ny, tl.nz);
  // layer 0 (1 -> 8)
  k_wgrad<1, C><<<grid, kT * kwg(1), 0, s>>>(x, g1, part, n, tl.ny, tl.nz);
  k_part_reduce<<<C * 27 + C, kT, 0, s>>>(part, rows, C * 27 + C, net->grad + W0);
}

void adam(ace_convnet* net, double lr) {
  const double b1 = 0.9, b2 = 0.999;
  net->t += 1;
  const float c1 = (float)(1.0 - std::pow(b1, (double)net->t));
  const float c2 = (float)(1.0 - std::pow(b2, (double)net->t));
  k_adam<<<(NPAR + kT - 1) / kT, kT, 0, net->stream>>>(net->w, net->m, net->v, net->grad, NPAR,
                                                       (float)lr, (float)b1, (float)b2, 1e-8f,
                                                       c1, c2, net->weff);
}

}  // namespace

namespace ace {
// preconditioner application for the SCF driver: y_j = net(x_j), FP32 grid vectors
int convnet_apply_internal(ace_convnet* net, int n, const float* x, int nb, float* y,
                           hipStream_t s) {
  hipStream_t keep = net->stream;
  net->stream = s;
  int rc = net_ensure(net, n, nb, false);
  if (!rc) forward(net, n, x, nb, y);
  net->stream = keep;
  return rc ? rc : hip_check(hipGetLastError());
}
}  // namespace ace

extern "C" {

int convnet_create(void* hip_stream, ace_convnet** out) {
  if (!out) return ACE_ERR_INVALID;
  *out = nullptr;
  ace_convnet* net = new (std::nothrow) ace_convnet();
  if (!net) return ACE_ERR_OOM;
  net->stream = (hipStream_t)hip_stream;
  int rc = net_alloc(net);
  if (!rc) {
    std::vector<float> zero(NPAR, 0.f);
    for (float* b : {net->w, net->weff, net->m, net->v, net->grad})
      if (hipMemcpy(b, zero.data(), NPAR * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        rc = ACE_ERR_HIP;
  }
  if (rc) {
    (void)hipGetLastError();
    convnet_destroy(net);
    return rc;
  }
  *out = net;
  return ACE_OK;
}

int convnet_destroy(ace_convnet* net) {
  if (!net) return ACE_OK;
  (void)hipStreamSynchronize(net->stream);
  for (float* b : {net->w, net->weff, net->m, net->v, net->grad, net->wt1, net->wt2})
    if (b) (void)hipFree(b);
  if (net->loss) (void)hipFree(net->loss);
  for (Buf* b : {&net->a1, &net->a2, &net->y, &net->g, &net->g2, &net->g1, &net->part,
                 &net->lpart, &net->xb, &net->tb, &net->lhist})
    if (b->p) (void)hipFree(b->p);
  delete net;
  return ACE_OK;
}

int convnet_set_params(ace_convnet* net, const float* params) {
  if (!net || !params) return ACE_ERR_INVALID;
  hipStream_t s = net->stream;
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(net->w, params, NPAR * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
    return ACE_ERR_HIP;
  std::vector<float> zero(NPAR, 0.f);
  if (hipMemcpy(net->m, zero.data(), NPAR * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(net->v, zero.data(), NPAR * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
    return ACE_ERR_HIP;
  net->t = 0;
  k_round_params<<<(NPAR + kT - 1) / kT, kT, 0, s>>>(net->w, NPAR, net->weff);
  if (hipStreamSynchronize(s) != hipSuccess) return ACE_ERR_HIP;
  return hip_check(hipGetLastError());
}

int convnet_get_params(ace_convnet* net, float* params, int rounded) {
  if (!net || !params) return ACE_ERR_INVALID;
  if (hipStreamSynchronize(net->stream) != hipSuccess ||
      hipMemcpy(params, rounded ? net->weff : net->w, NPAR * sizeof(float),
                hipMemcpyDeviceToHost) != hipSuccess)
    return ACE_ERR_HIP;
  return ACE_OK;
}

int convnet_forward(ace_convnet* net, int n, const float* x, int nb, float* y) {
  if (!net || !x || !y || n < 1 || nb < 1) return ACE_ERR_INVALID;
  int rc = net_ensure(net, n, nb, false);
  if (rc) return rc;
  forward(net, n, x, nb, y);
  return hip_check(hipGetLastError());
}

int convnet_gradient(ace_convnet* net, int n, const float* x, const float* t, int nb,
                     double* loss, float* grad) {
  if (!net || !x || !t || n < 1 || nb < 1) return ACE_ERR_INVALID;
  int rc = net_ensure(net, n, nb, true);
  if (rc) return rc;
  forward(net, n, x, nb, (float*)net->y.p);
  backward(net, n, x, t, nb);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(net->stream) != hipSuccess)
    return ACE_ERR_HIP;
  if (loss && hipMemcpy(loss, net->loss, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return ACE_ERR_HIP;
  if (grad && hipMemcpy(grad, net->grad, NPAR * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return ACE_ERR_HIP;
  return ACE_OK;
}

int convnet_train(ace_convnet* net, int n, const float* inputs, const float* targets, int count,
                  int steps, int batch, double lr, unsigned long long seed, int flags,
                  double* loss_hist) {
  if (!net || !inputs || !targets || n < 1 || count < 1 || steps < 1 || batch < 1 ||
      !(lr > 0.0))
    return ACE_ERR_INVALID;
  const bool random = (flags & ACE_TRAIN_RANDOM) != 0;
  if (!random && batch != count) return ACE_ERR_INVALID;
  const size_t ng = (size_t)n * n * n;
  hipStream_t s = net->stream;
  int rc = net_ensure(net, n, batch, true);
  if (!rc) rc = ensure_on(s, net->xb, sizeof(float) * ng * batch);
  if (!rc) rc = ensure_on(s, net->tb, sizeof(float) * ng * batch);
  if (!rc) rc = ensure_on(s, net->lhist, sizeof(double) * steps);
  if (rc) return rc;
  double* lh = (double*)net->lhist.p;
  for (int st = 0; st < steps; ++st) {
    const float* xb = inputs;
    const float* tb = targets;
    if (random) {
      dim3 g((unsigned)std::min<size_t>(1024, (ng + kT - 1) / kT), batch);
      k_gather<<<g, kT, 0, s>>>(inputs, targets, count, ng, seed, net->t, batch, 1,
                                (float*)net->xb.p, (float*)net->tb.p);
      xb = (const float*)net->xb.p;
      tb = (const float*)net->tb.p;
    }
    forward(net, n, xb, batch, (float*)net->y.p);
    backward(net, n, xb, tb, batch);
    if (hipMemcpyAsync(lh + st, net->loss, sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
      return ACE_ERR_HIP;
    adam(net, lr);
  }
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return ACE_ERR_HIP;
  if (loss_hist &&
      hipMemcpy(loss_hist, lh, sizeof(double) * steps, hipMemcpyDeviceToHost) != hipSuccess)
    return ACE_ERR_HIP;
  return ACE_OK;
}

}  // extern "C"
