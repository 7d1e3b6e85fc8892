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

#include "poisson_body.hpp"

namespace ace {

namespace {

// Z-forward pass of one launch sequence: workgroup (x, p).
template <typename T, int N, bool RP, typename R>
__global__ __launch_bounds__(zf_threads<N>()) void k_zfwd(R res, C2<T>* __restrict__ work,
                                                   const TwE<T>* __restrict__ twg) {
  constexpr int P = 2 * N;
  C2<T>* buf = lds<T>();
  const TwE<T>* tw = stage_twiddles<T, P>(buf, (size_t)N * (P + 1), twg);
  __syncthreads();
  const int p = blockIdx.y;
  zfwd_plane<T, N, RP, R>(res, p, blockIdx.x, work + (size_t)p * P * N * N, tw, buf,
                          threadIdx.x, zf_threads<N>());
}

// XY pass of one system: workgroup (blockIdx.x, p) takes planes K blockIdx.x .. + K - 1 of
// transform p, with NT threads.
template <typename T, int N, int K, int NT>
__global__ __launch_bounds__(NT) void k_xy(C2<T>* __restrict__ work, const T* __restrict__ gpos,
                                           const TwE<T>* __restrict__ twg) {
  constexpr int P = 2 * N;
  C2<T>* pl = lds<T>();
  const TwE<T>* tw = stage_twiddles<T, P>(pl, (size_t)K * P * (P + 1), twg);
  __syncthreads();
  const int qz0 = blockIdx.x * K, p = blockIdx.y;
  xy_planes<T, N, K>(work + ((size_t)p * P + qz0) * N * N, (size_t)N * N,
                     gpos + (size_t)qz0 * P * P, pl, tw, threadIdx.x, NT);
}

// XY pass with the rows-and-strips layout (planes larger than the LDS): workgroup (qz, p).
template <typename T, int N, int NT>
__global__ __launch_bounds__(NT) void k_xy_strips(C2<T>* __restrict__ work,
                                                  const T* __restrict__ gpos,
                                                  const TwE<T>* __restrict__ twg) {
  constexpr int P = 2 * N, SW = strip_width<T, N>();
  C2<T>* pl = lds<T>();
  const TwE<T>* tw = stage_twiddles<T, P>(pl, (size_t)N * (P + 1) + (size_t)P * (SW + 1), twg);
  __syncthreads();
  const int qz = blockIdx.x, p = blockIdx.y;
  xy_strips<T, N, SW>(work + ((size_t)p * P + qz) * N * N, gpos + (size_t)qz * P * P, pl, tw,
                      threadIdx.x, NT);
}

// Z-inverse pass of one launch sequence: workgroup (x, p).
template <typename T, int N, bool RP, typename R>
__global__ __launch_bounds__(zi_threads<N>()) void k_zinv(const C2<T>* __restrict__ work, R res,
                                                   const TwE<T>* __restrict__ twg) {
  constexpr int P = 2 * N;
  C2<T>* buf = lds<T>();
  const TwE<T>* tw = stage_twiddles<T, P>(buf, (size_t)N * (P + 1), twg);
  __syncthreads();
  const int p = blockIdx.y;
  zinv_plane<T, N, RP, R>(work + (size_t)p * P * N * N, res, p, blockIdx.x, tw, buf,
                          threadIdx.x, zi_threads<N>());
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
    if constexpr (fits<T, N>()) {
      constexpr int nt = xy_threads<T, N>();
      allow_lds(k_xy<T, N, 1, nt>, lds_xy);
      k_xy<T, N, 1, nt><<<gxy, nt, lds_xy, s>>>(w, gh, t);
    } else {
      allow_lds(k_xy_strips<T, N, 512>, strip_lds<T, N>());
      k_xy_strips<T, N, 512><<<gxy, 512, strip_lds<T, N>(), s>>>(w, gh, t);
    }
  }
  {
    TraceScope ts(tr, TR_ZINV);
    if (rp)
      k_zinv<T, N, true, R><<<gz, zi_threads<N>(), lds_z, s>>>(w, res, t);
    else
      k_zinv<T, N, false, R><<<gz, zi_threads<N>(), lds_z, s>>>(w, res, t);
  }
}

}  // namespace

bool poisson_size_supported(int n, bool fp64) {
#define ACE_CASE(NN) \
  case NN:           \
    return fp64 ? supported<double, NN>() : supported<float, NN>();
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
    if constexpr (supported<double, NN>()) {                                              \
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

template <typename T, int N>
static void xy_edge(int nt, void* work, int count, const void* gpos, const void* tw,
                    hipStream_t s) {
  constexpr int P = 2 * N;
  const size_t lds = lds_with_twiddles<T, P>((size_t)P * (P + 1));
  dim3 grid(P, count);
  C2<T>* w = reinterpret_cast<C2<T>*>(work);
  const T* g = reinterpret_cast<const T*>(gpos);
  const TwE<T>* t = reinterpret_cast<const TwE<T>*>(tw);
  if constexpr (!fits<T, N>()) {
    allow_lds(k_xy_strips<T, N, 512>, strip_lds<T, N>());
    k_xy_strips<T, N, 512><<<grid, 512, strip_lds<T, N>(), s>>>(w, g, t);
  } else if (nt == 512) {
    allow_lds(k_xy<T, N, 1, 512>, lds);
    k_xy<T, N, 1, 512><<<grid, 512, lds, s>>>(w, g, t);
  } else {
    allow_lds(k_xy<T, N, 1, 1024>, lds);
    k_xy<T, N, 1, 1024><<<grid, 1024, lds, s>>>(w, g, t);
  }
}

int launch_xy_edge(int n, bool fp64, int nt, void* work, int count, const void* gpos,
                   const void* tw, hipStream_t s) {
  if (count <= 0) return 0;
#define ACE_CASE(NN)                                                       \
  case NN:                                                                 \
    if constexpr (supported<double, NN>()) {                                    \
      if (fp64) {                                                          \
        xy_edge<double, NN>(nt, work, count, gpos, tw, s);                 \
        return 0;                                                          \
      }                                                                    \
    }                                                                      \
    if (fp64) return -1;                                                   \
    xy_edge<float, NN>(nt, work, count, gpos, tw, s);                      \
    return 0;
  switch (n) {
    ACE_SIZES(ACE_CASE)
    default:
      return -1;
  }
#undef ACE_CASE
}

void launch_pair_poisson(int n, bool fp64, bool real_packed, const void* phi_a, int na,
                         const void* phi_b, int nb, const int* pairs_dev, int np, void* work,
                         void* v_out, const void* ghat, const void* tw, int* status,
                         hipStream_t s, Trace* tr) {
  PairsByIndex res{phi_a, phi_b, pairs_dev, v_out, np, na, nb, status};
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
