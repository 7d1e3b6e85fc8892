// Persistent pair-Poisson passes over many independent systems of any box edges in one launch
// per pass (the uneven multi-molecule batch: the ACE rebuild of Sec. 3.1 for many systems at
// once).  The host lists every transform of every system as a job and every plane of a job as
// an item, largest box edge first; a grid of as many workgroups as the device holds at once
// walks the item list with a fixed stride, each item dispatched on its box edge to the same
// per-plane bodies as the one-system passes (poisson_body.hpp), so every transform gets the
// same bits as in a one-system build.  The XY items of an edge take K consecutive qz planes
// (K chosen per edge by the tuner of the batch), which keeps a workgroup sized for the largest
// plane of the launch busy on the smaller edges.
#include <algorithm>

#include "poisson_body.hpp"

namespace ace {

namespace {

// Pair resolver of one job: index 0 is p0, index 1 is p1 (real-packed couples).
struct JobPairs {
  const QJob* j;
  int np;
  template <typename E>
  __device__ __forceinline__ const E* a(int q, size_t) const {
    return reinterpret_cast<const E*>(q == 0 ? j->p0.a : j->p1.a);
  }
  template <typename E>
  __device__ __forceinline__ const E* b(int q, size_t) const {
    return reinterpret_cast<const E*>(q == 0 ? j->p0.b : j->p1.b);
  }
  template <typename E>
  __device__ __forceinline__ E* v(int q, size_t) const {
    return reinterpret_cast<E*>(q == 0 ? j->p0.v : j->p1.v);
  }
  __device__ __forceinline__ int kind(int) const { return j->p0.kind; }
  template <typename E>
  __device__ __forceinline__ E* v2(int, size_t) const {
    return reinterpret_cast<E*>(j->p0.v2);
  }
};

template <typename T, int N, int K>
constexpr bool xy_k_fits() {
  return fits<T, N>() && (2 * N) % K == 0 &&
         lds_with_twiddles<T, 2 * N>((size_t)K * 2 * N * (2 * N + 1)) <= kMaxLds;
}

// ---- per-item dispatch on the box edge ---------------------------------------------------
template <typename T, int N, bool RP>
__device__ __attribute__((noinline)) void zfwd_item_n(const QJob* jb, int x, C2<T>* buf, int nt) {
  constexpr int P = 2 * N;
  const TwE<T>* tw =
      stage_twiddles<T, P>(buf, (size_t)N * (P + 1), reinterpret_cast<const TwE<T>*>(jb->tw));
  __syncthreads();
  const JobPairs res{jb, jb->np};
  zfwd_plane<T, N, RP, JobPairs>(res, 0, x, reinterpret_cast<C2<T>*>(jb->work), tw, buf,
                                 threadIdx.x, nt);
}

template <typename T, int N, bool RP>
__device__ __attribute__((noinline)) void zinv_item_n(const QJob* jb, int x, C2<T>* buf, int nt) {
  constexpr int P = 2 * N;
  const TwE<T>* tw =
      stage_twiddles<T, P>(buf, (size_t)N * (P + 1), reinterpret_cast<const TwE<T>*>(jb->tw));
  const JobPairs res{jb, jb->np};
  // the twiddles are first read after the pass's own barrier
  zinv_plane<T, N, RP, JobPairs>(reinterpret_cast<const C2<T>*>(jb->work), res, 0, x, tw, buf,
                                 threadIdx.x, nt);
}

template <typename T, int N, int K>
__device__ __attribute__((noinline)) void xy_item_nk(const QJob* jb, int qz0, C2<T>* pl, int nt) {
  constexpr int P = 2 * N;
  const TwE<T>* tw = stage_twiddles<T, P>(pl, (size_t)K * P * (P + 1),
                                          reinterpret_cast<const TwE<T>*>(jb->tw));
  __syncthreads();
  xy_planes<T, N, K>(reinterpret_cast<C2<T>*>(jb->work) + (size_t)qz0 * N * N, (size_t)N * N,
                     reinterpret_cast<const T*>(jb->gpos) + (size_t)qz0 * P * P, pl, tw,
                     threadIdx.x, nt);
}

template <typename T, bool RP>
__device__ __forceinline__ void zfwd_item(const QJob* jb, int x, C2<T>* buf, int nt) {
  switch (jb->edge) {
#define ACE_CASE(NN)                                                  \
  case NN:                                                            \
    if constexpr (supported<T, NN>()) zfwd_item_n<T, NN, RP>(jb, x, buf, nt); \
    break;
    ACE_SIZES(ACE_CASE)
#undef ACE_CASE
  }
}

template <typename T, bool RP>
__device__ __forceinline__ void zinv_item(const QJob* jb, int x, C2<T>* buf, int nt) {
  switch (jb->edge) {
#define ACE_CASE(NN)                                                  \
  case NN:                                                            \
    if constexpr (supported<T, NN>()) zinv_item_n<T, NN, RP>(jb, x, buf, nt); \
    break;
    ACE_SIZES(ACE_CASE)
#undef ACE_CASE
  }
}

template <typename T, int N>
__device__ __attribute__((noinline)) void xy_strip_item_n(const QJob* jb, int qz, C2<T>* pl,
                                                          int nt) {
  constexpr int P = 2 * N, SW = strip_width<T, N>();
  const TwE<T>* tw = stage_twiddles<T, P>(pl, (size_t)N * (P + 1) + (size_t)P * (SW + 1),
                                          reinterpret_cast<const TwE<T>*>(jb->tw));
  __syncthreads();
  xy_strips<T, N, SW>(reinterpret_cast<C2<T>*>(jb->work) + (size_t)qz * N * N,
                      reinterpret_cast<const T*>(jb->gpos) + (size_t)qz * P * P, pl, tw,
                      threadIdx.x, nt);
}

template <typename T>
__device__ __forceinline__ void xy_item(const QJob* jb, int qz0, C2<T>* pl, int nt) {
  const int k = jb->k;
  switch (jb->edge) {
#define ACE_CASE(NN)                                                                       \
  case NN:                                                                                 \
    if constexpr (!fits<T, NN>() && supported<T, NN>()) {                                  \
      xy_strip_item_n<T, NN>(jb, qz0, pl, nt);                                            \
    }                                                                                      \
    if constexpr (xy_k_fits<T, NN, 1>()) {                                                 \
      if (k == 1) xy_item_nk<T, NN, 1>(jb, qz0, pl, nt);                                  \
    }                                                                                      \
    if constexpr (xy_k_fits<T, NN, 2>()) {                                                 \
      if (k == 2) xy_item_nk<T, NN, 2>(jb, qz0, pl, nt);                                  \
    }                                                                                      \
    if constexpr (xy_k_fits<T, NN, 4>()) {                                                 \
      if (k == 4) xy_item_nk<T, NN, 4>(jb, qz0, pl, nt);                                  \
    }                                                                                      \
    break;
    ACE_SIZES(ACE_CASE)
#undef ACE_CASE
  }
}

// ---- the persistent kernels ---------------------------------------------------------------
// Workgroup b takes items b, b + G, b + 2G, ... (G = gridDim.x); every workgroup leaves the
// loop after its last item, and the LDS is handed from one item to the next by a barrier.
template <typename T, bool RP, int NT>
__global__ __launch_bounds__(NT) void k_zfwd_q(const QJob* __restrict__ jobs,
                                               const QItem* __restrict__ items, int nitems) {
  C2<T>* buf = lds<T>();
  for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
    const QItem it = items[i];
    __syncthreads();
    zfwd_item<T, RP>(jobs + it.job, it.idx, buf, NT);
  }
}

template <typename T, bool RP, int NT>
__global__ __launch_bounds__(NT) void k_zinv_q(const QJob* __restrict__ jobs,
                                               const QItem* __restrict__ items, int nitems) {
  C2<T>* buf = lds<T>();
  for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
    const QItem it = items[i];
    __syncthreads();
    zinv_item<T, RP>(jobs + it.job, it.idx, buf, NT);
  }
}

// ---- per-edge forms of the z passes -------------------------------------------------------
// One launch over consecutive jobs of one box edge N (jobs[blockIdx.y], x-plane blockIdx.x)
// with the thread count and LDS of the one-system kernels, so that every edge runs at its own
// occupancy instead of that of a workgroup sized for the largest edge; same bodies, same bits.
template <typename T, int N, bool RP>
__global__ __launch_bounds__(zf_threads<N>()) void k_zfwd_e(const QJob* __restrict__ jobs) {
  constexpr int P = 2 * N;
  const QJob* jb = jobs + blockIdx.y;
  C2<T>* buf = lds<T>();
  const TwE<T>* tw =
      stage_twiddles<T, P>(buf, (size_t)N * (P + 1), reinterpret_cast<const TwE<T>*>(jb->tw));
  __syncthreads();
  const JobPairs res{jb, jb->np};
  zfwd_plane<T, N, RP, JobPairs>(res, 0, blockIdx.x, reinterpret_cast<C2<T>*>(jb->work), tw,
                                 buf, threadIdx.x, zf_threads<N>());
}

template <typename T, int N, bool RP>
__global__ __launch_bounds__(zi_threads<N>()) void k_zinv_e(const QJob* __restrict__ jobs) {
  constexpr int P = 2 * N;
  const QJob* jb = jobs + blockIdx.y;
  C2<T>* buf = lds<T>();
  const TwE<T>* tw =
      stage_twiddles<T, P>(buf, (size_t)N * (P + 1), reinterpret_cast<const TwE<T>*>(jb->tw));
  const JobPairs res{jb, jb->np};
  // the twiddles are first read after the pass's own barrier
  zinv_plane<T, N, RP, JobPairs>(reinterpret_cast<const C2<T>*>(jb->work), res, 0, blockIdx.x,
                                 tw, buf, threadIdx.x, zi_threads<N>());
}

template <typename T, int N, bool RP>
void z_edge(bool forward, const QJob* jobs, int count, hipStream_t s) {
  constexpr int P = 2 * N;
  const size_t lds = lds_with_twiddles<T, P>((size_t)N * (P + 1));
  dim3 grid(N, count);
  if (forward) {
    allow_lds(k_zfwd_e<T, N, RP>, lds);
    k_zfwd_e<T, N, RP><<<grid, zf_threads<N>(), lds, s>>>(jobs);
  } else {
    allow_lds(k_zinv_e<T, N, RP>, lds);
    k_zinv_e<T, N, RP><<<grid, zi_threads<N>(), lds, s>>>(jobs);
  }
}

template <typename T>
int z_edge_any(bool forward, int n, bool rp, const QJob* jobs, int count, hipStream_t s) {
  switch (n) {
#define ACE_CASE(NN)                                                       \
  case NN:                                                                 \
    if constexpr (supported<T, NN>()) {                                    \
      rp ? z_edge<T, NN, true>(forward, jobs, count, s)                    \
         : z_edge<T, NN, false>(forward, jobs, count, s);                  \
      return 0;                                                            \
    }                                                                      \
    return -1;
    ACE_SIZES(ACE_CASE)
#undef ACE_CASE
  }
  return -1;
}

constexpr int kXyQueueThreads = 1024;

// One 1024-thread workgroup per CU: the per-edge bodies are separate functions (inlined into
// one kernel they spill), each allowed the 128 registers of four waves per SIMD.
template <typename T>
__global__ __launch_bounds__(kXyQueueThreads) void k_xy_q(const QJob* __restrict__ jobs,
                                                         const QItem* __restrict__ items,
                                                         int nitems) {
  C2<T>* pl = lds<T>();
  for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
    const QItem it = items[i];
    __syncthreads();
    xy_item<T>(jobs + it.job, it.idx, pl, kXyQueueThreads);
  }
}

// workgroups of a persistent launch: every CU filled to the kernel's occupancy at this LDS size
template <typename Kern>
int persistent_grid(Kern kernel, int nt, size_t lds, int nitems) {
  allow_lds(kernel, lds);
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel),
                                                   nt, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return std::max(1, std::min(nitems, cus * per_cu));
}

template <typename T, bool RP>
void launch_z_passes(bool forward, const QJob* jobs, const QItem* items, int n, size_t lds,
                     int nt, hipStream_t s) {
  if (n <= 0) return;
  if (forward) {
    if (nt == 1024) {
      const int g = persistent_grid(k_zfwd_q<T, RP, 1024>, 1024, lds, n);
      k_zfwd_q<T, RP, 1024><<<g, 1024, lds, s>>>(jobs, items, n);
    } else {
      const int g = persistent_grid(k_zfwd_q<T, RP, 512>, 512, lds, n);
      k_zfwd_q<T, RP, 512><<<g, 512, lds, s>>>(jobs, items, n);
    }
  } else {
    if (nt == 1024) {
      const int g = persistent_grid(k_zinv_q<T, RP, 1024>, 1024, lds, n);
      k_zinv_q<T, RP, 1024><<<g, 1024, lds, s>>>(jobs, items, n);
    } else {
      const int g = persistent_grid(k_zinv_q<T, RP, 512>, 512, lds, n);
      k_zinv_q<T, RP, 512><<<g, 512, lds, s>>>(jobs, items, n);
    }
  }
}

template <typename T>
void launch_xy_pass(const QJob* jobs, const QItem* items, int n, size_t lds, hipStream_t s) {
  if (n <= 0) return;
  const int g = persistent_grid(k_xy_q<T>, kXyQueueThreads, lds, n);
  k_xy_q<T><<<g, kXyQueueThreads, lds, s>>>(jobs, items, n);
}

template <typename T>
bool k_ok(int n, int k) {
  switch (n) {
#define ACE_CASE(NN)                                                           \
  case NN:                                                                     \
    return (k == 1 && (xy_k_fits<T, NN, 1>() || supported<T, NN>())) ||        \
           (k == 2 && xy_k_fits<T, NN, 2>()) || (k == 4 && xy_k_fits<T, NN, 4>());
    ACE_SIZES(ACE_CASE)
#undef ACE_CASE
  }
  return false;
}

template <typename T>
size_t xy_lds(int n, int k) {
  switch (n) {
#define ACE_CASE(NN)                                                                        \
  case NN:                                                                                  \
    return fits<T, NN>() ? lds_with_twiddles<T, 2 * NN>((size_t)k * 2 * NN * (2 * NN + 1)) \
                         : strip_lds<T, NN>();
    ACE_SIZES(ACE_CASE)
#undef ACE_CASE
  }
  return 0;
}

}  // namespace

bool queue_xy_k_ok(int n, bool fp64, int k) { return fp64 ? k_ok<double>(n, k) : k_ok<float>(n, k); }

size_t queue_xy_lds(int n, bool fp64, int k) { return fp64 ? xy_lds<double>(n, k) : xy_lds<float>(n, k); }

size_t queue_z_lds(int n, bool fp64) {
  const size_t p = 2 * (size_t)n, e = fp64 ? 16 : 8;
  return ((size_t)n * (p + 1) * e + 15) / 16 * 16 + p * 16;
}

int launch_zfwd_queue(bool fp64, bool rp, const QJob* jobs, const QItem* zitems, int nz,
                      size_t lds_z, int nt, hipStream_t s) {
  if (lds_z > kMaxLds) return -1;
  if (fp64)
    rp ? launch_z_passes<double, true>(true, jobs, zitems, nz, lds_z, nt, s)
       : launch_z_passes<double, false>(true, jobs, zitems, nz, lds_z, nt, s);
  else
    rp ? launch_z_passes<float, true>(true, jobs, zitems, nz, lds_z, nt, s)
       : launch_z_passes<float, false>(true, jobs, zitems, nz, lds_z, nt, s);
  return 0;
}

int launch_z_edge(bool forward, int n, bool fp64, bool rp, const QJob* jobs, int count,
                  hipStream_t s) {
  if (count <= 0) return 0;
  return fp64 ? z_edge_any<double>(forward, n, rp, jobs, count, s)
              : z_edge_any<float>(forward, n, rp, jobs, count, s);
}

int launch_xy_queue(bool fp64, const QJob* jobs, const QItem* xyitems, int nxy, size_t lds_xy,
                    hipStream_t s) {
  if (lds_xy > kMaxLds) return -1;
  if (fp64)
    launch_xy_pass<double>(jobs, xyitems, nxy, lds_xy, s);
  else
    launch_xy_pass<float>(jobs, xyitems, nxy, lds_xy, s);
  return 0;
}

int launch_zinv_queue(bool fp64, bool rp, const QJob* jobs, const QItem* zitems, int nz,
                      size_t lds_z, int nt, hipStream_t s) {
  if (lds_z > kMaxLds) return -1;
  if (fp64)
    rp ? launch_z_passes<double, true>(false, jobs, zitems, nz, lds_z, nt, s)
       : launch_z_passes<double, false>(false, jobs, zitems, nz, lds_z, nt, s);
  else
    rp ? launch_z_passes<float, true>(false, jobs, zitems, nz, lds_z, nt, s)
       : launch_z_passes<float, false>(false, jobs, zitems, nz, lds_z, nt, s);
  return 0;
}

int launch_pair_queue(bool fp64, bool rp, const QJob* jobs, const QItem* zitems, int nz,
                      const QItem* xyitems, int nxy, size_t lds_z, size_t lds_xy, QShape sh,
                      hipStream_t s, Trace* tr) {
  int rc = 0;
  {
    TraceScope ts(tr, TR_ZFWD);
    rc |= launch_zfwd_queue(fp64, rp, jobs, zitems, nz, lds_z, sh.zf_nt, s);
  }
  {
    TraceScope ts(tr, TR_XY);
    rc |= launch_xy_queue(fp64, jobs, xyitems, nxy, lds_xy, s);
  }
  {
    TraceScope ts(tr, TR_ZINV);
    rc |= launch_zinv_queue(fp64, rp, jobs, zitems, nz, lds_z, sh.zi_nt, s);
  }
  return rc || hipGetLastError() != hipSuccess ? -1 : 0;
}

}  // namespace ace
