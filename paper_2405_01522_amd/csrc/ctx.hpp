// Host-side state shared by the C ABI translation units: the context object, device buffers,
// the launch tracer and the pair-solve launch sequence.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/ace.h"
#include "internal.hpp"

namespace ace {
namespace host {

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

inline size_t elem_bytes(int dt) {
  switch (dt) {
    case ACE_C128: return 16;
    case ACE_C64: return 8;
    case ACE_R64: return 8;
    case ACE_R32: return 4;
  }
  return 0;
}
inline bool is_fp64(int dt) { return dt == ACE_C128 || dt == ACE_R64; }
inline bool is_cplx(int dt) { return dt == ACE_C128 || dt == ACE_C64; }
inline int max_orbitals(int dt) { return is_cplx(dt) ? ACE_MAX_ORBITALS_COMPLEX : ACE_MAX_ORBITALS; }

struct Blob {
  Buf dev;
  std::vector<unsigned char> cache;
  unsigned char* pinned = nullptr;
  size_t pinned_cap = 0;
};

inline int ensure_on(hipStream_t s, Buf& b, size_t bytes) {
  if (bytes <= b.cap) return ACE_OK;
  if (b.p) {
    if (hipStreamSynchronize(s) != hipSuccess) return ACE_ERR_HIP;
    (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
  }
  size_t want = bytes + bytes / 8;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return ACE_ERR_OOM;
  }
  b.cap = want;
  return ACE_OK;
}

// Copy host bytes to the blob's device buffer on stream s, unless identical to the last upload.
inline int upload_blob(hipStream_t s, Blob& b, const void* host, size_t bytes) {
  if (b.cache.size() == bytes && std::memcmp(b.cache.data(), host, bytes) == 0) return ACE_OK;
  int rc = ensure_on(s, b.dev, bytes);
  if (rc) return rc;
  if (hipStreamSynchronize(s) != hipSuccess) return ACE_ERR_HIP;  // staging may be in flight
  if (b.pinned_cap < bytes) {
    if (b.pinned) (void)hipHostFree(b.pinned);
    b.pinned = nullptr;
    b.pinned_cap = 0;
    if (hipHostMalloc((void**)&b.pinned, bytes) != hipSuccess) return ACE_ERR_OOM;
    b.pinned_cap = bytes;
  }
  std::memcpy(b.pinned, host, bytes);
  if (hipMemcpyAsync(b.dev.p, b.pinned, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
    return ACE_ERR_HIP;
  b.cache.assign((const unsigned char*)host, (const unsigned char*)host + bytes);
  return ACE_OK;
}

inline void free_blob(Blob& b) {
  if (b.dev.p) (void)hipFree(b.dev.p);
  if (b.pinned) (void)hipHostFree(b.pinned);
  b = Blob();
}

inline int hip_check(hipError_t e) { return e == hipSuccess ? ACE_OK : ACE_ERR_HIP; }

struct DevBuf {
  double* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  int alloc(size_t n) {
    if (hipMalloc(&p, n * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return ACE_ERR_OOM;
    }
    return ACE_OK;
  }
};

}  // namespace host
}  // namespace ace

// Event tracer: one event pair per traced launch group, pooled events, totals per kernel class.
struct ace::Trace {
  bool on = false;
  hipStream_t stream = nullptr;
  struct Rec {
    int id;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  double total_ms[ace::TR_COUNT] = {};
  long long count[ace::TR_COUNT] = {};
  int depth = 0;

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  int collect() {
    if (pending.empty()) return ACE_OK;
    if (hipStreamSynchronize(stream) != hipSuccess) return ACE_ERR_HIP;
    for (Rec& r : pending) {
      float ms = 0.f;
      if (r.a && r.b && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        total_ms[r.id] += ms;
        count[r.id] += 1;
      }
      if (r.a) pool.push_back(r.a);
      if (r.b) pool.push_back(r.b);
    }
    pending.clear();
    return ACE_OK;
  }
  void release() {
    (void)hipStreamSynchronize(stream);
    for (Rec& r : pending) {
      if (r.a) pool.push_back(r.a);
      if (r.b) pool.push_back(r.b);
    }
    pending.clear();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
  }
};

struct ace_ctx {
  int n = 0, dtype = 0;
  double h = 0;
  size_t ng = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  double* ghat64 = nullptr;
  float* ghat32 = nullptr;
  void* gpos = nullptr;      // kernel spectrum in FFT position order, compute precision
  void* tw = nullptr;        // P twiddles exp(-2 pi i m / P) in the compute precision
  int* status = nullptr;     // device: [code, info]
  ace::host::Buf work, vbuf, wbuf, part, small, pairs, tda;
  // ace_build_apply: Gram partials of W^H psi (M's are in `part` at the same time) and the
  // reduced W^H psi dV
  ace::host::Buf part2, ybuf;
  ace::host::Blob tda_items;                // pair pointers of the TDA solves
  std::vector<int> pairs_cached;
  int* pinned_pairs = nullptr;
  size_t pinned_cap = 0;
  ace::Trace trace;
  ace::Trace* tr() {
    trace.stream = stream;
    return trace.on ? &trace : nullptr;
  }
};

namespace ace {
namespace host {


inline int ensure(ace_ctx* c, Buf& b, size_t bytes) {
  if (bytes <= b.cap) return ACE_OK;
  if (b.p) {
    if (hipStreamSynchronize(c->stream) != hipSuccess) return ACE_ERR_HIP;
    (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
  }
  size_t want = bytes + bytes / 8;
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return ACE_ERR_OOM;
  }
  b.cap = want;
  return ACE_OK;
}

// Upload a pair list to the context's device pair buffer (skipped if unchanged).
inline int upload_pairs(ace_ctx* c, const int* host, int count) {
  const size_t bytes = sizeof(int) * 2 * (size_t)count;
  if ((int)c->pairs_cached.size() == 2 * count &&
      std::memcmp(c->pairs_cached.data(), host, bytes) == 0)
    return ACE_OK;
  int rc = ensure(c, c->pairs, bytes);
  if (rc) return rc;
  // the pinned staging buffer may still feed an earlier copy: wait for the stream
  if (hipStreamSynchronize(c->stream) != hipSuccess) return ACE_ERR_HIP;
  if (c->pinned_cap < bytes) {
    if (c->pinned_pairs) (void)hipHostFree(c->pinned_pairs);
    c->pinned_pairs = nullptr;
    if (hipHostMalloc((void**)&c->pinned_pairs, bytes) != hipSuccess) {
      c->pinned_cap = 0;
      return ACE_ERR_OOM;
    }
    c->pinned_cap = bytes;
  }
  std::memcpy(c->pinned_pairs, host, bytes);
  if (hipMemcpyAsync(c->pairs.p, c->pinned_pairs, bytes, hipMemcpyHostToDevice, c->stream) !=
      hipSuccess)
    return ACE_ERR_HIP;
  c->pairs_cached.assign(host, host + 2 * count);
  return ACE_OK;
}

// Pair solves in batches bounded by the FFT workspace; pairs already on the device, indices
// into na orbitals of pa and nb of pb.
inline int run_pairs(ace_ctx* c, const void* pa, int na, const void* pb, int nb,
                     const int* pairs_dev, int np, void* vout) {
  const bool fp64 = is_fp64(c->dtype), rp = !is_cplx(c->dtype);
  const size_t per_item = poisson_work_bytes_per_item(c->n, fp64);
  const int items = rp ? (np + 1) / 2 : np;
  const size_t budget = size_t(1) << 30;  // 1 GiB of FFT volumes per launch sequence
  int batch = (int)std::max<size_t>(1, std::min<size_t>((size_t)items, budget / per_item));
  int rc = ensure(c, c->work, per_item * (size_t)batch);
  if (rc) return rc;
  const void* gh = c->gpos;
  const size_t eb = elem_bytes(c->dtype);
  for (int i0 = 0; i0 < items; i0 += batch) {
    const int ni = std::min(batch, items - i0);
    const int p0 = rp ? 2 * i0 : i0;
    const int npb = rp ? std::min(2 * ni, np - p0) : ni;
    launch_pair_poisson(c->n, fp64, rp, pa, na, pb, nb, pairs_dev + 2 * p0, npb, c->work.p,
                        (char*)vout + eb * c->ng * (size_t)p0, gh, c->tw, c->status, c->stream,
                        c->tr());
  }
  return hip_check(hipGetLastError());
}

// Complex transforms of launch_pair_slots (4 ints per transform, absolute output indices),
// in launches bounded like run_pairs.
inline int run_slots(ace_ctx* c, const void* phi, const int* slots_dev, int nslots, void* vout) {
  const bool fp64 = is_fp64(c->dtype);
  const size_t per_item = poisson_work_bytes_per_item(c->n, fp64);
  const size_t budget = size_t(1) << 30;
  int batch = (int)std::max<size_t>(1, std::min<size_t>((size_t)nslots, budget / per_item));
  int rc = ensure(c, c->work, per_item * (size_t)batch);
  if (rc) return rc;
  for (int i0 = 0; i0 < nslots; i0 += batch) {
    const int ni = std::min(batch, nslots - i0);
    launch_pair_slots(c->n, fp64, phi, slots_dev + 4 * (size_t)i0, ni, c->work.p, vout, c->gpos,
                      c->tw, c->stream, c->tr());
  }
  return hip_check(hipGetLastError());
}

}  // namespace host
}  // namespace ace
