// C ABI of libace: argument checking, workspace management and the launch sequences of the
// exchange / ACE / TDA calls.  Everything numerical happens in the kernels of poisson.hip,
// ace_kernels.hip and tda.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/ace.h"
#include "ace_kernels.hpp"
#include "common.hpp"
#include "internal.hpp"
#include "ctx.hpp"
#include "tda.hpp"

using namespace ace;
using namespace ace::host;

namespace {
constexpr double kC0 = 2.380077363979553;  // 3 ln(2 + sqrt 3) - pi/2

// Real pair solves of an explicit pointer list (two pairs per complex FFT), in batches bounded
// by the FFT workspace; the list goes to the device through the context's cached blob.
int solve_pair_list(ace_ctx* c, const std::vector<PairPtrs>& items) {
  const int np = (int)items.size();
  int rc = upload_blob(c->stream, c->tda_items, items.data(), sizeof(PairPtrs) * items.size());
  if (rc) return rc;
  const bool fp64 = is_fp64(c->dtype);
  const size_t per_item = poisson_work_bytes_per_item(c->n, fp64);
  const size_t nit = ((size_t)np + 1) / 2;
  const size_t batch = std::max<size_t>(1, std::min<size_t>(nit, (size_t(1) << 30) / per_item));
  rc = ensure(c, c->work, per_item * batch);
  if (rc) return rc;
  const PairPtrs* dev = (const PairPtrs*)c->tda_items.dev.p;
  for (size_t i0 = 0; i0 < nit; i0 += batch) {
    const size_t ni = std::min(batch, nit - i0);
    const size_t p0 = 2 * i0, npb = std::min(2 * ni, (size_t)np - p0);
    launch_pair_poisson_ptrs(c->n, fp64, true, dev + p0, (int)npb, c->work.p, c->gpos, c->tw,
                             c->stream, c->tr());
  }
  return hip_check(hipGetLastError());
}
}  // namespace

// ---------------------------------------------------------------------------------------
// Static scratch of ace_apply_noalloc: the Gram partial sums and the reduced xi^H psi block
// live in this array instead of a context workspace.  Host code never uses the symbol itself
// as an address; the per-device address comes from hipGetSymbolAddress once per device.
namespace {
constexpr size_t kNoallocScratch = ACE_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocScratch];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's copy of `scratch` (looked up once, with `dev` current).
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return ACE_ERR_INVALID;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return ACE_ERR_HIP;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return ACE_ERR_HIP;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return ACE_ERR_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ACE_OK;
}
}  // namespace

void ace::trace_begin(Trace* t, int id) {
  if (!t || !t->on) return;
  Trace::Rec r{id, t->get(), nullptr};
  if (r.a) (void)hipEventRecord(r.a, t->stream);
  t->pending.push_back(r);
}

void ace::trace_end(Trace* t, int id) {
  if (!t || !t->on) return;
  for (auto it = t->pending.rbegin(); it != t->pending.rend(); ++it)
    if (it->id == id && it->b == nullptr) {
      it->b = t->get();
      if (it->b) (void)hipEventRecord(it->b, t->stream);
      return;
    }
}



extern "C" {

int ace_size_supported(int n, int dtype) {
  if (dtype < ACE_C128 || dtype > ACE_R32) return 0;
  return poisson_size_supported(n, is_fp64(dtype)) ? 1 : 0;
}

int ace_ctx_create(int n, double h, int dtype, void* hip_stream, ace_ctx** out) {
  if (!out || !(h > 0.0) || !std::isfinite(h)) return ACE_ERR_INVALID;
  if (dtype < ACE_C128 || dtype > ACE_R32) return ACE_ERR_INVALID;
  *out = nullptr;
  if (!ace_size_supported(n, dtype)) return ACE_ERR_UNSUPPORTED;
  ace_ctx* c = new (std::nothrow) ace_ctx();
  if (!c) return ACE_ERR_OOM;
  c->n = n;
  c->h = h;
  c->dtype = dtype;
  c->ng = (size_t)n * n * n;
  c->stream = (hipStream_t)hip_stream;
  (void)hipGetDevice(&c->device);
  {
    // set-up of the no-allocation entry point's scratch on this device
    void* sp = nullptr;
    const int src = scratch_address(c->device, &sp);
    if (src) {
      ace_ctx_destroy(c);
      return src;
    }
  }
  const int p = 2 * n, ho = p / 2 + 1;
  const size_t oct = (size_t)ho * ho * ho;
  // cosine weights w(a) cos(2 pi k a / P) for the real-even kernel transform
  std::vector<double> cosw((size_t)ho * ho);
  for (int k = 0; k < ho; ++k)
    for (int a = 0; a < ho; ++a) {
      const double w = (a == 0 || a == p / 2) ? 1.0 : 2.0;
      cosw[(size_t)k * ho + a] = w * cossin_2pi((long long)k * a, p).c;
    }
  const bool fp64 = is_fp64(dtype);
  // table twiddles exp(-2 pi i m / P): FP64, or FP32 pairs of unit magnitude (unit_twiddle_f)
  std::vector<TwE<double>> tw64((size_t)p);
  std::vector<TwE<float>> tw32((size_t)p);
  for (int m = 0; m < p; ++m) {
    CosSin cs = cossin_2pi(m, p);
    tw64[m] = {cs.c, -cs.s};
    tw32[m] = unit_twiddle_f(cs.c, -cs.s);
  }
  static_assert(sizeof(TwE<double>) == 16 && sizeof(TwE<float>) == 8, "twiddle sizes");
  double *d_cos = nullptr, *t0 = nullptr, *t1 = nullptr;
  int rc = ACE_OK;
  if (hipMalloc(&c->ghat64, oct * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->ghat32, oct * sizeof(float)) != hipSuccess ||
      hipMalloc(&c->tw, 16 * (size_t)p) != hipSuccess ||
      hipMalloc(&c->gpos, (fp64 ? 8 : 4) * (size_t)p * p * p) != hipSuccess ||
      hipMalloc(&c->status, 4 * sizeof(int)) != hipSuccess ||
      hipMalloc(&d_cos, cosw.size() * sizeof(double)) != hipSuccess ||
      hipMalloc(&t0, oct * sizeof(double)) != hipSuccess ||
      hipMalloc(&t1, oct * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    rc = ACE_ERR_OOM;
  }
  if (!rc) {
    if (hipMemcpy(d_cos, cosw.data(), cosw.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->tw, fp64 ? (const void*)tw64.data() : (const void*)tw32.data(),
                  (fp64 ? sizeof(TwE<double>) : sizeof(TwE<float>)) * (size_t)p,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemsetAsync(c->status, 0, 4 * sizeof(int), c->stream) != hipSuccess)
      rc = ACE_ERR_HIP;
  }
  if (!rc) {
    launch_kernel_setup(n, h, kC0, d_cos, t0, t1, c->ghat64, c->ghat32, c->stream);
    launch_kernel_positions(n, fp64, c->ghat64, c->gpos, c->stream);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
      rc = ACE_ERR_HIP;
  }
  if (d_cos) (void)hipFree(d_cos);
  if (t0) (void)hipFree(t0);
  if (t1) (void)hipFree(t1);
  if (rc) {
    ace_ctx_destroy(c);
    return rc;
  }
  *out = c;
  return ACE_OK;
}

int ace_ctx_destroy(ace_ctx* c) {
  if (!c) return ACE_OK;
  (void)hipStreamSynchronize(c->stream);
  c->trace.stream = c->stream;
  c->trace.release();
  for (Buf* b : {&c->work, &c->vbuf, &c->wbuf, &c->part, &c->small, &c->pairs, &c->tda,
                 &c->part2, &c->ybuf})
    if (b->p) (void)hipFree(b->p);
  if (c->ghat64) (void)hipFree(c->ghat64);
  if (c->ghat32) (void)hipFree(c->ghat32);
  if (c->tw) (void)hipFree(c->tw);
  if (c->gpos) (void)hipFree(c->gpos);
  if (c->status) (void)hipFree(c->status);
  if (c->pinned_pairs) (void)hipHostFree(c->pinned_pairs);
  free_blob(c->tda_items);
  delete c;
  return ACE_OK;
}

int ace_ctx_set_stream(ace_ctx* c, void* s) {
  if (!c) return ACE_ERR_INVALID;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return ACE_ERR_HIP;
  c->trace.stream = c->stream;
  int rc = c->trace.collect();
  c->stream = (hipStream_t)s;
  return rc;
}

int pair_poisson_batched(ace_ctx* c, const void* phi_a, int na, const void* phi_b, int nb,
                         const int32_t* pairs, int np, void* v_out) {
  if (!c || !phi_a || !phi_b || !pairs || !v_out || na < 1 || nb < 1 || np < 1)
    return ACE_ERR_INVALID;
  for (int p = 0; p < np; ++p)
    if (pairs[2 * p] < 0 || pairs[2 * p] >= na || pairs[2 * p + 1] < 0 || pairs[2 * p + 1] >= nb)
      return ACE_ERR_INVALID;
  int rc = upload_pairs(c, pairs, np);
  if (rc) return rc;
  return run_pairs(c, phi_a, na, phi_b, nb, (const int*)c->pairs.p, np, v_out);
}

int pair_poisson_batched_dev(ace_ctx* c, const void* phi_a, int na, const void* phi_b, int nb,
                             const int32_t* pairs_dev, int np, void* v_out) {
  if (!c || !phi_a || !phi_b || !pairs_dev || !v_out || na < 1 || nb < 1 || np < 1)
    return ACE_ERR_INVALID;
  return run_pairs(c, phi_a, na, phi_b, nb, (const int*)pairs_dev, np, v_out);
}

}  // extern "C"

namespace {

// The pair solves of an ACE build (Eqs. (11), (2)) into c->vbuf, and the workspace of the
// steps after them (W in c->wbuf, Gram partials in c->part, M and L^{-H} in c->small).
int build_pairs(ace_ctx* c, const void* phi, int n) {
  const size_t eb = elem_bytes(c->dtype), ng = c->ng;
  const int np = n * (n + 1) / 2;
  const bool cplx = is_cplx(c->dtype);
  // real storage: the pair list in pair_index order (two real pairs per transform); complex
  // storage: 4-int transform slots (off-diagonal pairs, then the real diagonal densities two
  // per transform, orbitals 2m and 2m + 1 together)
  std::vector<int> pl;
  int nitems = np;
  if (!cplx) {
    pl.resize(2 * (size_t)np);
    for (int b = 0; b < n; ++b)
      for (int a = 0; a <= b; ++a) {
        const int p = b * (b + 1) / 2 + a;
        pl[2 * p] = a;
        pl[2 * p + 1] = b;
      }
  } else {
    for (int b = 0; b < n; ++b)
      for (int a = 0; a < b; ++a) pl.insert(pl.end(), {a, b, b * (b + 1) / 2 + a, -1});
    for (int a = 0; a < n; a += 2) {
      const int d0 = a * (a + 1) / 2 + a;
      if (a + 1 < n)
        pl.insert(pl.end(), {a, a + 1, d0, (a + 1) * (a + 2) / 2 + a + 1});
      else
        pl.insert(pl.end(), {a, a, d0, -2});
    }
    nitems = (int)(pl.size() / 4);
  }
  const size_t wide = cplx ? 16 : 8;
  size_t chunk;
  const int nblk = gram_blocks(ng, &chunk);
  // (upload_pairs counts 2-int records: a 4-int slot is two of them)
  int rc = upload_pairs(c, pl.data(), (int)(pl.size() / 2));
  if (!rc) rc = ensure(c, c->vbuf, eb * ng * (size_t)np);
  if (!rc) rc = ensure(c, c->wbuf, eb * ng * (size_t)n);
  if (!rc) rc = ensure(c, c->part, wide * (size_t)nblk * n * n);
  if (!rc) rc = ensure(c, c->small, wide * 2 * (size_t)n * n);
  if (rc) return rc;
  return cplx ? run_slots(c, phi, (const int*)c->pairs.p, nitems, c->vbuf.p)
              : run_pairs(c, phi, n, phi, n, (const int*)c->pairs.p, np, c->vbuf.p);
}

}  // namespace

extern "C" {

int ace_build(ace_ctx* c, const void* phi, int n, void* xi_out, double* M_out, double* ex_out) {
  if (!c || !phi || !xi_out || n < 1 || n > max_orbitals(c->dtype)) return ACE_ERR_INVALID;
  const size_t ng = c->ng, wide = is_cplx(c->dtype) ? 16 : 8;
  int rc = build_pairs(c, phi, n);
  if (rc) return rc;
  char* mred = (char*)c->small.p;
  char* linvh = mred + wide * (size_t)n * n;
  launch_wacc_gram(c->dtype, phi, c->vbuf.p, n, ng, c->wbuf.p, c->part.p, c->h * c->h * c->h,
                   mred, c->stream, c->tr());
  launch_chol_trsm(c->dtype, mred, n, M_out, ex_out, linvh, c->status, c->wbuf.p, ng, xi_out,
                   c->stream, c->tr());
  return hip_check(hipGetLastError());
}

int ace_build_apply(ace_ctx* c, const void* phi, int n, const void* psi, int nv, void* xi_out,
                    double* M_out, double* ex_out, void* kpsi_out) {
  if (!c || !phi || !psi || !xi_out || !kpsi_out || n < 1 || n > max_orbitals(c->dtype) ||
      nv < 1)
    return ACE_ERR_INVALID;
  const size_t eb = elem_bytes(c->dtype), ng = c->ng;
  const size_t wide = is_cplx(c->dtype) ? 16 : 8;
  const double dv = c->h * c->h * c->h;
  // vectors per Gram / update pass, as in ace_apply
  const int chunk_v = std::max(1, std::min(nv, 64));
  size_t chunk;
  const int nblk = gram_blocks(ng, &chunk);
  int rc = ensure(c, c->part2, wide * (size_t)nblk * n * chunk_v);
  if (!rc) rc = ensure(c, c->ybuf, wide * (size_t)n * nv);
  if (!rc) rc = build_pairs(c, phi, n);
  if (rc) return rc;
  char* mred = (char*)c->small.p;
  char* linvh = mred + wide * (size_t)n * n;
  char* y = (char*)c->ybuf.p;
  Trace* tr = c->tr();
  auto psi_at = [&](int v0) { return (const char*)psi + eb * ng * (size_t)v0; };
  const bool partials =
      launch_wacc_partials(c->dtype, phi, c->vbuf.p, n, ng, c->wbuf.p, c->part.p, c->stream, tr);
  // xi^H psi dV = L^{-1} Y with Y = W^H psi dV, so Y needs only W: for complex storage and
  // n <= 8 its Gram shares a launch with the reduction of M, and its reduction and L^{-1} one
  // with the Cholesky and xi (the first pass of vectors); otherwise the steps run one after
  // another and the update forms L^{-1} Y itself
  const int cv0 = std::min(chunk_v, nv);
  int first = 0;
  if (partials && launch_gram_y_reduce_m(c->dtype, c->wbuf.p, n, psi, cv0, ng, c->part2.p,
                                         c->part.p, dv, mred, c->stream, tr)) {
    launch_chol_trsm_zcol(c->dtype, mred, n, M_out, ex_out, linvh, c->status, c->wbuf.p, ng,
                          xi_out, c->part2.p, cv0, y, dv, c->stream, tr);
    launch_apply_out(c->dtype, xi_out, n, ng, y, cv0, kpsi_out, c->stream, tr);
    first = cv0;
  } else {
    launch_wacc_finish(c->dtype, partials, phi, n, ng, c->wbuf.p, c->part.p, dv, mred, c->stream,
                       tr);
    launch_chol_trsm(c->dtype, mred, n, M_out, ex_out, linvh, c->status, c->wbuf.p, ng, xi_out,
                     c->stream, tr);
  }
  for (int v0 = first; v0 < nv; v0 += chunk_v) {
    const int cv = std::min(chunk_v, nv - v0);
    launch_gram(c->dtype, c->wbuf.p, n, psi_at(v0), cv, ng, c->part2.p, dv,
                y + wide * (size_t)n * v0, c->stream, tr);
  }
  for (int v0 = first; v0 < nv; v0 += chunk_v) {
    const int cv = std::min(chunk_v, nv - v0);
    launch_apply_from_y(c->dtype, xi_out, n, ng, linvh, y + wide * (size_t)n * v0, cv,
                        (char*)kpsi_out + eb * ng * (size_t)v0, c->stream, tr);
  }
  return hip_check(hipGetLastError());
}

int ace_build_targets(ace_ctx* c, const void* phi_occ, int no, const void* psi, int nt,
                      void* xi_out, double* M_out) {
  if (!c || !phi_occ || !psi || !xi_out || no < 1 || nt < 1 || no > max_orbitals(c->dtype) ||
      nt > max_orbitals(c->dtype))
    return ACE_ERR_INVALID;
  const size_t eb = elem_bytes(c->dtype), ng = c->ng;
  const size_t wide = is_cplx(c->dtype) ? 16 : 8;
  size_t chunk;
  const int nblk = gram_blocks(ng, &chunk);
  int rc = ensure(c, c->wbuf, eb * ng * (size_t)nt);
  if (!rc) rc = ensure(c, c->part, wide * (size_t)nblk * nt * nt);
  if (!rc) rc = ensure(c, c->small, wide * 2 * (size_t)nt * nt);
  if (rc) return rc;
  // W_t = K[phi_occ] psi_t: one pair solve per (occupied, target) pair (Eq. (2))
  rc = exchange_apply_direct(c, phi_occ, no, psi, nt, c->wbuf.p);
  if (rc) return rc;
  char* mred = (char*)c->small.p;
  char* linvh = mred + wide * (size_t)nt * nt;
  launch_gram(c->dtype, psi, nt, c->wbuf.p, nt, ng, c->part.p, c->h * c->h * c->h, mred, c->stream,
              c->tr());
  launch_chol_trsm(c->dtype, mred, nt, M_out, nullptr, linvh, c->status, c->wbuf.p, ng, xi_out,
                   c->stream, c->tr());
  return hip_check(hipGetLastError());
}

int ace_apply(ace_ctx* c, const void* xi, int n, const void* psi, int nv, void* out) {
  if (!c || !xi || !psi || !out || n < 1 || n > max_orbitals(c->dtype) || nv < 1) return ACE_ERR_INVALID;
  const size_t eb = elem_bytes(c->dtype), ng = c->ng;
  const size_t wide = is_cplx(c->dtype) ? 16 : 8;
  // vectors per Gram / update pass (bounds the partial-sum workspace)
  const int chunk_v = std::max(1, std::min(nv, 64));
  size_t chunk;
  const int nblk = gram_blocks(ng, &chunk);
  int rc = ensure(c, c->part, wide * (size_t)nblk * n * chunk_v);
  if (!rc) rc = ensure(c, c->small, wide * (size_t)n * chunk_v + wide * 2 * 32 * 32);
  if (rc) return rc;
  for (int v0 = 0; v0 < nv; v0 += chunk_v) {
    const int cv = std::min(chunk_v, nv - v0);
    const char* ps = (const char*)psi + eb * ng * (size_t)v0;
    char* o = (char*)out + eb * ng * (size_t)v0;
    launch_gram(c->dtype, xi, n, ps, cv, ng, c->part.p, c->h * c->h * c->h, c->small.p, c->stream,
                c->tr());
    launch_apply_out(c->dtype, xi, n, ng, c->small.p, cv, o, c->stream, c->tr());
  }
  return hip_check(hipGetLastError());
}

int ace_apply_noalloc(ace_ctx* c, const void* xi, int n, const void* psi, int nv, void* out) {
  if (!c || !xi || !psi || !out || n < 1 || n > max_orbitals(c->dtype) || nv < 1)
    return ACE_ERR_INVALID;
  const size_t eb = elem_bytes(c->dtype), ng = c->ng;
  const size_t wide = is_cplx(c->dtype) ? 16 : 8;
  size_t chunk;
  const int nblk = gram_blocks(ng, &chunk);
  // per vector: nblk partial rows of n entries and the reduced column of Z (each part
  // 256-byte aligned); as many vectors per pass as the scratch holds, at most 64 as in
  // ace_apply (so both give the same passes and the same bits)
  const size_t per_vec = wide * (size_t)n * ((size_t)nblk + 1);
  const size_t room = kNoallocScratch - 512;
  if (per_vec > room) return ACE_ERR_SCRATCH;
  const int chunk_v = (int)std::min<size_t>({(size_t)nv, 64, room / per_vec});
  void* base = nullptr;
  int rc = scratch_address(c->device, &base);
  if (rc) return rc;
  char* part = (char*)base;
  const size_t part_bytes = (wide * (size_t)nblk * n * chunk_v + 255) / 256 * 256;
  char* z = part + part_bytes;
  for (int v0 = 0; v0 < nv; v0 += chunk_v) {
    const int cv = std::min(chunk_v, nv - v0);
    const char* ps = (const char*)psi + eb * ng * (size_t)v0;
    char* o = (char*)out + eb * ng * (size_t)v0;
    launch_gram(c->dtype, xi, n, ps, cv, ng, part, c->h * c->h * c->h, z, c->stream, nullptr);
    launch_apply_out(c->dtype, xi, n, ng, z, cv, o, c->stream, nullptr);
  }
  return hip_check(hipGetLastError());
}

int exchange_apply_direct(ace_ctx* c, const void* phi, int n, const void* psi, int nv, void* out) {
  if (!c || !phi || !psi || !out || n < 1 || n > max_orbitals(c->dtype) || nv < 1) return ACE_ERR_INVALID;
  const size_t eb = elem_bytes(c->dtype), ng = c->ng;
  // vectors in groups so that the pair volumes stay within about 1 GiB
  const size_t per_vec = eb * ng * (size_t)n;
  const int gv = (int)std::max<size_t>(1, std::min<size_t>((size_t)nv, (size_t(1) << 30) / per_vec));
  int rc = ensure(c, c->vbuf, per_vec * (size_t)gv);
  if (rc) return rc;
  for (int v0 = 0; v0 < nv; v0 += gv) {
    const int cv = std::min(gv, nv - v0);
    std::vector<int> pl(2 * (size_t)n * cv);
    for (int v = 0; v < cv; ++v)
      for (int j = 0; j < n; ++j) {
        pl[2 * ((size_t)v * n + j)] = j;
        pl[2 * ((size_t)v * n + j) + 1] = v;
      }
    rc = upload_pairs(c, pl.data(), n * cv);
    if (rc) return rc;
    const char* ps = (const char*)psi + eb * ng * (size_t)v0;
    rc = run_pairs(c, phi, n, ps, cv, (const int*)c->pairs.p, n * cv, c->vbuf.p);
    if (rc) return rc;
    launch_direct_acc(c->dtype, phi, n, c->vbuf.p, cv, ng, (char*)out + eb * ng * (size_t)v0,
                      c->stream, c->tr());
  }
  return hip_check(hipGetLastError());
}

int tda_coupling(ace_ctx* c, const void* phi_occ, int no, const void* phi_virt, int nv,
                 int delta_M, double* C_out) {
  return tdhf_coupling(c, phi_occ, no, phi_virt, nv, delta_M, C_out, nullptr);
}

int tdhf_coupling(ace_ctx* c, const void* phi_occ, int no, const void* phi_virt, int nv,
                  int delta_M, double* C_out, double* B_out) {
  if (!c || !phi_occ || !phi_virt || !C_out || no < 1 || nv < 1) return ACE_ERR_INVALID;
  if (delta_M != 0 && delta_M != 2) return ACE_ERR_INVALID;
  if (is_cplx(c->dtype)) return ACE_ERR_UNSUPPORTED;
  const size_t eb = elem_bytes(c->dtype), ng = c->ng;
  const int nov = no * nv, noo = no * (no + 1) / 2, np = nov + noo;
  const size_t vbytes = eb * ng * (size_t)np;
  int rc = ensure(c, c->vbuf, vbytes);
  if (rc) return rc;
  char* v_ov = (char*)c->vbuf.p;
  char* v_oo = v_ov + eb * ng * (size_t)nov;
  // one list of pair pointers: ov pairs (j, b) at row j*nv + b, then occupied pairs (a <= b)
  std::vector<PairPtrs> items((size_t)np);
  for (int j = 0; j < no; ++j)
    for (int b = 0; b < nv; ++b) {
      PairPtrs& t = items[(size_t)j * nv + b];
      t.a = (const char*)phi_occ + eb * ng * j;
      t.b = (const char*)phi_virt + eb * ng * b;
      t.v = v_ov + eb * ng * ((size_t)j * nv + b);
    }
  for (int b = 0; b < no; ++b)
    for (int a = 0; a <= b; ++a) {
      const size_t q = (size_t)b * (b + 1) / 2 + a;
      PairPtrs& t = items[nov + q];
      t.a = (const char*)phi_occ + eb * ng * a;
      t.b = (const char*)phi_occ + eb * ng * b;
      t.v = v_oo + eb * ng * q;
    }
  rc = solve_pair_list(c, items);
  if (rc) return rc;
  TdaWork tw;
  rc = ensure(c, c->tda, tda_workspace_bytes(no, nv, ng, is_fp64(c->dtype), &tw));
  if (rc) return rc;
  launch_tda(is_fp64(c->dtype), phi_occ, no, phi_virt, nv, v_ov, v_oo, ng, c->h * c->h * c->h,
             delta_M, c->tda.p, tw, C_out, B_out, c->stream, c->tr());
  return hip_check(hipGetLastError());
}

int uhf_coupling(ace_ctx* c, const void* occ_a, int no_a, const void* virt_a, int nv_a,
                 const void* occ_b, int no_b, const void* virt_b, int nv_b, double* C_out,
                 double* B_out) {
  if (!c || !occ_a || !virt_a || !occ_b || !virt_b || !C_out || no_a < 1 || nv_a < 1 ||
      no_b < 1 || nv_b < 1)
    return ACE_ERR_INVALID;
  if (is_cplx(c->dtype)) return ACE_ERR_UNSUPPORTED;
  const size_t eb = elem_bytes(c->dtype), ng = c->ng;
  UhfSpin sp[2] = {{occ_a, virt_a, no_a, nv_a, nullptr, nullptr},
                   {occ_b, virt_b, no_b, nv_b, nullptr, nullptr}};
  size_t nvol = 0;
  for (const UhfSpin& x : sp) nvol += (size_t)x.no * x.nv + (size_t)x.no * (x.no + 1) / 2;
  int rc = ensure(c, c->vbuf, eb * ng * nvol);
  if (rc) return rc;
  std::vector<PairPtrs> items;
  items.reserve(nvol);
  char* vp = (char*)c->vbuf.p;
  for (UhfSpin& x : sp) {
    x.v_ov = vp;
    for (int j = 0; j < x.no; ++j)
      for (int b = 0; b < x.nv; ++b) {
        items.push_back({(const char*)x.occ + eb * ng * j, (const char*)x.virt + eb * ng * b, vp});
        vp += eb * ng;
      }
    x.v_oo = vp;
    for (int b = 0; b < x.no; ++b)
      for (int a = 0; a <= b; ++a) {
        items.push_back({(const char*)x.occ + eb * ng * a, (const char*)x.occ + eb * ng * b, vp});
        vp += eb * ng;
      }
  }
  rc = solve_pair_list(c, items);
  if (rc) return rc;
  UhfWork uw;
  rc = ensure(c, c->tda, uhf_workspace_bytes(sp, ng, is_fp64(c->dtype), &uw));
  if (rc) return rc;
  launch_uhf(is_fp64(c->dtype), sp, ng, c->h * c->h * c->h, c->tda.p, uw, C_out, B_out, c->stream,
             c->tr());
  return hip_check(hipGetLastError());
}

int ace_ctx_status(ace_ctx* c, int* status, int* info) {
  if (!c || !status) return ACE_ERR_INVALID;
  int st[4] = {0, 0, 0, 0};
  if (hipStreamSynchronize(c->stream) != hipSuccess) return ACE_ERR_HIP;
  if (hipMemcpy(st, c->status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return ACE_ERR_HIP;
  if (hipMemset(c->status, 0, sizeof(st)) != hipSuccess) return ACE_ERR_HIP;
  *status = st[0];
  if (info) *info = st[1];
  return ACE_OK;
}

int ace_trace_enable(ace_ctx* c, int on) {
  if (!c) return ACE_ERR_INVALID;
  c->trace.stream = c->stream;
  int rc = c->trace.collect();
  c->trace.on = on != 0;
  return rc;
}

int ace_trace_read(ace_ctx* c, int id, double* total_ms, long long* count) {
  if (!c || id < 0 || id >= TR_COUNT || !total_ms) return ACE_ERR_INVALID;
  c->trace.stream = c->stream;
  int rc = c->trace.collect();
  *total_ms = c->trace.total_ms[id];
  if (count) *count = c->trace.count[id];
  return rc;
}

int ace_trace_reset(ace_ctx* c) {
  if (!c) return ACE_ERR_INVALID;
  c->trace.stream = c->stream;
  int rc = c->trace.collect();
  for (int i = 0; i < TR_COUNT; ++i) {
    c->trace.total_ms[i] = 0.0;
    c->trace.count[i] = 0;
  }
  return rc;
}

const char* ace_trace_name(int id) {
  static const char* names[TR_COUNT] = {"poisson_zfwd", "poisson_xy", "poisson_zinv", "w_accumulate",
                                        "gram", "cholesky", "xi_trsm", "apply_update",
                                        "direct_accumulate", "tda_gemm", "tda_reduce", "setup"};
  if (id < 0 || id >= TR_COUNT) return "";
  return names[id];
}

int ace_trace_count(void) { return TR_COUNT; }

const char* ace_strerror(int code) {
  switch (code) {
    case ACE_OK: return "ok";
    case ACE_ERR_INVALID: return "invalid argument";
    case ACE_ERR_UNSUPPORTED: return "unsupported box size or dtype";
    case ACE_ERR_HIP: return "HIP runtime error";
    case ACE_ERR_OOM: return "device out of memory";
    case ACE_ERR_NOT_POSDEF: return "-M is not positive definite";
    case ACE_ERR_NONFINITE: return "non-finite value in M";
    case ACE_ERR_SCRATCH: return "problem does not fit the static scratch of the no-allocation call";
  }
  return "unknown error";
}

}  // extern "C"


// ---------------------------------------------------------------------------------------
// Tamm-Dancoff excitations (Sec. 2: A X = omega X with A = diag(eps_a - eps_i) + C) by a
// block Davidson iteration on the device: subspace products and Rayleigh-Ritz with the small
// dense kernels of linalg.hip, diagonal (eps_a - eps_i - theta) correction, canonical
// orthonormalisation of each new block.  The host only steers (residual norms, block sizes).

#include "linalg.hpp"
#include "scf.hpp"

extern "C" {

int sym_eig_small(int n, const double* A, int lda, double* w, double* V, int ldv, void* stream) {
  if (n < 1 || n > kJacobiMax || !A || !w || !V || lda < n || ldv < n) return ACE_ERR_INVALID;
  launch_jacobi(n, A, lda, w, V, ldv, 60, 1e-15, (hipStream_t)stream);
  return hip_check(hipGetLastError());
}

int dense_gemm(int ta, int tb, int M, int N, int K, double alpha, const double* A, int lda,
               const double* B, int ldb, double beta, double* C, int ldc, void* stream) {
  if (M < 1 || N < 1 || K < 1 || !A || !B || !C) return ACE_ERR_INVALID;
  launch_dgemm(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, (hipStream_t)stream);
  return hip_check(hipGetLastError());
}

}  // extern "C"

namespace {

// Davidson for the k lowest eigenpairs of the dense symmetric n x n device matrix A:
// subspace products and Rayleigh-Ritz with the small dense kernels of linalg.hip, diagonal
// correction (theta - d_i)^{-1} with d (host) the diagonal of A, canonical orthonormalisation of
// each new block; the start vectors are the unit vectors of the k smallest d_i.
int davidson_core(ace_ctx* c, const double* Ain, const std::vector<double>& d, int n, int k,
                  double tol, int max_iter, double* omega_out, double* X_out, int* iterations) {
  hipStream_t s = c->stream;
  const int mmax = std::min(n, std::min(kJacobiMax, std::max(4 * k, 2 * k + 8)));
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return d[x] < d[y]; });
  std::vector<double> v0((size_t)k * n, 0.0);
  for (int j = 0; j < k; ++j) v0[(size_t)j * n + order[j]] = 1.0;
  DevBuf dd, V, AV, H, th, S, X, AX, R, T, G, nrm, Sm, lam, U, Y, sc;
  int rc = ACE_OK;
  for (auto pr : {std::make_pair(&dd, (size_t)n),
                  std::make_pair(&V, (size_t)mmax * n), std::make_pair(&AV, (size_t)mmax * n),
                  std::make_pair(&H, (size_t)mmax * mmax), std::make_pair(&th, (size_t)mmax),
                  std::make_pair(&S, (size_t)mmax * mmax), std::make_pair(&X, (size_t)k * n),
                  std::make_pair(&AX, (size_t)k * n), std::make_pair(&R, (size_t)k * n),
                  std::make_pair(&T, (size_t)k * n), std::make_pair(&G, (size_t)mmax * k),
                  std::make_pair(&nrm, (size_t)k), std::make_pair(&Sm, (size_t)k * k),
                  std::make_pair(&lam, (size_t)k), std::make_pair(&U, (size_t)k * k),
                  std::make_pair(&Y, (size_t)k * n), std::make_pair(&sc, (size_t)k)})
    if (!rc) rc = pr.first->alloc(pr.second);
  if (rc) return rc;
  if (hipMemcpyAsync(dd.p, d.data(), sizeof(double) * n, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(V.p, v0.data(), sizeof(double) * v0.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    return ACE_ERR_HIP;
  const double* Ap = Ain;
  launch_dgemm(0, 1, k, n, n, 1.0, V.p, n, Ap, n, 0.0, AV.p, n, s);
  int m = k, it = 0;
  bool done = false;
  std::vector<double> h_n(k), h_l(k);
  for (it = 1; it <= max_iter && !done; ++it) {
    launch_dgemm(0, 1, m, m, n, 1.0, V.p, n, AV.p, n, 0.0, H.p, m, s);
    launch_jacobi(m, H.p, m, th.p, S.p, m, 60, 1e-15, s);
    launch_dgemm(1, 0, k, n, m, 1.0, S.p, m, V.p, n, 0.0, X.p, n, s);
    launch_dgemm(1, 0, k, n, m, 1.0, S.p, m, AV.p, n, 0.0, AX.p, n, s);
    launch_residual(X.p, AX.p, th.p, n, k, R.p, nrm.p, s);
    if (hipMemcpyAsync(h_n.data(), nrm.p, sizeof(double) * k, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return ACE_ERR_HIP;
    double worst = 0.0;
    for (int j = 0; j < k; ++j) worst = std::max(worst, std::sqrt(h_n[j]));
    if (worst < tol) {
      done = true;
      break;
    }
    if (m + k > mmax) {  // restart from the current Ritz vectors
      if (hipMemcpyAsync(V.p, X.p, sizeof(double) * k * n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
          hipMemcpyAsync(AV.p, AX.p, sizeof(double) * k * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return ACE_ERR_HIP;
      m = k;
      continue;
    }
    launch_dav_precond(R.p, dd.p, th.p, n, k, T.p, s);
    for (int pass = 0; pass < 2; ++pass) {  // project out the subspace, twice
      launch_dgemm(0, 1, m, k, n, 1.0, V.p, n, T.p, n, 0.0, G.p, k, s);
      launch_dgemm(1, 0, k, n, m, -1.0, G.p, k, V.p, n, 1.0, T.p, n, s);
    }
    // canonical orthonormalisation of the new block: T T^T = U diag(l) U^T, Y = l^{-1/2} U^T T
    launch_dgemm(0, 1, k, k, n, 1.0, T.p, n, T.p, n, 0.0, Sm.p, k, s);
    launch_jacobi(k, Sm.p, k, lam.p, U.p, k, 60, 1e-15, s);
    if (hipMemcpyAsync(h_l.data(), lam.p, sizeof(double) * k, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return ACE_ERR_HIP;
    const double lmax = h_l[k - 1];
    std::vector<double> scale(k, 0.0);
    int first = k;
    for (int j = k - 1; j >= 0; --j)
      if (h_l[j] > 1e-12 * std::max(lmax, 1e-300) && h_l[j] > 1e-24) {
        scale[j] = 1.0 / std::sqrt(h_l[j]);
        first = j;
      }
    const int kk = k - first;
    if (kk == 0) break;  // no new direction: the subspace is exhausted
    launch_dgemm(1, 0, k, n, k, 1.0, U.p, k, T.p, n, 0.0, Y.p, n, s);
    if (hipMemcpyAsync(sc.p, scale.data(), sizeof(double) * k, hipMemcpyHostToDevice, s) != hipSuccess)
      return ACE_ERR_HIP;
    launch_scale_rows(Y.p, sc.p, n, k, s);
    if (hipMemcpyAsync(V.p + (size_t)m * n, Y.p + (size_t)first * n, sizeof(double) * kk * n,
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
      return ACE_ERR_HIP;
    launch_dgemm(0, 1, kk, n, n, 1.0, V.p + (size_t)m * n, n, Ap, n, 0.0, AV.p + (size_t)m * n, n, s);
    m += kk;
    if (hipStreamSynchronize(s) != hipSuccess) return ACE_ERR_HIP;  // host vectors reused
  }
  if (hipMemcpyAsync(omega_out, th.p, sizeof(double) * k, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return ACE_ERR_HIP;
  if (X_out && hipMemcpyAsync(X_out, X.p, sizeof(double) * k * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return ACE_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return ACE_ERR_HIP;
  if (iterations) *iterations = done ? it : -it;
  return hip_check(hipGetLastError());
}

}  // namespace

extern "C" {

int tda_excitations(ace_ctx* c, const double* C, const double* eps_occ, int no,
                    const double* eps_virt, int nv, int nstates, double tol, int max_iter,
                    double* omega_out, double* X_out, int* iterations) {
  if (!c || !C || !eps_occ || !eps_virt || !omega_out || no < 1 || nv < 1) return ACE_ERR_INVALID;
  std::vector<double> d((size_t)no * nv);
  for (int i = 0; i < no; ++i)
    for (int a = 0; a < nv; ++a) d[(size_t)i * nv + a] = eps_virt[a] - eps_occ[i];
  return tda_excitations_diag(c, C, d.data(), no * nv, nstates, tol, max_iter, omega_out, X_out,
                              iterations);
}

int tda_excitations_diag(ace_ctx* c, const double* C, const double* d, int n, int nstates,
                         double tol, int max_iter, double* omega_out, double* X_out,
                         int* iterations) {
  if (!c || !C || !d || !omega_out || n < 1) return ACE_ERR_INVALID;
  if (nstates < 1 || nstates > 16 || nstates > n || !(tol > 0.0) || max_iter < 1)
    return ACE_ERR_INVALID;
  DevBuf A, dd;
  int rc = A.alloc((size_t)n * n);
  if (!rc) rc = dd.alloc((size_t)n);
  if (rc) return rc;
  if (hipMemcpyAsync(dd.p, d, sizeof(double) * n, hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return ACE_ERR_HIP;
  launch_add_diag(C, dd.p, n, A.p, c->stream);
  std::vector<double> dv(d, d + n);
  return davidson_core(c, A.p, dv, n, nstates, tol, max_iter, omega_out, X_out, iterations);
}

int tdhf_excitations(ace_ctx* c, const double* C, const double* B, const double* d, int n,
                     int nstates, double tol, int max_iter, double* omega_out, double* XpY_out,
                     int* iterations) {
  if (!c || !C || !B || !d || !omega_out || n < 1) return ACE_ERR_INVALID;
  if (nstates < 1 || nstates > 16 || nstates > n || !(tol > 0.0) || max_iter < 1)
    return ACE_ERR_INVALID;
  hipStream_t s = c->stream;
  DevBuf P, M, T1, H, dd, Z, sc;
  int rc = ACE_OK;
  for (auto pr : {std::make_pair(&P, (size_t)n * n), std::make_pair(&M, (size_t)n * n),
                  std::make_pair(&T1, (size_t)n * n), std::make_pair(&H, (size_t)n * n),
                  std::make_pair(&dd, (size_t)n), std::make_pair(&Z, (size_t)nstates * n),
                  std::make_pair(&sc, (size_t)nstates)})
    if (!rc) rc = pr.first->alloc(pr.second);
  if (rc) return rc;
  int* info = c->status + 2;  // scratch word of the status area
  if (hipMemsetAsync(info, 0, sizeof(int), s) != hipSuccess ||
      hipMemcpyAsync(dd.p, d, sizeof(double) * n, hipMemcpyHostToDevice, s) != hipSuccess)
    return ACE_ERR_HIP;
  // (A + B)(X + Y) = omega (X - Y), (A - B)(X - Y) = omega (X + Y): with A - B = L L^T,
  // L^T (A + B) L z = omega^2 z, X + Y = L z / sqrt(omega)  (Hermitian half-size form, Sec. 2)
  launch_pm(C, B, dd.p, n, P.p, M.p, s);
  launch_potrf(M.p, n, n, info, s);
  launch_dgemm(1, 0, n, n, n, 1.0, M.p, n, P.p, n, 0.0, T1.p, n, s);
  launch_dgemm(0, 0, n, n, n, 1.0, T1.p, n, M.p, n, 0.0, H.p, n, s);
  std::vector<double> dh(n);
  int hinfo = 0;
  DevBuf hd;
  rc = hd.alloc((size_t)n);
  if (rc) return rc;
  launch_diag(H.p, n, n, hd.p, s);
  if (hipMemcpyAsync(dh.data(), hd.p, sizeof(double) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return ACE_ERR_HIP;
  if (hinfo) return ACE_ERR_NOT_POSDEF;  // A - B not positive definite: unstable reference
  rc = davidson_core(c, H.p, dh, n, nstates, tol, max_iter, omega_out, Z.p, iterations);
  if (rc) return rc;
  launch_sqrt_and_inv(omega_out, sc.p, nstates, s);
  if (XpY_out) {
    launch_dgemm(0, 1, nstates, n, n, 1.0, Z.p, n, M.p, n, 0.0, XpY_out, n, s);
    launch_scale_rows(XpY_out, sc.p, n, nstates, s);
  }
  if (hipStreamSynchronize(s) != hipSuccess) return ACE_ERR_HIP;  // scratch freed on return
  return hip_check(hipGetLastError());
}

int tda_oscillator_strengths(ace_ctx* c, const void* phi_occ, int no, const void* phi_virt, int nv,
                             const double* X, const double* omega, int nstates, double* f_out,
                             double* d_out) {
  if (!c || !phi_occ || !phi_virt || !X || !omega || !f_out || no < 1 || nv < 1 || nstates < 1)
    return ACE_ERR_INVALID;
  if (is_cplx(c->dtype)) return ACE_ERR_UNSUPPORTED;
  const int nov = no * nv;
  DevBuf D, dk;
  int rc = D.alloc((size_t)3 * nov);
  if (!rc) rc = dk.alloc((size_t)3 * nstates);
  if (rc) return rc;
  launch_dipoles(is_fp64(c->dtype), phi_occ, no, phi_virt, nv, c->n, c->h, D.p, c->stream);
  // d_k[c] = sum_ia X_k[ia] D[c][ia]
  launch_dgemm(0, 1, nstates, 3, nov, 1.0, X, nov, D.p, nov, 0.0, dk.p, 3, c->stream);
  launch_oscillator(omega, dk.p, nstates, f_out, c->stream);
  if (d_out && hipMemcpyAsync(d_out, dk.p, sizeof(double) * 3 * nstates, hipMemcpyDeviceToDevice,
                              c->stream) != hipSuccess)
    return ACE_ERR_HIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return ACE_ERR_HIP;  // scratch freed on return
  return hip_check(hipGetLastError());
}

int strength_function(const double* omega, const double* f, int nstates, double w0, double dw,
                      int nw, double gamma, double* S_out, void* stream) {
  if (!omega || !f || !S_out || nstates < 1 || nw < 1 || !(gamma > 0.0)) return ACE_ERR_INVALID;
  launch_strength(omega, f, nstates, w0, dw, nw, gamma, S_out, (hipStream_t)stream);
  return hip_check(hipGetLastError());
}

}  // extern "C"
