// Uneven batches: many independent systems (box edge, spacing and orbital count each their
// own) built by one call -- the ACE rebuild of Sec. 3.1 (Eqs. (11)-(12)) for many molecules at
// once.  Every pass is one launch over all systems of every edge:
//   * the three pair-Poisson passes are persistent launches over a list of items (transform
//     planes) of all systems, largest box edge first (poisson_queue.hip);
//   * W + the partials of M, the reduction of M, the Cholesky / E_x and xi = W L^{-H} are one
//     launch each over all systems (flat grids, ace_kernels.hip).
// The XY pass, the compute-bound one, runs either as one persistent launch over the planes of
// every edge (K planes per workgroup per edge, one 1024-thread workgroup per CU since the LDS
// is sized for the largest plane) or as one launch per box edge with the one-system kernel
// (its own occupancy and thread count per edge); a tuner times both on the first eager call
// for each (dtype, set of edges), together with the threads of the z passes, and keeps its
// choices in memory and, when ACE_TUNE_CACHE names a file, in that file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ace.h"
#include "ace_kernels.hpp"
#include "ctx.hpp"
#include "internal.hpp"

using namespace ace;
using namespace ace::host;

namespace {

// One distinct (edge, spacing): its kernel spectrum and twiddles live in a context.
struct BatchGrid {
  int n = 0;
  double h = 0;
  ace_ctx* ctx = nullptr;
};

// Launch shape of the passes for one (dtype, set of edges).
struct Tune {
  int k[65] = {};   // XY planes per item of the persistent XY launch, by box edge
  int nt[65] = {};  // threads of the per-edge XY launches, by box edge
  int per_edge = 0; // 1: XY as one launch per edge; 0: one persistent launch
  int zf_nt = 512, zi_nt = 512;  // threads of the persistent z passes; 0: one launch per edge
  std::string source = "default";
};

constexpr size_t kWorkBudget = size_t(12) << 30;  // FFT work volumes resident at once

// the tuning cache shared by all batches of the process
std::mutex g_tune_mu;
std::map<std::string, Tune> g_tune;
bool g_tune_loaded = false;

const char* cache_path() {
  const char* p = std::getenv("ACE_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

// cache file lines:  <key> xy=<edge>:<planes>:<threads>,... mode=<queue|edge> zf=<nt> zi=<nt>
// (zf / zi 0: the z pass as one launch per edge)
void load_cache_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[1024];
  while (std::fgets(line, sizeof(line), f)) {
    char key[512], xy[400], mode[16];
    int zf = 0, zi = 0;
    if (std::sscanf(line, "%511s xy=%399s mode=%15s zf=%d zi=%d", key, xy, mode, &zf, &zi) != 5)
      continue;
    Tune t;
    t.zf_nt = zf == 1024 || zf == 0 ? zf : 512;
    t.zi_nt = zi == 1024 || zi == 0 ? zi : 512;
    t.per_edge = std::strcmp(mode, "edge") == 0;
    for (char* tok = std::strtok(xy, ","); tok; tok = std::strtok(nullptr, ",")) {
      int n = 0, k = 0, nt = 0;
      if (std::sscanf(tok, "%d:%d:%d", &n, &k, &nt) == 3 && n > 0 && n <= 64 &&
          (k == 1 || k == 2 || k == 4) && (nt == 512 || nt == 1024)) {
        t.k[n] = k;
        t.nt[n] = nt;
      }
    }
    t.source = "cache";
    g_tune[key] = t;
  }
  std::fclose(f);
}

std::string tune_line(const std::string& key, const Tune& t, const std::vector<int>& edges) {
  std::string s = key + " xy=";
  for (size_t i = 0; i < edges.size(); ++i) {
    char b[48];
    const int e = edges[i];
    std::snprintf(b, sizeof(b), "%s%d:%d:%d", i ? "," : "", e, t.k[e] ? t.k[e] : 1,
                  t.nt[e] ? t.nt[e] : 1024);
    s += b;
  }
  char b[96];
  std::snprintf(b, sizeof(b), " mode=%s zf=%d zi=%d", t.per_edge ? "edge" : "queue", t.zf_nt,
                t.zi_nt);
  return s + b;
}

void store_cache_locked(const std::string& line) {
  const char* path = cache_path();
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s\n", line.c_str());
  std::fclose(f);
}

}  // namespace

struct ace_batch {
  int dtype = 0;
  hipStream_t stream = nullptr;
  std::vector<BatchGrid> grids;
  Buf work, vbuf, wbuf, part, mred, linvh, status;
  size_t status_n = 0;
  Blob desc;  // [QJob x njobs][QItem z][QItem xy][MolArgs x nmol][int bsys]
  std::string last_tuning;
  ace::Trace trace;
  ace::Trace* tr() {
    trace.stream = stream;
    return trace.on ? &trace : nullptr;
  }
};

namespace {

// XY planes per item for edge n: the tuned value if it is compiled and fits, else 1
int planes_for(const Tune& t, int n, bool fp64) {
  const int k = t.k[n] ? t.k[n] : 1;
  return queue_xy_k_ok(n, fp64, k) ? k : 1;
}

// Average milliseconds of reps calls of f (launches on stream s); synchronises.  -1 on error.
template <typename F>
double time_ms(hipStream_t s, int reps, F f) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0;
  }
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) f();
  (void)hipEventRecord(e1, s);
  float ms = -1.f;
  if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
    ms = -1.f;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms < 0 ? -1.0 : (double)ms / reps;
}

void build_items(const std::vector<QJob>& jobs, size_t j0, size_t j1, std::vector<QItem>& z,
                 std::vector<QItem>& xy) {
  for (size_t j = j0; j < j1; ++j) {
    const QJob& q = jobs[j];
    for (int x = 0; x < q.edge; ++x) z.push_back({(int)j, x});
    for (int qz = 0; qz < 2 * q.edge; qz += q.k) xy.push_back({(int)j, qz});
  }
}

size_t xy_lds_of(const std::vector<QJob>& jobs, size_t j0, size_t j1, bool fp64) {
  size_t m = 0;
  for (size_t j = j0; j < j1; ++j) m = std::max(m, queue_xy_lds(jobs[j].edge, fp64, jobs[j].k));
  return m;
}

size_t z_lds_of(const std::vector<QJob>& jobs, size_t j0, size_t j1, bool fp64) {
  size_t m = 0;
  for (size_t j = j0; j < j1; ++j) m = std::max(m, queue_z_lds(jobs[j].edge, fp64));
  return m;
}

}  // namespace

extern "C" {

int ace_batch_create(int dtype, void* hip_stream, ace_batch** out) {
  if (!out || dtype < ACE_C128 || dtype > ACE_R32) return ACE_ERR_INVALID;
  *out = nullptr;
  ace_batch* b = new (std::nothrow) ace_batch();
  if (!b) return ACE_ERR_OOM;
  b->dtype = dtype;
  b->stream = (hipStream_t)hip_stream;
  *out = b;
  return ACE_OK;
}

int ace_batch_destroy(ace_batch* b) {
  if (!b) return ACE_OK;
  (void)hipStreamSynchronize(b->stream);
  for (Buf* x : {&b->work, &b->vbuf, &b->wbuf, &b->part, &b->mred, &b->linvh, &b->status})
    if (x->p) (void)hipFree(x->p);
  free_blob(b->desc);
  for (BatchGrid& g : b->grids) ace_ctx_destroy(g.ctx);
  b->trace.stream = b->stream;
  b->trace.release();
  delete b;
  return ACE_OK;
}

int ace_batch_set_stream(ace_batch* b, void* s) {
  if (!b) return ACE_ERR_INVALID;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return ACE_ERR_HIP;
  b->trace.stream = b->stream;
  int rc = b->trace.collect();
  b->stream = (hipStream_t)s;
  return rc;
}

int ace_build_batched(ace_batch* b, const ace_mol* mols, int nmol) {
  if (!b || !mols || nmol < 1) return ACE_ERR_INVALID;
  const int dt = b->dtype;
  for (int m = 0; m < nmol; ++m) {
    const ace_mol& x = mols[m];
    if (!x.phi || !x.xi || x.norb < 1 || x.norb > max_orbitals(dt) || !(x.h > 0.0) ||
        !std::isfinite(x.h))
      return ACE_ERR_INVALID;
    if (!ace_size_supported(x.n, dt)) return ACE_ERR_UNSUPPORTED;
  }
  const bool fp64 = is_fp64(dt), cplx = is_cplx(dt), rp = !cplx;
  const size_t eb = elem_bytes(dt), wide = cplx ? 16 : 8;
  hipStream_t s = b->stream;
  // status words, one pair per system (cleared when grown; ace_batch_status clears after reads)
  if (b->status_n < (size_t)nmol) {
    if (ensure_on(s, b->status, sizeof(int) * 2 * (size_t)nmol)) return ACE_ERR_OOM;
    if (hipMemsetAsync(b->status.p, 0, sizeof(int) * 2 * (size_t)nmol, s) != hipSuccess)
      return ACE_ERR_HIP;
    b->status_n = nmol;
  }
  // kernel spectrum and twiddles per distinct (edge, spacing)
  std::vector<int> grid_of(nmol);
  std::vector<int> edges;
  for (int m = 0; m < nmol; ++m) {
    int gi = -1;
    for (size_t g = 0; g < b->grids.size(); ++g)
      if (b->grids[g].n == mols[m].n && b->grids[g].h == mols[m].h) gi = (int)g;
    if (gi < 0) {
      BatchGrid g;
      g.n = mols[m].n;
      g.h = mols[m].h;
      const int rc = ace_ctx_create(g.n, g.h, dt, s, &g.ctx);
      if (rc) return rc;
      b->grids.push_back(g);
      gi = (int)b->grids.size() - 1;
    }
    grid_of[m] = gi;
    if (std::find(edges.begin(), edges.end(), mols[m].n) == edges.end()) edges.push_back(mols[m].n);
  }
  std::sort(edges.begin(), edges.end());

  // sizes and offsets of every system's buffers
  std::vector<size_t> off_v(nmol), off_w(nmol), off_p(nmol), off_m(nmol);
  size_t tot_v = 0, tot_w = 0, tot_p = 0, tot_m = 0;
  int nmax = 0;
  long long nblk = 0;
  bool vec = true;
  for (int m = 0; m < nmol; ++m) {
    const size_t k = mols[m].norb, ng = (size_t)mols[m].n * mols[m].n * mols[m].n;
    const size_t blocks = (ng + 255) / 256;
    off_v[m] = tot_v; tot_v += eb * ng * (k * (k + 1) / 2);
    off_w[m] = tot_w; tot_w += eb * ng * k;
    off_p[m] = tot_p; tot_p += wide * blocks * k * k;
    off_m[m] = tot_m; tot_m += wide * k * k;
    nmax = std::max(nmax, (int)k);
    nblk += (long long)blocks;
    vec = vec && ng % 4 == 0;
  }
  if (nblk > (1LL << 31) - 1) return ACE_ERR_UNSUPPORTED;
  int rc = ensure_on(s, b->vbuf, tot_v);
  if (!rc) rc = ensure_on(s, b->wbuf, tot_w);
  if (!rc) rc = ensure_on(s, b->part, tot_p);
  if (!rc) rc = ensure_on(s, b->mred, tot_m);
  if (!rc) rc = ensure_on(s, b->linvh, tot_m);
  if (rc) return rc;

  // jobs (transforms) of every system; the same transforms as a one-system build
  std::vector<QJob> jobs;
  std::vector<MolArgs> ma(nmol);
  std::vector<int> bsys;
  bsys.reserve((size_t)nblk);
  int blk0 = 0;
  for (int m = 0; m < nmol; ++m) {
    const ace_mol& x = mols[m];
    const int k = x.norb;
    const size_t ng = (size_t)x.n * x.n * x.n;
    const BatchGrid& g = b->grids[grid_of[m]];
    MolArgs a{};
    a.phi = x.phi;
    a.v = (char*)b->vbuf.p + off_v[m];
    a.w = (char*)b->wbuf.p + off_w[m];
    a.xi = x.xi;
    a.part = (char*)b->part.p + off_p[m];
    a.mred = (char*)b->mred.p + off_m[m];
    a.linvh = (char*)b->linvh.p + off_m[m];
    a.m_out = x.M;
    a.ex_out = x.ex;
    a.status = (int*)b->status.p + 2 * m;
    a.n = k;
    a.blk0 = blk0;
    a.ng = ng;
    a.dv = x.h * x.h * x.h;
    ma[m] = a;
    const int blocks = (int)((ng + 255) / 256);
    for (int i = 0; i < blocks; ++i) bsys.push_back(m);
    blk0 += blocks;
    auto orb = [&](int j) { return (const char*)x.phi + eb * ng * j; };
    auto vol = [&](int j, int i) { return (char*)a.v + eb * ng * ((size_t)i * (i + 1) / 2 + j); };
    QJob base{};
    base.gpos = g.ctx->gpos;
    base.tw = g.ctx->tw;
    base.edge = x.n;
    base.k = 1;
    if (rp) {
      // pairs in pair-index order, two per transform
      std::vector<PairPtrs> pl((size_t)k * (k + 1) / 2);
      for (int q = 0; q < k; ++q)
        for (int p = 0; p <= q; ++p) pl[(size_t)q * (q + 1) / 2 + p] = {orb(p), orb(q), vol(p, q)};
      for (size_t i = 0; i < pl.size(); i += 2) {
        QJob j = base;
        j.p0 = pl[i];
        j.np = 1;
        if (i + 1 < pl.size()) {
          j.p1 = pl[i + 1];
          j.np = 2;
        }
        jobs.push_back(j);
      }
    } else {
      // off-diagonal pair densities, then the real diagonal densities two per transform
      for (int q = 0; q < k; ++q)
        for (int p = 0; p < q; ++p) {
          QJob j = base;
          j.p0 = {orb(p), orb(q), vol(p, q)};
          j.np = 1;
          jobs.push_back(j);
        }
      for (int d = 0; d < k; d += 2) {
        QJob j = base;
        j.p0.a = orb(d);
        j.p0.v = vol(d, d);
        if (d + 1 < k) {
          j.p0.b = orb(d + 1);
          j.p0.v2 = vol(d + 1, d + 1);
          j.p0.kind = 1;
        } else {
          j.p0.b = orb(d);
          j.p0.kind = 2;
        }
        j.np = 1;
        jobs.push_back(j);
      }
    }
  }
  // largest box edge first (the longest items start first; every workgroup's share mixes all)
  std::stable_sort(jobs.begin(), jobs.end(), [](const QJob& a, const QJob& c) {
    return a.edge != c.edge ? a.edge > c.edge : a.gpos < c.gpos;
  });

  // launch shape: tuned once per (dtype, edge set), from the cache when present
  std::string key = "dtype=" + std::to_string(dt) + ",edges=";
  for (size_t i = 0; i < edges.size(); ++i) key += (i ? "-" : "") + std::to_string(edges[i]);
  Tune tune;
  bool have = false;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    load_cache_locked();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      tune = it->second;
      have = true;
    }
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess) cap = hipStreamCaptureStatusNone;
  const bool may_tune = !have && cap == hipStreamCaptureStatusNone;

  // work volumes: per job N*N*P elements, in chunks of jobs within the budget
  auto work_bytes = [&](const QJob& j) { return poisson_work_bytes_per_item(j.edge, fp64); };
  std::vector<size_t> chunk_start{0};
  size_t cur = 0, max_chunk = 0;
  for (size_t j = 0; j < jobs.size(); ++j) {
    const size_t wbytes = work_bytes(jobs[j]);
    if (cur + wbytes > kWorkBudget && cur > 0) {
      chunk_start.push_back(j);
      max_chunk = std::max(max_chunk, cur);
      cur = 0;
    }
    jobs[j].work = (void*)cur;  // offset within the chunk, made a pointer below
    cur += wbytes;
  }
  max_chunk = std::max(max_chunk, cur);
  chunk_start.push_back(jobs.size());
  rc = ensure_on(s, b->work, max_chunk);
  if (rc) return rc;
  for (QJob& j : jobs) j.work = (char*)b->work.p + (size_t)j.work;

  auto set_k = [&](const Tune& t) {
    for (QJob& j : jobs) j.k = planes_for(t, j.edge, fp64);
  };
  // descriptors of the current shape: jobs, items per chunk, systems, block map
  std::vector<QItem> zi, xyi;
  std::vector<size_t> z_off, xy_off;
  auto upload = [&]() -> int {
    zi.clear();
    xyi.clear();
    z_off.assign(1, 0);
    xy_off.assign(1, 0);
    for (size_t c = 0; c + 1 < chunk_start.size(); ++c) {
      build_items(jobs, chunk_start[c], chunk_start[c + 1], zi, xyi);
      z_off.push_back(zi.size());
      xy_off.push_back(xyi.size());
    }
    const size_t nb = sizeof(QJob) * jobs.size() + sizeof(QItem) * (zi.size() + xyi.size()) +
                      sizeof(MolArgs) * ma.size() + sizeof(int) * bsys.size();
    std::vector<unsigned char> blob(nb);
    unsigned char* q = blob.data();
    std::memcpy(q, jobs.data(), sizeof(QJob) * jobs.size());
    q += sizeof(QJob) * jobs.size();
    std::memcpy(q, zi.data(), sizeof(QItem) * zi.size());
    q += sizeof(QItem) * zi.size();
    std::memcpy(q, xyi.data(), sizeof(QItem) * xyi.size());
    q += sizeof(QItem) * xyi.size();
    std::memcpy(q, ma.data(), sizeof(MolArgs) * ma.size());
    q += sizeof(MolArgs) * ma.size();
    std::memcpy(q, bsys.data(), sizeof(int) * bsys.size());
    return upload_blob(s, b->desc, blob.data(), blob.size());
  };
  auto dev_jobs = [&]() { return (const QJob*)b->desc.dev.p; };
  auto dev_z = [&]() { return (const QItem*)(dev_jobs() + jobs.size()); };
  auto dev_xy = [&]() { return dev_z() + zi.size(); };
  auto dev_mols = [&]() { return (const MolArgs*)(dev_xy() + xyi.size()); };
  auto dev_bsys = [&]() { return (const int*)(dev_mols() + ma.size()); };
  // the XY pass of chunk c: one persistent launch, or one launch per run of jobs of one
  // (edge, spacing) with the one-system kernel
  auto xy_pass = [&](const Tune& t, size_t c) -> int {
    const size_t j0 = chunk_start[c], j1 = chunk_start[c + 1];
    if (!t.per_edge)
      return launch_xy_queue(fp64, dev_jobs(), dev_xy() + xy_off[c],
                             (int)(xy_off[c + 1] - xy_off[c]), xy_lds_of(jobs, j0, j1, fp64), s);
    for (size_t g0 = j0; g0 < j1;) {
      size_t g1 = g0;
      while (g1 < j1 && jobs[g1].edge == jobs[g0].edge && jobs[g1].gpos == jobs[g0].gpos) ++g1;
      const int e = jobs[g0].edge;
      if (launch_xy_edge(e, fp64, t.nt[e] ? t.nt[e] : 1024, jobs[g0].work, (int)(g1 - g0),
                         jobs[g0].gpos, jobs[g0].tw, s))
        return -1;
      g0 = g1;
    }
    return 0;
  };
  // a z pass of chunk c: the persistent launch with nt threads over its items, or (nt 0) one
  // launch per run of jobs of one edge
  auto z_pass = [&](bool forward, int nt, size_t c) -> int {
    const size_t j0 = chunk_start[c], j1 = chunk_start[c + 1];
    if (nt > 0) {
      const int nz = (int)(z_off[c + 1] - z_off[c]);
      const size_t lz = z_lds_of(jobs, j0, j1, fp64);
      return forward ? launch_zfwd_queue(fp64, rp, dev_jobs(), dev_z() + z_off[c], nz, lz, nt, s)
                     : launch_zinv_queue(fp64, rp, dev_jobs(), dev_z() + z_off[c], nz, lz, nt, s);
    }
    for (size_t g0 = j0; g0 < j1;) {
      size_t g1 = g0;
      while (g1 < j1 && jobs[g1].edge == jobs[g0].edge) ++g1;
      if (launch_z_edge(forward, jobs[g0].edge, fp64, rp, dev_jobs() + g0, (int)(g1 - g0), s))
        return -1;
      g0 = g1;
    }
    return 0;
  };
  auto run_passes = [&](const Tune& t, ace::Trace* trp) -> int {
    for (size_t c = 0; c + 1 < chunk_start.size(); ++c) {
      int r = 0;
      {
        TraceScope ts(trp, TR_ZFWD);
        r |= z_pass(true, t.zf_nt, c);
      }
      {
        TraceScope ts(trp, TR_XY);
        r |= xy_pass(t, c);
      }
      {
        TraceScope ts(trp, TR_ZINV);
        r |= z_pass(false, t.zi_nt, c);
      }
      if (r) return ACE_ERR_UNSUPPORTED;
    }
    return ACE_OK;
  };

  if (may_tune) {
    // Tuner.  XY: the persistent launch with K planes per item, edge by edge (largest first);
    // the per-edge launches with 512 or 1024 threads, edge by edge; each candidate timed over
    // the whole XY pass of this batch, the faster form kept.  Then the threads of the z
    // passes.  The z-forward pass is re-run before every XY timing (the XY pass works in
    // place).
    tune = Tune();
    tune.source = "tuned";
    for (int e : edges) {
      tune.k[e] = 1;
      tune.nt[e] = 1024;
    }
    auto time_xy = [&](const Tune& t) -> double {
      set_k(t);
      if (upload()) return -1.0;
      double tot = 0.0;
      for (size_t c = 0; c + 1 < chunk_start.size(); ++c) {
        if (z_pass(true, t.zf_nt, c)) return -1.0;
        const double ms = time_ms(s, 2, [&]() { (void)xy_pass(t, c); });
        if (ms < 0) return -1.0;
        tot += ms;
      }
      return tot;
    };
    Tune tq = tune;
    double best_q = time_xy(tq);
    for (auto e = edges.rbegin(); e != edges.rend(); ++e)
      for (int k : {2, 4}) {
        if (!queue_xy_k_ok(*e, fp64, k)) continue;
        Tune t = tq;
        t.k[*e] = k;
        const double ms = time_xy(t);
        if (ms >= 0 && (best_q < 0 || ms < best_q)) {
          best_q = ms;
          tq = t;
        }
      }
    Tune te = tq;
    te.per_edge = 1;
    double best_e = time_xy(te);
    for (auto e = edges.rbegin(); e != edges.rend(); ++e) {
      Tune t = te;
      t.nt[*e] = 512;
      const double ms = time_xy(t);
      if (ms >= 0 && (best_e < 0 || ms < best_e)) {
        best_e = ms;
        te = t;
      }
    }
    tune = (best_e >= 0 && (best_q < 0 || best_e < best_q)) ? te : tq;
    set_k(tune);
    if (upload()) return ACE_ERR_HIP;
    // z passes: persistent with 512 or 1024 threads, or one launch per edge; timed over the
    // whole pass (both passes are idempotent)
    for (int pass = 0; pass < 2; ++pass) {
      double tbest = -1.0;
      int nbest = 512;
      for (int nt : {512, 1024, 0}) {
        const double ms = time_ms(s, 2, [&]() {
          for (size_t c = 0; c + 1 < chunk_start.size(); ++c) (void)z_pass(pass == 0, nt, c);
        });
        if (ms >= 0 && (tbest < 0 || ms < tbest)) {
          tbest = ms;
          nbest = nt;
        }
      }
      (pass == 0 ? tune.zf_nt : tune.zi_nt) = nbest;
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[key] = tune;
    store_cache_locked(tune_line(key, tune, edges));
  } else {
    set_k(tune);
    rc = upload();
    if (rc) return rc;
  }
  b->last_tuning = tune_line(key, tune, edges) + " source=" + tune.source;

  ace::Trace* trp = b->tr();
  rc = run_passes(tune, trp);
  if (rc) return rc;
  launch_ace_steps_flat(dt, dev_mols(), dev_bsys(), nmol, vec ? (int)nblk : -(int)nblk, nmax, s,
                        trp);
  return hip_check(hipGetLastError());
}

int ace_batch_tuning(ace_batch* b, char* buf, int len) {
  if (!b || !buf || len < 1) return ACE_ERR_INVALID;
  std::snprintf(buf, (size_t)len, "%s", b->last_tuning.c_str());
  return ACE_OK;
}

int ace_batch_status(ace_batch* b, int* status, int* mol, int* info) {
  if (!b || !status) return ACE_ERR_INVALID;
  *status = 0;
  if (mol) *mol = -1;
  if (info) *info = 0;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return ACE_ERR_HIP;
  if (!b->status_n) return ACE_OK;
  std::vector<int> st(2 * b->status_n);
  if (hipMemcpy(st.data(), b->status.p, sizeof(int) * st.size(), hipMemcpyDeviceToHost) != hipSuccess)
    return ACE_ERR_HIP;
  for (size_t m = 0; m < b->status_n; ++m)
    if (st[2 * m]) {
      *status = st[2 * m];
      if (mol) *mol = (int)m;
      if (info) *info = st[2 * m + 1];
      break;
    }
  if (hipMemset(b->status.p, 0, sizeof(int) * st.size()) != hipSuccess) return ACE_ERR_HIP;
  return ACE_OK;
}

int ace_batch_trace_enable(ace_batch* b, int on) {
  if (!b) return ACE_ERR_INVALID;
  b->trace.stream = b->stream;
  int rc = b->trace.collect();
  b->trace.on = on != 0;
  return rc;
}

int ace_batch_trace_read(ace_batch* b, int id, double* total_ms, long long* count) {
  if (!b || id < 0 || id >= TR_COUNT || !total_ms) return ACE_ERR_INVALID;
  b->trace.stream = b->stream;
  int rc = b->trace.collect();
  *total_ms = b->trace.total_ms[id];
  if (count) *count = b->trace.count[id];
  return rc;
}

}  // extern "C"
