// Closed-shell Hartree-Fock ground state on the device: the SCF cycle of the paper (Eq. (1),
// ACE rebuilt from the current orbitals every iteration as in Sec. 3.1, linear mixing of the
// states, Eq. (14), and the relative density error stop test, Eq. (15)) around a block
// eigensolver (LOBPCG: Rayleigh-Ritz over the current vectors, their preconditioned
// residuals and the previous search directions) whose preconditioner is either the kinetic
// one (damped Jacobi on T + shift) or the learned convolutional network of convnet.hip.
// Grid work runs in the kernels of scf.hip, ace_kernels.hip and poisson.hip; the small dense
// steps (Gram matrices, canonical orthonormalisation, Jacobi eigensolver) run on the device
// in FP64.  The host only steers: residual norms and the density error are read once per
// eigensolver step / SCF iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "../../include/ace.h"
#include "ace_kernels.hpp"
#include "ctx.hpp"
#include "linalg.hpp"
#include "scf.hpp"

namespace ace {
int convnet_apply_internal(ace_convnet* net, int n, const float* x, int nb, float* y,
                           hipStream_t s);
}

using namespace ace;
using namespace ace::host;

namespace {

struct Mem {
  void* p = nullptr;
  Mem() = default;
  Mem(const Mem&) = delete;
  Mem& operator=(const Mem&) = delete;
  ~Mem() {
    if (p) (void)hipFree(p);
  }
  int alloc(size_t bytes) {
    if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return ACE_ERR_OOM;
    }
    return ACE_OK;
  }
  double* d() const { return (double*)p; }
  float* f() const { return (float*)p; }
};

bool real_ctx(const ace_ctx* c) { return c->dtype == ACE_R64 || c->dtype == ACE_R32; }

struct Recorder {
  float* in = nullptr;
  float* tgt = nullptr;
  int cap = 0;
  int count = 0;
  int stride = 1;
  long long tick = 0;  // residual evaluations seen
};

// steps between explicit recomputations of F V in the FP32 block eigensolver
constexpr int kRefresh = 10;

// Workspace and steps of the block eigensolver for k vectors.
struct Eig {
  ace_ctx* c = nullptr;
  bool fp64 = false;
  size_t ng = 0, eb = 0;
  int n = 0, k = 0, mmax = 0, nw = 1;
  int kconv = 0;  // the lowest kconv Ritz pairs decide convergence (0: all k)
  double h = 0, dv = 0;
  hipStream_t s = nullptr;
  Mem V, HV, V2, HV2, R, tmp, nin, nout;
  Mem S, G, Ss, Gs, D, ws, U, T, TG, A, th, Y, Cm, Gr, rd, scale, part, zl, cholok;
  const void* lock = nullptr;  // converged vectors the search space is kept orthogonal to
  int nlock = 0;
  std::vector<double> h_rd;

  int init(ace_ctx* c_, int k_, bool want_net, int nlock_ = 0) {
    c = c_;
    k = k_;
    fp64 = c->dtype == ACE_R64;
    ng = c->ng;
    n = c->n;
    h = c->h;
    dv = h * h * h;
    eb = fp64 ? 8 : 4;
    s = c->stream;
    // basis blocks: X, one preconditioned-residual block per preconditioner (the learned
    // one is used beside the kinetic one, which stays as the fallback direction), and the
    // previous search directions P when the Rayleigh-Ritz order allows
    nw = want_net ? 2 : 1;
    const int lim = std::min(kCombineMax, kJacobiMax);
    if ((1 + nw) * k > lim) return ACE_ERR_UNSUPPORTED;
    mmax = (2 + nw) * k <= lim ? (2 + nw) * k : (1 + nw) * k;
    const size_t vec = eb * ng;
    int rc = ACE_OK;
    for (Mem* m : {&V, &HV, &V2, &HV2})
      if (!rc) rc = m->alloc(vec * mmax);
    for (Mem* m : {&R, &tmp})
      if (!rc) rc = m->alloc(vec * k);
    if (want_net) {
      if (!rc) rc = nin.alloc(sizeof(float) * ng * k);
      if (!rc) rc = nout.alloc(sizeof(float) * ng * k);
    }
    const size_t sq = sizeof(double) * kJacobiMax * kJacobiMax;
    for (Mem* m : {&S, &G, &Ss, &Gs, &U, &T, &TG, &A, &Y, &Cm})
      if (!rc) rc = m->alloc(sq);
    for (Mem* m : {&D, &ws, &th, &rd, &scale})
      if (!rc) rc = m->alloc(sizeof(double) * kJacobiMax);
    if (!rc) rc = Gr.alloc(sizeof(double) * k * k);
    if (!rc) rc = cholok.alloc(sizeof(int));
    size_t chunk;
    const int nblk = gram_blocks(ng, &chunk);
    nlock = nlock_;
    const size_t pw = std::max((size_t)mmax * mmax, (size_t)nlock * nw * k);
    if (!rc) rc = part.alloc(sizeof(double) * (size_t)nblk * pw);
    if (!rc && nlock) rc = zl.alloc(sizeof(double) * (size_t)nlock * nw * k);
    h_rd.assign(k, 0.0);
    return rc;
  }

  char* vec(const Mem& m, int j) const { return (char*)m.p + eb * ng * (size_t)j; }

  // Y <- Y - L (L^T Y dV) for the locked vectors L (dV-orthonormal eigenvectors of F)
  void deflate(void* Y, int nv) {
    if (!nlock) return;
    launch_gram(c->dtype, lock, nlock, Y, nv, ng, part.p, dv, zl.p, s, nullptr);
    launch_project_out(fp64, lock, nlock, zl.d(), nv, ng, Y, s);
  }

  void gram(const void* A_, int na, const void* B_, int nb, double scale_, double* out) {
    launch_gram(c->dtype, A_, na, B_, nb, ng, part.p, scale_, out, s, nullptr);
  }

  // out = F in for nv vectors: T + vloc (+ K_ACE when nxi > 0)
  int fock(const void* vloc, const void* xi, int nxi, const void* in, int nv, void* out) {
    if (nxi > 0) {
      int rc = ace_apply(c, xi, nxi, in, nv, out);
      if (rc) return rc;
      launch_fock_local(fp64, in, nv, n, h, vloc, 1, out, s);
    } else {
      launch_fock_local(fp64, in, nv, n, h, vloc, 0, out, s);
    }
    return ACE_OK;
  }

  // Rayleigh-Ritz over m basis vectors with Gram S and projected operator G (both in S, G):
  // scaled orthonormalisation, Ritz values in th (ascending), coefficients of the k lowest
  // Ritz vectors in Cm (m x k, row-major).  The orthonormalisation is by Cholesky when the
  // scaled Gram matrix is provably far from singular (its smallest eigenvalue above chol_min:
  // canonical orthonormalisation would drop nothing, so both span the same space and give the
  // same Ritz pairs); otherwise, decided on the device, by the canonical one (Jacobi
  // eigenvectors, directions below rel * max dropped).  The Cholesky form loses about
  // eps * cond(S) of orthonormality (cond(S) <= m / lambda_min, the diagonal being 1):
  // chol_min keeps that below 1e-9 for FP32 storage and below 2e-12 for FP64.
  void rr(int m) {
    const double rel = fp64 ? 1e-12 : 1e-6;
    // Jacobi off-diagonal tolerance: far below the rounding of the grid vectors
    const double jtol = fp64 ? 1e-14 : 1e-11;
    launch_sym_scale(S.d(), G.d(), m, Ss.d(), Gs.d(), D.d(), s);
    int* ok = (int*)cholok.p;
    const double chol_min = fp64 ? 1e-2 : std::max(m * rel, 1e-5);
    launch_chol_orth(m, Ss.d(), chol_min, T.d(), ws.d(), ok, s);
    launch_jacobi(m, Ss.d(), m, ws.d(), U.d(), m, 60, jtol, s, ok);
    launch_canon(ws.d(), U.d(), m, rel, T.d(), s, ok);
    launch_dgemm(1, 0, m, m, m, 1.0, T.d(), m, Gs.d(), m, 0.0, TG.d(), m, s);
    launch_dgemm(0, 0, m, m, m, 1.0, TG.d(), m, T.d(), m, 0.0, A.d(), m, s);
    launch_drop_diag(A.d(), m, ws.d(), rel, s);
    launch_jacobi(m, A.d(), m, th.d(), Y.d(), m, 60, jtol, s);
    launch_dgemm(0, 0, m, k, m, 1.0, T.d(), m, Y.d(), m, 0.0, Cm.d(), k, s);
    launch_scale_coeff_rows(Cm.d(), k, D.d(), m, k, s);
  }

  // preconditioned residual blocks from the k residuals in R (scale = their inverse RMS):
  // z[0:k] = kinetic (or plain copy), z[k:2k] = learned network when nw == 2
  int precondition(const ace_eig_opts* o, void* z) {
    if (o->precond == ACE_PRECOND_NONE)
      return hip_check(hipMemcpyAsync(z, R.p, eb * ng * k, hipMemcpyDeviceToDevice, s));
    launch_precond_kinetic(fp64, R.p, k, n, h, o->shift, o->sweeps, o->omega, z, tmp.p, s);
    if (o->precond != ACE_PRECOND_NET) return ACE_OK;
    void* zn = (char*)z + eb * ng * (size_t)k;
    launch_scale_to_f32(fp64, R.p, scale.d(), k, ng, nin.f(), s);
    float* y = fp64 ? nout.f() : (float*)zn;
    int rc = convnet_apply_internal(o->net, n, nin.f(), k, y, s);
    if (rc) return rc;
    if (fp64) launch_from_f32(true, nout.f(), ng * k, zn, s);
    return ACE_OK;
  }

  // residuals of the current Ritz pairs (V[0:k], th) into R; norms to h_rd (host, dV norm)
  int residuals(double* maxres) {
    launch_residual_grid(fp64, V.p, HV.p, th.d(), k, ng, R.p, s);
    gram(R.p, k, R.p, k, 1.0, Gr.d());
    launch_inv_rms(Gr.d(), k, k, (double)ng, scale.d(), s);
    launch_diag(Gr.d(), k, k, rd.d(), s);
    if (hipMemcpyAsync(h_rd.data(), rd.p, sizeof(double) * k, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return ACE_ERR_HIP;
    double worst = 0.0;
    const int kc = kconv > 0 ? std::min(kconv, k) : k;
    for (int j = 0; j < k; ++j) {
      h_rd[j] = std::sqrt(std::max(h_rd[j], 0.0) * dv);
      if (j < kc) worst = std::max(worst, h_rd[j]);
    }
    *maxres = worst;
    return ACE_OK;
  }

  // LOBPCG for the k lowest states of F from the vectors X (overwritten with the Ritz
  // vectors); Ritz values stay in th[0:k], residual norms in h_rd.
  int run(const void* vloc, const void* xi, int nxi, void* X, const ace_eig_opts* o,
          Recorder* rec, int* steps_out, double* maxres) {
    const size_t vb = eb * ng;
    int rc = hip_check(hipMemcpyAsync(V.p, X, vb * k, hipMemcpyDeviceToDevice, s));
    deflate(V.p, k);
    if (!rc) rc = fock(vloc, xi, nxi, V.p, k, HV.p);
    if (rc) return rc;
    // Rayleigh-Ritz on the starting block alone (orthonormalises it)
    gram(V.p, k, V.p, k, dv, S.d());
    gram(V.p, k, HV.p, k, dv, G.d());
    rr(k);
    launch_combine(fp64, V.p, k, ng, Cm.d(), k, k, V2.p, s);
    launch_combine(fp64, HV.p, k, ng, Cm.d(), k, k, HV2.p, s);
    std::swap(V.p, V2.p);
    std::swap(HV.p, HV2.p);
    bool haveP = false;
    int steps = 0;
    for (;;) {
      rc = residuals(maxres);
      if (rc) return rc;
      if (rec && rec->in && rec->count < rec->cap && (rec->tick++ % rec->stride) == 0) {
        const int nr = std::min(k, rec->cap - rec->count);
        launch_scale_to_f32(fp64, R.p, scale.d(), nr, ng, rec->in + (size_t)rec->count * ng, s);
        launch_scale_to_f32(fp64, V.p, scale.d(), nr, ng, rec->tgt + (size_t)rec->count * ng, s);
        rec->count += nr;
      }
      if (*maxres < o->tol || steps >= o->max_steps) break;
      rc = precondition(o, vec(V, k));
      deflate(vec(V, k), nw * k);
      if (!rc) rc = fock(vloc, xi, nxi, vec(V, k), nw * k, vec(HV, k));
      if (rc) return rc;
      const int pb = (1 + nw) * k;  // first vector of the P block
      const int m = (haveP && mmax > pb) ? mmax : pb;
      gram(V.p, m, V.p, m, dv, S.d());
      gram(V.p, m, HV.p, m, dv, G.d());
      rr(m);
      launch_combine(fp64, V.p, m, ng, Cm.d(), k, k, V2.p, s);
      launch_combine(fp64, HV.p, m, ng, Cm.d(), k, k, HV2.p, s);
      if (mmax > pb) {  // new search directions: the non-X part of the update
        launch_combine(fp64, vec(V, k), m - k, ng, Cm.d() + (size_t)k * k, k, k, vec(V2, pb), s);
        launch_combine(fp64, vec(HV, k), m - k, ng, Cm.d() + (size_t)k * k, k, k, vec(HV2, pb), s);
        haveP = true;
      }
      std::swap(V.p, V2.p);
      std::swap(HV.p, HV2.p);
      ++steps;
      // F V of the kept blocks is carried along by the same combinations as V.  In FP32
      // storage the two drift apart by rounding, step after step, until the computed
      // residuals stall near 1e-4 (64^3, h = 0.2); every kRefresh steps F V is recomputed.
      if (!fp64 && steps % kRefresh == 0) {
        rc = fock(vloc, xi, nxi, V.p, k, HV.p);
        if (!rc && haveP) rc = fock(vloc, xi, nxi, vec(V, pb), k, vec(HV, pb));
        if (rc) return rc;
      }
    }
    rc = hip_check(hipMemcpyAsync(X, V.p, vb * k, hipMemcpyDeviceToDevice, s));
    *steps_out = steps;
    return rc ? rc : hip_check(hipGetLastError());
  }
};

int check_eig_opts(const ace_ctx* c, const ace_eig_opts* o) {
  if (!o || o->max_steps < 0 || !(o->tol >= 0.0)) return ACE_ERR_INVALID;
  if (o->precond != ACE_PRECOND_NONE &&
      (o->sweeps < 1 || !(o->shift > -1e300) || !(o->omega > 0.0) || !(o->omega < 2.0)))
    return ACE_ERR_INVALID;
  if (o->precond == ACE_PRECOND_NET && !o->net) return ACE_ERR_INVALID;
  if (o->precond < ACE_PRECOND_NONE || o->precond > ACE_PRECOND_NET) return ACE_ERR_INVALID;
  (void)c;
  return ACE_OK;
}

int hartree(ace_ctx* c, const void* rho, const void* ones, void* vh) {
  const int pr[2] = {0, 0};
  int rc = upload_pairs(c, pr, 1);
  if (rc) return rc;
  return run_pairs(c, ones, 1, rho, 1, (const int*)c->pairs.p, 1, vh);
}

// energy terms of closed-shell orbitals (device scratch from the caller), host results
int energies(ace_ctx* c, Eig& e, const void* v_ext, const void* phi, int k, const void* ones,
             void* rho, void* vh, void* xi, double* out) {
  const bool fp64 = e.fp64;
  hipStream_t s = c->stream;
  Mem sm;
  int rc = sm.alloc(sizeof(double) * (k * k + 4));
  if (rc) return rc;
  double* kin = sm.d();
  double* ex = kin + k * k;
  launch_density(fp64, phi, k, c->ng, rho, s);
  rc = hartree(c, rho, ones, vh);
  if (rc) return rc;
  launch_fock_local(fp64, phi, k, c->n, c->h, nullptr, 0, e.R.p, s);  // T phi
  e.gram(phi, k, e.R.p, k, e.dv, kin);
  e.gram(rho, 1, v_ext, 1, e.dv, ex + 1);
  e.gram(rho, 1, vh, 1, e.dv, ex + 2);
  rc = ace_build(c, phi, k, xi, nullptr, ex);
  if (rc) return rc;
  std::vector<double> h(k * k + 4);
  if (hipMemcpyAsync(h.data(), sm.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return ACE_ERR_HIP;
  double ekin = 0.0;
  for (int i = 0; i < k; ++i) ekin += 2.0 * h[(size_t)i * k + i];
  const double eext = h[k * k + 1], eh = 0.5 * h[k * k + 2];
  const double exx = 2.0 * h[k * k];  // ACE's E_x counts one electron per orbital
  out[0] = ekin + eext + eh + exx;
  out[1] = ekin;
  out[2] = eext;
  out[3] = eh;
  out[4] = exx;
  int st = 0;
  rc = ace_ctx_status(c, &st, nullptr);
  if (rc) return rc;
  return st ? st : ACE_OK;
}

}  // namespace

extern "C" {

int fock_local_apply(ace_ctx* c, const void* v_local, const void* psi, int nv, int accumulate,
                     void* out) {
  if (!c || !psi || !out || nv < 1) return ACE_ERR_INVALID;
  if (!real_ctx(c)) return ACE_ERR_UNSUPPORTED;
  launch_fock_local(c->dtype == ACE_R64, psi, nv, c->n, c->h, v_local, accumulate ? 1 : 0, out,
                    c->stream);
  return hip_check(hipGetLastError());
}

int scf_density(ace_ctx* c, const void* phi, int k, void* rho) {
  if (!c || !phi || !rho || k < 1) return ACE_ERR_INVALID;
  if (!real_ctx(c)) return ACE_ERR_UNSUPPORTED;
  launch_density(c->dtype == ACE_R64, phi, k, c->ng, rho, c->stream);
  return hip_check(hipGetLastError());
}

int hartree_potential(ace_ctx* c, const void* rho, void* v_h) {
  if (!c || !rho || !v_h) return ACE_ERR_INVALID;
  if (!real_ctx(c)) return ACE_ERR_UNSUPPORTED;
  Mem ones;
  int rc = ones.alloc(elem_bytes(c->dtype) * c->ng);
  if (rc) return rc;
  launch_fill(c->dtype == ACE_R64, 1.0, c->ng, ones.p, c->stream);
  rc = hartree(c, rho, ones.p, v_h);
  if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) rc = ACE_ERR_HIP;  // before free
  return rc;
}

int kinetic_precondition(ace_ctx* c, const void* r, int nv, double shift, int sweeps,
                         double omega, void* z) {
  if (!c || !r || !z || nv < 1 || sweeps < 1 || !(omega > 0.0) || !(omega < 2.0))
    return ACE_ERR_INVALID;
  if (!real_ctx(c)) return ACE_ERR_UNSUPPORTED;
  Mem tmp;
  if (sweeps > 1) {
    int rc = tmp.alloc(elem_bytes(c->dtype) * c->ng * nv);
    if (rc) return rc;
  }
  launch_precond_kinetic(c->dtype == ACE_R64, r, nv, c->n, c->h, shift, sweeps, omega, z, tmp.p,
                         c->stream);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
    return ACE_ERR_HIP;
  return ACE_OK;
}

int fock_lowest_states(ace_ctx* c, const void* v_local, const void* xi, int nxi, void* phi,
                       int k, const ace_eig_opts* o, double* eigval, double* resnorm,
                       int* steps) {
  if (!c || !phi || k < 1 || k > ACE_MAX_ORBITALS || nxi < 0 || nxi > ACE_MAX_ORBITALS ||
      (nxi > 0 && !xi))
    return ACE_ERR_INVALID;
  if (!real_ctx(c)) return ACE_ERR_UNSUPPORTED;
  int rc = check_eig_opts(c, o);
  if (rc) return rc;
  Eig e;
  rc = e.init(c, k, o->precond == ACE_PRECOND_NET);
  if (rc) return rc;
  int st = 0;
  double maxres = 0.0;
  rc = e.run(v_local, xi, nxi, phi, o, nullptr, &st, &maxres);
  if (rc) return rc;
  std::vector<double> th(k);
  if (hipMemcpyAsync(th.data(), e.th.p, sizeof(double) * k, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return ACE_ERR_HIP;
  if (eigval) std::copy(th.begin(), th.end(), eigval);
  if (resnorm) std::copy(e.h_rd.begin(), e.h_rd.end(), resnorm);
  if (steps) *steps = st;
  return ACE_OK;
}

int unocc_states(ace_ctx* c, const void* v_local, const void* phi_occ, int no, void* psi, int nv,
                 int nconv, const ace_eig_opts* o, int max_outer, double* eigval,
                 double* resnorm, int* outer, int* steps) {
  if (!c || !v_local || !phi_occ || !psi || no < 1 || nv < 1 || max_outer < 1 ||
      no + nv > ACE_MAX_ORBITALS || nconv < 0 || nconv > nv)
    return ACE_ERR_INVALID;
  if (!real_ctx(c)) return ACE_ERR_UNSUPPORTED;
  int rc = check_eig_opts(c, o);
  if (rc) return rc;
  Eig e;
  rc = e.init(c, nv, o->precond == ACE_PRECOND_NET, no);
  if (rc) return rc;
  e.lock = phi_occ;
  e.kconv = nconv;
  const int nt = no + nv;
  const size_t vb = elem_bytes(c->dtype) * c->ng;
  hipStream_t s = c->stream;
  Mem targets, xi;
  if (!rc) rc = targets.alloc(vb * nt);
  if (!rc) rc = xi.alloc(vb * nt);
  if (rc) return rc;
  if (hipMemcpyAsync(targets.p, phi_occ, vb * no, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return ACE_ERR_HIP;
  // the unoccupied start vectors: orthogonal to the occupied ones
  e.deflate(psi, nv);
  int it = 0, total = 0;
  double maxres = 0.0;
  for (it = 0; it < max_outer; ++it) {
    // ACE over occupied + current unoccupied orbitals, then eigensolver steps with it
    if (hipMemcpyAsync((char*)targets.p + vb * no, psi, vb * nv, hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
      return ACE_ERR_HIP;
    rc = ace_build_targets(c, phi_occ, no, targets.p, nt, xi.p, nullptr);
    if (rc) return rc;
    int st = 0;
    rc = e.run(v_local, xi.p, nt, psi, o, nullptr, &st, &maxres);
    if (rc) return rc;
    total += st;
    int stc = 0;
    rc = ace_ctx_status(c, &stc, nullptr);
    if (rc) return rc;
    if (stc) return stc;
    // the first residual of a run is taken right after the rebuild, where K_ACE equals K on
    // the current vectors: no step taken means every residual of the true operator is small
    if (st == 0) {
      ++it;
      break;
    }
  }
  std::vector<double> th(nv);
  if (hipMemcpyAsync(th.data(), e.th.p, sizeof(double) * nv, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return ACE_ERR_HIP;
  if (eigval) std::copy(th.begin(), th.end(), eigval);
  if (resnorm) std::copy(e.h_rd.begin(), e.h_rd.end(), resnorm);
  if (outer) *outer = it;
  if (steps) *steps = total;
  return ACE_OK;
}

int scf_energies(ace_ctx* c, const void* v_ext, const void* phi, int k, double* energy) {
  if (!c || !v_ext || !phi || !energy || k < 1 || k > ACE_MAX_ORBITALS) return ACE_ERR_INVALID;
  if (!real_ctx(c)) return ACE_ERR_UNSUPPORTED;
  Eig e;
  int rc = e.init(c, k, false);
  Mem ones, rho, vh, xi;
  const size_t vb = elem_bytes(c->dtype) * c->ng;
  if (!rc) rc = ones.alloc(vb);
  if (!rc) rc = rho.alloc(vb);
  if (!rc) rc = vh.alloc(vb);
  if (!rc) rc = xi.alloc(vb * k);
  if (rc) return rc;
  launch_fill(e.fp64, 1.0, c->ng, ones.p, c->stream);
  return energies(c, e, v_ext, phi, k, ones.p, rho.p, vh.p, xi.p, energy);
}

// residual target of the continued inner solve, relative to the density error (Eq. (15))
#ifndef ACE_SCF_INEXACT
#define ACE_SCF_INEXACT 10.0
#endif
constexpr double kInexact = ACE_SCF_INEXACT;

int scf_run(ace_ctx* c, const void* v_ext, void* phi, int k, const ace_scf_opts* o,
            ace_scf_result* res, double* eigval, double* err_hist) {
  if (!c || !v_ext || !phi || !o || !res || k < 1 || k > ACE_MAX_ORBITALS) return ACE_ERR_INVALID;
  if (!real_ctx(c)) return ACE_ERR_UNSUPPORTED;
  if (!(o->alpha >= 0.0) || !(o->alpha < 1.0) || !(o->tol > 0.0) || o->max_iter < 1)
    return ACE_ERR_INVALID;
  int rc = check_eig_opts(c, &o->eig);
  if (rc) return rc;
  const bool want_rec = o->rec_in || o->rec_tgt;
  if (want_rec && (!o->rec_in || !o->rec_tgt || o->rec_cap < 1 || o->rec_stride < 1))
    return ACE_ERR_INVALID;
  if ((want_rec || o->eig.precond == ACE_PRECOND_NET) && c->dtype != ACE_R32)
    return ACE_ERR_UNSUPPORTED;
  *res = ace_scf_result{};
  Eig e;
  rc = e.init(c, k, o->eig.precond == ACE_PRECOND_NET);
  const bool fp64 = e.fp64;
  const size_t ng = c->ng, vb = elem_bytes(c->dtype) * ng;
  hipStream_t s = c->stream;
  Mem xold, xal, xi, rho_in, rho_out, vh, vloc, ones, small;
  for (auto pr : {std::make_pair(&xold, vb * k), std::make_pair(&xal, vb * k),
                  std::make_pair(&xi, vb * k), std::make_pair(&rho_in, vb),
                  std::make_pair(&rho_out, vb), std::make_pair(&vh, vb),
                  std::make_pair(&vloc, vb), std::make_pair(&ones, vb),
                  std::make_pair(&small, sizeof(double) * (6 * 64 * 64 + kAbsParts + 8))})
    if (!rc) rc = pr.first->alloc(pr.second);
  if (rc) return rc;
  double* O = small.d();
  double* Aq = O + 64 * 64;
  double* w = Aq + 64 * 64;
  double* U = w + 64 * 64;
  double* B = U + 64 * 64;
  double* Q = B + 64 * 64;
  double* apart = Q + 64 * 64;
  double* err_d = apart + kAbsParts;
  double* exd = err_d + 1;
  launch_fill(fp64, 1.0, ng, ones.p, s);
  Recorder rec;
  rec.in = o->rec_in;
  rec.tgt = o->rec_tgt;
  rec.cap = o->rec_cap;
  rec.stride = std::max(1, o->rec_stride);
  bool converged = false;
  int it = 0, eig_total = 0;
  double err = 0.0, maxres = 0.0;
  for (it = 0; it < o->max_iter; ++it) {
    // Fock operator of the current orbitals: Hartree potential and the ACE rebuild
    launch_density(fp64, phi, k, ng, rho_in.p, s);
    rc = hartree(c, rho_in.p, ones.p, vh.p);
    if (rc) return rc;
    launch_axpby(fp64, v_ext, vh.p, 1.0, 1.0, ng, vloc.p, s);
    rc = ace_build(c, phi, k, xi.p, nullptr, exd);
    if (rc) return rc;
    if (hipMemcpyAsync(xold.p, phi, vb * k, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return ACE_ERR_HIP;
    // eigensolver steps on the fixed operator, from the current orbitals
    int st = 0;
    rc = e.run(vloc.p, xi.p, k, phi, &o->eig, want_rec ? &rec : nullptr, &st, &maxres);
    if (rc) return rc;
    eig_total += st;
    // Inexact inner solves: a fixed number of steps per iteration leaves residuals that, near
    // self-consistency, hold the density error on a plateau (seen in FP32 and FP64 alike).  When
    // the residuals are above the tolerance and large against the previous iteration's density
    // error, the eigensolver continues (up to three times the base count) until they fall below
    // max(tol, kInexact * that error).
    if (it > 0 && o->eig.tol > 0.0 && o->eig.max_steps > 0) {
      const double target = std::max(o->eig.tol, kInexact * err);
      if (maxres > target) {
        ace_eig_opts more = o->eig;
        more.max_steps = 3 * o->eig.max_steps;
        more.tol = target;
        st = 0;
        rc = e.run(vloc.p, xi.p, k, phi, &more, want_rec ? &rec : nullptr, &st, &maxres);
        if (rc) return rc;
        eig_total += st;
      }
    }
    // align the new occupied set with the old one (orthogonal Procrustes: Q = polar(O))
    e.gram(phi, k, xold.p, k, e.dv, O);
    launch_dgemm(1, 0, k, k, k, 1.0, O, k, O, k, 0.0, Aq, k, s);
    launch_jacobi(k, Aq, k, w, U, k, 60, 1e-15, s);
    launch_inv_sqrt_from_eig(w, U, k, B, s);
    launch_dgemm(0, 0, k, k, k, 1.0, O, k, B, k, 0.0, Q, k, s);
    launch_combine(fp64, phi, k, ng, Q, k, k, xal.p, s);
    // relative density error, Eq. (15)
    launch_density(fp64, xal.p, k, ng, rho_out.p, s);
    launch_abs_diff_sum(fp64, rho_out.p, rho_in.p, ng, e.dv / (2.0 * k), apart, err_d, s);
    int stc[4] = {0, 0, 0, 0};
    if (hipMemcpyAsync(&err, err_d, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(stc, c->status, sizeof(stc), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return ACE_ERR_HIP;
    if (stc[0]) {
      (void)hipMemsetAsync(c->status, 0, sizeof(stc), s);
      return stc[0];
    }
    if (err_hist) err_hist[it] = err;
    const bool states_ok = !(o->eig.tol > 0.0) || maxres < o->eig.tol;
    if (err < o->tol && states_ok) {
      if (hipMemcpyAsync(phi, xal.p, vb * k, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return ACE_ERR_HIP;
      converged = true;
      ++it;
      break;
    }
    // states mixing, Eq. (14), then Loewdin re-orthonormalisation
    launch_axpby(fp64, xold.p, xal.p, o->alpha, 1.0 - o->alpha, ng * k, xal.p, s);
    e.gram(xal.p, k, xal.p, k, e.dv, Aq);
    launch_jacobi(k, Aq, k, w, U, k, 60, 1e-15, s);
    launch_inv_sqrt_from_eig(w, U, k, B, s);
    launch_combine(fp64, xal.p, k, ng, B, k, k, phi, s);
  }
  std::vector<double> th(k);
  if (hipMemcpyAsync(th.data(), e.th.p, sizeof(double) * k, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return ACE_ERR_HIP;
  if (eigval) std::copy(th.begin(), th.end(), eigval);
  rc = energies(c, e, v_ext, phi, k, ones.p, rho_in.p, vh.p, xi.p, res->energy);
  if (rc) return rc;
  res->iterations = it;
  res->eig_steps = eig_total;
  res->converged = converged ? 1 : 0;
  res->density_error = err;
  res->max_residual = maxres;
  res->rec_count = rec.count;
  return ACE_OK;
}

int precond_targets(ace_ctx* c, const void* phi, int k, float* tgt, int count) {
  if (!c || !phi || !tgt || k < 1 || k > ACE_MAX_ORBITALS || count < 1) return ACE_ERR_INVALID;
  if (c->dtype != ACE_R32) return ACE_ERR_UNSUPPORTED;
  const size_t ng = c->ng;
  const int chunk = 64;
  size_t pts;
  const int nblk = gram_blocks(ng, &pts);
  Mem part, z, g, sc;
  int rc = part.alloc(sizeof(double) * (size_t)nblk * std::max(k, chunk) * chunk);
  if (!rc) rc = z.alloc(sizeof(double) * (size_t)k * chunk);
  if (!rc) rc = g.alloc(sizeof(double) * (size_t)chunk * chunk);
  if (!rc) rc = sc.alloc(sizeof(double) * (size_t)chunk);
  if (rc) return rc;
  const double dv = c->h * c->h * c->h;
  for (int v0 = 0; v0 < count; v0 += chunk) {
    const int cv = std::min(chunk, count - v0);
    float* t = tgt + (size_t)v0 * ng;
    launch_gram(ACE_R32, phi, k, t, cv, ng, part.p, dv, z.p, c->stream, nullptr);
    launch_project_complement(false, phi, k, z.d(), cv, ng, t, c->stream);
    // unit RMS: only the direction of a correction matters to the eigensolver
    launch_gram(ACE_R32, t, cv, t, cv, ng, part.p, 1.0, g.p, c->stream, nullptr);
    launch_inv_rms(g.d(), cv, cv, (double)ng, sc.d(), c->stream);
    launch_scale_inplace(false, t, sc.d(), cv, ng, c->stream);
  }
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
    return ACE_ERR_HIP;
  return ACE_OK;
}

}  // extern "C"
