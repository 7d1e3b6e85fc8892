// Launchers of the ACE kernels (ace_kernels.hip), called from the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "internal.hpp"

namespace ace {

// One system of an ACE build: orbitals, pair volumes and the workspaces / outputs of the
// steps after the pair solves.  Several of them (same box edge) can be processed by one
// launch per step (launch_ace_steps_batched).
struct MolArgs {
  const void* phi;   // [n][ng] orbitals
  const void* v;     // [n(n+1)/2][ng] pair potentials, pair (a<=b) at b(b+1)/2 + a
  void* w;           // [n][ng] W
  void* xi;          // [n][ng] output (may alias w)
  void* part;        // Gram partials [gram_blocks(ng)][n*n] (FP64, complex or real)
  void* mred;        // [n*n] reduced M (FP64)
  void* linvh;       // [n*n] L^{-H} (FP64)
  void* m_out;       // [n*n] M for the caller, or null
  double* ex_out;    // E_x for the caller, or null
  int* status;       // [2] device status word of this system
  int n;             // orbitals
  int blk0;          // first 256-point block of this system in a launch over many systems
  size_t ng;         // grid points of this system's box
  double dv;         // volume element h^3 of this system's grid
};

// storage element types (same numbering as the public ace_dtype)
enum { ET_C128 = 0, ET_C64 = 1, ET_R64 = 2, ET_R32 = 3 };

// number of Gram partial chunks for ng points (and the points per chunk)
int gram_blocks(size_t ng, size_t* chunk);


void launch_wacc(int et, const void* phi, const void* v, int n, size_t ng, void* w, hipStream_t s, Trace* tr);
// W accumulation and M = scale * Phi^H W into mred (n*n FP64, complex or real).  W and the
// Gram partials come from one fused kernel when the orbitals fit its LDS tile (n <= 16; 8 for
// complex FP64), else from the separate kernels.  part: gram_blocks(ng) * n * n partials.
void launch_wacc_gram(int et, const void* phi, const void* v, int n, size_t ng, void* w,
                      void* part, double scale, void* mred, hipStream_t s, Trace* tr);
// launch_wacc_gram in two steps: W (and, from the fused kernel, the Gram partials: the
// result is true then) ...
bool launch_wacc_partials(int et, const void* phi, const void* v, int n, size_t ng, void* w,
                          void* part, hipStream_t s, Trace* tr);
// ... then M into mred: the reduction of the partials, or the Gram of Phi and W.
void launch_wacc_finish(int et, bool partials, const void* phi, int n, size_t ng, const void* w,
                        void* part, double scale, void* mred, hipStream_t s, Trace* tr);
// launch_chol followed by launch_trsm (one fused kernel for n <= 8).
void launch_chol_trsm(int et, const void* mred, int n, void* m_out, double* ex_out, void* linvh,
                      int* status, const void* w, size_t ng, void* xi, hipStream_t s, Trace* tr);
// out[k*nb + l] = scale * sum_r conj(A_k(r)) B_l(r), FP64 (complex or real), any na, nb.
// part: gram_blocks(ng) * na * nb FP64 elements.
void launch_gram(int et, const void* A, int na, const void* B, int nb, size_t ng, void* part,
                 double scale, void* out, hipStream_t s, Trace* tr);
void launch_chol(int et, const void* mred, int n, void* m_out, double* ex_out, void* linvh,
                 int* status, hipStream_t s, Trace* tr);
void launch_trsm(int et, const void* w, int n, size_t ng, const void* linvh, void* xi, hipStream_t s, Trace* tr);
void launch_apply_out(int et, const void* xi, int n, size_t ng, const void* z, int nv, void* out,
                      hipStream_t s, Trace* tr);
// The same update from y = W^H psi dV ([n][nv] FP64): Z = L^{-1} y is formed per workgroup
// from linvh = L^{-H} ([n][n] FP64, as written by launch_chol / launch_chol_trsm).
void launch_apply_from_y(int et, const void* xi, int n, size_t ng, const void* linvh,
                         const void* y, int nv, void* out, hipStream_t s, Trace* tr);
// Complex storage, n <= 8, one system (false, nothing launched, otherwise): the Gram
// partials of y = W^H psi (nv <= 64 vectors) into part_y, and in the same launch M into mred
// from the partials part_m of launch_wacc_partials -- the bits of launch_wacc_finish.
bool launch_gram_y_reduce_m(int et, const void* w, int n, const void* psi, int nv, size_t ng,
                            void* part_y, const void* part_m, double scale, void* mred,
                            hipStream_t s, Trace* tr);
// After it: launch_chol_trsm's Cholesky and xi (same bits), and in the same launch
// z = L^{-1} Y ([n][nv] FP64, = xi^H psi dV) from Y = scale * sum of part_y, the layout of
// launch_gram's partials for na = n, nb = nv.
void launch_chol_trsm_zcol(int et, const void* mred, int n, void* m_out, double* ex_out,
                           void* linvh, int* status, const void* w, size_t ng, void* xi,
                           const void* part_y, int nv, void* z, double scale, hipStream_t s,
                           Trace* tr);

// Direct exchange accumulation: out_v = -sum_j phi_j v[v*n + j]  (v: [nv][n][ng] pair volumes).
void launch_direct_acc(int et, const void* phi, int n, const void* v, int nv, size_t ng, void* out,
                       hipStream_t s, Trace* tr);

// W accumulation, M Gram + reduction, Cholesky / E_x and xi for nmol systems of any box edges
// and spacings, one launch per step: their MolArgs (ng, blk0 and dv set) are in device memory,
// bsys maps each of the nblk 256-point blocks of all systems to its system; nmax = largest
// orbital count.
void launch_ace_steps_flat(int et, const MolArgs* mols_dev, const int* bsys_dev, int nmol,
                           int nblk, int nmax, hipStream_t s, Trace* tr);

}  // namespace ace
