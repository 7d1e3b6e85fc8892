// Tamm-Dancoff coupling block assembly (tda.hip), called from the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "internal.hpp"

namespace ace {

struct TdaWork {
  int nsplit = 1;       // split-K factor of the two contractions
  size_t kchunk = 0;    // points per split
  size_t off_pj = 0, off_pk = 0, off_cj = 0, off_ck = 0;  // byte offsets in the workspace
};

size_t tda_workspace_bytes(int no, int nv, size_t ng, bool fp64, TdaWork* w);

// v_ov: [no*nv][ng] pair potentials of (j, b) at row j*nv + b; v_oo: [no(no+1)/2][ng] of the
// occupied pairs a <= b at row b(b+1)/2 + a.  Writes C_out[(no*nv)^2] (FP64) and, if b_out is
// not null, the RHF B block B[ia][jb] = delta_M (ia|bj) - (ib|aj).
void launch_tda(bool fp64, const void* occ, int no, const void* virt, int nv, const void* v_ov,
                const void* v_oo, size_t ng, double dv, int delta_m, void* ws, const TdaWork& w,
                double* c_out, double* b_out, hipStream_t s, Trace* tr);

// One spin channel of a UHF reference: orbitals and their pair potentials (layouts as above).
struct UhfSpin {
  const void* occ;
  const void* virt;
  int no, nv;
  const void* v_ov;  // [no*nv][ng]
  const void* v_oo;  // [no(no+1)/2][ng]
};

struct UhfWork {
  int nsplit = 1;
  size_t kchunk = 0;
  size_t off_part = 0, off_g1[2][2] = {{0, 0}, {0, 0}}, off_g2[2] = {0, 0};
};

size_t uhf_workspace_bytes(const UhfSpin* sp, size_t ng, bool fp64, UhfWork* w);

// UHF A - diag and B over both spins (real orbitals): index alpha transitions i*nv_a + a first,
// then beta.  C[x][y] = (ia|jb) - delta_st (ij|ab), B[x][y] = (ia|jb) - delta_st (ib|ja).
void launch_uhf(bool fp64, const UhfSpin* sp, size_t ng, double dv, void* ws, const UhfWork& w,
                double* c_out, double* b_out, hipStream_t s, Trace* tr);

// D[c][i*nv + a] = <i| x_c |a> (c = x, y, z) on the box grid of edge n, spacing h
void launch_dipoles(bool fp64, const void* occ, int no, const void* virt, int nv, int n, double h,
                    double* D, hipStream_t s);
// f_k = 2/3 omega_k |d_k|^2
void launch_oscillator(const double* omega, const double* d, int k, double* f, hipStream_t s);
// S(w_i) = sum_k f_k L_gamma(w_i - omega_k), w_i = w0 + i dw
void launch_strength(const double* omega, const double* f, int k, double w0, double dw, int nw,
                     double gamma, double* S, hipStream_t s);

}  // namespace ace
