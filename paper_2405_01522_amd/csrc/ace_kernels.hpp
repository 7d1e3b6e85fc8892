// Launchers of the ACE kernels (ace_kernels.hip), called from the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "internal.hpp"

namespace ace {

// storage element types (same numbering as the public ace_dtype)
enum { ET_C128 = 0, ET_C64 = 1, ET_R64 = 2, ET_R32 = 3 };

// number of Gram partial chunks for ng points (and the points per chunk)
int gram_blocks(size_t ng, size_t* chunk);

void launch_wacc(int et, const void* phi, const void* v, int n, size_t ng, void* w, hipStream_t s, Trace* tr);
// out[k*nb + l] = scale * sum_r conj(A_k(r)) B_l(r), FP64 (complex or real), any na, nb.
// part: gram_blocks(ng) * na * nb FP64 elements.
void launch_gram(int et, const void* A, int na, const void* B, int nb, size_t ng, void* part,
                 double scale, void* out, hipStream_t s, Trace* tr);
void launch_chol(int et, const void* mred, int n, void* m_out, double* ex_out, void* linvh,
                 int* status, hipStream_t s, Trace* tr);
void launch_trsm(int et, const void* w, int n, size_t ng, const void* linvh, void* xi, hipStream_t s, Trace* tr);
void launch_apply_out(int et, const void* xi, int n, size_t ng, const void* z, int nv, void* out,
                      hipStream_t s, Trace* tr);

// Direct exchange accumulation: out_v = -sum_j phi_j v[v*n + j]  (v: [nv][n][ng] pair volumes).
void launch_direct_acc(int et, const void* phi, int n, const void* v, int nv, size_t ng, void* out,
                       hipStream_t s, Trace* tr);

}  // namespace ace
