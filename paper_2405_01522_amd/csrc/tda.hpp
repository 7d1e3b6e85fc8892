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
// occupied pairs a <= b at row b(b+1)/2 + a.  Writes C_out[(no*nv)^2] (FP64).
void launch_tda(bool fp64, const void* occ, int no, const void* virt, int nv, const void* v_ov,
                const void* v_oo, size_t ng, double dv, int delta_m, void* ws, const TdaWork& w,
                double* c_out, hipStream_t s, Trace* tr);

}  // namespace ace
