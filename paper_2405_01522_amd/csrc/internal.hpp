// Internal launcher interface between the C ABI (abi.cpp) and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ace {

// Kernel classes timed by the optional event tracer (ace_trace_* in the C ABI).
enum TraceId {
  TR_ZFWD = 0, TR_XY, TR_ZINV, TR_WACC, TR_GRAM, TR_CHOL, TR_TRSM, TR_APPLY, TR_DIRECT,
  TR_TDA_GEMM, TR_TDA_REDUCE, TR_SETUP, TR_COUNT
};

// Event-pair tracer bound to one stream; begin/end are no-ops when tracing is off.
struct Trace;
void trace_begin(Trace* t, int id);
void trace_end(Trace* t, int id);

// RAII helper: times the launches made while it is alive.
struct TraceScope {
  Trace* t;
  int id;
  TraceScope(Trace* t_, int id_) : t(t_), id(id_) { trace_begin(t, id); }
  ~TraceScope() { trace_end(t, id); }
};

// Box edges for which the pair-Poisson passes are compiled (padded edge P = 2N).
bool poisson_size_supported(int n, bool fp64);

// Bytes of FFT workspace needed per pair item (one complex FFT volume of N*N*P elements).
size_t poisson_work_bytes_per_item(int n, bool fp64);

// Kernel spectrum setup on the device, FP64: writes the real-even octant (P/2+1)^3 scaled by
// dV / P^3 into ghat64 and its FP32 rounding into ghat32.  cosw: (P/2+1)^2 FP64 weights
// w(a) cos(2 pi k a / P), tmp: two octant-sized FP64 scratch arrays.
void launch_kernel_setup(int n, double h, double c0, const double* cosw, double* tmp0,
                         double* tmp1, double* ghat64, float* ghat32, hipStream_t s);

// Kernel spectrum reordered to the position order of the FFT passes, full (2N)^3 array in
// the compute precision (double if fp64 else float), from the FP64 octant.
void launch_kernel_positions(int n, bool fp64, const double* oct, void* gpos, hipStream_t s);

// Pair Poisson solves for items [0, nitems).  Complex mode: item p is pair (pairs[2p],
// pairs[2p+1]) and v[p] = G (*) (conj(a_j) b_i).  Real-packed mode: item p covers pairs 2p
// and 2p+1 of the list (np pairs in total) and v is real, one volume per pair.
// phi_*: orbital arrays; work: nitems * work_bytes_per_item; v_out: output volumes;
// ghat: the position-ordered kernel spectrum of launch_kernel_positions.
void launch_pair_poisson(int n, bool fp64, bool real_packed, const void* phi_a,
                         const void* phi_b, const int* pairs_dev, int np, void* work,
                         void* v_out, const void* ghat, const void* tw, hipStream_t s,
                         Trace* tr);

// Pointers of one pair solve: v = G (*) (conj(a) b) (complex), or v = G (*) (a b) (real).
// Complex mode only: kind 1 packs the two real densities |a|^2 and |b|^2 into one transform
// (v and v2 receive them with zero imaginary part), kind 2 solves |a|^2 alone into v.
struct PairPtrs {
  const void* a;
  const void* b;
  void* v;
  void* v2 = nullptr;
  int kind = 0;
};

// Complex pair solves from an index list of 4 ints per transform (a, b, out0, out1) into
// v_out + out * ng: out1 == -1 is the pair v[out0] = G (*) (conj(phi_a) phi_b); out1 >= 0 packs
// the real densities |phi_a|^2 -> v[out0] and |phi_b|^2 -> v[out1] (zero imaginary parts);
// out1 == -2 solves |phi_a|^2 -> v[out0] alone.
void launch_pair_slots(int n, bool fp64, const void* phi, const int* slots_dev, int nslots,
                       void* work, void* v_out, const void* ghat, const void* tw, hipStream_t s,
                       Trace* tr);

// Same passes with explicit pointers per pair (pairs of many systems of one box edge in one
// launch).  items: device array of np entries; real-packed mode pairs items 2p and 2p+1.
void launch_pair_poisson_ptrs(int n, bool fp64, bool real_packed, const PairPtrs* items, int np,
                              void* work, const void* ghat, const void* tw, hipStream_t s,
                              Trace* tr);

}  // namespace ace
