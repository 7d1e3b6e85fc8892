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
// ghat: the position-ordered kernel spectrum of launch_kernel_positions.  Indices are clamped
// to [0, na) / [0, nb) and an index out of range is recorded in status (may be NULL).
void launch_pair_poisson(int n, bool fp64, bool real_packed, const void* phi_a, int na,
                         const void* phi_b, int nb, const int* pairs_dev, int np, void* work,
                         void* v_out, const void* ghat, const void* tw, int* status,
                         hipStream_t s, Trace* tr);

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

// ---------------------------------------------------------------------------------------
// Persistent passes over many systems of any box edges (poisson_queue.hip).  A job is one
// transform (one complex pair density or a couple of real ones); an item is one plane of a
// job: an x-plane for the z passes, K consecutive qz planes for the XY pass.  Items are
// listed largest box edge first and walked by a fixed grid of workgroups with a fixed stride.
struct QJob {
  PairPtrs p0, p1;   // the pair (complex) or one or two pairs (real-packed) of this transform
  void* work;        // this transform's N*N*P complex work volume
  const void* gpos;  // kernel spectrum in position order of this edge and spacing
  const void* tw;    // table twiddles of this edge
  int edge;          // box edge N
  int np;            // pairs of the transform: 1, or 2 for a real-packed couple
  int k;             // qz planes per XY item
};
struct QItem {
  int job;
  int idx;  // x-plane (z passes) or first qz plane (XY pass)
};
// Threads per workgroup of the three passes (z passes: 512 or 1024; XY: 1024).
struct QShape {
  int zf_nt, zi_nt;
};
// 1 if K qz planes per XY item are compiled for this edge and dtype (and fit in LDS).
bool queue_xy_k_ok(int n, bool fp64, int k);
// LDS bytes of one XY item of K planes / of one z-pass item at edge n.
size_t queue_xy_lds(int n, bool fp64, int k);
size_t queue_z_lds(int n, bool fp64);
// The passes over every job, each one launch of as many workgroups as fit on the device at
// once: z-forward and z-inverse over zitems (nz), XY over xyitems (nxy); lds_z / lds_xy: the
// largest item's LDS bytes of the pass; nt: threads of a z pass (512 or 1024).  Return 0, or
// -1 if the LDS does not fit.
int launch_zfwd_queue(bool fp64, bool real_packed, const QJob* jobs, const QItem* zitems, int nz,
                      size_t lds_z, int nt, hipStream_t s);
int launch_xy_queue(bool fp64, const QJob* jobs, const QItem* xyitems, int nxy, size_t lds_xy,
                    hipStream_t s);
int launch_zinv_queue(bool fp64, bool real_packed, const QJob* jobs, const QItem* zitems, int nz,
                      size_t lds_z, int nt, hipStream_t s);
// The z-forward (forward) or z-inverse pass of count consecutive jobs of one box edge n
// (jobs: device pointer to the first), one workgroup per (x-plane, job) with the one-system
// kernels' shapes.  -1 if the edge is not compiled for the precision.
int launch_z_edge(bool forward, int n, bool fp64, bool real_packed, const QJob* jobs, int count,
                  hipStream_t s);
// XY pass of count consecutive transforms of one box edge n (their N*N*P work volumes back to
// back from work) with the one-system kernel at nt threads (512 or 1024), one plane per
// workgroup.  -1 if the edge is not compiled for the precision.
int launch_xy_edge(int n, bool fp64, int nt, void* work, int count, const void* gpos,
                   const void* tw, hipStream_t s);
// The three in order, each timed by the tracer when it is on.
int launch_pair_queue(bool fp64, bool real_packed, const QJob* jobs, const QItem* zitems, int nz,
                      const QItem* xyitems, int nxy, size_t lds_z, size_t lds_xy, QShape sh,
                      hipStream_t s, Trace* tr);

}  // namespace ace
