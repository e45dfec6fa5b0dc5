// Internal interface of the batched solver (tip_batch.hip) for the host
// driver (tip_api.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tip_device.h"
#include "tip_launch.h"

namespace tip {

constexpr int kBatchMaxRestarts = 8;       // FP64 restarts of one solve, as in the single-problem solver

// One problem of a batch as the kernels see it.
struct BatchProb {
  const double* mass_field;    // [V] or null
  double mass;
  const double* coupling;      // [ndim][V] or null
  const void* links;           // covariant: [ndim][9][V] double2 (kernel layout), else null
  const void* links32;         // its single-precision copy (mixed precision), else null
  uint64_t seed;
  int32_t mask;
  int32_t max_iter;
  double tol2;
};

// A block of 2^logB right-hand sides of one problem.  The kernels read its
// geometry in place (a reference into device memory: a private copy would be
// indexed by dimension at run time and go to scratch memory).
struct BatchJob {
  Geom g;                      // the problem's lattice and probe kind, with the job's probe class
  int32_t prob;                // index into the BatchProb array
  int32_t logB;
  int32_t nb;                  // lanes holding a right-hand side (the rest are padding)
  int64_t rhs0;                // right-hand side of lane 0 (class-local index with a class)
  uint32_t item0, nitems;      // its work items
  int32_t lane0;               // global index of lane 0
  uint32_t site_bytes;         // algorithmic bytes per site of the operator (links, couplings, mass field)
  uint32_t esz;                // bytes per element of the group's working vectors
  uint32_t pad;
  uint64_t off;                // element offset of its vectors ([ncomp][V][B]) in the group's arrays
};

// Device tables of a batch and the launch-specific item base.
struct BatchArgs {
  const BatchJob* jobs;
  const BatchProb* probs;
  const uint32_t* item_job;    // [items] job of each work item
  const int32_t* lane_job;     // [lanes] job of each lane
  uint32_t item_base;          // first item of the launch's group
  int32_t item_sites;          // sites per work item (a power of two >= 256)
  size_t PI;                   // partials per lane row (the most items of any job)
  int32_t march;               // kb_stencil: bit 0 slices in bands of item_sites / TS, bit 1 job items split per XCD
  unsigned long long* bytes;   // when profiling: algorithmic bytes the stencil launches moved, or null
};

// Jobs sharing one operator kind, element type and precision: one launch per
// CG phase covers all of them.
struct BatchGroup {
  int kind;
  Elem elem;
  Prec prec;
  uint32_t item_base, nitems;
  int lane_base, nlanes;
  int ndim;                    // the dimension every job of the group has, or 0 when they differ
  int min_logB;                // log2 of the smallest block of right-hand sides among its jobs
};

hipError_t launch_batch_scalars_init(const BatchArgs& a, const CgScalars& sc, int nlanes, hipStream_t st);
// x64 = 0 (and xh = 0 when given), r = p = b in the group's working precision
hipError_t launch_batch_init(const BatchArgs& a, const BatchGroup& gr, void* x64, void* xh, void* r, void* p,
                             hipStream_t st);
// One CG iteration of every live lane of the group: w = A p, alpha, r -= alpha w,
// beta, x += alpha p, p = r + beta p.  ev0 / ev1 (or null) are recorded
// around the stencil launch.
hipError_t launch_batch_iteration(const BatchArgs& a, const BatchGroup& gr, const CgScalars& sc, void* x, void* r,
                                  void* p, void* w, double* partial, size_t rowstride, double eps, double tau2,
                                  hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);
// Mixed precision: reliable updates (mode 0) or the final FP64 check (mode 1);
// partial holds 5 rows rowstride apart.
hipError_t launch_batch_reliable(const BatchArgs& a, const BatchGroup& gr, const CgScalars& sc, int mode, void* x64,
                                 void* xh, void* r, void* p, double* partial, size_t rowstride, hipStream_t st);
// FP64: the true-residual check of the frozen lanes (3 partial rows).
hipError_t launch_batch_true_residual(const BatchArgs& a, const BatchGroup& gr, const CgScalars& sc, void* x,
                                      void* r, void* p, double* partial, size_t rowstride, hipStream_t st);

}  // namespace tip
