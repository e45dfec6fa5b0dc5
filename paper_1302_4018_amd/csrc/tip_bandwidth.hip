// Practical HBM ceiling of MI355X measured with plain streaming kernels, for
// stating the stencil's rate against what a kernel that only moves data
// reaches on the same machine (beside the published 8 TB/s).
//
// Each kernel walks its arrays once per pass with 16-byte loads and stores,
// 256-thread workgroups and four independent accesses in flight per thread
// (grid-stride, one pass = every element once).  Arrays are far larger than
// the 256 MB last-level cache, so every pass streams from HBM.
//   kind 0  read only: partial sums of a (one partial per workgroup)
//   kind 1  copy:      b = a
//   kind 2  three reads, one write: d = a + b + c (the read:write mix of the
//           dominant half-lattice stencil is about 2.7:1)

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>

#include "../../include/tip.h"
#include "tip_launch.h"

namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;

__global__ __launch_bounds__(kThreads) void k_read(size_t n, const double2* __restrict__ a,
                                                   double* __restrict__ partial) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  double2 s[kUnroll];
#pragma unroll
  for (int k = 0; k < kUnroll; ++k) s[k] = make_double2(0.0, 0.0);
  for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
    double2 v[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) v[k] = a[i + k * stride];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) s[k].x += v[k].x, s[k].y += v[k].y;
  }
  for (; i < n; i += stride) s[0].x += a[i].x, s[0].y += a[i].y;
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < kUnroll; ++k) t += s[k].x + s[k].y;
  for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
  __shared__ double lds[kThreads / 64];
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

__global__ __launch_bounds__(kThreads) void k_copy(size_t n, const double2* __restrict__ a, double2* __restrict__ b) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
    double2 v[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) v[k] = a[i + k * stride];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) b[i + k * stride] = v[k];
  }
  for (; i < n; i += stride) b[i] = a[i];
}

__global__ __launch_bounds__(kThreads) void k_sum3(size_t n, const double2* __restrict__ a,
                                                   const double2* __restrict__ b, const double2* __restrict__ c,
                                                   double2* __restrict__ d) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
    double2 va[kUnroll], vb[kUnroll], vc[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      va[k] = a[i + k * stride];
      vb[k] = b[i + k * stride];
      vc[k] = c[i + k * stride];
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k)
      d[i + k * stride] = make_double2(va[k].x + vb[k].x + vc[k].x, va[k].y + vb[k].y + vc[k].y);
  }
  for (; i < n; i += stride)
    d[i] = make_double2(a[i].x + b[i].x + c[i].x, a[i].y + b[i].y + c[i].y);
}

__global__ __launch_bounds__(kThreads) void k_fill2(size_t n, double2* __restrict__ a, double v) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) a[i] = make_double2(v, -v);
}

}  // namespace

extern "C" {

tip_status tip_stream_ceiling(int32_t kind, int64_t bytes, int32_t reps, int32_t grid, double* seconds_per_pass,
                              double* bytes_per_pass, void* stream) {
  if (kind < 0 || kind > 2 || bytes < (int64_t)(1 << 20) || reps < 1 || grid < 0 || !seconds_per_pass ||
      !bytes_per_pass) {
    tip::set_last_error("tip_stream_ceiling: kind in 0..2, bytes >= 1 MiB, reps >= 1, grid >= 0 and output "
                        "pointers needed");
    return TIP_EINVAL;
  }
  const int narr = kind == 0 ? 1 : kind == 1 ? 2 : 4;
  const size_t per = (size_t)bytes / narr / sizeof(double2) * sizeof(double2);   // bytes per array
  const size_t n = per / sizeof(double2);
  hipStream_t st = (hipStream_t)stream;
  const unsigned g = grid > 0 ? (unsigned)grid : 256u * 16u;   // 16 workgroups per compute unit
  double2* arr[4] = {nullptr, nullptr, nullptr, nullptr};
  double* partial = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  tip_status ret = TIP_OK;
  auto fail = [&](tip_status s, const char* what, hipError_t e) {
    char buf[256];
    snprintf(buf, sizeof buf, "tip_stream_ceiling: %s: %s", what, hipGetErrorString(e));
    tip::set_last_error(buf);
    ret = s;
  };
  for (int k = 0; k < narr && ret == TIP_OK; ++k)
    if (const hipError_t e = hipMalloc(&arr[k], per); e != hipSuccess) fail(TIP_ENOMEM, "hipMalloc", e);
  if (ret == TIP_OK)
    if (const hipError_t e = hipMalloc(&partial, g * sizeof(double)); e != hipSuccess) fail(TIP_ENOMEM, "hipMalloc", e);
  if (ret == TIP_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    fail(TIP_EDEVICE, "hipEventCreate", hipGetLastError());
  auto pass = [&]() {
    if (kind == 0) k_read<<<g, kThreads, 0, st>>>(n, arr[0], partial);
    else if (kind == 1) k_copy<<<g, kThreads, 0, st>>>(n, arr[0], arr[1]);
    else k_sum3<<<g, kThreads, 0, st>>>(n, arr[0], arr[1], arr[2], arr[3]);
  };
  if (ret == TIP_OK) {
    for (int k = 0; k < narr; ++k) k_fill2<<<g, kThreads, 0, st>>>(n, arr[k], 1.0 + k);
    pass();                                                       // warm-up
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r) pass();
    (void)hipEventRecord(e1, st);
    if (const hipError_t e = hipEventSynchronize(e1); e != hipSuccess) {
      fail(TIP_EDEVICE, "streaming kernels", e);
    } else {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      *seconds_per_pass = ms * 1e-3 / reps;
      *bytes_per_pass = (double)per * narr;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (int k = 0; k < narr; ++k)
    if (arr[k]) (void)hipFree(arr[k]);
  if (partial) (void)hipFree(partial);
  return ret;
}

}  // extern "C"
