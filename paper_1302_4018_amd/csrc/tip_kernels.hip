// HIP kernels of libtip for gfx950 (MI355X).
//
// Data layout in HBM (site index s = x1 + n1 (x2 + n2 (x3 + n3 x4))):
//   vectors   [B][ncomp][V] of T (T = double for real scalar problems,
//             double2 = (re, im) otherwise): one coalesced 8/16-byte word per
//             lane for every (rhs, component);
//   links     [ndim][9][V] double2: element (a, b) of U_mu(s) at
//             [mu][3a+b][s], so a wave reads each matrix element of 64
//             consecutive sites as one contiguous 1 KiB run;
//   coupling  [ndim][V] double, mass_field [V] double (caller layout).
// Workgroups are 256 threads; blockIdx.x tiles sites, blockIdx.y selects a
// group of R right-hand sides that one thread carries in registers, so each
// link is read once per R right-hand sides.
//
// All reductions are two-stage and deterministic: each workgroup writes one
// partial per right-hand side, a second kernel sums the partials in a fixed
// order.  No floating-point atomics are used.

#include "tip_device.h"
#include "tip_launch.h"

namespace tip {

// ---------------------------------------------------------------------------
// Stencils: hop(s) = sum_mu [w_mu(s) U_mu(s) x(s+mu) + w_mu(s-mu) U_mu(s-mu)^H x(s-mu)],
// diag(s) = m(s) + sum_mu [w_mu(s) + w_mu(s-mu)],  (A x)(s) = diag(s) x(s) - hop(s).
// ---------------------------------------------------------------------------

template <int R>
__device__ __forceinline__ void cov_hop(const Geom& g, uint32_t s, const double2* __restrict__ U,
                                        const double* __restrict__ w, const double2* __restrict__ in,
                                        double2 (&hop)[R][3], double& diag) {
  const size_t V = g.V;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) hop[r][a] = make_double2(0.0, 0.0);
  for (int mu = 0; mu < g.ndim; ++mu) {
    const uint32_t sf = nbr_fwd(s, g, mu);
    const uint32_t sb = nbr_bwd(s, g, mu);
    const double wf = w ? w[(size_t)mu * V + s] : 1.0;
    const double wb = w ? w[(size_t)mu * V + sb] : 1.0;
    diag += wf + wb;
    const double2* Um = U + (size_t)mu * 9 * V;
    {
      double2 u[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) u[e] = Um[(size_t)e * V + s];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double2 xv[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) xv[b] = in[((size_t)r * 3 + b) * V + sf];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          double2 t = make_double2(0.0, 0.0);
#pragma unroll
          for (int b = 0; b < 3; ++b) t = cfma(u[3 * a + b], xv[b], t);
          hop[r][a].x = fma(wf, t.x, hop[r][a].x);
          hop[r][a].y = fma(wf, t.y, hop[r][a].y);
        }
      }
    }
    {
      double2 u[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) u[e] = Um[(size_t)e * V + sb];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double2 xv[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) xv[b] = in[((size_t)r * 3 + b) * V + sb];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          double2 t = make_double2(0.0, 0.0);
#pragma unroll
          for (int b = 0; b < 3; ++b) t = cfma_conj(u[3 * b + a], xv[b], t);
          hop[r][a].x = fma(wb, t.x, hop[r][a].x);
          hop[r][a].y = fma(wb, t.y, hop[r][a].y);
        }
      }
    }
  }
}

template <class T, int R>
__device__ __forceinline__ void scalar_hop(const Geom& g, uint32_t s, const double* __restrict__ w,
                                           const T* __restrict__ in, T (&hop)[R], double& diag) {
  const size_t V = g.V;
#pragma unroll
  for (int r = 0; r < R; ++r) hop[r] = zero<T>();
  for (int mu = 0; mu < g.ndim; ++mu) {
    const uint32_t sf = nbr_fwd(s, g, mu);
    const uint32_t sb = nbr_bwd(s, g, mu);
    const double wf = w ? w[(size_t)mu * V + s] : 1.0;
    const double wb = w ? w[(size_t)mu * V + sb] : 1.0;
    diag += wf + wb;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      hop[r] = axpy(wf, in[(size_t)r * V + sf], hop[r]);
      hop[r] = axpy(wb, in[(size_t)r * V + sb], hop[r]);
    }
  }
}

// out = A in for R right-hand sides per thread; partial[j][bx] = Re(in_j^H out_j)
// summed over the workgroup's sites (p^H A p in CG).  partial may be null.
template <int R>
__global__ __launch_bounds__(kBlock) void k_cov_matvec(Geom g, const double2* __restrict__ U,
                                                       const double* __restrict__ mass_field, double mass,
                                                       const double* __restrict__ w,
                                                       const double2* __restrict__ in,
                                                       double2* __restrict__ out,
                                                       double* __restrict__ partial,
                                                       const int* __restrict__ active, int* __restrict__ ran) {
  if (active && *active == 0) return;
  if (ran && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *ran = 1;
  __shared__ double lds[R * 4];
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  const size_t V = g.V;
  const size_t off = (size_t)blockIdx.y * R * 3 * V;
  in += off;
  out += off;
  double dot[R];
#pragma unroll
  for (int r = 0; r < R; ++r) dot[r] = 0.0;
  if (s < g.V) {
    double2 hop[R][3];
    double diag = mass_field ? mass_field[s] : mass;
    cov_hop<R>(g, s, U, w, in, hop, diag);
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const size_t i = ((size_t)r * 3 + a) * V + s;
        const double2 x = in[i];
        double2 y;
        y.x = fma(diag, x.x, -hop[r][a].x);
        y.y = fma(diag, x.y, -hop[r][a].y);
        out[i] = y;
        dot[r] += redot(x, y);
      }
    }
  }
  if (partial) {
    block_sum<R>(dot, lds);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) partial[(size_t)(blockIdx.y * R + r) * gridDim.x + blockIdx.x] = dot[r];
    }
  }
}

template <class T, int R>
__global__ __launch_bounds__(kBlock) void k_scalar_matvec(Geom g, const double* __restrict__ mass_field,
                                                          double mass, const double* __restrict__ w,
                                                          const T* __restrict__ in, T* __restrict__ out,
                                                          double* __restrict__ partial,
                                                          const int* __restrict__ active, int* __restrict__ ran) {
  if (active && *active == 0) return;
  if (ran && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *ran = 1;
  __shared__ double lds[R * 4];
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  const size_t V = g.V;
  const size_t off = (size_t)blockIdx.y * R * V;
  in += off;
  out += off;
  double dot[R];
#pragma unroll
  for (int r = 0; r < R; ++r) dot[r] = 0.0;
  if (s < g.V) {
    T hop[R];
    double diag = mass_field ? mass_field[s] : mass;
    scalar_hop<T, R>(g, s, w, in, hop, diag);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const size_t i = (size_t)r * V + s;
      const T x = in[i];
      const T y = axpy(diag, x, axpy(-1.0, hop[r], zero<T>()));
      out[i] = y;
      dot[r] += redot(x, y);
    }
  }
  if (partial) {
    block_sum<R>(dot, lds);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) partial[(size_t)(blockIdx.y * R + r) * gridDim.x + blockIdx.x] = dot[r];
    }
  }
}

// ---------------------------------------------------------------------------
// CG passes.  RHS j of the block is global right-hand side rhs0 + j, i.e.
// spatial probe m = (rhs0 + j) / ncomp and component c = (rhs0 + j) % ncomp.
// ---------------------------------------------------------------------------

// x = 0, r = p = b_j (generated from the site index), zero for padding RHS.
template <class T>
__global__ __launch_bounds__(kBlock) void k_init(Geom g, int64_t rhs0, int nb, uint64_t seed, int mask,
                                                 T* __restrict__ x, T* __restrict__ r, T* __restrict__ p) {
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const int j = blockIdx.y;
  const size_t V = g.V;
  const uint32_t P = hier_perm(s, g);
  const int64_t rg = rhs0 + j;
  const int cj = (int)(rg % g.ncomp);
  const uint32_t col = hadamard_column((uint32_t)(rg / g.ncomp), g.L);
  for (int c = 0; c < g.ncomp; ++c) {
    const size_t i = ((size_t)j * g.ncomp + c) * V + s;
    T b = zero<T>();
    if (j < nb && c == cj) b = from_c<T>(probe_value(s, P, col, c, g, seed, mask));
    x[i] = zero<T>();
    r[i] = b;
    p[i] = b;
  }
}

// x += alpha p; r -= alpha Ap; partial = ||r||^2  (active right-hand sides only)
template <class T>
__global__ __launch_bounds__(kBlock) void k_update(Geom g, const CgScalars sc, T* __restrict__ x,
                                                   T* __restrict__ r, const T* __restrict__ p,
                                                   const T* __restrict__ Ap, double* __restrict__ partial) {
  const int j = blockIdx.y;
  if (*sc.active == 0 || sc.state[j] != kActive) return;
  __shared__ double lds[4];
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  const size_t V = g.V;
  const double a = sc.alpha[j];
  double acc[1] = {0.0};
  if (s < g.V) {
    for (int c = 0; c < g.ncomp; ++c) {
      const size_t i = ((size_t)j * g.ncomp + c) * V + s;
      x[i] = axpy(a, p[i], x[i]);
      const T ri = axpy(-a, Ap[i], r[i]);
      r[i] = ri;
      acc[0] += norm2(ri);
    }
  }
  block_sum<1>(acc, lds);
  if (threadIdx.x == 0) partial[(size_t)j * gridDim.x + blockIdx.x] = acc[0];
}

// p = r + beta p  (active right-hand sides only)
template <class T>
__global__ __launch_bounds__(kBlock) void k_direction(Geom g, const CgScalars sc, const T* __restrict__ r,
                                                      T* __restrict__ p) {
  const int j = blockIdx.y;
  if (*sc.active == 0 || sc.state[j] != kActive) return;
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const size_t V = g.V;
  const double b = sc.beta[j];
  for (int c = 0; c < g.ncomp; ++c) {
    const size_t i = ((size_t)j * g.ncomp + c) * V + s;
    p[i] = axpy(b, p[i], r[i]);
  }
}

// True residual: rt = b - A x in FP64, with b regenerated; r = p = rt.
// partial[0] = ||rt||^2, partial[1], partial[2] = Re, Im of b^H x.
template <int R>
__global__ __launch_bounds__(kBlock) void k_cov_true_residual(Geom g, const double2* __restrict__ U,
                                                              const double* __restrict__ mass_field, double mass,
                                                              const double* __restrict__ w, int64_t rhs0, int nb,
                                                              uint64_t seed, int mask,
                                                              const double2* __restrict__ x,
                                                              double2* __restrict__ r, double2* __restrict__ p,
                                                              double* __restrict__ partial, size_t pstride) {
  __shared__ double lds[3 * R * 4];
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  const size_t V = g.V;
  const int j0 = blockIdx.y * R;
  const size_t off = (size_t)j0 * 3 * V;
  double acc[3 * R];
#pragma unroll
  for (int i = 0; i < 3 * R; ++i) acc[i] = 0.0;
  if (s < g.V) {
    double2 hop[R][3];
    double diag = mass_field ? mass_field[s] : mass;
    cov_hop<R>(g, s, U, w, x + off, hop, diag);
    const uint32_t P = hier_perm(s, g);
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int j = j0 + rr;
      const int64_t rg = rhs0 + j;
      const int cj = (int)(rg % 3);
      const uint32_t col = hadamard_column((uint32_t)(rg / 3), g.L);
      const double2 bval = j < nb ? probe_value(s, P, col, cj, g, seed, mask) : make_double2(0.0, 0.0);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const size_t i = ((size_t)j * 3 + a) * V + s;
        const double2 xv = x[i];
        const double2 b = a == cj ? bval : make_double2(0.0, 0.0);
        double2 rt;
        rt.x = b.x - fma(diag, xv.x, -hop[rr][a].x);
        rt.y = b.y - fma(diag, xv.y, -hop[rr][a].y);
        r[i] = rt;
        p[i] = rt;
        acc[3 * rr + 0] += norm2(rt);
        acc[3 * rr + 1] += redot(b, xv);
        acc[3 * rr + 2] += imdot(b, xv);
      }
    }
  }
  block_sum<3 * R>(acc, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        partial[k * pstride + (size_t)(j0 + rr) * gridDim.x + blockIdx.x] = acc[3 * rr + k];
  }
}

template <class T, int R>
__global__ __launch_bounds__(kBlock) void k_scalar_true_residual(Geom g, const double* __restrict__ mass_field,
                                                                 double mass, const double* __restrict__ w,
                                                                 int64_t rhs0, int nb, uint64_t seed, int mask,
                                                                 const T* __restrict__ x, T* __restrict__ r,
                                                                 T* __restrict__ p, double* __restrict__ partial,
                                                                 size_t pstride) {
  __shared__ double lds[3 * R * 4];
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  const size_t V = g.V;
  const int j0 = blockIdx.y * R;
  const size_t off = (size_t)j0 * V;
  double acc[3 * R];
#pragma unroll
  for (int i = 0; i < 3 * R; ++i) acc[i] = 0.0;
  if (s < g.V) {
    T hop[R];
    double diag = mass_field ? mass_field[s] : mass;
    scalar_hop<T, R>(g, s, w, x + off, hop, diag);
    const uint32_t P = hier_perm(s, g);
#pragma unroll
    for (int rr = 0; rr < R; ++rr) {
      const int j = j0 + rr;
      const int64_t rg = rhs0 + j;
      const uint32_t col = hadamard_column((uint32_t)rg, g.L);
      const T b = j < nb ? from_c<T>(probe_value(s, P, col, 0, g, seed, mask)) : zero<T>();
      const size_t i = (size_t)j * V + s;
      const T xv = x[i];
      const T ax = axpy(diag, xv, axpy(-1.0, hop[rr], zero<T>()));
      const T rt = axpy(-1.0, ax, b);
      r[i] = rt;
      p[i] = rt;
      acc[3 * rr + 0] += norm2(rt);
      acc[3 * rr + 1] += redot(b, xv);
      acc[3 * rr + 2] += imdot(b, xv);
    }
  }
  block_sum<3 * R>(acc, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int rr = 0; rr < R; ++rr)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        partial[k * pstride + (size_t)(j0 + rr) * gridDim.x + blockIdx.x] = acc[3 * rr + k];
  }
}

// ---------------------------------------------------------------------------
// Scalar bookkeeping of CG, one workgroup per right-hand side.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int n) {
  __shared__ double lds[4];
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += kBlock) v[0] += part[i];
  block_sum<1>(v, lds);
  return v[0];
}

__global__ void k_scalars_init(CgScalars sc, int nb, int B, double bnorm2, int start_frozen) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) *sc.active = start_frozen ? 0 : nb;
  if (j >= B) return;
  const bool valid = j < nb;
  sc.state[j] = valid ? (start_frozen ? kFrozen : kActive) : kPadding;
  sc.bnorm2[j] = valid ? bnorm2 : 0.0;
  sc.rho[j] = valid ? bnorm2 : 0.0;
  sc.alpha[j] = 0.0;
  sc.beta[j] = 0.0;
  sc.iters[j] = 0;
  sc.restarts[j] = 0;
  sc.relres2[j] = 0.0;
  sc.q[2 * j] = 0.0;
  sc.q[2 * j + 1] = 0.0;
}

// alpha = rho / p^H A p; breakdown when p^H A p is not positive and finite.
__global__ __launch_bounds__(kBlock) void k_reduce_alpha(CgScalars sc, const double* __restrict__ partial, int gx) {
  const int j = blockIdx.x;
  if (*sc.active == 0) return;
  const double pAp = sum_partials(partial + (size_t)j * gx, gx);
  if (threadIdx.x != 0) return;
  if (sc.state[j] != kActive) {
    sc.alpha[j] = 0.0;
    return;
  }
  if (!(pAp > 0.0) || !isfinite(pAp)) {
    sc.state[j] = kBreakdown;
    sc.alpha[j] = 0.0;
    atomicSub(sc.active, 1);
    return;
  }
  sc.alpha[j] = sc.rho[j] / pAp;
}

// rho' = ||r||^2; beta = rho'/rho; freeze on the recursive residual, or stop at max_iter.
__global__ __launch_bounds__(kBlock) void k_reduce_beta(CgScalars sc, const double* __restrict__ partial, int gx,
                                                        double tol2, int max_iter) {
  const int j = blockIdx.x;
  if (*sc.active == 0) return;
  if (sc.state[j] != kActive) return;        // uniform per workgroup
  const double rho_new = sum_partials(partial + (size_t)j * gx, gx);
  if (threadIdx.x != 0) return;
  const int it = sc.iters[j] + 1;
  sc.iters[j] = it;
  sc.beta[j] = rho_new / sc.rho[j];
  sc.rho[j] = rho_new;
  if (!isfinite(rho_new)) {
    sc.state[j] = kBreakdown;
    atomicSub(sc.active, 1);
  } else if (rho_new <= tol2 * sc.bnorm2[j]) {
    sc.state[j] = kFrozen;
    atomicSub(sc.active, 1);
  } else if (it >= max_iter) {
    sc.state[j] = kNoConv;
    atomicSub(sc.active, 1);
  }
}

// Accept a frozen solve when its true residual passes, else restart CG from x.
__global__ __launch_bounds__(kBlock) void k_reduce_true(CgScalars sc, const double* __restrict__ partial, int gx,
                                                        size_t pstride, double tol2, int max_iter, int max_restarts) {
  const int j = blockIdx.x;
  if (sc.state[j] != kFrozen) return;
  const double rt2 = sum_partials(partial + (size_t)j * gx, gx);
  const double qre = sum_partials(partial + pstride + (size_t)j * gx, gx);
  const double qim = sum_partials(partial + 2 * pstride + (size_t)j * gx, gx);
  if (threadIdx.x != 0) return;
  sc.relres2[j] = rt2 / sc.bnorm2[j];
  if (rt2 <= tol2 * sc.bnorm2[j]) {
    sc.state[j] = kAccepted;
    sc.q[2 * j] = qre;
    sc.q[2 * j + 1] = qim;
  } else if (sc.restarts[j] < max_restarts && sc.iters[j] < max_iter && isfinite(rt2)) {
    sc.state[j] = kActive;
    sc.rho[j] = rt2;
    sc.restarts[j] += 1;
    atomicAdd(sc.active, 1);
  } else {
    sc.state[j] = kNoConv;
  }
}

// ---------------------------------------------------------------------------
// Generator entry points and layout conversion.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_hier_perm(Geom g, uint32_t* __restrict__ out) {
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s < g.V) out[s] = hier_perm(s, g);
}

__global__ __launch_bounds__(kBlock) void k_probe_vectors(Geom g, uint64_t seed, int mask, int64_t m0, int comp,
                                                          double2* __restrict__ out) {
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const int64_t m = m0 + blockIdx.y;
  const uint32_t P = hier_perm(s, g);
  out[(size_t)blockIdx.y * g.V + s] = probe_value(s, P, hadamard_column((uint32_t)m, g.L), comp, g, seed, mask);
}

// [ndim][V][3][3] complex (caller) -> [ndim][9][V] complex (kernels)
__global__ __launch_bounds__(kBlock) void k_repack_links(Geom g, const double2* __restrict__ src,
                                                         double2* __restrict__ dst) {
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const int mu = blockIdx.y;
  const size_t V = g.V;
#pragma unroll
  for (int e = 0; e < 9; ++e) dst[((size_t)mu * 9 + e) * V + s] = src[((size_t)mu * V + s) * 9 + e];
}

// [n][V][nc] <-> [n][nc][V]
template <class T>
__global__ __launch_bounds__(kBlock) void k_site_major_to_comp_major(Geom g, const T* __restrict__ src,
                                                                     T* __restrict__ dst) {
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const size_t V = g.V, j = blockIdx.y, nc = g.ncomp;
  for (size_t c = 0; c < nc; ++c) dst[(j * nc + c) * V + s] = src[(j * V + s) * nc + c];
}
template <class T>
__global__ __launch_bounds__(kBlock) void k_comp_major_to_site_major(Geom g, const T* __restrict__ src,
                                                                     T* __restrict__ dst) {
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const size_t V = g.V, j = blockIdx.y, nc = g.ncomp;
  for (size_t c = 0; c < nc; ++c) dst[(j * V + s) * nc + c] = src[(j * nc + c) * V + s];
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------

static inline dim3 site_grid(const Geom& g, unsigned y) { return dim3((g.V + kBlock - 1) / kBlock, y); }

hipError_t launch_matvec(const OpDev& op, const Geom& g, Elem elem, int R, int B, const void* in, void* out,
                         double* partial, const int* active, int* ran, hipStream_t st) {
  const dim3 grid = site_grid(g, B / R);
  if (op.kind == 1) {
    const double2* U = (const double2*)op.links;
    const double2* x = (const double2*)in;
    double2* y = (double2*)out;
    switch (R) {
      case 1: k_cov_matvec<1><<<grid, kBlock, 0, st>>>(g, U, op.mass_field, op.mass, op.coupling, x, y, partial, active, ran); break;
      case 2: k_cov_matvec<2><<<grid, kBlock, 0, st>>>(g, U, op.mass_field, op.mass, op.coupling, x, y, partial, active, ran); break;
      case 4: k_cov_matvec<4><<<grid, kBlock, 0, st>>>(g, U, op.mass_field, op.mass, op.coupling, x, y, partial, active, ran); break;
      case 8: k_cov_matvec<8><<<grid, kBlock, 0, st>>>(g, U, op.mass_field, op.mass, op.coupling, x, y, partial, active, ran); break;
      default: return hipErrorInvalidValue;
    }
  } else if (elem == Elem::kReal) {
    const double* x = (const double*)in;
    double* y = (double*)out;
    switch (R) {
      case 1: k_scalar_matvec<double, 1><<<grid, kBlock, 0, st>>>(g, op.mass_field, op.mass, op.coupling, x, y, partial, active, ran); break;
      case 2: k_scalar_matvec<double, 2><<<grid, kBlock, 0, st>>>(g, op.mass_field, op.mass, op.coupling, x, y, partial, active, ran); break;
      case 4: k_scalar_matvec<double, 4><<<grid, kBlock, 0, st>>>(g, op.mass_field, op.mass, op.coupling, x, y, partial, active, ran); break;
      case 8: k_scalar_matvec<double, 8><<<grid, kBlock, 0, st>>>(g, op.mass_field, op.mass, op.coupling, x, y, partial, active, ran); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    const double2* x = (const double2*)in;
    double2* y = (double2*)out;
    switch (R) {
      case 1: k_scalar_matvec<double2, 1><<<grid, kBlock, 0, st>>>(g, op.mass_field, op.mass, op.coupling, x, y, partial, active, ran); break;
      case 2: k_scalar_matvec<double2, 2><<<grid, kBlock, 0, st>>>(g, op.mass_field, op.mass, op.coupling, x, y, partial, active, ran); break;
      case 4: k_scalar_matvec<double2, 4><<<grid, kBlock, 0, st>>>(g, op.mass_field, op.mass, op.coupling, x, y, partial, active, ran); break;
      case 8: k_scalar_matvec<double2, 8><<<grid, kBlock, 0, st>>>(g, op.mass_field, op.mass, op.coupling, x, y, partial, active, ran); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_true_residual(const OpDev& op, const Geom& g, Elem elem, int R, int B, int64_t rhs0, int nb,
                                uint64_t seed, int mask, const void* x, void* r, void* p, double* partial,
                                size_t pstride, hipStream_t st) {
  const dim3 grid = site_grid(g, B / R);
  if (op.kind == 1) {
    const double2* U = (const double2*)op.links;
    auto X = (const double2*)x;
    auto Rr = (double2*)r;
    auto Pp = (double2*)p;
#define TIP_TR(RR) k_cov_true_residual<RR><<<grid, kBlock, 0, st>>>(g, U, op.mass_field, op.mass, op.coupling, rhs0, nb, seed, mask, X, Rr, Pp, partial, pstride)
    switch (R) {
      case 1: TIP_TR(1); break;
      case 2: TIP_TR(2); break;
      case 4: TIP_TR(4); break;
      case 8: TIP_TR(8); break;
      default: return hipErrorInvalidValue;
    }
#undef TIP_TR
  } else if (elem == Elem::kReal) {
    auto X = (const double*)x;
    auto Rr = (double*)r;
    auto Pp = (double*)p;
#define TIP_TR(RR) k_scalar_true_residual<double, RR><<<grid, kBlock, 0, st>>>(g, op.mass_field, op.mass, op.coupling, rhs0, nb, seed, mask, X, Rr, Pp, partial, pstride)
    switch (R) {
      case 1: TIP_TR(1); break;
      case 2: TIP_TR(2); break;
      case 4: TIP_TR(4); break;
      case 8: TIP_TR(8); break;
      default: return hipErrorInvalidValue;
    }
#undef TIP_TR
  } else {
    auto X = (const double2*)x;
    auto Rr = (double2*)r;
    auto Pp = (double2*)p;
#define TIP_TR(RR) k_scalar_true_residual<double2, RR><<<grid, kBlock, 0, st>>>(g, op.mass_field, op.mass, op.coupling, rhs0, nb, seed, mask, X, Rr, Pp, partial, pstride)
    switch (R) {
      case 1: TIP_TR(1); break;
      case 2: TIP_TR(2); break;
      case 4: TIP_TR(4); break;
      case 8: TIP_TR(8); break;
      default: return hipErrorInvalidValue;
    }
#undef TIP_TR
  }
  return hipGetLastError();
}

hipError_t launch_init(const Geom& g, Elem elem, int B, int64_t rhs0, int nb, uint64_t seed, int mask, void* x,
                       void* r, void* p, hipStream_t st) {
  const dim3 grid = site_grid(g, B);
  if (elem == Elem::kReal)
    k_init<double><<<grid, kBlock, 0, st>>>(g, rhs0, nb, seed, mask, (double*)x, (double*)r, (double*)p);
  else
    k_init<double2><<<grid, kBlock, 0, st>>>(g, rhs0, nb, seed, mask, (double2*)x, (double2*)r, (double2*)p);
  return hipGetLastError();
}

hipError_t launch_update(const Geom& g, Elem elem, int B, const CgScalars& sc, void* x, void* r, const void* p,
                         const void* Ap, double* partial, hipStream_t st) {
  const dim3 grid = site_grid(g, B);
  if (elem == Elem::kReal)
    k_update<double><<<grid, kBlock, 0, st>>>(g, sc, (double*)x, (double*)r, (const double*)p, (const double*)Ap, partial);
  else
    k_update<double2><<<grid, kBlock, 0, st>>>(g, sc, (double2*)x, (double2*)r, (const double2*)p, (const double2*)Ap, partial);
  return hipGetLastError();
}

hipError_t launch_direction(const Geom& g, Elem elem, int B, const CgScalars& sc, const void* r, void* p,
                            hipStream_t st) {
  const dim3 grid = site_grid(g, B);
  if (elem == Elem::kReal)
    k_direction<double><<<grid, kBlock, 0, st>>>(g, sc, (const double*)r, (double*)p);
  else
    k_direction<double2><<<grid, kBlock, 0, st>>>(g, sc, (const double2*)r, (double2*)p);
  return hipGetLastError();
}

hipError_t launch_scalars_init(const CgScalars& sc, int nb, int B, double bnorm2, int start_frozen, hipStream_t st) {
  k_scalars_init<<<(B + 255) / 256, 256, 0, st>>>(sc, nb, B, bnorm2, start_frozen);
  return hipGetLastError();
}

hipError_t launch_reduce_alpha(const CgScalars& sc, int B, const double* partial, int gx, hipStream_t st) {
  k_reduce_alpha<<<B, kBlock, 0, st>>>(sc, partial, gx);
  return hipGetLastError();
}

hipError_t launch_reduce_beta(const CgScalars& sc, int B, const double* partial, int gx, double tol2, int max_iter,
                              hipStream_t st) {
  k_reduce_beta<<<B, kBlock, 0, st>>>(sc, partial, gx, tol2, max_iter);
  return hipGetLastError();
}

hipError_t launch_reduce_true(const CgScalars& sc, int B, const double* partial, int gx, size_t pstride, double tol2,
                              int max_iter, int max_restarts, hipStream_t st) {
  k_reduce_true<<<B, kBlock, 0, st>>>(sc, partial, gx, pstride, tol2, max_iter, max_restarts);
  return hipGetLastError();
}

hipError_t launch_hier_perm(const Geom& g, uint32_t* out, hipStream_t st) {
  k_hier_perm<<<site_grid(g, 1), kBlock, 0, st>>>(g, out);
  return hipGetLastError();
}

hipError_t launch_probe_vectors(const Geom& g, uint64_t seed, int mask, int64_t m0, int count, int comp, double2* out,
                                hipStream_t st) {
  k_probe_vectors<<<site_grid(g, count), kBlock, 0, st>>>(g, seed, mask, m0, comp, out);
  return hipGetLastError();
}

hipError_t launch_repack_links(const Geom& g, const double2* src, double2* dst, hipStream_t st) {
  k_repack_links<<<site_grid(g, g.ndim), kBlock, 0, st>>>(g, src, dst);
  return hipGetLastError();
}

hipError_t launch_layout(const Geom& g, Elem elem, int n, const void* src, void* dst, bool to_comp_major,
                         hipStream_t st) {
  const dim3 grid = site_grid(g, n);
  if (elem == Elem::kReal) {
    if (to_comp_major) k_site_major_to_comp_major<double><<<grid, kBlock, 0, st>>>(g, (const double*)src, (double*)dst);
    else k_comp_major_to_site_major<double><<<grid, kBlock, 0, st>>>(g, (const double*)src, (double*)dst);
  } else {
    if (to_comp_major) k_site_major_to_comp_major<double2><<<grid, kBlock, 0, st>>>(g, (const double2*)src, (double2*)dst);
    else k_comp_major_to_site_major<double2><<<grid, kBlock, 0, st>>>(g, (const double2*)src, (double2*)dst);
  }
  return hipGetLastError();
}

}  // namespace tip
