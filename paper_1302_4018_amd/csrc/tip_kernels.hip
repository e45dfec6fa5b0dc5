// HIP kernels of libtip for gfx950 (MI355X).
//
// Data layout in HBM (site index s = x1 + n1 (x2 + n2 (x3 + n3 x4))):
//   vectors   a block of B right-hand sides (B a power of two <= 64) is one
//             array [ncomp][V][B] of T (T = double for real scalar problems,
//             double2 = (re, im) otherwise): right-hand side fastest.  A
//             thread owns one (site, rhs) pair, the B lanes of a site are
//             adjacent, so a wave reads 64/B sites x B rhs as one contiguous
//             1 KiB (or 512 B) run and every per-site operand (links,
//             couplings, mass) is one address shared by B lanes;
//   links     [ndim][9][V] double2: element (a, b) of U_mu(s) at [mu][3a+b][s];
//   coupling  [ndim][V] double, mass_field [V] double (caller layout).
//
// The stencil marches along the last lattice dimension ("t"): a workgroup
// owns a tile of 256/B sites of the other dimensions and a chunk of t values.
// Each t-link is read once and used twice (forward hop of t, and the
// backward hop of t+1, carried in registers), x(t-1), x(t), x(t+1) stay in
// registers, and tiles are ordered so that one XCD keeps a contiguous slab
// of tiles in flight (neighbour loads then hit its own L2).
//
// CG (Hestenes-Stiefel, per right-hand side j) uses three passes per
// iteration, with one-workgroup-per-RHS reductions in between:
//   matvec:  w = A p, partial p^H w            -> alpha = rho / p^H w
//   update:  r -= alpha w, partial ||r||^2     -> beta = rho' / rho
//   direct:  x += alpha p; p = r + beta p
// All reductions are two-stage and deterministic: each workgroup writes one
// partial per right-hand side and a second kernel sums them in a fixed
// order.  No floating-point atomics are used.

#include <algorithm>

#include "tip_device.h"
#include "tip_kernel_common.h"
#include "tip_launch.h"

namespace tip {

// ---------------------------------------------------------------------------
// Stencil kernels
// ---------------------------------------------------------------------------

// Generic stencil, one (site, rhs) per thread: out = A in for lanes whose rhs
// is live (state == kActive, or every lane when state is null); partial[j][bx]
// = Re(in_j^H out_j) over the tile.
template <class Op>
__global__ __launch_bounds__(kBlock) void k_stencil(Geom g, TileMap tm, Op op, const double* __restrict__ mass_field,
                                                    double mass, const double* __restrict__ w, const int* __restrict__ state,
                                                    const int* __restrict__ active, const typename Op::T* __restrict__ in,
                                                    typename Op::T* __restrict__ out, double* __restrict__ partial,
                                                    int* __restrict__ ran) {
  using T = typename Op::T;
  constexpr int NC = Op::NC;
  if (active && *active == 0) return;
  if (ran && blockIdx.x == 0 && threadIdx.x == 0) *ran = 1;
  __shared__ double lds[4 * 64];
  const int B = 1 << tm.logB;
  const int j = threadIdx.x & (B - 1);
  const uint32_t s = tile_first_site(blockIdx.x, tm) + (threadIdx.x >> tm.logB);
  double dot[1] = {0.0};
  if (s < g.V && (!state || state[j] == kActive)) {
    T xs[NC], y[NC];
    stencil_site(op, g, tm.logB, s, j, mass_field, mass, w, in, xs, y);
    store_vec<T, NC>(out, g.V, tm.logB, s, j, y);
#pragma unroll
    for (int c = 0; c < NC; ++c) dot[0] += redot(xs[c], y[c]);
  }
  if (partial) {
    seg_sum<1>(dot, B, lds);
    if ((int)threadIdx.x < B) partial[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = dot[0];
  }
}

// Marching stencil (ndim >= 2): workgroup b owns spatial tile q (TS sites of
// the first ndim-1 dimensions, V3 = V / n_t sites per t-plane) and the t
// values [c Tc, (c+1) Tc).  Same arithmetic, same summation order as
// stencil_site.
//
// kLdsLinks (covariant operator): at every t the workgroup first copies the
// links its TS sites use -- the forward link of every dimension and the
// backward link U_mu(s-mu) of every marched-over dimension -- into LDS with
// one coalesced 16-byte load per element, then the B lanes of a site read
// them from there.  Without it every lane would fetch the 3x3 matrices
// itself, so the L1 would deliver each link B times.
template <class Op, bool kLdsLinks, int kLogB = -1, int kHasW = -1>
__global__ __launch_bounds__(kBlock) void k_stencil_march(Geom g, MarchMap mm, Op op,
                                                          const double* __restrict__ mass_field, double mass,
                                                          const double* __restrict__ w, const int* __restrict__ state,
                                                          const int* __restrict__ active,
                                                          const typename Op::T* __restrict__ in,
                                                          typename Op::T* __restrict__ out,
                                                          double* __restrict__ partial, int* __restrict__ ran) {
  using T = typename Op::T;
  constexpr int NC = Op::NC;
  if (active && *active == 0) return;
  if (ran && blockIdx.x == 0 && threadIdx.x == 0) *ran = 1;
  __shared__ double lds[4 * 64];
  // [2 ndim - 1][9][TS] link elements when kLdsLinks
  T* lds_links = reinterpret_cast<T*>(tip_dyn_lds);
  // kLogB >= 0 / kHasW >= 0 fix the block size / the presence of couplings at
  // compile time (LDS offsets become immediates, unit weights disappear)
  const int logB = kLogB >= 0 ? kLogB : mm.logB;
  const int B = 1 << logB;
  const int TS = kBlock >> logB;
  if (kHasW == 0) w = nullptr;
  const int j = threadIdx.x & (B - 1);
  const int si = threadIdx.x >> logB;
  uint32_t q, chunk;
  march_tile(mm, blockIdx.x, q, chunk);
  const uint32_t s3_first = q * (uint32_t)TS;
  const uint32_t s3 = s3_first + (uint32_t)si;
  const size_t V = g.V;
  const uint32_t V3 = mm.V3;
  const int nt = mm.nt;
  const int mt = g.ndim - 1;                      // marching dimension
  const bool live = !state || state[j] == kActive;
  const int t0 = (int)chunk * mm.Tc;
  double dot[1] = {0.0};
  T carry[NC], xc[NC];
  double wprev = 1.0;
  if (live) {
    // prologue: x(t0-1) and the link from t0-1 give the backward t hop of t0
    const int tp = t0 == 0 ? nt - 1 : t0 - 1;
    const uint32_t sp = s3 + V3 * (uint32_t)tp;
    T xp[NC];
    load_vec<T, NC>(in, V, logB, sp, j, xp);
    hop_term(op, V, mt, sp, true, xp, carry);
    wprev = w ? w[(size_t)mt * V + sp] : 1.0;
    load_vec<T, NC>(in, V, logB, s3 + V3 * (uint32_t)t0, j, xc);
  }
  for (int t = t0; t < t0 + mm.Tc; ++t) {
    const uint32_t s = s3 + V3 * (uint32_t)t;
    if constexpr (kLdsLinks) {
      // every thread helps to stage the tile's links, live or not
      const int nitems = (2 * g.ndim - 1) * 9 * TS;
      __syncthreads();
      for (int it = threadIdx.x; it < nitems; it += kBlock) {
        const int site = it & (TS - 1);
        const int es = it >> (8 - logB);          // it / TS
        const int e = es % 9;
        const int slot = es / 9;
        const uint32_t ss = s3_first + (uint32_t)site + V3 * (uint32_t)t;
        const int mu = slot < g.ndim ? slot : slot - g.ndim;
        const uint32_t sl = slot < g.ndim ? ss : nbr_bwd_p2(ss, g, mu);
        lds_links[it] = op.U[((size_t)mu * 9 + e) * V + sl];
      }
      __syncthreads();
    }
    if (!live) continue;
    const uint32_t sn = s3 + V3 * (uint32_t)(t + 1 == nt ? 0 : t + 1);
    T hop[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) hop[c] = zero<T>();
    double diag = mass_field ? mass_field[s] : mass;
    for (int mu = 0; mu < mt; ++mu) {
      const uint32_t sf = nbr_fwd_p2(s, g, mu);
      const uint32_t sb = nbr_bwd_p2(s, g, mu);
      const double wf = w ? w[(size_t)mu * V + s] : 1.0;
      const double wb = w ? w[(size_t)mu * V + sb] : 1.0;
      diag += wf + wb;
      T xn[NC], h[NC];
      load_vec<T, NC>(in, V, logB, sf, j, xn);
      if constexpr (kLdsLinks) {
        T u[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = lds_links[(mu * 9 + e) * TS + si];
        mul_u(u, xn, h);
      } else {
        hop_term(op, V, mu, s, false, xn, h);
      }
      add_weighted<T, NC>(wf, h, hop);
      load_vec<T, NC>(in, V, logB, sb, j, xn);
      if constexpr (kLdsLinks) {
        T u[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = lds_links[((g.ndim + mu) * 9 + e) * TS + si];
        mul_uh(u, xn, h);
      } else {
        hop_term(op, V, mu, sb, true, xn, h);
      }
      add_weighted<T, NC>(wb, h, hop);
    }
    // t direction: forward hop with the link of s, backward hop carried
    const double wt = w ? w[(size_t)mt * V + s] : 1.0;
    diag += wt + wprev;
    T xn[NC], h[NC];
    load_vec<T, NC>(in, V, logB, sn, j, xn);
    if constexpr (NC == 3) {
      T u[9];
      if constexpr (kLdsLinks) {
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = lds_links[(mt * 9 + e) * TS + si];
      } else {
        load_link(op, V, mt, s, u);
      }
      mul_u(u, xn, h);
      add_weighted<T, NC>(wt, h, hop);
      add_weighted<T, NC>(wprev, carry, hop);
      mul_uh(u, xc, carry);                    // backward hop of t+1
    } else {
      add_weighted<T, NC>(wt, xn, hop);
      add_weighted<T, NC>(wprev, carry, hop);
      carry[0] = xc[0];
    }
    wprev = wt;
    T y[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      y[c] = axpy(diag, xc[c], axpy(-1.0, hop[c], zero<T>()));
      dot[0] += redot(xc[c], y[c]);
    }
    store_vec<T, NC>(out, V, logB, s, j, y);
#pragma unroll
    for (int c = 0; c < NC; ++c) xc[c] = xn[c];
  }
  if (partial) {
    seg_sum<1>(dot, B, lds);
    if ((int)threadIdx.x < B) partial[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = dot[0];
  }
}

// 4-D covariant marching stencil, specialised: the three marched-over
// dimensions are unrolled, each thread's spatial neighbour offsets are fixed
// for the whole march (its x, y, z never change), and every global access is
// a kernel-argument base plus a 32-bit byte offset (the host checks that all
// arrays fit), so the loop body is the 3x3 complex algebra plus little
// address arithmetic.  Same arithmetic and summation order as stencil_site.
template <class C>
__device__ __forceinline__ C ld_off(const C* __restrict__ base, uint32_t byte_off) {
  return *reinterpret_cast<const C*>(reinterpret_cast<const char*>(base) + byte_off);
}
#ifndef TIP_STENCIL_NT_STORE
#define TIP_STENCIL_NT_STORE 1
#endif
template <class C>
__device__ __forceinline__ void st_off(C* __restrict__ base, uint32_t byte_off, C v) {
  if constexpr (TIP_STENCIL_NT_STORE) {
    // streaming store: the written line is not kept in L2 for reuse
    auto* d = reinterpret_cast<decltype(v.x)*>(reinterpret_cast<char*>(base) + byte_off);
    __builtin_nontemporal_store(v.x, d);
    __builtin_nontemporal_store(v.y, d + 1);
  } else {
    *reinterpret_cast<C*>(reinterpret_cast<char*>(base) + byte_off) = v;
  }
}
__device__ __forceinline__ double ld_offd(const double* __restrict__ base, uint32_t byte_off) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + byte_off);
}

#ifndef TIP_MARCH4_WAVES
#define TIP_MARCH4_WAVES 1
#endif
template <class C, int LOGB, bool HASW>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(TIP_MARCH4_WAVES))) void k_stencil_march4(Geom g, MarchMap mm, const C* __restrict__ U,
                                                           const double* __restrict__ mass_field, double mass,
                                                           const double* __restrict__ w,
                                                           const int* __restrict__ state,
                                                           const int* __restrict__ active, const C* __restrict__ in,
                                                           C* __restrict__ out, double* __restrict__ partial,
                                                           int* __restrict__ ran) {
  constexpr int B = 1 << LOGB;
  constexpr int TS = kBlock >> LOGB;
  constexpr int SZ = (int)sizeof(C);
  constexpr int NSLOT = 7;                        // 4 forward links + 3 backward (x, y, z)
  if (active && *active == 0) return;
  if (ran && blockIdx.x == 0 && threadIdx.x == 0) *ran = 1;
  __shared__ double lds[4 * 64];
  C* lds_links = reinterpret_cast<C*>(tip_dyn_lds);   // [7][9][TS]
  const int j = threadIdx.x & (B - 1);
  const int si = threadIdx.x >> LOGB;
  uint32_t q, chunk;
  march_tile(mm, blockIdx.x, q, chunk);
  const uint32_t V = g.V;
  const uint32_t V3 = mm.V3;
  const uint32_t s3_first = q * (uint32_t)TS;
  const uint32_t s3 = s3_first + (uint32_t)si;
  const uint32_t cstride = (V << LOGB) * SZ;      // bytes between components
  const uint32_t lstride = V * SZ;                // bytes between link elements
  // fixed spatial neighbour offsets (in sites) of this thread
  int32_t dfw[3], dbw[3];
#pragma unroll
  for (int mu = 0; mu < 3; ++mu) {
    const uint32_t n = 1u << g.logn[mu], stride = 1u << g.shift[mu];
    const uint32_t x = (s3 >> g.shift[mu]) & (n - 1u);
    dfw[mu] = x == n - 1u ? -(int32_t)((n - 1u) * stride) : (int32_t)stride;
    dbw[mu] = x == 0u ? (int32_t)((n - 1u) * stride) : -(int32_t)stride;
  }
  auto vec_off = [&](uint32_t site) -> uint32_t { return ((site << LOGB) + (uint32_t)j) * SZ; };
  const bool live = !state || state[j] == kActive;
  const int nt = mm.nt;
  const int t0 = (int)chunk * mm.Tc;
  double dot[1] = {0.0};
  C carry[3], xc[3];
  double wprev = 1.0;
  if (live) {
    const int tp = t0 == 0 ? nt - 1 : t0 - 1;
    const uint32_t sp = s3 + V3 * (uint32_t)tp;
    C u[9], xp[3];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = ld_off(U, (27u + (uint32_t)e) * lstride + sp * SZ);
#pragma unroll
    for (int c = 0; c < 3; ++c) xp[c] = ld_off(in, c * cstride + vec_off(sp));
    mul_uh(u, xp, carry);
    if constexpr (HASW) wprev = ld_offd(w, (3u * V + sp) * 8u);
#pragma unroll
    for (int c = 0; c < 3; ++c) xc[c] = ld_off(in, c * cstride + vec_off(s3 + V3 * (uint32_t)t0));
  }
  for (int t = t0; t < t0 + mm.Tc; ++t) {
    const uint32_t s = s3 + V3 * (uint32_t)t;
    // stage the tile's links: slots 0..3 forward U_mu(s), 4..6 backward U_mu(s - mu)
    __syncthreads();
    for (int it = threadIdx.x; it < NSLOT * 9 * TS; it += kBlock) {
      const int site = it & (TS - 1);
      const int es = it >> (8 - LOGB);
      const int e = es % 9;
      const int slot = es / 9;
      const uint32_t ss = s3_first + (uint32_t)site + V3 * (uint32_t)t;
      uint32_t sl = ss;
      int mu = slot;
      if (slot >= 4) {
        mu = slot - 4;
        const uint32_t n = 1u << g.logn[mu], stride = 1u << g.shift[mu];
        sl = ((ss >> g.shift[mu]) & (n - 1u)) == 0u ? ss + (n - 1u) * stride : ss - stride;
      }
      lds_links[it] = ld_off(U, ((uint32_t)mu * 9u + (uint32_t)e) * lstride + sl * SZ);
    }
    __syncthreads();
    if (!live) continue;
    const uint32_t sn = s3 + V3 * (uint32_t)(t + 1 == nt ? 0 : t + 1);
    C hop[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) hop[c] = zero<C>();
    double diag = mass_field ? ld_offd(mass_field, s * 8u) : mass;
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
      const uint32_t sf = (uint32_t)((int32_t)s + dfw[mu]);
      const uint32_t sb = (uint32_t)((int32_t)s + dbw[mu]);
      double wf = 1.0, wb = 1.0;
      if constexpr (HASW) {
        wf = ld_offd(w, ((uint32_t)mu * V + s) * 8u);
        wb = ld_offd(w, ((uint32_t)mu * V + sb) * 8u);
      }
      diag += wf + wb;
      C xn[3], h[3], u[9];
#pragma unroll
      for (int c = 0; c < 3; ++c) xn[c] = ld_off(in, c * cstride + vec_off(sf));
#pragma unroll
      for (int e = 0; e < 9; ++e) u[e] = lds_links[(mu * 9 + e) * TS + si];
      mul_u(u, xn, h);
      add_weighted<C, 3>(wf, h, hop);
#pragma unroll
      for (int c = 0; c < 3; ++c) xn[c] = ld_off(in, c * cstride + vec_off(sb));
#pragma unroll
      for (int e = 0; e < 9; ++e) u[e] = lds_links[((4 + mu) * 9 + e) * TS + si];
      mul_uh(u, xn, h);
      add_weighted<C, 3>(wb, h, hop);
    }
    double wt = 1.0;
    if constexpr (HASW) wt = ld_offd(w, (3u * V + s) * 8u);
    diag += wt + wprev;
    C xn[3], h[3], u[9];
#pragma unroll
    for (int c = 0; c < 3; ++c) xn[c] = ld_off(in, c * cstride + vec_off(sn));
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = lds_links[(3 * 9 + e) * TS + si];
    mul_u(u, xn, h);
    add_weighted<C, 3>(wt, h, hop);
    add_weighted<C, 3>(wprev, carry, hop);
    mul_uh(u, xc, carry);
    wprev = wt;
    C y[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      y[c] = axpy(diag, xc[c], axpy(-1.0, hop[c], zero<C>()));
      dot[0] += redot(xc[c], y[c]);
      st_off(out, c * cstride + vec_off(s), y[c]);
      xc[c] = xn[c];
    }
  }
  if (partial) {
    seg_sum<1>(dot, B, lds);
    if ((int)threadIdx.x < B) partial[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = dot[0];
  }
}

// ---------------------------------------------------------------------------
// CG vector passes over the flat block [ncomp][V][B]: element i has rhs i mod B.
// ---------------------------------------------------------------------------

// r -= alpha w for active right-hand sides; partial = ||r||^2.  Grid-stride:
// the stride is a multiple of 256, so a thread always meets the same rhs and
// the number of partials per rhs is the (moderate) grid size.
#ifndef TIP_UPD_UNROLL
#define TIP_UPD_UNROLL 4
#endif
template <class T>
__global__ __launch_bounds__(kBlock) void k_update_r(size_t n, int logB, const CgScalars sc, T* __restrict__ r,
                                                     const T* __restrict__ Ap, double* __restrict__ partial) {
  __shared__ double lds[4 * 64];
  const int B = 1 << logB;
  const int j = threadIdx.x & (B - 1);
  double acc[1] = {0.0};
  if (sc.state[j] == kActive) {
    const double a = sc.alpha[j];
    const size_t stride = (size_t)gridDim.x * kBlock;
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    constexpr int U = TIP_UPD_UNROLL;
    for (; i + (U - 1) * stride < n; i += U * stride) {      // U independent loads in flight
      T rr[U], ww[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        rr[k] = r[i + k * stride];
        ww[k] = Ap[i + k * stride];
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        rr[k] = axpy(-a, ww[k], rr[k]);
        r[i + k * stride] = rr[k];
        acc[0] += norm2(rr[k]);
      }
    }
    for (; i < n; i += stride) {
      const T ri = axpy(-a, Ap[i], r[i]);
      r[i] = ri;
      acc[0] += norm2(ri);
    }
  }
  seg_sum<1>(acc, B, lds);
  if ((int)threadIdx.x < B) partial[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = acc[0];
}

// x += xalpha p (the update of this iteration, also for a rhs that just
// converged); p = r + beta p for right-hand sides still iterating.
template <class T>
__global__ __launch_bounds__(kBlock) void k_direction(size_t n, int logB, const CgScalars sc, T* __restrict__ x,
                                                      const T* __restrict__ r, T* __restrict__ p) {
  const int B = 1 << logB;
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const int j = threadIdx.x & (B - 1);
  if (i >= n) return;
  const double a = sc.xalpha[j];
  const bool live = sc.state[j] == kActive;
  if (a == 0.0 && !live) return;
  const T pi = p[i];
  if (a != 0.0) x[i] = axpy(a, pi, x[i]);
  if (live) p[i] = axpy(sc.beta[j], pi, r[i]);
}

// ---------------------------------------------------------------------------
// Right-hand sides, initial state and the true residual.  Lane j of the block
// is global right-hand side rhs0 + j: spatial probe m = (rhs0 + j) / ncomp
// (through class_probe when the call solves one class of probes),
// component c = (rhs0 + j) % ncomp.
// ---------------------------------------------------------------------------

// Parity of the first ndim-1 coordinates of a site (or of a spatial index);
// power-of-two sides (the even-odd kernels run only there).
__device__ __forceinline__ uint32_t spatial_parity(uint32_t s3, const Geom& g) {
  uint32_t sum = 0;
#pragma unroll
  for (int mu = 0; mu < kMaxDim - 1; ++mu)
    if (mu < g.ndim - 1) sum += coord_p2(s3, g, mu);
  return sum & 1u;
}

// x = 0, r = p = b for every lane (zero for padding lanes j >= nb).
template <class T, int NC>
__global__ __launch_bounds__(kBlock) void k_init(Geom g, int logB, int64_t rhs0, int nb, uint64_t seed, int mask,
                                                 T* __restrict__ x, T* __restrict__ r, T* __restrict__ p) {
  const int B = 1 << logB;
  const int j = threadIdx.x & (B - 1);
  const uint32_t s = blockIdx.x * (kBlock >> logB) + (threadIdx.x >> logB);
  if (s >= g.V) return;
  T b[NC], z[NC];
  rhs_at<T, NC>(g, s, rhs0, j, nb, seed, mask, b);
#pragma unroll
  for (int c = 0; c < NC; ++c) z[c] = zero<T>();
  store_vec<T, NC>(x, g.V, logB, s, j, z);
  store_vec<T, NC>(r, g.V, logB, s, j, b);
  store_vec<T, NC>(p, g.V, logB, s, j, b);
}

// For lanes in state kFrozen: rt = b - A x in FP64 with b regenerated;
// r = p = rt.  partial[k] (k = 0, 1, 2): ||rt||^2, Re b^H x, Im b^H x.
template <class Op>
__global__ __launch_bounds__(kBlock) void k_true_residual(Geom g, TileMap tm, Op op,
                                                          const double* __restrict__ mass_field, double mass,
                                                          const double* __restrict__ w, const int* __restrict__ state,
                                                          int64_t rhs0, int nb, uint64_t seed, int mask,
                                                          const typename Op::T* __restrict__ x,
                                                          typename Op::T* __restrict__ r, typename Op::T* __restrict__ p,
                                                          double* __restrict__ partial, size_t pstride) {
  using T = typename Op::T;
  constexpr int NC = Op::NC;
  __shared__ double lds[3 * 4 * 64];
  const int B = 1 << tm.logB;
  const int j = threadIdx.x & (B - 1);
  double acc[3] = {0.0, 0.0, 0.0};
  // grid-stride over the tiles: one partial per workgroup, so the reduction
  // that follows reads gridDim.x values per rhs, not one per tile
  for (uint32_t tile = blockIdx.x; tile < tm.grid && state[j] == kFrozen; tile += gridDim.x) {
    const uint32_t s = tile_first_site(tile, tm) + (threadIdx.x >> tm.logB);
    if (s >= g.V) continue;
    T xs[NC], ax[NC], b[NC], rt[NC];
    stencil_site(op, g, tm.logB, s, j, mass_field, mass, w, x, xs, ax);
    rhs_at<T, NC>(g, s, rhs0, j, nb, seed, mask, b);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      rt[c] = axpy(-1.0, ax[c], b[c]);
      acc[0] += norm2(rt[c]);
      acc[1] += redot(b[c], xs[c]);
      acc[2] += imdot(b[c], xs[c]);
    }
    store_vec<T, NC>(r, g.V, tm.logB, s, j, rt);
    store_vec<T, NC>(p, g.V, tm.logB, s, j, rt);
  }
  seg_sum<3>(acc, B, lds);
  if ((int)threadIdx.x < B) {
#pragma unroll
    for (int k = 0; k < 3; ++k) partial[k * pstride + (size_t)threadIdx.x * gridDim.x + blockIdx.x] = acc[k];
  }
}

// ---------------------------------------------------------------------------
// Scalar bookkeeping of CG, one workgroup per right-hand side.
// ---------------------------------------------------------------------------

__global__ void k_scalars_init(CgScalars sc, int nb, int B, double bnorm2, int start_frozen) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) {
    *sc.active = start_frozen ? 0 : nb;
    *sc.n_ru = 0;
    *sc.ru_count = 0;
  }
  if (j >= B) return;
  const bool valid = j < nb;
  sc.state[j] = valid ? (start_frozen ? kFrozen : kActive) : kPadding;
  sc.bnorm2[j] = valid ? bnorm2 : 0.0;
  sc.rho[j] = valid ? bnorm2 : 0.0;
  sc.alpha[j] = 0.0;
  sc.xalpha[j] = 0.0;
  sc.beta[j] = 0.0;
  sc.rho_ref[j] = valid ? bnorm2 : 0.0;
  sc.pp[j] = valid ? bnorm2 : 0.0;
  sc.anorm[j] = 0.0;
  sc.xhn[j] = 0.0;
  sc.dev[j] = 0.0;
  sc.ru[j] = 0;
  sc.iters[j] = 0;
  sc.restarts[j] = 0;
  sc.relres2[j] = 0.0;
  sc.q[2 * j] = 0.0;
  sc.q[2 * j + 1] = 0.0;
}

// alpha = rho / p^H A p (lane_alpha).  force_iter > 0 (tests) treats
// iteration force_iter of a solve that has not restarted as a breakdown.
__global__ __launch_bounds__(kBlock) void k_reduce_alpha(CgScalars sc, const double* __restrict__ partial, int gx,
                                                         int soft, int force_iter) {
  const int j = blockIdx.x;
  if (*sc.active == 0 || sc.state[j] != kActive) return;     // uniform per workgroup
  const bool forced = force_iter > 0 && sc.restarts[j] == 0 && sc.iters[j] + 1 == force_iter;
  const double pAp = sum_partials(partial + (size_t)j * gx, gx);
  if (threadIdx.x != 0) return;
  lane_alpha(sc, j, pAp, soft, forced);
}

// rho' = ||r||^2 over up to 32768 update-pass partials, then lane_beta.
__global__ __launch_bounds__(kWideBlock) void k_reduce_beta(CgScalars sc, const double* __restrict__ partial, int gx,
                                                        double tol2, int max_iter, double delta2, double first2,
                                                        double eps, double tau2) {
  const int j = blockIdx.x;
  if (sc.state[j] != kActive) {                // uniform per workgroup
    if (threadIdx.x == 0) sc.xalpha[j] = 0.0;
    return;
  }
  const BetaIn in = lane_beta_read(sc, j);    // uniform addresses: one load per wave
  const double rho_new = sum_partials_wide(partial + (size_t)j * gx, gx);
  if (threadIdx.x != 0) return;
  lane_beta(sc, j, in, rho_new, tol2, max_iter, delta2, first2, eps, tau2);
}

// Accept a frozen solve when its true residual passes, else restart CG from x.
__global__ __launch_bounds__(kBlock) void k_reduce_true(CgScalars sc, const double* __restrict__ partial,
                                                        const double* __restrict__ partial2, int gx, size_t pstride,
                                                        double tol2, int max_iter, int max_restarts) {
  const int j = blockIdx.x;
  if (threadIdx.x == 0) sc.xalpha[j] = 0.0;
  if (sc.state[j] != kFrozen) return;
  const double rt2 = sum_partials2(partial, partial2, (size_t)j * gx, gx);
  const double qre = sum_partials2(partial, partial2, pstride + (size_t)j * gx, gx);
  const double qim = sum_partials2(partial, partial2, 2 * pstride + (size_t)j * gx, gx);
  if (threadIdx.x != 0) return;
  lane_true(sc, j, rt2, qre, qim, tol2, max_iter, max_restarts);
}

// ---------------------------------------------------------------------------
// Mixed precision: CG in FP32 (links and vectors stored and combined in
// single precision) with FP64 reliable updates (Sleijpen & van der Vorst,
// Computing 56 (1996) 141): when the FP32 recursive residual has fallen by
// the factor delta since the last update, x (FP64) absorbs the FP32
// correction and the residual is recomputed from x with the FP64 operator.
// The final acceptance is the same FP64 true-residual test as in plain FP64.
// Lanes are selected by mode: 0 = flagged for a reliable update and still
// iterating, 1 = frozen (final check).
// ---------------------------------------------------------------------------

// x64 = 0, xh = 0, rh = ph = b (exact in single precision).
template <class T64, class T32, int NC>
__global__ __launch_bounds__(kBlock) void k_init_mixed(Geom g, int logB, int64_t rhs0, int nb, uint64_t seed,
                                                       int mask, T64* __restrict__ x, T32* __restrict__ xh,
                                                       T32* __restrict__ rh, T32* __restrict__ ph) {
  const int B = 1 << logB;
  const int j = threadIdx.x & (B - 1);
  const uint32_t s = blockIdx.x * (kBlock >> logB) + (threadIdx.x >> logB);
  if (s >= g.V) return;
  T32 b[NC], z[NC];
  T64 z64[NC];
  rhs_at<T32, NC>(g, s, rhs0, j, nb, seed, mask, b);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    z[c] = zero<T32>();
    z64[c] = zero<T64>();
  }
  store_vec<T64, NC>(x, g.V, logB, s, j, z64);
  store_vec<T32, NC>(xh, g.V, logB, s, j, z);
  store_vec<T32, NC>(rh, g.V, logB, s, j, b);
  store_vec<T32, NC>(ph, g.V, logB, s, j, b);
}

// x64 += xh, xh = 0 for the selected lanes (flat [ncomp][V][B] elements,
// grid-stride with a stride that is a multiple of 256).  Mode 0 runs after
// every CG iteration and returns at once when no update is pending.
template <class T64, class T32>
__global__ __launch_bounds__(kBlock) void k_ru_accumulate(size_t n, int logB, const CgScalars sc, int mode,
                                                          T64* __restrict__ x, T32* __restrict__ xh) {
  if (mode == 0 && *sc.n_ru == 0) return;
  const int B = 1 << logB;
  const int j = threadIdx.x & (B - 1);
  if (!ru_selected(sc, mode, j)) return;
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    x[i] = axpy(1.0, from_c<T64>(to_c(xh[i])), x[i]);
    xh[i] = zero<T32>();
  }
}

// r = b - A x with the FP64 operator for the selected lanes; rh = r rounded
// to single; in mode 1 also ph = rh (restart direction).  partial[k] for
// k = 0..4: ||r||^2, Re b^H x, Im b^H x, Re x^H r, Im x^H r.
template <class Op64, class T32>
__global__ __launch_bounds__(kBlock) void k_ru_residual(Geom g, TileMap tm, Op64 op,
                                                        const double* __restrict__ mass_field, double mass,
                                                        const double* __restrict__ w, const CgScalars sc, int mode,
                                                        int64_t rhs0, int nb, uint64_t seed, int mask,
                                                        const typename Op64::T* __restrict__ x, T32* __restrict__ rh,
                                                        T32* __restrict__ ph, double* __restrict__ partial,
                                                        size_t pstride) {
  using T = typename Op64::T;
  constexpr int NC = Op64::NC;
  if (mode == 0 && *sc.n_ru == 0) return;
  __shared__ double lds[5 * 4 * 64];
  const int B = 1 << tm.logB;
  const int j = threadIdx.x & (B - 1);
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (ru_selected(sc, mode, j)) {
    // grid-stride over the tiles: one partial per workgroup
    for (uint32_t tile = blockIdx.x; tile < tm.grid; tile += gridDim.x) {
      const uint32_t s = tile_first_site(tile, tm) + (threadIdx.x >> tm.logB);
      if (s >= g.V) continue;
      T xs[NC], ax[NC], b[NC];
      T32 r32[NC];
      stencil_site(op, g, tm.logB, s, j, mass_field, mass, w, x, xs, ax);
      rhs_at<T, NC>(g, s, rhs0, j, nb, seed, mask, b);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const T rt = axpy(-1.0, ax[c], b[c]);
        acc[0] += norm2(rt);
        acc[1] += redot(b[c], xs[c]);
        acc[2] += imdot(b[c], xs[c]);
        acc[3] += redot(xs[c], rt);
        acc[4] += imdot(xs[c], rt);
        r32[c] = to_single(rt);
      }
      store_vec<T32, NC>(rh, g.V, tm.logB, s, j, r32);
      if (mode == 1) store_vec<T32, NC>(ph, g.V, tm.logB, s, j, r32);
    }
  }
  seg_sum<5>(acc, B, lds);
  if ((int)threadIdx.x < B) {
#pragma unroll
    for (int k = 0; k < 5; ++k) partial[k * pstride + (size_t)threadIdx.x * gridDim.x + blockIdx.x] = acc[k];
  }
}

// Sums of the reliable-update pass's five partial rows, then lane_ru.
__global__ __launch_bounds__(kBlock) void k_reduce_ru(CgScalars sc, const double* __restrict__ partial,
                                                      const double* __restrict__ partial2, int gx, size_t pstride,
                                                      int mode, double tol2, int max_iter, int max_restarts) {
  const int j = blockIdx.x;
  if (mode == 0 && *sc.n_ru == 0) return;
  if (!ru_selected(sc, mode, j)) return;      // uniform per workgroup
  double v[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) v[k] = sum_partials2(partial, partial2, k * pstride + (size_t)j * gx, gx);
  if (threadIdx.x != 0) return;
  lane_ru(sc, j, v, mode, tol2, max_iter, max_restarts);
}

// Mixed even-odd start: r = p = single(b_hat), x_h = 0 (flat half vectors).
template <class T64, class T32>
__global__ __launch_bounds__(kBlock) void k_eo_cast_init(size_t n, const T64* __restrict__ bh, T32* __restrict__ r,
                                                         T32* __restrict__ p, T32* __restrict__ xh) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const T32 v = to_single(bh[i]);
  r[i] = v;
  p[i] = v;
  xh[i] = zero<T32>();
}

// FP64 links [ndim][9][V] -> single-precision copy, same layout.
__global__ __launch_bounds__(kBlock) void k_cast_links(size_t n, const double2* __restrict__ src,
                                                       float2* __restrict__ dst) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = make_float2((float)src[i].x, (float)src[i].y);
}

// ---------------------------------------------------------------------------
// Gradient of the estimate with respect to the mass field and the couplings.
// T = (1/s) sum_j b_j^H A^-1 b_j, so with the probes fixed
// dT/dtheta = -(1/s) sum_j b_j^H A^-1 (dA/dtheta) A^-1 b_j = -(1/s) sum_j x_j^H (dA/dtheta) x_j
// (A Hermitian: the adjoint solves are the forward ones).  dA/dm(x) is the
// identity on site x; dA/dw_mu(x) is the edge Laplacian L_e of e = (x, x+mu),
// whose quadratic form is ||x(x) - U_mu(x) x(x+mu)||^2.  One pass per block
// adds the raw sums sum_j x_j^H (dA/dtheta) x_j; the B lanes of a site are
// summed with shuffles and written by one lane, so there are no atomics.
// ---------------------------------------------------------------------------

template <class Op>
__global__ __launch_bounds__(kBlock) void k_grad_accum(Geom g, int logB, int nb, Op op,
                                                       const typename Op::T* __restrict__ x,
                                                       double* __restrict__ gm, double* __restrict__ gw) {
  using T = typename Op::T;
  constexpr int NC = Op::NC;
  const int B = 1 << logB;
  const int j = threadIdx.x & (B - 1);
  const uint32_t s = blockIdx.x * (kBlock >> logB) + (threadIdx.x >> logB);
  if (s >= g.V) return;                                  // whole site groups leave together
  const size_t V = g.V;
  T xs[NC];
  load_vec<T, NC>(x, V, logB, s, j, xs);
  const bool use = j < nb;
  double vm = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) vm += norm2(xs[c]);
  double vw[kMaxDim] = {0.0, 0.0, 0.0, 0.0};
  if (gw) {
    for (int mu = 0; mu < g.ndim; ++mu) {
      T xf[NC], h[NC];
      load_vec<T, NC>(x, V, logB, nbr_fwd(s, g, mu), j, xf);
      hop_term(op, V, mu, s, false, xf, h);          // U_mu(s) x(s+mu)
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < NC; ++c) acc += norm2(axpy(-1.0, h[c], xs[c]));
      vw[mu] = acc;
    }
  }
  if (!use) {
    vm = 0.0;
    for (int mu = 0; mu < kMaxDim; ++mu) vw[mu] = 0.0;
  }
  for (int off = B >> 1; off > 0; off >>= 1) {
    vm += __shfl_down(vm, off, 64);
#pragma unroll
    for (int mu = 0; mu < kMaxDim; ++mu) vw[mu] += __shfl_down(vw[mu], off, 64);
  }
  if (j == 0) {
    if (gm) gm[s] += vm;
    if (gw)
      for (int mu = 0; mu < g.ndim; ++mu) gw[(size_t)mu * V + s] += vw[mu];
  }
}

__global__ __launch_bounds__(kBlock) void k_scale(size_t n, double* __restrict__ a, double f) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) a[i] *= f;
}

__global__ __launch_bounds__(kBlock) void k_fill(size_t n, double* __restrict__ a, double v) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) a[i] = v;
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
  out[(size_t)blockIdx.y * g.V + s] = probe_entry(s, (uint64_t)m, comp, g, seed, mask);
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

// one vector: [V][nc] <-> lane `lane` of the block layout [nc][V][2^logB]
template <class T>
__global__ __launch_bounds__(kBlock) void k_site_major_to_comp_major(Geom g, int logB, int lane,
                                                                     const T* __restrict__ src, T* __restrict__ dst) {
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const size_t V = g.V, nc = g.ncomp;
  for (size_t c = 0; c < nc; ++c) dst[((c * V + s) << logB) + lane] = src[s * nc + c];
}
template <class T>
__global__ __launch_bounds__(kBlock) void k_comp_major_to_site_major(Geom g, int logB, int lane,
                                                                     const T* __restrict__ src, T* __restrict__ dst) {
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const size_t V = g.V, nc = g.ncomp;
  for (size_t c = 0; c < nc; ++c) dst[s * nc + c] = src[((c * V + s) << logB) + lane];
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------

static inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Even-odd (red-black) reduction of A x = b.  With every side even the torus
// is bipartite: A = D - H, D = diag(m(x) + sum_mu [w_mu(x) + w_mu(x - mu)])
// (x) I and the hopping H couples sites of opposite parity only -- the
// red-black colouring of Sec. 2.  Eliminating the odd sites leaves the Schur
// complement
//     S x_e = b_e + H_eo D_o^-1 b_o,   S = D_e - H_eo D_o^-1 H_oe,
// which is Hermitian positive definite and better conditioned than A (for a
// diagonal-dominated A with D^-1 H of spectral radius rho, the condition
// number drops from (1 + rho)/(1 - rho) to 1/(1 - rho^2)), after which
// x_o = D_o^-1 (b_o + H_oe x_e).  With x_o formed this way the full residual
// b - A x is zero on odd sites and equals the reduced residual on even ones,
// so CG on S stopped at ||r_e|| <= tol ||b|| meets the same criterion.
//
// Half-lattice layout: the sites of one parity, numbered h = x + V3 (t >> 1)
// with x the index of the first ndim-1 coordinates (V3 of them) and t the last
// coordinate; vectors are [ncomp][V/2][B].  At fixed x the sites of parity P
// have t = 2 tau + delta(x), delta(x) = (P + |x|) mod 2, |x| the coordinate sum.
// For an output site of parity P at slice tau, its spatial neighbours (parity
// 1 - P) sit in the same slice tau of the input vector and its neighbours
// along t in slices tau + delta (forward) and tau - 1 + delta (backward), so
// the kernel marches tau like the full stencil and carries the backward input
// from the previous step.
//
// One kernel, four uses (MODE):
//   0  out = D^-1 H in                  (t_o = D_o^-1 H_oe p_e)
//   1  out = D cin - H in, partial Re cin^H out   (w_e = S p_e)
//   2  out = out2 = b + H in, out3 = 0, partial ||out||^2   (reduced rhs, CG start)
//   3  out = D^-1 (b + H in)   (x_o from x_e; also at full-lattice sites
//      into out2 when given); partials (5 rows, pstride apart) of the odd
//      sites' part of the true residual: ||y - D out||^2 with y = b + H in
//      (zero up to rounding), Re/Im b^H x_o, Re/Im x_o^H r_o
//   4  (FP64) out32 = single(cin2 - (D cin - H in)), partial ||.||^2, lanes
//      flagged in ru only   (reliable update of the reduced residual)
//   5  r_e = b - (D cin - H in), the even sites' part of the true residual
//      b - A x with x_e = cin, x_o = in; partials ||r_e||^2, Re/Im b^H x_e,
//      Re/Im x_e^H r_e.  With state given, lanes in state kActive (those the
//      check just restarted) store r_e to out and out2 (FP64 restart) or,
//      rounded to single, to out32 and to out3 read as single precision
//      (mixed restart: r and p)
// With x_o formed by mode 3, b - A x vanishes on the odd sites up to
// rounding and equals the reduced residual b_hat - S x_e on the even ones, so
// modes 3 and 5 together give the full FP64 true residual and the quadrature
// in two half-lattice passes.
// b is the probing right-hand side, regenerated from site indices.
// ---------------------------------------------------------------------------

// The link staging of the half-lattice hops with the address arithmetic done
// once per workgroup instead of once per march step.  At step tau the tile's
// links [2 ndim][9][TS] (slots 0..ndim-1 forward U_mu(s), ndim..2 ndim-1
// backward U_mu(s - mu)) come from the even-odd link layout
// [parity][mu][9][V/2] at half-lattice index x + V3 tau' with x the tile
// site or its backward spatial neighbour, and tau' = tau except for the
// backward t-link of a site with delta = 0, which sits one slice behind
// (tau' = tau - 1, wrapping to ntau - 1 at tau = 0).  Thread tid copies
// elements it = tid + k kNT, k < KMAX; each keeps its element index at
// tau' = 0 and whether it is such a trailing t-link.
template <int KMAX>
struct EoLinkStage {
  uint32_t base[KMAX];
  uint32_t trail;                 // bit k: element k trails by one slice
  int n;                          // 2 ndim 9 TS
  __device__ __forceinline__ EoLinkStage(const Geom& g, uint32_t V3, int P, uint32_t s3_first, int TS, int kNT) {
    const int ndim = g.ndim, tdim = ndim - 1;
    const uint32_t Vh = g.V >> 1;
    n = 2 * ndim * 9 * TS;
    trail = 0u;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int it = (int)threadIdx.x + k * kNT;
      base[k] = 0u;
      if (it >= n) continue;
      const int site = it % TS;
      const int es = it / TS;
      const int e = es % 9;
      const int slot = es / 9;
      const uint32_t x3 = s3_first + (uint32_t)site;
      uint32_t hl, par;
      int mu;
      if (slot < ndim) {
        mu = slot;
        par = (uint32_t)P;
        hl = x3;
      } else {
        mu = slot - ndim;
        par = 1u - (uint32_t)P;
        if (mu < tdim) {
          hl = nbr_bwd_p2(x3, g, mu);
        } else {
          hl = x3;
          const uint32_t dl = ((uint32_t)P + spatial_parity(x3, g)) & 1u;
          if (dl == 0u) trail |= 1u << k;
        }
      }
      base[k] = (((par * (uint32_t)ndim + (uint32_t)mu) * 9u + (uint32_t)e) * Vh) + hl;
    }
  }
  // copy step tau's links into lds (the caller synchronises around it)
  template <class C>
  __device__ __forceinline__ void stage(const C* __restrict__ U, C* lds, uint32_t V3, uint32_t tau, uint32_t ntau,
                                        int kNT) const {
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int it = (int)threadIdx.x + k * kNT;
      if (it >= n) break;
      const uint32_t tt = (trail >> k) & 1u ? (tau == 0u ? ntau : tau) - 1u : tau;
      lds[it] = U[base[k] + V3 * tt];
    }
  }
};

#ifndef TIP_EO_STREAMING
#define TIP_EO_STREAMING 1
#endif
template <class Op, int MODE, int kLogB, int kNT = kBlock, bool kCacheProbe = false>
__global__ __launch_bounds__(kNT) void k_eo_hop(Geom g, MarchMap mm, int P, Op op,
                                                   const double* __restrict__ diag, const double* __restrict__ w,
                                                   const int* __restrict__ state, const int* __restrict__ active,
                                                   const typename Op::T* __restrict__ in,
                                                   const typename Op::T* __restrict__ cin,
                                                   typename Op::T* __restrict__ out, typename Op::T* __restrict__ out2,
                                                   typename Op::T* __restrict__ out3, int64_t rhs0, int nb,
                                                   uint64_t seed, int mask, double* __restrict__ partial,
                                                   int* __restrict__ ran, const int* __restrict__ ru,
                                                   const typename Op::T* __restrict__ cin2, void* __restrict__ out32,
                                                   size_t pstride) {
  using T = typename Op::T;
  constexpr int NC = Op::NC;
  constexpr bool kCov = NC == 3;
  constexpr bool kResidual = MODE == 3 || MODE == 5;      // true-residual passes: 5 partial rows
  constexpr int NP = kResidual ? 5 : 1;
  const int logB = kLogB >= 0 ? kLogB : mm.logB;
  const int B = 1 << logB;
  const int TS = kNT >> logB;
  if (active && *active == 0) return;
  if (ran && blockIdx.x == 0 && threadIdx.x == 0) *ran = 1;
  __shared__ double lds[NP * (kNT / 64) * 64];
  T* lds_links = reinterpret_cast<T*>(tip_dyn_lds);   // covariant: [2 ndim][9][TS]
  // scalar operator with couplings: the tile's weights [2 ndim][TS] (forward
  // w_mu(s), backward w_mu(s - mu)), read once per site instead of per lane
  __shared__ double lds_w[kCov ? 1 : 2 * kMaxDim * kNT];
  // kCacheProbe (passes that regenerate b, hierarchical probes): P(x) and the
  // mask of each of the tile's sites, computed once per site and march step
  // (instead of once per rhs lane) and read by the site's B lanes
  static_assert(!kCacheProbe || MODE == 2 || kResidual, "only the passes that regenerate b cache probes");
  __shared__ ProbeSiteCode lds_probe[kCacheProbe ? kNT : 1];
  const int j = threadIdx.x & (B - 1);
  const int si = threadIdx.x >> logB;
  uint32_t q, chunk;
  march_tile(mm, blockIdx.x, q, chunk);
  const uint32_t V = g.V;
  const uint32_t V3 = mm.V3;
  const uint32_t Vh = V >> 1;
  const int ndim = g.ndim;
  const int tdim = ndim - 1;
  const uint32_t nt = 1u << g.logn[tdim];
  const uint32_t ntau = nt >> 1;
  const uint32_t s3_first = q * (uint32_t)TS;
  const uint32_t s3 = s3_first + (uint32_t)si;
  const uint32_t delta = ((uint32_t)P + spatial_parity(s3, g)) & 1u;
  const bool live = kResidual || ((!state || state[j] == kActive) && (!ru || ru[j] != 0));
  // compile-time B: the link staging's addresses once per workgroup
  constexpr int kStageK = kLogB >= 0 ? (2 * kMaxDim * 9 * (kNT >> (kLogB >= 0 ? kLogB : 0)) + kNT - 1) / kNT : 1;
  const EoLinkStage<kStageK> stage(g, V3, P, s3_first, TS, kNT);
  const LaneProbe lane = lane_probe<NC>(g, rhs0, j, nb);
  double acc[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) acc[k] = 0.0;
  const uint32_t tau0 = chunk * (uint32_t)mm.Tc;
  T xprev[NC];
  if (live) load_vec<T, NC>(in, Vh, logB, s3 + V3 * ((tau0 + ntau - 1u + delta) % ntau), j, xprev);
  for (uint32_t tau = tau0; tau < tau0 + (uint32_t)mm.Tc; ++tau) {
    const uint32_t t = 2u * tau + delta;
    const uint32_t s = s3 + V3 * t;                     // full-lattice output site
    const uint32_t h = s3 + V3 * tau;                   // its half-lattice index
    if constexpr (kCov && kLogB >= 0) {
      __syncthreads();
      stage.stage(op.U, lds_links, V3, tau, ntau, kNT);
      __syncthreads();
    } else if constexpr (kCov) {
      // stage the tile's links: slots 0..ndim-1 forward U_mu(s), ndim..2ndim-1 backward U_mu(s - mu)
      __syncthreads();
      const int nslot = 2 * ndim;
      // op.U holds the even-odd link layout [parity][mu][9][V/2]: forward
      // links of the tile's own sites (parity P, index x + V3 tau), backward
      // ones at the neighbours of parity 1 - P (same slice for spatial mu,
      // slice tau - 1 + delta along t)
      for (int it = threadIdx.x; it < nslot * 9 * TS; it += kNT) {
        const int site = it % TS;
        const int es = it / TS;
        const int e = es % 9;
        const int slot = es / 9;
        const uint32_t x3 = s3_first + (uint32_t)site;
        uint32_t hl, par;
        int mu;
        if (slot < ndim) {
          mu = slot;
          par = (uint32_t)P;
          hl = x3 + V3 * tau;
        } else {
          mu = slot - ndim;
          par = 1u - (uint32_t)P;
          if (mu < tdim) {
            hl = nbr_bwd_p2(x3, g, mu) + V3 * tau;
          } else {
            const uint32_t dl = ((uint32_t)P + spatial_parity(x3, g)) & 1u;
            hl = x3 + V3 * ((tau + ntau - 1u + dl) % ntau);
          }
        }
        lds_links[it] = op.U[(((size_t)par * ndim + mu) * 9 + e) * Vh + hl];
      }
      __syncthreads();
    } else {
      if (w) {
        __syncthreads();
        const int nslot = 2 * ndim;
        for (int it = threadIdx.x; it < nslot * TS; it += kNT) {
          const int site = it % TS;
          const int slot = it / TS;
          const uint32_t x3 = s3_first + (uint32_t)site;
          const uint32_t dl = ((uint32_t)P + spatial_parity(x3, g)) & 1u;
          const uint32_t sf = x3 + V3 * (2u * tau + dl);        // full-lattice site of the tile
          const int mu = slot < ndim ? slot : slot - ndim;
          lds_w[it] = w[(size_t)mu * V + (slot < ndim ? sf : nbr_bwd_p2(sf, g, mu))];
        }
        __syncthreads();
      }
    }
    if constexpr (kCacheProbe) {
      __syncthreads();                                  // the previous step's readers are done
      if ((int)threadIdx.x < TS) {
        const uint32_t x3 = s3_first + threadIdx.x;
        const uint32_t dl = ((uint32_t)P + spatial_parity(x3, g)) & 1u;
        lds_probe[threadIdx.x] = probe_site_code(x3 + V3 * (2u * tau + dl), g, seed, mask);
      }
      __syncthreads();
    }
    if (!live) continue;
    T hop[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) hop[c] = zero<T>();
    // spatial directions: neighbours in the same slice
#pragma unroll
    for (int mu = 0; mu < kMaxDim - 1; ++mu) {
      if (mu >= tdim) break;
      const uint32_t nf = nbr_fwd_p2(s3, g, mu), nbk = nbr_bwd_p2(s3, g, mu);
      double wf = 1.0, wb = 1.0;
      if (w) {
        if constexpr (kCov) {
          wf = w[(size_t)mu * V + s];
          wb = w[(size_t)mu * V + nbr_bwd_p2(s, g, mu)];
        } else {
          wf = lds_w[mu * TS + si];
          wb = lds_w[(ndim + mu) * TS + si];
        }
      }
      T xn[NC], hh[NC];
      load_vec<T, NC>(in, Vh, logB, nf + V3 * tau, j, xn);
      if constexpr (kCov) {
        T u[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = lds_links[(mu * 9 + e) * TS + si];
        mul_u(u, xn, hh);
      } else {
        hh[0] = xn[0];
      }
      add_weighted<T, NC>(wf, hh, hop);
      load_vec<T, NC>(in, Vh, logB, nbk + V3 * tau, j, xn);
      if constexpr (kCov) {
        T u[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = lds_links[((ndim + mu) * 9 + e) * TS + si];
        mul_uh(u, xn, hh);
      } else {
        hh[0] = xn[0];
      }
      add_weighted<T, NC>(wb, hh, hop);
    }
    // the marching direction: forward input in slice tau + delta, backward one carried
    {
      double wf = 1.0, wb = 1.0;
      if (w) {
        if constexpr (kCov) {
          wf = w[(size_t)tdim * V + s];
          wb = w[(size_t)tdim * V + nbr_bwd_p2(s, g, tdim)];
        } else {
          wf = lds_w[tdim * TS + si];
          wb = lds_w[(ndim + tdim) * TS + si];
        }
      }
      T xn[NC], hh[NC];
      load_vec<T, NC>(in, Vh, logB, s3 + V3 * ((tau + delta) % ntau), j, xn);
      if constexpr (kCov) {
        T u[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = lds_links[(tdim * 9 + e) * TS + si];
        mul_u(u, xn, hh);
      } else {
        hh[0] = xn[0];
      }
      add_weighted<T, NC>(wf, hh, hop);
      if constexpr (kCov) {
        T u[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = lds_links[((ndim + tdim) * 9 + e) * TS + si];
        mul_uh(u, xprev, hh);
      } else {
        hh[0] = xprev[0];
      }
      add_weighted<T, NC>(wb, hh, hop);
#pragma unroll
      for (int c = 0; c < NC; ++c) xprev[c] = xn[c];
    }
    const double d = diag[s];
    T y[NC];
    if constexpr (MODE == 0) {
      const double f = diag[(size_t)V + s];
#pragma unroll
      for (int c = 0; c < NC; ++c) y[c] = axpy(f, hop[c], zero<T>());
      if constexpr (TIP_EO_STREAMING) store_vec_nt<T, NC>(out, Vh, logB, h, j, y);
      else store_vec<T, NC>(out, Vh, logB, h, j, y);
    } else if constexpr (MODE == 1) {
      T cv[NC];
      if constexpr (TIP_EO_STREAMING) load_vec_nt<T, NC>(cin, Vh, logB, h, j, cv);
      else load_vec<T, NC>(cin, Vh, logB, h, j, cv);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        y[c] = axpy(d, cv[c], axpy(-1.0, hop[c], zero<T>()));
        acc[0] += redot(cv[c], y[c]);
      }
      if constexpr (TIP_EO_STREAMING) store_vec_nt<T, NC>(out, Vh, logB, h, j, y);
      else store_vec<T, NC>(out, Vh, logB, h, j, y);
    } else if constexpr (MODE == 4) {
      if constexpr (sizeof(typename SingleOf<T>::type) * 2 == sizeof(T)) {
        // reliable update of the reduced system: r = b_hat - (D x_e - H t_o),
        // b_hat = cin2, x_e = cin, t_o = in; rounded to single into out32
        using T32 = typename SingleOf<T>::type;
        T xv[NC], bv[NC];
        T32 r32[NC];
        load_vec<T, NC>(cin, Vh, logB, h, j, xv);
        load_vec<T, NC>(cin2, Vh, logB, h, j, bv);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const T sx = axpy(d, xv[c], axpy(-1.0, hop[c], zero<T>()));
          y[c] = axpy(-1.0, sx, bv[c]);
          acc[0] += norm2(y[c]);
          r32[c] = to_single(y[c]);
        }
        store_vec<T32, NC>(reinterpret_cast<T32*>(out32), Vh, logB, h, j, r32);
      }
    } else {
      T b[NC];
      if constexpr (kCacheProbe) rhs_from_code<T, NC>(lds_probe[si], lane, b);
      else rhs_at<T, NC>(g, s, rhs0, j, nb, seed, mask, b);
      if constexpr (MODE == 2) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          y[c] = j < nb ? axpy(1.0, hop[c], b[c]) : zero<T>();
          acc[0] += norm2(y[c]);
        }
        T z[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) z[c] = zero<T>();
        store_vec<T, NC>(out, Vh, logB, h, j, y);
        if (out2) store_vec<T, NC>(out2, Vh, logB, h, j, y);
        if (out3) store_vec<T, NC>(out3, Vh, logB, h, j, z);
      } else if constexpr (MODE == 3) {
        const double f = diag[(size_t)V + s];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const T yv = axpy(1.0, hop[c], b[c]);              // b_o + H_oe x_e
          y[c] = axpy(f, yv, zero<T>());                       // x_o
          const T ro = axpy(-d, y[c], yv);                     // b_o + H_oe x_e - D_o x_o
          acc[0] += norm2(ro);
          acc[1] += redot(b[c], y[c]);
          acc[2] += imdot(b[c], y[c]);
          acc[3] += redot(y[c], ro);
          acc[4] += imdot(y[c], ro);
        }
        store_vec<T, NC>(out, Vh, logB, h, j, y);
        if (out2) store_vec<T, NC>(out2, V, logB, s, j, y);
      } else if constexpr (MODE == 5) {
        T xv[NC];
        load_vec<T, NC>(cin, Vh, logB, h, j, xv);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const T ax = axpy(d, xv[c], axpy(-1.0, hop[c], zero<T>()));   // D_e x_e - H_eo x_o
          y[c] = axpy(-1.0, ax, b[c]);
          acc[0] += norm2(y[c]);
          acc[1] += redot(b[c], xv[c]);
          acc[2] += imdot(b[c], xv[c]);
          acc[3] += redot(xv[c], y[c]);
          acc[4] += imdot(xv[c], y[c]);
        }
        if (state && state[j] == kActive) {
          if (out) store_vec<T, NC>(out, Vh, logB, h, j, y);
          if (out2) store_vec<T, NC>(out2, Vh, logB, h, j, y);
          if constexpr (sizeof(typename SingleOf<T>::type) * 2 == sizeof(T)) {
            using T32 = typename SingleOf<T>::type;
            if (out32) {
              T32 r32[NC];
#pragma unroll
              for (int c = 0; c < NC; ++c) r32[c] = to_single(y[c]);
              store_vec<T32, NC>(reinterpret_cast<T32*>(out32), Vh, logB, h, j, r32);
              if (out3) store_vec<T32, NC>(reinterpret_cast<T32*>(out3), Vh, logB, h, j, r32);
            }
          }
        }
      }
    }
  }
  if (partial) {
    seg_sum<NP, kNT / 64>(acc, B, lds);
    if ((int)threadIdx.x < B) {
#pragma unroll
      for (int k = 0; k < NP; ++k) partial[k * pstride + (size_t)threadIdx.x * gridDim.x + blockIdx.x] = acc[k];
    }
  }
}

// The two hops of the CG iteration (modes 0 and 1 of k_eo_hop) with two
// right-hand sides per thread, for the operators whose lane element is 8
// bytes: the single-precision covariant operator (float2) and the FP64 real
// scalar one (double).  A block of 32 rhs in [ncomp][V/2][32] holds rhs 2l and
// 2l + 1 of a site and colour in one aligned 16-byte pair, so thread l of a
// site loads both with one instruction: the bytes per load of the FP64
// covariant kernel, 16 threads per site and 16 sites per workgroup (against
// 8), which also halves the share of x1 neighbours that lie in the next tile.
// Each rhs is computed exactly as in k_eo_hop; the partials of mode 1 are
// written per rhs.
typedef float tip_f4 __attribute__((ext_vector_type(4)));
typedef double tip_d2 __attribute__((ext_vector_type(2)));
template <class T> struct PairOf;
template <> struct PairOf<float2> {
  using V = tip_f4;
  __device__ static void split(const V& x, float2& a, float2& b) {
    a = make_float2(x.x, x.y);
    b = make_float2(x.z, x.w);
  }
};
template <> struct PairOf<double> {
  using V = tip_d2;
  __device__ static void split(const V& x, double& a, double& b) {
    a = x.x;
    b = x.y;
  }
};

template <bool kNT, class T, int NC>
__device__ __forceinline__ void load_pair(const T* __restrict__ v, size_t Vh, uint32_t h, int l, T (&a)[NC],
                                          T (&b)[NC]) {
  using PV = typename PairOf<T>::V;
  const PV* p = reinterpret_cast<const PV*>(v);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const PV* q = p + ((((size_t)c * Vh + h)) << 4) + l;
    PV x;
    if constexpr (kNT) x = __builtin_nontemporal_load(q);
    else x = *q;
    PairOf<T>::split(x, a[c], b[c]);
  }
}
// Two 8-byte streaming stores to adjacent addresses (merged into one 16-byte
// store); packing the pair into one vector first put it on the stack.
template <class T, int NC>
__device__ __forceinline__ void store_pair_nt(T* __restrict__ v, size_t Vh, uint32_t h, int l, const T (&a)[NC],
                                              const T (&b)[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    T* q = v + ((((size_t)c * Vh + h)) << 5) + 2 * l;
    st_nt(q, a[c]);
    st_nt(q + 1, b[c]);
  }
}

template <class Op, int MODE, int kNT = kBlock>
__global__ __launch_bounds__(kNT) void k_eo_hop_pair(Geom g, MarchMap mm, int P, Op op,
                                                        const double* __restrict__ diag,
                                                        const double* __restrict__ w,
                                                        const int* __restrict__ state, const int* __restrict__ active,
                                                        const typename Op::T* __restrict__ in,
                                                        const typename Op::T* __restrict__ cin,
                                                        typename Op::T* __restrict__ out,
                                                        double* __restrict__ partial, int* __restrict__ ran) {
  static_assert(MODE == 0 || MODE == 1, "pair kernel: the two hops of the CG iteration");
  using T = typename Op::T;
  constexpr int NC = Op::NC;
  constexpr bool kCov = NC == 3;
  static_assert(sizeof(T) == 8, "pair kernel: 8-byte lane elements");
  constexpr int kLP = 4;                          // 16 pair lanes per site: rhs 2l, 2l + 1
  constexpr int NL = 1 << kLP;
  constexpr int TS = kNT >> kLP;                  // 16 sites per 256-thread workgroup
  if (active && *active == 0) return;
  if (ran && blockIdx.x == 0 && threadIdx.x == 0) *ran = 1;
  __shared__ double lds[2 * (kNT / 64) * 64];
  T* lds_links = reinterpret_cast<T*>(tip_dyn_lds);   // covariant: [2 ndim][9][TS]
  __shared__ double lds_w[kCov ? 1 : 2 * kMaxDim * TS];   // scalar with couplings: [2 ndim][TS]
  const int l = threadIdx.x & (NL - 1);
  const int si = threadIdx.x >> kLP;
  uint32_t q, chunk;
  march_tile(mm, blockIdx.x, q, chunk);
  const uint32_t V = g.V;
  const uint32_t V3 = mm.V3;
  const uint32_t Vh = V >> 1;
  const int ndim = g.ndim;
  const int tdim = ndim - 1;
  const uint32_t ntau = (1u << g.logn[tdim]) >> 1;
  const uint32_t s3_first = q * (uint32_t)TS;
  const uint32_t s3 = s3_first + (uint32_t)si;
  const uint32_t delta = ((uint32_t)P + spatial_parity(s3, g)) & 1u;
  const bool live = !state || state[2 * l] == kActive || state[2 * l + 1] == kActive;
  const EoLinkStage<(2 * kMaxDim * 9 * TS + kNT - 1) / kNT> stage(g, V3, P, s3_first, TS, kNT);
  double acc[2] = {0.0, 0.0};
  const uint32_t tau0 = chunk * (uint32_t)mm.Tc;
  T pa[NC], pb[NC];                               // backward t input, carried along the march
  auto ld = [&](uint32_t hh, T (&xa)[NC], T (&xb)[NC]) { load_pair<false, T, NC>(in, Vh, hh, l, xa, xb); };
  if (live) ld(s3 + V3 * ((tau0 + ntau - 1u + delta) % ntau), pa, pb);
  for (uint32_t tau = tau0; tau < tau0 + (uint32_t)mm.Tc; ++tau) {
    const uint32_t t = 2u * tau + delta;
    const uint32_t s = s3 + V3 * t;
    const uint32_t h = s3 + V3 * tau;
    const int nslot = 2 * ndim;
    if constexpr (kCov) {
      // the tile's links, as in k_eo_hop: forward U_mu of the tile's sites,
      // backward ones at the opposite-parity neighbours
      __syncthreads();
      stage.stage(op.U, lds_links, V3, tau, ntau, kNT);
      __syncthreads();
    } else if (w) {
      // the tile's couplings, as in k_eo_hop: forward w_mu(s), backward w_mu(s - mu)
      __syncthreads();
      for (int it = threadIdx.x; it < nslot * TS; it += kNT) {
        const int site = it % TS;
        const int slot = it / TS;
        const uint32_t x3 = s3_first + (uint32_t)site;
        const uint32_t dl = ((uint32_t)P + spatial_parity(x3, g)) & 1u;
        const uint32_t sf = x3 + V3 * (2u * tau + dl);
        const int mu = slot < ndim ? slot : slot - ndim;
        lds_w[it] = w[(size_t)mu * V + (slot < ndim ? sf : nbr_bwd_p2(sf, g, mu))];
      }
      __syncthreads();
    }
    if (!live) continue;
    T ha[NC], hb[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) ha[c] = hb[c] = zero<T>();
    // one hop: y = U x (forward) or U^H x (backward) for both rhs, weighted
    auto hop = [&](int slot, bool fwd, const T (&xa)[NC], const T (&xb)[NC]) {
      if constexpr (kCov) {
        // unit weights: the products go straight into the sums
        T u[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = lds_links[(slot * 9 + e) * TS + si];
        if (fwd) {
          mul_u_acc(u, xa, ha);
          mul_u_acc(u, xb, hb);
        } else {
          mul_uh_acc(u, xa, ha);
          mul_uh_acc(u, xb, hb);
        }
      } else {
        double wt = 1.0;
        if (w) wt = lds_w[slot * TS + si];
        T ya[NC], yb[NC];
        ya[0] = xa[0];
        yb[0] = xb[0];
        add_weighted<T, NC>(wt, ya, ha);
        add_weighted<T, NC>(wt, yb, hb);
      }
    };
#pragma unroll
    for (int mu = 0; mu < kMaxDim - 1; ++mu) {
      if (mu >= tdim) break;
      T xa[NC], xb[NC];
      ld(nbr_fwd_p2(s3, g, mu) + V3 * tau, xa, xb);
      hop(mu, true, xa, xb);
      ld(nbr_bwd_p2(s3, g, mu) + V3 * tau, xa, xb);
      hop(ndim + mu, false, xa, xb);
    }
    {
      T xa[NC], xb[NC];
      ld(s3 + V3 * ((tau + delta) % ntau), xa, xb);
      hop(tdim, true, xa, xb);
      hop(ndim + tdim, false, pa, pb);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        pa[c] = xa[c];
        pb[c] = xb[c];
      }
    }
    const double d = diag[s];
    T ya[NC], yb[NC];
    if constexpr (MODE == 0) {
      const double f = diag[(size_t)V + s];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        ya[c] = axpy(f, ha[c], zero<T>());
        yb[c] = axpy(f, hb[c], zero<T>());
      }
    } else {
      T ca[NC], cb[NC];
      load_pair<true, T, NC>(cin, Vh, h, l, ca, cb);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        ya[c] = axpy(d, ca[c], axpy(-1.0, ha[c], zero<T>()));
        yb[c] = axpy(d, cb[c], axpy(-1.0, hb[c], zero<T>()));
        acc[0] += redot(ca[c], ya[c]);
        acc[1] += redot(cb[c], yb[c]);
      }
    }
    store_pair_nt<T, NC>(out, Vh, h, l, ya, yb);
  }
  if constexpr (MODE == 1) {
    seg_sum<2, kNT / 64>(acc, NL, lds);
    if ((int)threadIdx.x < NL) {
      partial[(size_t)(2 * threadIdx.x) * gridDim.x + blockIdx.x] = acc[0];
      partial[(size_t)(2 * threadIdx.x + 1) * gridDim.x + blockIdx.x] = acc[1];
    }
  }
}

// Half-lattice index <-> full-lattice site of parity P (see above).
__device__ __forceinline__ uint32_t eo_site(uint32_t h, int P, const Geom& g) {
  const int tdim = g.ndim - 1;
  const uint32_t V3 = 1u << g.shift[tdim];
  const uint32_t s3 = h & (V3 - 1u), tau = h >> g.shift[tdim];
  const uint32_t delta = ((uint32_t)P + spatial_parity(s3, g)) & 1u;
  return s3 + V3 * (2u * tau + delta);
}

// t_o = D_o^-1 b_o on the odd half-lattice (zero for padding lanes).
template <class T, int NC>
__global__ __launch_bounds__(kBlock) void k_eo_init_odd(Geom g, int logB, int64_t rhs0, int nb, uint64_t seed,
                                                        int mask, const double* __restrict__ diag,
                                                        T* __restrict__ to) {
  const int B = 1 << logB;
  const int j = threadIdx.x & (B - 1);
  const uint32_t h = blockIdx.x * (kBlock >> logB) + (threadIdx.x >> logB);
  const uint32_t Vh = g.V >> 1;
  if (h >= Vh) return;
  const uint32_t s = eo_site(h, 1, g);
  T b[NC];
  rhs_at<T, NC>(g, s, rhs0, j, nb, seed, mask, b);
  const double f = diag[(size_t)g.V + s];
#pragma unroll
  for (int c = 0; c < NC; ++c) b[c] = axpy(f, b[c], zero<T>());
  store_vec<T, NC>(to, Vh, logB, h, j, b);
}

// x (full lattice) at even sites = x_e (half lattice).
template <class T, int NC>
__global__ __launch_bounds__(kBlock) void k_eo_scatter_even(Geom g, int logB, const T* __restrict__ xe,
                                                            T* __restrict__ x) {
  const int B = 1 << logB;
  const int j = threadIdx.x & (B - 1);
  const uint32_t h = blockIdx.x * (kBlock >> logB) + (threadIdx.x >> logB);
  const uint32_t Vh = g.V >> 1;
  if (h >= Vh) return;
  T v[NC];
  load_vec<T, NC>(xe, Vh, logB, h, j, v);
  store_vec<T, NC>(x, g.V, logB, eo_site(h, 0, g), j, v);
}

// D(x) = m(x) + sum_mu [w_mu(x) + w_mu(x - mu)].
__global__ __launch_bounds__(kBlock) void k_diag(Geom g, const double* __restrict__ mass_field, double mass,
                                                 const double* __restrict__ w, double* __restrict__ out) {
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  double d = mass_field ? mass_field[s] : mass;
  for (int mu = 0; mu < g.ndim; ++mu) {
    const double wf = w ? w[(size_t)mu * g.V + s] : 1.0;
    const double wb = w ? w[(size_t)mu * g.V + nbr_bwd(s, g, mu)] : 1.0;
    d += wf + wb;
  }
  out[s] = d;
  out[(size_t)g.V + s] = 1.0 / d;   // D^-1 of the even-odd passes, rounded once here
}

// rho = rho_ref = ||r||^2 of the reduced start residual.
__global__ __launch_bounds__(kBlock) void k_reduce_rho0(CgScalars sc, const double* __restrict__ partial, int gx) {
  const int j = blockIdx.x;
  if (sc.state[j] != kActive) return;            // uniform per workgroup
  const double v = sum_partials(partial + (size_t)j * gx, gx);
  if (threadIdx.x != 0) return;
  sc.rho[j] = v;
  sc.rho_ref[j] = v;
  sc.pp[j] = v;                                // p = r
}

size_t march_lds_bytes(const Geom& g, const MarchMap& mm, Prec prec) {
  const size_t need = (size_t)(2 * g.ndim - 1) * 9 * mm.TS * (prec == Prec::kF64 ? sizeof(double2) : sizeof(float2));
  const int cap = prec == Prec::kF64 ? mm.wgs_per_cu64 : mm.wgs_per_cu32;
  if (cap < 2) return need;
  // reserve enough LDS that at most `cap` workgroups fit on one CU (160 KiB),
  // counting the 2 KiB of static LDS of the reduction
  const size_t pad = (size_t)kLdsPerCu / (size_t)(cap + 1) + 512 - 2048;
  return need > pad ? need : pad;
}

// Calls f(op_policy) for the operator / element / precision combination.
template <class F>
static hipError_t dispatch(const OpDev& od, Elem elem, Prec prec, F&& f) {
  if (prec == Prec::kF64) {
    if (od.kind == 1) f(CovOp<double2>{(const double2*)od.links});
    else if (elem == Elem::kReal) f(ScalarOp<double>{});
    else f(ScalarOp<double2>{});
  } else {
    if (od.kind == 1) f(CovOp<float2>{(const float2*)od.links});
    else if (elem == Elem::kReal) f(ScalarOp<float>{});
    else f(ScalarOp<float2>{});
  }
  return hipGetLastError();
}

// FP64 operators only (true residual, reliable updates).
template <class F>
static hipError_t dispatch64(const OpDev& od, Elem elem, F&& f) {
  if (od.kind == 1) f(CovOp<double2>{(const double2*)od.links});
  else if (elem == Elem::kReal) f(ScalarOp<double>{});
  else f(ScalarOp<double2>{});
  return hipGetLastError();
}

// Calls f(T) with a value of the vector element type.
template <class F>
static hipError_t by_elem(Elem elem, Prec prec, F&& f) {
  if (prec == Prec::kF64) {
    if (elem == Elem::kReal) f(double{});
    else f(double2{});
  } else {
    if (elem == Elem::kReal) f(float{});
    else f(float2{});
  }
  return hipGetLastError();
}

hipError_t launch_stencil(const OpDev& od, const Geom& g, const TileMap& tm, const MarchMap* mm, Elem elem, Prec prec,
                          const int* state, const int* active, const void* in, void* out, double* partial, int* ran,
                          hipStream_t st) {
  return dispatch(od, elem, prec, [&](auto op) {
    using Op = decltype(op);
    using T = typename Op::T;
    if constexpr (Op::NC == 3) {
      if (mm && mm->lds_links && mm->spec4) {
        const size_t lds = march_lds_bytes(g, *mm, prec);
        const bool hw = od.coupling != nullptr;
        auto go4 = [&](auto kern) {
          kern<<<mm->grid, kBlock, lds, st>>>(g, *mm, op.U, od.mass_field, od.mass, od.coupling, state, active,
                                              (const T*)in, (T*)out, partial, ran);
        };
        switch (mm->logB * 2 + (hw ? 1 : 0)) {
          case 4: go4(k_stencil_march4<T, 2, false>); return;
          case 5: go4(k_stencil_march4<T, 2, true>); return;
          case 6: go4(k_stencil_march4<T, 3, false>); return;
          case 7: go4(k_stencil_march4<T, 3, true>); return;
          case 8: go4(k_stencil_march4<T, 4, false>); return;
          case 9: go4(k_stencil_march4<T, 4, true>); return;
          case 10: go4(k_stencil_march4<T, 5, false>); return;
          case 11: go4(k_stencil_march4<T, 5, true>); return;
          default: break;
        }
      }
      if (mm && mm->lds_links) {
        const size_t lds = march_lds_bytes(g, *mm, prec);
        auto go = [&](auto kern) {
          kern<<<mm->grid, kBlock, lds, st>>>(g, *mm, op, od.mass_field, od.mass, od.coupling, state, active,
                                              (const T*)in, (T*)out, partial, ran);
        };
        const bool hw = od.coupling != nullptr;
        switch (mm->logB * 2 + (hw ? 1 : 0)) {
          case 4: go(k_stencil_march<Op, true, 2, 0>); break;
          case 5: go(k_stencil_march<Op, true, 2, 1>); break;
          case 6: go(k_stencil_march<Op, true, 3, 0>); break;
          case 7: go(k_stencil_march<Op, true, 3, 1>); break;
          case 8: go(k_stencil_march<Op, true, 4, 0>); break;
          case 9: go(k_stencil_march<Op, true, 4, 1>); break;
          default: go(k_stencil_march<Op, true>); break;
        }
        return;
      }
    }
    if (mm)
      k_stencil_march<Op, false><<<mm->grid, kBlock, 0, st>>>(g, *mm, op, od.mass_field, od.mass, od.coupling, state,
                                                              active, (const T*)in, (T*)out, partial, ran);
    else
      k_stencil<Op><<<tm.grid, kBlock, 0, st>>>(g, tm, op, od.mass_field, od.mass, od.coupling, state, active,
                                                (const T*)in, (T*)out, partial, ran);
  });
}

hipError_t launch_true_residual(const OpDev& od, const Geom& g, const TileMap& tm, Elem elem, const int* state,
                                int64_t rhs0, int nb, uint64_t seed, int mask, const void* x, void* r, void* p,
                                double* partial, size_t pstride, hipStream_t st) {
  return dispatch64(od, elem, [&](auto op) {
    using Op = decltype(op);
    using T = typename Op::T;
    k_true_residual<Op><<<ru_grid(tm), kBlock, 0, st>>>(g, tm, op, od.mass_field, od.mass, od.coupling, state, rhs0, nb,
                                                    seed, mask, (const T*)x, (T*)r, (T*)p, partial, pstride);
  });
}

hipError_t launch_init(const Geom& g, Elem elem, int logB, int64_t rhs0, int nb, uint64_t seed, int mask, void* x,
                       void* r, void* p, hipStream_t st) {
  const unsigned grid = cdiv(g.V, (size_t)(kBlock >> logB));
  if (g.ncomp == 3)
    k_init<double2, 3><<<grid, kBlock, 0, st>>>(g, logB, rhs0, nb, seed, mask, (double2*)x, (double2*)r, (double2*)p);
  else if (elem == Elem::kReal)
    k_init<double, 1><<<grid, kBlock, 0, st>>>(g, logB, rhs0, nb, seed, mask, (double*)x, (double*)r, (double*)p);
  else
    k_init<double2, 1><<<grid, kBlock, 0, st>>>(g, logB, rhs0, nb, seed, mask, (double2*)x, (double2*)r, (double2*)p);
  return hipGetLastError();
}

// workgroups of the grid-stride update pass: more spread the 3-vector stream
// better, but the reduction after it reads one partial per workgroup and rhs
// (32^4 covariant, k_update_r + k_reduce_beta: 487 us at 8192, 466 at 32768,
// 479 at 65536)
#ifndef TIP_UPD_GRID
#define TIP_UPD_GRID 32768u
#endif
unsigned update_grid(size_t n) { return std::min<unsigned>(cdiv(n, kBlock), TIP_UPD_GRID); }
unsigned ru_grid(const TileMap& tm) { return std::min<unsigned>(tm.grid, 4096u); }

hipError_t launch_update_r(size_t n, int logB, Elem elem, Prec prec, const CgScalars& sc, void* r, const void* Ap,
                           double* partial, hipStream_t st) {
  const unsigned grid = update_grid(n);
  return by_elem(elem, prec, [&](auto tv) {
    using T = decltype(tv);
    k_update_r<T><<<grid, kBlock, 0, st>>>(n, logB, sc, (T*)r, (const T*)Ap, partial);
  });
}

hipError_t launch_direction(size_t n, int logB, Elem elem, Prec prec, const CgScalars& sc, void* x, const void* r,
                            void* p, hipStream_t st) {
  const unsigned grid = cdiv(n, kBlock);
  return by_elem(elem, prec, [&](auto tv) {
    using T = decltype(tv);
    k_direction<T><<<grid, kBlock, 0, st>>>(n, logB, sc, (T*)x, (const T*)r, (T*)p);
  });
}

hipError_t launch_init_mixed(const Geom& g, Elem elem, int logB, int64_t rhs0, int nb, uint64_t seed, int mask,
                             void* x64, void* xh, void* rh, void* ph, hipStream_t st) {
  const unsigned grid = cdiv(g.V, (size_t)(kBlock >> logB));
  if (g.ncomp == 3)
    k_init_mixed<double2, float2, 3><<<grid, kBlock, 0, st>>>(g, logB, rhs0, nb, seed, mask, (double2*)x64,
                                                              (float2*)xh, (float2*)rh, (float2*)ph);
  else if (elem == Elem::kReal)
    k_init_mixed<double, float, 1><<<grid, kBlock, 0, st>>>(g, logB, rhs0, nb, seed, mask, (double*)x64, (float*)xh,
                                                            (float*)rh, (float*)ph);
  else
    k_init_mixed<double2, float2, 1><<<grid, kBlock, 0, st>>>(g, logB, rhs0, nb, seed, mask, (double2*)x64,
                                                              (float2*)xh, (float2*)rh, (float2*)ph);
  return hipGetLastError();
}

hipError_t launch_ru_accumulate(size_t n, int logB, Elem elem, const CgScalars& sc, int mode, void* x64, void* xh,
                                hipStream_t st) {
  // launched every iteration and returning at once while no update is
  // pending: a smaller grid than the update pass keeps that cheap
  const unsigned grid = std::min<unsigned>(cdiv(n, kBlock), 8192u);
  if (elem == Elem::kReal)
    k_ru_accumulate<double, float><<<grid, kBlock, 0, st>>>(n, logB, sc, mode, (double*)x64, (float*)xh);
  else
    k_ru_accumulate<double2, float2><<<grid, kBlock, 0, st>>>(n, logB, sc, mode, (double2*)x64, (float2*)xh);
  return hipGetLastError();
}

hipError_t launch_ru_residual(const OpDev& od64, const Geom& g, const TileMap& tm, Elem elem, const CgScalars& sc,
                              int mode, int64_t rhs0, int nb, uint64_t seed, int mask, const void* x64, void* rh,
                              void* ph, double* partial, size_t pstride, hipStream_t st) {
  return dispatch64(od64, elem, [&](auto op) {
    using Op = decltype(op);
    using T = typename Op::T;
    using T32 = typename SingleOf<T>::type;
    k_ru_residual<Op, T32><<<ru_grid(tm), kBlock, 0, st>>>(g, tm, op, od64.mass_field, od64.mass, od64.coupling, sc, mode,
                                                       rhs0, nb, seed, mask, (const T*)x64, (T32*)rh, (T32*)ph,
                                                       partial, pstride);
  });
}

hipError_t launch_reduce_ru(const CgScalars& sc, int B, const double* partial, int gx, size_t pstride, int mode,
                            double tol2, int max_iter, int max_restarts, hipStream_t st, const double* partial2) {
  k_reduce_ru<<<B, kBlock, 0, st>>>(sc, partial, partial2, gx, pstride, mode, tol2, max_iter, max_restarts);
  return hipGetLastError();
}

size_t eo_lds_bytes(const Geom& g, const MarchMap& mm, Prec prec) {
  return (size_t)(2 * g.ndim) * 9 * mm.TS * (prec == Prec::kF64 ? sizeof(double2) : sizeof(float2));
}

hipError_t launch_eo_hop(int mode, const OpDev& od, const Geom& g, const MarchMap& mm, int P, Elem elem, Prec prec,
                         const double* diag, const int* state, const int* active, const void* in, const void* cin,
                         void* out, void* out2, void* out3, int64_t rhs0, int nb, uint64_t seed, int mask,
                         double* partial, int* ran, hipStream_t st, const int* ru, const void* cin2, void* out32,
                         size_t pstride) {
  OpDev oe = od;
  oe.links = od.links_eo;
  return dispatch(oe, elem, prec, [&](auto op) {
    using Op = decltype(op);
    using T = typename Op::T;
    const size_t lds = Op::NC == 3 ? eo_lds_bytes(g, mm, prec) : 0;
    auto go = [&](auto kern) {
      kern<<<mm.grid, kBlock, lds, st>>>(g, mm, P, op, diag, od.coupling, state, active, (const T*)in,
                                          (const T*)cin, (T*)out, (T*)out2, (T*)out3, rhs0, nb, seed, mask, partial,
                                          ran, ru, (const T*)cin2, out32, pstride);
    };
    const bool b32 = mm.logB == 5;
    const bool hier = g.probe == kProbeHierarchical;     // b from the per-site probe cache
    switch (mode) {
      case 0: b32 ? go(k_eo_hop<Op, 0, 5>) : go(k_eo_hop<Op, 0, -1>); break;
      case 1: b32 ? go(k_eo_hop<Op, 1, 5>) : go(k_eo_hop<Op, 1, -1>); break;
      case 2:
        if (hier) b32 ? go(k_eo_hop<Op, 2, 5, kBlock, true>) : go(k_eo_hop<Op, 2, -1, kBlock, true>);
        else b32 ? go(k_eo_hop<Op, 2, 5>) : go(k_eo_hop<Op, 2, -1>);
        break;
      case 3:
        if (hier) b32 ? go(k_eo_hop<Op, 3, 5, kBlock, true>) : go(k_eo_hop<Op, 3, -1, kBlock, true>);
        else b32 ? go(k_eo_hop<Op, 3, 5>) : go(k_eo_hop<Op, 3, -1>);
        break;
      case 5:
        if (hier) b32 ? go(k_eo_hop<Op, 5, 5, kBlock, true>) : go(k_eo_hop<Op, 5, -1, kBlock, true>);
        else b32 ? go(k_eo_hop<Op, 5, 5>) : go(k_eo_hop<Op, 5, -1>);
        break;
      default:
        if constexpr (sizeof(typename SingleOf<T>::type) * 2 == sizeof(T)) {
          if (b32) go(k_eo_hop<Op, 4, 5>);
          else go(k_eo_hop<Op, 4, -1>);
        }
        break;
    }
  });
}

// FP64 covariant modes 0 and 1 with 512-thread workgroups: one rhs per lane as
// in k_eo_hop, 16 sites per tile (the march map built for that tile size).
// Measured at 32^4 against 256 threads (8 sites per tile): 749 against 772 us
// for the dominant hop; 1024 threads (a whole x1 row per tile) gained nothing.
hipError_t launch_eo_hop_wide(int mode, const OpDev& od, const Geom& g, const MarchMap& mm, int P,
                              const double* diag, const int* state, const int* active, const void* in,
                              const void* cin, void* out, double* partial, int* ran, hipStream_t st) {
  using Op = CovOp<double2>;
  constexpr int kNT = 2 * kBlock;
  Op op{reinterpret_cast<const double2*>(od.links_eo)};
  const size_t lds = eo_lds_bytes(g, mm, Prec::kF64);
  const double2* x = (const double2*)in;
  const double2* c = (const double2*)cin;
  auto go = [&](auto kern) {
    kern<<<mm.grid, kNT, lds, st>>>(g, mm, P, op, diag, od.coupling, state, active, x, c, (double2*)out, nullptr,
                                    nullptr, 0, 0, 0, 0, mode == 1 ? partial : nullptr, ran, nullptr, nullptr,
                                    nullptr, 0);
  };
  if (mode == 0) go(k_eo_hop<Op, 0, 5, kNT>);
  else go(k_eo_hop<Op, 1, 5, kNT>);
  return hipGetLastError();
}

// Every FP64 covariant mode in 512-thread workgroups (B = 32, 16 sites per
// tile, on the march map built for that tile size): the iteration's hops of
// the FP64 solver, and the once-per-block passes and reliable updates of both
// solvers.
hipError_t launch_eo_hop512(int mode, const OpDev& od, const Geom& g, const MarchMap& mm, int P, const double* diag,
                            const int* state, const int* active, const void* in, const void* cin, void* out,
                            void* out2, void* out3, int64_t rhs0, int nb, uint64_t seed, int mask, double* partial,
                            int* ran, hipStream_t st, const int* ru, const void* cin2, void* out32, size_t pstride) {
  using Op = CovOp<double2>;
  constexpr int kNT = 2 * kBlock;
  Op op{reinterpret_cast<const double2*>(od.links_eo)};
  const size_t lds = eo_lds_bytes(g, mm, Prec::kF64);
  using T = double2;
  auto go = [&](auto kern) {
    kern<<<mm.grid, kNT, lds, st>>>(g, mm, P, op, diag, od.coupling, state, active, (const T*)in, (const T*)cin,
                                    (T*)out, (T*)out2, (T*)out3, rhs0, nb, seed, mask, partial, ran, ru,
                                    (const T*)cin2, out32, pstride);
  };
  const bool hier = g.probe == kProbeHierarchical;     // b from the per-site probe cache
  switch (mode) {
    case 0: go(k_eo_hop<Op, 0, 5, kNT>); break;
    case 1: go(k_eo_hop<Op, 1, 5, kNT>); break;
    case 2: hier ? go(k_eo_hop<Op, 2, 5, kNT, true>) : go(k_eo_hop<Op, 2, 5, kNT>); break;
    case 3: hier ? go(k_eo_hop<Op, 3, 5, kNT, true>) : go(k_eo_hop<Op, 3, 5, kNT>); break;
    case 4: go(k_eo_hop<Op, 4, 5, kNT>); break;
    default: hier ? go(k_eo_hop<Op, 5, 5, kNT, true>) : go(k_eo_hop<Op, 5, 5, kNT>); break;
  }
  return hipGetLastError();
}

hipError_t launch_eo_hop_pair(int mode, const OpDev& od, const Geom& g, const MarchMap& mm, int P, Prec prec,
                              const double* diag, const int* state, const int* active, const void* in,
                              const void* cin, void* out, double* partial, int* ran, hipStream_t st) {
  auto go = [&](auto op) {
    using Op = decltype(op);
    using T = typename Op::T;
    const size_t lds = Op::NC == 3 ? eo_lds_bytes(g, mm, prec) : 0;
    if (mm.TS == 2 * (kBlock >> 4)) {             // 32-site tiles (the scalar form): 512 threads
      if (mode == 0)
        k_eo_hop_pair<Op, 0, 2 * kBlock><<<mm.grid, 2 * kBlock, lds, st>>>(
            g, mm, P, op, diag, od.coupling, state, active, (const T*)in, nullptr, (T*)out, nullptr, ran);
      else
        k_eo_hop_pair<Op, 1, 2 * kBlock><<<mm.grid, 2 * kBlock, lds, st>>>(
            g, mm, P, op, diag, od.coupling, state, active, (const T*)in, (const T*)cin, (T*)out, partial, ran);
      return;
    }
    if (mode == 0)
      k_eo_hop_pair<Op, 0><<<mm.grid, kBlock, lds, st>>>(g, mm, P, op, diag, od.coupling, state, active,
                                                        (const T*)in, nullptr, (T*)out, nullptr, ran);
    else
      k_eo_hop_pair<Op, 1><<<mm.grid, kBlock, lds, st>>>(g, mm, P, op, diag, od.coupling, state, active,
                                                        (const T*)in, (const T*)cin, (T*)out, partial, ran);
  };
  if (od.kind == 1 && prec == Prec::kF32) go(CovOp<float2>{reinterpret_cast<const float2*>(od.links_eo)});
  else if (od.kind == 0 && prec == Prec::kF64) go(ScalarOp<double>{});
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_eo_init_odd(const Geom& g, Elem elem, Prec prec, int logB, int64_t rhs0, int nb, uint64_t seed,
                              int mask, const double* diag, void* to, hipStream_t st) {
  const unsigned grid = cdiv(g.V >> 1, (size_t)(kBlock >> logB));
  return by_elem(elem, prec, [&](auto tv) {
    using T = decltype(tv);
    if (g.ncomp == 3) k_eo_init_odd<T, 3><<<grid, kBlock, 0, st>>>(g, logB, rhs0, nb, seed, mask, diag, (T*)to);
    else k_eo_init_odd<T, 1><<<grid, kBlock, 0, st>>>(g, logB, rhs0, nb, seed, mask, diag, (T*)to);
  });
}

hipError_t launch_eo_scatter_even(const Geom& g, Elem elem, Prec prec, int logB, const void* xe, void* x,
                                  hipStream_t st) {
  const unsigned grid = cdiv(g.V >> 1, (size_t)(kBlock >> logB));
  return by_elem(elem, prec, [&](auto tv) {
    using T = decltype(tv);
    if (g.ncomp == 3) k_eo_scatter_even<T, 3><<<grid, kBlock, 0, st>>>(g, logB, (const T*)xe, (T*)x);
    else k_eo_scatter_even<T, 1><<<grid, kBlock, 0, st>>>(g, logB, (const T*)xe, (T*)x);
  });
}

hipError_t launch_diag(const Geom& g, const double* mass_field, double mass, const double* w, double* out,
                       hipStream_t st) {
  k_diag<<<cdiv(g.V, kBlock), kBlock, 0, st>>>(g, mass_field, mass, w, out);
  return hipGetLastError();
}

hipError_t launch_reduce_rho0(const CgScalars& sc, int B, const double* partial, int gx, hipStream_t st) {
  k_reduce_rho0<<<B, kBlock, 0, st>>>(sc, partial, gx);
  return hipGetLastError();
}

hipError_t launch_grad_accum(const OpDev& od64, const Geom& g, Elem elem, int logB, int nb, const void* x, double* gm,
                             double* gw, hipStream_t st) {
  const unsigned grid = cdiv(g.V, (size_t)(kBlock >> logB));
  return dispatch64(od64, elem, [&](auto op) {
    using Op = decltype(op);
    using T = typename Op::T;
    k_grad_accum<Op><<<grid, kBlock, 0, st>>>(g, logB, nb, op, (const T*)x, gm, gw);
  });
}

hipError_t launch_scale(size_t n, double* a, double f, hipStream_t st) {
  k_scale<<<cdiv(n, kBlock), kBlock, 0, st>>>(n, a, f);
  return hipGetLastError();
}

hipError_t launch_fill(size_t n, double* a, double v, hipStream_t st) {
  k_fill<<<cdiv(n, kBlock), kBlock, 0, st>>>(n, a, v);
  return hipGetLastError();
}

hipError_t launch_eo_cast_init(size_t n, Elem elem, const void* bh, void* r, void* p, void* xh, hipStream_t st) {
  const unsigned grid = cdiv(n, kBlock);
  if (elem == Elem::kReal)
    k_eo_cast_init<double, float><<<grid, kBlock, 0, st>>>(n, (const double*)bh, (float*)r, (float*)p, (float*)xh);
  else
    k_eo_cast_init<double2, float2><<<grid, kBlock, 0, st>>>(n, (const double2*)bh, (float2*)r, (float2*)p,
                                                             (float2*)xh);
  return hipGetLastError();
}

hipError_t launch_cast_links(size_t n, const double2* src, float2* dst, hipStream_t st) {
  k_cast_links<<<cdiv(n, kBlock), kBlock, 0, st>>>(n, src, dst);
  return hipGetLastError();
}

hipError_t launch_scalars_init(const CgScalars& sc, int nb, int B, double bnorm2, int start_frozen, hipStream_t st) {
  k_scalars_init<<<(B + 255) / 256, 256, 0, st>>>(sc, nb, B, bnorm2, start_frozen);
  return hipGetLastError();
}

hipError_t launch_reduce_alpha(const CgScalars& sc, int B, const double* partial, int gx, hipStream_t st, int soft,
                               int force_iter) {
  k_reduce_alpha<<<B, kBlock, 0, st>>>(sc, partial, gx, soft, force_iter);
  return hipGetLastError();
}

hipError_t launch_reduce_beta(const CgScalars& sc, int B, const double* partial, int gx, double tol2, int max_iter,
                              double delta2, hipStream_t st, double first2, double eps, double tau2) {
  k_reduce_beta<<<B, kWideBlock, 0, st>>>(sc, partial, gx, tol2, max_iter, delta2, first2 > 0.0 ? first2 : tol2,
                                          eps, tau2);
  return hipGetLastError();
}

hipError_t launch_reduce_true(const CgScalars& sc, int B, const double* partial, int gx, size_t pstride, double tol2,
                              int max_iter, int max_restarts, hipStream_t st, const double* partial2) {
  k_reduce_true<<<B, kBlock, 0, st>>>(sc, partial, partial2, gx, pstride, tol2, max_iter, max_restarts);
  return hipGetLastError();
}

hipError_t launch_hier_perm(const Geom& g, uint32_t* out, hipStream_t st) {
  k_hier_perm<<<cdiv(g.V, kBlock), kBlock, 0, st>>>(g, out);
  return hipGetLastError();
}

hipError_t launch_probe_vectors(const Geom& g, uint64_t seed, int mask, int64_t m0, int count, int comp, double2* out,
                                hipStream_t st) {
  k_probe_vectors<<<dim3(cdiv(g.V, kBlock), count), kBlock, 0, st>>>(g, seed, mask, m0, comp, out);
  return hipGetLastError();
}

// Links of the even-odd kernels: [parity][mu][9][V/2], the site of parity P at
// half-lattice index h holding U_mu(site) at [P][mu][e][h].  A tile of
// consecutive h then reads whole cache lines of links (in the full-lattice
// layout its sites alternate between two t planes).
__global__ __launch_bounds__(kBlock) void k_repack_links_eo(Geom g, const double2* __restrict__ links,
                                                            double2* __restrict__ dst) {
  const uint32_t s = blockIdx.x * kBlock + threadIdx.x;
  if (s >= g.V) return;
  const int mu = blockIdx.y;
  const int tdim = g.ndim - 1;
  const uint32_t t = coord_p2(s, g, tdim);
  const uint32_t P = (spatial_parity(s, g) + t) & 1u;
  const uint32_t V3 = 1u << g.shift[tdim];
  const uint32_t h = (s & (V3 - 1u)) + V3 * (t >> 1);
  const size_t V = g.V, Vh = V >> 1;
#pragma unroll
  for (int e = 0; e < 9; ++e) dst[(((size_t)P * g.ndim + mu) * 9 + e) * Vh + h] = links[((size_t)mu * 9 + e) * V + s];
}

hipError_t launch_repack_links_eo(const Geom& g, const double2* links, double2* dst, hipStream_t st) {
  k_repack_links_eo<<<dim3(cdiv(g.V, kBlock), g.ndim), kBlock, 0, st>>>(g, links, dst);
  return hipGetLastError();
}

hipError_t launch_repack_links(const Geom& g, const double2* src, double2* dst, hipStream_t st) {
  k_repack_links<<<dim3(cdiv(g.V, kBlock), g.ndim), kBlock, 0, st>>>(g, src, dst);
  return hipGetLastError();
}

hipError_t launch_layout(const Geom& g, Elem elem, int logB, int lane, const void* src, void* dst,
                         bool to_comp_major, hipStream_t st) {
  const unsigned grid = cdiv(g.V, kBlock);
  if (elem == Elem::kReal) {
    if (to_comp_major)
      k_site_major_to_comp_major<double><<<grid, kBlock, 0, st>>>(g, logB, lane, (const double*)src, (double*)dst);
    else
      k_comp_major_to_site_major<double><<<grid, kBlock, 0, st>>>(g, logB, lane, (const double*)src, (double*)dst);
  } else {
    if (to_comp_major)
      k_site_major_to_comp_major<double2><<<grid, kBlock, 0, st>>>(g, logB, lane, (const double2*)src,
                                                                    (double2*)dst);
    else
      k_comp_major_to_site_major<double2><<<grid, kBlock, 0, st>>>(g, logB, lane, (const double2*)src,
                                                                    (double2*)dst);
  }
  return hipGetLastError();
}

}  // namespace tip
