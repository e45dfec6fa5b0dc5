// Device building blocks shared by the single-problem kernels (tip_kernels.hip)
// and the batched ones (tip_batch.hip): operator policies, vector access in
// the block layout [ncomp][V][B], the stencil at one (site, rhs), the
// per-rhs workgroup sums, the probing right-hand side at a site, the
// fixed-order partial sums of the CG reductions, and the per-rhs scalar
// steps of CG (alpha, beta, the true-residual check, the reliable update).
#pragma once

#include "tip_device.h"
#include "tip_launch.h"

namespace tip {

extern __shared__ __align__(16) unsigned char tip_dyn_lds[];

// ---------------------------------------------------------------------------
// Operator policies and small helpers
// ---------------------------------------------------------------------------

template <class C>
struct CovOp {                         // 3 complex components, links U_mu (C = double2 or float2)
  using T = C;
  static constexpr int NC = 3;
  const C* __restrict__ U;
};

template <class TT>
struct ScalarOp {                      // 1 component, real or complex vectors
  using T = TT;
  static constexpr int NC = 1;
};

// Single-precision type of an FP64 vector element.
template <class T> struct SingleOf;
template <> struct SingleOf<double> { using type = float; };
template <> struct SingleOf<double2> { using type = float2; };
template <> struct SingleOf<float> { using type = float; };      // already single
template <> struct SingleOf<float2> { using type = float2; };

// y = U x and y = U^H x for a 3x3 complex matrix u[3a+b].
template <class C>
__device__ __forceinline__ void mul_u(const C (&u)[9], const C (&x)[3], C (&y)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    C t = zero<C>();
#pragma unroll
    for (int b = 0; b < 3; ++b) t = cfma(u[3 * a + b], x[b], t);
    y[a] = t;
  }
}
template <class C>
__device__ __forceinline__ void mul_uh(const C (&u)[9], const C (&x)[3], C (&y)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    C t = zero<C>();
#pragma unroll
    for (int b = 0; b < 3; ++b) t = cfma_conj(u[3 * b + a], x[b], t);
    y[a] = t;
  }
}

// y += U x and y += U^H x, accumulated straight into y (one FMA chain per
// component, no separate product and add); the single-precision pair hops
// use them.
template <class C>
__device__ __forceinline__ void mul_u_acc(const C (&u)[9], const C (&x)[3], C (&y)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) y[a] = cfma(u[3 * a + b], x[b], y[a]);
}
template <class C>
__device__ __forceinline__ void mul_uh_acc(const C (&u)[9], const C (&x)[3], C (&y)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) y[a] = cfma_conj(u[3 * b + a], x[b], y[a]);
}

template <class C>
__device__ __forceinline__ void load_link(const CovOp<C>& op, size_t V, int mu, uint32_t s, C (&u)[9]) {
  const C* Um = op.U + (size_t)mu * 9 * V;
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = Um[(size_t)e * V + s];
}

// x at (site s, rhs lane j) for all components: in[(c V + s) B + j]
template <class T, int NC>
__device__ __forceinline__ void load_vec(const T* __restrict__ in, size_t V, int logB, uint32_t s, int j, T (&x)[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) x[c] = in[((((size_t)c * V + s)) << logB) + j];
}
template <class T, int NC>
__device__ __forceinline__ void store_vec(T* __restrict__ out, size_t V, int logB, uint32_t s, int j, const T (&x)[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) out[((((size_t)c * V + s)) << logB) + j] = x[c];
}

// Streaming forms for data a kernel touches once: the lines are not kept in
// L2, which leaves room for the neighbour data that other workgroups reuse.
__device__ __forceinline__ void st_nt(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_nt(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_nt(double2* p, double2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}
__device__ __forceinline__ void st_nt(float2* p, float2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}
__device__ __forceinline__ double ld_nt(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ld_nt(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ double2 ld_nt(const double2* p) {
  return make_double2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}
__device__ __forceinline__ float2 ld_nt(const float2* p) {
  return make_float2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}
template <class T, int NC>
__device__ __forceinline__ void store_vec_nt(T* __restrict__ out, size_t V, int logB, uint32_t s, int j,
                                             const T (&x)[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) st_nt(&out[((((size_t)c * V + s)) << logB) + j], x[c]);
}
template <class T, int NC>
__device__ __forceinline__ void load_vec_nt(const T* __restrict__ in, size_t V, int logB, uint32_t s, int j,
                                            T (&x)[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) x[c] = ld_nt(&in[((((size_t)c * V + s)) << logB) + j]);
}

// One hop term h = U x (fwd) or U^H x (bwd) for the operator policy.
template <class Op>
__device__ __forceinline__ void hop_term(const Op&, size_t, int, uint32_t, bool,
                                         const typename Op::T (&x)[Op::NC], typename Op::T (&h)[Op::NC]) {
  h[0] = x[0];
}
template <class C>
__device__ __forceinline__ void hop_term(const CovOp<C>& op, size_t V, int mu, uint32_t s_link, bool backward,
                                         const C (&x)[3], C (&h)[3]) {
  C u[9];
  load_link(op, V, mu, s_link, u);
  if (backward) mul_uh(u, x, h);
  else mul_u(u, x, h);
}

// acc += wgt * h
template <class T, int NC>
__device__ __forceinline__ void add_weighted(double wgt, const T (&h)[NC], T (&acc)[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = axpy(wgt, h[c], acc[c]);
}

// Sum per right-hand side over a 256-thread workgroup whose lane l holds rhs
// l mod B: a shuffle tree inside each wave down to B lanes, then the four
// wave results through LDS.  Threads tid < B end with the totals of rhs tid.
template <int N, int W = 4>
__device__ __forceinline__ void seg_sum(double (&v)[N], int B, double* lds /* [N][W][64] */) {
#pragma unroll
  for (int i = 0; i < N; ++i)
    for (int off = 32; off >= B; off >>= 1) v[i] += __shfl_down(v[i], off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane < B) {
#pragma unroll
    for (int i = 0; i < N; ++i) lds[(i * W + wave) * 64 + lane] = v[i];
  }
  __syncthreads();
  if ((int)threadIdx.x < B) {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      // pairs of waves, then pairs of pairs: a fixed order for any W
      double q[W];
#pragma unroll
      for (int w = 0; w < W; ++w) q[w] = lds[(i * W + w) * 64 + t];
#pragma unroll
      for (int h = 1; h < W; h <<= 1)
#pragma unroll
        for (int w = 0; w + h < W; w += 2 * h) q[w] += q[w + h];
      v[i] = q[0];
    }
  }
}

// ---------------------------------------------------------------------------
// Site tiles: a workgroup owns TS = 256/B sites x B right-hand sides.
// ---------------------------------------------------------------------------

// First site of tile b in the generic (one site per thread) kernels.
// Workgroups are dispatched round-robin over the XCDs (b mod 8), so tile b
// and tile b+1 land on different L2 caches.  When the geometry allows, XCD k
// instead gets a contiguous chunk of pc planes of the last (slowest)
// dimension and walks it with that dimension innermost, so the +-mu
// neighbours a tile needs were fetched into the same L2 by tiles dispatched
// shortly before it.  The map is a bijection of the tiles; it changes only
// which workgroup computes which sites, never the arithmetic of a site.
__device__ __forceinline__ uint32_t tile_first_site(uint32_t b, const TileMap& tm) {
  if (tm.pc == 0) return b * (uint32_t)tm.TS;
  const uint32_t xcd = b % kNumXcd, slot = b / kNumXcd;
  const uint32_t t_local = slot % (uint32_t)tm.pc, q = slot / (uint32_t)tm.pc;
  return ((xcd * (uint32_t)tm.pc + t_local) * (uint32_t)tm.P + q) * (uint32_t)tm.TS;
}

// Stencil at one (site, rhs): y = diag x(s) - sum_mu [w_mu(s) U_mu(s) x(s+mu)
// + w_mu(s-mu) U_mu(s-mu)^H x(s-mu)], with the hop terms summed in the order
// mu = 0..ndim-1, forward before backward (the marching kernel keeps it).
// Nbr gives the periodic neighbours of s: nbr(mu, fwd).
template <class Op, class Nbr>
__device__ __forceinline__ void stencil_site_at(const Op& op, const Geom& g, int logB, uint32_t s, int j,
                                                const double* __restrict__ mass_field, double mass,
                                                const double* __restrict__ w, const typename Op::T* __restrict__ in,
                                                const Nbr& nbr, typename Op::T (&xs)[Op::NC],
                                                typename Op::T (&y)[Op::NC]) {
  using T = typename Op::T;
  constexpr int NC = Op::NC;
  const size_t V = g.V;
  T hop[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) hop[c] = zero<T>();
  double diag = mass_field ? mass_field[s] : mass;
#pragma unroll
  for (int mu = 0; mu < kMaxDim; ++mu) {
    if (mu >= g.ndim) break;
    const uint32_t sf = nbr(mu, true);
    const uint32_t sb = nbr(mu, false);
    const double wf = w ? w[(size_t)mu * V + s] : 1.0;
    const double wb = w ? w[(size_t)mu * V + sb] : 1.0;
    diag += wf + wb;
    T xn[NC], h[NC];
    load_vec<T, NC>(in, V, logB, sf, j, xn);
    hop_term(op, V, mu, s, false, xn, h);
    add_weighted<T, NC>(wf, h, hop);
    load_vec<T, NC>(in, V, logB, sb, j, xn);
    hop_term(op, V, mu, sb, true, xn, h);
    add_weighted<T, NC>(wb, h, hop);
  }
  load_vec<T, NC>(in, V, logB, s, j, xs);
#pragma unroll
  for (int c = 0; c < NC; ++c) y[c] = axpy(diag, xs[c], axpy(-1.0, hop[c], zero<T>()));
}

// The same site, with every load of the site (the 2 ndim neighbours, the
// site itself, the couplings and the mass) issued before any arithmetic, so a
// wave has them all in flight at once instead of one round trip per
// neighbour.  The arithmetic and its order are stencil_site_at's, so the
// result is the same bit for bit.  (The covariant operator's links are still
// loaded inside hop_term.)
template <class Op, class Nbr>
__device__ __forceinline__ void stencil_site_gather(const Op& op, const Geom& g, int logB, uint32_t s, int j,
                                                    const double* __restrict__ mass_field, double mass,
                                                    const double* __restrict__ w,
                                                    const typename Op::T* __restrict__ in, const Nbr& nbr,
                                                    typename Op::T (&xs)[Op::NC], typename Op::T (&y)[Op::NC]) {
  using T = typename Op::T;
  constexpr int NC = Op::NC;
  const size_t V = g.V;
  T xf[kMaxDim][NC], xb[kMaxDim][NC];
  double wf[kMaxDim], wb[kMaxDim];
  uint32_t sbk[kMaxDim];
#pragma unroll
  for (int mu = 0; mu < kMaxDim; ++mu) {
    if (mu >= g.ndim) break;
    const uint32_t sf = nbr(mu, true);
    sbk[mu] = nbr(mu, false);
    wf[mu] = w ? w[(size_t)mu * V + s] : 1.0;
    wb[mu] = w ? w[(size_t)mu * V + sbk[mu]] : 1.0;
    load_vec<T, NC>(in, V, logB, sf, j, xf[mu]);
    load_vec<T, NC>(in, V, logB, sbk[mu], j, xb[mu]);
  }
  load_vec<T, NC>(in, V, logB, s, j, xs);
  double diag = mass_field ? mass_field[s] : mass;
  T hop[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) hop[c] = zero<T>();
#pragma unroll
  for (int mu = 0; mu < kMaxDim; ++mu) {
    if (mu >= g.ndim) break;
    diag += wf[mu] + wb[mu];
    T h[NC];
    hop_term(op, V, mu, s, false, xf[mu], h);
    add_weighted<T, NC>(wf[mu], h, hop);
    hop_term(op, V, mu, sbk[mu], true, xb[mu], h);
    add_weighted<T, NC>(wb[mu], h, hop);
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) y[c] = axpy(diag, xs[c], axpy(-1.0, hop[c], zero<T>()));
}

// Scalar operators in a workgroup pass whose steps are synchronised anyway:
// the 2 ndim + 1 scalars of site s (w_mu(s) for mu < ndim, w_mu(s - e_mu),
// then m(s)) are read once per site, value k by lane k of the site's B lanes
// (lanes k, k + B, ... when B < 2 ndim + 1), into sv[k]; after the barrier
// stencil_site_lds takes them from there.  One load per site instead of one
// per lane: with every lane loading them, the scalars took as many address
// cycles as the vector entries.
template <class Nbr>
__device__ __forceinline__ void site_scalars_split(const Geom& g, uint32_t s, int j, int B,
                                                   const double* __restrict__ mass_field, double mass,
                                                   const double* __restrict__ w, const Nbr& nbr, double* sv) {
  const int nd = g.ndim, nv = 2 * nd + 1;
  for (int k = j; k < nv; k += B) {
    double v;
    if (k < 2 * nd) {
      const int mu = k < nd ? k : k - nd;
      uint32_t sk = s;
      if (k >= nd) {
#pragma unroll
        for (int m = 0; m < kMaxDim; ++m)
          if (m == mu) sk = nbr(m, false);
      }
      v = w ? w[(size_t)mu * g.V + sk] : 1.0;
    } else {
      v = mass_field ? mass_field[s] : mass;
    }
    sv[k] = v;
  }
}
constexpr int kSiteScalarStride = 2 * kMaxDim + 2;   // doubles per site in sv

// stencil_site_gather for the scalar operators with the site's scalars from
// sv (site_scalars_split); the same arithmetic in the same order.
template <class T, class Nbr>
__device__ __forceinline__ void stencil_site_lds(const Geom& g, int logB, uint32_t s, int j, const double* sv,
                                                 const T* __restrict__ in, const Nbr& nbr, T (&xs)[1], T (&y)[1]) {
  const size_t V = g.V;
  T xf[kMaxDim][1], xb[kMaxDim][1];
#pragma unroll
  for (int mu = 0; mu < kMaxDim; ++mu) {
    if (mu >= g.ndim) break;
    load_vec<T, 1>(in, V, logB, nbr(mu, true), j, xf[mu]);
    load_vec<T, 1>(in, V, logB, nbr(mu, false), j, xb[mu]);
  }
  load_vec<T, 1>(in, V, logB, s, j, xs);
  double diag = sv[2 * g.ndim];
  T hop = zero<T>();
#pragma unroll
  for (int mu = 0; mu < kMaxDim; ++mu) {
    if (mu >= g.ndim) break;
    const double wf = sv[mu], wb = sv[g.ndim + mu];
    diag += wf + wb;
    hop = axpy(wf, xf[mu][0], hop);
    hop = axpy(wb, xb[mu][0], hop);
  }
  y[0] = axpy(diag, xs[0], axpy(-1.0, hop, zero<T>()));
}

template <class Op>
__device__ __forceinline__ void stencil_site(const Op& op, const Geom& g, int logB, uint32_t s, int j,
                                             const double* __restrict__ mass_field, double mass,
                                             const double* __restrict__ w, const typename Op::T* __restrict__ in,
                                             typename Op::T (&xs)[Op::NC], typename Op::T (&y)[Op::NC]) {
  auto nbr = [&](int mu, bool fwd) { return fwd ? nbr_fwd(s, g, mu) : nbr_bwd(s, g, mu); };
  stencil_site_at(op, g, logB, s, j, mass_field, mass, w, in, nbr, xs, y);
}

// A site index with its coordinates, stepped forward without division on
// any sides: the periodic neighbours then follow from the coordinates.
struct SiteWalk {
  uint32_t s;
  uint32_t x[kMaxDim];
  __device__ __forceinline__ SiteWalk(uint32_t s0, const Geom& g) : s(s0) {
#pragma unroll
    for (int mu = 0; mu < kMaxDim; ++mu) x[mu] = mu < g.ndim ? coord(s0, g, mu) : 0u;
  }
  // s += d with the carries through the coordinates (d >= 0)
  __device__ __forceinline__ void advance(uint32_t d, const Geom& g) {
    s += d;
    uint32_t carry = d;
#pragma unroll
    for (int mu = 0; mu < kMaxDim; ++mu) {
      if (mu >= g.ndim || carry == 0u) break;
      uint32_t v = x[mu] + carry;
      const uint32_t n = g.n[mu];
      carry = 0u;
      if (v >= n) {
        if (v < 2u * n) {
          v -= n;
          carry = 1u;
        } else {
          carry = v / n;
          v -= carry * n;
        }
      }
      x[mu] = v;
    }
  }
  // periodic neighbour of s along mu
  __device__ __forceinline__ uint32_t nbr(int mu, bool fwd, const Geom& g) const {
    const uint32_t n = g.n[mu], st = g.stride[mu];
    if (fwd) return x[mu] == n - 1u ? s - (n - 1u) * st : s + st;
    return x[mu] == 0u ? s + (n - 1u) * st : s - st;
  }
};


// Entry (s, c) of right-hand side rhs0 + j (spatial probe (rhs0 + j) / ncomp
// through class_probe, component (rhs0 + j) % ncomp), for every component:
// zero except component c; zero for padding lanes j >= nb.
template <class T, int NC>
__device__ __forceinline__ void rhs_at(const Geom& g, uint32_t s, int64_t rhs0, int j, int nb,
                                       uint64_t seed, int mask, T (&b)[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) b[c] = zero<T>();
  if (j >= nb) return;
  const int64_t rg = rhs0 + j;
  const int cj = (int)(rg % NC);
  const T v = from_c<T>(probe_entry(s, class_probe((uint64_t)(rg / NC), g), cj, g, seed, mask));
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (c == cj) b[c] = v;
}

// The part of a hierarchical probe entry that depends on the site only
// (power-of-two sides, mask sweep 0, i.e. probes m < V): the site's location
// P(x) and, per component c, the mask value z0(x, c) = i^code (Z2: code 0 or
// 2; no mask: 0), two bits per component.
struct ProbeSiteCode {
  uint32_t P;
  uint32_t codes;
};
__device__ __forceinline__ ProbeSiteCode probe_site_code(uint32_t s, const Geom& g, uint64_t seed, int mask) {
  ProbeSiteCode pc;
  pc.P = hier_perm(s, g);
  pc.codes = 0u;
  if (mask != kMaskNone)
    for (int c = 0; c < g.ncomp; ++c) {
      const uint64_t u = splitmix64_at(seed, (uint64_t)s * (uint64_t)g.ncomp + (uint64_t)c);
      const uint32_t code = mask == kMaskZ2 ? ((u >> 63) ? 2u : 0u) : (uint32_t)(u >> 62);
      pc.codes |= code << (2 * c);
    }
  return pc;
}

// The part of the same entry that depends on the lane only: right-hand side
// rhs0 + j = m ncomp + c has its component c and Hadamard column bitrev_L(m);
// cj < 0 marks a padding lane (j >= nb).  Computed once per thread.
struct LaneProbe {
  int cj;
  uint32_t col;
};
template <int NC>
__device__ __forceinline__ LaneProbe lane_probe(const Geom& g, int64_t rhs0, int j, int nb) {
  LaneProbe lp{-1, 0u};
  if (j < nb) {
    const int64_t rg = rhs0 + j;
    lp.cj = (int)(rg % NC);
    lp.col = hadamard_column((uint32_t)(rg / NC), g.L);
  }
  return lp;
}

// b of a lane from its site's ProbeSiteCode: z0(x, c) H(P(x), bitrev_L(m)) on
// component c (the same exact value rhs_at computes), zero elsewhere.
template <class T, int NC>
__device__ __forceinline__ void rhs_from_code(const ProbeSiteCode& pc, const LaneProbe& lp, T (&b)[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) b[c] = zero<T>();
  if (lp.cj < 0) return;
  const double h = (__popc(pc.P & lp.col) & 1) ? -1.0 : 1.0;
  double2 v;
  switch ((pc.codes >> (2 * lp.cj)) & 3u) {            // i^code h
    case 0: v = make_double2(h, 0.0); break;
    case 1: v = make_double2(0.0, h); break;
    case 2: v = make_double2(-h, 0.0); break;
    default: v = make_double2(0.0, -h); break;
  }
  const T e = from_c<T>(v);
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (c == lp.cj) b[c] = e;
}

// ---------------------------------------------------------------------------
// Fixed-order sums of per-workgroup partials (the second stage of every CG
// reduction).
// ---------------------------------------------------------------------------

__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int n) {
  __shared__ double lds[4];
  // four independent running sums keep four loads in flight per thread; the
  // order of the additions is fixed, so the result is reproducible
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = threadIdx.x;
  for (; i + 3 * kBlock < n; i += 4 * kBlock) {
    a0 += part[i];
    a1 += part[i + kBlock];
    a2 += part[i + 2 * kBlock];
    a3 += part[i + 3 * kBlock];
  }
  for (; i < n; i += kBlock) a0 += part[i];
  double v[1] = {(a0 + a1) + (a2 + a3)};
  block_sum<1>(v, lds);
  return v[0];
}

// The same sum with a 1024-thread workgroup, for the update pass's partials
// (up to 32768 per rhs): four times the loads in flight of sum_partials.  Each
// thread keeps four running sums in a fixed order, then a shuffle tree per
// wave and the 16 wave results in order through LDS, so the result is
// reproducible.
constexpr int kWideBlock = 1024;
__device__ __forceinline__ double sum_partials_wide(const double* __restrict__ part, int n) {
  __shared__ double lds[kWideBlock / 64];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = threadIdx.x;
  for (; i + 3 * kWideBlock < n; i += 4 * kWideBlock) {
    a0 += part[i];
    a1 += part[i + kWideBlock];
    a2 += part[i + 2 * kWideBlock];
    a3 += part[i + 3 * kWideBlock];
  }
  for (; i < n; i += kWideBlock) a0 += part[i];
  double v = (a0 + a1) + (a2 + a3);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWideBlock / 64; ++w) t += lds[w];
    v = t;
  }
  return v;
}

// The same sum over two partial arrays (two passes that each cover part of
// the lattice); partial2 may be NULL.
__device__ __forceinline__ double sum_partials2(const double* __restrict__ p1, const double* __restrict__ p2,
                                                size_t off, int n) {
  const double a = sum_partials(p1 + off, n);
  return p2 ? a + sum_partials(p2 + off, n) : a;
}

// ---------------------------------------------------------------------------
// Per-rhs scalar steps of CG.  Each takes the sums of its reduction and runs
// on one thread for right-hand side j; the kernels that call them (one
// workgroup per rhs) differ only in where the partials of rhs j lie.
// ---------------------------------------------------------------------------

// alpha = rho / p^H A p; breakdown when p^H A p is not positive and finite.
// soft (mixed precision): a single-precision p^H A p <= 0 says nothing about
// the FP64 operator, so the solve is frozen instead and the FP64 true
// residual decides.  forced (tests): treat this iteration as a breakdown.
__device__ __forceinline__ void lane_alpha(const CgScalars& sc, int j, double pAp, int soft, bool forced) {
  if (!(pAp > 0.0) || !isfinite(pAp) || forced) {
    sc.state[j] = soft ? kFrozen : kBreakdown;
    atomicSub(sc.active, 1);
    return;
  }
  const double pp = sc.pp[j];
  sc.alpha[j] = sc.rho[j] / pAp;
  if (pp > 0.0) sc.anorm[j] = fmax(sc.anorm[j], pAp / pp);
}

// The rhs's scalars that the beta step reads, loaded before the reduction so
// that their latency overlaps it.
struct BetaIn {
  double alpha, rho_old, pp, xh0, dev0, anorm, rho_ref, bnorm2;
  int it, restarted, flagged;
};
__device__ __forceinline__ BetaIn lane_beta_read(const CgScalars& sc, int j) {
  BetaIn b;
  b.alpha = sc.alpha[j];
  b.rho_old = sc.rho[j];
  b.pp = sc.pp[j];
  b.xh0 = sc.xhn[j];
  b.dev0 = sc.dev[j];
  b.anorm = sc.anorm[j];
  b.rho_ref = sc.rho_ref[j];
  b.bnorm2 = sc.bnorm2[j];
  b.it = sc.iters[j] + 1;
  b.restarted = sc.restarts[j];
  b.flagged = sc.ru[j];
  return b;
}

// rho' = ||r||^2; beta = rho'/rho; freeze on the recursive residual, or stop
// at max_iter.  xalpha = the x update the direction pass applies this
// iteration.
//
// Mixed precision (eps = the single-precision unit roundoff; 0 in FP64): the
// gap between the true residual b - A x and the recursive r grows by the
// rounding of x_h += alpha p and of r -= alpha A p.  Following van der Vorst &
// Ye (SIAM J. Sci. Comput. 22 (2000) 835) it is bounded from scalars CG
// already has, d += eps (||A|| (||x_h|| + |alpha| ||p||) + ||r|| + ||r'||), with
// ||A|| estimated by the largest Rayleigh quotient, ||p||^2 by its recurrence
// and ||x_h|| <= sum |alpha| ||p||.  A reliable update (residual replacement)
// is asked for once d^2 > tau2 ||r'||^2, so the recursive residual stays
// within a factor 1 +- sqrt(tau2) of the true one, and (delta2 > 0) also
// when ||r'||^2 has fallen by delta2 since the last update.
__device__ __forceinline__ void lane_beta(const CgScalars& sc, int j, const BetaIn& in, double rho_new, double tol2,
                                          int max_iter, double delta2, double first2, double eps, double tau2) {
  sc.xalpha[j] = in.alpha;
  sc.iters[j] = in.it;
  const double beta = rho_new / in.rho_old;
  sc.beta[j] = beta;
  sc.rho[j] = rho_new;
  const double step = fabs(in.alpha) * sqrt(in.pp);
  const double xh = in.xh0 + step;
  const double dev = in.dev0 + eps * (in.anorm * (xh + step) + sqrt(in.rho_old) + sqrt(rho_new));
  sc.xhn[j] = xh;
  sc.dev[j] = dev;
  sc.pp[j] = rho_new + beta * beta * in.pp;
  if (!isfinite(rho_new)) {
    sc.state[j] = kBreakdown;
    atomicSub(sc.active, 1);
  } else if (rho_new <= (in.restarted == 0 ? first2 : tol2) * in.bnorm2) {
    sc.state[j] = kFrozen;
    atomicSub(sc.active, 1);
  } else if (in.it >= max_iter) {
    sc.state[j] = kNoConv;
    atomicSub(sc.active, 1);
  } else if (in.flagged == 0 && (dev * dev > tau2 * rho_new || rho_new < delta2 * in.rho_ref)) {
    sc.ru[j] = 1;                              // ask for a reliable update
    atomicAdd(sc.n_ru, 1);
  }
}

// FP64 check of a frozen solve: accept when the true residual passes (with
// the quadrature b^H x), else restart CG from x (r and p already hold the
// true residual) while the restart budget lasts.
__device__ __forceinline__ void lane_true(const CgScalars& sc, int j, double rt2, double qre, double qim, double tol2,
                                          int max_iter, int max_restarts) {
  sc.relres2[j] = rt2 / sc.bnorm2[j];
  if (rt2 <= tol2 * sc.bnorm2[j]) {
    sc.state[j] = kAccepted;
    sc.q[2 * j] = qre;
    sc.q[2 * j + 1] = qim;
  } else if (sc.restarts[j] < max_restarts && sc.iters[j] < max_iter && isfinite(rt2)) {
    sc.state[j] = kActive;
    sc.rho[j] = rt2;
    sc.pp[j] = rt2;                            // p = r
    sc.restarts[j] += 1;
    atomicAdd(sc.active, 1);
  } else {
    sc.state[j] = kNoConv;
  }
}

// Mixed precision.  Mode 0: the recursive residual restarts from the true one
// (a reliable update).  Mode 1: accept with the variational quadrature
// b^H x + x^H r = 2 Re(b^H x) - x^H A x, whose error r^H A^-1 r is second
// order in the residual, or restart CG from x.  v: ||r||^2, Re/Im b^H x,
// Re/Im x^H r.
__device__ __forceinline__ void lane_ru(const CgScalars& sc, int j, const double (&v)[5], int mode, double tol2,
                                        int max_iter, int max_restarts) {
  const double rt2 = v[0];
  if (sc.ru[j]) {
    sc.ru[j] = 0;
    atomicSub(sc.n_ru, 1);
  }
  sc.xhn[j] = 0.0;                             // x_h is in x now; r is the true residual
  sc.dev[j] = 0.0;
  if (mode == 0) {
    sc.rho[j] = rt2;
    sc.rho_ref[j] = rt2;
    atomicAdd(sc.ru_count, 1);
    if (sc.ru_lanes) sc.ru_lanes[j] += 1;
    return;
  }
  sc.relres2[j] = rt2 / sc.bnorm2[j];
  if (rt2 <= tol2 * sc.bnorm2[j]) {
    sc.state[j] = kAccepted;
    sc.q[2 * j] = v[1] + v[3];
    sc.q[2 * j + 1] = v[2] + v[4];
  } else if (sc.restarts[j] < max_restarts && sc.iters[j] < max_iter && isfinite(rt2)) {
    sc.state[j] = kActive;
    sc.rho[j] = rt2;
    sc.rho_ref[j] = rt2;
    sc.pp[j] = rt2;                            // p = r
    sc.restarts[j] += 1;
    atomicAdd(sc.active, 1);
  } else {
    sc.state[j] = kNoConv;
  }
}

// Lanes a reliable-update pass works on: 0 = flagged for an update and still
// iterating, 1 = frozen (final check).
__device__ __forceinline__ bool ru_selected(const CgScalars& sc, int mode, int j) {
  return mode == 0 ? (sc.ru[j] != 0 && sc.state[j] == kActive) : sc.state[j] == kFrozen;
}

}  // namespace tip
