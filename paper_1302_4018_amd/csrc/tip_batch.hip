// Batched kernels: many independent problems (e.g. 64 tori of uneven sides,
// Sec. 3.4) solved together, one launch per CG phase for every problem of a
// group.
//
// Each problem's right-hand sides are split into jobs: blocks of B = 2^logB
// right-hand sides in the block layout [ncomp][V][B] of that problem, placed
// one after another in the group's vector arrays.  A job's sites are cut
// into work items of `item_sites` consecutive sites (a multiple of the tile
// of 256 / B sites); workgroup b of a launch takes item item_base + b, finds
// its job in item_job[] and walks the item one tile (256 threads = 256 / B
// sites x B rhs) at a time.  Lanes are numbered globally (job lane0 + j), so
// one array of CG scalars serves every problem, and the partials of a
// per-rhs reduction are stored per lane: partial[lane * PI + item - item0],
// PI = the most items any job has.  The scalar steps are those of the
// single-problem solver (lane_alpha, lane_beta, lane_true, lane_ru), with each
// problem's own tolerance and iteration cap.
//
// A workgroup none of whose rhs is live returns at once, so problems that
// have converged cost a launch slot each, not memory traffic.

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "tip_batch.h"
#include "tip_kernel_common.h"

namespace tip {

namespace {

// CG scalars of job J (lane j of the job is entry j of every array).
__device__ __forceinline__ CgScalars job_scalars(const CgScalars& sc, int lane0) {
  CgScalars s = sc;
  s.rho += lane0;
  s.alpha += lane0;
  s.xalpha += lane0;
  s.beta += lane0;
  s.rho_ref += lane0;
  s.pp += lane0;
  s.anorm += lane0;
  s.xhn += lane0;
  s.dev += lane0;
  s.bnorm2 += lane0;
  s.relres2 += lane0;
  s.q += 2 * lane0;
  s.state += lane0;
  s.iters += lane0;
  s.restarts += lane0;
  s.ru += lane0;
  return s;
}

// Operator policy of a problem: the links in the vector type's precision.
template <class Op> struct BatchOpOf;
template <class TT> struct BatchOpOf<ScalarOp<TT>> {
  __device__ static ScalarOp<TT> get(const BatchProb&) { return ScalarOp<TT>{}; }
};
template <class C> struct BatchOpOf<CovOp<C>> {
  __device__ static CovOp<C> get(const BatchProb& P) {
    return CovOp<C>{(const C*)(sizeof(C) == sizeof(float2) ? P.links32 : P.links)};
  }
};

// Per-lane sum of a workgroup's values, stored as partial row entry of lane
// lane0 + j and item `local` (threads j < B hold the totals after seg_sum).
template <int N>
__device__ __forceinline__ void store_partials(double (&acc)[N], int B, double* lds, double* __restrict__ partial,
                                               size_t rowstride, size_t PI, int lane0, uint32_t local) {
  seg_sum<N, kBlock / 64>(acc, B, lds);
  if ((int)threadIdx.x < B) {
#pragma unroll
    for (int k = 0; k < N; ++k) partial[k * rowstride + (size_t)(lane0 + (int)threadIdx.x) * PI + local] = acc[k];
  }
}

// Hierarchical probes on any sides, split like the even-odd passes' probe
// cache: the part of an entry that depends on the site (P(x) and the colour
// of the three-colouring level) once per site and step, shared by the site's
// B lanes through LDS, and the part that depends on the lane (its component,
// its column through class_probe and probe_column) once per thread.  The
// entry is then probe_value's, bit for bit.
struct SiteCode {
  uint32_t P, c3;
};
__device__ __forceinline__ SiteCode site_code(uint32_t s, const Geom& g) {
  return {hier_perm(s, g), g.has3 ? three_colour(s, g) : 0u};
}
struct LaneCode {
  int cj;                      // component; -1 for a padding lane
  ProbeCol pc;
};
template <int NC>
__device__ __forceinline__ LaneCode lane_code(const Geom& g, int64_t rhs0, int j, int nb) {
  LaneCode lc{-1, {0u, 0u, 0u}};
  if (j < nb) {
    const int64_t rg = rhs0 + j;
    lc.cj = (int)(rg % NC);
    lc.pc = probe_column(class_probe((uint64_t)(rg / NC), g), g);
  }
  return lc;
}
template <class T, int NC>
__device__ __forceinline__ void rhs_coded(const SiteCode& sc, const LaneCode& lc, uint32_t s, const Geom& g,
                                          uint64_t seed, int mask, T (&b)[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) b[c] = zero<T>();
  if (lc.cj < 0) return;
  const T v = from_c<T>(probe_value_c3(s, sc.P, sc.c3, lc.pc, lc.cj, g, seed, mask));
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (c == lc.cj) b[c] = v;
}

}  // namespace

// x = 0 and r = p = b (FP64); mixed: x64 = 0, xh = 0, r = p = single(b).
template <class T64, class TW, int NC>
__global__ __launch_bounds__(kBlock) void kb_init(BatchArgs a, T64* __restrict__ x64, TW* __restrict__ xh,
                                                  TW* __restrict__ r, TW* __restrict__ p) {
  __shared__ SiteCode lds_code[kBlock];
  const uint32_t item = a.item_base + blockIdx.x;
  const BatchJob& J = a.jobs[a.item_job[item]];
  const BatchProb P = a.probs[J.prob];
  const Geom g = J.g;
  const int logB = J.logB, B = 1 << logB;
  const int j = threadIdx.x & (B - 1), si = threadIdx.x >> logB;
  const uint32_t s0 = (item - J.item0) * (uint32_t)a.item_sites;
  const uint32_t s1 = min(g.V, s0 + (uint32_t)a.item_sites);
  const uint32_t TS = (uint32_t)(kBlock >> logB);
  const bool hier = g.probe == kProbeHierarchical;
  const LaneCode lc = lane_code<NC>(g, J.rhs0, j, J.nb);
  T64* xj = x64 + J.off;
  for (uint32_t base = s0; base < s1; base += TS) {
    const uint32_t s = base + (uint32_t)si;
    if (hier) {
      __syncthreads();
      if (j == 0 && s < s1) lds_code[si] = site_code(s, g);
      __syncthreads();
    }
    if (s >= s1) continue;
    TW b[NC], zw[NC];
    T64 z64[NC];
    if (hier) rhs_coded<TW, NC>(lds_code[si], lc, s, g, P.seed, P.mask, b);
    else rhs_at<TW, NC>(g, s, J.rhs0, j, J.nb, P.seed, P.mask, b);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      zw[c] = zero<TW>();
      z64[c] = zero<T64>();
    }
    store_vec<T64, NC>(xj, g.V, logB, s, j, z64);
    if (xh) store_vec<TW, NC>(xh + J.off, g.V, logB, s, j, zw);
    store_vec<TW, NC>(r + J.off, g.V, logB, s, j, b);
    store_vec<TW, NC>(p + J.off, g.V, logB, s, j, b);
  }
}

// The iteration's stencil visits a job's sites in march order.  The job's
// plane (its first ndim - 1 dimensions, Vp sites) is cut into columns of TS =
// 256 / B consecutive plane sites; march index o runs through column c, slice
// t (the last coordinate) and offset i as o = (c nt + t) TS + i, and through
// the last column, when TS does not divide Vp, as o = F + t wl + i (wl its
// width, F the indices of the whole columns).  A thread that starts at o0 + i
// and steps by TS keeps its plane site and moves one slice per step: the
// workgroup marches its column through the slices, so a site's t-neighbours
// are the sites of its previous and next steps, and the plane neighbours lie
// in the columns that the neighbouring work items march at the same time.
struct MarchOrder {
  uint32_t nt, Vp, TS, full, F, wl;
  __device__ __forceinline__ MarchOrder(const Geom& g, uint32_t TS_) : TS(TS_) {
    nt = 1u;
#pragma unroll
    for (int mu = 0; mu < kMaxDim; ++mu)   // constant indices keep g in registers
      if (mu == g.ndim - 1) nt = g.n[mu];
    Vp = g.V / nt;
    full = Vp / TS * TS;
    F = full * nt;
    wl = Vp - full;
  }
  // site of march index o, and its slice
  __device__ __forceinline__ uint32_t site(uint32_t o, uint32_t& t) const {
    if (o < F) {
      const uint32_t c = o / (TS * nt), rem = o - c * TS * nt;
      t = rem / TS;
      return c * TS + (rem - t * TS) + Vp * t;
    }
    const uint32_t r = o - F;
    t = r / wl;
    return full + (r - t * wl) + Vp * t;
  }
};

// Work item of a job of n items taken by the job's bl-th workgroup when the
// items are dealt to the 8 XCDs in contiguous parts: workgroups go round
// robin to the XCDs, so those with the same bl mod 8 share one XCD, and that
// XCD gets the part x = bl mod 8 of the job's items (parts of n / 8 or
// n / 8 + 1 items), in order.  A bijection of [0, n).
__device__ __forceinline__ uint32_t xcd_part(uint32_t bl, uint32_t n) {
  const uint32_t x = bl & 7u, k = bl >> 3, q = n >> 3, r = n & 7u;
  return x * q + min(x, r) + k;
}

// A load through a pointer the compiler cannot place (read from a table in
// memory) is a flat load, which also counts against the LDS wait counter;
// the couplings and masses are in global memory.
__device__ __forceinline__ double ld_global(const double* p) {
  return *(const __attribute__((address_space(1))) double*)p;
}

// A site of a D-dimensional lattice with its coordinates (D known at
// compile time: the coordinate and neighbour arithmetic stays in registers
// with no per-dimension branch).
template <int D>
struct WalkD {
  uint32_t s;
  uint32_t x[D];
  __device__ __forceinline__ void set(uint32_t s0, const Geom& g) {
    s = s0;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) x[mu] = (s0 / g.stride[mu]) % g.n[mu];
  }
  // s += d (d >= 0) within the plane of the first D - 1 coordinates, with
  // the carries; the last coordinate is left alone (s stays below the plane)
  __device__ __forceinline__ void advance_plane(uint32_t d, const Geom& g) {
    s += d;
    uint32_t carry = d;
#pragma unroll
    for (int mu = 0; mu + 1 < D; ++mu) {
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
  __device__ __forceinline__ uint32_t fwd(int mu, const Geom& g) const {
    return x[mu] == g.n[mu] - 1u ? s - (g.n[mu] - 1u) * g.stride[mu] : s + g.stride[mu];
  }
  __device__ __forceinline__ uint32_t bwd(int mu, const Geom& g) const {
    return x[mu] == 0u ? s + (g.n[mu] - 1u) * g.stride[mu] : s - g.stride[mu];
  }
};

// The march of kb_stencil for the scalar operators on a D-dimensional job.
//
// A site needs 2D + 1 scalars besides its vector entries: the couplings
// w_mu(x) and w_mu(x - e_mu) and the mass m(x).  Read by every lane of the
// site, each would cost the address unit as much as a vector entry while
// carrying 8 bytes for B lanes; here lane k of the site's B lanes reads value
// k (lanes k, k + B, ... when B < 2D + 1) and the site's lanes take them from
// LDS.  The B lanes of a site sit in one wave, so the exchange needs only a
// wave-level barrier.  Along the march a thread also keeps p at its site and
// at its forward t-neighbour, which are the next step's backward neighbour
// and site: a step in the middle of a column loads 2D - 1 vector entries
// instead of 2D + 1.  The arithmetic is stencil_site_gather's, in the same
// order, so w is the same bit for bit.
//
// The march order is MarchOrder's with the slices cut into bands of L (the
// last band shorter): the march runs through band h's columns (each marched
// through the band's Lh slices), then its narrower last column, then band h +
// 1.  With L = item_sites / TS a whole column of a band is one work item's
// worth, so consecutive items march neighbouring columns through the same
// slices; with L = nt it is MarchOrder's order.

template <class Op, int D>
__device__ __forceinline__ void march_scalar(const Geom& g, const BatchProb& P, int logB, int j, int si, bool live,
                                             uint32_t L, uint32_t o0, uint32_t o1,
                                             const typename Op::T* __restrict__ inj, typename Op::T* __restrict__ outj,
                                             double* __restrict__ lds_site, double& dot) {
  using T = typename Op::T;
  constexpr int NV = 2 * D + 1;
  constexpr int NVS = (NV + 1) & ~1;                 // per-site LDS stride: pairs stay 16-byte aligned
  const int B = 1 << logB;
  const size_t V = g.V;
  const double* __restrict__ w = P.coupling;
  const double* __restrict__ mf = P.mass_field;
  double* my = lds_site + si * NVS;
  const uint32_t TS = (uint32_t)(kBlock >> logB);
  const uint32_t nt = g.n[D - 1], Vp = g.stride[D - 1];
  const uint32_t full = Vp & ~(TS - 1u), wl = Vp - full;
  auto ld = [&](uint32_t site) { return inj[((size_t)site << logB) + j]; };
  // position in the march: band of slices [t0, t0 + Lh), slice tb within it;
  // the band's whole columns end at march index Fb
  uint32_t o = o0 + (uint32_t)si, t0 = 0u, Lh = 1u, tb = 0u, Fb = 0u;
  auto site_of = [&](uint32_t oo) -> uint32_t {
    const uint32_t h = oo / (Vp * L);
    t0 = h * L;
    Lh = min(L, nt - t0);
    const uint32_t ob = oo - t0 * Vp;
    Fb = oo - ob + full * Lh;
    if (oo < Fb) {
      const uint32_t c = ob / (TS * Lh), rem = ob - c * TS * Lh;
      tb = rem >> (8 - logB);
      return c * TS + (rem & (TS - 1u)) + Vp * (t0 + tb);
    }
    const uint32_t r = oo - Fb;
    tb = r / wl;
    return full + (r - tb * wl) + Vp * (t0 + tb);
  };
  WalkD<D> wk;
  wk.set(site_of(o), g);
  bool carry = false;
  T xs = zero<T>(), xft = zero<T>();          // p at the site and at its forward t-neighbour, carried
  // scalar k of site s with backward neighbours sb: the load goes out as a
  // global (not flat) load, which the LDS waits do not count
  auto scalar = [&](int k, uint32_t s, const uint32_t (&sb)[D]) -> double {
    if (k < 2 * D) {
      uint32_t sk = s;
      int mk = k;
#pragma unroll
      for (int mu = 0; mu < D; ++mu)
        if (k == D + mu) {
          sk = sb[mu];
          mk = mu;
        }
      return w ? ld_global(w + (size_t)mk * V + sk) : 1.0;
    }
    return mf ? ld_global(mf + s) : P.mass;
  };
  while (o < o1) {
    const uint32_t s = wk.s;
    uint32_t sb[D];
#pragma unroll
    for (int mu = 0; mu < D; ++mu) sb[mu] = wk.bwd(mu, g);
    // the lane's site scalar first, then the vector entries
    double sv = 0.0;
    if (j < NV) sv = scalar(j, s, sb);
    T xf[D], xb[D], xfn = zero<T>();
    if (live) {                                // lanes whose solve has stopped load and store nothing
      if (carry) {                             // values of the previous step, already waited for
        xb[D - 1] = xs;
        xs = xft;
      }
#pragma unroll
      for (int mu = 0; mu + 1 < D; ++mu) {
        xf[mu] = ld(wk.fwd(mu, g));
        xb[mu] = ld(sb[mu]);
      }
      xfn = ld(wk.fwd(D - 1, g));
      if (!carry) {
        xb[D - 1] = ld(sb[D - 1]);
        xs = ld(s);
      }
    }
    if (j < NV) my[j] = sv;
    for (int k = j + B; k < NV; k += B) my[k] = scalar(k, s, sb);   // B < 2D + 1 only
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (live) {
      xf[D - 1] = xfn;
      double diag = my[2 * D];
      T hop = zero<T>();
#pragma unroll
      for (int mu = 0; mu < D; ++mu) {
        const double wf = my[mu], wb = my[D + mu];
        diag += wf + wb;
        hop = axpy(wf, xf[mu], hop);
        hop = axpy(wb, xb[mu], hop);
      }
      const T y = axpy(diag, xs, axpy(-1.0, hop, zero<T>()));
      outj[((size_t)s << logB) + j] = y;
      dot += redot(xs, y);
      xft = xfn;
    }
    // every lane has read the site's values before the next step writes them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    o += TS;
    if (o >= o1) break;
    if (o < Fb) {
      if (tb + 1u < Lh) {                      // next slice of the column: p there was loaded as xf[D - 1]
        ++tb;
        wk.s += Vp;
        wk.x[D - 1] = t0 + tb;
        carry = true;
      } else {                                 // first slice of the band in the next column
        wk.s -= Vp * tb;
        tb = 0u;
        wk.x[D - 1] = t0;
        wk.advance_plane(TS, g);
        carry = false;
      }
    } else {
      wk.set(site_of(o), g);                   // the band's narrower last column, or the next band
      carry = false;
    }
  }
}

// w = A p for the live lanes, partial p^H w per lane (per work item of
// item_sites march indices).
//
// D > 0 (scalar operators, every job of the launch D-dimensional): the march
// of march_scalar.  D = 0: any dimension, every lane loading its site's
// values itself (stencil_site_gather; the covariant operator keeps the plain
// form, which needs about half the registers).  One kernel for all D would
// hold every D's registers: 80-108 VGPRs against 60-84 for D = 3 alone.
template <class Op, int D>
__global__ __launch_bounds__(kBlock) void kb_stencil(BatchArgs a, CgScalars sc, const typename Op::T* __restrict__ in,
                                                     typename Op::T* __restrict__ out, double* __restrict__ partial) {
  using T = typename Op::T;
  constexpr int NC = Op::NC;
  __shared__ double lds[4 * 64];
  const uint32_t item = a.item_base + blockIdx.x;
  const BatchJob& J = a.jobs[a.item_job[item]];
  // the geometry and operator in registers: read through the tables, every
  // field would be reloaded after each store (the tables might alias it)
  const Geom g = J.g;
  const BatchProb P = a.probs[J.prob];
  const int logB = J.logB, B = 1 << logB;
  const int j = threadIdx.x & (B - 1), si = threadIdx.x >> logB;
  const bool live = sc.state[J.lane0 + j] == kActive;
  // live rhs of the job (threads si == 0 hold lanes 0..B-1); none: its partials are not read
  const int nlive = __syncthreads_count(live && si == 0);
  if (nlive == 0) return;
  const Op op = BatchOpOf<Op>::get(P);
  const uint32_t local = (a.march & 2) ? xcd_part(item - J.item0, J.nitems) : item - J.item0;
  const uint32_t o0 = local * (uint32_t)a.item_sites;
  const uint32_t o1 = min(g.V, o0 + (uint32_t)a.item_sites);
  if (a.bytes && threadIdx.x == 0)   // each link, coupling and mass read once, p read and w written per live rhs
    atomicAdd(a.bytes, (unsigned long long)(o1 - o0) * (J.site_bytes + 2ull * (unsigned)NC * (unsigned)nlive * J.esz));
  const T* inj = in + J.off;
  T* outj = out + J.off;
  double dot[1] = {0.0};
  if constexpr (NC == 1 && D > 0) {
    (void)op;
    // [256 / B of the group's narrowest job][stride]: sized at launch, so
    // that blocks of 16 rhs take 1-1.3 KB of LDS, not the 20 KB of B = 1
    extern __shared__ __align__(16) double lds_site[];
    const uint32_t L = (a.march & 1) ? (uint32_t)a.item_sites >> (8 - logB) : g.n[D - 1];
    march_scalar<Op, D>(g, P, logB, j, si, live, L, o0, o1, inj, outj, lds_site, dot[0]);
  } else if (live) {
    const uint32_t TS = (uint32_t)(kBlock >> logB);
    const MarchOrder mo(g, TS);
    const int last = g.ndim - 1;
    uint32_t o = o0 + (uint32_t)si, t;
    SiteWalk w(mo.site(o, t), g);
    auto nbr = [&](int mu, bool fwd) { return w.nbr(mu, fwd, g); };
    while (o < o1) {
      T xs[NC], y[NC];
      if constexpr (NC == 1)
        stencil_site_gather(op, g, logB, w.s, j, P.mass_field, P.mass, P.coupling, inj, nbr, xs, y);
      else
        stencil_site_at(op, g, logB, w.s, j, P.mass_field, P.mass, P.coupling, inj, nbr, xs, y);
      store_vec<T, NC>(outj, g.V, logB, w.s, j, y);
#pragma unroll
      for (int c = 0; c < NC; ++c) dot[0] += redot(xs[c], y[c]);
      o += TS;
      if (o >= o1) break;
      if (o < mo.F) {
        if (t + 1u < mo.nt) {                    // next slice of the column
          ++t;
          w.s += mo.Vp;
        } else {                                 // first slice of the next column
          t = 0u;
          w.s -= mo.Vp * (mo.nt - 1u);
        }
#pragma unroll
        for (int mu = 0; mu < kMaxDim; ++mu)
          if (mu == last) w.x[mu] = t;
        // the plane site moves on by TS when the column changes; it stays
        // below full <= Vp, so no carry reaches the last coordinate
        if (t == 0u) w.advance(TS, g);
      } else {
        w = SiteWalk(mo.site(o, t), g);          // the last, narrower column
      }
    }
  }
  store_partials<1>(dot, B, lds, partial, 0, a.PI, J.lane0, local);
}

// r -= alpha w for the live lanes, partial ||r||^2.
template <class T>
__global__ __launch_bounds__(kBlock) void kb_update_r(BatchArgs a, CgScalars sc, T* __restrict__ r,
                                                      const T* __restrict__ w, double* __restrict__ partial) {
  __shared__ double lds[4 * 64];
  const uint32_t item = a.item_base + blockIdx.x;
  const BatchJob& J = a.jobs[a.item_job[item]];
  const Geom& gp = J.g;
  const uint32_t V = gp.V;
  const int nc = gp.ncomp;
  const int logB = J.logB, B = 1 << logB;
  const int j = threadIdx.x & (B - 1), si = threadIdx.x >> logB;
  const bool live = sc.state[J.lane0 + j] == kActive;
  if (!__syncthreads_or(live)) return;
  const uint32_t s0 = (item - J.item0) * (uint32_t)a.item_sites;
  const uint32_t s1 = min(V, s0 + (uint32_t)a.item_sites);
  double acc[1] = {0.0};
  if (live) {
    const double al = sc.alpha[J.lane0 + j];
    // the item's elements of one component are contiguous: walk them flat,
    // four loads in flight per thread (256 is a multiple of B, so the lane of
    // element threadIdx.x + 256 k is always j)
    const size_t n = (size_t)(s1 - s0) << logB;
    for (int c = 0; c < nc; ++c) {
      T* rj = r + J.off + (((size_t)c * V + s0) << logB);
      const T* wj = w + J.off + (((size_t)c * V + s0) << logB);
      size_t i = threadIdx.x;
      for (; i + 3 * kBlock < n; i += 4 * kBlock) {
        T rr[4], ww[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          rr[u] = rj[i + u * kBlock];
          ww[u] = wj[i + u * kBlock];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          rr[u] = axpy(-al, ww[u], rr[u]);
          rj[i + u * kBlock] = rr[u];
          acc[0] += norm2(rr[u]);
        }
      }
      for (; i < n; i += kBlock) {
        const T ri = axpy(-al, wj[i], rj[i]);
        rj[i] = ri;
        acc[0] += norm2(ri);
      }
    }
  }
  store_partials<1>(acc, B, lds, partial, 0, a.PI, J.lane0, item - J.item0);
}

// x += xalpha p (also for a rhs that converged this iteration); p = r + beta p
// for the lanes still iterating.
template <class T>
__global__ __launch_bounds__(kBlock) void kb_direction(BatchArgs a, CgScalars sc, T* __restrict__ x,
                                                       const T* __restrict__ r, T* __restrict__ p, int parts) {
  const uint32_t item = a.item_base + blockIdx.x / (uint32_t)parts;
  const uint32_t part = blockIdx.x % (uint32_t)parts;
  const BatchJob& J = a.jobs[a.item_job[item]];
  const Geom& gp = J.g;
  const uint32_t V = gp.V;
  const int nc = gp.ncomp;
  const int logB = J.logB, B = 1 << logB;
  const int j = threadIdx.x & (B - 1), si = threadIdx.x >> logB;
  const double xa = sc.xalpha[J.lane0 + j];
  const bool live = sc.state[J.lane0 + j] == kActive;
  if (!__syncthreads_or(live || xa != 0.0)) return;
  if (!live && xa == 0.0) return;
  const double be = sc.beta[J.lane0 + j];
  const uint32_t s0 = (item - J.item0) * (uint32_t)a.item_sites;
  const uint32_t s1 = min(V, s0 + (uint32_t)a.item_sites);
  const size_t ni = (size_t)(s1 - s0) << logB;       // flat, as in kb_update_r
  // this workgroup's part of the item: whole 256-element runs (lane = element mod B)
  const size_t chunk = ((ni + parts - 1) / parts + kBlock - 1) / kBlock * kBlock;
  const size_t e0 = part * chunk, n = min(ni, e0 + chunk);
  for (int c = 0; c < nc; ++c) {
    const size_t base = J.off + (((size_t)c * V + s0) << logB);
    T* xj = x + base;
    const T* rj = r + base;
    T* pj = p + base;
    size_t i = e0 + threadIdx.x;
    for (; i + 3 * kBlock < n; i += 4 * kBlock) {
      // Loads and stores for every lane, the lane's conditions applied as
      // selects (a lane that updates nothing writes back what it read): with
      // the conditions as branches the compiler sank loads into them and each
      // join waited for the loads before it.  The extra bytes are in
      // segments that the block's live lanes fetch and write anyway.
      T pp[4], xx[4], rr[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        pp[u] = pj[i + u * kBlock];
        xx[u] = xj[i + u * kBlock];
        rr[u] = rj[i + u * kBlock];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xj[i + u * kBlock] = xa != 0.0 ? axpy(xa, pp[u], xx[u]) : xx[u];
        pj[i + u * kBlock] = live ? axpy(be, pp[u], rr[u]) : pp[u];
      }
    }
    for (; i < n; i += kBlock) {
      const T pi = pj[i];
      if (xa != 0.0) xj[i] = axpy(xa, pi, xj[i]);
      if (live) pj[i] = axpy(be, pi, rj[i]);
    }
  }
}

// FP64 check of the frozen lanes: rt = b - A x with b regenerated; r = p = rt
// (the restart direction); partial rows ||rt||^2, Re b^H x, Im b^H x.
template <class Op>
__global__ __launch_bounds__(kBlock) void kb_true_residual(BatchArgs a, CgScalars sc,
                                                           const typename Op::T* __restrict__ x,
                                                           typename Op::T* __restrict__ r,
                                                           typename Op::T* __restrict__ p, double* __restrict__ partial,
                                                           size_t rowstride) {
  using T = typename Op::T;
  constexpr int NC = Op::NC;
  __shared__ double lds[3 * 4 * 64];
  __shared__ SiteCode lds_code[kBlock];
  extern __shared__ __align__(16) double lds_sv[];   // scalar operators: [256 / B of the narrowest job][stride]
  const uint32_t item = a.item_base + blockIdx.x;
  const BatchJob& J = a.jobs[a.item_job[item]];
  const int logB = J.logB, B = 1 << logB;
  const int j = threadIdx.x & (B - 1), si = threadIdx.x >> logB;
  const bool live = sc.state[J.lane0 + j] == kFrozen;
  if (!__syncthreads_or(live)) return;
  const Geom g = J.g;                            // in registers (see kb_stencil)
  const BatchProb P = a.probs[J.prob];
  const Op op = BatchOpOf<Op>::get(P);
  const uint32_t s0 = (item - J.item0) * (uint32_t)a.item_sites;
  const uint32_t s1 = min(g.V, s0 + (uint32_t)a.item_sites);
  const uint32_t TS = (uint32_t)(kBlock >> logB);
  const bool hier = g.probe == kProbeHierarchical;
  const LaneCode lc = lane_code<NC>(g, J.rhs0, j, J.nb);
  const T* xj = x + J.off;
  double acc[3] = {0.0, 0.0, 0.0};
  SiteWalk w(s0 + (uint32_t)si, g);
  auto nbr = [&](int mu, bool fwd) { return w.nbr(mu, fwd, g); };
  for (uint32_t base = s0; base < s1; base += TS, w.advance(TS, g)) {
    const bool in = w.s < s1;
    if (hier || NC == 1) {
      __syncthreads();
      if (hier && j == 0 && in) lds_code[si] = site_code(w.s, g);
      if (NC == 1 && in)
        site_scalars_split(g, w.s, j, B, P.mass_field, P.mass, P.coupling, nbr, lds_sv + si * kSiteScalarStride);
      __syncthreads();
    }
    if (!live || !in) continue;
    const uint32_t s = w.s;
    T xs[NC], ax[NC], b[NC], rt[NC];
    if constexpr (NC == 1)
      stencil_site_lds(g, logB, s, j, lds_sv + si * kSiteScalarStride, xj, nbr, xs, ax);
    else
      stencil_site_at(op, g, logB, s, j, P.mass_field, P.mass, P.coupling, xj, nbr, xs, ax);
    if (hier) rhs_coded<T, NC>(lds_code[si], lc, s, g, P.seed, P.mask, b);
    else rhs_at<T, NC>(g, s, J.rhs0, j, J.nb, P.seed, P.mask, b);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      rt[c] = axpy(-1.0, ax[c], b[c]);
      acc[0] += norm2(rt[c]);
      acc[1] += redot(b[c], xs[c]);
      acc[2] += imdot(b[c], xs[c]);
    }
    store_vec<T, NC>(r + J.off, g.V, logB, s, j, rt);
    store_vec<T, NC>(p + J.off, g.V, logB, s, j, rt);
  }
  store_partials<3>(acc, B, lds, partial, rowstride, a.PI, J.lane0, item - J.item0);
}

// Mixed precision: x64 += xh, xh = 0 for the selected lanes (mode 0 flagged
// for a reliable update, mode 1 frozen).  Mode 0 runs after every iteration
// and returns at once while no update is pending.
template <class T64, class T32>
__global__ __launch_bounds__(kBlock) void kb_ru_accumulate(BatchArgs a, CgScalars sc, int mode,
                                                           T64* __restrict__ x, T32* __restrict__ xh) {
  if (mode == 0 && *sc.n_ru == 0) return;
  const uint32_t item = a.item_base + blockIdx.x;
  const BatchJob& J = a.jobs[a.item_job[item]];
  const Geom& gp = J.g;
  const uint32_t V = gp.V;
  const int nc = gp.ncomp;
  const int logB = J.logB, B = 1 << logB;
  const int j = threadIdx.x & (B - 1), si = threadIdx.x >> logB;
  const CgScalars sj = job_scalars(sc, J.lane0);
  if (!ru_selected(sj, mode, j)) return;
  const uint32_t s0 = (item - J.item0) * (uint32_t)a.item_sites;
  const uint32_t s1 = min(V, s0 + (uint32_t)a.item_sites);
  T64* xj = x + J.off;
  T32* hj = xh + J.off;
  for (int c = 0; c < nc; ++c)
    for (uint32_t s = s0 + (uint32_t)si; s < s1; s += (uint32_t)(kBlock >> logB)) {
      const size_t i = (((size_t)c * V + s) << logB) + j;
      xj[i] = axpy(1.0, from_c<T64>(to_c(hj[i])), xj[i]);
      hj[i] = zero<T32>();
    }
}

// Mixed precision: r = b - A x64 with the FP64 operator for the selected lanes,
// rh = single(r), in mode 1 also ph = rh; partial rows ||r||^2, Re/Im b^H x,
// Re/Im x^H r.
template <class Op64, class T32>
__global__ __launch_bounds__(kBlock) void kb_ru_residual(BatchArgs a, CgScalars sc, int mode,
                                                         const typename Op64::T* __restrict__ x,
                                                         T32* __restrict__ rh, T32* __restrict__ ph,
                                                         double* __restrict__ partial, size_t rowstride) {
  using T = typename Op64::T;
  constexpr int NC = Op64::NC;
  if (mode == 0 && *sc.n_ru == 0) return;
  __shared__ double lds[5 * 4 * 64];
  __shared__ SiteCode lds_code[kBlock];
  extern __shared__ __align__(16) double lds_sv[];   // scalar operators: [256 / B of the narrowest job][stride]
  const uint32_t item = a.item_base + blockIdx.x;
  const BatchJob& J = a.jobs[a.item_job[item]];
  const int logB = J.logB, B = 1 << logB;
  const int j = threadIdx.x & (B - 1), si = threadIdx.x >> logB;
  const CgScalars sj = job_scalars(sc, J.lane0);
  const bool live = ru_selected(sj, mode, j);
  if (!__syncthreads_or(live)) return;
  const Geom g = J.g;                            // in registers (see kb_stencil)
  const BatchProb P = a.probs[J.prob];
  const Op64 op = BatchOpOf<Op64>::get(P);
  const uint32_t s0 = (item - J.item0) * (uint32_t)a.item_sites;
  const uint32_t s1 = min(g.V, s0 + (uint32_t)a.item_sites);
  const uint32_t TS = (uint32_t)(kBlock >> logB);
  const bool hier = g.probe == kProbeHierarchical;
  const LaneCode lc = lane_code<NC>(g, J.rhs0, j, J.nb);
  const T* xj = x + J.off;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  SiteWalk w(s0 + (uint32_t)si, g);
  auto nbr = [&](int mu, bool fwd) { return w.nbr(mu, fwd, g); };
  // every thread takes every step (the probe codes and the scalar operators'
  // site scalars are shared through LDS)
  for (uint32_t base = s0; base < s1; base += TS, w.advance(TS, g)) {
    const bool in = w.s < s1;
    if (hier || NC == 1) {
      __syncthreads();
      if (hier && j == 0 && in) lds_code[si] = site_code(w.s, g);
      if (NC == 1 && in)
        site_scalars_split(g, w.s, j, B, P.mass_field, P.mass, P.coupling, nbr, lds_sv + si * kSiteScalarStride);
      __syncthreads();
    }
    if (!live || !in) continue;
    const uint32_t s = w.s;
    T xs[NC], ax[NC], b[NC];
    T32 r32[NC];
    if constexpr (NC == 1)
      stencil_site_lds(g, logB, s, j, lds_sv + si * kSiteScalarStride, xj, nbr, xs, ax);
    else
      stencil_site_at(op, g, logB, s, j, P.mass_field, P.mass, P.coupling, xj, nbr, xs, ax);
    if (hier) rhs_coded<T, NC>(lds_code[si], lc, s, g, P.seed, P.mask, b);
    else rhs_at<T, NC>(g, s, J.rhs0, j, J.nb, P.seed, P.mask, b);
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
    store_vec<T32, NC>(rh + J.off, g.V, logB, s, j, r32);
    if (mode == 1) store_vec<T32, NC>(ph + J.off, g.V, logB, s, j, r32);
  }
  store_partials<5>(acc, B, lds, partial, rowstride, a.PI, J.lane0, item - J.item0);
}

// ---- per-lane scalar steps -------------------------------------------------

__global__ void kb_scalars_init(BatchArgs a, CgScalars sc, int nlanes) {
  const int L = blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= nlanes) return;
  const BatchJob& J = a.jobs[a.lane_job[L]];
  const int j = L - J.lane0;
  const bool valid = j < J.nb;
  const double bnorm2 = (double)J.g.V;   // unit-modulus entries on one component per site
  sc.state[L] = valid ? kActive : kPadding;
  sc.bnorm2[L] = valid ? bnorm2 : 0.0;
  sc.rho[L] = valid ? bnorm2 : 0.0;
  sc.alpha[L] = 0.0;
  sc.xalpha[L] = 0.0;
  sc.beta[L] = 0.0;
  sc.rho_ref[L] = valid ? bnorm2 : 0.0;
  sc.pp[L] = valid ? bnorm2 : 0.0;
  sc.anorm[L] = 0.0;
  sc.xhn[L] = 0.0;
  sc.dev[L] = 0.0;
  sc.ru[L] = 0;
  sc.iters[L] = 0;
  sc.restarts[L] = 0;
  sc.relres2[L] = 0.0;
  sc.q[2 * L] = 0.0;
  sc.q[2 * L + 1] = 0.0;
}

// One wave per lane: four lanes per 256-thread workgroup.  Each wave sums its
// lane's partials in a fixed order (four running sums per thread, then a
// shuffle tree), so the result is reproducible; the lane's scalar step runs
// on the wave's first thread.
constexpr int kLanesPerBlock = kBlock / 64;

__device__ __forceinline__ double wave_sum(const double* __restrict__ part, int n) {
  const int t = threadIdx.x & 63;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int i = t;
  for (; i + 192 < n; i += 256) {
    a0 += part[i];
    a1 += part[i + 64];
    a2 += part[i + 128];
    a3 += part[i + 192];
  }
  for (; i < n; i += 64) a0 += part[i];
  double v = (a0 + a1) + (a2 + a3);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__global__ __launch_bounds__(kBlock) void kb_reduce_alpha(BatchArgs a, CgScalars sc, int lane_base, int nlanes,
                                                          const double* __restrict__ partial, int soft) {
  const int l = blockIdx.x * kLanesPerBlock + (int)(threadIdx.x >> 6);
  if (l >= nlanes) return;
  const int L = lane_base + l;
  if (*sc.active == 0 || sc.state[L] != kActive) return;     // uniform per wave
  const BatchJob& J = a.jobs[a.lane_job[L]];
  const double pAp = wave_sum(partial + (size_t)L * a.PI, (int)J.nitems);
  if ((threadIdx.x & 63) != 0) return;
  lane_alpha(sc, L, pAp, soft, false);
}

__global__ __launch_bounds__(kBlock) void kb_reduce_beta(BatchArgs a, CgScalars sc, int lane_base, int nlanes,
                                                         const double* __restrict__ partial, double eps, double tau2) {
  const int l = blockIdx.x * kLanesPerBlock + (int)(threadIdx.x >> 6);
  if (l >= nlanes) return;
  const int L = lane_base + l;
  if (sc.state[L] != kActive) {                // uniform per wave
    if ((threadIdx.x & 63) == 0) sc.xalpha[L] = 0.0;
    return;
  }
  const BatchJob& J = a.jobs[a.lane_job[L]];
  const BatchProb& P = a.probs[J.prob];
  const BetaIn in = lane_beta_read(sc, L);
  const double rho_new = wave_sum(partial + (size_t)L * a.PI, (int)J.nitems);
  if ((threadIdx.x & 63) != 0) return;
  lane_beta(sc, L, in, rho_new, P.tol2, P.max_iter, 0.0, P.tol2, eps, tau2);
}

__global__ __launch_bounds__(kBlock) void kb_reduce_true(BatchArgs a, CgScalars sc, int lane_base, int nlanes,
                                                         const double* __restrict__ partial, size_t rowstride) {
  const int l = blockIdx.x * kLanesPerBlock + (int)(threadIdx.x >> 6);
  if (l >= nlanes) return;
  const int L = lane_base + l;
  if ((threadIdx.x & 63) == 0) sc.xalpha[L] = 0.0;
  if (sc.state[L] != kFrozen) return;
  const BatchJob& J = a.jobs[a.lane_job[L]];
  const BatchProb& P = a.probs[J.prob];
  const double* row = partial + (size_t)L * a.PI;
  const double rt2 = wave_sum(row, (int)J.nitems);
  const double qre = wave_sum(row + rowstride, (int)J.nitems);
  const double qim = wave_sum(row + 2 * rowstride, (int)J.nitems);
  if ((threadIdx.x & 63) != 0) return;
  lane_true(sc, L, rt2, qre, qim, P.tol2, P.max_iter, kBatchMaxRestarts);
}

__global__ __launch_bounds__(kBlock) void kb_reduce_ru(BatchArgs a, CgScalars sc, int lane_base, int nlanes,
                                                       const double* __restrict__ partial, size_t rowstride, int mode) {
  const int l = blockIdx.x * kLanesPerBlock + (int)(threadIdx.x >> 6);
  if (l >= nlanes) return;
  const int L = lane_base + l;
  if (mode == 0 && *sc.n_ru == 0) return;
  if (!ru_selected(sc, mode, L)) return;      // uniform per wave
  const BatchJob& J = a.jobs[a.lane_job[L]];
  const BatchProb& P = a.probs[J.prob];
  double v[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) v[k] = wave_sum(partial + k * rowstride + (size_t)L * a.PI, (int)J.nitems);
  if ((threadIdx.x & 63) != 0) return;
  lane_ru(sc, L, v, mode, P.tol2, P.max_iter, kBatchMaxRestarts);
}

// ---- launchers -------------------------------------------------------------

namespace {

// Operator policy for a group: (kind, element type, precision).
template <class F>
hipError_t batch_dispatch(int kind, Elem elem, Prec prec, F&& f) {
  if (kind == 1) {
    if (prec == Prec::kF32) f(CovOp<float2>{nullptr});
    else f(CovOp<double2>{nullptr});
  } else if (elem == Elem::kReal) {
    if (prec == Prec::kF32) f(ScalarOp<float>{});
    else f(ScalarOp<double>{});
  } else {
    if (prec == Prec::kF32) f(ScalarOp<float2>{});
    else f(ScalarOp<double2>{});
  }
  return hipGetLastError();
}

template <class T> struct Wide;
template <> struct Wide<float> { using type = double; };
template <> struct Wide<double> { using type = double; };
template <> struct Wide<float2> { using type = double2; };
template <> struct Wide<double2> { using type = double2; };

template <class T> struct is_single
    : std::integral_constant<bool, std::is_same<T, float>::value || std::is_same<T, float2>::value> {};

template <class Op> struct FP64Op;
template <class TT> struct FP64Op<ScalarOp<TT>> { using type = ScalarOp<typename Wide<TT>::type>; };
template <class C> struct FP64Op<CovOp<C>> { using type = CovOp<typename Wide<C>::type>; };

unsigned lane_grid(const BatchGroup& gr) { return (unsigned)((gr.nlanes + kLanesPerBlock - 1) / kLanesPerBlock); }

}  // namespace

hipError_t launch_batch_init(const BatchArgs& a, const BatchGroup& gr, void* x64, void* xh, void* r, void* p,
                             hipStream_t st) {
  return batch_dispatch(gr.kind, gr.elem, gr.prec, [&](auto op) {
    using Op = decltype(op);
    using TW = typename Op::T;
    using T64 = typename Wide<TW>::type;
    kb_init<T64, TW, Op::NC><<<gr.nitems, kBlock, 0, st>>>(a, (T64*)x64, (TW*)xh, (TW*)r, (TW*)p);
  });
}

// Workgroups per work item in the direction pass: 8 for FP64 vectors (an
// item of 16 rhs is then 4-8 KB per vector and workgroup, and the workgroups
// that run together stream through neighbouring memory), one for FP32.
// Measured on the 64 uneven tori (FP64 quadratures/s): 19 020-19 120 with
// one, 19 210-19 230 with 2, 19 300-19 330 with 4, 19 500-19 530 with 8; in
// mixed precision 2 and 4 changed nothing and 8 lost 6%.
template <class T>
static int direction_parts() {
  if (const char* e = std::getenv("TIP_BATCH_VQ")) return std::max(1, std::min(16, std::atoi(e)));   // experiments
  return is_single<T>::value ? 1 : 8;
}

hipError_t launch_batch_iteration(const BatchArgs& a, const BatchGroup& gr, const CgScalars& sc, void* x, void* r,
                                  void* p, void* w, double* partial, size_t rowstride, double eps, double tau2,
                                  hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  return batch_dispatch(gr.kind, gr.elem, gr.prec, [&](auto op) {
    using Op = decltype(op);
    using T = typename Op::T;
    if (ev0) (void)hipEventRecord(ev0, st);
    auto stencil = [&](auto dim) {
      constexpr int D = decltype(dim)::value;
      if constexpr (D > 0) {
        constexpr int NVS = (2 * D + 2) & ~1;
        const size_t lds = (size_t)(kBlock >> gr.min_logB) * NVS * sizeof(double);
        kb_stencil<Op, D><<<gr.nitems, kBlock, lds, st>>>(a, sc, (const T*)p, (T*)w, partial);
      } else {
        kb_stencil<Op, 0><<<gr.nitems, kBlock, 0, st>>>(a, sc, (const T*)p, (T*)w, partial);
      }
    };
    if constexpr (Op::NC == 1) {
      switch (gr.ndim) {
        case 1: stencil(std::integral_constant<int, 1>{}); break;
        case 2: stencil(std::integral_constant<int, 2>{}); break;
        case 3: stencil(std::integral_constant<int, 3>{}); break;
        case 4: stencil(std::integral_constant<int, 4>{}); break;
        default: stencil(std::integral_constant<int, 0>{}); break;
      }
    } else {
      stencil(std::integral_constant<int, 0>{});
    }
    if (ev1) (void)hipEventRecord(ev1, st);
    kb_reduce_alpha<<<lane_grid(gr), kBlock, 0, st>>>(a, sc, gr.lane_base, gr.nlanes, partial,
                                                         gr.prec == Prec::kF32 ? 1 : 0);
    kb_update_r<T><<<gr.nitems, kBlock, 0, st>>>(a, sc, (T*)r, (const T*)w, partial + rowstride);
    kb_reduce_beta<<<lane_grid(gr), kBlock, 0, st>>>(a, sc, gr.lane_base, gr.nlanes, partial + rowstride, eps,
                                                        tau2);
    const int vp = direction_parts<T>();
    kb_direction<T><<<gr.nitems * (uint32_t)vp, kBlock, 0, st>>>(a, sc, (T*)x, (const T*)r, (T*)p, vp);
  });
}

hipError_t launch_batch_reliable(const BatchArgs& a, const BatchGroup& gr, const CgScalars& sc, int mode, void* x64,
                                 void* xh, void* r, void* p, double* partial, size_t rowstride, hipStream_t st) {
  return batch_dispatch(gr.kind, gr.elem, Prec::kF32, [&](auto op) {
    using Op = decltype(op);
    using T32 = typename Op::T;
    if constexpr (is_single<T32>::value) {
      using Op64 = typename FP64Op<Op>::type;
      using T64 = typename Op64::T;
      kb_ru_accumulate<T64, T32><<<gr.nitems, kBlock, 0, st>>>(a, sc, mode, (T64*)x64, (T32*)xh);
      const size_t lds = Op64::NC == 1 ? (size_t)(kBlock >> gr.min_logB) * kSiteScalarStride * sizeof(double) : 0;
      kb_ru_residual<Op64, T32><<<gr.nitems, kBlock, lds, st>>>(a, sc, mode, (const T64*)x64, (T32*)r, (T32*)p,
                                                                partial, rowstride);
      kb_reduce_ru<<<lane_grid(gr), kBlock, 0, st>>>(a, sc, gr.lane_base, gr.nlanes, partial, rowstride, mode);
    }
  });
}

hipError_t launch_batch_true_residual(const BatchArgs& a, const BatchGroup& gr, const CgScalars& sc, void* x,
                                      void* r, void* p, double* partial, size_t rowstride, hipStream_t st) {
  return batch_dispatch(gr.kind, gr.elem, Prec::kF64, [&](auto op) {
    using Op = decltype(op);
    using T = typename Op::T;
    if constexpr (!is_single<T>::value) {
      const size_t lds = Op::NC == 1 ? (size_t)(kBlock >> gr.min_logB) * kSiteScalarStride * sizeof(double) : 0;
      kb_true_residual<Op><<<gr.nitems, kBlock, lds, st>>>(a, sc, (const T*)x, (T*)r, (T*)p, partial, rowstride);
      kb_reduce_true<<<lane_grid(gr), kBlock, 0, st>>>(a, sc, gr.lane_base, gr.nlanes, partial, rowstride);
    }
  });
}

hipError_t launch_batch_scalars_init(const BatchArgs& a, const CgScalars& sc, int nlanes, hipStream_t st) {
  kb_scalars_init<<<(nlanes + 255) / 256, 256, 0, st>>>(a, sc, nlanes);
  return hipGetLastError();
}

}  // namespace tip
