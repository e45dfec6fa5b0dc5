// Device-side building blocks shared by the HIP kernels of libtip.
//
// Lattice geometry, the hierarchical permutation of Sec. 3 (Alg. 5 with the
// Red-Black order in the closed form of Lemma 3.3), the probing-vector entry
// of eq. row-col-permutation, the bias mask of Sec. 4 and small complex
// helpers.  Everything here is computed per site from its index; nothing is
// tabulated in memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tip {

constexpr int kMaxDim = 4;
constexpr int kBlock = 256;        // threads per workgroup (4 wave64)
constexpr int kMaxLevels = 31;

// Per-call lattice description, passed by value to every kernel.
struct Geom {
  int32_t ndim;
  int32_t ncomp;
  uint32_t V;
  int32_t L;                 // sum_j k_j = log2 V (power-of-two sides)
  int32_t nlevels;           // max_j k_j (power-of-two sides)
  int32_t logn[kMaxDim];     // k_j (power-of-two sides)
  int32_t shift[kMaxDim];    // log2 of the site-index stride of dimension j (power-of-two sides)
  // any sides
  int32_t pow2;              // every side a power of two: logn / shift above are valid
  uint32_t n[kMaxDim];       // sides
  uint32_t stride[kMaxDim];  // site-index stride of dimension j
  // levels of the probing colouring (Sec. 3; Sec. 3.4 for odd factors)
  int32_t k2[kMaxDim];       // 2-adic valuation of n_j
  int32_t B;                 // binary levels (= nlevels for power-of-two sides)
  int32_t LB;                // bits of the binary colour (= L for power-of-two sides)
  int32_t has3;              // a three-colouring level follows the binary ones
  uint32_t sub[kMaxDim];     // sides n_j >> B of the sub-torus it colours
  uint32_t gamma;            // colours of one sweep: 2^LB, times 3 with that level
  int32_t probe;             // probe kind of the call (ProbeKind)
  int32_t stop;              // stopped hierarchy: bit-levels of the colouring kept
  // probe classes: with cls_gamma > 0 a call solves only the probes whose
  // F_3 digit is cls_j3, numbered i = 0, 1, ...: probe(i) = (i / cls_nbc)
  // cls_gamma + cls_j3 cls_nbc + i mod cls_nbc, with cls_nbc = 2^LB
  int32_t cls_gamma, cls_nbc, cls_j3;
};

// The probe index of class-local probe i (identity without classes).
__host__ __device__ inline uint64_t class_probe(uint64_t i, const Geom& g) {
  if (g.cls_gamma == 0) return i;
  const uint64_t nbc = (uint64_t)g.cls_nbc;
  return (i / nbc) * (uint64_t)g.cls_gamma + (uint64_t)g.cls_j3 * nbc + i % nbc;
}

constexpr int kLdsPerCu = 160 * 1024;   // gfx950 LDS per CU
constexpr int kNumXcd = 8;   // MI355X: 8 XCDs, each with its own L2

// Coordinate and periodic neighbours of a site.  The _p2 forms use shifts
// and serve the kernels that only run on power-of-two sides; the plain forms
// take any sides.
__device__ __forceinline__ uint32_t coord_p2(uint32_t s, const Geom& g, int mu) {
  return (s >> g.shift[mu]) & ((1u << g.logn[mu]) - 1u);
}
__device__ __forceinline__ uint32_t nbr_fwd_p2(uint32_t s, const Geom& g, int mu) {
  const uint32_t n = 1u << g.logn[mu];
  const uint32_t stride = 1u << g.shift[mu];
  return coord_p2(s, g, mu) == n - 1u ? s - (n - 1u) * stride : s + stride;
}
__device__ __forceinline__ uint32_t nbr_bwd_p2(uint32_t s, const Geom& g, int mu) {
  const uint32_t n = 1u << g.logn[mu];
  const uint32_t stride = 1u << g.shift[mu];
  return coord_p2(s, g, mu) == 0u ? s + (n - 1u) * stride : s - stride;
}
__device__ __forceinline__ uint32_t coord(uint32_t s, const Geom& g, int mu) {
  if (g.pow2) return coord_p2(s, g, mu);
  return (s / g.stride[mu]) % g.n[mu];
}
__device__ __forceinline__ uint32_t nbr_fwd(uint32_t s, const Geom& g, int mu) {
  return coord(s, g, mu) == g.n[mu] - 1u ? s - (g.n[mu] - 1u) * g.stride[mu] : s + g.stride[mu];
}
__device__ __forceinline__ uint32_t nbr_bwd(uint32_t s, const Geom& g, int mu) {
  return coord(s, g, mu) == 0u ? s + (g.n[mu] - 1u) * g.stride[mu] : s - g.stride[mu];
}

// Location of site s in the hierarchical permutation (Sec. 3.3, Alg. 5).
// Level m (0-based here) gathers bit m of every dimension that still has one,
// first dimension most significant, and appends its Red-Black position
// RB_a(i) = floor(i/2) + parity(i) 2^{a-1} (Lemma 3.3 with c_a(i) = parity of
// the one-bits of i, which is what c_j = [c_{j-1}, not c_{j-1}] unrolls to).
// The Theorem of Sec. 3.3 makes the a-dimensional table the one to use when
// only a dimensions are active, so no d-dimensional table is needed.
// With odd factors in the sides only the B binary levels are taken (dimension
// j active at level m while m < k_j, its 2-adic valuation); the result is
// then the binary colour of the site, in [0, 2^LB).
__device__ __forceinline__ uint32_t hier_perm(uint32_t s, const Geom& g) {
  uint32_t x[kMaxDim];
#pragma unroll
  for (int mu = 0; mu < kMaxDim; ++mu) x[mu] = mu < g.ndim ? coord(s, g, mu) : 0u;
  uint32_t loc = 0;
  for (int m = 0; m < g.B; ++m) {
    uint32_t idx = 0;
    int a = 0;
#pragma unroll
    for (int mu = 0; mu < kMaxDim; ++mu) {
      if (mu < g.ndim && m < g.k2[mu]) {
        idx = (idx << 1) | ((x[mu] >> m) & 1u);
        ++a;
      }
    }
    const uint32_t rb = (idx >> 1) | ((uint32_t)(__popc(idx) & 1) << (a - 1));
    loc = (loc << a) | rb;
  }
  return loc;
}

// Column of the Hadamard matrix used by probe m: eq. HpermSequence is the
// L-bit reversal of m.
__device__ __forceinline__ uint32_t hadamard_column(uint32_t m, int L) {
  return L == 0 ? 0u : (__brev(m) >> (32 - L));
}

// H(P, col) = (-1)^{popcount(P & col)} (eq. HadamardElements), as +1 / -1.
__device__ __forceinline__ double hadamard_sign(uint32_t P, uint32_t col) {
  return (__popc(P & col) & 1) ? -1.0 : 1.0;
}

// Output n of SplitMix64(seed) (Steele, Lea & Flood 2014): the generator's
// state after n+1 steps is seed + (n+1) * gamma; the output mixes that state.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t n) {
  uint64_t z = seed + (n + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

enum MaskKind { kMaskNone = 0, kMaskZ2 = 1, kMaskZ4 = 2 };

// Three-colouring of Sec. 3.4 on the sub-torus y_j = x_j >> B (sides sub_j):
// C = (sum_j y_j + sum_j delta_j) mod 3, delta_j = 1 iff y_j = sub_j - 1 and
// (sub_j - 1) mod 3 = 0; sides of 1 take no part.
__device__ __forceinline__ uint32_t three_colour(uint32_t s, const Geom& g) {
  uint32_t total = 0;
#pragma unroll
  for (int mu = 0; mu < kMaxDim; ++mu) {
    if (mu >= g.ndim || g.sub[mu] <= 1u) continue;
    const uint32_t y = coord(s, g, mu) >> g.B;
    total += y + ((y == g.sub[mu] - 1u && (g.sub[mu] - 1u) % 3u == 0u) ? 1u : 0u);
  }
  return total % 3u;
}

// Column of probe m: sweep r = m / gamma, within it column j = m mod gamma
// with binary part j mod 2^LB (Hadamard column through eq. HpermSequence)
// and F_3 part j3 = j >> LB (eq. Hperm-general-recursive, newest level's
// column most significant).
struct ProbeCol {
  uint32_t col;   // Hadamard column
  uint32_t j3;    // F_3 column, 0 without the three-colouring level
  uint32_t r;     // mask sweep
};
__device__ __forceinline__ ProbeCol probe_column(uint64_t m, const Geom& g) {
  ProbeCol pc;
  pc.r = (uint32_t)(m / g.gamma);
  const uint64_t j = m % g.gamma;
  pc.j3 = (uint32_t)(j >> g.LB);
  pc.col = hadamard_column((uint32_t)(j & ((1ull << g.LB) - 1ull)), g.LB);
  return pc;
}

// Probe kinds (the comparison probes of Sec. 5 run through the same path):
// hierarchical (above); natural-order Hadamard, z_m(x) = H(s(x), m) on the
// natural site numbering; random, z_m = the mask of sweep m alone; the
// hierarchy stopped after g.stop levels; Fourier-grouped columns.  The last
// two take power-of-two sides.
enum ProbeKind { kProbeHierarchical = 0, kProbeNatural = 1, kProbeRandom = 2, kProbeStopped = 3, kProbeFourier = 4 };

// Red-Black index of Alg. 5 level m (0-based) of a site with coordinates x
// on power-of-two sides, and the number a of dimensions active at it.
__device__ __forceinline__ uint32_t level_rb(const uint32_t (&x)[kMaxDim], const Geom& g, int m, int& a) {
  uint32_t idx = 0;
  a = 0;
#pragma unroll
  for (int mu = 0; mu < kMaxDim; ++mu) {
    if (mu < g.ndim && m < g.logn[mu]) {
      idx = (idx << 1) | ((x[mu] >> m) & 1u);
      ++a;
    }
  }
  return (idx >> 1) | ((uint32_t)(__popc(idx) & 1) << (a - 1));
}

// Stopped hierarchy (Sec. 5.1): the recursion of Sec. 3 run for g.stop
// levels leaves the members of each colour class in natural order.  On
// power-of-two sides a class after k levels fixes the low k bits of every
// coordinate and its members differ in y_j = x_j >> min(k, k_j), so the
// location is the Alg. 5 string of levels 0..k-1 (t bits) followed by the
// natural index of y on the sub-torus of sides n_j >> min(k, k_j).
__device__ __forceinline__ uint32_t stopped_perm(uint32_t s, const Geom& g) {
  uint32_t x[kMaxDim];
#pragma unroll
  for (int mu = 0; mu < kMaxDim; ++mu) x[mu] = mu < g.ndim ? coord_p2(s, g, mu) : 0u;
  const int kmax = g.stop < g.nlevels ? g.stop : g.nlevels;
  uint32_t loc = 0;
  int t = 0;
  for (int m = 0; m < kmax; ++m) {
    int a;
    const uint32_t rb = level_rb(x, g, m, a);
    loc = (loc << a) | rb;
    t += a;
  }
  uint32_t nat = 0;
  int sh = 0;
#pragma unroll
  for (int mu = 0; mu < kMaxDim; ++mu) {
    if (mu >= g.ndim) break;
    const int cut = kmax < g.logn[mu] ? kmax : g.logn[mu];
    nat |= (x[mu] >> cut) << sh;
    sh += g.logn[mu] - cut;
  }
  return t == 0 ? nat : ((loc << (g.L - t)) | nat);
}

// w16^e = exp(2 pi i e / 16) from the doubles nearest cos(pi/8), sin(pi/8)
// and sqrt(2)/2, rotated by i^(e >> 2).
__device__ __forceinline__ double2 omega16(uint32_t e) {
  const double c = 0.9238795325112867, sn = 0.3826834323650898, h = 0.7071067811865476;
  double2 v;
  switch (e & 3u) {
    case 0: v = make_double2(1.0, 0.0); break;
    case 1: v = make_double2(c, sn); break;
    case 2: v = make_double2(h, h); break;
    default: v = make_double2(sn, c); break;
  }
  for (uint32_t q = (e >> 2) & 3u; q > 0; --q) v = make_double2(-v.y, v.x);
  return v;
}

// Fourier-grouped columns: eq. Hperm-general-recursive with the a bits of one
// Alg. 5 level taken as one level of c = 2^a colours, so probe
// m = sum_l j_l prod_{l' < l} c_{l'} is prod_l F_c(s_l(x), j_l) with s_l the
// level's Red-Black index and F_n(i, j) = exp(2 pi i i j / n) (eq.
// FourierElements).  With c <= 16 the entry is w16^e,
// e = sum_l (s_l j_l mod c_l) 16 / c_l.
__device__ __forceinline__ uint32_t fourier_exponent(uint32_t s, uint64_t m, const Geom& g) {
  uint32_t x[kMaxDim];
#pragma unroll
  for (int mu = 0; mu < kMaxDim; ++mu) x[mu] = mu < g.ndim ? coord_p2(s, g, mu) : 0u;
  uint32_t e = 0;
  uint64_t rest = m;
  for (int l = 0; l < g.nlevels; ++l) {
    int a;
    const uint32_t sl = level_rb(x, g, l, a);
    const uint32_t c = 1u << a;
    const uint32_t j = (uint32_t)(rest & (c - 1u));
    rest >>= a;
    e += ((sl * j) & (c - 1u)) << (4 - a);
  }
  return e & 15u;
}

// Entry (s, comp) of the probing right-hand side b_{m,comp} = z0_r .* z_m:
// (re, im), each exactly 0 or +-1 except the F_3 factor w^k, whose parts are
// -1/2 and +-(the double nearest sqrt(3)/2).  z0_r takes outputs
// (r V + s) ncomp + comp of SplitMix64(seed).
// c3 is the site's colour of the three-colouring level (three_colour), read
// only when pc.j3 != 0.
__device__ __forceinline__ double2 probe_value_c3(uint32_t s, uint32_t P, uint32_t c3, ProbeCol pc, int comp,
                                                  const Geom& g, uint64_t seed, int mask) {
  const double h = hadamard_sign(P, pc.col);
  double2 v = make_double2(h, 0.0);
  if (mask != kMaskNone) {
    const uint64_t n = ((uint64_t)pc.r * (uint64_t)g.V + (uint64_t)s) * (uint64_t)g.ncomp + (uint64_t)comp;
    const uint64_t u = splitmix64_at(seed, n);
    if (mask == kMaskZ2) {
      v = make_double2((u >> 63) ? -h : h, 0.0);
    } else {
      switch ((int)(u >> 62)) {            // i^t
        case 0: v = make_double2(h, 0.0); break;
        case 1: v = make_double2(0.0, h); break;
        case 2: v = make_double2(-h, 0.0); break;
        default: v = make_double2(0.0, -h); break;
      }
    }
  }
  if (pc.j3 != 0u) {
    const uint32_t k = (c3 * pc.j3) % 3u;
    if (k != 0u) {
      const double wr = -0.5, wi = k == 1u ? 0.8660254037844386 : -0.8660254037844386;
      v = make_double2(v.x * wr - v.y * wi, v.x * wi + v.y * wr);
    }
  }
  return v;
}

__device__ __forceinline__ double2 probe_value(uint32_t s, uint32_t P, ProbeCol pc, int comp, const Geom& g,
                                               uint64_t seed, int mask) {
  return probe_value_c3(s, P, pc.j3 != 0u ? three_colour(s, g) : 0u, pc, comp, g, seed, mask);
}

// Entry (s, comp) of right-hand side m for the call's probe kind.
__device__ __forceinline__ double2 probe_entry(uint32_t s, uint64_t m, int comp, const Geom& g, uint64_t seed,
                                               int mask) {
  ProbeCol pc;
  if (g.probe == kProbeNatural) {
    pc.col = (uint32_t)m;
    pc.j3 = 0u;
    pc.r = 0u;
    return probe_value(s, s, pc, comp, g, seed, mask);
  }
  if (g.probe == kProbeRandom) {
    pc.col = 0u;
    pc.j3 = 0u;
    pc.r = (uint32_t)m;
    return probe_value(s, 0u, pc, comp, g, seed, mask);
  }
  if (g.probe == kProbeStopped) {
    pc.col = hadamard_column((uint32_t)m, g.L);
    pc.j3 = 0u;
    pc.r = 0u;
    return probe_value(s, stopped_perm(s, g), pc, comp, g, seed, mask);
  }
  if (g.probe == kProbeFourier) {
    pc.col = 0u;
    pc.j3 = 0u;
    pc.r = 0u;
    const double2 z0 = probe_value(s, 0u, pc, comp, g, seed, mask);   // the mask entry
    const double2 w = omega16(fourier_exponent(s, m, g));
    return make_double2(z0.x * w.x - z0.y * w.y, z0.x * w.y + z0.y * w.x);
  }
  return probe_value(s, hier_perm(s, g), probe_column(m, g), comp, g, seed, mask);
}


// ---- complex helpers (double2 = re, im) ----------------------------------
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double a, double2 b) { return make_double2(a * b.x, a * b.y); }
// acc + u * v
__device__ __forceinline__ double2 cfma(double2 u, double2 v, double2 acc) {
  acc.x = fma(u.x, v.x, acc.x);
  acc.x = fma(-u.y, v.y, acc.x);
  acc.y = fma(u.x, v.y, acc.y);
  acc.y = fma(u.y, v.x, acc.y);
  return acc;
}
// acc + conj(u) * v
__device__ __forceinline__ double2 cfma_conj(double2 u, double2 v, double2 acc) {
  acc.x = fma(u.x, v.x, acc.x);
  acc.x = fma(u.y, v.y, acc.x);
  acc.y = fma(u.x, v.y, acc.y);
  acc.y = fma(-u.y, v.x, acc.y);
  return acc;
}

// FP32 complex helpers (single-precision storage and arithmetic).
__device__ __forceinline__ float2 cfma(float2 u, float2 v, float2 acc) {
  acc.x = fmaf(u.x, v.x, acc.x);
  acc.x = fmaf(-u.y, v.y, acc.x);
  acc.y = fmaf(u.x, v.y, acc.y);
  acc.y = fmaf(u.y, v.x, acc.y);
  return acc;
}
__device__ __forceinline__ float2 cfma_conj(float2 u, float2 v, float2 acc) {
  acc.x = fmaf(u.x, v.x, acc.x);
  acc.x = fmaf(u.y, v.y, acc.x);
  acc.y = fmaf(u.x, v.y, acc.y);
  acc.y = fmaf(-u.y, v.x, acc.y);
  return acc;
}

// Generic element helpers for real (double, float) and complex (double2,
// float2) vectors.  Scalars are passed in double and applied in the vector's
// own precision; dot products and norms are always returned in double.
__device__ __forceinline__ double axpy(double a, double x, double y) { return fma(a, x, y); }
__device__ __forceinline__ double2 axpy(double a, double2 x, double2 y) {
  return make_double2(fma(a, x.x, y.x), fma(a, x.y, y.y));
}
__device__ __forceinline__ double norm2(double a) { return a * a; }
__device__ __forceinline__ double norm2(double2 a) { return fma(a.x, a.x, a.y * a.y); }
// Re(conj(a) b)
__device__ __forceinline__ double redot(double a, double b) { return a * b; }
__device__ __forceinline__ double redot(double2 a, double2 b) { return fma(a.x, b.x, a.y * b.y); }
// Im(conj(a) b)
__device__ __forceinline__ double imdot(double, double) { return 0.0; }
__device__ __forceinline__ double imdot(double2 a, double2 b) { return fma(a.x, b.y, -a.y * b.x); }
__device__ __forceinline__ float axpy(double a, float x, float y) { return fmaf((float)a, x, y); }
__device__ __forceinline__ float2 axpy(double a, float2 x, float2 y) {
  const float af = (float)a;
  return make_float2(fmaf(af, x.x, y.x), fmaf(af, x.y, y.y));
}
__device__ __forceinline__ double norm2(float a) { return (double)a * (double)a; }
__device__ __forceinline__ double norm2(float2 a) { return fma((double)a.x, (double)a.x, (double)a.y * (double)a.y); }
__device__ __forceinline__ double redot(float a, float b) { return (double)a * (double)b; }
__device__ __forceinline__ double redot(float2 a, float2 b) {
  return fma((double)a.x, (double)b.x, (double)a.y * (double)b.y);
}
__device__ __forceinline__ double imdot(float, float) { return 0.0; }
__device__ __forceinline__ double imdot(float2 a, float2 b) {
  return fma((double)a.x, (double)b.y, -(double)a.y * (double)b.x);
}
template <class T> __device__ __forceinline__ T zero();
template <> __device__ __forceinline__ double zero<double>() { return 0.0; }
template <> __device__ __forceinline__ double2 zero<double2>() { return make_double2(0.0, 0.0); }
template <> __device__ __forceinline__ float zero<float>() { return 0.0f; }
template <> __device__ __forceinline__ float2 zero<float2>() { return make_float2(0.0f, 0.0f); }
// exact values (probes) or FP64 vectors converted to the vector type
template <class T> __device__ __forceinline__ T from_c(double2 v);
template <> __device__ __forceinline__ double from_c<double>(double2 v) { return v.x; }
template <> __device__ __forceinline__ double2 from_c<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float from_c<float>(double2 v) { return (float)v.x; }
template <> __device__ __forceinline__ float2 from_c<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ double2 to_c(double v) { return make_double2(v, 0.0); }
__device__ __forceinline__ double2 to_c(double2 v) { return v; }
__device__ __forceinline__ double2 to_c(float v) { return make_double2((double)v, 0.0); }
__device__ __forceinline__ double2 to_c(float2 v) { return make_double2((double)v.x, (double)v.y); }
// element of an FP64 vector converted to the single-precision type
__device__ __forceinline__ float to_single(double v) { return (float)v; }
__device__ __forceinline__ float2 to_single(double2 v) { return make_float2((float)v.x, (float)v.y); }

// Sum of N per-thread values over a 256-thread workgroup; thread 0 gets the
// totals.  A shuffle tree inside each wave64 first, then the 4 wave results through LDS; the
// order is fixed, so results are reproducible run to run.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* lds /* [N][4] */) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_down(v[i], off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();   // lds may still be read by thread 0 from a previous call
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) lds[i * 4 + wave] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = (lds[i * 4 + 0] + lds[i * 4 + 1]) + (lds[i * 4 + 2] + lds[i * 4 + 3]);
  }
}

}  // namespace tip
