// Internal interface between the host driver (tip_api.hip) and the kernels
// (tip_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tip_device.h"

namespace tip {

// Message returned by tip_last_error() for the calling thread.
void set_last_error(const char* msg);

enum class Elem { kReal, kComplex };
enum class Prec { kF64, kF32 };            // storage and arithmetic of the CG vectors and links

// Per right-hand-side CG state codes.
enum : int { kActive = 0, kFrozen = 1, kAccepted = 2, kBreakdown = 3, kNoConv = 4, kPadding = 5 };

// Operator as the kernels see it (device pointers, kernel layouts).
struct OpDev {
  int kind;                    // 0 scalar, 1 covariant
  double mass;
  const double* mass_field;    // [V] or null
  const double* coupling;      // [ndim][V] or null
  const double* links;         // [ndim][9][V] double2 (covariant)
  const double* links_eo;      // [2][ndim][9][V/2] double2, even-odd kernels (covariant, or null)
};

// Per right-hand-side CG scalars, device arrays of length B (q: 2B).
struct CgScalars {
  double* rho;
  double* alpha;
  double* xalpha;              // x update the direction pass applies this iteration
  double* beta;
  double* rho_ref;             // residual norm^2 at the last reliable update (mixed precision)
  double* pp;                  // ||p||^2 by the recurrence ||r'||^2 + beta^2 ||p||^2
  double* anorm;               // largest Rayleigh quotient p^H A p / ||p||^2 seen (estimate of ||A||)
  double* xhn;                 // bound on ||x_h||, the single-precision x since the last update
  double* dev;                 // bound on ||(b - A x) - r|| accumulated since the last update
  double* bnorm2;
  double* relres2;
  double* q;
  int* state;
  int* iters;
  int* restarts;
  int* active;                 // number of right-hand sides still iterating
  int* ru;                     // reliable update requested (mixed precision)
  int* n_ru;                   // number of such right-hand sides
  int* ru_count;               // reliable updates done in the block
  int* ru_lanes;               // reliable updates per rhs (batched solver), or null
};

// Generic site kernels: workgroup b owns TS = 256/B sites (tile_first_site).
struct TileMap {
  int32_t logB;
  int32_t TS;
  int32_t pc, P;               // XCD-aware order, pc = 0 for plain order
  uint32_t grid;
};

// Marching stencil: workgroup -> (spatial tile of TS sites, chunk of Tc t values).
struct MarchMap {
  int32_t logB;
  int32_t TS;
  uint32_t V3;                 // sites per plane of the marching dimension
  int32_t Q;                   // spatial tiles, V3 / TS
  int32_t nt, Tc;
  int32_t xcd_order;           // workgroup -> tile order, see march_tile
  int32_t ord_n1t, ord_n2;     // order 2: x1 tiles per row, n2
  int32_t ord_g2;              // order 2: XCD regions along x2 (8 / ord_g2 along x3)
  int32_t ord_r2, ord_r3;      // order 2: rows per XCD region
  int32_t ord_b2, ord_b3;      // order 2: rows per round
  int32_t lds_links;           // stage links in LDS (covariant, TS <= 64)
  int32_t wgs_per_cu64;        // >= 2: cap resident workgroups per CU through LDS (FP64 / FP32 kernels)
  int32_t wgs_per_cu32;
  int32_t spec4;               // 4-D specialised kernel (32-bit offsets fit, 4 <= B <= 32)
  uint32_t grid;               // Q * nt / Tc
};

// Workgroup -> (spatial tile q, t-chunk) of the marching stencils.  Workgroups
// are dealt to the 8 XCDs round robin (workgroup b runs on XCD b mod 8), and
// each XCD has its own L2, so the order decides which tiles share an L2 while
// they run.
//   0: tile-major;
//   1: each XCD takes a contiguous range of tiles;
//   2: 3-D blocks (4-D lattices with whole x1 rows per tile group): XCD k owns
//      a region of r2 x r3 rows (x2, x3) and runs it in rounds of b2 x b3 rows
//      (all x1 tiles), each round through all its t-chunks before the next,
//      so the workgroups resident on one XCD at a time cover a compact block
//      at the same few t slices: they load each other's x2 +- 1 and x3 +- 1
//      neighbour rows, and the previous chunk's slices, into the same L2.
__host__ __device__ inline void march_tile(const MarchMap& mm, uint32_t b, uint32_t& q, uint32_t& chunk) {
  if (mm.xcd_order == 2) {
    const uint32_t xcd = b % kNumXcd, slot = b / kNumXcd;
    const uint32_t n1t = (uint32_t)mm.ord_n1t, b2 = (uint32_t)mm.ord_b2, b3 = (uint32_t)mm.ord_b3;
    const uint32_t r2 = (uint32_t)mm.ord_r2, r3 = (uint32_t)mm.ord_r3;
    const uint32_t bs = n1t * b2 * b3;                     // tiles per round
    const uint32_t span = bs * (uint32_t)(mm.nt / mm.Tc);  // workgroups per round (all chunks)
    const uint32_t blk = slot / span, k = slot % span;
    chunk = k / bs;
    const uint32_t w = k % bs;
    const uint32_t x1t = w % n1t, y = (w / n1t) % b2, z = w / (n1t * b2);
    const uint32_t nb2 = r2 / b2;
    const uint32_t g2 = (uint32_t)mm.ord_g2;
    const uint32_t x2 = (xcd % g2) * r2 + (blk % nb2) * b2 + y;
    const uint32_t x3 = (xcd / g2) * r3 + (blk / nb2) * b3 + z;
    q = x1t + n1t * (x2 + (uint32_t)mm.ord_n2 * x3);
  } else if (mm.xcd_order == 1) {
    const uint32_t per = (uint32_t)mm.Q / kNumXcd;        // spatial tiles per XCD
    const uint32_t xcd = b % kNumXcd, slot = b / kNumXcd;
    q = xcd * per + slot % per;
    chunk = slot / per;
  } else {
    q = b % (uint32_t)mm.Q;
    chunk = b / (uint32_t)mm.Q;
  }
}

// Dynamic LDS of the marching stencil when it stages links.
size_t march_lds_bytes(const Geom& g, const MarchMap& mm, Prec prec);

hipError_t launch_stencil(const OpDev& op, const Geom& g, const TileMap& tm, const MarchMap* mm, Elem elem,
                          Prec prec, const int* state, const int* active, const void* in, void* out, double* partial, int* ran,
                          hipStream_t st);
hipError_t launch_true_residual(const OpDev& op, const Geom& g, const TileMap& tm, Elem elem, const int* state,
                                int64_t rhs0, int nb, uint64_t seed, int mask, const void* x, void* r, void* p,
                                double* partial, size_t pstride, hipStream_t st);
hipError_t launch_init(const Geom& g, Elem elem, int logB, int64_t rhs0, int nb, uint64_t seed, int mask, void* x,
                       void* r, void* p, hipStream_t st);
// Workgroups of the update pass (= partials per right-hand side).
unsigned update_grid(size_t n);
// Workgroups of the reliable-update residual pass (= its partials per rhs).
unsigned ru_grid(const TileMap& tm);
hipError_t launch_update_r(size_t n, int logB, Elem elem, Prec prec, const CgScalars& sc, void* r, const void* Ap,
                           double* partial, hipStream_t st);
hipError_t launch_direction(size_t n, int logB, Elem elem, Prec prec, const CgScalars& sc, void* x, const void* r,
                            void* p, hipStream_t st);
// mixed precision (FP32 CG, FP64 reliable updates); mode 0 = flagged lanes, 1 = frozen lanes
hipError_t launch_init_mixed(const Geom& g, Elem elem, int logB, int64_t rhs0, int nb, uint64_t seed, int mask,
                             void* x64, void* xh, void* rh, void* ph, hipStream_t st);
hipError_t launch_ru_accumulate(size_t n, int logB, Elem elem, const CgScalars& sc, int mode, void* x64, void* xh,
                                hipStream_t st);
hipError_t launch_ru_residual(const OpDev& od64, const Geom& g, const TileMap& tm, Elem elem, const CgScalars& sc,
                              int mode, int64_t rhs0, int nb, uint64_t seed, int mask, const void* x64, void* rh,
                              void* ph, double* partial, size_t pstride, hipStream_t st);
hipError_t launch_reduce_ru(const CgScalars& sc, int B, const double* partial, int gx, size_t pstride, int mode,
                            double tol2, int max_iter, int max_restarts, hipStream_t st,
                            const double* partial2 = nullptr);
hipError_t launch_cast_links(size_t n, const double2* src, float2* dst, hipStream_t st);
// gradient: gm[s] += sum_j ||x_j(s)||^2, gw[mu][s] += sum_j ||x_j(s) - U_mu(s) x_j(s+mu)||^2 over lanes j < nb
hipError_t launch_grad_accum(const OpDev& od64, const Geom& g, Elem elem, int logB, int nb, const void* x, double* gm,
                             double* gw, hipStream_t st);
hipError_t launch_scale(size_t n, double* a, double f, hipStream_t st);
// even-odd reduced system (half-lattice vectors [ncomp][V/2][B], see k_eo_hop)
size_t eo_lds_bytes(const Geom& g, const MarchMap& mm, Prec prec);
// Modes 0 and 1 with two rhs per thread (B = 32, 16 lanes per site) for the
// single-precision covariant and the FP64 real scalar operators, with 256
// threads when the march map has 16 sites per tile and 512 when it has 32;
// hipErrorInvalidValue for any other operator.
// FP64 covariant modes 0 and 1 with 512-thread workgroups (B = 32, 16 sites per
// tile; the same march map as the pair kernel).
hipError_t launch_eo_hop_wide(int mode, const OpDev& od, const Geom& g, const MarchMap& mm, int P,
                              const double* diag, const int* state, const int* active, const void* in,
                              const void* cin, void* out, double* partial, int* ran, hipStream_t st);
// Any FP64 covariant mode (as launch_eo_hop) with 512-thread workgroups, B = 32,
// on a march map of 16-site tiles.
hipError_t launch_eo_hop512(int mode, const OpDev& od, const Geom& g, const MarchMap& mm, int P, const double* diag,
                            const int* state, const int* active, const void* in, const void* cin, void* out,
                            void* out2, void* out3, int64_t rhs0, int nb, uint64_t seed, int mask, double* partial,
                            int* ran, hipStream_t st, const int* ru, const void* cin2, void* out32, size_t pstride);
hipError_t launch_eo_hop_pair(int mode, const OpDev& od, const Geom& g, const MarchMap& mm, int P, Prec prec,
                              const double* diag, const int* state, const int* active, const void* in,
                              const void* cin, void* out, double* partial, int* ran, hipStream_t st);
hipError_t launch_eo_hop(int mode, const OpDev& od, const Geom& g, const MarchMap& mm, int P, Elem elem, Prec prec,
                         const double* diag, const int* state, const int* active, const void* in, const void* cin,
                         void* out, void* out2, void* out3, int64_t rhs0, int nb, uint64_t seed, int mask,
                         double* partial, int* ran, hipStream_t st, const int* ru = nullptr,
                         const void* cin2 = nullptr, void* out32 = nullptr, size_t pstride = 0);
hipError_t launch_eo_cast_init(size_t n, Elem elem, const void* bh, void* r, void* p, void* xh, hipStream_t st);
hipError_t launch_eo_init_odd(const Geom& g, Elem elem, Prec prec, int logB, int64_t rhs0, int nb, uint64_t seed,
                              int mask, const double* diag, void* to, hipStream_t st);
hipError_t launch_eo_scatter_even(const Geom& g, Elem elem, Prec prec, int logB, const void* xe, void* x,
                                  hipStream_t st);
// out [2][V]: D(x), then 1 / D(x)
hipError_t launch_diag(const Geom& g, const double* mass_field, double mass, const double* w, double* out,
                       hipStream_t st);
hipError_t launch_reduce_rho0(const CgScalars& sc, int B, const double* partial, int gx, hipStream_t st);
hipError_t launch_fill(size_t n, double* a, double v, hipStream_t st);
hipError_t launch_scalars_init(const CgScalars& sc, int nb, int B, double bnorm2, int start_frozen, hipStream_t st);
// soft: freeze instead of failing on p^H A p <= 0 (mixed precision); force_iter: test hook
hipError_t launch_reduce_alpha(const CgScalars& sc, int B, const double* partial, int gx, hipStream_t st,
                               int soft = 0, int force_iter = 0);
// first2 > 0: freeze threshold for solves not yet restarted (tol2 otherwise);
// eps, tau2: residual-replacement bound of mixed precision (eps = 0 turns it off)
hipError_t launch_reduce_beta(const CgScalars& sc, int B, const double* partial, int gx, double tol2, int max_iter,
                              double delta2, hipStream_t st, double first2 = 0.0, double eps = 0.0,
                              double tau2 = 0.0);
hipError_t launch_reduce_true(const CgScalars& sc, int B, const double* partial, int gx, size_t pstride, double tol2,
                              int max_iter, int max_restarts, hipStream_t st, const double* partial2 = nullptr);
hipError_t launch_hier_perm(const Geom& g, uint32_t* out, hipStream_t st);
hipError_t launch_probe_vectors(const Geom& g, uint64_t seed, int mask, int64_t m0, int count, int comp, double2* out,
                                hipStream_t st);
hipError_t launch_repack_links_eo(const Geom& g, const double2* links, double2* dst, hipStream_t st);
hipError_t launch_repack_links(const Geom& g, const double2* src, double2* dst, hipStream_t st);
// [V][ncomp] <-> lane `lane` of the block layout [ncomp][V][2^logB] (FP64)
hipError_t launch_layout(const Geom& g, Elem elem, int logB, int lane, const void* src, void* dst,
                         bool to_comp_major, hipStream_t st);

}  // namespace tip
