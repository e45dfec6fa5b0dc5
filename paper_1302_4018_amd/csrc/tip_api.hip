// Host side of libtip: the C ABI declared in include/tip.h.
//
// trace_inv_probe_op drives the hot path.  Right-hand sides (spatial probe m,
// internal component c) are solved B at a time.  For each block the kernels
// generate b in place, run CG with per-RHS scalars kept on the device, and
// confirm convergence on the true FP64 residual; the host only polls one
// counter every few iterations.  Quadratures are then combined per probe and
// summed in probe order with Neumaier compensation into the estimates at
// s = 2^k.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>
#include <atomic>
#include <memory>
#include <mutex>

#include "../../include/tip.h"
#include "tip_batch.h"
#include "tip_launch.h"

using namespace tip;

namespace {

thread_local std::string g_err;
int g_profiling = 0;

tip_status fail(tip_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define TIP_HIP(call)                                                                             \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess) return fail(TIP_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)

bool is_pow2(int64_t n) { return n >= 1 && (n & (n - 1)) == 0; }
int ilog2(int64_t n) { int k = 0; while ((int64_t(1) << k) < n) ++k; return k; }

tip_status make_geom(int32_t ndim, const int64_t* dims, int ncomp, Geom* g) {
  if (ndim < 1 || ndim > kMaxDim) return fail(TIP_EINVAL, "ndim = %d, expected 1..4", ndim);
  if (!dims) return fail(TIP_EINVAL, "dims is NULL");
  std::memset(g, 0, sizeof *g);
  g->ndim = ndim;
  g->ncomp = ncomp;
  int64_t V = 1;
  bool pow2 = true;
  for (int j = 0; j < ndim; ++j) {
    if (dims[j] < 1) return fail(TIP_EINVAL, "dims[%d] = %lld must be >= 1", j, (long long)dims[j]);
    if (V * dims[j] > (int64_t(1) << 31)) return fail(TIP_EINVAL, "lattice volume exceeds 2^31 sites");
    g->n[j] = (uint32_t)dims[j];
    g->stride[j] = (uint32_t)V;
    V *= dims[j];
    pow2 = pow2 && is_pow2(dims[j]);
  }
  g->V = (uint32_t)V;
  g->pow2 = pow2 ? 1 : 0;
  if (pow2) {
    int shift = 0;
    for (int j = 0; j < ndim; ++j) {
      const int k = ilog2(dims[j]);
      g->logn[j] = k;
      g->shift[j] = shift;
      shift += k;
      g->nlevels = std::max(g->nlevels, k);
    }
    g->L = shift;
  }
  // levels of the probing colouring: binary levels while every side with a
  // remaining size above 1 is even, then one three-colouring level when a
  // side has an odd factor (Sec. 3.4)
  int kmin_odd = 1 << 30, kmax = 0;
  bool odd = false;
  for (int j = 0; j < ndim; ++j) {
    int64_t n = dims[j];
    int k = 0;
    while (n % 2 == 0) n /= 2, ++k;
    g->k2[j] = k;
    kmax = std::max(kmax, k);
    if (n > 1) odd = true, kmin_odd = std::min(kmin_odd, k);
  }
  g->B = odd ? kmin_odd : kmax;
  g->LB = 0;
  for (int m = 0; m < g->B; ++m)
    for (int j = 0; j < ndim; ++j) g->LB += g->k2[j] > m ? 1 : 0;
  g->has3 = odd ? 1 : 0;
  for (int j = 0; j < ndim; ++j) g->sub[j] = (uint32_t)(dims[j] >> g->B);
  const uint64_t gamma = (uint64_t(1) << g->LB) * (odd ? 3u : 1u);
  g->gamma = (uint32_t)std::min<uint64_t>(gamma, uint64_t(1) << 31);
  return TIP_OK;
}

// Device allocation, frees, stream creation and device-wide synchronisation
// may synchronise the device, which must not happen while another thread
// captures a HIP graph (trace_inv_probe_batch runs calls on several threads).
// They and the captures take this lock.
std::mutex g_device_mu;

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  ~DevBuf() {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_device_mu);
    (void)hipFree(p);
  }
  hipError_t ensure(size_t bytes) {
    if (bytes <= n) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_device_mu);
    if (p) { (void)hipFree(p); p = nullptr; n = 0; }
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipSuccess) n = bytes;
    return e;
  }
};

struct HostPinned {
  void* p = nullptr;
  size_t n = 0;
  ~HostPinned() {
    if (!p) return;
    std::lock_guard<std::mutex> lk(g_device_mu);
    (void)hipHostFree(p);
  }
  hipError_t ensure(size_t bytes) {
    if (bytes <= n) return hipSuccess;
    std::lock_guard<std::mutex> lk(g_device_mu);
    if (p) { (void)hipHostFree(p); p = nullptr; n = 0; }
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
    if (e == hipSuccess) n = bytes;
    return e;
  }
};

}  // namespace

void tip::set_last_error(const char* msg) { g_err = msg; }

struct tip_op_s {
  Geom geom{};                 // ncomp filled from kind
  int kind = 0;
  double mass = 0.0;
  DevBuf links, mass_field, coupling;
  DevBuf links32;              // single-precision copy, made on first mixed-precision use
  DevBuf diag;                 // [2][V] FP64: D(x) = m(x) + sum_mu [w_mu(x) + w_mu(x - mu)], then 1 / D(x)
  DevBuf links_eo;             // covariant, every side even: links by parity (see k_repack_links_eo)
  DevBuf links_eo32;           // its single-precision copy, made on first mixed-precision use
  bool has_links_eo = false, has_links_eo32 = false;
  bool has_mass_field = false, has_coupling = false, has_links32 = false;
  // lower bound of the spectrum: A = sum_e w_e L_e + diag(m) with L_e PSD, so
  // lambda_min >= min m(x) whenever every w_e >= 0 (NaN when not known)
  double lambda_lb = 0.0;
  // workspace, grown on demand
  DevBuf vec, partial, scal;
  HostPinned host;
  std::vector<hipEvent_t> events;
  // a non-blocking stream of the handle's own, used when the caller passes the
  // null stream (which cannot be captured into a graph); calls synchronise it
  // before they return
  hipStream_t own_stream = nullptr;

  OpDev dev(bool single = false) const {
    OpDev o;
    o.kind = kind;
    o.mass = mass;
    o.mass_field = has_mass_field ? (const double*)mass_field.p : nullptr;
    o.coupling = has_coupling ? (const double*)coupling.p : nullptr;
    o.links = kind == 1 ? (const double*)(single ? links32.p : links.p) : nullptr;
    o.links_eo = kind != 1 ? nullptr
                 : single ? (has_links_eo32 ? (const double*)links_eo32.p : nullptr)
                          : (has_links_eo ? (const double*)links_eo.p : nullptr);
    return o;
  }
  ~tip_op_s() {
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    if (own_stream) {
      std::lock_guard<std::mutex> lk(g_device_mu);
      (void)hipStreamDestroy(own_stream);
    }
  }
};

namespace {

tip_status validate_op(const tip_operator* op, Geom* g) {
  if (!op) return fail(TIP_EINVAL, "operator is NULL");
  if (op->kind != TIP_KIND_SCALAR && op->kind != TIP_KIND_COVARIANT)
    return fail(TIP_EINVAL, "unknown operator kind %d", op->kind);
  tip_status st = make_geom(op->ndim, op->dims, op->kind == TIP_KIND_COVARIANT ? 3 : 1, g);
  if (st != TIP_OK) return st;
  if (op->kind == TIP_KIND_COVARIANT && !op->links) return fail(TIP_EINVAL, "covariant operator needs links");
  if (!op->mass_field && !std::isfinite(op->mass)) return fail(TIP_EINVAL, "mass is not finite");
  return TIP_OK;
}

tip_status create_handle(const tip_operator* op, hipStream_t st, tip_op_s** out) {
  Geom g;
  tip_status s = validate_op(op, &g);
  if (s != TIP_OK) return s;
  tip_op_s* h = new (std::nothrow) tip_op_s();
  if (!h) return fail(TIP_ENOMEM, "out of host memory");
  h->geom = g;
  h->kind = op->kind;
  h->mass = op->mass;
  const size_t V = g.V;
  auto bail = [&](tip_status code) { delete h; return code; };
  if (op->mass_field) {
    if (const hipError_t e_ = h->mass_field.ensure(V * sizeof(double)); e_ != hipSuccess)
      return bail(fail(TIP_ENOMEM, "hipMalloc mass_field: %s", hipGetErrorString(e_)));
    if (hipMemcpyAsync(h->mass_field.p, op->mass_field, V * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
      return bail(fail(TIP_EDEVICE, "copy of mass_field failed"));
    h->has_mass_field = true;
  }
  if (op->coupling) {
    const size_t n = (size_t)g.ndim * V * sizeof(double);
    if (const hipError_t e_ = h->coupling.ensure(n); e_ != hipSuccess)
      return bail(fail(TIP_ENOMEM, "hipMalloc coupling: %s", hipGetErrorString(e_)));
    if (hipMemcpyAsync(h->coupling.p, op->coupling, n, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return bail(fail(TIP_EDEVICE, "copy of coupling failed"));
    h->has_coupling = true;
  }
  if (op->kind == TIP_KIND_COVARIANT) {
    const size_t n = (size_t)g.ndim * 9 * V * sizeof(double2);
    if (const hipError_t e_ = h->links.ensure(n); e_ != hipSuccess)
      return bail(fail(TIP_ENOMEM, "hipMalloc links (%zu bytes): %s", n, hipGetErrorString(e_)));
    if (launch_repack_links(g, (const double2*)op->links, (double2*)h->links.p, st) != hipSuccess)
      return bail(fail(TIP_EDEVICE, "link repack launch failed"));
    bool bip = g.pow2 != 0;
    for (int mu = 0; mu < g.ndim; ++mu) bip = bip && g.logn[mu] >= 1;
    if (bip) {
      if (const hipError_t e_ = h->links_eo.ensure(n); e_ != hipSuccess)
      return bail(fail(TIP_ENOMEM, "hipMalloc even-odd links (%zu bytes): %s", n, hipGetErrorString(e_)));
      if (launch_repack_links_eo(g, (const double2*)h->links.p, (double2*)h->links_eo.p, st) != hipSuccess)
        return bail(fail(TIP_EDEVICE, "even-odd link repack launch failed"));
      h->has_links_eo = true;
    }
  }
  if (const hipError_t e_ = h->diag.ensure(2 * V * sizeof(double)); e_ != hipSuccess)
      return bail(fail(TIP_ENOMEM, "hipMalloc diagonal: %s", hipGetErrorString(e_)));
  if (launch_diag(g, h->has_mass_field ? (const double*)h->mass_field.p : nullptr, op->mass,
                  h->has_coupling ? (const double*)h->coupling.p : nullptr, (double*)h->diag.p, st) != hipSuccess)
    return bail(fail(TIP_EDEVICE, "diagonal launch failed"));
  if (hipStreamSynchronize(st) != hipSuccess) return bail(fail(TIP_EDEVICE, "operator setup failed on the device"));
  {
    double lb = op->mass;
    if (op->mass_field) {
      std::vector<double> m(V);
      hipError_t e;
      {
        std::lock_guard<std::mutex> lk(g_device_mu);   // a null-stream copy
        e = hipMemcpy(m.data(), op->mass_field, V * sizeof(double), hipMemcpyDeviceToHost);
      }
      if (e != hipSuccess) return bail(fail(TIP_EDEVICE, "reading mass_field failed"));
      lb = *std::min_element(m.begin(), m.end());
    }
    if (op->coupling) {
      std::vector<double> w((size_t)g.ndim * V);
      hipError_t e;
      {
        std::lock_guard<std::mutex> lk(g_device_mu);   // a null-stream copy
        e = hipMemcpy(w.data(), op->coupling, w.size() * sizeof(double), hipMemcpyDeviceToHost);
      }
      if (e != hipSuccess) return bail(fail(TIP_EDEVICE, "reading coupling failed"));
      if (*std::min_element(w.begin(), w.end()) < 0.0) lb = std::nan("");
    }
    h->lambda_lb = lb;
  }
  *out = h;
  return TIP_OK;
}

// Neumaier running sum.
struct Compensated {
  double s = 0.0, c = 0.0;
  void add(double v) {
    const double t = s + v;
    if (std::fabs(s) >= std::fabs(v)) c += (s - t) + v;
    else c += (v - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

int num_checkpoints(int64_t n) {
  if (n < 1) return 0;
  int k = 0;
  while ((int64_t(1) << (k + 1)) <= n) ++k;
  return k + 1 + (is_pow2(n) ? 0 : 1);
}

int64_t checkpoint_size(int64_t n, int idx) {
  const int npow = num_checkpoints(n) - (is_pow2(n) ? 0 : 1);
  return idx < npow ? (int64_t(1) << idx) : n;
}

struct Plan {
  Elem elem;
  int mask;
  int B, logB; // right-hand sides per block (power of two <= 64), one per lane
  size_t esz;  // bytes per vector element
  TileMap tm;  // generic site kernels
  MarchMap mm; // marching stencil (valid when use_march)
  bool use_march;
  bool eo = false;  // CG on the even-odd reduced system
  MarchMap me;      // half-lattice march (valid when eo)
  bool pair = false;  // single-precision covariant hops with two rhs per thread (B = 32)
  bool wide = false;  // FP64 covariant hops with 512-thread workgroups (B = 32)
  MarchMap me2;       // the march of either (16 sites per tile)
  bool eo512 = false; // FP64 once-per-block and reliable-update passes in 512-thread workgroups on me2
};

bool env_off(const char* name) {
  const char* e = std::getenv(name);
  return e && e[0] == '0';
}

TileMap make_tilemap(const Geom& g, int logB) {
  TileMap tm{};
  tm.logB = logB;
  tm.TS = kBlock >> logB;
  const int64_t V = g.V, ntiles = (V + tm.TS - 1) / tm.TS;
  tm.grid = (uint32_t)ntiles;
  // XCD-aware order: whole tiles, a tile count divisible by the XCD count and
  // whole planes of the last dimension per XCD chunk (TIP_TILE_ORDER=0: off).
  const int64_t n_last = g.n[g.ndim - 1];
  if (g.pow2 && !env_off("TIP_TILE_ORDER") && V % tm.TS == 0 && ntiles % kNumXcd == 0 && ntiles % n_last == 0) {
    const int64_t P = ntiles / n_last, C = ntiles / kNumXcd;
    if (C % P == 0) {
      tm.pc = (int32_t)(C / P);
      tm.P = (int32_t)P;
    }
  }
  return tm;
}

// Marching stencil map, or false when the geometry does not fit it
// (TIP_MARCH=0 turns it off; TIP_MARCH_TC fixes the chunk length).
bool env_on(const char* name) {
  const char* e = std::getenv(name);
  return e && std::atoi(e) != 0;
}

// Parameters of tile order 2 (see march_tile) for a 4-D lattice marched
// along x4: split the (x2, x3) rows over the 8 XCDs into slabs as thin along x2
// (and so as long along x3) as the sides allow, then pick the round (b2 x b3
// rows of n1/TS tiles each) of at most `round_tiles` tiles that leaves the
// fewest x2 / x3 neighbour rows outside it.  Measured at 32^4 (FP64 / mixed
// solves/s, one box): slabs of 4 x 32 rows with rounds of 4 x 16 rows 951-953 /
// 1492 against 940-941 / 1479 for the squarest regions (8 x 16 rows, rounds of
// 8 x 8), and 902-920 for regions of 16 x 8 rows.  TIP_MARCH_ORDER="g2,b2,b3"
// overrides the choice.
bool plan_block_order(const Geom& g, int TS, MarchMap* mm, int round_tiles) {
  const int n1 = 1 << g.logn[0], n2 = 1 << g.logn[1], n3 = 1 << g.logn[2];
  if (TS > n1 || n1 % TS != 0) return false;
  const int n1t = n1 / TS;
  if (const char* e = std::getenv("TIP_ROUND_TILES")) round_tiles = std::max(1, std::atoi(e));   // experiments
  int best_g2 = -1;
  for (int g2 = 1; g2 <= kNumXcd; g2 *= 2) {
    const int g3 = kNumXcd / g2;
    if (g2 > n2 || g3 > n3) continue;
    best_g2 = g2;                                   // the largest split of x2 that fits
  }
  if (best_g2 < 0) return false;
  int g2 = best_g2, b2 = 0, b3 = 0;
  int r2 = n2 / g2, r3 = n3 / (kNumXcd / g2);
  double best_cost = 1e30;
  for (int c2 = 1; c2 <= r2; c2 *= 2)
    for (int c3 = 1; c3 <= r3; c3 *= 2) {
      if (n1t * c2 * c3 > round_tiles) continue;
      const double cost = (c2 < n2 ? 2.0 / c2 : 0.0) + (c3 < n3 ? 2.0 / c3 : 0.0);
      if (cost < best_cost || (cost == best_cost && c2 * c3 > b2 * b3)) best_cost = cost, b2 = c2, b3 = c3;
    }
  if (const char* e = std::getenv("TIP_MARCH_ORDER")) {
    int a = 0, b = 0, c = 0;
    if (std::sscanf(e, "%d,%d,%d", &a, &b, &c) == 3 && a >= 1 && a <= kNumXcd && (a & (a - 1)) == 0 && a <= n2 &&
        kNumXcd / a <= n3) {
      const int rr2 = n2 / a, rr3 = n3 / (kNumXcd / a);
      if (b >= 1 && c >= 1 && rr2 % b == 0 && rr3 % c == 0) g2 = a, r2 = rr2, r3 = rr3, b2 = b, b3 = c;
    }
  }
  if (b2 < 1 || b3 < 1) return false;
  mm->ord_n1t = n1t;
  mm->ord_n2 = n2;
  mm->ord_g2 = g2;
  mm->ord_r2 = r2;
  mm->ord_r3 = r3;
  mm->ord_b2 = b2;
  mm->ord_b3 = b3;
  return true;
}

// Every workgroup of the grid must get a distinct (tile, chunk) in range;
// checked on the host before order 2 is used (grids up to 2^22 workgroups).
bool block_order_is_permutation(const MarchMap& mm) {
  const uint32_t nchunk = mm.grid / (uint32_t)mm.Q;
  if (mm.grid > (1u << 22) || mm.grid % kNumXcd != 0) return false;
  std::vector<unsigned char> seen(mm.grid, 0);
  for (uint32_t b = 0; b < mm.grid; ++b) {
    uint32_t q = 0, chunk = 0;
    march_tile(mm, b, q, chunk);
    if (q >= (uint32_t)mm.Q || chunk >= nchunk) return false;
    unsigned char& v = seen[(size_t)chunk * mm.Q + q];
    if (v) return false;
    v = 1;
  }
  return true;
}

// halve_t: march the half-lattice of the even-odd system (t slices of two).
// round_tiles / tc: per-call tuning (0 = the defaults below).
bool make_marchmap(const Geom& g, int logB, MarchMap* mm, bool halve_t = false, int round_tiles = 0, int tc = 0) {
  if (!g.pow2) return false;                         // the marching kernels index with shifts
  if (!halve_t && (env_off("TIP_MARCH") || g.ndim < 2)) return false;
  const int nt = (1 << g.logn[g.ndim - 1]) >> (halve_t ? 1 : 0);
  if (nt < (halve_t ? 1 : 2)) return false;
  const int TS = kBlock >> logB;
  const uint32_t V3 = g.V >> g.logn[g.ndim - 1];
  if (V3 % (uint32_t)TS != 0) return false;
  mm->logB = logB;
  mm->TS = TS;
  mm->V3 = V3;
  mm->Q = (int32_t)(V3 / TS);
  mm->nt = nt;
  int Tc = nt;
  const char* env_tc = std::getenv("TIP_MARCH_TC");
  const int want_tc = tc > 0 ? tc : (env_tc ? std::atoi(env_tc) : 0);
  if (want_tc >= 1 && want_tc <= nt && (want_tc & (want_tc - 1)) == 0) {
    Tc = want_tc;
  } else {
    while (Tc > 1 && (int64_t)mm->Q * (nt / Tc) < 2048) Tc /= 2;
  }
  mm->Tc = Tc;
  mm->xcd_order = !env_off("TIP_TILE_ORDER") && mm->Q % kNumXcd == 0;
  // rounds of 128 tiles for the full stencil, 256 for the half-lattice one
  // (measured on the 32^4 covariant workload)
  if (mm->xcd_order && g.ndim == 4 && plan_block_order(g, TS, mm, round_tiles > 0 ? round_tiles : (halve_t ? 256 : 128)))
    mm->xcd_order = 2;
  if (const char* e = std::getenv("TIP_TILE_ORDER")) {
    if (std::atoi(e) == 1 && mm->xcd_order == 2) mm->xcd_order = 1;
  }
  mm->lds_links = !env_off("TIP_LDS_LINKS") && TS <= 64;
  mm->wgs_per_cu64 = 0;
  mm->wgs_per_cu32 = 0;
  if (const char* e = std::getenv("TIP_WGS_PER_CU64")) mm->wgs_per_cu64 = std::atoi(e);
  if (const char* e = std::getenv("TIP_WGS_PER_CU32")) mm->wgs_per_cu32 = std::atoi(e);
  // the 4-D specialised kernel addresses every array with 32-bit byte
  // offsets: 3 components x V x B x 16 bytes and the links must fit in 4 GiB
  const double vec_bytes = 3.0 * g.V * (double)(1 << logB) * 16.0;
  const double link_bytes = 4.0 * 9.0 * g.V * 16.0;
  mm->spec4 = !env_off("TIP_SPEC4") && g.ndim == 4 && logB >= 2 && logB <= 5 && vec_bytes < 4294967296.0 &&
              link_bytes < 4294967296.0;
  mm->grid = (uint32_t)mm->Q * (uint32_t)(nt / Tc);
  if (mm->xcd_order == 2 && !block_order_is_permutation(*mm)) mm->xcd_order = 1;
  return true;
}

// Common validation of the solve parameters; resolves the mask.
tip_status check_params(const tip_op_s* h, const tip_params* p, int* mask_out) {
  if (!p) return fail(TIP_EINVAL, "params is NULL");
  const int64_t V = h->geom.V;
  if (p->n_vectors < 1 || p->n_vectors > V)
    return fail(TIP_EINVAL, "n_vectors = %lld must be in [1, V = %lld]", (long long)p->n_vectors, (long long)V);
  if (p->m_begin < 0 || p->m_begin > p->n_vectors)
    return fail(TIP_EINVAL, "m_begin = %lld must be in [0, n_vectors]", (long long)p->m_begin);
  if (!(p->tol > 0.0) || !std::isfinite(p->tol)) return fail(TIP_EINVAL, "tol must be positive and finite");
  if (p->max_iter < 0) return fail(TIP_EINVAL, "max_iter must be >= 0");
  if (p->rhs_block < 0) return fail(TIP_EINVAL, "rhs_block must be >= 0");
  if (p->precision != TIP_PREC_FP64 && p->precision != TIP_PREC_MIXED)
    return fail(TIP_EINVAL, "unknown precision %d", p->precision);
  if (!(p->reliable_delta >= 0.0 && p->reliable_delta < 1.0))
    return fail(TIP_EINVAL, "reliable_delta must be in [0, 1)");
  int mask = p->mask;
  if (mask == TIP_MASK_DEFAULT) mask = h->kind == TIP_KIND_COVARIANT ? TIP_MASK_Z4 : TIP_MASK_Z2;
  if (mask < TIP_MASK_NONE || mask > TIP_MASK_Z4) return fail(TIP_EINVAL, "unknown mask %d", p->mask);
  if (p->probe < TIP_PROBE_HIERARCHICAL || p->probe > TIP_PROBE_FOURIER)
    return fail(TIP_EINVAL, "unknown probe kind %d", p->probe);
  if (p->round_tiles < 0 || p->march_tc < 0) return fail(TIP_EINVAL, "round_tiles and march_tc must be >= 0");
  if ((p->probe == TIP_PROBE_NATURAL || p->probe == TIP_PROBE_STOPPED || p->probe == TIP_PROBE_FOURIER) &&
      !h->geom.pow2)
    return fail(TIP_EINVAL, "probe kind %d needs power-of-two sides", p->probe);
  if (p->stop_levels < 0) return fail(TIP_EINVAL, "stop_levels must be >= 0");
  if (p->probe == TIP_PROBE_RANDOM && mask == TIP_MASK_NONE)
    return fail(TIP_EINVAL, "random probes need a Z2 or Z4 mask");
  *mask_out = mask;
  return TIP_OK;
}

// CG over blocks of right-hand sides on one prepared operator.
//   FP64:  x, r, p, w in FP64; one FP64 true-residual check per solve.
//   mixed: x in FP64; correction xh, r, p, w in FP32 with FP32 links; FP64
//          reliable updates whenever the bound on the drift of the FP32
//          residual from b - A x asks for one (k_reduce_beta), and the same
//          FP64 true-residual check at the end.
struct Solver {
  tip_op_s* h;
  const tip_params* p;
  Geom geom;                 // the operator's lattice with this call's probe kind
  hipStream_t st;
  Plan pl;
  bool mixed = false;
  bool need_x = false;          // even-odd: assemble x on the full lattice (gradient, solve_probe)
  int force_elem = -1;          // 0 real, 1 complex solves (the caller knows the right-hand sides); -1 automatic
  int64_t rhs_hint = 0;         // > 0: right-hand sides of this pass (bounds the block size when rhs_block = 0)
  Prec prec = Prec::kF64;
  int max_iter, max_restarts = 8;
  double tol2, delta2 = 0.0, ru_eps = 0.0, ru_tau2 = 0.0;
  double freeze2;               // recursive-residual freeze threshold (tol2 unless TIP_FREEZE_SLACK)
  int force_breakdown = 0;      // TIP_FORCE_BREAKDOWN = k (tests): iteration k of a fresh solve breaks down
  size_t vbytes, vbytes64, pstride, nscal, nelem, nvec;
  int gx_m, gx_u, gx_t;       // partials per rhs written by matvec, update, true residual
  int gx_p;                   // partials per rhs of the iteration's matvec (gx_m unless pair)
  void *X, *Rv, *Pv, *W, *XH; // FP64 path: X, Rv, Pv, W; mixed: X (FP64) + XH, Rv, Pv, W (FP32)
  void *Xe = nullptr, *Tv = nullptr;   // even-odd: x_e and t_o (half lattice)
  void *Bh = nullptr, *T64 = nullptr;  // mixed even-odd: b_hat and an FP64 t_o (half lattice)
  double* part;
  CgScalars sc;
  int* ran_dev;
  double *h_q, *h_relres2;
  int *h_state, *h_iters, *h_restarts, *h_active, *h_ran;
  OpDev od, od64;
  double mv_bytes;              // dominant stencil kernel, per launch
  double hop_bytes = 0.0;       // even-odd: the other half-lattice kernel, per launch
  int64_t matvecs = 0;
  double matvec_seconds = 0.0, matvec_bytes = 0.0;
  int predicted = 8;
  int64_t reliable_updates = 0;
  int64_t restarts = 0;          // solves restarted after a failed true-residual check
  // stencil accounting
  int64_t stencil_launches = 0;
  double stencil_seconds = 0.0, stencil_bytes = 0.0;
  struct Timed { hipEvent_t a, b, c; };
  size_t ev_used = 0;
  static constexpr int kMaxChunk = 4096;

  hipError_t next_event(hipEvent_t* e) {
    if (ev_used == h->events.size()) {
      hipEvent_t ne;
      hipError_t r = hipEventCreate(&ne);
      if (r != hipSuccess) return r;
      h->events.push_back(ne);
    }
    *e = h->events[ev_used++];
    return hipSuccess;
  }

  tip_status setup(tip_op_s* handle, const tip_params* params, int mask) {
    h = handle;
    p = params;
    geom = h->geom;
    geom.probe = p->probe;
    geom.stop = p->stop_levels;
    st = (hipStream_t)p->stream;
    if (!st && !env_off("TIP_GRAPH")) {
      if (!h->own_stream) {
        std::lock_guard<std::mutex> lk(g_device_mu);
        if (hipStreamCreateWithFlags(&h->own_stream, hipStreamNonBlocking) != hipSuccess) h->own_stream = nullptr;
      }
      if (h->own_stream) {
        // work the caller queued on the null stream comes first
        TIP_HIP(hipStreamSynchronize(nullptr));
        st = h->own_stream;
      }
    }
    mixed = p->precision == TIP_PREC_MIXED;
    prec = mixed ? Prec::kF32 : Prec::kF64;
    const Geom& g = geom;
    const int64_t V = g.V;
    const int ncomp = g.ncomp;
    pl.mask = mask;
    // complex solves: covariant operator, Z4 mask, or a probe past the binary
    // columns (F_3 columns of the three-colouring level are complex)
    const bool f3 = g.has3 && p->n_vectors > (int64_t(1) << g.LB);
    const bool fourier = p->probe == TIP_PROBE_FOURIER;          // roots of unity w16^e
    pl.elem = (h->kind == TIP_KIND_COVARIANT || mask == TIP_MASK_Z4 || f3 || fourier) ? Elem::kComplex : Elem::kReal;
    if (force_elem >= 0) pl.elem = force_elem ? Elem::kComplex : Elem::kReal;
    const size_t esz64 = pl.elem == Elem::kReal ? sizeof(double) : sizeof(double2);
    pl.esz = mixed ? esz64 / 2 : esz64;
    // block size: a power of two <= 64; 32 shares each link among 32 solves;
    // small lattices take more right-hand sides per block to fill the GPU.
    // B depends only on the operator and rhs_block, so a right-hand side is
    // solved with the same arithmetic whichever block it falls in (resumed
    // runs reproduce uninterrupted ones bit for bit), except in the probe
    // classes of odd-sided real problems below.
    int B = 1;
    if (p->rhs_block > 0) {
      while (B < p->rhs_block && B < 64) B *= 2;
    } else {
      B = 32;
      while (B < 64 && V * B < (int64_t(1) << 18)) B *= 2;
    }
    // a pass over fewer right-hand sides than that (a probe class of an
    // odd-sided lattice) takes the smallest power of two that holds them
    if (p->rhs_block <= 0 && rhs_hint > 0)
      while (B > 1 && B / 2 >= rhs_hint) B /= 2;
    // keep the CG vectors of a block within 32 GiB
    while (B > 1 && 4.5 * B * ncomp * (double)V * esz64 > 32.0 * (1ull << 30)) B /= 2;
    pl.B = B;
    pl.logB = 0;
    while ((1 << pl.logB) < B) ++pl.logB;
    pl.tm = make_tilemap(g, pl.logB);
    pl.use_march = make_marchmap(g, pl.logB, &pl.mm, false, p->round_tiles, p->march_tc);
    // even-odd reduction: bipartite torus (every side >= 2, all powers of two
    // are then even) and a positive diagonal (lambda_lb > 0 implies D > 0)
    {
      bool bip = g.pow2 != 0;
      for (int mu = 0; mu < g.ndim; ++mu) bip = bip && g.logn[mu] >= 1;
      pl.eo = bip && h->lambda_lb > 0.0 && !env_off("TIP_EO") &&
              make_marchmap(g, pl.logB, &pl.me, true, p->round_tiles, p->march_tc);
      // the covariant half-lattice kernel stages its tile's links in LDS
      if (pl.eo && h->kind == TIP_KIND_COVARIANT && (eo_lds_bytes(g, pl.me, prec) > 65536 || !h->has_links_eo))
        pl.eo = false;
      // 32 rhs with 8-byte lane elements (single-precision covariant without
      // couplings, FP64 real scalar): the iteration's two hops load two rhs
      // per thread (TIP_EO_PAIR=0 turns this off); rounds of 128 of these
      // tiles cover as many sites as 256 of the others
      const bool pair_op = (mixed && h->kind == TIP_KIND_COVARIANT && !h->has_coupling) ||
                           (!mixed && h->kind == TIP_KIND_SCALAR && pl.elem == Elem::kReal);
      // the scalar form runs 512 threads (32 sites per tile) where 32 sites
      // divide a plane: 1457 against 1483 us on a 256^3 torus
      const auto pair_map = [&](int lb) {
        return make_marchmap(g, lb, &pl.me2, true, p->round_tiles > 0 ? p->round_tiles : (lb == 3 ? 64 : 128),
                             p->march_tc);
      };
      pl.pair = pl.eo && pair_op && pl.B == 32 && !env_off("TIP_EO_PAIR") &&
                ((h->kind == TIP_KIND_SCALAR && pair_map(3)) || pair_map(4)) &&
                (h->kind != TIP_KIND_COVARIANT || eo_lds_bytes(g, pl.me2, prec) <= 65536);
      // FP64 covariant, 32 rhs: the same tiles of 16 sites with one rhs per
      // lane, in 512-thread workgroups (TIP_EO_WIDE=0 turns this off)
      pl.wide = !pl.pair && pl.eo && !mixed && h->kind == TIP_KIND_COVARIANT && pl.B == 32 &&
                !env_off("TIP_EO_WIDE") &&
                make_marchmap(g, 4, &pl.me2, true, p->round_tiles > 0 ? p->round_tiles : 128, p->march_tc) &&
                eo_lds_bytes(g, pl.me2, prec) <= 65536;
      // the FP64 passes outside the iteration (reduced right-hand side, true
      // residual, reliable updates) stay in 256-thread workgroups: with 180-200
      // VGPRs they run 2 waves per SIMD, i.e. two 256-thread workgroups per CU
      // against one of 512, and measured 10-12% faster that way.
      // TIP_EO_WIDE_ONCE=1 puts them on the 16-site tiles in 512 threads.
      pl.eo512 = (pl.wide || pl.pair) && h->kind == TIP_KIND_COVARIANT && pl.B == 32 &&
                 eo_lds_bytes(g, pl.me2, Prec::kF64) <= 65536 && env_on("TIP_EO_WIDE_ONCE");
    }
    max_iter = p->max_iter > 0 ? p->max_iter : (int)std::min<int64_t>(10 * V * ncomp, 1 << 20);
    tol2 = p->tol * p->tol;
    // TIP_FREEZE_SLACK = f > 1 (tests): freeze a solve that has not restarted
    // once its recursive residual is below f tol, so the first FP64
    // true-residual check fails and the solve restarts from x -- the path a
    // drifting recursive residual takes; after that the threshold is tol
    freeze2 = tol2;
    if (const char* e = std::getenv("TIP_FORCE_BREAKDOWN")) force_breakdown = std::max(0, std::atoi(e));
    if (const char* e = std::getenv("TIP_FREEZE_SLACK")) {
      const double f = std::atof(e);
      if (f > 1.0 && std::isfinite(f)) freeze2 = tol2 * f * f;
    }
    if (mixed) {
      // residual replacement once the drift bound passes tau ||r||, tau = 2^-5.
      // Measured against tau = 2^-12 (sqrt of the unit roundoff) and 2^-8: at
      // 32^4 one FP64 update per solve instead of two (1308 against 1204
      // solves/s), and on free fields at kappa 1e4..1e6 no restarts and at most
      // 4% more iterations.
      ru_eps = 0x1p-24;
      ru_tau2 = 0x1p-10;
      delta2 = p->reliable_delta * p->reliable_delta;
    }

    nelem = (size_t)B * ncomp * V;
    vbytes = nelem * pl.esz;                      // one CG vector of the block
    vbytes64 = nelem * esz64;
    nvec = pl.eo ? nelem / 2 : nelem;             // elements the CG vector passes touch
    gx_m = (int)(pl.eo ? pl.me.grid : (pl.use_march ? pl.mm.grid : pl.tm.grid));
    gx_p = (pl.pair || pl.wide) ? (int)pl.me2.grid : gx_m;
    gx_u = (int)update_grid(nvec);
    gx_t = (int)ru_grid(pl.tm);
    pstride = (size_t)B * std::max(std::max(gx_m, gx_p), std::max(gx_u, gx_t));
    nscal = (size_t)B;
    // FP64: x, r, p, w; mixed: x (FP64) + xh, r, p, w (FP32); even-odd: x on the
    // full lattice + x_e, r, p, w, t on the half lattice
    // mixed even-odd: x (FP64, full lattice), x_e, b_hat, t (FP64, half) and
    // x_h, r, p, w, t (FP32, half)
    const size_t vec_total = pl.eo ? (mixed ? vbytes64 + 3 * (vbytes64 / 2) + 5 * (vbytes / 2)
                                            : vbytes + 5 * (vbytes / 2))
                                   : (mixed ? vbytes64 + 4 * vbytes : 4 * vbytes);
    if (const hipError_t e_ = h->vec.ensure(vec_total); e_ != hipSuccess)
      return fail(TIP_ENOMEM, "hipMalloc of %zu bytes of CG vectors failed: %s", vec_total, hipGetErrorString(e_));
    // 5 rows of per-workgroup partials, and 5 more for the second pass of the
    // even-odd true residual
    if (const hipError_t e_ = h->partial.ensure(10 * pstride * sizeof(double)); e_ != hipSuccess)
      return fail(TIP_ENOMEM, "hipMalloc partials: %s", hipGetErrorString(e_));
    const size_t scal_bytes = nscal * (13 * sizeof(double) + 4 * sizeof(int)) + 128 + kMaxChunk * sizeof(int);
    if (const hipError_t e_ = h->scal.ensure(scal_bytes); e_ != hipSuccess)
      return fail(TIP_ENOMEM, "hipMalloc scalars: %s", hipGetErrorString(e_));
    const size_t host_bytes = nscal * (3 * sizeof(double) + 3 * sizeof(int)) + 128 + kMaxChunk * sizeof(int);
    if (const hipError_t e_ = h->host.ensure(host_bytes); e_ != hipSuccess)
      return fail(TIP_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e_));
    if (mixed && h->kind == TIP_KIND_COVARIANT && !h->has_links32) {
      const size_t n = (size_t)g.ndim * 9 * V;
      if (const hipError_t e_ = h->links32.ensure(n * sizeof(float2)); e_ != hipSuccess)
      return fail(TIP_ENOMEM, "hipMalloc FP32 links: %s", hipGetErrorString(e_));
      TIP_HIP(launch_cast_links(n, (const double2*)h->links.p, (float2*)h->links32.p, st));
      h->has_links32 = true;
    }
    if (mixed && pl.eo && h->kind == TIP_KIND_COVARIANT && !h->has_links_eo32) {
      const size_t n = (size_t)g.ndim * 9 * V;
      if (const hipError_t e_ = h->links_eo32.ensure(n * sizeof(float2)); e_ != hipSuccess)
      return fail(TIP_ENOMEM, "hipMalloc FP32 links: %s", hipGetErrorString(e_));
      TIP_HIP(launch_cast_links(n, (const double2*)h->links_eo.p, (float2*)h->links_eo32.p, st));
      h->has_links_eo32 = true;
    }

    char* vb = (char*)h->vec.p;
    X = vb;
    if (mixed && pl.eo) {
      const size_t h64 = vbytes64 / 2, h32 = vbytes / 2;
      char* q = vb + vbytes64;
      Xe = q;
      Bh = q + h64;
      T64 = q + 2 * h64;
      q += 3 * h64;
      XH = q;
      Rv = q + h32;
      Pv = q + 2 * h32;
      W = q + 3 * h32;
      Tv = q + 4 * h32;
      if (pl.pair && (((uintptr_t)Pv | (uintptr_t)Tv | (uintptr_t)W) & 15u))
        return fail(TIP_EDEVICE, "internal: single-precision half vectors not 16-byte aligned");
    } else if (mixed) {
      XH = vb + vbytes64;
      Rv = vb + vbytes64 + vbytes;
      Pv = vb + vbytes64 + 2 * vbytes;
      W = vb + vbytes64 + 3 * vbytes;
    } else if (pl.eo) {
      const size_t hb = vbytes / 2;
      XH = nullptr;
      Xe = vb + vbytes;
      Rv = vb + vbytes + hb;
      Pv = vb + vbytes + 2 * hb;
      W = vb + vbytes + 3 * hb;
      Tv = vb + vbytes + 4 * hb;
      if (pl.pair && (((uintptr_t)Pv | (uintptr_t)Tv | (uintptr_t)W) & 15u))
        return fail(TIP_EDEVICE, "internal: half vectors not 16-byte aligned");
    } else {
      XH = nullptr;
      Rv = vb + vbytes;
      Pv = vb + 2 * vbytes;
      W = vb + 3 * vbytes;
    }
    part = (double*)h->partial.p;
    double* d = (double*)h->scal.p;
    sc.rho = d;
    sc.alpha = d + nscal;
    sc.xalpha = d + 2 * nscal;
    sc.beta = d + 3 * nscal;
    sc.rho_ref = d + 4 * nscal;
    sc.bnorm2 = d + 5 * nscal;
    sc.relres2 = d + 6 * nscal;
    sc.q = d + 7 * nscal;            // 2 * nscal
    sc.pp = d + 9 * nscal;
    sc.anorm = d + 10 * nscal;
    sc.xhn = d + 11 * nscal;
    sc.dev = d + 12 * nscal;
    int* iv = (int*)(d + 13 * nscal);
    sc.state = iv;
    sc.iters = iv + nscal;
    sc.restarts = iv + 2 * nscal;
    sc.ru = iv + 3 * nscal;
    sc.active = iv + 4 * nscal;
    sc.n_ru = sc.active + 1;
    sc.ru_count = sc.active + 2;
    sc.ru_lanes = nullptr;
    ran_dev = sc.active + 32;
    char* hb = (char*)h->host.p;
    h_q = (double*)hb;
    h_relres2 = h_q + 2 * nscal;
    h_state = (int*)(h_relres2 + nscal);
    h_iters = h_state + nscal;
    h_restarts = h_iters + nscal;
    h_active = h_restarts + nscal;   // [0] active, [2] reliable updates of the block
    h_ran = h_active + 32;

    od = h->dev(mixed);
    od64 = h->dev(false);
    // Algorithmic bytes of one stencil launch: per site, each link, coupling
    // and mass read once (shared by the B right-hand sides), p read and
    // w = A p written once per right-hand side.
    double per_site = 0.0;
    if (h->kind == TIP_KIND_COVARIANT) per_site += (double)g.ndim * 9 * 2 * (mixed ? 4 : 8);
    if (h->has_coupling) per_site += (double)g.ndim * 8;
    if (h->has_mass_field) per_site += 8.0;
    mv_bytes = per_site * V + 2.0 * (double)vbytes;
    if (pl.eo) {
      // the two half-lattice kernels of S p: each reads every link and
      // coupling once and D at its output sites; t_o = D_o^-1 H_oe p_e reads
      // p_e and writes t_o, S p reads t_o and p_e and writes w_e
      double link_site = 0.0;
      if (h->kind == TIP_KIND_COVARIANT) link_site += (double)g.ndim * 9 * 2 * (mixed ? 4 : 8);
      if (h->has_coupling) link_site += (double)g.ndim * 8;
      const double half = (double)vbytes / 2.0;
      hop_bytes = link_site * V + 4.0 * V + 2.0 * half;
      mv_bytes = link_site * V + 4.0 * V + 3.0 * half;
    }
    return TIP_OK;
  }

  // An FP64 even-odd pass (the operator's FP64 form) and the workgroups, that
  // is the partials per rhs, it writes.
  hipError_t eo_pass(int mode, int P, const int* state, const int* active, const void* in, const void* cin,
                     void* out, void* out2, void* out3, int64_t rhs0, int nb, double* partial,
                     const int* ru = nullptr, const void* cin2 = nullptr, void* out32 = nullptr) {
    const double* diag = (const double*)h->diag.p;
    if (pl.eo512)
      return launch_eo_hop512(mode, od64, geom, pl.me2, P, diag, state, active, in, cin, out, out2, out3, rhs0, nb,
                              p->seed, pl.mask, partial, nullptr, st, ru, cin2, out32, pstride);
    return launch_eo_hop(mode, od64, geom, pl.me, P, pl.elem, Prec::kF64, diag, state, active, in, cin, out, out2,
                         out3, rhs0, nb, p->seed, pl.mask, partial, nullptr, st, ru, cin2, out32, pstride);
  }
  int gx_eo() const { return pl.eo512 ? (int)pl.me2.grid : gx_m; }

  // Reliable updates of flagged right-hand sides (mode 0, enqueued after
  // every iteration; the kernels return at once when none is pending) or the
  // final check of frozen ones (mode 1) in the mixed solver.
  tip_status reliable(int64_t rhs0, int nb, int mode) {
    const Geom& g = geom;
    if (pl.eo) {
      const double* diag = (const double*)h->diag.p;
      TIP_HIP(launch_ru_accumulate(nvec, pl.logB, pl.elem, sc, mode, Xe, XH, st));
      if (mode == 0) {
        // r_e = b_hat - S x_e in FP64 for the flagged lanes (the kernels return
        // at once while no reliable update is pending: n_ru doubles as the
        // active counter)
        TIP_HIP(eo_pass(0, 1, sc.state, sc.n_ru, Xe, nullptr, T64, nullptr, nullptr, 0, 0, nullptr, sc.ru));
        TIP_HIP(eo_pass(4, 0, sc.state, sc.n_ru, T64, Xe, nullptr, nullptr, nullptr, 0, 0, part, sc.ru, Bh, Rv));
        TIP_HIP(launch_reduce_ru(sc, pl.B, part, gx_eo(), pstride, 0, tol2, max_iter, max_restarts, st));
        return TIP_OK;
      }
      // final check: the FP64 true residual b - A x in two half-lattice passes,
      // x_o = D_o^-1 (b_o + H_oe x_e) with the odd sites' part, then the even
      // sites' part (restart_residual stores r_e for lanes that fail)
      TIP_HIP(eo_pass(3, 1, nullptr, nullptr, Xe, nullptr, T64, need_x ? X : nullptr, nullptr, rhs0, nb, part));
      if (need_x) TIP_HIP(launch_eo_scatter_even(g, pl.elem, Prec::kF64, pl.logB, Xe, X, st));
      TIP_HIP(eo_pass(5, 0, nullptr, nullptr, T64, Xe, nullptr, nullptr, nullptr, rhs0, nb, part + 5 * pstride));
      TIP_HIP(launch_reduce_ru(sc, pl.B, part, gx_eo(), pstride, 1, tol2, max_iter, max_restarts, st,
                               part + 5 * pstride));
      return TIP_OK;
    }
    TIP_HIP(launch_ru_accumulate(nelem, pl.logB, pl.elem, sc, mode, X, XH, st));
    TIP_HIP(launch_ru_residual(od64, g, pl.tm, pl.elem, sc, mode, rhs0, nb, p->seed, pl.mask, X, Rv, Pv, part,
                               pstride, st));
    TIP_HIP(launch_reduce_ru(sc, pl.B, part, (int)ru_grid(pl.tm), pstride, mode, tol2, max_iter, max_restarts, st));
    return TIP_OK;
  }

  // Solve right-hand sides rhs0 .. rhs0+nb-1; x (FP64) stays in X.  Fills the
  // host mirrors h_q, h_relres2, h_state, h_iters for those nb right-hand sides.
  // One CG iteration of the block: w = A p (with p^H w), alpha, r -= alpha w
  // (with ||r||^2), beta, x += alpha p and p = r + beta p, then in mixed
  // precision any pending reliable update.  tv: events around the operator
  // application, or NULL.
  tip_status enqueue_iteration(int it, const Timed* tv, int64_t rhs0, int nb, void* xdir) {
    const Geom& g = geom;
    const MarchMap* mm = pl.use_march ? &pl.mm : nullptr;
    const double* diag = (const double*)h->diag.p;
    if (tv) TIP_HIP(hipEventRecord(tv->a, st));
    if (pl.pair) {
      TIP_HIP(launch_eo_hop_pair(0, od, g, pl.me2, 1, prec, diag, sc.state, sc.active, Pv, nullptr, Tv, nullptr,
                                 nullptr, st));
      if (tv) TIP_HIP(hipEventRecord(tv->b, st));
      TIP_HIP(launch_eo_hop_pair(1, od, g, pl.me2, 0, prec, diag, sc.state, sc.active, Tv, Pv, W, part, ran_dev + it,
                                 st));
    } else if (pl.wide) {
      TIP_HIP(launch_eo_hop_wide(0, od, g, pl.me2, 1, diag, sc.state, sc.active, Pv, nullptr, Tv, nullptr, nullptr,
                                 st));
      if (tv) TIP_HIP(hipEventRecord(tv->b, st));
      TIP_HIP(launch_eo_hop_wide(1, od, g, pl.me2, 0, diag, sc.state, sc.active, Tv, Pv, W, part, ran_dev + it, st));
    } else if (pl.eo) {
      // w_e = S p_e: t_o = D_o^-1 H_oe p_e, then w_e = D_e p_e - H_eo t_o
      TIP_HIP(launch_eo_hop(0, od, g, pl.me, 1, pl.elem, prec, diag, sc.state, sc.active, Pv, nullptr, Tv,
                            nullptr, nullptr, 0, 0, 0, 0, nullptr, nullptr, st));
      if (tv) TIP_HIP(hipEventRecord(tv->b, st));
      TIP_HIP(launch_eo_hop(1, od, g, pl.me, 0, pl.elem, prec, diag, sc.state, sc.active, Tv, Pv, W, nullptr,
                            nullptr, 0, 0, 0, 0, part, ran_dev + it, st));
    } else {
      if (tv) TIP_HIP(hipEventRecord(tv->b, st));
      TIP_HIP(launch_stencil(od, g, pl.tm, mm, pl.elem, prec, sc.state, sc.active, Pv, W, part, ran_dev + it,
                             st));
    }
    if (tv) TIP_HIP(hipEventRecord(tv->c, st));
    TIP_HIP(launch_reduce_alpha(sc, pl.B, part, gx_p, st, mixed ? 1 : 0, force_breakdown));
    TIP_HIP(launch_update_r(nvec, pl.logB, pl.elem, prec, sc, Rv, W, part + pstride, st));
    TIP_HIP(launch_reduce_beta(sc, pl.B, part + pstride, gx_u, tol2, max_iter, delta2, st, freeze2, ru_eps,
                               ru_tau2));
    TIP_HIP(launch_direction(nvec, pl.logB, pl.elem, prec, sc, xdir, Rv, Pv, st));
    if (mixed) {
      tip_status s = reliable(rhs0, nb, 0);
      if (s != TIP_OK) return s;
    }
    return TIP_OK;
  }

  // Chunks of CG iterations replayed as HIP graphs (kernel nodes only): one
  // graph per chunk length, captured on first use and replayed for every
  // later chunk of that length in this call.  The reset of the per-launch
  // flags stays outside the graph.  Eager launches instead: with profiling on
  // (per-kernel hipEvent timing needs events on the stream), in plain-CG
  // mixed precision (its reliable updates regenerate b, which ties a chunk to
  // its block), with TIP_GRAPH=0, and for the rest of the call after a failed
  // capture.
  struct GraphEntry {
    int chunk;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  bool graphs_ok = true;

  int graph_for(int chunk, int64_t rhs0, int nb, void* xdir) {
    if (!graphs_ok || g_profiling || (mixed && !pl.eo) || env_off("TIP_GRAPH")) return -1;
    for (size_t i = 0; i < graphs.size(); ++i)
      if (graphs[i].chunk == chunk) return (int)i;
    GraphEntry ge{chunk, nullptr};
    std::lock_guard<std::mutex> lk(g_device_mu);
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      graphs_ok = false;
      (void)hipGetLastError();
      return -1;
    }
    tip_status s = TIP_OK;
    for (int it = 0; it < chunk && s == TIP_OK; ++it)
      s = enqueue_iteration(it, nullptr, rhs0, nb, xdir);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    hipError_t ei = hipErrorUnknown;
    if (s == TIP_OK && e == hipSuccess && graph) ei = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      graphs_ok = false;
      (void)hipGetLastError();
      return -1;
    }
    graphs.push_back(ge);
    return (int)graphs.size() - 1;
  }

  ~Solver() {
    if (graphs.empty()) return;
    std::lock_guard<std::mutex> lk(g_device_mu);
    for (GraphEntry& ge : graphs)
      if (ge.exec) (void)hipGraphExecDestroy(ge.exec);
  }

  tip_status solve_block(int64_t rhs0, int nb) {
    const Geom& g = geom;
    TIP_HIP(launch_scalars_init(sc, nb, pl.B, (double)g.V, p->tol >= 1.0 ? 1 : 0, st));
    const double* diag = (const double*)h->diag.p;
    if (pl.eo && mixed) {
      // b_hat in FP64 (kept for the reliable updates), x_e = 0; r = p = single(b_hat), x_h = 0
      TIP_HIP(launch_eo_init_odd(g, pl.elem, Prec::kF64, pl.logB, rhs0, nb, p->seed, pl.mask, diag, T64, st));
      TIP_HIP(eo_pass(2, 0, nullptr, nullptr, T64, nullptr, Bh, nullptr, Xe, rhs0, nb, part));
      TIP_HIP(launch_reduce_rho0(sc, pl.B, part, gx_eo(), st));
      TIP_HIP(launch_eo_cast_init(nvec, pl.elem, Bh, Rv, Pv, XH, st));
    } else if (pl.eo) {
      // reduced right-hand side b_e + H_eo D_o^-1 b_o; x_e = 0, r = p = it
      TIP_HIP(launch_eo_init_odd(g, pl.elem, prec, pl.logB, rhs0, nb, p->seed, pl.mask, diag, Tv, st));
      TIP_HIP(eo_pass(2, 0, nullptr, nullptr, Tv, nullptr, Rv, Pv, Xe, rhs0, nb, part));
      TIP_HIP(launch_reduce_rho0(sc, pl.B, part, gx_eo(), st));
    } else if (mixed) {
      TIP_HIP(launch_init_mixed(g, pl.elem, pl.logB, rhs0, nb, p->seed, pl.mask, X, XH, Rv, Pv, st));
    } else {
      TIP_HIP(launch_init(g, pl.elem, pl.logB, rhs0, nb, p->seed, pl.mask, X, Rv, Pv, st));
    }
    void* xdir = mixed ? XH : (pl.eo ? Xe : X);     // vector the direction pass updates
    bool first_chunk = true;
    std::vector<Timed> window;
    for (;;) {
      // CG iterations, polled every `chunk` iterations; launches issued after
      // every rhs of the block stopped return at once (ran flag stays 0)
      for (;;) {
        const int chunk = first_chunk ? std::min(kMaxChunk, std::max(1, predicted - 1)) : 2;
        first_chunk = false;
        window.clear();
        ev_used = 0;
        TIP_HIP(hipMemsetAsync(ran_dev, 0, chunk * sizeof(int), st));
        const int gi = graph_for(chunk, rhs0, nb, xdir);
        if (gi >= 0) {
          TIP_HIP(hipGraphLaunch(graphs[(size_t)gi].exec, st));
        } else {
          for (int it = 0; it < chunk; ++it) {
            Timed tv{};
            if (g_profiling) {
              TIP_HIP(next_event(&tv.a));
              TIP_HIP(next_event(&tv.b));
              TIP_HIP(next_event(&tv.c));
              window.push_back(tv);
            }
            tip_status s = enqueue_iteration(it, g_profiling ? &tv : nullptr, rhs0, nb, xdir);
            if (s != TIP_OK) return s;
          }
        }
        TIP_HIP(hipMemcpyAsync(h_ran, ran_dev, chunk * sizeof(int), hipMemcpyDeviceToHost, st));
        TIP_HIP(hipMemcpyAsync(h_active, sc.active, sizeof(int), hipMemcpyDeviceToHost, st));
        TIP_HIP(hipStreamSynchronize(st));
        for (int i = 0; i < chunk; ++i) {
          if (!h_ran[i]) continue;
          ++stencil_launches;
          ++matvecs;
          stencil_bytes += mv_bytes;
          matvec_bytes += mv_bytes + hop_bytes;
          if (g_profiling) {
            float ms = 0.f, ms_all = 0.f;
            TIP_HIP(hipEventElapsedTime(&ms, window[i].b, window[i].c));
            TIP_HIP(hipEventElapsedTime(&ms_all, window[i].a, window[i].c));
            stencil_seconds += ms * 1e-3;
            matvec_seconds += ms_all * 1e-3;
          }
        }
        if (h_active[0] == 0) break;
      }
      // FP64 true residual: accept, or restart CG from x
      if (mixed) {
        tip_status s = reliable(rhs0, nb, 1);
        if (s != TIP_OK) return s;
      } else {
        if (pl.eo) {
          // the true residual b - A x in two half-lattice passes: x_o = D_o^-1
          // (b_o + H_oe x_e) with the odd sites' part, then the even sites'
          // part r_e = b_e - D_e x_e + H_eo x_o (the restart r = p for lanes
          // that fail); x on the full lattice only when the caller reads it
          TIP_HIP(eo_pass(3, 1, nullptr, nullptr, Xe, nullptr, Tv, need_x ? X : nullptr, nullptr, rhs0, nb, part));
          if (need_x) TIP_HIP(launch_eo_scatter_even(g, pl.elem, prec, pl.logB, Xe, X, st));
          TIP_HIP(eo_pass(5, 0, nullptr, nullptr, Tv, Xe, nullptr, nullptr, nullptr, rhs0, nb, part + 5 * pstride));
          TIP_HIP(launch_reduce_true(sc, pl.B, part, gx_eo(), pstride, tol2, max_iter, max_restarts, st,
                                     part + 5 * pstride));
        } else {
          TIP_HIP(launch_true_residual(od, g, pl.tm, pl.elem, sc.state, rhs0, nb, p->seed, pl.mask, X, Rv, Pv, part,
                                       pstride, st));
          TIP_HIP(launch_reduce_true(sc, pl.B, part, gx_t, pstride, tol2, max_iter, max_restarts, st));
        }
      }
      TIP_HIP(hipMemcpyAsync(h_active, sc.active, sizeof(int), hipMemcpyDeviceToHost, st));
      TIP_HIP(hipStreamSynchronize(st));
      if (h_active[0] == 0) break;
      if (pl.eo) {
        // some lanes failed the check and are active again: their CG restarts
        // from r = p = the reduced residual (the even sites' part of b - A x;
        // the x_o of the check is still in the t buffer)
        const double* diag = (const double*)h->diag.p;
        if (mixed)
          TIP_HIP(eo_pass(5, 0, sc.state, nullptr, T64, Xe, nullptr, nullptr, Pv, rhs0, nb, nullptr, nullptr, nullptr,
                          Rv));
        else
          TIP_HIP(eo_pass(5, 0, sc.state, nullptr, Tv, Xe, Rv, Pv, nullptr, rhs0, nb, nullptr));
      }
    }
    TIP_HIP(hipMemcpyAsync(h_q, sc.q, 2 * nb * sizeof(double), hipMemcpyDeviceToHost, st));
    TIP_HIP(hipMemcpyAsync(h_relres2, sc.relres2, nb * sizeof(double), hipMemcpyDeviceToHost, st));
    TIP_HIP(hipMemcpyAsync(h_state, sc.state, nb * sizeof(int), hipMemcpyDeviceToHost, st));
    TIP_HIP(hipMemcpyAsync(h_iters, sc.iters, nb * sizeof(int), hipMemcpyDeviceToHost, st));
    TIP_HIP(hipMemcpyAsync(h_restarts, sc.restarts, nb * sizeof(int), hipMemcpyDeviceToHost, st));
    TIP_HIP(hipMemcpyAsync(h_active + 2, sc.ru_count, sizeof(int), hipMemcpyDeviceToHost, st));
    TIP_HIP(hipStreamSynchronize(st));
    reliable_updates += h_active[2];
    for (int j = 0; j < nb; ++j) restarts += h_restarts[j];
    int blk_max = 0;
    for (int j = 0; j < nb; ++j) blk_max = std::max(blk_max, h_iters[j]);
    predicted = std::max(1, blk_max);
    return TIP_OK;
  }

  void fill_stats(tip_stats* stats) const {
    stats->stencil_launches = stencil_launches;
    stats->stencil_seconds = g_profiling ? stencil_seconds : 0.0;
    stats->stencil_bytes = stencil_bytes;
    stats->matvecs = matvecs;
    stats->matvec_seconds = g_profiling ? matvec_seconds : 0.0;
    stats->matvec_bytes = matvec_bytes;
    stats->even_odd = pl.eo ? 1 : 0;
    stats->reliable_updates = reliable_updates;
    stats->restarts = restarts;
  }
};

}  // namespace

extern "C" {

int32_t tip_num_checkpoints(int64_t n_vectors) { return num_checkpoints(n_vectors); }

const char* tip_last_error(void) { return g_err.c_str(); }

void tip_set_profiling(int32_t on) { g_profiling = on ? 1 : 0; }

tip_status tip_op_create(const tip_operator* op, void* stream, tip_op_handle* out) {
  if (!out) return fail(TIP_EINVAL, "out is NULL");
  tip_op_s* h = nullptr;
  tip_status s = create_handle(op, (hipStream_t)stream, &h);
  if (s == TIP_OK) *out = h;
  return s;
}

tip_status tip_op_destroy(tip_op_handle h) {
  if (!h) return fail(TIP_EINVAL, "handle is NULL");
  {
    std::lock_guard<std::mutex> lk(g_device_mu);
    (void)hipDeviceSynchronize();
  }
  delete h;
  return TIP_OK;
}

}  // extern "C"

namespace {

// Per-rhs results of one probing run: slot k = (m - m_begin) * ncomp + c for
// probe m and component c.
struct RunResult {
  std::vector<double> qre, qim, relres;
  std::vector<int> state, iters;
  std::vector<char> copied;        // quadrature taken from the conjugate partner, not solved
  tip_stats acc{};                 // stencil / matvec timing, reliable updates, restarts, even_odd
  explicit RunResult(int64_t n_rhs)
      : qre((size_t)n_rhs, 0.0), qim((size_t)n_rhs, 0.0), relres((size_t)n_rhs, 0.0),
        state((size_t)n_rhs, kPadding), iters((size_t)n_rhs, 0), copied((size_t)n_rhs, 0) {}
};

// Conjugate F_3 columns (Sec. 3.4, eq. Hperm-general-recursive): for a real
// operator and a real mask, probe column j3 = 2 of a sweep is the complex
// conjugate of column j3 = 1 (w^2 = conj w), so its quadrature is the
// conjugate of that one, and the j3 = 0 columns are real.  Then the j3 = 0
// probes are solved in real arithmetic, the j3 = 1 ones in complex, and the
// j3 = 2 ones take conj(q) of their partner probe m - 2^LB: half the work of
// complex solves for all of them.  Not with the gradient (it needs every x).
bool conj_split(const Geom& gg, int kind, int mask, const tip_params* p, bool want_grad) {
  const int64_t nb_cols = int64_t(1) << gg.LB;
  return gg.has3 && kind == TIP_KIND_SCALAR && (mask == TIP_MASK_Z2 || mask == TIP_MASK_NONE) &&
         p->probe == TIP_PROBE_HIERARCHICAL && !want_grad && p->n_vectors > nb_cols && !env_off("TIP_CONJ_SPLIT");
}

// The classes of the split: class j3 numbers its probes i = 0, 1, ...
// (class_probe); the members in [m_begin, n_vectors) have consecutive i.
struct ClassMap {
  int64_t gam, nbc;
  int64_t index(int64_t m, int j3) const { return (m / gam) * nbc + (m % gam - j3 * nbc); }
  int64_t first_member(int64_t m, int j3) const {      // smallest member >= m
    const int64_t r = m / gam, j = m % gam;
    if (j < j3 * nbc) return r * gam + j3 * nbc;
    if (j < (j3 + 1) * nbc) return m;
    return (r + 1) * gam + j3 * nbc;
  }
};

// The j3 = 2 probes of a split run: the conjugate of the partner's quadrature
// (and its state); from the earlier call's quadratures when the partner lies
// before m_begin.
void conj_copies(const Geom& gg, const tip_params* p, int ncomp, RunResult& rr) {
  const int64_t gam = (int64_t)gg.gamma, nb_cols = int64_t(1) << gg.LB;
  for (int64_t m = p->m_begin; m < p->n_vectors; ++m) {
    if ((m % gam) / nb_cols != 2) continue;
    for (int c = 0; c < ncomp; ++c) {
      const size_t k = (size_t)((m - p->m_begin) * ncomp + c);
      const int64_t mp = m - nb_cols;                   // same sweep, column j3 = 1
      rr.copied[k] = 1;
      if (mp < p->m_begin) {                              // from the earlier call's quadratures
        if (ncomp != 1) { rr.state[k] = kNoConv; continue; }
        rr.qre[k] = p->quadratures[2 * mp];
        rr.qim[k] = -p->quadratures[2 * mp + 1];
        rr.state[k] = kAccepted;
        continue;
      }
      const size_t kp = (size_t)((mp - p->m_begin) * ncomp + c);
      rr.qre[k] = rr.qre[kp];
      rr.qim[k] = -rr.qim[kp];
      rr.state[k] = rr.state[kp] == kPadding ? kNoConv : rr.state[kp];
      rr.relres[k] = rr.relres[kp];
    }
  }
}

// Quadratures per probe, compensated sums into the estimates at s = 2^k,
// stats, and the status of the first probe (in probe order) that was not
// accepted.
tip_status finish_run(const tip_op_s* h, const tip_params* p, const RunResult& rr, double* estimates,
                      tip_stats* stats, std::chrono::steady_clock::time_point t_start) {
  const int ncomp = h->geom.ncomp;
  const int64_t probes = p->n_vectors - p->m_begin;
  const int64_t n_rhs = probes * ncomp;
  int64_t first_bad_rhs = -1;
  tip_status bad_status = TIP_OK;
  for (int64_t k = 0; k < n_rhs; ++k)
    if (rr.state[(size_t)k] != kAccepted) {
      first_bad_rhs = k;
      bad_status = rr.state[(size_t)k] == kBreakdown ? TIP_EBREAKDOWN : TIP_ENOCONV;
      break;
    }
  const int64_t n = p->n_vectors;
  const int64_t good_probes = first_bad_rhs < 0 ? probes : first_bad_rhs / ncomp;
  const int64_t m_end = p->m_begin + good_probes;      // probes [0, m_end) are valid
  std::vector<double> q_all_re((size_t)m_end), q_all_im((size_t)m_end);
  for (int64_t m = 0; m < p->m_begin; ++m) {
    q_all_re[m] = p->quadratures[2 * m];
    q_all_im[m] = p->quadratures[2 * m + 1];
  }
  for (int64_t m = p->m_begin; m < m_end; ++m) {
    double re = 0.0, im = 0.0;
    for (int c = 0; c < ncomp; ++c) {
      re += rr.qre[(size_t)((m - p->m_begin) * ncomp + c)];
      im += rr.qim[(size_t)((m - p->m_begin) * ncomp + c)];
    }
    q_all_re[m] = re;
    q_all_im[m] = im;
  }
  if (p->quadratures)
    for (int64_t m = p->m_begin; m < m_end; ++m) {
      p->quadratures[2 * m] = q_all_re[m];
      p->quadratures[2 * m + 1] = q_all_im[m];
    }
  if (p->residuals)
    for (int64_t k = 0; k < n_rhs; ++k)
      p->residuals[p->m_begin * ncomp + k] = rr.state[(size_t)k] == kAccepted ? rr.relres[(size_t)k] : std::nan("");
  const int nck = num_checkpoints(n);
  int done = 0;
  {
    Compensated sre, sim;
    int64_t m = 0;
    for (int k = 0; k < nck; ++k) {
      const int64_t sz = checkpoint_size(n, k);
      if (sz > m_end) break;
      for (; m < sz; ++m) {
        sre.add(q_all_re[m]);
        sim.add(q_all_im[m]);
      }
      estimates[2 * k] = sre.value() / (double)sz;
      estimates[2 * k + 1] = sim.value() / (double)sz;
      done = k + 1;
    }
  }
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    double mx_rr = 0.0;
    int64_t tot = 0;
    int mx_it = 0, solved = 0;
    for (int64_t k = 0; k < n_rhs; ++k) {
      if (rr.state[k] == kPadding || rr.copied[(size_t)k]) continue;
      ++solved;
      tot += rr.iters[k];
      mx_it = std::max(mx_it, rr.iters[k]);
      if (rr.state[k] == kAccepted) mx_rr = std::max(mx_rr, rr.relres[k]);
    }
    stats->solves = solved;
    stats->total_iters = tot;
    stats->max_iters = mx_it;
    stats->n_checkpoints_done = done;
    stats->max_true_relres = mx_rr;
    // error of one quadrature: r^H A^-1 r <= ||r||^2 / lambda_min, ||b||^2 = V
    stats->max_quad_err_bound = mx_rr * mx_rr * (double)h->geom.V / h->lambda_lb;
    stats->stencil_launches = rr.acc.stencil_launches;
    stats->stencil_seconds = rr.acc.stencil_seconds;
    stats->stencil_bytes = rr.acc.stencil_bytes;
    stats->matvecs = rr.acc.matvecs;
    stats->matvec_seconds = rr.acc.matvec_seconds;
    stats->matvec_bytes = rr.acc.matvec_bytes;
    stats->reliable_updates = rr.acc.reliable_updates;
    stats->restarts = rr.acc.restarts;
    stats->even_odd = rr.acc.even_odd;
    int64_t reused = 0;
    for (char c : rr.copied) reused += c ? 1 : 0;
    stats->reused = reused;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  }
  if (first_bad_rhs >= 0) {
    const int64_t bad_m = p->m_begin + first_bad_rhs / ncomp;
    return fail(bad_status, "solve of probe %lld component %d %s", (long long)bad_m, (int)(first_bad_rhs % ncomp),
                bad_status == TIP_EBREAKDOWN ? "broke down (p^H A p <= 0)" : "did not converge within max_iter");
  }
  return TIP_OK;
}

// The probing run behind trace_inv_probe_op and trace_inv_probe_grad; grad_mass
// and grad_coupling (device, or NULL) receive the gradient of the estimate at
// s = n_vectors, accumulated block by block from the solutions in the workspace.
tip_status run_probe(tip_op_handle h, const tip_params* p, double* estimates, double* grad_mass,
                     double* grad_coupling, tip_stats* stats) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!h) return fail(TIP_EINVAL, "handle is NULL");
  if (!estimates) return fail(TIP_EINVAL, "estimates is NULL");
  int mask = 0;
  tip_status s = check_params(h, p, &mask);
  if (s != TIP_OK) return s;
  if (p->m_begin > 0 && !p->quadratures) return fail(TIP_EINVAL, "m_begin > 0 needs the earlier quadratures");
  const bool want_grad = grad_mass || grad_coupling;
  if (want_grad && p->m_begin != 0) return fail(TIP_EINVAL, "the gradient needs every solve: m_begin must be 0");
  const int ncomp = h->geom.ncomp;
  const int64_t probes = p->n_vectors - p->m_begin;
  const int64_t n_rhs = probes * ncomp;
  const Geom& gg = h->geom;
  const size_t V = gg.V;
  RunResult rr(n_rhs);
  bool failed = false;
  hipStream_t st_used = nullptr;
  // Solve right-hand sides [r0, r1) in blocks: rhs r (lane rhs of the kernels)
  // is result slot slot(r); stops at the first block holding a failed solve.
  auto run_range = [&](Solver& sv, int64_t r0, int64_t r1, auto slot) -> tip_status {
    for (int64_t blk0 = r0; blk0 < r1 && !failed; blk0 += sv.pl.B) {
      const int nb = (int)std::min<int64_t>(sv.pl.B, r1 - blk0);
      tip_status s2 = sv.solve_block(blk0, nb);
      if (s2 != TIP_OK) return s2;
      if (want_grad)
        TIP_HIP(launch_grad_accum(sv.od64, gg, sv.pl.elem, sv.pl.logB, nb, sv.X, grad_mass, grad_coupling, sv.st));
      for (int j = 0; j < nb; ++j) {
        const size_t k = slot(blk0 + j);
        rr.qre[k] = sv.h_q[2 * j];
        rr.qim[k] = sv.h_q[2 * j + 1];
        rr.state[k] = sv.h_state[j];
        rr.iters[k] = sv.h_iters[j];
        rr.relres[k] = std::sqrt(sv.h_relres2[j]);
        if (sv.h_state[j] != kAccepted) failed = true;
      }
    }
    return TIP_OK;
  };
  auto add_stats = [&](const Solver& sv) {
    tip_stats t;
    std::memset(&t, 0, sizeof t);
    sv.fill_stats(&t);
    rr.acc.stencil_launches += t.stencil_launches;
    rr.acc.stencil_seconds += t.stencil_seconds;
    rr.acc.stencil_bytes += t.stencil_bytes;
    rr.acc.matvecs += t.matvecs;
    rr.acc.matvec_seconds += t.matvec_seconds;
    rr.acc.matvec_bytes += t.matvec_bytes;
    rr.acc.reliable_updates += t.reliable_updates;
    rr.acc.restarts += t.restarts;
    rr.acc.even_odd = rr.acc.even_odd || t.even_odd;
  };
  if (!conj_split(gg, h->kind, mask, p, want_grad)) {
    Solver sv;
    sv.need_x = want_grad;
    s = sv.setup(h, p, mask);
    if (s != TIP_OK) return s;
    st_used = sv.st;
    if (grad_mass) TIP_HIP(launch_fill(V, grad_mass, 0.0, sv.st));
    if (grad_coupling) TIP_HIP(launch_fill((size_t)gg.ndim * V, grad_coupling, 0.0, sv.st));
    const int64_t base = p->m_begin * ncomp;
    s = run_range(sv, base, base + n_rhs, [&](int64_t r) { return (size_t)(r - base); });
    if (s != TIP_OK) return s;
    add_stats(sv);
  } else {
    const ClassMap cm{(int64_t)gg.gamma, int64_t(1) << gg.LB};
    // each class runs up to its own first failure; the checkpoints then stop
    // at the first probe, in probe order, that is not accepted
    for (int pass = 0; pass < 2; ++pass) {
      failed = false;
      const int64_t m0 = cm.first_member(p->m_begin, pass);
      if (m0 >= p->n_vectors) continue;
      const int64_t i0 = cm.index(m0, pass);
      const int64_t i1 = cm.index(cm.first_member(p->n_vectors, pass), pass);   // one past the last member
      Solver sv;
      sv.force_elem = pass;          // j3 = 0: real, j3 = 1: complex
      sv.rhs_hint = (i1 - i0) * ncomp;
      s = sv.setup(h, p, mask);
      if (s != TIP_OK) return s;
      sv.geom.cls_gamma = (int32_t)cm.gam;
      sv.geom.cls_nbc = (int32_t)cm.nbc;
      sv.geom.cls_j3 = pass;
      st_used = sv.st;
      s = run_range(sv, i0 * ncomp, i1 * ncomp, [&](int64_t r) {
        const int64_t m = (int64_t)class_probe((uint64_t)(r / ncomp), sv.geom);
        return (size_t)((m - p->m_begin) * ncomp + r % ncomp);
      });
      if (s != TIP_OK) return s;
      add_stats(sv);
    }
    conj_copies(gg, p, ncomp, rr);
  }
  s = finish_run(h, p, rr, estimates, stats, t_start);
  if (s == TIP_OK && want_grad) {
    const double f = -1.0 / (double)p->n_vectors;
    if (grad_mass) TIP_HIP(launch_scale(V, grad_mass, f, st_used));
    if (grad_coupling) TIP_HIP(launch_scale((size_t)gg.ndim * V, grad_coupling, f, st_used));
    TIP_HIP(hipStreamSynchronize(st_used));
  }
  return s;
}

// ---------------------------------------------------------------------------
// Many independent problems solved together (trace_inv_probe_batch).
//
// Every problem's right-hand sides are cut into blocks (jobs) exactly as a
// single call would solve them (probe classes of the conjugate F_3 split
// included), and all jobs of one (operator kind, element type, precision)
// group advance together: each CG phase is one launch over the work items
// of every job of the group (tip_batch.hip), and one chunk of iterations for
// the whole batch is captured once as a HIP graph and replayed.  One host
// thread does all of it (each group's chain on a side stream inside the
// captured chunk); the host polls one counter per chunk.
// ---------------------------------------------------------------------------

struct HandleDel {
  void operator()(tip_op_s* h) const { delete h; }
};

// Batch arguments valid for every problem (estimates may be NULL when only
// the parameters are checked).
tip_status validate_batch(const tip_operator* ops, const tip_params* params, int32_t count, double* const* estimates) {
  if (count < 0) return fail(TIP_EINVAL, "count = %d must be >= 0", count);
  if (count > 0 && (!ops || !params)) return fail(TIP_EINVAL, "ops or params is NULL");
  for (int32_t i = 0; i < count; ++i) {
    Geom g;
    tip_status s = validate_op(&ops[i], &g);
    if (s != TIP_OK) return fail(s, "torus %d: %s", i, g_err.c_str());
    if (estimates && !estimates[i]) return fail(TIP_EINVAL, "torus %d: estimates is NULL", i);
    if (params[i].n_vectors < 1 || params[i].n_vectors > (int64_t)g.V)
      return fail(TIP_EINVAL, "torus %d: n_vectors = %lld must be in [1, V = %u]", i,
                  (long long)params[i].n_vectors, g.V);
    if (params[i].m_begin > 0 && !params[i].quadratures)
      return fail(TIP_EINVAL, "torus %d: m_begin > 0 needs the earlier quadratures", i);
    if (params[i].item_sites < 0) return fail(TIP_EINVAL, "torus %d: item_sites must be >= 0", i);
  }
  return TIP_OK;
}

// A range of right-hand sides of one problem solved in one element type.
struct BatchClass {
  int prob;
  int j3;                      // F_3 class of the conjugate split, -1 for none
  Elem elem;
  Prec prec;
  int64_t r0, r1;              // right-hand sides (class-local with a class)
  int B;
};

constexpr int kBatchChunk = 8;              // CG iterations per poll of the active counter
constexpr int kBatchItemSites = 512;        // default sites per work item

tip_status run_batch(const tip_operator* ops, const tip_params* params, int32_t count, double* const* estimates,
                     tip_stats* stats, int32_t* statuses, const tip_tuning* tune) {
  const auto t_start = std::chrono::steady_clock::now();
  // one stream for the whole batch: the first problem's, or one of the call's own
  hipStream_t st = (hipStream_t)params[0].stream;
  struct OwnStream {
    hipStream_t s = nullptr;
    ~OwnStream() {
      if (!s) return;
      std::lock_guard<std::mutex> lk(g_device_mu);
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  } own;
  if (!st) {
    {
      std::lock_guard<std::mutex> lk(g_device_mu);
      if (hipStreamCreateWithFlags(&own.s, hipStreamNonBlocking) != hipSuccess)
        return fail(TIP_EDEVICE, "hipStreamCreateWithFlags failed");
    }
    TIP_HIP(hipStreamSynchronize(nullptr));        // work queued on the null stream comes first
    st = own.s;
  }
  // operators: link repack, diagonal, lower spectral bound; the call's masks
  std::vector<std::unique_ptr<tip_op_s, HandleDel>> hs((size_t)count);
  std::vector<int> masks((size_t)count);
  for (int32_t i = 0; i < count; ++i) {
    tip_op_s* h = nullptr;
    tip_status s = create_handle(&ops[i], st, &h);
    if (s != TIP_OK) return fail(s, "torus %d: %s", i, g_err.c_str());
    hs[(size_t)i].reset(h);
    s = check_params(h, &params[i], &masks[(size_t)i]);
    if (s != TIP_OK) return fail(s, "torus %d: %s", i, g_err.c_str());
    if (params[i].precision == TIP_PREC_MIXED && h->kind == TIP_KIND_COVARIANT && !h->has_links32) {
      const size_t n = (size_t)h->geom.ndim * 9 * h->geom.V;
      if (const hipError_t e_ = h->links32.ensure(n * sizeof(float2)); e_ != hipSuccess)
        return fail(TIP_ENOMEM, "torus %d: hipMalloc FP32 links: %s", i, hipGetErrorString(e_));
      TIP_HIP(launch_cast_links(n, (const double2*)h->links.p, (float2*)h->links32.p, st));
      h->has_links32 = true;
    }
  }
  // classes of right-hand sides
  std::vector<BatchClass> classes;
  for (int32_t i = 0; i < count; ++i) {
    const tip_op_s* h = hs[(size_t)i].get();
    const tip_params& p = params[i];
    const Geom& g = h->geom;
    const int ncomp = g.ncomp;
    const Prec prec = p.precision == TIP_PREC_MIXED ? Prec::kF32 : Prec::kF64;
    const int rb = tune ? tune->rhs_block : p.rhs_block;
    auto pick_b = [&](int64_t nrhs) {
      int b = 1;
      if (rb > 0) {
        while (b < rb && b < 64) b *= 2;
      } else {
        b = 32;
      }
      while (b > 1 && b / 2 >= nrhs) b /= 2;
      return b;
    };
    if (conj_split(g, h->kind, masks[(size_t)i], &p, false)) {
      const ClassMap cm{(int64_t)g.gamma, int64_t(1) << g.LB};
      for (int pass = 0; pass < 2; ++pass) {
        const int64_t m0 = cm.first_member(p.m_begin, pass);
        if (m0 >= p.n_vectors) continue;
        const int64_t i0 = cm.index(m0, pass), i1 = cm.index(cm.first_member(p.n_vectors, pass), pass);
        classes.push_back({i, pass, pass ? Elem::kComplex : Elem::kReal, prec, i0 * ncomp, i1 * ncomp,
                           pick_b((i1 - i0) * ncomp)});
      }
    } else {
      const bool f3 = g.has3 && p.n_vectors > (int64_t(1) << g.LB);
      const bool cplx = h->kind == TIP_KIND_COVARIANT || masks[(size_t)i] == TIP_MASK_Z4 || f3 ||
                        p.probe == TIP_PROBE_FOURIER;
      if (p.n_vectors > p.m_begin)
        classes.push_back({i, -1, cplx ? Elem::kComplex : Elem::kReal, prec, p.m_begin * ncomp, p.n_vectors * ncomp,
                           pick_b((p.n_vectors - p.m_begin) * ncomp)});
    }
  }
  // groups and jobs; work items of item_sites sites
  int item_sites = tune && tune->item_sites > 0 ? tune->item_sites
                   : params[0].item_sites > 0   ? params[0].item_sites
                                                : kBatchItemSites;
  if (const char* e = std::getenv("TIP_BATCH_ITEM")) item_sites = std::max(1, std::atoi(e));   // experiments
  {
    int v = 256;
    while (v < item_sites && v < (1 << 20)) v *= 2;
    item_sites = v;                              // a power of two >= 256: whole tiles for every B
  }
  std::vector<int> order(classes.size());
  for (size_t c = 0; c < classes.size(); ++c) order[c] = (int)c;
  auto key = [&](const BatchClass& c) {
    return hs[(size_t)c.prob]->kind * 4 + (c.elem == Elem::kComplex ? 2 : 0) + (c.prec == Prec::kF32 ? 1 : 0);
  };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key(classes[x]) < key(classes[y]); });
  std::vector<BatchJob> jobs;
  std::vector<int> job_class;
  std::vector<uint32_t> item_job;
  std::vector<int32_t> lane_job;
  std::vector<BatchGroup> groups;
  std::vector<size_t> group_elems;
  size_t PI = 1;
  for (size_t oi = 0; oi < order.size();) {
    const BatchClass& c0 = classes[(size_t)order[oi]];
    BatchGroup gr{hs[(size_t)c0.prob]->kind, c0.elem, c0.prec, (uint32_t)item_job.size(), 0, (int)lane_job.size(), 0,
                  hs[(size_t)c0.prob]->geom.ndim, 6};
    uint64_t off = 0;
    for (; oi < order.size() && key(classes[(size_t)order[oi]]) == key(c0); ++oi) {
      const BatchClass& c = classes[(size_t)order[oi]];
      const tip_op_s* h = hs[(size_t)c.prob].get();
      const tip_params& p = params[c.prob];
      if (h->geom.ndim != gr.ndim) gr.ndim = 0;
      Geom gj = h->geom;
      gj.probe = p.probe;
      gj.stop = p.stop_levels;
      gj.cls_gamma = c.j3 >= 0 ? (int32_t)gj.gamma : 0;
      gj.cls_nbc = c.j3 >= 0 ? (int32_t)(1u << gj.LB) : 0;
      gj.cls_j3 = c.j3 >= 0 ? c.j3 : 0;
      int logB = 0;
      while ((1 << logB) < c.B) ++logB;
      gr.min_logB = std::min(gr.min_logB, logB);
      const uint32_t nitems = (uint32_t)((gj.V + (uint32_t)item_sites - 1) / (uint32_t)item_sites);
      PI = std::max<size_t>(PI, nitems);
      const bool single = c.prec == Prec::kF32;
      uint32_t site_bytes = 0;
      if (h->kind == TIP_KIND_COVARIANT) site_bytes += (uint32_t)gj.ndim * 9 * 2 * (single ? 4 : 8);
      if (h->has_coupling) site_bytes += (uint32_t)gj.ndim * 8;
      if (h->has_mass_field) site_bytes += 8;
      const uint32_t esz = (c.elem == Elem::kComplex ? 2u : 1u) * (single ? 4u : 8u);
      for (int64_t blk0 = c.r0; blk0 < c.r1; blk0 += c.B) {
        BatchJob J{};
        J.g = gj;
        J.prob = c.prob;
        J.logB = logB;
        J.nb = (int32_t)std::min<int64_t>(c.B, c.r1 - blk0);
        J.rhs0 = blk0;
        J.item0 = (uint32_t)item_job.size();
        J.nitems = nitems;
        J.lane0 = (int32_t)lane_job.size();
        J.site_bytes = site_bytes;
        J.esz = esz;
        J.off = off;
        const uint32_t jidx = (uint32_t)jobs.size();
        jobs.push_back(J);
        job_class.push_back(order[oi]);
        item_job.insert(item_job.end(), nitems, jidx);
        lane_job.insert(lane_job.end(), (size_t)c.B, (int32_t)jidx);
        off += (uint64_t)gj.ncomp * gj.V * (uint64_t)c.B;
      }
    }
    gr.nitems = (uint32_t)item_job.size() - gr.item_base;
    gr.nlanes = (int)lane_job.size() - gr.lane_base;
    groups.push_back(gr);
    group_elems.push_back(off);
  }
  const int L = (int)lane_job.size();
  std::vector<RunResult> results;
  results.reserve((size_t)count);
  for (int32_t i = 0; i < count; ++i)
    results.emplace_back((params[i].n_vectors - params[i].m_begin) * hs[(size_t)i]->geom.ncomp);
  if (L > 0) {
    // device memory: per group x (FP64) and r, p, w (and x_h in mixed precision)
    // in the working precision; 6 partial rows; the CG scalars; the tables
    auto al = [](size_t n) { return (n + 255) & ~size_t(255); };
    struct GroupVec { size_t x, xh, r, p, w; };
    std::vector<GroupVec> gv(groups.size());
    size_t vec_bytes = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      const size_t e64 = groups[gi].elem == Elem::kComplex ? 16 : 8;
      const size_t ew = groups[gi].prec == Prec::kF32 ? e64 / 2 : e64;
      const size_t n = group_elems[gi];
      gv[gi].x = vec_bytes;
      vec_bytes += al(n * e64);
      gv[gi].xh = vec_bytes;
      if (groups[gi].prec == Prec::kF32) vec_bytes += al(n * ew);
      gv[gi].r = vec_bytes;
      vec_bytes += al(n * ew);
      gv[gi].p = vec_bytes;
      vec_bytes += al(n * ew);
      gv[gi].w = vec_bytes;
      vec_bytes += al(n * ew);
    }
    const size_t rowstride = (size_t)L * PI;
    DevBuf vec, part, scal, tab;
    if (const hipError_t e_ = vec.ensure(vec_bytes); e_ != hipSuccess)
      return fail(TIP_ENOMEM, "hipMalloc of %zu bytes of batch vectors failed: %s", vec_bytes, hipGetErrorString(e_));
    if (const hipError_t e_ = part.ensure(6 * rowstride * sizeof(double)); e_ != hipSuccess)
      return fail(TIP_ENOMEM, "hipMalloc batch partials: %s", hipGetErrorString(e_));
    const size_t scal_bytes = (size_t)L * (13 * sizeof(double) + 5 * sizeof(int)) + 256;
    if (const hipError_t e_ = scal.ensure(scal_bytes); e_ != hipSuccess)
      return fail(TIP_ENOMEM, "hipMalloc batch scalars: %s", hipGetErrorString(e_));
    std::vector<BatchProb> probs((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
      const tip_op_s* h = hs[(size_t)i].get();
      BatchProb& P = probs[(size_t)i];
      P.mass_field = h->has_mass_field ? (const double*)h->mass_field.p : nullptr;
      P.mass = h->mass;
      P.coupling = h->has_coupling ? (const double*)h->coupling.p : nullptr;
      P.links = h->kind == TIP_KIND_COVARIANT ? h->links.p : nullptr;
      P.links32 = h->has_links32 ? h->links32.p : nullptr;
      P.seed = params[i].seed;
      P.mask = masks[(size_t)i];
      P.max_iter = params[i].max_iter > 0 ? params[i].max_iter
                                          : (int)std::min<int64_t>(10 * (int64_t)h->geom.V * h->geom.ncomp, 1 << 20);
      P.tol2 = params[i].tol * params[i].tol;
    }
    const size_t t_jobs = 0, t_probs = al(jobs.size() * sizeof(BatchJob));
    const size_t t_items = t_probs + al(probs.size() * sizeof(BatchProb));
    const size_t t_lanes = t_items + al(item_job.size() * sizeof(uint32_t));
    const size_t t_bytes = t_lanes + al(lane_job.size() * sizeof(int32_t));
    if (const hipError_t e_ = tab.ensure(t_bytes + 256); e_ != hipSuccess)
      return fail(TIP_ENOMEM, "hipMalloc batch tables: %s", hipGetErrorString(e_));
    char* tb = (char*)tab.p;
    TIP_HIP(hipMemcpyAsync(tb + t_jobs, jobs.data(), jobs.size() * sizeof(BatchJob), hipMemcpyHostToDevice, st));
    TIP_HIP(hipMemcpyAsync(tb + t_probs, probs.data(), probs.size() * sizeof(BatchProb), hipMemcpyHostToDevice, st));
    TIP_HIP(hipMemcpyAsync(tb + t_items, item_job.data(), item_job.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                           st));
    TIP_HIP(hipMemcpyAsync(tb + t_lanes, lane_job.data(), lane_job.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                           st));
    BatchArgs args{};
    args.jobs = (const BatchJob*)(tb + t_jobs);
    args.probs = (const BatchProb*)(tb + t_probs);
    args.item_job = (const uint32_t*)(tb + t_items);
    args.lane_job = (const int32_t*)(tb + t_lanes);
    args.item_sites = item_sites;
    args.PI = PI;
    // kb_stencil: slices in bands of item_sites / TS and each job's items in
    // one contiguous part per XCD; together they halve the stencil's fetched
    // bytes on the 64 uneven tori (its time falls by about 2%)
    args.march = 3;
    if (const char* e = std::getenv("TIP_BATCH_MARCH")) args.march = std::atoi(e) & 3;   // experiments
    args.bytes = g_profiling ? (unsigned long long*)(tb + t_bytes) : nullptr;
    CgScalars sc{};
    double* d = (double*)scal.p;
    sc.rho = d;
    sc.alpha = d + L;
    sc.xalpha = d + 2 * (size_t)L;
    sc.beta = d + 3 * (size_t)L;
    sc.rho_ref = d + 4 * (size_t)L;
    sc.bnorm2 = d + 5 * (size_t)L;
    sc.relres2 = d + 6 * (size_t)L;
    sc.q = d + 7 * (size_t)L;                      // 2 L
    sc.pp = d + 9 * (size_t)L;
    sc.anorm = d + 10 * (size_t)L;
    sc.xhn = d + 11 * (size_t)L;
    sc.dev = d + 12 * (size_t)L;
    int* iv = (int*)(d + 13 * (size_t)L);
    sc.state = iv;
    sc.iters = iv + L;
    sc.restarts = iv + 2 * (size_t)L;
    sc.ru = iv + 3 * (size_t)L;
    sc.ru_lanes = iv + 4 * (size_t)L;
    sc.active = iv + 5 * (size_t)L;
    sc.n_ru = sc.active + 1;
    sc.ru_count = sc.active + 2;
    TIP_HIP(hipMemsetAsync(sc.ru_lanes, 0, (size_t)L * sizeof(int) + 64, st));
    if (args.bytes) TIP_HIP(hipMemsetAsync(args.bytes, 0, sizeof(unsigned long long), st));
    int live_lanes = 0;
    for (const BatchJob& J : jobs) live_lanes += J.nb;
    HostPinned host;
    if (const hipError_t e_ = host.ensure((size_t)L * (3 * sizeof(double) + 4 * sizeof(int)) + 256); e_ != hipSuccess)
      return fail(TIP_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e_));
    int* h_active = (int*)host.p;
    h_active[0] = live_lanes;
    TIP_HIP(launch_batch_scalars_init(args, sc, L, st));
    TIP_HIP(hipMemcpyAsync(sc.active, h_active, sizeof(int), hipMemcpyHostToDevice, st));
    char* vb = (char*)vec.p;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      BatchArgs ga = args;
      ga.item_base = groups[gi].item_base;
      const bool mixed = groups[gi].prec == Prec::kF32;
      TIP_HIP(launch_batch_init(ga, groups[gi], vb + gv[gi].x, mixed ? vb + gv[gi].xh : nullptr, vb + gv[gi].r,
                                vb + gv[gi].p, st));
    }
    double* pt = (double*)part.p;
    // residual replacement in single precision: the constants of the single-problem solver
    const double eps32 = 0x1p-24, tau2 = 0x1p-10;
    int64_t stencil_launches = 0;
    double stencil_seconds = 0.0;
    std::vector<hipEvent_t> evs;
    // In a captured chunk each group's iterations form a chain of their own,
    // forked from the capturing stream onto a side stream and joined back, so
    // the groups' launches overlap: the groups share no vector, partial entry
    // or CG scalar (lanes are disjoint), and the counters they share (active
    // lanes, pending reliable updates) are updated atomically and only gate
    // early exits.  Eager chunks stay on the one stream.
    struct SideStreams {
      std::vector<hipStream_t> s;              // only ever captured into: no work runs on them
      std::vector<hipEvent_t> e;               // [0] fork, then one join per side stream
      ~SideStreams() {
        if (s.empty() && e.empty()) return;
        std::lock_guard<std::mutex> lk(g_device_mu);
        for (hipStream_t x : s) (void)hipStreamDestroy(x);
        for (hipEvent_t x : e) (void)hipEventDestroy(x);
      }
    } side;
    auto stream_of = [&](size_t gi, bool captured) {
      return captured && gi > 0 && !side.s.empty() ? side.s[(gi - 1) % side.s.size()] : st;
    };
    auto enqueue_chunk = [&](int chunk, bool timed, bool captured) -> tip_status {
      for (int it = 0; it < chunk; ++it)
        for (size_t gi = 0; gi < groups.size(); ++gi) {
          const hipStream_t sg = stream_of(gi, captured);
          BatchArgs ga = args;
          ga.item_base = groups[gi].item_base;
          const bool mixed = groups[gi].prec == Prec::kF32;
          hipEvent_t e0 = nullptr, e1 = nullptr;
          if (timed) {
            TIP_HIP(hipEventCreate(&e0));
            evs.push_back(e0);
            TIP_HIP(hipEventCreate(&e1));
            evs.push_back(e1);
          }
          TIP_HIP(launch_batch_iteration(ga, groups[gi], sc, vb + (mixed ? gv[gi].xh : gv[gi].x), vb + gv[gi].r,
                                         vb + gv[gi].p, vb + gv[gi].w, pt, rowstride, mixed ? eps32 : 0.0,
                                         mixed ? tau2 : 0.0, sg, e0, e1));
          if (mixed)
            TIP_HIP(launch_batch_reliable(ga, groups[gi], sc, 0, vb + gv[gi].x, vb + gv[gi].xh, vb + gv[gi].r,
                                          vb + gv[gi].p, pt + rowstride, rowstride, sg));
        }
      return TIP_OK;
    };
    auto enqueue_captured_chunk = [&](int chunk) -> tip_status {
      if (side.s.empty()) return enqueue_chunk(chunk, false, false);
      TIP_HIP(hipEventRecord(side.e[0], st));
      for (hipStream_t x : side.s) TIP_HIP(hipStreamWaitEvent(x, side.e[0], 0));
      const tip_status cs = enqueue_chunk(chunk, false, true);
      for (size_t k = 0; k < side.s.size(); ++k) {  // join every side stream, also after a failed launch
        TIP_HIP(hipEventRecord(side.e[k + 1], side.s[k]));
        TIP_HIP(hipStreamWaitEvent(st, side.e[k + 1], 0));
      }
      return cs;
    };
    // chunks of iterations replayed as one HIP graph for the whole batch
    hipGraphExec_t graph = nullptr;
    struct GraphDel {
      hipGraphExec_t* g;
      ~GraphDel() {
        if (*g) (void)hipGraphExecDestroy(*g);
      }
    } graph_del{&graph};
    bool use_graph = !g_profiling && !env_off("TIP_GRAPH");
    if (use_graph && groups.size() > 1 && !env_off("TIP_BATCH_FORK")) {
      std::lock_guard<std::mutex> lk(g_device_mu);
      const size_t ns = std::min<size_t>(groups.size() - 1, 3);
      for (size_t k = 0; k < ns; ++k) {
        hipStream_t x = nullptr;
        if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) break;
        side.s.push_back(x);
      }
      for (size_t k = 0; k <= side.s.size(); ++k) {
        hipEvent_t x = nullptr;
        if (hipEventCreateWithFlags(&x, hipEventDisableTiming) != hipSuccess) break;
        side.e.push_back(x);
      }
      if (side.e.size() != side.s.size() + 1 || side.s.empty()) {    // fall back to one chain
        for (hipStream_t x : side.s) (void)hipStreamDestroy(x);
        for (hipEvent_t x : side.e) (void)hipEventDestroy(x);
        side.s.clear();
        side.e.clear();
        (void)hipGetLastError();
      }
    }
    auto poll = [&]() -> tip_status {
      TIP_HIP(hipMemcpyAsync(h_active, sc.active, sizeof(int), hipMemcpyDeviceToHost, st));
      TIP_HIP(hipStreamSynchronize(st));
      return TIP_OK;
    };
    for (;;) {
      for (;;) {
        if (use_graph && !graph) {
          std::lock_guard<std::mutex> lk(g_device_mu);
          if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            use_graph = false;
            (void)hipGetLastError();
          } else {
            const tip_status cs = enqueue_captured_chunk(kBatchChunk);
            hipGraph_t gr = nullptr;
            const hipError_t e = hipStreamEndCapture(st, &gr);
            hipError_t ei = hipErrorUnknown;
            if (cs == TIP_OK && e == hipSuccess && gr) ei = hipGraphInstantiate(&graph, gr, nullptr, nullptr, 0);
            if (gr) (void)hipGraphDestroy(gr);
            if (ei != hipSuccess) {
              graph = nullptr;
              use_graph = false;
              (void)hipGetLastError();
            }
          }
        }
        if (use_graph && graph) {
          TIP_HIP(hipGraphLaunch(graph, st));
        } else {
          tip_status cs = enqueue_chunk(kBatchChunk, g_profiling != 0, false);
          if (cs != TIP_OK) return cs;
        }
        tip_status ps = poll();
        if (ps != TIP_OK) return ps;
        for (size_t k = 0; k + 1 < evs.size(); k += 2) {
          float ms = 0.f;
          TIP_HIP(hipEventElapsedTime(&ms, evs[k], evs[k + 1]));
          stencil_seconds += ms * 1e-3;
          ++stencil_launches;
        }
        for (hipEvent_t e : evs) (void)hipEventDestroy(e);
        evs.clear();
        if (h_active[0] == 0) break;
      }
      // the FP64 check of every frozen solve: accept, or restart CG from x
      for (size_t gi = 0; gi < groups.size(); ++gi) {
        BatchArgs ga = args;
        ga.item_base = groups[gi].item_base;
        if (groups[gi].prec == Prec::kF32)
          TIP_HIP(launch_batch_reliable(ga, groups[gi], sc, 1, vb + gv[gi].x, vb + gv[gi].xh, vb + gv[gi].r,
                                        vb + gv[gi].p, pt + rowstride, rowstride, st));
        else
          TIP_HIP(launch_batch_true_residual(ga, groups[gi], sc, vb + gv[gi].x, vb + gv[gi].r, vb + gv[gi].p,
                                             pt + rowstride, rowstride, st));
      }
      tip_status ps = poll();
      if (ps != TIP_OK) return ps;
      if (h_active[0] == 0) break;
    }
    // per-lane results back to the problems
    double* h_q = (double*)((char*)host.p + 64);
    double* h_rr = h_q + 2 * (size_t)L;
    int* h_state = (int*)(h_rr + L);
    int* h_iters = h_state + L;
    int* h_restarts = h_iters + L;
    int* h_ru = h_restarts + L;
    TIP_HIP(hipMemcpyAsync(h_q, sc.q, 2 * (size_t)L * sizeof(double), hipMemcpyDeviceToHost, st));
    TIP_HIP(hipMemcpyAsync(h_rr, sc.relres2, (size_t)L * sizeof(double), hipMemcpyDeviceToHost, st));
    TIP_HIP(hipMemcpyAsync(h_state, sc.state, (size_t)L * sizeof(int), hipMemcpyDeviceToHost, st));
    TIP_HIP(hipMemcpyAsync(h_iters, sc.iters, (size_t)L * sizeof(int), hipMemcpyDeviceToHost, st));
    TIP_HIP(hipMemcpyAsync(h_restarts, sc.restarts, (size_t)L * sizeof(int), hipMemcpyDeviceToHost, st));
    TIP_HIP(hipMemcpyAsync(h_ru, sc.ru_lanes, (size_t)L * sizeof(int), hipMemcpyDeviceToHost, st));
    unsigned long long bytes_moved = 0;
    if (args.bytes) TIP_HIP(hipMemcpyAsync(&bytes_moved, args.bytes, sizeof bytes_moved, hipMemcpyDeviceToHost, st));
    TIP_HIP(hipStreamSynchronize(st));
    for (size_t ji = 0; ji < jobs.size(); ++ji) {
      const BatchJob& J = jobs[ji];
      const BatchClass& c = classes[(size_t)job_class[ji]];
      const tip_params& p = params[J.prob];
      const int ncomp = J.g.ncomp;
      RunResult& rr = results[(size_t)J.prob];
      for (int j = 0; j < J.nb; ++j) {
        const int lane = J.lane0 + j;
        const int64_t r = J.rhs0 + j;
        const int64_t m = c.j3 >= 0 ? (int64_t)class_probe((uint64_t)(r / ncomp), J.g) : r / ncomp;
        const size_t k = (size_t)((m - p.m_begin) * ncomp + r % ncomp);
        rr.qre[k] = h_q[2 * lane];
        rr.qim[k] = h_q[2 * lane + 1];
        rr.state[k] = h_state[lane];
        rr.iters[k] = h_iters[lane];
        rr.relres[k] = std::sqrt(h_rr[lane]);
        rr.acc.restarts += h_restarts[lane];
        rr.acc.reliable_updates += h_ru[lane];
      }
    }
    for (int32_t i = 0; i < count; ++i) {
      tip_stats& a = results[(size_t)i].acc;
      a.stencil_launches = stencil_launches;
      a.stencil_seconds = g_profiling ? stencil_seconds : 0.0;
      a.stencil_bytes = (double)bytes_moved;
    }
  }
  // estimates and stats per problem; conjugate F_3 columns from their partners
  tip_status first = TIP_OK;
  int32_t first_i = -1;
  std::string first_msg;
  for (int32_t i = 0; i < count; ++i) {
    const tip_op_s* h = hs[(size_t)i].get();
    if (conj_split(h->geom, h->kind, masks[(size_t)i], &params[i], false))
      conj_copies(h->geom, &params[i], h->geom.ncomp, results[(size_t)i]);
    const tip_status si =
        finish_run(h, &params[i], results[(size_t)i], estimates[i], stats ? &stats[i] : nullptr, t_start);
    if (statuses) statuses[i] = si;
    if (si != TIP_OK && first_i < 0) first = si, first_i = i, first_msg = g_err;
  }
  if (first_i >= 0) return fail(first, "torus %d: %s", first_i, first_msg.c_str());
  return TIP_OK;
}

}  // namespace

extern "C" {

tip_status trace_inv_probe_op(tip_op_handle h, const tip_params* p, double* estimates, tip_stats* stats) {
  return run_probe(h, p, estimates, nullptr, nullptr, stats);
}

tip_status trace_inv_probe_grad(tip_op_handle h, const tip_params* p, double* estimates, double* grad_mass,
                                double* grad_coupling, tip_stats* stats) {
  if (!grad_mass && !grad_coupling) return fail(TIP_EINVAL, "grad_mass and grad_coupling are both NULL");
  return run_probe(h, p, estimates, grad_mass, grad_coupling, stats);
}

tip_status tip_solve_probe(tip_op_handle h, const tip_params* p, int64_t m, int32_t comp, double* x_out,
                           double* q_out, tip_stats* stats) {
  const auto t_start = std::chrono::steady_clock::now();
  if (!h) return fail(TIP_EINVAL, "handle is NULL");
  if (!p) return fail(TIP_EINVAL, "params is NULL");
  tip_params one = *p;           // one right-hand side; probe-count fields do not apply
  one.n_vectors = 1;
  one.m_begin = 0;
  one.rhs_block = 0;             // the block size trace_inv_probe uses: same arithmetic
  int mask = 0;
  tip_status s = check_params(h, &one, &mask);
  if (s != TIP_OK) return s;
  const Geom& g = h->geom;
  if (m < 0 || m >= (int64_t)g.V) return fail(TIP_EINVAL, "probe %lld outside [0, V)", (long long)m);
  if (comp < 0 || comp >= g.ncomp) return fail(TIP_EINVAL, "comp = %d out of range", comp);
  if (!x_out) return fail(TIP_EINVAL, "x_out is NULL");
  Solver sv;
  sv.need_x = true;
  s = sv.setup(h, &one, mask);
  if (s != TIP_OK) return s;
  s = sv.solve_block(m * g.ncomp + comp, 1);
  if (s != TIP_OK) return s;
  TIP_HIP(launch_layout(g, sv.pl.elem, sv.pl.logB, 0, sv.X, x_out, false, sv.st));
  TIP_HIP(hipStreamSynchronize(sv.st));
  if (q_out) {
    q_out[0] = sv.h_q[0];
    q_out[1] = sv.h_q[1];
  }
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    stats->solves = 1;
    stats->total_iters = sv.h_iters[0];
    stats->max_iters = sv.h_iters[0];
    stats->max_true_relres = std::sqrt(sv.h_relres2[0]);
    stats->max_quad_err_bound = sv.h_relres2[0] * (double)g.V / h->lambda_lb;
    sv.fill_stats(stats);
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  }
  if (sv.h_state[0] == kBreakdown) return fail(TIP_EBREAKDOWN, "solve broke down (p^H A p <= 0)");
  if (sv.h_state[0] != kAccepted) return fail(TIP_ENOCONV, "solve did not converge within max_iter");
  return TIP_OK;
}

tip_status tip_autotune(tip_op_handle h, const tip_params* p, int64_t sample_vectors, tip_tuning* best,
                        tip_tuning* tried, int32_t max_tried, int32_t* n_tried) {
  if (!h) return fail(TIP_EINVAL, "handle is NULL");
  if (!p) return fail(TIP_EINVAL, "params is NULL");
  if (!best) return fail(TIP_EINVAL, "best is NULL");
  if (max_tried < 0 || (max_tried > 0 && !tried)) return fail(TIP_EINVAL, "tried is NULL");
  const Geom& g = h->geom;
  tip_params q = *p;
  q.n_vectors = std::max<int64_t>(1, std::min<int64_t>(sample_vectors > 0 ? sample_vectors : 64, g.V));
  q.m_begin = 0;
  q.quadratures = nullptr;
  int mask = 0;
  tip_status s = check_params(h, &q, &mask);
  if (s != TIP_OK) return s;
  // candidates: right-hand sides per block, and (4-D power-of-two lattices,
  // where the XCD block order applies) the tiles per round
  std::vector<int> blocks = p->rhs_block > 0 ? std::vector<int>{p->rhs_block} : std::vector<int>{16, 32, 64};
  std::vector<int> rounds{0};
  if (g.pow2 && g.ndim == 4 && p->round_tiles == 0) rounds = {0, 64, 128, 256, 512};
  else if (p->round_tiles > 0) rounds = {p->round_tiles};
  std::vector<double> est((size_t)num_checkpoints(q.n_vectors) * 2);
  int count = 0;
  double best_t = 1e300;
  for (int b : blocks)
    for (int r : rounds) {
      q.rhs_block = b;
      q.round_tiles = r;
      tip_stats st{};
      s = trace_inv_probe_op(h, &q, est.data(), &st);            // warm-up (allocation, first launches)
      if (s != TIP_OK) return s;
      s = trace_inv_probe_op(h, &q, est.data(), &st);
      if (s != TIP_OK) return s;
      tip_tuning t{};
      t.rhs_block = b;
      t.round_tiles = r;
      t.march_tc = q.march_tc;
      t.seconds_per_solve = st.seconds / (double)std::max<int64_t>(1, st.solves);
      if (count < max_tried) tried[count] = t;
      ++count;
      if (t.seconds_per_solve < best_t) best_t = t.seconds_per_solve, *best = t;
    }
  if (n_tried) *n_tried = count;
  return TIP_OK;
}

tip_status trace_inv_probe(const tip_operator* op, const tip_params* p, double* estimates, tip_stats* stats) {
  if (!p) return fail(TIP_EINVAL, "params is NULL");
  if (!estimates) return fail(TIP_EINVAL, "estimates is NULL");
  Geom g;
  tip_status s = validate_op(op, &g);
  if (s != TIP_OK) return s;
  if (p->n_vectors < 1 || p->n_vectors > (int64_t)g.V)
    return fail(TIP_EINVAL, "n_vectors = %lld must be in [1, V = %u]", (long long)p->n_vectors, g.V);
  tip_op_s* h = nullptr;
  s = create_handle(op, (hipStream_t)p->stream, &h);
  if (s != TIP_OK) return s;
  s = trace_inv_probe_op(h, p, estimates, stats);
  const std::string msg = g_err;
  (void)hipStreamSynchronize((hipStream_t)p->stream);
  delete h;
  g_err = msg;
  return s;
}

tip_status trace_inv_probe_batch(const tip_operator* ops, const tip_params* params, int32_t count, int32_t n_streams,
                                 double* const* estimates, tip_stats* stats, int32_t* statuses) {
  if (n_streams < 0) return fail(TIP_EINVAL, "n_streams = %d must be >= 0", n_streams);
  tip_status s = validate_batch(ops, params, count, estimates);
  if (s != TIP_OK || count == 0) return s;
  return run_batch(ops, params, count, estimates, stats, statuses, nullptr);
}

tip_status tip_autotune_batch(const tip_operator* ops, const tip_params* params, int32_t count,
                              int64_t sample_vectors, tip_tuning* best, tip_tuning* tried, int32_t max_tried,
                              int32_t* n_tried) {
  if (!best) return fail(TIP_EINVAL, "best is NULL");
  if (max_tried < 0 || (max_tried > 0 && !tried)) return fail(TIP_EINVAL, "tried is NULL");
  tip_status s = validate_batch(ops, params, count, nullptr);
  if (s != TIP_OK) return s;
  if (count == 0) return fail(TIP_EINVAL, "count = 0: nothing to tune");
  // the sample: the first sample_vectors probes of every problem, fresh runs
  const int64_t want = sample_vectors > 0 ? sample_vectors : 64;
  std::vector<tip_params> q(params, params + count);
  std::vector<std::vector<double>> est((size_t)count);
  std::vector<double*> est_ptr((size_t)count);
  int64_t solves = 0;
  for (int32_t i = 0; i < count; ++i) {
    q[(size_t)i].n_vectors = std::max<int64_t>(1, std::min<int64_t>(want, params[i].n_vectors));
    q[(size_t)i].m_begin = 0;
    q[(size_t)i].quadratures = nullptr;
    est[(size_t)i].assign((size_t)num_checkpoints(q[(size_t)i].n_vectors) * 2, 0.0);
    est_ptr[(size_t)i] = est[(size_t)i].data();
    solves += q[(size_t)i].n_vectors * (ops[i].kind == TIP_KIND_COVARIANT ? 3 : 1);
  }
  std::vector<int> blocks = params[0].rhs_block > 0 ? std::vector<int>{params[0].rhs_block} : std::vector<int>{16, 32, 64};
  std::vector<int> items = params[0].item_sites > 0 ? std::vector<int>{params[0].item_sites}
                                                    : std::vector<int>{256, 512, 1024, 2048};
  int cnt = 0;
  double best_t = 1e300;
  for (int bsz : blocks)
    for (int it : items) {
      tip_tuning t{};
      t.rhs_block = bsz;
      t.item_sites = it;
      double secs = 0.0;
      for (int rep = 0; rep < 2; ++rep) {                 // the first run warms up
        const auto t0 = std::chrono::steady_clock::now();
        s = run_batch(ops, q.data(), count, est_ptr.data(), nullptr, nullptr, &t);
        if (s != TIP_OK) return s;
        secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      }
      t.seconds_per_solve = secs / (double)std::max<int64_t>(1, solves);
      if (cnt < max_tried) tried[cnt] = t;
      ++cnt;
      if (t.seconds_per_solve < best_t) best_t = t.seconds_per_solve, *best = t;
    }
  if (n_tried) *n_tried = cnt;
  return TIP_OK;
}

tip_status tip_apply_operator(const tip_operator* op, int32_t nrhs, const double* x, double* y, void* stream) {
  Geom g;
  tip_status s = validate_op(op, &g);
  if (s != TIP_OK) return s;
  if (nrhs < 1) return fail(TIP_EINVAL, "nrhs = %d must be >= 1", nrhs);
  if (!x || !y) return fail(TIP_EINVAL, "x or y is NULL");
  hipStream_t st = (hipStream_t)stream;
  tip_op_s* h = nullptr;
  s = create_handle(op, st, &h);
  if (s != TIP_OK) return s;
  const Elem elem = op->kind == TIP_KIND_COVARIANT ? Elem::kComplex : Elem::kReal;
  const size_t esz = elem == Elem::kReal ? sizeof(double) : sizeof(double2);
  const size_t bytes = (size_t)g.ncomp * g.V * esz;       // one vector
  const TileMap tm = make_tilemap(g, 0);
  tip_status ret = TIP_OK;
  if (h->vec.ensure(2 * bytes) != hipSuccess) ret = fail(TIP_ENOMEM, "hipMalloc apply buffers");
  for (int k = 0; k < nrhs && ret == TIP_OK; ++k) {
    char* in = (char*)h->vec.p;
    char* out = in + bytes;
    const char* xk = (const char*)x + k * bytes;
    char* yk = (char*)y + k * bytes;
    if (launch_layout(g, elem, 0, 0, xk, in, true, st) != hipSuccess ||
        launch_stencil(h->dev(), g, tm, nullptr, elem, Prec::kF64, nullptr, nullptr, in, out, nullptr, nullptr, st) != hipSuccess ||
        launch_layout(g, elem, 0, 0, out, yk, false, st) != hipSuccess)
      ret = fail(TIP_EDEVICE, "apply launch failed");
  }
  if (ret == TIP_OK && hipStreamSynchronize(st) != hipSuccess) ret = fail(TIP_EDEVICE, "apply failed on the device");
  delete h;
  return ret;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Operator application without allocation.  Its workspace (repacked links and
// the block-layout input and output vectors) lives in `scratch`, a file-scope
// device array of kScratchBytes: every GPU the library runs on holds its own
// copy until the process ends, and calls on one GPU share it (overlapping
// calls on one GPU race).  In host code the array's name is only a stand-in
// for the variable; its device address is taken once per device with
// hipGetSymbolAddress, with that device current, and only that address is
// handed to kernels.  Every byte a call reads from the scratch was written
// earlier in the same call, so nothing needs clearing between calls.
// ---------------------------------------------------------------------------

namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;     // 64 MiB per device
constexpr int kMaxScratchDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device.
tip_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(TIP_EDEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(TIP_EUNSUPPORTED, "device %d: the no-allocation scratch covers devices 0..%d", dev,
                kMaxScratchDevices - 1);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(TIP_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return TIP_OK;
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

extern "C" {

tip_status tip_apply_operator_noalloc(const tip_operator* op, int32_t nrhs, const double* x, double* y,
                                      void* stream) {
  Geom g;
  tip_status s = validate_op(op, &g);
  if (s != TIP_OK) return s;
  if (nrhs < 1) return fail(TIP_EINVAL, "nrhs = %d must be >= 1", nrhs);
  if (!x || !y) return fail(TIP_EINVAL, "x or y is NULL");
  const bool cov = op->kind == TIP_KIND_COVARIANT;
  const Elem elem = cov ? Elem::kComplex : Elem::kReal;
  const size_t esz = cov ? sizeof(double2) : sizeof(double);
  const size_t bytes = (size_t)g.ncomp * g.V * esz;                   // one vector
  const size_t link_bytes = cov ? (size_t)g.ndim * 9 * g.V * sizeof(double2) : 0;
  const size_t need = align256(link_bytes) + 2 * align256(bytes);
  if (need > kScratchBytes)
    return fail(TIP_EINVAL, "lattice needs %zu bytes of workspace; the no-allocation scratch holds %zu", need,
                kScratchBytes);
  void* base = nullptr;
  s = scratch_address(&base);
  if (s != TIP_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char* links = (char*)base;
  char* in = links + align256(link_bytes);
  char* out = in + align256(bytes);
  // the caller's mass field and couplings are read in place; the links are
  // repacked into the scratch ([ndim][9][V], as the kernels read them)
  OpDev od{};
  od.kind = op->kind;
  od.mass = op->mass;
  od.mass_field = op->mass_field;
  od.coupling = op->coupling;
  od.links = cov ? (const double*)links : nullptr;
  od.links_eo = nullptr;
  if (cov && launch_repack_links(g, (const double2*)op->links, (double2*)links, st) != hipSuccess)
    return fail(TIP_EDEVICE, "link repack launch failed");
  const TileMap tm = make_tilemap(g, 0);
  for (int k = 0; k < nrhs; ++k) {
    const char* xk = (const char*)x + k * bytes;
    char* yk = (char*)y + k * bytes;
    if (launch_layout(g, elem, 0, 0, xk, in, true, st) != hipSuccess ||
        launch_stencil(od, g, tm, nullptr, elem, Prec::kF64, nullptr, nullptr, in, out, nullptr, nullptr, st) !=
            hipSuccess ||
        launch_layout(g, elem, 0, 0, out, yk, false, st) != hipSuccess)
      return fail(TIP_EDEVICE, "apply launch failed");
  }
  if (hipStreamSynchronize(st) != hipSuccess) return fail(TIP_EDEVICE, "apply failed on the device");
  return TIP_OK;
}

tip_status tip_hier_perm(int32_t ndim, const int64_t* dims, uint32_t* P_out, void* stream) {
  Geom g;
  tip_status s = make_geom(ndim, dims, 1, &g);
  if (s != TIP_OK) return s;
  if (!P_out) return fail(TIP_EINVAL, "P_out is NULL");
  hipStream_t st = (hipStream_t)stream;
  TIP_HIP(launch_hier_perm(g, P_out, st));
  TIP_HIP(hipStreamSynchronize(st));
  return TIP_OK;
}

tip_status tip_probe_vectors(int32_t ndim, const int64_t* dims, int32_t ncomp, int32_t mask, uint64_t seed,
                             int64_t m0, int64_t count, int32_t comp, int32_t probe, int32_t stop_levels,
                             double* out, void* stream) {
  if (ncomp != 1 && ncomp != 3) return fail(TIP_EINVAL, "ncomp = %d, expected 1 or 3", ncomp);
  Geom g;
  tip_status s = make_geom(ndim, dims, ncomp, &g);
  if (s != TIP_OK) return s;
  if (mask == TIP_MASK_DEFAULT) mask = ncomp == 1 ? TIP_MASK_Z2 : TIP_MASK_Z4;
  if (mask < TIP_MASK_NONE || mask > TIP_MASK_Z4) return fail(TIP_EINVAL, "unknown mask %d", mask);
  if (probe < TIP_PROBE_HIERARCHICAL || probe > TIP_PROBE_FOURIER) return fail(TIP_EINVAL, "unknown probe kind %d", probe);
  if ((probe == TIP_PROBE_NATURAL || probe == TIP_PROBE_STOPPED || probe == TIP_PROBE_FOURIER) && !g.pow2)
    return fail(TIP_EINVAL, "probe kind %d needs power-of-two sides", probe);
  if (probe == TIP_PROBE_RANDOM && mask == TIP_MASK_NONE) return fail(TIP_EINVAL, "random probes need a Z2 or Z4 mask");
  if (stop_levels < 0) return fail(TIP_EINVAL, "stop_levels must be >= 0");
  g.probe = probe;
  g.stop = stop_levels;
  if (comp < 0 || comp >= ncomp) return fail(TIP_EINVAL, "comp = %d out of range", comp);
  if (m0 < 0 || count < 0 || m0 + count > (int64_t)g.V) return fail(TIP_EINVAL, "probe range outside [0, V)");
  if (!out && count > 0) return fail(TIP_EINVAL, "out is NULL");
  hipStream_t st = (hipStream_t)stream;
  for (int64_t done = 0; done < count; done += 65535) {
    const int c = (int)std::min<int64_t>(65535, count - done);
    TIP_HIP(launch_probe_vectors(g, seed, mask, m0 + done, c, comp, (double2*)out + (size_t)done * g.V, st));
  }
  TIP_HIP(hipStreamSynchronize(st));
  return TIP_OK;
}

}  // extern "C"
