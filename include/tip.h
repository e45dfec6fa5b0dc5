/*
 * tip.h -- Tr(A^-1) by hierarchical probing on toroidal lattices, MI355X (gfx950).
 *
 * C ABI of libtip.so.  Method: Stathopoulos, Laeuchli, Orginos, "Hierarchical
 * probing for estimating the trace of the matrix inverse on toroidal lattices"
 * (arXiv:1302.4018).  The library
 *   1. generates probing vectors in-kernel from site indices: the hierarchical
 *      lattice permutation (Sec. 3, Alg. 5 with the Red-Black order of Alg. 3 in
 *      the closed form of Lemma 3.3), Hadamard columns in the order of
 *      eq. HpermSequence read through eq. row-col-permutation, and the random
 *      vector z0 of Sec. 4 (eq. removebias);
 *   2. solves A x = z by conjugate gradients with a lattice stencil (Sec. 1.1.2:
 *      quadratures through linear solves);
 *   3. accumulates z^H x into the estimator (1/s) sum_m z_m^H A^-1 z_m
 *      (Sec. 1, Hutchinson) reported at every s = 2^k (Sec. 1.1.4, and the
 *      nesting Z(k-1) = Z(k)(:, 1:2^{k-1}) after eq. Hperm-recursive).
 *   The solves run CG on the even-odd reduced system whenever every side is a
 *   power of two >= 2 and the diagonal is positive (both precisions): the red-black
 *   colouring of Sec. 2 makes the torus bipartite, A = D - H with H joining
 *   opposite parities only, and CG iterates on the Schur complement
 *   S = D_e - H_eo D_o^-1 H_oe over the even sites (half the vector length,
 *   about half the iterations), then forms x_o = D_o^-1 (b_o + H_oe x_e).  The
 *   acceptance test is the same FP64 true residual of the full system.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice: ndim in 1..4, sides dims[0..ndim-1] = n_1..n_ndim >= 1; V = prod n_j
 *   <= 2^31.  Sites are numbered s = x_1 + n_1 (x_2 + n_2 (x_3 + n_3 x_4)).
 *   Sides that are powers of two give the hierarchical probing of Sec. 3 and
 *   the fastest kernels.  Other sides n_j = 2^{k_j} p_j (p_j odd) follow
 *   Sec. 3.4: binary red-black levels while every side with a remaining size
 *   above 1 is even, then one level coloured by the three-colouring theorem of
 *   Sec. 3.4 (see "Right-hand sides").
 * Operator: A = sum_e w_e L_e + diag(m(x)) (x) I_ncomp over the edges e = (x, x+mu)
 *   of the torus (the shifted periodic Laplacian of Sec. 5), with
 *     TIP_KIND_SCALAR    (ncomp = 1): L_e = [[1, -1], [-1, 1]];
 *     TIP_KIND_COVARIANT (ncomp = 3): L_e = [[I, -U_mu(x)], [-U_mu(x)^H, I]],
 *   i.e. (A x)(s) = (m(s) + sum_mu [w_mu(s) + w_mu(s-mu)]) x(s)
 *                 - sum_mu [w_mu(s) U_mu(s) x(s+mu) + w_mu(s-mu) U_mu(s-mu)^H x(s-mu)].
 *   A is Hermitian positive definite when every m(x) > 0.
 * Right-hand sides: spatial probe m (0-based) and internal component c give
 *   b_{m,c}(y, c') = delta_{c c'} z0(y, c) H(P(y), bitrev_L(m)), L = log2 V,
 *   H(i, j) = (-1)^{popcount(i & j)} (eq. HadamardElements), P the location of
 *   site y in the hierarchical permutation (Alg. 5; the bits of the first
 *   active dimension are the most significant of each Red-Black index, and
 *   earlier levels occupy more significant bits of P).
 *   z0(y, c) uses counter n = y * ncomp + c of SplitMix64(seed) (state
 *   seed + (n+1) * 0x9E3779B97F4A7C15, then the published 64-bit mix):
 *   Z2: +1 / -1 from the top output bit; Z4: i^t, t = the top two bits.
 *   Sides with odd factors: P(y) is the binary colour over the B binary
 *   levels (LB bits) and gamma = 2^LB (x 3 with a three-colouring level)
 *   colours make one sweep.  Probe m = r gamma + j takes column j of the
 *   general recursion eq. Hperm-general-recursive: H(P(y), bitrev_LB(j mod
 *   2^LB)) times w^{(j >> LB) C(y)}, w = -1/2 + i sqrt(3)/2 and C the
 *   three-colouring of the sub-torus y >> B; sweep r uses mask outputs
 *   n = (r V + y) ncomp + c.  Probes past 2^LB are complex (complex solves).
 *   For the scalar (real) operator with a Z2 or no mask, column j3 = 2 of a
 *   sweep is the conjugate of column j3 = 1 (w^2 = conj w), so its quadrature
 *   is the conjugate of the one of probe m - 2^LB and is not solved again
 *   (stats->reused), and the j3 = 0 probes are solved in real arithmetic.
 * Memory: every pointer documented as "device" is caller-owned device memory
 *   and is never freed by the library; "host" pointers likewise.  Complex
 *   numbers are interleaved (re, im) float64 pairs.
 * Streams: `stream` is a hipStream_t.  All work of a call is enqueued on that
 *   stream; calls that return synchronise it.  With NULL the library first
 *   synchronises the null stream, then works on a non-blocking stream of the
 *   operator handle, so that chunks of CG iterations can be replayed as HIP
 *   graphs (set TIP_GRAPH=0 to keep the null stream and eager launches).
 * Errors: no exception crosses the ABI.  Argument validation fails with
 *   TIP_EINVAL before any output is written or any device work is enqueued;
 *   tip_last_error() then returns a thread-local message.
 */
#ifndef TIP_H
#define TIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TIP_OK = 0,
  TIP_EINVAL = -1,       /* invalid argument (nothing written)                   */
  TIP_ENOMEM = -2,       /* device or host allocation failed                     */
  TIP_ENOCONV = -3,      /* a solve hit max_iter (completed checkpoints written) */
  TIP_EBREAKDOWN = -4,   /* CG breakdown: p^H A p <= 0 or not finite             */
  TIP_EDEVICE = -5,      /* a HIP runtime call failed                            */
  TIP_EUNSUPPORTED = -6  /* valid request this build does not implement          */
} tip_status;

enum { TIP_KIND_SCALAR = 0, TIP_KIND_COVARIANT = 1 };
enum { TIP_MASK_DEFAULT = -1, TIP_MASK_NONE = 0, TIP_MASK_Z2 = 1, TIP_MASK_Z4 = 2 };
/* Precision of the CG solves.  FP64: vectors, links and arithmetic in FP64.
 * MIXED: CG vectors and links stored and combined in FP32, with FP64 kept for
 * the solution x, the CG scalars, reliable updates (the FP32 correction folded
 * into x and the residual recomputed from x with the FP64 operator; Sleijpen &
 * van der Vorst 1996) and the final true-residual test, so a solve is
 * accepted on the same FP64 criterion as in FP64 mode.  An update is made
 * when a bound on the drift of the FP32 residual from b - A x, accumulated
 * from the CG scalars (van der Vorst & Ye 2000), passes 2^-5 of the residual
 * norm, and also, if reliable_delta > 0, when the residual has fallen by
 * reliable_delta since the last update.  The drift bound grows with
 * ||A|| ||x_h||, so ill-conditioned operators get the updates they need:
 * free fields at condition numbers 1e4, 1e5 and 1e6 converge to 1e-10 with
 * 1.3x, 1.9x and 3.1x the FP64 iteration count.  FP32 pays on the
 * well-conditioned end (the 32^4 covariant workload: 12 iterations either
 * way, one update per solve).
 * In MIXED a single-precision p^H A p <= 0 (rounding on a badly conditioned
 * operator) is not a breakdown: the solve goes to the FP64 check and restarts
 * from the FP64 residual (counted in tip_stats.restarts; TIP_ENOCONV once the
 * restart budget is spent).
 * MIXED reports the variational quadrature 2 Re(b^H x) - x^H A x = b^H x + x^H r,
 * whose error r^H A^-1 r <= ||r||^2 / lambda_min is second order in the
 * residual. */
enum { TIP_PREC_FP64 = 0, TIP_PREC_MIXED = 1 };
/* Probe kinds.  HIERARCHICAL: the probes described above (default).  The
 * comparison probes of Sec. 5 run through the same solver and estimator:
 * NATURAL, Hadamard columns in natural order on the natural site numbering,
 * b_{m,c}(y, c) = z0(y, c) H(y, m) (power-of-two sides); RANDOM, plain Monte
 * Carlo (Sec. 1, Hutchinson): b_{m,c}(y, c) = z0_m(y, c), the mask of sweep m
 * (SplitMix64 outputs (m V + y) ncomp + c), so every probe is an independent
 * Z2 / Z4 noise vector (a Z2 or Z4 mask is required).
 * STOPPED (Sec. 5.1, power-of-two sides): the colouring recursion stopped
 * after stop_levels bit-levels; each colour class keeps its natural order, so
 * P_k(y) = [Alg. 5 string of levels 1..k | natural index of the coarse
 * coordinates y_j >> min(k, k_j)] and b = z0 H(P_k(y), bitrev_L(m)).  k = 0 is
 * the natural site order, k >= max k_j the full hierarchy.
 * FOURIER (power-of-two sides, complex solves): eq. Hperm-general-recursive
 * with the a active bits of one Alg. 5 level taken as one level of 2^a colours,
 * z_m(y) = prod_l exp(2 pi i s_l(y) j_l / 2^{a_l}), m = sum_l j_l 2^{a_1 + .. + a_{l-1}},
 * s_l the level's Red-Black index (Lemma 3.3); entries are 16th roots of unity
 * made of the doubles nearest cos(pi/8), sin(pi/8) and sqrt(2)/2.  Equal to the
 * hierarchical estimate at every level boundary s = 2^{a_1 + .. + a_k}. */
enum { TIP_PROBE_HIERARCHICAL = 0, TIP_PROBE_NATURAL = 1, TIP_PROBE_RANDOM = 2, TIP_PROBE_STOPPED = 3,
       TIP_PROBE_FOURIER = 4 };

/* Operator description.  Arrays are DEVICE pointers, read only. */
typedef struct {
  int32_t ndim;              /* 1..4                                              */
  int64_t dims[4];           /* n_1..n_ndim >= 1 (see "Lattice" above)             */
  int32_t kind;              /* TIP_KIND_SCALAR or TIP_KIND_COVARIANT              */
  double mass;               /* m(x) = mass when mass_field is NULL                */
  const double* mass_field;  /* [V] m(x), or NULL                                  */
  const double* coupling;    /* [ndim][V] w_mu(x) of edge x -> x+mu, or NULL (= 1) */
  const double* links;       /* covariant: [ndim][V][3][3] complex128, row-major,
                                (U x)_a = sum_b U[a][b] x_b; ignored for scalar    */
} tip_operator;

typedef struct {
  int64_t n_vectors;    /* spatial probes s, 1 <= n_vectors <= V                   */
  int64_t m_begin;      /* first probe solved; 0 for a fresh run (see quadratures) */
  double tol;           /* accept a solve when ||b - A x||_2 <= tol ||b||_2, with the
                           residual recomputed in FP64 (Sec. 1.1.2 stops on the
                           residual; its square bounds the quadrature error)        */
  int32_t max_iter;     /* CG iterations per solve; 0 = min(10 V ncomp, 2^20)      */
  uint64_t seed;        /* seed of z0                                              */
  int32_t mask;         /* TIP_MASK_*; DEFAULT = Z2 for scalar, Z4 for covariant   */
  int32_t rhs_block;    /* right-hand sides solved together; 0 = library choice   */
  int32_t precision;    /* TIP_PREC_FP64 or TIP_PREC_MIXED                         */
  void* stream;         /* hipStream_t or NULL                                     */
  double* quadratures;  /* HOST [n_vectors][2] q_m = sum_c b_{m,c}^H x_{m,c}, or NULL.
                           Entries [m_begin, n_vectors) are written.  When m_begin > 0
                           entries [0, m_begin) must hold the q_m of an earlier call
                           (same operator, seed, mask) and are read: this resumes a
                           run, reusing earlier levels' quadratures.                */
  double reliable_delta; /* MIXED: also update when the FP32 residual norm has
                            fallen by this factor since the last update; 0 = the
                            drift bound alone                                      */
  int32_t probe;         /* TIP_PROBE_*; 0 = hierarchical                           */
  int32_t round_tiles;   /* 4-D power-of-two lattices: stencil tiles per XCD round of the
                            workgroup order (0 = library choice; see tip_autotune) */
  int32_t march_tc;      /* lattice slices one stencil workgroup marches (power of two;
                            0 = library choice)                                    */
  int32_t stop_levels;   /* TIP_PROBE_STOPPED: bit-levels of the colouring kept (>= 0) */
  int32_t item_sites;    /* trace_inv_probe_batch: lattice sites one workgroup walks per
                            work item (rounded up to a power of two >= 256; 0 = library
                            choice, 512; see tip_autotune_batch); ignored elsewhere  */
  double* residuals;     /* HOST [n_vectors][ncomp] or NULL: entries [m_begin, n_vectors)
                            receive ||b - A x|| / ||b|| of each solve's accepted FP64 true
                            residual (the partner's for a reused conjugate; NaN for a solve
                            that was not accepted).  With ||b||^2 = V and lambda_lb of
                            tip_stats.max_quad_err_bound, (1/s) sum_{m<s,c} V res^2 /
                            lambda_lb bounds the error of the estimate at s.         */
} tip_params;

typedef struct {
  int64_t solves;              /* right-hand sides solved by this call             */
  int64_t total_iters;         /* CG iterations summed over those solves           */
  int32_t max_iters;           /* largest iteration count of one solve             */
  int32_t n_checkpoints_done;  /* leading estimates[] entries that are valid       */
  double max_true_relres;      /* max ||b - A x|| / ||b|| over accepted solves     */
  double seconds;              /* wall time of the call                            */
  int64_t stencil_launches;    /* stencil-kernel launches (timed when profiling on) */
  double stencil_seconds;      /* summed device time of those launches (hipEvents), 0 if off */
  double stencil_bytes;        /* algorithmic HBM bytes of those launches          */
  int64_t reliable_updates;    /* MIXED: reliable updates done (all right-hand sides) */
  double max_quad_err_bound;   /* max over solves of ||b - A x||^2 / lambda_lb, with
                                  lambda_lb = min m(x) (valid when every coupling is
                                  >= 0, NaN otherwise): bounds each quadrature's error */
  int64_t matvecs;             /* operator applications inside CG (one per iteration of a block) */
  double matvec_seconds;       /* their summed device time (hipEvents), 0 if profiling off */
  double matvec_bytes;         /* their algorithmic HBM bytes                              */
  int32_t even_odd;            /* 1 when CG ran on the even-odd reduced system (see below) */
  int64_t restarts;            /* restarts of CG from x after a failed FP64 true-residual
                                  check (the recursive residual had drifted)               */
  int64_t reused;              /* right-hand sides whose quadrature is the conjugate of an
                                  already solved one (conjugate F_3 columns of a real
                                  operator, see TIP_PROBE_HIERARCHICAL); not in solves     */
} tip_stats;

/* Number of estimates written by trace_inv_probe: floor(log2 n) + 1, plus one
 * more (at s = n) when n is not a power of two. */
int32_t tip_num_checkpoints(int64_t n_vectors);

/* Tr(A^-1) estimates.  estimates: HOST [tip_num_checkpoints(n_vectors)][2];
 * entry k is T = (1/s) sum_{m<s} q_m at s = 2^k (last entry at s = n_vectors),
 * summed in m order with Neumaier compensation.  stats may be NULL.
 * Builds a temporary operator handle (link repack) for the call.
 * On TIP_ENOCONV / TIP_EBREAKDOWN the checkpoints completed before the first
 * failing probe are written and stats->n_checkpoints_done says how many. */
tip_status trace_inv_probe(const tip_operator* op, const tip_params* p,
                           double* estimates, tip_stats* stats);

/* Many independent problems in one call, e.g. a batch of uneven 3-D tori.
 * Problem i is ops[i] with params[i] and writes estimates[i] (HOST
 * [tip_num_checkpoints(params[i].n_vectors)][2]) and, when stats is not NULL,
 * stats[i].  All problems are solved together on params[0].stream (NULL: a
 * stream of the call's own, after the null stream has been synchronised):
 * each problem's right-hand sides are cut into blocks as trace_inv_probe
 * cuts them (params[i].rhs_block, default 32, fewer when the problem has
 * fewer right-hand sides; the conjugate F_3 columns of real odd-sided
 * problems are reused the same way), and every CG phase of every block of
 * every problem that shares the operator kind, element type and precision
 * is one kernel launch over work items of params[0].item_sites sites.  A
 * chunk of CG iterations of the whole batch is captured once as a HIP graph
 * and replayed; the host polls one counter per chunk.  Solves stop on each
 * problem's own tol and max_iter and are accepted on the FP64 true residual;
 * the batch runs plain CG (no even-odd reduction), so results agree with
 * separate trace_inv_probe calls to the solver tolerance, not bit for bit.
 * stats[i].seconds is the wall time of the whole call; stats[i].stencil_*
 * describe the batch's shared stencil launches (the same in every entry;
 * timed only with tip_set_profiling(1), which also turns the graph off).
 * n_streams is kept for compatibility and ignored (must be >= 0).
 * statuses: HOST [count] per-problem status, or NULL.  All arguments are
 * validated before any device work (TIP_EINVAL names the problem); otherwise
 * the return value is TIP_OK or the status of the lowest-numbered failing
 * problem. */
tip_status trace_inv_probe_batch(const tip_operator* ops, const tip_params* params, int32_t count,
                                 int32_t n_streams, double* const* estimates, tip_stats* stats,
                                 int32_t* statuses);

/* Operator handle: validates op and repacks links/couplings into the kernels'
 * layout in library-owned device memory (one time, on `stream`).  The caller's
 * arrays are not referenced after tip_op_create returns. */
typedef struct tip_op_s* tip_op_handle;
tip_status tip_op_create(const tip_operator* op, void* stream, tip_op_handle* out);
tip_status tip_op_destroy(tip_op_handle h);

/* trace_inv_probe on a prepared handle (no repack inside the call). */
tip_status trace_inv_probe_op(tip_op_handle h, const tip_params* p,
                              double* estimates, tip_stats* stats);

/* Launch configuration found by tip_autotune. */
typedef struct {
  int32_t rhs_block;          /* right-hand sides per block                         */
  int32_t round_tiles;        /* tiles per XCD round (0 = library choice)           */
  int32_t march_tc;           /* marched slices (0 = library choice)                */
  double seconds_per_solve;   /* measured on the sample                             */
  int32_t item_sites;         /* tip_autotune_batch: sites per work item            */
} tip_tuning;

/* Times trace_inv_probe_op on the first sample_vectors probes (0 = 64) for each
 * candidate launch configuration and returns the fastest in best: rhs_block in
 * {16, 32, 64} unless p->rhs_block fixes it, and on 4-D power-of-two lattices
 * round_tiles in {library choice, 64, 128, 256, 512} unless p->round_tiles
 * fixes it.  Every candidate runs twice (the first run warms up) and keeps
 * the other fields of p (precision, mask, probe, tol, stream).  tried: HOST
 * [max_tried] candidates in the order timed, or NULL with max_tried = 0;
 * n_tried: how many were timed (may exceed max_tried), or NULL.  Copy the
 * result into tip_params.rhs_block / round_tiles / march_tc.  Results differ
 * between block sizes in rounding only. */
tip_status tip_autotune(tip_op_handle h, const tip_params* p, int64_t sample_vectors, tip_tuning* best,
                        tip_tuning* tried, int32_t max_tried, int32_t* n_tried);

/* Times trace_inv_probe_batch on the first sample_vectors probes of every
 * problem (0 = 64; a sample that keeps the sizes of the probe classes, and so
 * the padding each block size leaves, close to the full run's) for each
 * candidate launch configuration: right-hand sides
 * per block in {16, 32, 64} unless params[0].rhs_block fixes it, times sites
 * per work item in {256, 512, 1024, 2048} unless params[0].item_sites fixes
 * it.  Every candidate runs twice (the first run warms up); the fastest goes
 * to best (its rhs_block and item_sites; round_tiles and march_tc are 0).
 * tried / max_tried / n_tried as in tip_autotune.  Copy the result into every
 * params[i].rhs_block and params[0].item_sites. */
tip_status tip_autotune_batch(const tip_operator* ops, const tip_params* params, int32_t count,
                              int64_t sample_vectors, tip_tuning* best, tip_tuning* tried,
                              int32_t max_tried, int32_t* n_tried);

/* trace_inv_probe_op plus the gradient of the last estimate, T = (1/s) sum_{m<s} q_m
 * at s = n_vectors, with respect to the operator's parameters, the probes held
 * fixed.  Differentiating the Hutchinson estimator of Sec. 1 with
 * d(A^-1) = -A^-1 (dA) A^-1, and using that A is Hermitian (the adjoint solves
 * are the forward solves x_{m,c} = A^-1 b_{m,c}):
 *   grad_mass[y]           = dT/dm(y)    = -(1/s) sum_{m<s,c} ||x_{m,c}(y)||^2
 *   grad_coupling[mu][y]   = dT/dw_mu(y) = -(1/s) sum_{m<s,c} ||x_{m,c}(y) - U_mu(y) x_{m,c}(y+mu)||^2
 * (U = 1 for the scalar operator).  This is the exact derivative of the
 * estimate up to the solver tolerance; for s = V and no mask it is the exact
 * -Tr(A^-1 (dA) A^-1).  With a NULL mass_field (coupling) the entries are the
 * derivatives with respect to a per-site mass (coupling) at the uniform value.
 * grad_mass: DEVICE float64 [V] or NULL; grad_coupling: DEVICE float64 [ndim][V]
 * or NULL; not both NULL.  Both are overwritten; on a status other than TIP_OK
 * their contents are unspecified.  p->m_begin must be 0 (TIP_EINVAL otherwise).
 * The sums over probes are taken block by block in a fixed order, so results
 * are reproducible run to run. */
tip_status trace_inv_probe_grad(tip_op_handle h, const tip_params* p, double* estimates,
                                double* grad_mass, double* grad_coupling, tip_stats* stats);

/* One solve A x = b_{m,comp} on a prepared handle, for checks of the solver
 * and for callers that need the solution itself.  Uses tol, max_iter, seed,
 * mask, precision and stream of p; its probe-count fields and rhs_block are
 * ignored: the solve runs in a block of the library's default size, so it
 * repeats the arithmetic of trace_inv_probe for this right-hand side.
 * x_out: DEVICE, [V][ncomp] complex128 when the solve is complex (covariant
 * operator, or Z4 mask), else [V] float64.  q_out: HOST [2] = b^H x, or NULL.
 * stats may be NULL.  Status as trace_inv_probe for a single solve. */
tip_status tip_solve_probe(tip_op_handle h, const tip_params* p, int64_t m, int32_t comp,
                           double* x_out, double* q_out, tip_stats* stats);

/* y = A x for nrhs vectors.  x, y: DEVICE [nrhs][V][ncomp] complex128 for the
 * covariant operator, [nrhs][V] float64 for the scalar one. */
tip_status tip_apply_operator(const tip_operator* op, int32_t nrhs,
                              const double* x, double* y, void* stream);

/* tip_apply_operator for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and arithmetic (results equal bit for bit),
 * with the caller's mass field and couplings read in place and the
 * workspace (repacked links and the input and output vectors in the kernels'
 * layout) in a fixed device array of the library, 64 MiB per GPU, held from
 * first use until the process ends.  No hipMalloc, hipFree or allocating
 * library routine is called; the first call on a device also resolves the
 * array's device address there (hipGetSymbolAddress).  Lattices whose
 * workspace exceeds 64 MiB (ndim * 9 * V * 16 bytes of links for the
 * covariant operator plus two vectors of ncomp * V elements, each part
 * rounded up to 256 bytes) fail with TIP_EINVAL before any device work.
 * Calls on one GPU share the array: calls that overlap on one GPU (from
 * several host threads, or on several streams) race and must be serialised
 * by the caller.  Every byte a call reads from the array it wrote earlier in
 * the same call, so nothing carries over between calls.  Synchronises
 * `stream` before returning. */
tip_status tip_apply_operator_noalloc(const tip_operator* op, int32_t nrhs,
                                      const double* x, double* y, void* stream);

/* Measurement aid, not part of the method: the practical HBM ceiling of the
 * device, for stating a kernel's rate against what a kernel that only moves
 * data reaches on the same machine beside the published peak.  Allocates
 * `bytes` of device memory split over the arrays of streaming kernel `kind`
 * (0: read only, one array; 1: copy, two arrays; 2: three arrays read and one
 * written, d = a + b + c), runs one warm-up pass and `reps` timed passes
 * (hipEvents on `stream`) with 16-byte accesses and `grid` workgroups of 256
 * threads (0 = 16 per compute unit), frees everything, and writes the device
 * time of one pass and the bytes one pass moves (HOST doubles).  bytes >= 1 MiB,
 * reps >= 1; pick bytes well above the 256 MB last-level cache. */
tip_status tip_stream_ceiling(int32_t kind, int64_t bytes, int32_t reps, int32_t grid,
                              double* seconds_per_pass, double* bytes_per_pass, void* stream);

/* P(x) of every site (Alg. 5): DEVICE uint32 [V].  With odd factors in the
 * sides: the binary colour over the B binary levels, in [0, 2^LB). */
tip_status tip_hier_perm(int32_t ndim, const int64_t* dims, uint32_t* P_out, void* stream);

/* Probing vectors b_{m,comp}(y, comp) = z0(y, comp) H(P(y), bitrev_L(m)) for
 * m = m0 .. m0+count-1 (or the probe kind given, with stop_levels for
 * TIP_PROBE_STOPPED): DEVICE complex128 [count][V].  mask as in tip_params
 * (DEFAULT resolves with ncomp: 1 -> Z2, 3 -> Z4). */
tip_status tip_probe_vectors(int32_t ndim, const int64_t* dims, int32_t ncomp, int32_t mask,
                             uint64_t seed, int64_t m0, int64_t count, int32_t comp,
                             int32_t probe, int32_t stop_levels, double* out, void* stream);

/* Turn per-launch hipEvent timing of the stencil kernel on (1) or off (0). */
void tip_set_profiling(int32_t on);

/* Message for the last non-OK status returned on this thread. */
const char* tip_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TIP_H */
