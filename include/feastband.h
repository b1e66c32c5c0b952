/*
 * feastband.h -- C ABI of the MI355X banded FEAST spectrum-slicing library.
 *
 * The library computes eigenpairs of a band Hermitian (or real symmetric)
 * matrix B slice by slice with FEAST: contour-integral filtering by shifted
 * band solves, orthonormalisation and Rayleigh-Ritz, with slices placed and
 * checked by Sylvester inertia (the spectrum-slicing stage of PDESHEP,
 * Section 3 of the paper, with Algorithm alg:FEAST of Section 2.2).
 *
 * Conventions for every entry point
 *  - Arrays are column-major and 0-based.  "dev" marks a device pointer
 *    (memory of the current HIP device), "host" a host pointer.
 *  - stream is a hipStream_t (NULL = the null stream).  Work is queued on
 *    it; entry points that return host results synchronise it.
 *  - Workspace: the caller owns all memory.  Calling with work == NULL is a
 *    query: the required size in bytes is written to *lwork, nothing is
 *    launched and 0 is returned.  Otherwise *lwork must be at least that
 *    size and work must be 256-byte aligned device memory.
 *  - Return value: 0 on success; -k when argument k (1-based) is invalid,
 *    with nothing launched; -1000 - e for a HIP error e; FB_ERR_* codes
 *    below for other failures; a positive value where an entry point says so.
 *  - Inputs are never modified unless documented as in/out.
 *  - Calls that overlap on one device must use distinct workspaces.
 */
#ifndef FEASTBAND_H
#define FEASTBAND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FB_REAL64 1     /* real symmetric, double */
#define FB_COMPLEX128 2 /* complex Hermitian, interleaved (re, im) doubles */

#define FB_ERR_SINGULAR (-2001)   /* an exactly zero pivot in a shifted LU */
#define FB_ERR_NOT_BUILT (-2002)  /* no kernel for this device */
#define FB_ERR_CERTIFY (-2003)    /* a slice boundary could not be certified */
#define FB_ERR_NOMEM (-2004)      /* workspace or HBM budget below one unit of work */
#define FB_ERR_NONFINITE (-2005)  /* NaN or Inf in an input block */
#define FB_ERR_INTERNAL (-2006)
#define FB_ERR_TOO_LARGE (-2007)  /* beyond the fixed scratch of band_inertia_noalloc */

/* A band Hermitian matrix in LAPACK lower band storage (the compact band form
 * the paper keeps on every process, Section 3 "Proposed algorithm"):
 * ab[(i-j) + j*ldab] = B(i, j) for 0 <= i-j <= b, ab dev, dtype FB_REAL64
 * (double) or FB_COMPLEX128 (two doubles).  Imaginary parts of the diagonal
 * are ignored.  Requires 0 <= b < n, ldab >= b+1. */
typedef struct {
  int64_t n;
  int32_t b;
  int32_t dtype;
  int64_t ldab;
  const void* ab;
} fb_band;

/* Sylvester inertia of B - shift_k I for every shift (Section 3.1 "Spectrum
 * Partition": the LDL^H factorisation of A - s I counts the eigenvalues below
 * s; Section 3.2 uses two such counts to check every slice).  Computed by a
 * band LDL^H without pivoting in FP64, one factorisation per shift, all
 * shifts in one batched launch.  A pivot of magnitude below
 * eps^2 * ||B||_1 is counted in n_zero and replaced by its negative bound.
 * shifts: host, nshift doubles.  n_neg/n_zero/n_pos: host, nshift int32
 * each (n_zero and n_pos may be NULL).  Synchronises the stream. */
int band_inertia(const fb_band* B, int32_t nshift, const double* shifts,
                 int32_t* n_neg, int32_t* n_zero, int32_t* n_pos,
                 void* work, size_t* lwork, void* stream);

/* Bytes of the library's fixed device scratch used by band_inertia_noalloc
 * (one copy per device, held from the library's load until the process
 * ends). */
#define FB_NOALLOC_SCRATCH_BYTES (64 << 20)

/* band_inertia for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same counts as band_inertia, computed in a fixed library-owned device
 * scratch of FB_NOALLOC_SCRATCH_BYTES instead of a caller workspace.  The
 * call makes no device allocation of any kind.  The problem must fit the
 * scratch: the internal band copy takes (max(b,1) + 1) * n * 16 bytes plus
 * about 1 KB per 16 shifts, so n * (b + 1) up to about 4.1e6 entries;
 * larger problems return FB_ERR_TOO_LARGE with nothing launched.  Argument
 * errors as band_inertia (-1 band, -2 nshift, -3 shifts, -4 n_neg).  Every
 * call on a device shares that device's scratch: calls that overlap on one
 * device (other host threads, other streams) race and must be serialised by
 * the caller.  Synchronises the stream. */
int band_inertia_noalloc(const fb_band* B, int32_t nshift, const double* shifts,
                         int32_t* n_neg, int32_t* n_zero, int32_t* n_pos, void* stream);

/* Options of the shifted band solves. */
typedef struct {
  int32_t precision; /* 0: complex128 LU and solves (plain FP64).
                        1: complex64 LU and solves with FP32 accumulation,
                           refined in FP64 (residual from the FP64 band) */
  double ir_tol;     /* precision 1: stop refining a column once
                        ||y - A x||_2 / ||y||_2 <= ir_tol */
  int32_t ir_max;    /* precision 1: at most this many correction passes; a
                        column group whose residual a pass did not halve has
                        stagnated and stops early (then, above ir_tol, the
                        complex128 fallback) */
  int32_t tile;      /* right-hand-side columns per work item; 0 = default */
} fb_solve_opts;

/* Batched shifted band solves, the building block of the FEAST filter
 * (Section 2.2, equation eq:feast_L2: one factorisation of (z_j I - B) per
 * integration node, then solves with many right-hand sides).
 * For every system s: factor A_s = z_s I - B by band LU with partial
 * pivoting, then X[s] = A_s^{-1} Y[s] and, if XH[s] != NULL,
 * XH[s] = A_s^{-H} Y[s].
 *  z      host, 2*nsys doubles: (re, im) of each shift
 *  m      host, nsys: columns of system s (0 allowed)
 *  Y      host array of nsys dev pointers to complex128 n x m[s] blocks,
 *         leading dimension ldy[s] >= n (systems may share a block)
 *  X, XH  host arrays of nsys dev pointers to complex128 outputs,
 *         leading dimension ldx[s] >= n; XH itself or XH[s] may be NULL
 *  resid  host, nsys or NULL: max over the columns of system s (N and H)
 *         of ||y - A x||_2 / ||y||_2 after the call, computed in FP64
 *  passes host, nsys or NULL: refinement passes used (precision 1); -1
 *         when the residual stayed above ir_tol after ir_max passes and the
 *         system was factored again and solved in complex128 (a warning:
 *         the solution is the FP64 one)
 * Returns FB_ERR_NONFINITE (nothing solved) when B or a Y block holds a
 * NaN or an infinity, FB_ERR_SINGULAR if a pivot is exactly zero.
 * Precision 1 returns the number of systems whose residual is still above
 * ir_tol after the complex128 fallback (0 when all converged). */
int band_shifted_solve(const fb_band* B, int32_t nsys, const double* z,
                       const int32_t* m, const void* const* Y,
                       const int64_t* ldy, void* const* X, void* const* XH,
                       const int64_t* ldx, double* resid, int32_t* passes,
                       const fb_solve_opts* o, void* work, size_t* lwork,
                       void* stream);

/* FEAST options. */
typedef struct {
  int32_t n_nodes;     /* Gauss-Legendre nodes on the upper half circle (8) */
  double tol;          /* eigen-residual ||Bx - lx||_2/||B||_1 target (1e-10) */
  int32_t max_iter;    /* FEAST iterations (20) */
  int32_t precision;   /* as fb_solve_opts.precision */
  double ir_tol;       /* as fb_solve_opts.ir_tol (1e-12) */
  int32_t ir_max;      /* as fb_solve_opts.ir_max (4) */
  int32_t batched;     /* 0: one launch sequence per slice; 1: all slices of
                          a sweep in shared batched launches */
  double hbm_budget;   /* bytes of device memory the workspace may take,
                          0 = half of the device's memory.  It sets how many
                          (node, direction) pairs share one batched launch:
                          each pair needs an n x m0 complex128 buffer per
                          slice (batched = 0 uses one) */
  int32_t pairs;       /* > 0: exactly this many pairs per batched launch
                          (capped at 2 n_nodes), overriding hbm_budget */
  int32_t rule;        /* quadrature of the contour integral (Section 2.2,
                          eq:integral): 0 Gauss-Legendre in the angle of the
                          upper half, 1 trapezoid (midpoint) rule with 2 n_nodes
                          equispaced angles on the whole curve, of which the
                          n_nodes on the upper half are used, 2 the Zolotarev
                          rational filter (Section 2.2 names it): the best
                          uniform rational approximation of sign composed
                          with a Moebius map of the slice, n_nodes poles on
                          the upper half of the circle through the slice
                          ends; within its error delta of 1 on the inner
                          fraction |lambda - c| <= ratio r and of 0 beyond
                          r / ratio (c, r: centre and half width) */
  double ratio;        /* rules 0 and 1: vertical over horizontal semi-axis
                          of the contour through the slice ends: 1 (or 0) the
                          circle, other positive values an ellipse
                          z(t) = c + r (cos t + i ratio sin t); rule 2: the
                          inner fraction, 0 < ratio < 1 */
  const char* tune_cache; /* path of a file written by fb_autotune, or NULL:
                          its choices of the solve variant are loaded first */
  int32_t graph;       /* feast_filter, batched with every (node, direction)
                          pair in one launch and a non-null stream: 1 captures
                          the sweep (factorisations, solves, the refinement
                          passes with their device-side decisions, node sum)
                          in a HIP graph on the first call and replays it on
                          later calls with the same pointers, sizes and
                          options; a refinement that stagnates is redone by
                          direct launches with the complex128 fallback */
  double ir_from;      /* feast_band_slice with precision 1: a slice's
                          complex64 solves run without refinement (and without
                          the FP64 residuals) while the m_i-th smallest
                          eigen-residual of its in-slice Ritz pairs is above
                          ir_from, for at most 3 iterations, then refined;
                          the convergence test is on FP64 eigen-residuals
                          either way.  0 refines from the first iteration */
} fb_feast_opts;

/* FEAST on the slices [lo_i, hi_i) of B (Algorithm alg:FEAST, Section 2.2,
 * with the slice validation of Section 3.2).  Nodes z_j = z(t_j) on the upper
 * half of the contour, weights w_j = (dt_j / (2 pi)) z'(t_j) / i with dt_j the
 * quadrature weight in the angle (Gauss-Legendre: (pi/2) omega_j; trapezoid:
 * pi / n_nodes):
 *   repeat: Q = sum_j [w_j (z_j I - B)^{-1} Y + conj(w_j)(z_j I - B)^{-H} Y]
 *           (real B: Q = sum_j 2 Re[w_j (z_j I - B)^{-1} Y]),
 *           orthonormalise Q, A_q = Q^H B Q, A_q W = W Lambda, X = Q W,
 *   until the number of Ritz pairs in [lo_i, hi_i) with
 *   ||B x - l x||_2 / ||B||_1 <= tol equals the exact count m_i; Y <- X.
 *  lo, hi      host, nslice doubles, lo_i < hi_i
 *  m0          host, nslice: subspace sizes (columns of Y[i]), m0_i >= 1
 *  m_expected  host, nslice or NULL: exact counts; NULL = computed here by
 *              band_inertia at lo_i and hi_i
 *  Y           host array of dev pointers, in/out: on entry the start block
 *              (n x m0_i, dtype of B), on exit all Ritz vectors, the
 *              converged in-slice pairs first in ascending order
 *  ldy         host, nslice: leading dimensions (>= n)
 *  evals,resid host arrays of dev pointers to m0_i doubles: Ritz values and
 *              eigen-residuals in the order of the columns of Y
 *  m_found, iters, info  host, nslice each.  info: 0 ok, 1 not converged in
 *              max_iter, 2 count mismatch (m0 too small or a missed
 *              eigenvalue: rerun with a larger m0), 3 converged, but a
 *              refined complex64 solve of the slice stagnated above ir_tol
 *              and was redone in complex128 (a warning), 4 rank-deficient
 *              filtered block (a truncated basis was used), 5 m0 < m
 * The filtered block is orthonormalised as band_rayleigh_ritz describes
 * (Cholesky QR twice, the eigen passes when it does not apply).
 * Returns 0, or the number of slices with info in {1, 2, 5};
 * FB_ERR_NONFINITE (nothing solved) when B or a start block holds a NaN or
 * an infinity. */
int feast_band_slice(const fb_band* B, int32_t nslice, const double* lo,
                     const double* hi, const int32_t* m0,
                     const int32_t* m_expected, void* const* Y,
                     const int64_t* ldy, double* const* evals,
                     double* const* resid, int32_t* m_found, int32_t* iters,
                     int32_t* info, const fb_feast_opts* o, void* work,
                     size_t* lwork, void* stream);

/* Orthonormalisation and Rayleigh-Ritz of given blocks, the step of
 * Algorithm alg:FEAST that follows the filter (Section 2.2): for every block
 * Q_i, an orthonormal basis U_i of span(Q_i), the Ritz values and vectors of
 * B on it (U_i^H B U_i W = W Lambda, X_i = U_i W, ascending) and their
 * residuals ||B x - l x||_2 / ||B||_1.  The basis is formed by Cholesky QR
 * applied twice to the column-equilibrated block (D scales every column to
 * unit norm: (Q D)^H (Q D) = R1^H R1, Q1 = Q D R1^{-1}, Q1^H Q1 = R2^H R2,
 * U = Q1 R2^{-1}) while every pivot r_jj^2 of both unit-diagonal Gram
 * matrices exceeds 1e-12; otherwise by two eigen-decomposition passes of the
 * Gram matrix that drop directions below 1e-14 of the largest (rank < m_i).
 *  m      host, nblk: columns of each block (0 allowed, at most 4096)
 *  Q      host array of dev pointers, n x m_i in the dtype of B, leading
 *         dimension ldq[i] >= n (not modified)
 *  X      host array of dev pointers, out: the Ritz vectors in the first
 *         rank_i columns (dtype of B), leading dimension ldx[i] >= n
 *  evals, resid  host arrays of dev pointers to m_i doubles (first rank_i)
 *  rank   host, nblk: dimension of the basis
 *  path   host, nblk or NULL: 0 Cholesky QR, 1 eigen-decomposition passes
 * Synchronises the stream. */
int band_rayleigh_ritz(const fb_band* B, int32_t nblk, const int32_t* m, const void* const* Q,
                       const int64_t* ldq, void* const* X, const int64_t* ldx,
                       double* const* evals, double* const* resid, int32_t* rank,
                       int32_t* path, void* work, size_t* lwork, void* stream);

#define FB_PLAN_EQUAL_WIDTH 0 /* Approach-2 of Section 3.1: equal widths */
#define FB_PLAN_EQUAL_COUNT 1 /* Approach-1 of Section 3.1: equal counts */
#define FB_PLAN_LEARNED 2     /* equal counts, search guided by the planner network */

typedef struct {
  int32_t mode;       /* FB_PLAN_* */
  int32_t K;          /* number of slices */
  double lo, hi;      /* interval; NaN = the Gershgorin bound moved outward by
                         4 cert_delta ||B||_1 + 1e-12 ||B||_1 (equal count and
                         LEARNED; EQUAL_WIDTH needs both) */
  double count_tol;   /* equal count: accept |n_-(s) - target| <= floor(tol*total/K) */
  double cert_delta;  /* boundaries keep eigenvalues farther than cert_delta*||B||_1 */
  int32_t max_rounds; /* bisection rounds */
  const void* planner;/* FB_PLAN_LEARNED: dev pointer to the network weights
                         (fb_planner_bytes() bytes), or NULL for a uniform
                         prior over [lo, hi] (interpolation search) */
  uint64_t seed;      /* FB_PLAN_LEARNED: probe seed of the features */
  int64_t nev;        /* equal count / LEARNED: > 0 places hi so that [lo, hi)
                         holds exactly the lowest nev eigenvalues above lo */
  const int32_t* targets; /* equal count / LEARNED: host, K desired slice
                         counts (their sum fixes hi exactly, as nev), or NULL
                         for equal counts */
} fb_plan_opts;

/* Slice placement by exact inertia (Section 3.1 "Spectrum Partition",
 * Approach-1 and Approach-2; slice counts m_i = n_-(s_i) - n_-(s_{i-1}) as in
 * Section 3.2).  Every boundary is certified: n_-(s - d) = n_-(s + d) with
 * d = cert_delta * ||B||_1, else it is moved to the first certified point of
 * s + 2 d k, k = 1, -1, 2, -2, ...  Equal count bisects all open boundaries
 * together, one batched inertia launch per round; the bisection that places
 * hi for nev (or targets) evaluates its next levels (up to 63 midpoints) in
 * one launch and keeps the points it visits.  LEARNED predicts the
 * eigenvalue distribution from the band features (band_features) with the
 * planner network and searches every boundary by inverting that prediction
 * inside the current bracket, rescaled by the exact counts at its ends (a
 * bracket that did not halve in two rounds is bisected); the final plan is
 * certified and exact whatever the network predicts.
 *  bounds host, K+1 doubles; counts host, K; n_inertia host (may be NULL):
 *  number of shifts factorised, speculative ones included.  Synchronises
 *  the stream. */
int slice_plan(const fb_band* B, const fb_plan_opts* o, double* bounds,
               int32_t* counts, int32_t* n_inertia, void* work, size_t* lwork,
               void* stream);

/* Options of slice placement from the previous eigenvalues of a sequence. */
typedef struct {
  int32_t K;          /* wanted slices; the clustering may return fewer */
  int64_t nev;        /* the lowest nev eigenvalues are covered, 1 <= nev <= nprev */
  double alpha;       /* relative step of the bound searches (1e-3) */
  int32_t m1;         /* gap multiple of the bound step (6) */
  double cert_delta;  /* as fb_plan_opts.cert_delta (1e-8) */
  int32_t max_sweeps; /* clustering sweeps (100) */
  int32_t max_steps;  /* steps of each bound search (1000) */
} fb_prev_opts;

/* Slices for the lowest nev eigenvalues of B from the eigenvalues of the
 * previous matrix of a sequence (Section 3.1 "K-means Clustering" with
 * Algorithm alg:kmeans; bounds of Section 3.2 "Validation and Other
 * Details", Algorithm alg:lower_upper):
 *   the previous d_1 <= ... <= d_nev are clustered into at most K groups of
 *   consecutive values (simplified one-dimensional k-means: initial groups of
 *   floor(nev/K) or floor(nev/K)+1 points, the first nev mod K larger; each
 *   sweep moves every boundary, in order, to the first point above the
 *   midpoint of the two neighbouring group centroids, a centroid being the
 *   midpoint of the group's extreme points; an emptied group is dropped;
 *   until no boundary moves or max_sweeps); an interior boundary is the
 *   midpoint of the points on its two sides;
 *   b_K = d_nev + s, s = max(alpha |d_nev|, m1 (d_nev - d_nev-1),
 *   4 cert_delta ||B||_1 + 1e-12 ||B||_1), advanced by s until
 *   n_-(b_K) >= nev; b_0 = d_1 - s0 (s0 likewise from d_1 and d_2 - d_1),
 *   moved down by s0 until n_-(b_0) = 0;
 *   every boundary is then certified as in slice_plan and the counts are
 *   exact inertia differences.
 *  prev    host, nprev ascending doubles
 *  bounds  host, K+1 doubles (the first K_out+1 are set); counts host, K
 *  K_out   host (may be NULL): slices returned, <= K
 *  n_inertia host (may be NULL): shifts factorised
 * Returns 0; -k for invalid argument k (nothing launched); FB_ERR_CERTIFY
 * when a boundary cannot be certified, a bound search does not end within
 * max_steps, or certified boundaries are out of order.  Synchronises the
 * stream. */
int slice_plan_prev(const fb_band* B, const double* prev, int64_t nprev,
                    const fb_prev_opts* o, double* bounds, int32_t* counts,
                    int32_t* K_out, int32_t* n_inertia, void* work, size_t* lwork,
                    void* stream);

/* Boundary certification for a matrix of a sequence whose slices were placed
 * on an earlier one (the per-slice validation of Section 3.2 before FEAST
 * runs on the new matrix): bounds[i] (host, nb ascending doubles, in/out)
 * is replaced by the first of s = bounds[i] + 2 d k, k = 0, 1, -1, ..., 32,
 * -32 (d = cert_delta ||B||_1) with n_-(s - d) = n_-(s + d), so that no
 * eigenvalue lies within d of it.  neg (host, nb) receives n_-(bounds[i]),
 * counts (host, nb - 1) the exact slice counts neg[i+1] - neg[i], and m0
 * (host, nb - 1, or NULL) the subspace sizes fb_m0_rule(counts[i]).
 * n_inertia (host or NULL): inertia evaluations used.  Returns 0,
 * FB_ERR_CERTIFY when a boundary cannot be certified or two of them meet,
 * or a negative argument index. */
int slice_certify(const fb_band* B, int32_t nb, double* bounds, double cert_delta,
                  int32_t* neg, int32_t* counts, int32_t* m0, int32_t* n_inertia,
                  void* work, size_t* lwork, void* stream);
/* Subspace size for a slice of m eigenvalues: max(ceil(1.5 m), m + 10) (the
 * paper's rule of a margin over the count, Section 3.2, with the 1.5 factor
 * of the configurations); -1 for m < 0.  Host only. */
int32_t fb_m0_rule(int32_t m);

/* Filter application only (the shifted solves of one FEAST iteration,
 * Section 2.2, eq:feast_L2 and the quadrature sum Q = sum_j w_j Q^(j)):
 * factor z_j I - B for every node of every slice, solve with Y[i]
 * (N and, for complex B, H), refine (precision 1) and accumulate
 *   Q[i] = sum_j [w_j (z_j I - B)^{-1} Y[i] + conj(w_j) (z_j I - B)^{-H} Y[i]]
 * (real B: Q[i] = sum_j 2 Re[w_j (z_j I - B)^{-1} Y[i]]), nodes in order.
 *  Y, Q   host arrays of dev pointers, n x m[i] in the dtype of B, leading
 *         dimensions ldy[i], ldq[i] >= n (Y is not modified)
 *  resid  host, nslice or NULL: max over nodes, directions and columns of
 *         ||y - A x||_2 / ||y||_2 in FP64 (extra residual pass for precision 0)
 *  passes host, nslice or NULL: most refinement passes of any tile; -1 when
 *         a system of the slice was refactored and solved in complex128
 *         after its refinement stayed above ir_tol
 * o->max_iter and o->tol are ignored; o->hbm_budget and o->pairs set how
 * many (node, direction) pairs share a launch.  Returns 0, or for
 * precision 1 the number of slices with a tile above ir_tol after ir_max. */
int feast_filter(const fb_band* B, int32_t nslice, const double* lo, const double* hi,
                 const int32_t* m, const void* const* Y, const int64_t* ldy,
                 void* const* Q, const int64_t* ldq, double* resid, int32_t* passes,
                 const fb_feast_opts* o, void* work, size_t* lwork, void* stream);

/* Launch timing, a tracing aid.  While enabled, every launch of the classes
 * below is bracketed by HIP events on its own stream.  fb_profile_enable
 * resets the counters; fb_profile_read waits for the recorded events and
 * returns, for one class, the number of launches, their summed duration in
 * milliseconds and their summed algorithmic work (flops; for FB_PROF_SOLVE
 * 24 n b per right-hand-side column, for FB_PROF_RESID 8 (2b+1) n per
 * column, for FB_PROF_LU 16 n b^2 per system, for FB_PROF_INERTIA 4 n b^2
 * per shift). */
#define FB_PROF_LU 0
#define FB_PROF_INVERT 1
#define FB_PROF_SOLVE 2
#define FB_PROF_RESID 3
#define FB_PROF_INERTIA 4
#define FB_PROF_JACOBI 5
#define FB_PROF_GEMM 6
#define FB_PROF_BANDMM 7
#define FB_PROF_NCLASS 8
int fb_profile_enable(int32_t on);
int fb_profile_read(int32_t cls, int64_t* launches, double* ms, double* work);

/* Autotuner of the block-solve kernel (the tile width of right-hand sides per
 * work item and whether factor fragments are prefetched a product ahead):
 * factors nsys shifted systems of B in the given precision (0: complex128,
 * 1: complex64), times every variant that fits in LDS on the N and H solves
 * of m right-hand sides each with HIP events, and keeps the fastest for this
 * precision and block size for the rest of the process.  When cache_path is
 * not NULL the choice is appended to it as one JSON line.  chosen/ms (host,
 * may be NULL) receive the variant and its time per sweep. */
int fb_autotune(const fb_band* B, int32_t precision, int32_t nsys, int32_t m,
                const char* cache_path, int32_t* chosen, double* ms, void* work,
                size_t* lwork, void* stream);
/* Load choices written by fb_autotune; returns how many were read, or -1. */
int fb_tune_load(const char* cache_path);

/* Stochastic Chebyshev moments of B, the density-of-states estimate the
 * paper names as the matrix-vector alternative to inertia (Section 3.1):
 * with Bh = (B - c I)/h, c = (g_lo + g_hi)/2, h = 1.01 (g_hi - g_lo)/2 from
 * the Gershgorin bounds, mu[p*(K+1) + k] = v_p^T T_k(Bh) v_p / n for
 * k = 0..K, the Rademacher probes being v_p(i) = 1 - 2 (SplitMix64(seed*2^40
 * + p*2^32 + i) & 1), p = 0..P-1.  mu host, P*(K+1) doubles; gersh host (may
 * be NULL), 3 doubles: g_lo, g_hi, ||B||_1.  Synchronises the stream. */
int band_cheb_moments(const fb_band* B, int32_t K, int32_t P, uint64_t seed, double* mu,
                      double* gersh, void* work, size_t* lwork, void* stream);

/* The 80 planner features of B (host, doubles): Gershgorin bounds over
 * ||B||_1, the mean and the spread over 20 probes of the Chebyshev moments
 * mu_1..mu_16, the Jackson-damped Chebyshev estimate of the fraction of
 * eigenvalues below 32 evenly spaced points of the Gershgorin interval, and
 * 14 band statistics (size, bandwidth, type, diagonal moments, off-diagonal
 * energy, norms).  Synchronises the stream. */
int band_features(const fb_band* B, uint64_t seed, double* feat, void* work, size_t* lwork,
                  void* stream);

/* Bytes of the planner network's FP32 weights: W1 (80 x 256), b1 (256),
 * W2 (256 x 256), b2 (256), W3 (256 x 64), b3 (64), row-major, packed. */
size_t fb_planner_bytes(void);

/* Network forward for a batch: x dev float [batch x 80] row-major, out dev
 * float [batch x 64]; ReLU hidden layers; every product takes its operands
 * rounded to BF16 and accumulates in FP32 (MFMA).  Workspace as above. */
int planner_forward(const void* weights, int32_t batch, const float* x, float* out,
                    void* work, size_t* lwork, void* stream);

/* One training step of the network on a batch: forward, mean squared error
 * against target (dev float [batch x 64]), backward (BF16 operands, FP32
 * accumulation), then, unless grads is given, Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected with step t >= 1) on the FP32 weights with
 * opt_state = [m | v] (dev, 2 fb_planner_bytes(), zero before step 1).
 * grads (dev, fb_planner_bytes(), may be NULL): receives the gradients and
 * no update is made.  loss (host, may be NULL): the batch loss; giving it
 * synchronises the stream. */
int planner_train_step(void* weights, void* opt_state, int32_t batch, const float* x,
                       const float* target, float lr, int32_t t, float* loss, void* grads,
                       void* work, size_t* lwork, void* stream);

const char* fb_strerror(int code);

/* Nodes z_j and weights w_j, j = 1..k, of the filter
 * r(x) = sum_j 2 Re[w_j / (z_j - x)] that FEAST applies on the slice
 * [lo, hi) (Section 2.2, the quadrature of eq:integral), for the rule and
 * ratio of fb_feast_opts; the lower half of the contour is the conjugate of
 * the upper.  z and w: caller-owned host arrays of 2k doubles, written as
 * interleaved (real, imaginary) pairs.  Host only: touches no device.
 * Returns 0; -1 / -2 for a non-finite lo or hi <= lo; -3 for k outside
 * 1..64; -4 for an unknown rule; -5 for a ratio the rule does not take;
 * -6 / -7 for a null z / w. */
int fb_contour(double lo, double hi, int32_t k, int32_t rule, double ratio, double* z,
               double* w);

/* Device properties used by the library (for reports): compute units and
 * the device name, written to name (cap bytes). */
int fb_device_info(int32_t* cus, char* name, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif /* FEASTBAND_H */
