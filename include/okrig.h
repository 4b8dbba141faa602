/*
 * okrig.h - C ABI of the MI355X edge-preserved ordinary-kriging library.
 *
 * The library fills the missing voxels between known 2D slices along Z
 * (Section 4.1 of "Fast 3D Volumetric Image Reconstruction from 2D MRI
 * Slices by Parallel Processing"): known slices are placed into the output
 * volume (Algorithm 1, step 3) and every missing voxel is estimated by
 * ordinary kriging (Appendix A with a single constant predictor) over its
 * neighbours in the two adjacent known slices, with neighbours that would
 * cross an edge of the supplied edge mask left out (Section 4.1.2).
 *
 * Conventions shared by every entry point
 *   - All array arguments named d_* are DEVICE pointers owned by the caller;
 *     the library never frees them and keeps no reference after the call's
 *     stream work completes. Arrays are C-contiguous, slice index slowest:
 *     slices[s][y][x], s < nslices, y < ny, x < nx.
 *   - Work is enqueued on the HIP stream given at plan creation and is
 *     asynchronous unless stated otherwise.
 *   - Every function returns an okr_status; no C++ exception crosses the ABI.
 *     Argument and shape errors are detected on the host before any device
 *     work is enqueued. okr_plan_last_error() returns a message for the last
 *     failing call on a plan.
 *   - A plan is not thread-safe; distinct plans are independent.
 *
 * Geometry (readings where the paper is silent; the oracle uses the same)
 *   - Output volume: (nslices-1)*upsample + 1 slices; known slice s is copied
 *     bit-exactly to z = s*upsample, where the kriging variance is 0.
 *   - Distances are Euclidean in output-voxel units (pixels in-plane, known
 *     slices `upsample` apart).
 *   - Candidate neighbours of target (x, y, g*f + t), 0 < t < f: offsets
 *     |dx|, |dy| <= radius in slices g ("lower", s = 0) and g+1 ("upper",
 *     s = 1); out-of-image candidates are dropped. Canonical candidate index
 *     c = s*W*W + (dy+radius)*W + (dx+radius), W = 2*radius + 1.
 *   - Edge rule: a candidate is kept iff no pixel of its discrete path from
 *     the centre is an edge in its own slice's mask; the path is
 *     p_k = (rha(k*dx/L), rha(k*dy/L)), k = 1..L, L = max(|dx|, |dy|), rha =
 *     round half away from zero. The centre (0, 0) is always kept.
 *   - Floor: with fewer than min_points kept, rejected in-image candidates are
 *     added in the order (dx^2+dy^2, lower slice first, dy, dx).
 *   - Covariance (GSLIB convention): Cov(0) = sill (total sill),
 *     Cov(h > 0) = (sill - nugget) * rho(h) with practical range a:
 *       spherical   rho = 1 - 1.5 h/a + 0.5 (h/a)^3 for h < a, else 0
 *       exponential rho = exp(-3 h / a)
 *       gaussian    rho = exp(-3 h^2 / a^2)
 *   - Estimate z_hat = sum_i w_i z_i and variance sill - w^T c0 - mu, with
 *     [[C, 1], [1^T, 0]] [w; mu] = [c0; 1] (Appendix A, extended covariance
 *     system with Lagrange multiplier).
 */
#ifndef OKRIG_H
#define OKRIG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t okr_status;
#define OKR_OK                0
#define OKR_E_INVALID_ARG     1  /* null pointer, bad enum or parameter value */
#define OKR_E_SHAPE           2  /* sizes out of range or overflowing */
#define OKR_E_NONFINITE       3  /* non-finite known voxel (reported at a sync) */
#define OKR_E_DEVICE          4  /* a HIP call failed */
#define OKR_E_OOM             5  /* device or pinned allocation failed */
#define OKR_E_UNSUPPORTED     6  /* valid request the library does not serve */
#define OKR_E_NOT_CONVERGED   7  /* strict mode: a system failed every precision */
#define OKR_E_CAPACITY        8  /* caller's output buffer too small (size reported) */

typedef enum { OKR_SPHERICAL = 0, OKR_EXPONENTIAL = 1, OKR_GAUSSIAN = 2 } okr_model;

/* Arithmetic of the factorisation. Assembly and read-out are FP32 except in
 * OKR_FP64. MIXED_* use split low-precision MFMA products (hi + lo parts) with
 * FP32 accumulation, optionally an FP64-residual correction of every system's
 * estimate (refine_max = 1), and an FP64 re-solve of systems whose pivots flag
 * instability or whose error bound exceeds refine_tol. */
typedef enum { OKR_FP32 = 0, OKR_MIXED_FP16 = 1, OKR_MIXED_BF16 = 2, OKR_FP64 = 3 } okr_precision;

/* BATCHED: selection, size bucketing and one persistent factorisation launch,
 * one Cholesky per (column, gap) shared by its f-1 targets.
 * PLAIN_PER_VOXEL: the comparison kernel: one wavefront per kriged voxel,
 * nothing shared between voxels: its own selection, covariances from the FP64
 * tables rounded to FP32, Cholesky of C in LDS (FP32), the bordered solution
 * from C^{-1} 1 and C^{-1} c0, and with refine_max = 1 one step of iterative
 * refinement with the FP64 residual of the bordered system; estimate and
 * variance summed in FP64.
 * PATTERN_CACHE: BATCHED, except that the systems keeping the whole window
 * (the same matrix for all of them, by translation invariance) take weights
 * and variances computed once per launch in FP64 and applied as FP64 dot
 * products, and the systems of the size classes that drop at most 32
 * candidates of the window take theirs from the window's FP64 inverse (the block-inverse identity, one k x k solve per
 * system for its k dropped candidates); the other systems are solved as in
 * BATCHED at the plan's precision. */
typedef enum { OKR_ALGO_BATCHED = 0, OKR_ALGO_PLAIN_PER_VOXEL = 1,
               OKR_ALGO_PATTERN_CACHE = 2 } okr_algo;

typedef struct {
  int32_t model;        /* okr_model */
  double  nugget;       /* 0 <= nugget < sill */
  double  sill;         /* total sill, > 0 */
  double  range;        /* practical range, > 0 */
} okr_variogram;

typedef struct {
  int32_t nx, ny;       /* slice width / height, 1..65535 */
  int32_t nslices;      /* known slices, 1..65535 */
  int32_t upsample;     /* f, 1..15: output has (nslices-1)*f + 1 slices */
  int32_t radius;       /* r, 0..3: window (2r+1) x (2r+1) x 2 */
  int32_t min_points;   /* neighbour floor, 1..2*(2r+1)^2; 4 is the usual value */
  int32_t precision;    /* okr_precision */
  int32_t algo;         /* okr_algo */
  double  refine_tol;   /* >= 0: per-voxel tolerance on the relative error
                           |z_hat - z*| / max(|z*|, 0.01*max|known voxel|) (0 = no
                           check). Precision control uses kappa_w, the 2-norm
                           condition number of the covariance matrix of the whole
                           window, computed on the host in FP64 for each new
                           variogram; every system's covariance matrix is a
                           principal submatrix of it, so no system is worse
                           conditioned (eigenvalue interlacing). With u the unit
                           roundoff of the factorisation (2^-24 FP32, 2^-22 split
                           FP16, 2^-16 split BF16):
                           MIXED_* with refine_max = 0: a system whose indicator
                           kappa_w*u*s / max(|z_hat|, 0.01*max|known voxel|)
                           exceeds refine_tol for some target (s: the power of
                           two above the spread of its data) is re-solved in FP64;
                           MIXED_* with refine_max = 1: every system takes the
                           FP64-residual correction, which is exact up to
                           (lambda - lambda~)'h (lambda~ = computed weights and
                           multipliers, h = FP64 residual of the dual system);
                           with the weights' relative error taken as
                           min(1, 10*kappa_w*u), a system whose resulting bound
                           min(1, 10*kappa_w*u) * (|w_t| |h_w| + |phi_t| |Q'nu_w|)
                           exceeds refine_tol * max(|z_hat|, 0.01*max|known voxel|)
                           for some target is unconverged: re-solved in FP64,
                           flagged (bit 32) and counted (n_refine_unconverged).
                           Where the full-window system itself fails its test
                           (FP32: kappa_w*2^-24 > refine_tol; refine_max = 0:
                           kappa_w*u > refine_tol; refine_max = 1:
                           min(1, 10*kappa_w*u)*kappa_w*u > refine_tol), every
                           system is solved in FP64 directly instead, flagged
                           (bit 4) and counted in n_fp64_fallback as re-solved
                           (results equal the FP64 launch bit for bit; the
                           environment variable OKR_NO_DIRECT_FP64=1 keeps the
                           low-precision pass with its per-system checks).
                           Ignored by FP64. Systems with a non-positive pivot are
                           always re-solved in FP64. */
  int32_t refine_max;   /* MIXED_*: 0 = no correction (the low-precision
                           factorisation's own read-out); 1 = the FP64-residual
                           correction, taken once (it squares the factorisation's
                           relative error; what it cannot reach is re-solved in
                           FP64, see refine_tol). Other values: OKR_E_INVALID_ARG. */
  int32_t strict;       /* 1: OKR_E_NOT_CONVERGED is returned at the next sync if a
                           system met a non-positive pivot in its FP64 re-solve */
  int32_t drift;        /* 0: ordinary kriging (Appendix A with the constant
                           predictor). 1: universal kriging with a linear trend
                           across the gap: Appendix A with the predictors 1 and
                           the point's slice (0 lower, 1 upper; t/f at target
                           t). Needs BATCHED or PATTERN_CACHE;
                           upsample <= 14. Systems always hold points of both
                           slices (the centres are always kept), so the
                           extended system is regular. */
} okr_problem;

typedef struct okr_plan okr_plan;   /* opaque: workspace, tables, launch state */

typedef struct {
  int64_t n_systems;          /* (column, gap) systems in the last execute */
  int64_t n_kriged;           /* kriged voxels in the last execute */
  int64_t bucket[128];        /* systems per neighbour count n (index n) */
  int64_t n_floor_filled;     /* systems whose neighbour set used the floor */
  int64_t n_refined;          /* systems that took the FP64-residual correction */
  int64_t n_fp64_fallback;    /* systems re-solved in FP64 */
  int64_t n_nonpositive_pivot;/* systems with a non-positive pivot in the first pass */
  double  max_kappa_est;      /* largest pivot-ratio condition estimate */
  double  phase_ms[13];       /* with profiling on: summed device time per phase since the
                                 last okr_stats_get: 0 placement, 1 tables, 2 selection,
                                 3 bucketing, 4 batched solve, 5 FP64 re-solve,
                                 6 plain per-voxel kernel, 7 leave-one-slice-out,
                                 8 full-window pattern weights + application (the
                                 systems served from the window's inverse count
                                 under 4),
                                 9 marching cubes, edge post-pass: 10 shearlet
                                 coefficients, 11 edge thinning, 12 chain tracing and
                                 re-routing (with the copy of the input to the output) */
  int64_t phase_calls[13];    /* launches timed per phase */
  int64_t n_not_converged;    /* systems whose FP64 re-solve also met a non-positive pivot */
  int64_t n_refine_unconverged; /* systems whose correction left refine_tol unmet (each
                                   re-solved in FP64, so also in n_fp64_fallback) */
  double  kappa_window;       /* condition number of the full-window covariance matrix
                                 used by the last execute's precision control (0 if
                                 refine_tol was 0) */
  int32_t direct_fp64;        /* 1 if the last execute solved every system in FP64
                                 directly (see refine_tol) */
} okr_stats;

#define OKR_PHASE_PLACE 0
#define OKR_PHASE_TABLES 1
#define OKR_PHASE_SELECT 2
#define OKR_PHASE_BUCKET 3
#define OKR_PHASE_SOLVE 4
#define OKR_PHASE_FALLBACK 5
#define OKR_PHASE_PLAIN 6
#define OKR_PHASE_LOSO 7
#define OKR_PHASE_PATTERN 8
#define OKR_PHASE_MESH 9
#define OKR_PHASE_EDGE_SHEAR 10
#define OKR_PHASE_EDGE_THIN 11
#define OKR_PHASE_EDGE_TRACE 12
#define OKR_NUM_PHASES 13

/* Create a plan for one problem shape. `hip_stream` is a hipStream_t (NULL =
 * the default stream). Validates every field (OKR_E_INVALID_ARG / SHAPE /
 * UNSUPPORTED), allocates the workspace (OKR_E_OOM) and returns the plan in
 * *out. The caller destroys it with okr_plan_destroy. */
okr_status okr_plan_create(const okr_problem* problem, void* hip_stream, okr_plan** out);

/* Reconstruct the volume (Algorithm 1 steps 3-4, Section 4.1.2).
 *   d_slices   float32 [nslices][ny][nx], required
 *   d_edge     uint8   [nslices][ny][nx], nonzero = edge; NULL = no mask
 *   d_volume   float32 [(nslices-1)*f+1][ny][nx], required
 *   d_variance float32, same shape as d_volume; NULL = not written
 *   d_flags    uint8 [(nslices-1)][ny][nx] per (column, gap) system; NULL =
 *              not written. Bits: 1 floor-filled, 2 FP64-residual correction,
 *              4 FP64 re-solve, 8 non-positive pivot in the first pass,
 *              16 non-positive pivot in the FP64 re-solve as well,
 *              32 correction did not reach refine_tol (re-solved in FP64).
 * Input and output buffers must not overlap. */
okr_status okr_execute(okr_plan* plan, const okr_variogram* vario,
                       const float* d_slices, const uint8_t* d_edge,
                       float* d_volume, float* d_variance, uint8_t* d_flags);

/* Neighbour selection only (the integer part of okr_execute), for callers
 * and tests that need the kept sets.
 *   d_bits  uint64 [(nslices-1)*ny*nx][2]: bit c of the 128-bit word of
 *           system (g, y, x) is canonical candidate c (word 0 = bits 0..63)
 *   d_count uint8  [(nslices-1)*ny*nx]: number of kept candidates */
okr_status okr_select(okr_plan* plan, const uint8_t* d_edge, uint64_t* d_bits, uint8_t* d_count);

/* Leave-one-slice-out loss of a variogram: every known slice s in
 * 1..nslices-2 is predicted from slices s-1 and s+1 (at distance 1 each, the
 * geometry of upsample 2) with the plan's window and edge rule, and
 * *d_loss (device double) receives the mean of (z_hat - z)^2 over all those
 * voxels. With a drift plan (problem.drift = 1) the predictions use the
 * slice predictor as the volume path does (q0 = (1, 1/2)). Requires a plan
 * with upsample == 2, nslices >= 3 and a batched algorithm. */
okr_status okr_loso_forward(okr_plan* plan, const okr_variogram* vario, const float* d_slices,
                            const uint8_t* d_edge, double* d_loss);

/* Gradient of the last okr_loso_forward loss on this plan with respect to
 * (nugget, sill, range), by the adjoint of the extended system of
 * Appendix A, K = [[C, Q], [Q^T, 0]] (Q = 1, or [1 s] with the drift):
 * nu = K^{-1} [e z; 0], dL/dtheta = nu_w^T dc0/dtheta - nu_w^T dC/dtheta w
 * (Q does not depend on the variogram).
 * d_grad: device double[3]. OKR_E_INVALID_ARG unless an okr_loso_forward
 * preceded it with no okr_execute, okr_select, okr_plan_autotune or
 * okr_krige_points on the plan in between (those overwrite the
 * selection and counters the adjoint reads). */
okr_status okr_loso_backward(okr_plan* plan, double* d_grad);

/* Ordinary kriging of explicitly given point sets (Appendix A with the single
 * constant predictor), in FP64 whatever the plan's precision: the test seam
 * for the closed forms and invariants of the method. System i has
 * n_i = d_count[i] points (1..98) starting at d_offset[i] (CSR, int64):
 *   d_xyz         float32 [total][3] point coordinates (x, y, z)
 *   d_val         float32 [total] point values
 *   d_target_xyz  float32 [nsys][3] one target per system
 *   d_est         float32 [nsys] estimate (required)
 *   d_var         float32 [nsys] kriging variance sill - w'c0 - mu (nullable)
 *   d_weights     float32 [total] weights w, CSR like d_val (nullable)
 * Covariance: Cov(0) = sill, Cov(h > 0) = (sill - nugget) rho(h) on Euclidean
 * distances. All device buffers are caller-owned; stream-ordered. A count
 * outside 1..98 gives NaN outputs for that system and OKR_E_SHAPE at the next
 * okr_stats_get; a non-positive pivot (e.g. coincident points with nugget 0)
 * gives NaN outputs and is counted in n_nonpositive_pivot; non-finite inputs
 * give OKR_E_NONFINITE at the next okr_stats_get. */
okr_status okr_krige_points(okr_plan* plan, const okr_variogram* vario, int64_t nsys,
                            const int32_t* d_count, const int64_t* d_offset, const float* d_xyz,
                            const float* d_val, const float* d_target_xyz, float* d_est,
                            float* d_var, float* d_weights);

/* Marching cubes (Appendix C) on a float32 volume of the plan's output shape
 * [nz][ny][nx], nz = (nslices-1)*upsample+1 -- e.g. the volume okr_execute
 * wrote: a surface through the unit cubes between neighbouring voxels where
 * the values cross iso. A corner is inside when its value >= iso (NaN is
 * outside); crossing points are interpolated on the cube edge from its lower
 * corner, t = (iso - A) / (B - A) in float32; on a face whose diagonal
 * corners agree the crossings are paired around the inside corners, so
 * neighbouring cubes join without holes; each polygon is oriented with its
 * normal from inside to outside and split into a fan from its lowest edge id
 * (corner c = x + 2y + 4z, edge 4a + u + 2w along axis a at (u, w) on the
 * other axes). Triangles come in order of the cube index
 * (z*(ny-1) + y)*(nx-1) + x:
 *   d_tris   float32 [max_tris][3][3] vertex coordinates (x, y, z), voxel units
 *   d_cube   int64 [max_tris] each triangle's cube index (nullable)
 * *n_tris (host) receives the total number of triangles. With max_tris = 0
 * (d_tris may then be NULL) only the count is taken; otherwise the first
 * min(total, max_tris) triangles are written and OKR_E_CAPACITY is returned if
 * total > max_tris. Non-finite values give NaN coordinates on their edges.
 * Synchronises the plan's stream; the workspace (a 4 KB table and 4 bytes per
 * 64 cubes of a row) is allocated by the first call. */
okr_status okr_marching_cubes(okr_plan* plan, const float* d_volume, float iso, float* d_tris,
                              int64_t* d_cube, int64_t max_tris, int64_t* n_tris);

/* The paper's edge post-pass (Section 4.1.2, Algorithm 2; shearlets of
 * Appendix B) on a float32 volume of the plan's output shape [nz][ny][nx],
 * nz = (nslices-1)*upsample+1, image by image along the YZ plane
 * (I_x(z, y) = V[z][y][x]; image rows z, columns y):
 *   1. FP64 coefficients SH_k(p) = sum_d psi_k(d) I(p + d) of 8 orientations
 *      (the filters okr_edge_filters returns; border replicated), summed with
 *      d2 (rows) outer and d1 (columns) inner, each product rounded before it
 *      is added; M = max_k |SH_k|, theta = the first k attaining it;
 *   2. p is an edge pixel iff M(p) >= tau and neither neighbour p +- n
 *      (n: the normal of theta rounded to 45 degrees, okr_edge_filters'
 *      normals; out-of-image neighbours do not count) has a larger M;
 *   3. chains: pixels in row-major order each start a chain at an edge pixel
 *      not yet visited; a chain moves to the first unvisited edge pixel among
 *      the 8 neighbours of its last pixel, searched clockwise (y right, z
 *      down: E, SE, S, SW, W, NW, N, NE) from three steps counter-clockwise of
 *      its last move (from E at the start); each full group of 16 consecutive
 *      chain pixels is a window;
 *   4. a window whose orientation changes at least 4 times between
 *      consecutive pixels is noise: its representative orientation is the
 *      most frequent one (ties: the first seen in the window); walking the
 *      window from its first pixel, each interior pixel with another
 *      orientation is replaced by the previous kept or new pixel plus the
 *      tangent t (the representative's rounded normal turned by 90 degrees,
 *      pointing from the first toward the last pixel; a replacement outside
 *      the image keeps the pixel);
 *   5. around each new edge pixel the 3 neighbours on each side of t (sign of
 *      t x d) that lie in the image take their median; windows apply in
 *      chain order, so later medians see earlier ones.
 * Arguments:
 *   d_volume  float32 [nz][ny][nx] input, finite (required)
 *   d_out     float32 [nz][ny][nx] the adjusted volume (required; may equal
 *             d_volume for an in-place pass, otherwise it must not overlap it)
 *   tau       edge threshold on M (finite)
 *   d_edge    uint8 [nz][ny][nx] edge map after the pass, 1 = edge (nullable)
 *   d_orient  uint8 [nz][ny][nx] orientation 0..7 after the pass (nullable)
 *   d_mag     float64 [nz][ny][nx] M of step 1 (nullable)
 * The workspace (9 bytes per voxel and one bit per pixel) is allocated by the
 * first call. Stream-ordered; the result does not depend on the launch
 * shape. Non-finite voxels give unspecified edges (no error is raised). */
okr_status okr_edge_postpass(okr_plan* plan, const float* d_volume, float* d_out, double tau,
                             uint8_t* d_edge, uint8_t* d_orient, double* d_mag);

/* The edge post-pass's filters and rounded normals as the library uses them
 * (host only, no device work): taps[k][d2 + 4][d1 + 4] for k < 8 (648
 * doubles) and normals[2k], normals[2k+1] = (d1, d2) of orientation k (16
 * int32). Either pointer may be NULL. */
okr_status okr_edge_filters(double* taps, int32_t* normals);

/* Counters of the last execute / loso call; synchronises the plan's stream and
 * returns any latched device-side error (e.g. OKR_E_NONFINITE). */
okr_status okr_stats_get(okr_plan* plan, okr_stats* out);

okr_status okr_plan_destroy(okr_plan* plan);

/* okr_execute without a plan and without any allocation, for callers that
 * cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. Same arguments and results as
 * okr_plan_create + okr_execute on the given problem (identical kernels;
 * the launch shape is the untuned default and no graph is used), except:
 *   - the workspace is a static device array of the library, 26.4 MB per GPU
 *     it runs on, held until the process ends: problems of at most 2^20
 *     (column, gap) systems ((nslices-1)*nx*ny <= 1048576), larger ones get
 *     OKR_E_SHAPE before any device work;
 *   - every call on one GPU shares that array: calls that overlap on one GPU
 *     (other streams, other threads) race and must be serialised by the
 *     caller; each call clears what it needs and leaves the last call's
 *     contents behind;
 *   - device-detected errors are not latched in a plan: with d_status
 *     (device int32, nullable) the call writes, stream-ordered, the status
 *     okr_stats_get would return (OKR_OK, OKR_E_NONFINITE, or with strict
 *     OKR_E_NOT_CONVERGED).
 * hip_stream is a hipStream_t (NULL = the default stream); work is
 * asynchronous. Argument errors are returned before any device work. */
okr_status okr_execute_noalloc(const okr_problem* problem, void* hip_stream,
                               const okr_variogram* vario, const float* d_slices,
                               const uint8_t* d_edge, float* d_volume, float* d_variance,
                               uint8_t* d_flags, int32_t* d_status);

/* Profiling: when enabled, every phase launch is bracketed by HIP events on the
 * plan's stream and okr_stats_get reports the summed device time per phase
 * (then clears it). Off by default; costs one event pair per phase. */
okr_status okr_plan_set_profiling(okr_plan* plan, int32_t enable);

/* Launch graph: when enabled, okr_execute records its launch sequence into a
 * HIP graph (captured on a private stream of the plan) the first time it is
 * called with a given variogram, buffer set and tuning, and afterwards
 * replays that graph on the plan's stream; a call with other arguments
 * re-captures. Results are those of the direct launches. With profiling on,
 * one mark (phase 4) spans the whole replay. Off by default. */
okr_status okr_plan_set_graph(okr_plan* plan, int32_t enable);

/* Autotuner: times the plan's own okr_execute on the given inputs (buffers as
 * in okr_execute; flags are not written) for each candidate launch shape --
 * 1 to 4 persistent workgroups per compute unit and, for MIXED_*, the split
 * low-precision or the FP32 trailing-update arithmetic (the FP32 form is at
 * least as accurate) -- as the median of three timed executes after one
 * warm-up, and keeps the fastest for later calls. The choice is cached for
 * the process, keyed by (device architecture, radius, upsample, precision,
 * algo, refine_max, drift): a later autotune of a plan with the same key
 * takes the cached shape without timing (okr_plan_get_tuning reports it).
 * Synchronises the plan's stream when it times. Every candidate computes the
 * same problem; the last one timed leaves its result in d_volume /
 * d_variance. */
okr_status okr_plan_autotune(okr_plan* plan, const okr_variogram* vario, const float* d_slices,
                             const uint8_t* d_edge, float* d_volume, float* d_variance);

/* The plan's launch shape: workgroups per compute unit, mixed update
 * arithmetic (-1: the precision's own, 0: FP32, 1: split FP16, 2: split BF16)
 * and, after okr_plan_autotune, the median time of each candidate in ms
 * (double[8], nullable; candidates in the order grid 1..4, each with the
 * precision's own then FP32 updates for MIXED_*, grid 1..4 otherwise; the
 * times of the run that made a cached choice), and whether the choice came
 * from the cache (from_cache, nullable: 1 cached, 0 timed by this plan). */
okr_status okr_plan_get_tuning(const okr_plan* plan, int32_t* grid_per_cu, int32_t* update_arith,
                               double* cand_ms, int32_t* from_cache);

const char* okr_status_string(okr_status status);
const char* okr_plan_last_error(const okr_plan* plan);

/* Library version as major*10000 + minor*100 + patch. */
int32_t okr_version(void);

/* Sizes in bytes of okr_problem, okr_variogram and okr_stats as compiled into
 * the library, written to out[0..2], so a binding can check its layouts. */
okr_status okr_abi_sizes(int64_t* out);

#ifdef __cplusplus
}
#endif

#endif /* OKRIG_H */
