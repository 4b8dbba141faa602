// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace okr {

constexpr int kMaxRadius = 3;
constexpr int kMaxWin = 2 * kMaxRadius + 1;        // W
constexpr int kMaxCand = 2 * kMaxWin * kMaxWin;    // 98 candidates
constexpr int kMaxUpsample = 15;                   // f; nb = f + 1 <= 16 border rows
constexpr int kMaxBlocks = 8;                      // 16-wide blocks of the augmented matrix
constexpr int kTcSize = 128;                       // pair-class table, index (ds<<6)|(|dy|<<3)|(|dx|)
constexpr int kT0Stride = 32;                      // target table: ((t-1)*2 + s)*16 + |dy|*4 + |dx|
constexpr int kT0Size = kMaxUpsample * kT0Stride;  // up to 14 targets used
constexpr int kHist = 128;                         // histogram bins over n

// Full-window weight cache (kernels_points.hip), one buffer of doubles:
//   W   [f-1][kMaxCand]        weights of the full window per target
//   var [kMaxUpsample]         their kriging variances
//   G   [kMaxCand][kMaxCand]   C^{-1} of the full window (row-major)
//   U   [kMaxUpsample][kMaxCand]  row 0: C^{-1} 1, row t: C^{-1} c0_t,
//                              last row: C^{-1} s (the slice predictor)
//   C0  [kMaxUpsample-1][kMaxCand] row t-1: c0_t of the full window
// Systems that drop at most kMaxDrop candidates of the full window take
// their weights from G and U (a k x k solve per system).
constexpr int kMaxDrop = 32;
constexpr int kPatW = 0;
constexpr int kPatVar = kPatW + (kMaxUpsample - 1) * kMaxCand;
constexpr int kPatG = kPatVar + kMaxUpsample;
constexpr int kPatU = kPatG + kMaxCand * kMaxCand;
constexpr int kPatC0 = kPatU + kMaxUpsample * kMaxCand;
constexpr int kPatDoubles = kPatC0 + (kMaxUpsample - 1) * kMaxCand;

// Per-system count byte: low 7 bits = n, bit 7 = floor-filled.
constexpr uint8_t kFloorBit = 0x80;

// Flag bits written per system (see okrig.h).
constexpr uint8_t kFlagFloor = 1, kFlagRefined = 2, kFlagFp64 = 4, kFlagBadPivot = 8,
                  kFlagFailed = 16, kFlagUnconverged = 32;

struct Geometry {
  int nx, ny, nslices, f, r, W, W2, ncand, min_points;
  int drift;              // 1: the slice of each point is a second predictor
  long long plane;        // nx * ny
  long long nsys;         // (nslices - 1) * plane
};

// Kernel-argument block of the selection rule.
struct SelectRule {
  uint64_t path[kMaxWin * kMaxWin];  // offset o=(dy+r)*W+(dx+r): window cells on its path
  uint8_t floor_order[kMaxCand];     // canonical indices in floor order
};

// Device tables, computed on the device in FP64 from the variogram.
struct TableSet {
  double* tc_d;   // [kTcSize]
  double* t0_d;   // [kT0Size]
  double* dtc_d;  // [3][kTcSize]  d/d(nugget, sill, range)
  double* dt0_d;  // [3][kT0Size]
  float* tc_f;    // FP32 copies
  float* t0_f;
};

struct Vario { int model; double nugget, sill, range; };

// Work-distribution and statistics block in device memory.
struct DevCounters {
  unsigned long long next;          // persistent-kernel work cursor
  unsigned long long hist[kHist];   // systems per n
  unsigned long long floor_filled;
  unsigned long long refined;
  unsigned long long fp64_fallback;
  unsigned long long bad_pivot;
  unsigned long long failed;        // systems whose FP64 re-solve also met a bad pivot
  unsigned long long unconverged;   // systems whose correction left the tolerance unmet
  unsigned int max_kappa_bits;      // float bits of the largest estimate
  unsigned int zmax_bits;           // float bits of the largest |known voxel|
  unsigned int nonfinite;           // nonzero if a known voxel is not finite
  unsigned int bad_input;           // nonzero if a point system had an invalid count
  unsigned long long offsets[kHist + 1];  // bucket starts (largest n first)
  unsigned long long cursor[kHist];
  unsigned long long next2;         // second-pass cursor
  unsigned long long cls_next[kMaxBlocks + 1][8];  // per size-class cursors, one per XCD
  unsigned long long n_fallback_list;
};

// ---- launchers (kernels_select.hip) ----
hipError_t launch_tables(const Vario& v, const Geometry& g, TableSet t, hipStream_t s);
hipError_t launch_reset(DevCounters* c, hipStream_t s);
hipError_t launch_status(const DevCounters* c, int strict, int32_t* out, hipStream_t s);
hipError_t launch_reset_cursors(DevCounters* c, hipStream_t s);
hipError_t launch_place(const float* slices, float* volume, float* variance, const Geometry& g,
                        DevCounters* c, hipStream_t s);
hipError_t launch_select(const uint8_t* edge, const Geometry& g, const SelectRule& rule,
                         uint64_t* bits, uint8_t* count, DevCounters* c, hipStream_t s);
// Size-sorted permutation: buckets by size class (nb border rows), largest first.
hipError_t launch_bucket(const uint8_t* count, const Geometry& g, int nb, uint32_t* perm,
                         DevCounters* c, hipStream_t s);

// ---- launchers (kernels_solve.hip) ----
struct SolveArgs {
  const float* slices;
  const uint64_t* bits;
  const uint8_t* count;
  const uint32_t* perm;
  float* volume;
  float* variance;
  uint8_t* flags;
  DevCounters* ctr;
  TableSet tab;
  Geometry geo;
  double sill;
  int nb;               // border rows: f + 1
  int precision;        // okr_precision
  double kappa_limit;   // condition estimate above which a system is re-solved in FP64
  double refine_kappa;  // mixed: condition estimate above which the FP64 correction runs
  int refine;           // mixed: 0 = factor read-out only, 1 = FP64 correction
  double route_tol;     // mixed read-out: error indicator above which a system is re-solved in FP64
  double route_scale;   // mixed read-out: kappa_w * u of the indicator kappa_w u s / max(|z_hat|, zfloor)
  double refine_tol;    // mixed corrected: per-voxel tolerance of the convergence test (0: none)
  double rho_hat;       // mixed corrected: bound on the error left per unit of correction
  double kappa_w;       // condition number of the full-window covariance matrix (0: not computed)
  int upd;              // mixed trailing updates: 0 FP32, 1 split FP16, 2 split BF16
  int nmax;             // largest neighbour count the size-class kernels take
  uint32_t* fallback;   // list of systems for the FP64 pass
  int step;             // upper bounding slice = lower + step (1: volume, 2: held-out slice)
  double* resid;        // leave-one-slice-out: z_hat - z per system
  double* gpart;        // leave-one-slice-out: per-system gradient [3]
  double inv_count;     // 1 / number of held-out voxels
  int as_resolve;       // 1: this FP64 launch stands in for the re-solve of every system
                        // (flags and counters as for re-solved systems)
};
hipError_t launch_solve(const SolveArgs& a, int grid, hipStream_t s);
hipError_t launch_solve_fallback(const SolveArgs& a, int grid, hipStream_t s);
int solve_blocks_needed(const Geometry& g);

hipError_t launch_solve_mixed(const SolveArgs& a, int grid, hipStream_t s);

// ---- launchers (kernels_points.hip) ----
// Smallest neighbour count whose systems the weight cache serves by the
// k x k solve (whole size classes of the solve kernels, at most kMaxDrop
// dropped candidates); ncand when none.
int pattern_downdate_floor(const Geometry& g);
// The full window's weights, inverse and solves, then its systems' estimates.
hipError_t launch_pattern(const float* slices, const uint8_t* count, DevCounters* c,
                          const Geometry& g, const Vario& v, double* pat, float* volume,
                          float* variance, uint8_t* flags, hipStream_t s);
// The systems with neighbour counts nlo .. ncand - 1 from the full window's
// inverse (after launch_pattern and the bucketing).
hipError_t launch_pattern_downdate(const float* slices, const uint64_t* bits,
                                   const uint8_t* count, const uint32_t* perm, DevCounters* c,
                                   const Geometry& g, const Vario& v, const double* pat, int nlo,
                                   float* volume, float* variance, uint8_t* flags, int grid,
                                   hipStream_t s);
hipError_t launch_points(const Vario& v, long long nsys, const int32_t* count,
                         const int64_t* offset, const float* xyz, const float* val,
                         const float* txyz, float* est, float* var, float* weights,
                         DevCounters* c, int grid, hipStream_t s);

// ---- launchers (kernels_adjoint.hip) ----
hipError_t launch_loso_forward(const SolveArgs& a, int grid, hipStream_t s);
hipError_t launch_loso_backward(const SolveArgs& a, int grid, hipStream_t s);
// Deterministic sum of x[i*stride + comp] over i < n (fixed order), comp < ncomp,
// scaled by `scale`, into out[comp]; partial needs 256 * ncomp doubles.
hipError_t launch_reduce(const double* x, long long n, int ncomp, double scale, double* partial,
                         double* out, bool square, hipStream_t s);
hipError_t launch_select_step(const uint8_t* edge, const Geometry& g, int step, int ngaps,
                              const SelectRule& rule, uint64_t* bits, uint8_t* count,
                              DevCounters* c, hipStream_t s);

// ---- launchers (kernels_plain.hip) ----
hipError_t launch_plain(const float* slices, const uint8_t* edge, float* volume, float* variance,
                        const Geometry& g, const SelectRule& rule, const Vario& v, TableSet tab,
                        int refine, int num_cu, hipStream_t s);

// ---- marching cubes (mcubes_table.cpp, kernels_mcubes.hip) ----
constexpr int kMcMaxTri = 5;     // triangles of one cube configuration, at most
constexpr int kMcRows = 64;      // rows of one wave's strip of 64 cubes (at most 64)
constexpr int kMcGroup = 4;      // rows whose loads the count pass issues together
struct McTable {
  uint8_t ntri[256];                  // triangles of configuration cfg
  uint8_t tri[256][3 * kMcMaxTri];    // their cube edges, three per triangle
};
const McTable& mc_table();            // built once on the host
// Work decomposition: waves over (z-slab, run of kMcRows rows, strip of 64
// cubes); one count per (row, strip), scanned in tiles of 1024.
struct McGrid {
  long long nstrip, nych, nwaves, ncnt, ntile;
};
McGrid mc_grid(long long nz, long long ny, long long nx);
hipError_t launch_mc_count(const float* vol, int nx, int ny, const McGrid& g, float iso,
                           const McTable* table, uint32_t* cnt, hipStream_t s);
// counts -> offsets within their tile (in place); tile[0..ntile) the tiles'
// offsets, tile[ntile] the total
hipError_t launch_mc_scan(uint32_t* cnt, const McGrid& g, unsigned long long* tile,
                          hipStream_t s);
hipError_t launch_mc_emit(const float* vol, int nx, int ny, const McGrid& g, float iso,
                          const McTable* table, const uint32_t* off_local,
                          const unsigned long long* tile_off, float* tris, long long* cube_id,
                          long long max_tris, hipStream_t s);

}  // namespace okr
