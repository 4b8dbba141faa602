// Host side of the okrig C ABI: validation, plan/workspace ownership, the
// neighbour-rule tables and the launch sequence of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/okrig.h"
#include "edge_filters.h"
#include "edge_internal.h"
#include "okrig_internal.h"

namespace okr {
hipError_t launch_select_step(const uint8_t* edge, const Geometry& g, int step, int ngaps,
                              const SelectRule& rule, uint64_t* bits, uint8_t* count,
                              DevCounters* c, hipStream_t s);
}  // namespace okr

struct okr_plan {
  okr_problem prob;
  okr::Geometry geo;
  okr::SelectRule rule;
  hipStream_t stream = nullptr;
  int device = 0;
  int num_cu = 256;
  // workspace
  uint64_t* bits = nullptr;
  uint8_t* count = nullptr;
  uint32_t* perm = nullptr;
  uint32_t* fallback = nullptr;
  double* pattern_w = nullptr;  // full-window weight cache (layout at kPatDoubles)
  okr::DevCounters* ctr = nullptr;
  double* tabs = nullptr;       // FP64 tables and derivatives
  float* tabs_f = nullptr;      // FP32 copies
  double* loso_resid = nullptr;   // per held-out voxel residual (z_hat - z)
  double* loso_gpart = nullptr;   // per held-out voxel gradient contribution [3]
  double* loso_partial = nullptr; // reduction partials
  okr::McTable* mc_tab = nullptr;       // marching cubes (first call): case table,
  uint32_t* mc_cnt = nullptr;           // triangles per (row, strip), then offsets,
  unsigned long long* mc_tile = nullptr;  // tile offsets and the total
  double* edge_mag = nullptr;           // edge post-pass (first call): M per voxel,
  uint8_t* edge_theta = nullptr;        // orientation per voxel,
  uint32_t* edge_bits = nullptr;        // per-image edge bitmaps
  int edge_lds_max = -1;                // largest dynamic LDS of one workgroup (bytes)
  bool loso_ready = false;
  okr_variogram loso_vario{};
  const float* loso_slices = nullptr;
  const uint8_t* loso_edge = nullptr;
  long long last_nsys = 0, last_kriged = 0;
  bool profiling = false;
  bool timers_off = false;      // no profiling marks while a graph is captured
  // 2-norm condition number of the full-window covariance matrix for the last
  // variogram it was computed for (every system's covariance matrix is a
  // principal submatrix of it, so bounds their condition numbers)
  bool last_direct64 = false;   // the last execute solved every system in FP64 directly
  bool kw_valid = false;
  okr_variogram kw_vario{};
  double kappa_w = 0.0;
  int grid_per_cu = 3;          // persistent workgroups per compute unit (autotuned)
  int upd = -1;                 // mixed trailing-update arithmetic (-1: from the precision)
  bool tuned = false;
  bool tune_cached = false;     // the shape came from the process-wide cache
  double tune_ms[8] = {0};      // autotune: median time per candidate, ms
  // launch graph of okr_execute, keyed by its arguments
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  struct GraphKey {
    okr_variogram v;
    const float* slices;
    const uint8_t* edge;
    float* volume;
    float* variance;
    uint8_t* flags;
    bool forced, no_direct;
    int grid_per_cu, upd;
  } gkey{};
  bool gkey_valid = false;
  long long graph_launches = 0, graph_captures = 0;
  struct Mark { int phase; hipEvent_t a, b; };
  std::vector<Mark> marks;
  double phase_ms[OKR_NUM_PHASES] = {0};
  long long phase_calls[OKR_NUM_PHASES] = {0};
  std::string err;
};

namespace {

okr_status fail(okr_plan* p, okr_status st, const std::string& msg) {
  if (p) p->err = msg;
  return st;
}

#define OKR_HIP(plan, call)                                                              \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(plan, OKR_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// round half away from zero of num/den, den > 0
int rha(int num, int den) {
  int q = (2 * std::abs(num) + den) / (2 * den);
  return num >= 0 ? q : -q;
}

void build_rule(int r, okr::SelectRule* rule) {
  std::memset(rule, 0, sizeof(*rule));
  const int W = 2 * r + 1, W2 = W * W;
  for (int dy = -r; dy <= r; ++dy) {
    for (int dx = -r; dx <= r; ++dx) {
      const int o = (dy + r) * W + (dx + r);
      const int L = std::max(std::abs(dx), std::abs(dy));
      uint64_t m = 0;
      for (int k = 1; k <= L; ++k) {
        const int px = rha(k * dx, L), py = rha(k * dy, L);
        m |= 1ull << ((py + r) * W + (px + r));
      }
      rule->path[o] = m;
    }
  }
  std::vector<int> idx(2 * W2);
  for (int i = 0; i < 2 * W2; ++i) idx[i] = i;
  auto key = [&](int c) {
    const int s = c >= W2, o = c - s * W2, dy = o / W - r, dx = o % W - r;
    return std::make_tuple(dx * dx + dy * dy, s, dy, dx);
  };
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return key(a) < key(b); });
  for (int i = 0; i < 2 * W2; ++i) rule->floor_order[i] = (uint8_t)idx[i];
}

okr_status validate_problem(const okr_problem* p, std::string* msg) {
  if (!p) { *msg = "problem is NULL"; return OKR_E_INVALID_ARG; }
  if (p->nx < 1 || p->ny < 1 || p->nslices < 1 || p->nx > 65535 || p->ny > 65535 ||
      p->nslices > 65535) {
    *msg = "nx, ny, nslices must be in 1..65535";
    return OKR_E_SHAPE;
  }
  if (p->upsample < 1 || p->upsample > okr::kMaxUpsample) {
    *msg = "upsample must be in 1..15";
    return OKR_E_SHAPE;
  }
  if (p->radius < 0 || p->radius > okr::kMaxRadius) {
    *msg = "radius must be in 0..3";
    return OKR_E_SHAPE;
  }
  const int W = 2 * p->radius + 1;
  if (p->min_points < 1 || p->min_points > 2 * W * W) {
    *msg = "min_points must be in 1..2*(2r+1)^2";
    return OKR_E_INVALID_ARG;
  }
  if (p->precision < OKR_FP32 || p->precision > OKR_FP64) {
    *msg = "unknown precision";
    return OKR_E_INVALID_ARG;
  }
  if (p->algo != OKR_ALGO_BATCHED && p->algo != OKR_ALGO_PLAIN_PER_VOXEL &&
      p->algo != OKR_ALGO_PATTERN_CACHE) {
    *msg = "unknown algo";
    return OKR_E_INVALID_ARG;
  }
  if (p->algo == OKR_ALGO_PLAIN_PER_VOXEL && p->precision != OKR_FP32) {
    *msg = "the plain per-voxel kernel is FP32 only";
    return OKR_E_UNSUPPORTED;
  }
  if (p->drift != 0 && p->drift != 1) {
    *msg = "drift must be 0 (ordinary kriging) or 1 (slice predictor)";
    return OKR_E_INVALID_ARG;
  }
  if (p->drift && p->algo == OKR_ALGO_PLAIN_PER_VOXEL) {
    *msg = "the slice predictor needs the batched or pattern-cache algorithm";
    return OKR_E_UNSUPPORTED;
  }
  if (p->drift && p->upsample > okr::kMaxUpsample - 1) {
    *msg = "with the slice predictor upsample must be in 1..14";
    return OKR_E_SHAPE;
  }
  if (!(p->refine_tol >= 0.0) || p->refine_max < 0 || p->refine_max > 1) {
    *msg = "refine_tol must be >= 0 and refine_max 0 or 1 (one FP64-residual correction "
           "squares the factorisation's relative error; systems it leaves above refine_tol "
           "are re-solved in FP64)";
    return OKR_E_INVALID_ARG;
  }
  const long long plane = (long long)p->nx * p->ny;
  const long long nsys = plane * (long long)(p->nslices > 1 ? p->nslices - 1 : 1);
  if (nsys > 0xffffffffLL) {
    *msg = "more than 2^32 systems";
    return OKR_E_SHAPE;
  }
  return OKR_OK;
}

okr_status validate_vario(const okr_variogram* v, std::string* msg) {
  if (!v) { *msg = "variogram is NULL"; return OKR_E_INVALID_ARG; }
  if (v->model < OKR_SPHERICAL || v->model > OKR_GAUSSIAN) {
    *msg = "unknown variogram model";
    return OKR_E_INVALID_ARG;
  }
  if (!(std::isfinite(v->sill) && std::isfinite(v->nugget) && std::isfinite(v->range)) ||
      !(v->sill > 0.0) || !(v->nugget >= 0.0) || !(v->nugget < v->sill) || !(v->range > 0.0)) {
    *msg = "variogram needs 0 <= nugget < sill and range > 0 (finite)";
    return OKR_E_INVALID_ARG;
  }
  return OKR_OK;
}

template <typename T>
okr_status dev_alloc(okr_plan* p, T** ptr, size_t count) {
  if (count == 0) count = 1;
  if (std::getenv("OKR_FAIL_ALLOC")) return fail(p, OKR_E_OOM, "allocation failure (forced)");
  hipError_t e = hipMalloc(reinterpret_cast<void**>(ptr), count * sizeof(T));
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return fail(p, OKR_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return OKR_OK;
}

void drain_marks(okr_plan* p);

void drop_graph(okr_plan* p) {
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->graph_exec = nullptr;
  p->graph = nullptr;
  p->gkey_valid = false;
}

void free_plan(okr_plan* p) {
  if (!p) return;
  drain_marks(p);
  drop_graph(p);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  hipFree(p->bits);
  hipFree(p->count);
  hipFree(p->perm);
  hipFree(p->fallback);
  hipFree(p->pattern_w);
  hipFree(p->ctr);
  hipFree(p->tabs);
  hipFree(p->tabs_f);
  hipFree(p->loso_resid);
  hipFree(p->loso_gpart);
  hipFree(p->loso_partial);
  hipFree(p->mc_tab);
  hipFree(p->mc_cnt);
  hipFree(p->mc_tile);
  hipFree(p->edge_mag);
  hipFree(p->edge_theta);
  hipFree(p->edge_bits);
  delete p;
}

// Problem, stream, geometry, selection rule and device of a plan (no
// allocation).
okr_status init_plan_shape(okr_plan* p, const okr_problem* problem, void* hip_stream) {
  p->prob = *problem;
  p->stream = static_cast<hipStream_t>(hip_stream);
  okr::Geometry& g = p->geo;
  g.nx = problem->nx;
  g.ny = problem->ny;
  g.nslices = problem->nslices;
  g.f = problem->upsample;
  g.r = problem->radius;
  g.W = 2 * g.r + 1;
  g.W2 = g.W * g.W;
  g.ncand = 2 * g.W2;
  g.min_points = problem->min_points;
  g.drift = problem->drift;
  g.plane = (long long)g.nx * g.ny;
  g.nsys = g.plane * (g.nslices > 1 ? g.nslices - 1 : 0);
  build_rule(g.r, &p->rule);
  if (hipGetDevice(&p->device) != hipSuccess) {
    (void)hipGetLastError();
    return OKR_E_DEVICE;
  }
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess &&
      cu > 0)
    p->num_cu = cu;
  return OKR_OK;
}

okr::TableSet tables_of(okr_plan* p) {
  okr::TableSet t;
  t.tc_d = p->tabs;
  t.t0_d = t.tc_d + okr::kTcSize;
  t.dtc_d = t.t0_d + okr::kT0Size;
  t.dt0_d = t.dtc_d + 3 * okr::kTcSize;
  t.tc_f = p->tabs_f;
  t.t0_f = t.tc_f + okr::kTcSize;
  return t;
}

okr::Vario vario_of(const okr_variogram* v) {
  okr::Vario o;
  o.model = v->model;
  o.nugget = v->nugget;
  o.sill = v->sill;
  o.range = v->range;
  return o;
}

okr::SolveArgs solve_args(okr_plan* p, const okr_variogram* v) {
  okr::SolveArgs a{};
  a.bits = p->bits;
  a.count = p->count;
  a.perm = p->perm;
  a.ctr = p->ctr;
  a.tab = tables_of(p);
  a.geo = p->geo;
  a.sill = v->sill;
  a.nb = p->geo.f + 1 + p->geo.drift;
  a.precision = p->prob.precision;
  a.kappa_limit = 1e300;
  a.refine_kappa = 0.0;
  a.refine = 0;
  a.route_tol = 0.0;
  a.route_scale = 0.0;
  a.refine_tol = 0.0;
  a.rho_hat = 1.0;
  a.kappa_w = 0.0;
  a.as_resolve = 0;
  a.upd = 1;
  a.nmax = okr::kHist - 1;
  a.fallback = nullptr;
  a.step = 1;
  a.resid = nullptr;
  a.gpart = nullptr;
  a.inv_count = 0.0;
  return a;
}

int persistent_grid(okr_plan* p) { return p->num_cu * p->grid_per_cu; }

constexpr double kUnitRoundoff32 = 5.9604644775390625e-8;   // 2^-24

// Brackets one phase's launches with events when profiling is on.
struct PhaseTimer {
  okr_plan* p;
  int phase;
  hipEvent_t a = nullptr, b = nullptr;
  PhaseTimer(okr_plan* plan, int ph) : p(plan), phase(ph) {
    if (!p->profiling || p->timers_off) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      (void)hipGetLastError();
      a = b = nullptr;
      return;
    }
    (void)hipEventRecord(a, p->stream);
  }
  ~PhaseTimer() {
    if (!a) return;
    (void)hipEventRecord(b, p->stream);
    p->marks.push_back({phase, a, b});
  }
};

void drain_marks(okr_plan* p) {
  for (auto& m : p->marks) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, m.a, m.b) == hipSuccess) {
      p->phase_ms[m.phase] += ms;
      p->phase_calls[m.phase] += 1;
    } else {
      (void)hipGetLastError();
    }
    (void)hipEventDestroy(m.a);
    (void)hipEventDestroy(m.b);
  }
  p->marks.clear();
}

}  // namespace

extern "C" {

int32_t okr_version(void) { return 100; }

okr_status okr_abi_sizes(int64_t* out) {
  if (!out) return OKR_E_INVALID_ARG;
  out[0] = (int64_t)sizeof(okr_problem);
  out[1] = (int64_t)sizeof(okr_variogram);
  out[2] = (int64_t)sizeof(okr_stats);
  return OKR_OK;
}

const char* okr_status_string(okr_status s) {
  switch (s) {
    case OKR_OK: return "ok";
    case OKR_E_INVALID_ARG: return "invalid argument";
    case OKR_E_SHAPE: return "shape out of range";
    case OKR_E_NONFINITE: return "non-finite known voxel";
    case OKR_E_DEVICE: return "device error";
    case OKR_E_OOM: return "out of memory";
    case OKR_E_UNSUPPORTED: return "unsupported";
    case OKR_E_NOT_CONVERGED: return "not converged";
    case OKR_E_CAPACITY: return "output buffer too small";
    default: return "unknown status";
  }
}

const char* okr_plan_last_error(const okr_plan* p) { return p ? p->err.c_str() : "plan is NULL"; }

okr_status okr_plan_create(const okr_problem* problem, void* hip_stream, okr_plan** out) {
  if (!out) return OKR_E_INVALID_ARG;
  *out = nullptr;
  std::string msg;
  okr_status st = validate_problem(problem, &msg);
  if (st != OKR_OK) return st;
  okr_plan* p = new (std::nothrow) okr_plan();
  if (!p) return OKR_E_OOM;
  if ((st = init_plan_shape(p, problem, hip_stream)) != OKR_OK) {
    free_plan(p);
    return st;
  }
  const okr::Geometry& g = p->geo;
  const size_t nsys = (size_t)std::max<long long>(g.nsys, 1);
  if ((st = dev_alloc(p, &p->ctr, 1)) != OKR_OK ||
      (st = dev_alloc(p, &p->tabs, 4 * okr::kTcSize + 4 * okr::kT0Size)) != OKR_OK ||
      (st = dev_alloc(p, &p->tabs_f, okr::kTcSize + okr::kT0Size)) != OKR_OK) {
    free_plan(p);
    return st;
  }
  if (problem->algo != OKR_ALGO_PLAIN_PER_VOXEL) {
    if ((st = dev_alloc(p, &p->pattern_w, okr::kPatDoubles)) !=
        OKR_OK) {
      free_plan(p);
      return st;
    }
    if ((st = dev_alloc(p, &p->bits, 2 * nsys)) != OKR_OK ||
        (st = dev_alloc(p, &p->count, nsys)) != OKR_OK ||
        (st = dev_alloc(p, &p->perm, nsys)) != OKR_OK ||
        (st = dev_alloc(p, &p->fallback, nsys)) != OKR_OK) {
      free_plan(p);
      return st;
    }
  }
  *out = p;
  return OKR_OK;
}

okr_status okr_plan_destroy(okr_plan* p) {
  if (!p) return OKR_E_INVALID_ARG;
  (void)hipStreamSynchronize(p->stream);
  free_plan(p);
  return OKR_OK;
}

}  // extern "C"

namespace {

bool force_fallback() {
  const char* force = std::getenv("OKR_FORCE_FALLBACK");
  return force && force[0] == '1';
}

// OKR_NO_DIRECT_FP64=1 keeps the low-precision pass where the precision
// control would otherwise solve every system in FP64 directly (tests use it
// to exercise the per-system checks on ill-conditioned windows).
bool no_direct_fp64() {
  const char* v = std::getenv("OKR_NO_DIRECT_FP64");
  return v && v[0] == '1';
}

// Covariance of lag h (GSLIB convention, the library's variogram models).
double host_cov(const okr_variogram& v, double h) {
  if (h == 0.0) return v.sill;
  const double q = h / v.range;
  double rho;
  if (v.model == OKR_SPHERICAL) rho = q < 1.0 ? 1.0 - 1.5 * q + 0.5 * q * q * q : 0.0;
  else if (v.model == OKR_EXPONENTIAL) rho = std::exp(-3.0 * q);
  else rho = std::exp(-3.0 * q * q);
  return (v.sill - v.nugget) * rho;
}

// Smallest and largest eigenvalue of a symmetric matrix (cyclic Jacobi
// rotations in FP64; a is overwritten).
void sym_eig_range(double* a, int n, double* lmin, double* lmax) {
  double fro = 0.0;
  for (int i = 0; i < n * n; ++i) fro += a[i] * a[i];
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += a[i * n + j] * a[i * n + j];
    if (off <= 1e-32 * fro) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p * n + q];
        if (std::fabs(apq) <= 1e-300) continue;
        const double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - sn * akq;
          a[k * n + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - sn * aqk;
          a[q * n + k] = sn * apk + c * aqk;
        }
      }
    }
  }
  double mn = a[0], mx = a[0];
  for (int i = 1; i < n; ++i) {
    mn = std::min(mn, a[i * n + i]);
    mx = std::max(mx, a[i * n + i]);
  }
  *lmin = mn;
  *lmax = mx;
}

// Condition number of the covariance matrix of the whole (2r+1)^2 x 2 window
// (known slices f apart). By eigenvalue interlacing no system's matrix, a
// principal submatrix, is worse conditioned. Cached per variogram.
double window_kappa(okr_plan* p, const okr_variogram& v) {
  if (p->kw_valid && p->kw_vario.model == v.model && p->kw_vario.nugget == v.nugget &&
      p->kw_vario.sill == v.sill && p->kw_vario.range == v.range)
    return p->kappa_w;
  const okr::Geometry& g = p->geo;
  const int n = g.ncand;
  double pts[3 * okr::kMaxCand];
  double a[okr::kMaxCand * okr::kMaxCand];
  for (int c = 0; c < n; ++c) {
    const int sl = c / g.W2, o = c % g.W2;
    pts[3 * c] = o % g.W - g.r;
    pts[3 * c + 1] = o / g.W - g.r;
    pts[3 * c + 2] = (double)sl * g.f;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double dx = pts[3 * i] - pts[3 * j], dy = pts[3 * i + 1] - pts[3 * j + 1],
                   dz = pts[3 * i + 2] - pts[3 * j + 2];
      a[(size_t)i * n + j] = host_cov(v, std::sqrt(dx * dx + dy * dy + dz * dz));
    }
  double lmin = 0.0, lmax = 0.0;
  sym_eig_range(a, n, &lmin, &lmax);
  p->kappa_w = lmin > 0.0 ? lmax / lmin : std::numeric_limits<double>::infinity();
  p->kw_vario = v;
  p->kw_valid = true;
  return p->kappa_w;
}

// Unit roundoff of the factorisation arithmetic: FP32 updates, split FP16
// products (hi + lo halves carry about 22 bits), split BF16 products (16 bits).
double factor_roundoff(int upd) {
  return upd == 2 ? std::ldexp(1.0, -16) : (upd == 1 ? std::ldexp(1.0, -22) : std::ldexp(1.0, -24));
}

// Process-wide autotune cache: the chosen launch shape per (device
// architecture, radius, upsample, precision, algo, refine_max, drift).
struct TuneKey {
  char arch[64];
  int r, f, precision, algo, refine_max, drift;
  bool operator==(const TuneKey& o) const {
    return std::strncmp(arch, o.arch, sizeof(arch)) == 0 && r == o.r && f == o.f &&
           precision == o.precision && algo == o.algo && refine_max == o.refine_max &&
           drift == o.drift;
  }
};
struct TuneVal {
  int grid, upd;
  double ms[8];
};
std::mutex g_tune_mu;
std::vector<std::pair<TuneKey, TuneVal>> g_tune_cache;

TuneKey tune_key(const okr_plan* p) {
  TuneKey k{};
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess)
    std::strncpy(k.arch, prop.gcnArchName, sizeof(k.arch) - 1);
  else
    (void)hipGetLastError();
  k.r = p->geo.r;
  k.f = p->geo.f;
  k.precision = p->prob.precision;
  k.algo = p->prob.algo;
  k.refine_max = p->prob.refine_max;
  k.drift = p->prob.drift;
  return k;
}

// The launch sequence of okr_execute on stream `strm` (the plan's stream, or
// the capture stream of its graph).
okr_status enqueue_execute(okr_plan* p, hipStream_t strm, const okr_variogram* vario,
                           const float* d_slices, const uint8_t* d_edge, float* d_volume,
                           float* d_variance, uint8_t* d_flags) {
  const okr::Geometry& g = p->geo;
  OKR_HIP(p, okr::launch_reset(p->ctr, strm));
  {
    PhaseTimer t(p, OKR_PHASE_PLACE);
    OKR_HIP(p, okr::launch_place(d_slices, d_volume, d_variance, g, p->ctr, strm));
  }
  if (g.nslices < 2 || g.f < 2) return OKR_OK;
  {
    PhaseTimer t(p, OKR_PHASE_TABLES);
    OKR_HIP(p, okr::launch_tables(vario_of(vario), g, tables_of(p), strm));
  }
  if (p->prob.algo == OKR_ALGO_PLAIN_PER_VOXEL) {
    PhaseTimer t(p, OKR_PHASE_PLAIN);
    OKR_HIP(p, okr::launch_plain(d_slices, d_edge, d_volume, d_variance, g, p->rule,
                                 vario_of(vario), tables_of(p), p->prob.refine_max > 0 ? 1 : 0,
                                 p->num_cu, strm));
    return OKR_OK;
  }
  {
    PhaseTimer t(p, OKR_PHASE_SELECT);
    OKR_HIP(p, okr::launch_select(d_edge, g, p->rule, p->bits, p->count, p->ctr, strm));
  }
  {
    PhaseTimer t(p, OKR_PHASE_BUCKET);
    OKR_HIP(p, okr::launch_bucket(p->count, g, g.f + 1 + g.drift, p->perm, p->ctr, strm));
  }
  okr::SolveArgs a = solve_args(p, vario);
  a.slices = d_slices;
  a.volume = d_volume;
  a.variance = d_variance;
  a.flags = d_flags;
  if (p->prob.algo == OKR_ALGO_PATTERN_CACHE) {
    // the full-window systems from the cached FP64 weights; the rest below
    PhaseTimer t(p, OKR_PHASE_PATTERN);
    OKR_HIP(p, okr::launch_pattern(d_slices, p->count, p->ctr, g, vario_of(vario), p->pattern_w,
                                   d_volume, d_variance, d_flags, strm));
  }
  if (p->prob.algo == OKR_ALGO_PATTERN_CACHE) {
    // the systems that drop at most kMaxDrop window candidates, from the
    // window's inverse (timed with the batched solve, whose systems they are)
    PhaseTimer t(p, OKR_PHASE_SOLVE);
    const int nlo = okr::pattern_downdate_floor(g);
    OKR_HIP(p, okr::launch_pattern_downdate(d_slices, p->bits, p->count, p->perm, p->ctr, g,
                                            vario_of(vario), p->pattern_w, nlo, d_volume,
                                            d_variance, d_flags, p->num_cu * 4, strm));
    a.nmax = nlo - 1;
  }
  const bool mixed = p->prob.precision == OKR_MIXED_FP16 || p->prob.precision == OKR_MIXED_BF16;
  // Precision control against refine_tol (per-voxel relative error), with the
  // window's condition number kappa_w bounding every system's:
  //   FP32: kappa_w 2^-24 above refine_tol sends every system to FP64;
  //   mixed read-out: per system, the indicator kappa_w u s / max(|z_hat|,
  //     0.01 Zmax) above refine_tol sends it to FP64;
  //   mixed with the correction: the error the correction leaves is at most
  //     the computed weights' relative error, taken as min(1, 10 kappa_w u),
  //     times |w_t| |h_w| + |phi_t| |Q'nu_w| (h the FP64 residual); a system
  //     where that exceeds refine_tol (same relative measure) is unconverged
  //     and re-solved in FP64.
  // Where the full-window system itself misses refine_tol by these bounds
  // (FP32: kappa_w 2^-24; read-out: kappa_w u; corrected: rho_hat kappa_w u,
  // the first-order error of its weights times rho_hat), the full-window
  // systems, most systems of a volume, would all be re-solved: every system
  // is then solved in FP64 directly (and flagged and counted as re-solved).
  // Systems with a non-positive pivot are always re-solved in FP64.
  const double tol = p->prob.refine_tol;
  const double kw = (tol > 0.0 && p->prob.precision != OKR_FP64) ? window_kappa(p, *vario) : 0.0;
  a.kappa_w = kw;
  if (p->prob.precision != OKR_FP64) a.fallback = p->fallback;
  bool direct64 = false;
  if (mixed) {
    a.refine = p->prob.refine_max > 0 ? 1 : 0;
    a.refine_kappa = 0.0;
    a.upd = p->upd >= 0 ? p->upd : (p->prob.precision == OKR_MIXED_BF16 ? 2 : 1);
    const double uf = factor_roundoff(a.upd);
    if (!a.refine) {
      a.route_tol = tol;
      a.route_scale = kw * uf;
      direct64 = tol > 0.0 && !(kw * uf <= tol);
    } else {
      a.refine_tol = tol;
      a.rho_hat = std::min(1.0, 10.0 * kw * uf);
      direct64 = tol > 0.0 && !(a.rho_hat * kw * uf <= tol);
    }
  } else if (p->prob.precision == OKR_FP32) {
    direct64 = tol > 0.0 && !(kw * kUnitRoundoff32 <= tol);
  }
  p->last_direct64 = direct64 && !no_direct_fp64() && !force_fallback();
  if (p->last_direct64) {
    a.precision = OKR_FP64;
    a.fallback = nullptr;
    a.as_resolve = 1;
    a.refine = 0;
  } else if (direct64 && p->prob.precision == OKR_FP32) {
    a.kappa_limit = 0.0;   // every system re-solved after the FP32 pass
  }
  if (force_fallback() && p->prob.precision != OKR_FP64) {
    a.kappa_limit = 0.0;
    a.fallback = p->fallback;
  }
  {
    PhaseTimer t(p, OKR_PHASE_SOLVE);
    if (mixed && !p->last_direct64)
      OKR_HIP(p, okr::launch_solve_mixed(a, persistent_grid(p), strm));
    else
      OKR_HIP(p, okr::launch_solve(a, persistent_grid(p), strm));
  }
  if (a.fallback) {
    PhaseTimer t(p, OKR_PHASE_FALLBACK);
    OKR_HIP(p, okr::launch_solve_fallback(a, persistent_grid(p), strm));
  }
  return OKR_OK;
}

bool same_key(const okr_plan::GraphKey& k, const okr_plan::GraphKey& q) {
  return k.v.model == q.v.model && k.v.nugget == q.v.nugget && k.v.sill == q.v.sill &&
         k.v.range == q.v.range && k.slices == q.slices && k.edge == q.edge &&
         k.volume == q.volume && k.variance == q.variance && k.flags == q.flags &&
         k.forced == q.forced && k.no_direct == q.no_direct && k.grid_per_cu == q.grid_per_cu &&
         k.upd == q.upd;
}

// Capture the launch sequence into a graph (on the plan's private stream) if
// the arguments differ from the captured ones, then launch it on the plan's
// stream.
okr_status execute_graph(okr_plan* p, const okr_variogram* vario, const float* d_slices,
                         const uint8_t* d_edge, float* d_volume, float* d_variance,
                         uint8_t* d_flags) {
  okr_plan::GraphKey key{};
  key.v = *vario;
  key.slices = d_slices;
  key.edge = d_edge;
  key.volume = d_volume;
  key.variance = d_variance;
  key.flags = d_flags;
  key.forced = force_fallback();
  key.no_direct = no_direct_fp64();
  key.grid_per_cu = p->grid_per_cu;
  key.upd = p->upd;
  if (!p->gkey_valid || !same_key(p->gkey, key)) {
    drop_graph(p);
    if (!p->cap_stream) OKR_HIP(p, hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    OKR_HIP(p, hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    p->timers_off = true;
    okr_status st =
        enqueue_execute(p, p->cap_stream, vario, d_slices, d_edge, d_volume, d_variance, d_flags);
    p->timers_off = false;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
    if (st != OKR_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return fail(p, OKR_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    p->graph = graph;
    e = hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      drop_graph(p);
      return fail(p, OKR_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    p->gkey = key;
    p->gkey_valid = true;
    p->graph_captures += 1;
  }
  PhaseTimer t(p, OKR_PHASE_SOLVE);
  OKR_HIP(p, hipGraphLaunch(p->graph_exec, p->stream));
  p->graph_launches += 1;
  return OKR_OK;
}

}  // namespace

extern "C" {

okr_status okr_execute(okr_plan* p, const okr_variogram* vario, const float* d_slices,
                       const uint8_t* d_edge, float* d_volume, float* d_variance,
                       uint8_t* d_flags) {
  if (!p) return OKR_E_INVALID_ARG;
  std::string msg;
  okr_status st = validate_vario(vario, &msg);
  if (st != OKR_OK) return fail(p, st, msg);
  if (!d_slices || !d_volume) return fail(p, OKR_E_INVALID_ARG, "slices and volume are required");
  const okr::Geometry& g = p->geo;
  p->loso_ready = false;
  p->last_nsys = g.nsys;
  p->last_kriged = g.nsys * (g.f - 1);
  if (p->use_graph)
    return execute_graph(p, vario, d_slices, d_edge, d_volume, d_variance, d_flags);
  return enqueue_execute(p, p->stream, vario, d_slices, d_edge, d_volume, d_variance, d_flags);
}

okr_status okr_plan_autotune(okr_plan* p, const okr_variogram* vario, const float* d_slices,
                             const uint8_t* d_edge, float* d_volume, float* d_variance) {
  if (!p) return OKR_E_INVALID_ARG;
  std::string msg;
  okr_status st = validate_vario(vario, &msg);
  if (st != OKR_OK) return fail(p, st, msg);
  if (!d_slices || !d_volume) return fail(p, OKR_E_INVALID_ARG, "slices and volume are required");
  // the timed executes overwrite the selection, permutation and counters that
  // a pending okr_loso_backward would read
  p->loso_ready = false;
  if (p->prob.algo == OKR_ALGO_PLAIN_PER_VOXEL || p->geo.nslices < 2 || p->geo.f < 2) {
    p->tuned = true;
    return OKR_OK;
  }
  const TuneKey key = tune_key(p);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    for (const auto& e : g_tune_cache) {
      if (e.first == key) {
        p->grid_per_cu = e.second.grid;
        p->upd = e.second.upd;
        std::memcpy(p->tune_ms, e.second.ms, sizeof(p->tune_ms));
        p->tuned = true;
        p->tune_cached = true;
        drop_graph(p);
        return OKR_OK;
      }
    }
  }
  const bool mixed = p->prob.precision == OKR_MIXED_FP16 || p->prob.precision == OKR_MIXED_BF16;
  const int own_upd = p->prob.precision == OKR_MIXED_BF16 ? 2 : 1;
  struct Cand { int grid, upd; };
  std::vector<Cand> cands;
  for (int gpc = 1; gpc <= 4; ++gpc) {
    cands.push_back({gpc, mixed ? own_upd : -1});
    if (mixed) cands.push_back({gpc, 0});   // FP32 updates are at least as accurate
  }
  const bool graph = p->use_graph, prof = p->profiling;
  p->use_graph = false;
  p->profiling = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  OKR_HIP(p, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(p, OKR_E_DEVICE, "hipEventCreate failed");
  }
  constexpr int kReps = 3;
  double best = 1e300;
  Cand pick = {p->grid_per_cu, p->upd};
  for (size_t i = 0; i < cands.size() && st == OKR_OK; ++i) {
    p->grid_per_cu = cands[i].grid;
    p->upd = cands[i].upd;
    st = enqueue_execute(p, p->stream, vario, d_slices, d_edge, d_volume, d_variance, nullptr);
    double ms[kReps];
    for (int k = 0; k < kReps && st == OKR_OK; ++k) {
      (void)hipEventRecord(e0, p->stream);
      st = enqueue_execute(p, p->stream, vario, d_slices, d_edge, d_volume, d_variance, nullptr);
      (void)hipEventRecord(e1, p->stream);
      if (st != OKR_OK) break;
      float t = 0.0f;
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
        st = fail(p, OKR_E_DEVICE, "autotune timing failed");
        break;
      }
      ms[k] = t;
    }
    if (st != OKR_OK) break;
    std::sort(ms, ms + kReps);
    const double med = ms[kReps / 2];
    if (i < 8) p->tune_ms[i] = med;
    if (med < best) {
      best = med;
      pick = cands[i];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->grid_per_cu = pick.grid;
  p->upd = pick.upd;
  p->use_graph = graph;
  p->profiling = prof;
  if (st == OKR_OK) {
    p->tuned = true;
    p->tune_cached = false;
    TuneVal v{pick.grid, pick.upd, {}};
    std::memcpy(v.ms, p->tune_ms, sizeof(v.ms));
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache.emplace_back(key, v);
  }
  drop_graph(p);
  return st;
}

okr_status okr_plan_get_tuning(const okr_plan* p, int32_t* grid_per_cu, int32_t* update_arith,
                               double* cand_ms, int32_t* from_cache) {
  if (!p) return OKR_E_INVALID_ARG;
  if (grid_per_cu) *grid_per_cu = p->grid_per_cu;
  if (update_arith) *update_arith = p->upd;
  if (cand_ms)
    for (int i = 0; i < 8; ++i) cand_ms[i] = p->tune_ms[i];
  if (from_cache) *from_cache = p->tune_cached ? 1 : 0;
  return OKR_OK;
}

okr_status okr_krige_points(okr_plan* p, const okr_variogram* vario, int64_t nsys,
                            const int32_t* d_count, const int64_t* d_offset, const float* d_xyz,
                            const float* d_val, const float* d_target_xyz, float* d_est,
                            float* d_var, float* d_weights) {
  if (!p) return OKR_E_INVALID_ARG;
  std::string msg;
  okr_status st = validate_vario(vario, &msg);
  if (st != OKR_OK) return fail(p, st, msg);
  if (nsys < 0) return fail(p, OKR_E_INVALID_ARG, "nsys must be >= 0");
  if (nsys > 0 && (!d_count || !d_offset || !d_xyz || !d_val || !d_target_xyz || !d_est))
    return fail(p, OKR_E_INVALID_ARG, "count, offset, xyz, val, target_xyz and est are required");
  p->loso_ready = false;
  OKR_HIP(p, okr::launch_reset(p->ctr, p->stream));
  OKR_HIP(p, okr::launch_points(vario_of(vario), (long long)nsys, d_count, d_offset, d_xyz, d_val,
                                d_target_xyz, d_est, d_var, d_weights, p->ctr, p->num_cu * 4,
                                p->stream));
  p->last_nsys = nsys;
  p->last_kriged = nsys;
  return OKR_OK;
}

okr_status okr_marching_cubes(okr_plan* p, const float* d_volume, float iso, float* d_tris,
                              int64_t* d_cube, int64_t max_tris, int64_t* n_tris) {
  if (!p) return OKR_E_INVALID_ARG;
  if (!d_volume || !n_tris) return fail(p, OKR_E_INVALID_ARG, "volume and n_tris are required");
  if (max_tris < 0) return fail(p, OKR_E_INVALID_ARG, "max_tris must be >= 0");
  if (max_tris > 0 && !d_tris) return fail(p, OKR_E_INVALID_ARG, "tris is required when max_tris > 0");
  *n_tris = 0;
  const okr::Geometry& g = p->geo;
  const long long nz = (long long)(g.nslices - 1) * g.f + 1, ny = g.ny, nx = g.nx;
  if (g.nslices < 1 || nz < 2 || ny < 2 || nx < 2) return OKR_OK;
  const okr::McGrid mg = okr::mc_grid(nz, ny, nx);
  if ((mg.nwaves + 3) / 4 > 0x7fffffffLL || mg.ntile > 0x7fffffffLL)
    return fail(p, OKR_E_SHAPE, "volume too large for marching cubes");
  if (!p->mc_tab) {
    const okr::McTable& t = okr::mc_table();
    if (hipMalloc(&p->mc_tab, sizeof(okr::McTable)) != hipSuccess ||
        hipMalloc(&p->mc_cnt, sizeof(uint32_t) * mg.ncnt) != hipSuccess ||
        hipMalloc(&p->mc_tile, sizeof(unsigned long long) * (mg.ntile + 1)) != hipSuccess) {
      (void)hipGetLastError();
      hipFree(p->mc_tab);
      hipFree(p->mc_cnt);
      hipFree(p->mc_tile);
      p->mc_tab = nullptr;
      p->mc_cnt = nullptr;
      p->mc_tile = nullptr;
      return fail(p, OKR_E_OOM, "marching cubes workspace");
    }
    OKR_HIP(p, hipMemcpy(p->mc_tab, &t, sizeof(t), hipMemcpyHostToDevice));
  }
  unsigned long long total = 0;
  {
    PhaseTimer t(p, OKR_PHASE_MESH);
    OKR_HIP(p, okr::launch_mc_count(d_volume, (int)nx, (int)ny, mg, iso, p->mc_tab, p->mc_cnt,
                                    p->stream));
    OKR_HIP(p, okr::launch_mc_scan(p->mc_cnt, mg, p->mc_tile, p->stream));
    if (max_tris > 0)
      OKR_HIP(p, okr::launch_mc_emit(d_volume, (int)nx, (int)ny, mg, iso, p->mc_tab, p->mc_cnt,
                                     p->mc_tile, d_tris, (long long*)d_cube, (long long)max_tris,
                                     p->stream));
  }
  OKR_HIP(p, hipMemcpyAsync(&total, p->mc_tile + mg.ntile, sizeof(total), hipMemcpyDeviceToHost,
                            p->stream));
  OKR_HIP(p, hipStreamSynchronize(p->stream));
  *n_tris = (int64_t)total;
  if (max_tris > 0 && (long long)total > max_tris)
    return fail(p, OKR_E_CAPACITY,
                "marching cubes: " + std::to_string(total) + " triangles, buffer holds " +
                    std::to_string(max_tris));
  return OKR_OK;
}

namespace {

// Rounded normals (d1, d2) of the eight orientations: the normal angle
// (atan s from the x1 axis for the horizontal cone, 90 degrees minus atan s
// for the vertical one) to the nearest multiple of 45 degrees.
void edge_normals(int n1[8], int n2[8]) {
  static const int off1[4] = {1, 1, 0, -1}, off2[4] = {0, 1, 1, 1};
  for (int k = 0; k < okr::edge::kOrient; ++k) {
    const double deg = std::atan(okr::edge::kShears[k].s) * (180.0 / M_PI);
    const double ang = okr::edge::kShears[k].cone == 0 ? deg : 90.0 - deg;
    const int q = (((int)std::nearbyint(ang / 45.0)) % 4 + 4) % 4;
    n1[k] = off1[q];
    n2[k] = off2[q];
  }
}

}  // namespace

okr_status okr_edge_filters(double* taps, int32_t* normals) {
  if (taps)
    std::memcpy(taps, &okr::edge::kTapTable, sizeof(okr::edge::kTapTable));
  if (normals) {
    int n1[8], n2[8];
    edge_normals(n1, n2);
    for (int k = 0; k < 8; ++k) {
      normals[2 * k] = n1[k];
      normals[2 * k + 1] = n2[k];
    }
  }
  return OKR_OK;
}

okr_status okr_edge_postpass(okr_plan* p, const float* d_volume, float* d_out, double tau,
                             uint8_t* d_edge, uint8_t* d_orient, double* d_mag) {
  if (!p) return OKR_E_INVALID_ARG;
  if (!d_volume || !d_out) return fail(p, OKR_E_INVALID_ARG, "volume and out are required");
  if (!std::isfinite(tau)) return fail(p, OKR_E_INVALID_ARG, "tau must be finite");
  if (std::sqrt(2.0) != okr::edge::kSqrt2)
    return fail(p, OKR_E_UNSUPPORTED, "host sqrt(2) differs from the filters' constant");
  const okr::Geometry& g = p->geo;
  const long long nz = (long long)(g.nslices - 1) * g.f + 1, ny = g.ny, nx = g.nx;
  const long long vox = nz * ny * nx;
  const int wr = okr::edge_words_per_row((int)ny);
  const long long words = (nz + 2) * wr;
  if (nz < 1 || vox <= 0) return OKR_OK;
  if (nz + 2 > 0x7fffffffLL || words > 0x7fffffffLL || (words + 3) / 4 > 0x7fffffffLL ||
      nz * ny > 0xffffffffLL)
    return fail(p, OKR_E_SHAPE, "volume too large for the edge post-pass");
  const char* vb = reinterpret_cast<const char*>(d_volume);
  const char* ob = reinterpret_cast<const char*>(d_out);
  const long long bytes = vox * (long long)sizeof(float);
  if (vb != ob && vb < ob + bytes && ob < vb + bytes)
    return fail(p, OKR_E_INVALID_ARG, "out overlaps volume without being equal to it");
  if (!p->edge_mag) {
    if (hipMalloc(&p->edge_mag, sizeof(double) * vox) != hipSuccess ||
        hipMalloc(&p->edge_theta, vox) != hipSuccess ||
        hipMalloc(&p->edge_bits, sizeof(uint32_t) * words * nx) != hipSuccess) {
      (void)hipGetLastError();
      hipFree(p->edge_mag);
      hipFree(p->edge_theta);
      hipFree(p->edge_bits);
      p->edge_mag = nullptr;
      p->edge_theta = nullptr;
      p->edge_bits = nullptr;
      return fail(p, OKR_E_OOM, "edge post-pass workspace");
    }
  }
  if (p->edge_lds_max < 0) {
    int v = 0;
    OKR_HIP(p, hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device));
    p->edge_lds_max = v;
  }
  okr::EdgeArgs a{};
  a.volume = d_volume;
  a.out = d_out;
  a.mag = d_mag ? d_mag : p->edge_mag;
  a.theta = p->edge_theta;
  a.bits = p->edge_bits;
  a.edge_out = d_edge;
  a.orient_out = d_orient;
  a.tau = tau;
  a.nz = (int)nz;
  a.ny = (int)ny;
  a.nx = (int)nx;
  a.wr = wr;
  int n1[8], n2[8];
  edge_normals(n1, n2);
  for (int k = 0; k < 8; ++k) {
    a.n1 |= (uint32_t)(n1[k] + 1) << (4 * k);
    a.n2 |= (uint32_t)(n2[k] + 1) << (4 * k);
  }
  {
    PhaseTimer t(p, OKR_PHASE_EDGE_SHEAR);
    OKR_HIP(p, okr::launch_edge_shear(a, p->stream));
  }
  {
    PhaseTimer t(p, OKR_PHASE_EDGE_THIN);
    OKR_HIP(p, okr::launch_edge_nms(a, p->stream));
  }
  {
    PhaseTimer t(p, OKR_PHASE_EDGE_TRACE);
    if (d_out != d_volume)
      OKR_HIP(p, hipMemcpyAsync(d_out, d_volume, bytes, hipMemcpyDeviceToDevice, p->stream));
    hipError_t err = hipSuccess;
    okr::launch_edge_trace(a, p->edge_lds_max, p->stream, &err);
    OKR_HIP(p, err);
  }
  return OKR_OK;
}

okr_status okr_plan_set_graph(okr_plan* p, int32_t enable) {
  if (!p) return OKR_E_INVALID_ARG;
  p->use_graph = enable != 0;
  if (!p->use_graph) drop_graph(p);
  return OKR_OK;
}

okr_status okr_select(okr_plan* p, const uint8_t* d_edge, uint64_t* d_bits, uint8_t* d_count) {
  if (!p) return OKR_E_INVALID_ARG;
  if (!d_bits || !d_count) return fail(p, OKR_E_INVALID_ARG, "bits and count are required");
  const okr::Geometry& g = p->geo;
  p->loso_ready = false;   // the counters a pending okr_loso_backward reads are reset
  if (g.nsys == 0) return OKR_OK;
  OKR_HIP(p, okr::launch_reset(p->ctr, p->stream));
  OKR_HIP(p, okr::launch_select(d_edge, g, p->rule, d_bits, d_count, p->ctr, p->stream));
  p->last_nsys = g.nsys;
  p->last_kriged = 0;
  return OKR_OK;
}

okr_status okr_plan_set_profiling(okr_plan* p, int32_t enable) {
  if (!p) return OKR_E_INVALID_ARG;
  p->profiling = enable != 0;
  return OKR_OK;
}

okr_status okr_loso_forward(okr_plan* p, const okr_variogram* vario, const float* d_slices,
                            const uint8_t* d_edge, double* d_loss) {
  if (!p) return OKR_E_INVALID_ARG;
  std::string msg;
  okr_status st = validate_vario(vario, &msg);
  if (st != OKR_OK) return fail(p, st, msg);
  if (!d_slices || !d_loss) return fail(p, OKR_E_INVALID_ARG, "slices and loss are required");
  if (p->prob.algo == OKR_ALGO_PLAIN_PER_VOXEL)
    return fail(p, OKR_E_UNSUPPORTED, "leave-one-slice-out needs a batched plan");
  if (p->geo.f != 2)
    return fail(p, OKR_E_UNSUPPORTED,
                "leave-one-slice-out uses the upsample-2 geometry (held-out slice half-way)");
  if (p->geo.nslices < 3) return fail(p, OKR_E_SHAPE, "leave-one-slice-out needs >= 3 slices");
  p->loso_ready = false;
  okr::Geometry gl = p->geo;
  gl.nsys = gl.plane * (gl.nslices - 2);
  const size_t nl = (size_t)gl.nsys;
  if (!p->loso_resid) {
    if ((st = dev_alloc(p, &p->loso_resid, nl)) != OKR_OK) return st;
    if ((st = dev_alloc(p, &p->loso_gpart, 3 * nl)) != OKR_OK) return st;
    if ((st = dev_alloc(p, &p->loso_partial, 256 * 3)) != OKR_OK) return st;
  }
  PhaseTimer t(p, OKR_PHASE_LOSO);
  OKR_HIP(p, okr::launch_reset(p->ctr, p->stream));
  OKR_HIP(p, okr::launch_tables(vario_of(vario), gl, tables_of(p), p->stream));
  OKR_HIP(p, okr::launch_select_step(d_edge, gl, 2, gl.nslices - 2, p->rule, p->bits, p->count,
                                     p->ctr, p->stream));
  OKR_HIP(p, okr::launch_bucket(p->count, gl, gl.f + 1 + gl.drift, p->perm, p->ctr, p->stream));
  okr::SolveArgs a = solve_args(p, vario);
  a.geo = gl;
  a.slices = d_slices;
  a.step = 2;
  a.resid = p->loso_resid;
  a.gpart = p->loso_gpart;
  a.inv_count = 1.0 / (double)gl.nsys;
  OKR_HIP(p, okr::launch_loso_forward(a, persistent_grid(p), p->stream));
  OKR_HIP(p, okr::launch_reduce(p->loso_resid, gl.nsys, 1, a.inv_count, p->loso_partial, d_loss,
                                true, p->stream));
  p->loso_ready = true;
  p->loso_vario = *vario;
  p->loso_slices = d_slices;
  p->loso_edge = d_edge;
  p->last_nsys = gl.nsys;
  p->last_kriged = gl.nsys;
  return OKR_OK;
}

okr_status okr_loso_backward(okr_plan* p, double* d_grad) {
  if (!p) return OKR_E_INVALID_ARG;
  if (!d_grad) return fail(p, OKR_E_INVALID_ARG, "grad is required");
  if (!p->loso_ready)
    return fail(p, OKR_E_INVALID_ARG, "okr_loso_backward needs a preceding okr_loso_forward");
  okr::Geometry gl = p->geo;
  gl.nsys = gl.plane * (gl.nslices - 2);
  PhaseTimer t(p, OKR_PHASE_LOSO);
  okr::SolveArgs a = solve_args(p, &p->loso_vario);
  a.geo = gl;
  a.slices = p->loso_slices;
  a.step = 2;
  a.resid = p->loso_resid;
  a.gpart = p->loso_gpart;
  a.inv_count = 1.0 / (double)gl.nsys;
  OKR_HIP(p, okr::launch_reset_cursors(p->ctr, p->stream));
  OKR_HIP(p, okr::launch_loso_backward(a, persistent_grid(p), p->stream));
  OKR_HIP(p, okr::launch_reduce(p->loso_gpart, gl.nsys, 3, 1.0, p->loso_partial, d_grad, false,
                                p->stream));
  return OKR_OK;
}

okr_status okr_stats_get(okr_plan* p, okr_stats* out) {
  if (!p || !out) return OKR_E_INVALID_ARG;
  OKR_HIP(p, hipStreamSynchronize(p->stream));
  okr::DevCounters c;
  OKR_HIP(p, hipMemcpy(&c, p->ctr, sizeof(c), hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof(*out));
  out->n_systems = p->last_nsys;
  out->n_kriged = p->last_kriged;
  for (int i = 0; i < okr::kHist && i < 128; ++i) out->bucket[i] = (int64_t)c.hist[i];
  out->n_floor_filled = (int64_t)c.floor_filled;
  out->n_refined = (int64_t)c.refined;
  out->n_fp64_fallback = (int64_t)c.fp64_fallback;
  out->n_nonpositive_pivot = (int64_t)c.bad_pivot;
  float k;
  std::memcpy(&k, &c.max_kappa_bits, sizeof(k));
  out->max_kappa_est = k;
  drain_marks(p);
  for (int i = 0; i < OKR_NUM_PHASES; ++i) {
    out->phase_ms[i] = p->phase_ms[i];
    out->phase_calls[i] = p->phase_calls[i];
    p->phase_ms[i] = 0.0;
    p->phase_calls[i] = 0;
  }
  out->n_not_converged = (int64_t)c.failed;
  out->n_refine_unconverged = (int64_t)c.unconverged;
  out->kappa_window = p->kw_valid ? p->kappa_w : 0.0;
  out->direct_fp64 = p->last_direct64 ? 1 : 0;
  if (c.nonfinite) return fail(p, OKR_E_NONFINITE, "a known voxel is not finite");
  if (c.bad_input) return fail(p, OKR_E_SHAPE, "a point system has a count outside 1..98");
  if (p->prob.strict && c.failed)
    return fail(p, OKR_E_NOT_CONVERGED, "a system met a non-positive pivot in FP64 as well");
  return OKR_OK;
}

}  // extern "C"

// ---- okr_execute_noalloc: okr_execute with a static workspace ----
namespace {

// The workspace of one execute of up to kStaticMaxSystems (column, gap)
// systems, in a file-scope device array that every GPU the library runs on
// holds until the process ends. Layout (each part 256-byte aligned): counters,
// FP64 and FP32 tables, full-window pattern weights, then per system the
// kept mask (2 x u64), the count byte, the size-sorted permutation (u32) and
// the FP64 re-solve list (u32).
constexpr long long kStaticMaxSystems = 1LL << 20;
constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kOffCtr = 0;
constexpr size_t kOffTabs = kOffCtr + align256(sizeof(okr::DevCounters));
constexpr size_t kOffTabsF = kOffTabs + align256(sizeof(double) * (4 * okr::kTcSize + 4 * okr::kT0Size));
constexpr size_t kOffPattern = kOffTabsF + align256(sizeof(float) * (okr::kTcSize + okr::kT0Size));
constexpr size_t kOffBits =
    kOffPattern + align256(sizeof(double) * okr::kPatDoubles);
constexpr size_t kOffCount = kOffBits + align256(sizeof(uint64_t) * 2 * kStaticMaxSystems);
constexpr size_t kOffPerm = kOffCount + align256(kStaticMaxSystems);
constexpr size_t kOffFallback = kOffPerm + align256(sizeof(uint32_t) * kStaticMaxSystems);
constexpr size_t kStaticBytes = kOffFallback + align256(sizeof(uint32_t) * kStaticMaxSystems);

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

// Device address of `scratch` per device, from hipGetSymbolAddress on the
// first call made with that device current (the array's host-side name is
// not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

okr_status static_workspace(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return OKR_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return OKR_E_DEVICE;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return OKR_OK;
}

}  // namespace

extern "C" {

okr_status okr_execute_noalloc(const okr_problem* problem, void* hip_stream,
                               const okr_variogram* vario, const float* d_slices,
                               const uint8_t* d_edge, float* d_volume, float* d_variance,
                               uint8_t* d_flags, int32_t* d_status) {
  std::string msg;
  okr_status st = validate_problem(problem, &msg);
  if (st != OKR_OK) return st;
  if (validate_vario(vario, &msg) != OKR_OK) return OKR_E_INVALID_ARG;
  if (!d_slices || !d_volume) return OKR_E_INVALID_ARG;
  const long long nsys =
      (long long)problem->nx * problem->ny * (problem->nslices > 1 ? problem->nslices - 1 : 0);
  if (nsys > kStaticMaxSystems) return OKR_E_SHAPE;
  okr_plan p;
  if ((st = init_plan_shape(&p, problem, hip_stream)) != OKR_OK) return st;
  unsigned char* base = nullptr;
  if ((st = static_workspace(p.device, &base)) != OKR_OK) return st;
  p.ctr = reinterpret_cast<okr::DevCounters*>(base + kOffCtr);
  p.tabs = reinterpret_cast<double*>(base + kOffTabs);
  p.tabs_f = reinterpret_cast<float*>(base + kOffTabsF);
  p.pattern_w = reinterpret_cast<double*>(base + kOffPattern);
  p.bits = reinterpret_cast<uint64_t*>(base + kOffBits);
  p.count = base + kOffCount;
  p.perm = reinterpret_cast<uint32_t*>(base + kOffPerm);
  p.fallback = reinterpret_cast<uint32_t*>(base + kOffFallback);
  st = enqueue_execute(&p, p.stream, vario, d_slices, d_edge, d_volume, d_variance, d_flags);
  if (st == OKR_OK && d_status &&
      okr::launch_status(p.ctr, problem->strict, d_status, p.stream) != hipSuccess) {
    (void)hipGetLastError();
    st = OKR_E_DEVICE;
  }
  // the plan's pointers belong to the static workspace: nothing to free
  p.ctr = nullptr; p.tabs = nullptr; p.tabs_f = nullptr; p.pattern_w = nullptr;
  p.bits = nullptr; p.count = nullptr; p.perm = nullptr; p.fallback = nullptr;
  return st;
}

}  // extern "C"
