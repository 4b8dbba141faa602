// Ordinary kriging of explicitly given point sets (the point entry point).
//
// Each system is a set of n neighbour points with 3-D coordinates and values
// and one target point. The covariance of every pair and of every point with
// the target is evaluated from the variogram in FP64 (Appendix A's extended
// covariance matrix and vector with the single constant predictor), and the
// bordered system [[C, 1], [1^T, 0]] [w; mu] = [c0; 1] is solved through a
// Cholesky factor of C:
//   x_1 = C^{-1} 1,  x_c = C^{-1} c0,  mu = (1'x_c - 1) / 1'x_1,
//   w = x_c - mu x_1,  z_hat = w'z,  sigma^2 = sill - w'c0 - mu.
// One wavefront per system; C is factored in place in LDS in FP64, lanes
// running over rows. Invalid counts and non-finite inputs are latched in the
// counters and reported at the next synchronising call; a non-positive pivot
// gives NaN outputs for that system and is counted.
#include <algorithm>

#include "okrig_internal.h"
#include "variogram.h"

namespace okr {
namespace {

constexpr int kPtMax = kMaxCand;        // points per system
constexpr int kPtLd = kPtMax + 1;       // row stride of the factor (odd: fewer bank conflicts)

__device__ __forceinline__ double lane_d(double x, int l) {
  long long b = __double_as_longlong(x);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return lane_d(x, 0);
}

// K wave sums at once, on the DPP network: quad_perm [1,0,3,2] and [2,3,0,1],
// row_ror:4 and row_ror:8 give every lane its 16-lane row's sum; row_bcast:15
// (into rows 1 and 3) and row_bcast:31 (into rows 2 and 3) then leave the
// wave's sum in lane 63, whose value is made uniform.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp64(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int K>
__device__ __forceinline__ void wave_sums_k(double (&x)[K]) {
#pragma unroll
  for (int q = 0; q < K; ++q) x[q] += dpp64<0xB1, 0xf>(x[q]);
#pragma unroll
  for (int q = 0; q < K; ++q) x[q] += dpp64<0x4E, 0xf>(x[q]);
#pragma unroll
  for (int q = 0; q < K; ++q) x[q] += dpp64<0x124, 0xf>(x[q]);
#pragma unroll
  for (int q = 0; q < K; ++q) x[q] += dpp64<0x128, 0xf>(x[q]);
#pragma unroll
  for (int q = 0; q < K; ++q) x[q] += dpp64<0x142, 0xa>(x[q]);
#pragma unroll
  for (int q = 0; q < K; ++q) x[q] += dpp64<0x143, 0xc>(x[q]);
#pragma unroll
  for (int q = 0; q < K; ++q) x[q] = lane_d(x[q], 63);
}


// C = L L^T in place in the lower triangle of A (row stride kPtLd), lanes over
// rows. Returns true (uniformly) on a non-positive pivot.
__device__ bool chol_lds(double* A, int n) {
  const int lane = threadIdx.x & 63;
  for (int k = 0; k < n; ++k) {
    const double d = A[k * kPtLd + k];
    if (!(d > 0.0)) return true;
    const double is = 1.0 / sqrt(d);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      if (i > k && i < n) A[i * kPtLd + k] *= is;
    }
    if (lane == 0) A[k * kPtLd + k] = d * is;   // L[k][k] = sqrt(d)
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      if (i > k && i < n) {
        const double lik = A[i * kPtLd + k];
        for (int j = k + 1; j <= i; ++j) A[i * kPtLd + j] -= lik * A[j * kPtLd + k];
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  return false;
}

// The factorisation of chol_lds by a whole workgroup, two columns per step:
// every thread reads the 2 x 2 pivot block, then each wave takes rows i of the
// trailing matrix (its lanes the columns j <= i) and applies both rank-1
// updates in turn, a_ij - l_i0 l_j0 - l_i1 l_j1 with l_i1 from the updated
// a_i,p+1, reading columns p and p + 1 as they were; after a barrier the two
// scaled columns are written. Each element sees the operations of two single
// steps in their order, so the factor is that of chol_lds. Returns true
// (uniformly) on a non-positive pivot.
__device__ bool chol_block(double* A, int n) {
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  int p = 0;
  for (; p + 1 < n; p += 2) {
    const double d0 = A[p * kPtLd + p];
    if (!(d0 > 0.0)) return true;
    const double is0 = 1.0 / sqrt(d0);
    const double l10 = A[(p + 1) * kPtLd + p] * is0;
    const double d1 = A[(p + 1) * kPtLd + p + 1] - l10 * l10;
    if (!(d1 > 0.0)) return true;
    const double is1 = 1.0 / sqrt(d1);
    // trailing rows over waves, the row's columns over lanes
    for (int i = p + 2 + (int)(threadIdx.x >> 6); i < n; i += nw) {
      const double li0 = A[i * kPtLd + p] * is0;
      const double li1 = (A[i * kPtLd + p + 1] - li0 * l10) * is1;
      for (int j = p + 2 + lane; j <= i; j += 64) {
        const double lj0 = A[j * kPtLd + p] * is0;
        const double lj1 = (A[j * kPtLd + p + 1] - lj0 * l10) * is1;
        A[i * kPtLd + j] = (A[i * kPtLd + j] - li0 * lj0) - li1 * lj1;
      }
    }
    __syncthreads();   // every read of columns p, p + 1 and of the pivots is done
    for (int i = p + 2 + (int)threadIdx.x; i < n; i += blockDim.x) {
      const double li0 = A[i * kPtLd + p] * is0;
      A[i * kPtLd + p] = li0;
      A[i * kPtLd + p + 1] = (A[i * kPtLd + p + 1] - li0 * l10) * is1;
    }
    if (threadIdx.x == 0) {
      A[p * kPtLd + p] = d0 * is0;               // L[p][p] = sqrt(d0)
      A[(p + 1) * kPtLd + p] = l10;
      A[(p + 1) * kPtLd + p + 1] = d1 * is1;     // L[p+1][p+1] = sqrt(d1)
    }
    __syncthreads();
  }
  if (p < n) {   // the last column of an odd n
    const double d = A[p * kPtLd + p];
    if (!(d > 0.0)) return true;
    const double is = 1.0 / sqrt(d);
    __syncthreads();   // every thread has read the pivot
    if (threadIdx.x == 0) A[p * kPtLd + p] = d * is;
    __syncthreads();
  }
  return false;
}

// Solves L L^T x = b for two right-hand sides held by rows (b[h] of lane l is
// row l + 64 h); on return b holds x.
__device__ void subst_lds(const double* A, int n, double (&b)[2], double (&c)[2]) {
  const int lane = threadIdx.x & 63;
  for (int k = 0; k < n; ++k) {
    const double lkk = A[k * kPtLd + k];
    const int hk = k >> 6, lk = k & 63;
    const double yb = (hk ? lane_d(b[1], lk) : lane_d(b[0], lk)) / lkk;
    const double yc = (hk ? lane_d(c[1], lk) : lane_d(c[0], lk)) / lkk;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      if (i == k) {
        b[h] = yb;
        c[h] = yc;
      } else if (i > k && i < n) {
        const double lik = A[i * kPtLd + k];
        b[h] -= lik * yb;
        c[h] -= lik * yc;
      }
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    const double lkk = A[k * kPtLd + k];
    const int hk = k >> 6, lk = k & 63;
    const double xb = (hk ? lane_d(b[1], lk) : lane_d(b[0], lk)) / lkk;
    const double xc = (hk ? lane_d(c[1], lk) : lane_d(c[0], lk)) / lkk;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      if (i == k) {
        b[h] = xb;
        c[h] = xc;
      } else if (i < k) {
        const double lki = A[k * kPtLd + i];
        b[h] -= lki * xb;
        c[h] -= lki * xc;
      }
    }
  }
}

// subst_lds for NR right-hand sides at once (the independent chains of one
// step interleave), with the reciprocal of each pivot taken once.
template <int NR>
__device__ void subst_lds_n(const double* A, int n, double (&b)[NR][2]) {
  const int lane = threadIdx.x & 63;
  for (int k = 0; k < n; ++k) {
    const double ikk = 1.0 / A[k * kPtLd + k];
    const int hk = k >> 6, lk = k & 63;
    const double l0 = (lane > k && lane < n) ? A[lane * kPtLd + k] : 0.0;
    const double l1 = (lane + 64 > k && lane + 64 < n) ? A[(lane + 64) * kPtLd + k] : 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double y = (hk ? lane_d(b[r][1], lk) : lane_d(b[r][0], lk)) * ikk;
      b[r][0] = lane == k ? y : b[r][0] - l0 * y;
      b[r][1] = lane + 64 == k ? y : b[r][1] - l1 * y;
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    const double ikk = 1.0 / A[k * kPtLd + k];
    const int hk = k >> 6, lk = k & 63;
    const double l0 = lane < k ? A[k * kPtLd + lane] : 0.0;
    const double l1 = lane + 64 < k ? A[k * kPtLd + lane + 64] : 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double x = (hk ? lane_d(b[r][1], lk) : lane_d(b[r][0], lk)) * ikk;
      b[r][0] = lane == k ? x : b[r][0] - l0 * x;
      b[r][1] = lane + 64 == k ? x : b[r][1] - l1 * x;
    }
  }
}

__global__ __launch_bounds__(64) void points_kernel(Vario v, long long nsys,
                                                    const int32_t* __restrict__ count,
                                                    const int64_t* __restrict__ offset,
                                                    const float* __restrict__ xyz,
                                                    const float* __restrict__ val,
                                                    const float* __restrict__ txyz,
                                                    float* __restrict__ est, float* __restrict__ var,
                                                    float* __restrict__ weights,
                                                    DevCounters* __restrict__ ctr) {
  __shared__ double A[kPtMax * kPtLd];
  __shared__ double px[kPtMax], py[kPtMax], pz[kPtMax];
  const int lane = threadIdx.x;
  for (long long sys = blockIdx.x; sys < nsys; sys += gridDim.x) {
    const int n = count[sys];
    const long long o = offset[sys];
    if (n < 1 || n > kPtMax || o < 0) {
      if (lane == 0) {
        atomicOr(&ctr->bad_input, 1u);
        est[sys] = __builtin_nanf("");
        if (var) var[sys] = __builtin_nanf("");
      }
      continue;
    }
    const double tx = txyz[3 * sys], ty = txyz[3 * sys + 1], tz = txyz[3 * sys + 2];
    // points: lane holds points i = lane and lane + 64
    double zv[2] = {0.0, 0.0}, c0[2] = {0.0, 0.0};
    bool finite = isfinite(tx) && isfinite(ty) && isfinite(tz);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      if (i < n) {
        const double x = xyz[3 * (o + i)], y = xyz[3 * (o + i) + 1], z = xyz[3 * (o + i) + 2];
        zv[h] = val[o + i];
        finite = finite && isfinite(x) && isfinite(y) && isfinite(z) && isfinite(zv[h]);
        px[i] = x;
        py[i] = y;
        pz[i] = z;
        const double dx = x - tx, dy = y - ty, dz = z - tz;
        c0[h] = cov_d(v, sqrt(dx * dx + dy * dy + dz * dz));
      }
    }
    if (__any(!finite) && lane == 0) atomicOr(&ctr->nonfinite, 1u);
    __builtin_amdgcn_wave_barrier();
    // C, lower triangle (rows i by lane)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      if (i < n) {
        for (int j = 0; j <= i; ++j) {
          const double dx = px[i] - px[j], dy = py[i] - py[j], dz = pz[i] - pz[j];
          A[i * kPtLd + j] = i == j ? v.sill : cov_d(v, sqrt(dx * dx + dy * dy + dz * dz));
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    const bool bad = chol_lds(A, n);
    if (bad) {
      if (lane == 0) {
        atomicAdd(&ctr->bad_pivot, 1ull);
        est[sys] = __builtin_nanf("");
        if (var) var[sys] = __builtin_nanf("");
      }
      if (weights) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (lane + 64 * h < n) weights[o + lane + 64 * h] = __builtin_nanf("");
      }
      continue;
    }
    // two right-hand sides: b = 1 and b = c0
    double b1[2], bc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      b1[h] = lane + 64 * h < n ? 1.0 : 0.0;
      bc[h] = c0[h];
    }
    subst_lds(A, n, b1, bc);
    const double s1 = wave_sum(b1[0] + b1[1]);
    const double sc = wave_sum(bc[0] + bc[1]);
    const double mu = (sc - 1.0) / s1;
    const double w0 = bc[0] - mu * b1[0], w1 = bc[1] - mu * b1[1];
    const double zh = wave_sum(w0 * zv[0] + w1 * zv[1]);
    const double wc = wave_sum(w0 * c0[0] + w1 * c0[1]);
    if (lane == 0) {
      est[sys] = (float)zh;
      if (var) var[sys] = (float)(v.sill - wc - mu);
    }
    if (weights) {
      if (lane < n) weights[o + lane] = (float)w0;
      if (lane + 64 < n) weights[o + lane + 64] = (float)w1;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// ---- exact cache of the full-window pattern ----
// Systems that keep every candidate of the window share their matrix: the
// covariances depend only on the offsets (translation invariance). Their
// weights w_t and variances are computed once per launch in FP64 (one wave),
// and each such system is then a gather of its values and f-1 dot products.
// With the slice predictor (Appendix A with predictors 1 and the slice s)
// the weights are still pure geometry: from X_1 = C^-1 1, X_s = C^-1 s and
// X_t = C^-1 c0_t, the multipliers solve G phi = (1'X_t - 1, s'X_t - t/f) with
// G = Q'C^-1 Q, w_t = X_t - phi_1 X_1 - phi_s X_s and
// sigma^2 = sill - w_t'c0_t - phi_1 - phi_s t/f.

// Candidate c of the window -> (dx, dy, s) with the canonical index
// c = s W^2 + (dy + r) W + (dx + r).
__device__ __forceinline__ void cand_xyz(int c, const Geometry& g, int* dx, int* dy, int* s) {
  *s = c >= g.W2;
  const int o = c - *s * g.W2;
  *dy = o / g.W - g.r;
  *dx = o - (o / g.W) * g.W - g.r;
}

__global__ __launch_bounds__(1024) void pattern_weights_kernel(Vario v, Geometry g, double* pat,
                                                               DevCounters* ctr) {
  __shared__ double A[kPtMax * kPtLd];
  double* W = pat + kPatW;
  double* wvar = pat + kPatVar;
  double* G = pat + kPatG;
  double* U = pat + kPatU;
  double* C0 = pat + kPatC0;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int n = g.ncand;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e - (e / n) * n;
    if (j > i) continue;
    int dxi, dyi, si, dxj, dyj, sj;
    cand_xyz(i, g, &dxi, &dyi, &si);
    cand_xyz(j, g, &dxj, &dyj, &sj);
    const double ddx = dxi - dxj, ddy = dyi - dyj, ddz = (double)(si - sj) * g.f;
    A[i * kPtLd + j] = i == j ? v.sill : cov_d(v, sqrt(ddx * ddx + ddy * ddy + ddz * ddz));
  }
  __syncthreads();
  if (chol_block(A, n)) {
    if (threadIdx.x == 0) atomicAdd(&ctr->bad_pivot, 1ull);
    for (int t = 0; t < g.f - 1; ++t) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) W[t * kMaxCand + i] = __builtin_nan("");
      if (threadIdx.x == 0) wvar[t] = __builtin_nan("");
    }
    for (int i = threadIdx.x; i < kMaxCand * kMaxCand; i += blockDim.x) G[i] = __builtin_nan("");
    for (int i = threadIdx.x; i < kMaxUpsample * kMaxCand; i += blockDim.x) U[i] = __builtin_nan("");
    return;
  }
  // G = C^{-1}, seven columns per wave (rows by symmetry: row c of G is
  // C^{-1} e_c); sixteen waves cover the 98 columns in one pass
  {
    constexpr int NR = 7;
    for (int c0 = NR * wid; c0 < n; c0 += NR * (int)(blockDim.x >> 6)) {
      double e[NR][2];
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int h = 0; h < 2; ++h) e[r][h] = lane + 64 * h == c0 + r ? 1.0 : 0.0;
      subst_lds_n<NR>(A, n, e);
#pragma unroll
      for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = lane + 64 * h;
          if (c0 + r < n && i < n) G[(c0 + r) * kMaxCand + i] = e[r][h];
        }
      __builtin_amdgcn_wave_barrier();
    }
  }
  // each wave solves the targets t = 1 + wid (mod waves) against the shared factor
  // slice of each candidate (0 lower, 1 upper) and, with the drift, X_s = C^-1 s
  double sl[2], xs[2] = {0.0, 0.0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = lane + 64 * h;
    int dx, dy, sc = 0;
    if (i < n) cand_xyz(i, g, &dx, &dy, &sc);
    sl[h] = i < n ? (double)sc : 0.0;
  }
  if (g.drift) {
    double unused[2] = {0.0, 0.0};
    xs[0] = sl[0];
    xs[1] = sl[1];
    subst_lds(A, n, xs, unused);
    // C^{-1} s in the last row of U (f <= kMaxUpsample - 1 with the predictor)
    if (wid == 0) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (lane + 64 * h < n) U[(kMaxUpsample - 1) * kMaxCand + lane + 64 * h] = xs[h];
    }
  }
  for (int t = 1 + wid; t < g.f; t += blockDim.x >> 6) {
    double b1[2], bc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      b1[h] = i < n ? 1.0 : 0.0;
      bc[h] = 0.0;
      if (i < n) {
        int dx, dy, sc;
        cand_xyz(i, g, &dx, &dy, &sc);
        const double dz = (double)sc * g.f - t;
        bc[h] = cov_d(v, sqrt((double)(dx * dx + dy * dy) + dz * dz));
      }
    }
    const double c0[2] = {bc[0], bc[1]};
    subst_lds(A, n, b1, bc);
    // the full-window solves C^{-1} 1 and C^{-1} c0_t, and c0_t, for the
    // systems that take their weights from G
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = lane + 64 * h;
      if (i < n) {
        if (t == 1) U[i] = b1[h];
        U[t * kMaxCand + i] = bc[h];
        C0[(t - 1) * kMaxCand + i] = c0[h];
      }
    }
    const double s1 = wave_sum(b1[0] + b1[1]);
    const double sc = wave_sum(bc[0] + bc[1]);
    double w0, w1, lagr;
    if (!g.drift) {
      const double mu = (sc - 1.0) / s1;
      w0 = bc[0] - mu * b1[0];
      w1 = bc[1] - mu * b1[1];
      lagr = mu;
    } else {
      const double qt = (double)t / g.f;
      const double g11 = s1, g12 = wave_sum(xs[0] + xs[1]);
      const double g22 = wave_sum(sl[0] * xs[0] + sl[1] * xs[1]);
      const double r1 = sc - 1.0, r2 = wave_sum(sl[0] * bc[0] + sl[1] * bc[1]) - qt;
      const double det = g11 * g22 - g12 * g12;
      const double p1 = (g22 * r1 - g12 * r2) / det, ps = (g11 * r2 - g12 * r1) / det;
      w0 = bc[0] - p1 * b1[0] - ps * xs[0];
      w1 = bc[1] - p1 * b1[1] - ps * xs[1];
      lagr = p1 + ps * qt;
    }
    const double wc = wave_sum(w0 * c0[0] + w1 * c0[1]);
    if (lane < n) W[(t - 1) * kMaxCand + lane] = w0;
    if (lane + 64 < n) W[(t - 1) * kMaxCand + lane + 64] = w1;
    if (lane == 0) wvar[t - 1] = v.sill - wc - lagr;
    __builtin_amdgcn_wave_barrier();
  }
}

// The full-window systems apply the cached weights as a stencil. A workgroup
// of 64 x 4 threads covers a 64 x 16 tile of one gap: both bounding slices of
// the tile and its window halo are staged once in LDS, converted to FP64, with
// coalesced row loads. Each thread computes a column of kRows pixels, window
// row by window row: the staged rows its pixels need at one window row are the
// rows of the previous window row shifted by one, so each step reads one new
// row from LDS and the rest stay in registers; the weights of a window row are
// wave-uniform (scalar loads, an FMA operand each), so LDS serves only the
// slice values. A pixel's sum runs over slice, window row, window column for
// each target in turn, the order of the per-system FP64 weighted sum; its
// result is stored when its kept window is the full window (count = ncand).
// Targets go in groups of three (the weights of a group's missing targets
// repeat the last one and are not stored).
constexpr int kPTX = 64, kRows = 4, kPTY = 4 * kRows, kTGroup = 3;

template <int R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
void pattern_apply_kernel(const float* __restrict__ slices, const uint8_t* __restrict__ count,
                          Geometry g, const double* __restrict__ W,
                          const double* __restrict__ wvar, float* __restrict__ volume,
                          float* __restrict__ variance, uint8_t* __restrict__ flags) {
  constexpr int Wn = 2 * R + 1, W2 = Wn * Wn;
  constexpr int kTX = kPTX + 2 * R, kTY = kPTY + 2 * R;
  __shared__ double tile[2][kTY][kTX];
  const int n = g.ncand, nt = g.f - 1;
  const int gap = blockIdx.z, x0 = blockIdx.x * kPTX, y0 = blockIdx.y * kPTY;
  const int lx = threadIdx.x & (kPTX - 1), ly0 = (threadIdx.x / kPTX) * kRows;
  const int x = x0 + lx;
  // The loads below are unconditional, from coordinates clamped into the
  // image (values from outside are replaced or unused), so that every load of
  // a thread is in flight before the first is used: first the neighbour counts
  // of the thread's pixels, then its share of the tile,
  // tile[s][ty][tx] = slice gap + s at (y0 - R + ty, x0 - R + tx), 0 outside.
  uint8_t cn[kRows];
#pragma unroll
  for (int p = 0; p < kRows; ++p)
    cn[p] = count[(long long)gap * g.plane + (long long)min(y0 + ly0 + p, g.ny - 1) * g.nx +
                  min(x, g.nx - 1)];
  constexpr int kStage = (2 * kTY * kTX + 255) / 256;
  float sv[kStage];
  bool in[kStage];
#pragma unroll
  for (int it = 0; it < kStage; ++it) {
    const int i = min((int)threadIdx.x + 256 * it, 2 * kTY * kTX - 1);
    const int sl = i / (kTY * kTX), rem = i - sl * (kTY * kTX);
    const int ty = rem / kTX, tx = rem - ty * kTX;
    const int yy = y0 - R + ty, xx = x0 - R + tx;
    in[it] = yy >= 0 && yy < g.ny && xx >= 0 && xx < g.nx;
    const int yc = min(max(yy, 0), g.ny - 1), xc = min(max(xx, 0), g.nx - 1);
    sv[it] = slices[(long long)(gap + sl) * g.plane + (long long)yc * g.nx + xc];
  }
#pragma unroll
  for (int it = 0; it < kStage; ++it) {
    const int i = threadIdx.x + 256 * it;
    if (i < 2 * kTY * kTX) (&tile[0][0][0])[i] = in[it] ? (double)sv[it] : 0.0;
  }
  __syncthreads();
  if (x >= g.nx) return;
  // which of the thread's pixels take the cached weights
  unsigned keep = 0;
#pragma unroll
  for (int p = 0; p < kRows; ++p) {
    const int y = y0 + ly0 + p;
    if (y < g.ny && x >= R && y >= R && x + R < g.nx && y + R < g.ny && (cn[p] & 0x7f) == n)
      keep |= 1u << p;
  }
  if (!keep) return;
  for (int t0 = 0; t0 < nt; t0 += kTGroup) {
    const double* w[kTGroup];
#pragma unroll
    for (int t = 0; t < kTGroup; ++t) w[t] = W + (long long)min(t0 + t, nt - 1) * kMaxCand;
    double acc[kRows][kTGroup];
#pragma unroll
    for (int p = 0; p < kRows; ++p)
#pragma unroll
      for (int t = 0; t < kTGroup; ++t) acc[p][t] = 0.0;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      double z[kRows][Wn];   // z[(p + yy) % kRows]: staged row ly0 + p + yy
#pragma unroll
      for (int q = 0; q < kRows - 1; ++q)
#pragma unroll
        for (int xx = 0; xx < Wn; ++xx) z[q][xx] = tile[sl][ly0 + q][lx + xx];
#pragma unroll
      for (int yy = 0; yy < Wn; ++yy) {
        // The weights of this window row (3 x W doubles in SGPRs). An opaque
        // row offset keeps the rows' loads apart (not merged into wide loads
        // of every row at the top): the 2 x W x W x 3 weights do not fit in
        // SGPRs.
        int off = (sl * Wn + yy) * Wn;   // slot sl * W2 + yy * Wn
        asm volatile("" : "+s"(off));
        double wr[kTGroup][Wn];
#pragma unroll
        for (int t = 0; t < kTGroup; ++t)
#pragma unroll
          for (int xx = 0; xx < Wn; ++xx) wr[t][xx] = w[t][off + xx];
        const int qn = (yy + kRows - 1) % kRows;   // row ly0 + kRows - 1 + yy
#pragma unroll
        for (int xx = 0; xx < Wn; ++xx) z[qn][xx] = tile[sl][ly0 + kRows - 1 + yy][lx + xx];
#pragma unroll
        for (int t = 0; t < kTGroup; ++t)
#pragma unroll
          for (int xx = 0; xx < Wn; ++xx)
#pragma unroll
            for (int p = 0; p < kRows; ++p)
              acc[p][t] = fma(wr[t][xx], z[(p + yy) % kRows][xx], acc[p][t]);
      }
    }
    // pinned here: otherwise each pixel's sums sink into its conditional
    // store, and every window row's weights stay live until then
#pragma unroll
    for (int p = 0; p < kRows; ++p)
#pragma unroll
      for (int t = 0; t < kTGroup; ++t) asm volatile("" : "+v"(acc[p][t]));
#pragma unroll
    for (int p = 0; p < kRows; ++p) {
      if (!(keep >> p & 1u)) continue;
      const long long pix = (long long)(y0 + ly0 + p) * g.nx + x;
#pragma unroll
      for (int t = 0; t < kTGroup; ++t) {
        if (t0 + t >= nt) break;
        const long long o = ((long long)gap * g.f + t0 + t + 1) * g.plane + pix;
        volume[o] = (float)acc[p][t];
        if (variance) variance[o] = (float)wvar[t0 + t];
      }
    }
  }
  if (flags) {
#pragma unroll
    for (int p = 0; p < kRows; ++p)
      if (keep >> p & 1u) flags[(long long)gap * g.plane + (long long)(y0 + ly0 + p) * g.nx + x] = 0;
  }
}

// Systems that keep all but k <= kMaxDrop candidates of the full window
// (drop set D, kept set K) take their weights from the full window's inverse
// G = C^{-1} and its solves u_r = G b_r (b_0 = 1, b_t = c0_t): by the block
// inverse of C, C_KK^{-1} = G_KK - G_KD G_DD^{-1} G_DK, and since
// u_D = G_DK b_K + G_DD b_D,
//   x_r = C_KK^{-1} b_K = u_K - G_KD y_r,   G_DD y_r = u_D,
// exactly (up to rounding) and whatever b holds at the dropped candidates.
// Per system one wave: the k x k matrix G_DD is gathered into LDS and
// factored two columns per step (columns over lanes), the k-vectors y_r are
// solved with lanes over rows, and x_r for the kept candidates (two per lane)
// follow from rows of G.
// Then mu_t = (1'x_t - 1) / 1'x_0, w_t = x_t - mu_t x_0, the estimate w_t'z
// and the variance sill - w_t'c0_t - mu_t, all in FP64. Targets go in groups
// of three (x_0 solved again for each group).
struct DowndateScratch {
  double a[kMaxDrop][kMaxDrop + 1];   // G_DD, then its Cholesky factor (lower triangle)
  double ip[kMaxDrop];                // 1 / L[p][p]
  double y[kMaxDrop][5];              // the solutions y_r by row
  int dl[kMaxDrop];                   // the dropped candidates, ascending
};

// 1/sqrt(x) in FP64: the hardware estimate (relative error about 5e-8) and
// one second-order Newton step in residual form, y = y0 + y0 e (1/2 + 3e/8)
// with e = 1 - x y0^2.
__device__ __forceinline__ double rsq64(double x) {
  const double y0 = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y0, y0, 1.0);
  return fma(y0 * e, fma(0.375, e, 0.5), y0);
}
constexpr int kDdWaves = 4;

// G_DD (lower triangle) into LDS, two rows per pass (lanes 0..31 and 32..63);
// every load is issued before the first store, from indices clamped to the
// list. PASSES * 2 >= k.
template <int PASSES>
__device__ __forceinline__ void gather_gdd(DowndateScratch& ws, const double* __restrict__ G,
                                           int k, int lane) {
  const int j = lane & 31, jc = ws.dl[min(j, k - 1)];
  double gv[PASSES];
#pragma unroll
  for (int q = 0; q < PASSES; ++q) {
    const int i = min(2 * q + (lane >> 5), k - 1);
    gv[q] = G[ws.dl[i] * kMaxCand + jc];
  }
#pragma unroll
  for (int q = 0; q < PASSES; ++q) {
    const int i = 2 * q + (lane >> 5);
    if (i < k && j <= i) ws.a[i][j] = gv[q];
  }
}

template <bool DRIFT>
__global__ __launch_bounds__(64 * kDdWaves) __attribute__((amdgpu_waves_per_eu(4)))
void pattern_downdate_kernel(
    const float* __restrict__ slices, const uint64_t* __restrict__ bits,
    const uint8_t* __restrict__ count, const uint32_t* __restrict__ perm,
    DevCounters* __restrict__ ctr, Geometry g, double sill, const double* __restrict__ pat,
    int nlo, float* __restrict__ volume, float* __restrict__ variance,
    uint8_t* __restrict__ flags) {
  __shared__ DowndateScratch wsa[kDdWaves];
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  DowndateScratch& ws = wsa[wid];
  const double* G = pat + kPatG;
  const double* U = pat + kPatU;
  const double* C0 = pat + kPatC0;
  const int nc = g.ncand, nt = g.f - 1;
  const unsigned long long start = ctr->offsets[nc - 1];
  const unsigned long long end = ctr->offsets[nlo] + ctr->hist[nlo];
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  // the lane's two candidates: in range, and their offset in the slice stack
  const bool in0 = lane < nc, in1 = lane + 64 < nc;
  long long off0 = 0, off1 = 0;
  int dy0 = 0, dx0 = 0, dy1 = 0, dx1 = 0;
  double sl0 = 0.0, sl1 = 0.0;   // the candidates' slices (the second predictor)
  {
    int s;
    if (in0) {
      cand_xyz(lane, g, &dx0, &dy0, &s);
      off0 = (long long)s * g.plane + (long long)dy0 * g.nx + dx0;
      sl0 = (double)s;
    }
    if (in1) {
      cand_xyz(lane + 64, g, &dx1, &dy1, &s);
      off1 = (long long)s * g.plane + (long long)dy1 * g.nx + dx1;
      sl1 = (double)s;
    }
  }
  for (unsigned long long it = start + (unsigned long long)blockIdx.x * kDdWaves + wid; it < end;
       it += (unsigned long long)gridDim.x * kDdWaves) {
    const unsigned sys = __builtin_amdgcn_readfirstlane(perm[it]);
    // uniform values made scalar, so that the loops over them stay scalar
    const int k = __builtin_amdgcn_readfirstlane(nc - (count[sys] & 0x7f));
    if (k < 1 || k > kMaxDrop) continue;   // not a system of this range
    const uint64_t lo = bits[2ull * sys], hi = bits[2ull * sys + 1];
    const bool keep0 = in0 && ((lo >> lane) & 1ull);
    const bool keep1 = in1 && ((hi >> lane) & 1ull);
    const uint64_t m0 = __ballot(in0 && !keep0), m1 = __ballot(in1 && !keep1);
    if (__popcll(m0) + __popcll(m1) != k) continue;   // count and mask disagree: not ours
    if (in0 && !keep0) ws.dl[__popcll(m0 & below)] = lane;
    if (in1 && !keep1) ws.dl[__popcll(m0) + __popcll(m1 & below)] = lane + 64;
    __builtin_amdgcn_wave_barrier();
    // G_DD, lower triangle
    if (k <= 8)
      gather_gdd<4>(ws, G, k, lane);
    else if (k <= 16)
      gather_gdd<8>(ws, G, k, lane);
    else
      gather_gdd<kMaxDrop / 2>(ws, G, k, lane);
    __builtin_amdgcn_wave_barrier();
    // Cholesky, right-looking, two columns per step. A step reads the 2 x 2
    // pivot block and columns p, p + 1, then updates the trailing triangle
    // (lane: column j = p + 2 + (lane & 31), rows i = p + 2 + 2q + (lane >> 5))
    // in chunks of eight rows, each chunk's reads before its writes, to
    // a_ij - l_i0 l_j0 - l_i1 l_j1 (the two rank-1 updates in turn), and writes
    // the two scaled columns last (no read of the step needs them).
    bool bad = false;
    {
      constexpr int kChunk = 4;   // row pairs per chunk
      const int ho = lane >> 5;
      int p = 0;
      for (; p + 1 < k; p += 2) {
        const double d0 = lane_d(ws.a[p][p], 0);
        const double a10 = lane_d(ws.a[p + 1][p], 0);
        const double a11 = lane_d(ws.a[p + 1][p + 1], 0);
        if (!(d0 > 0.0)) {
          bad = true;
          break;
        }
        const double is0 = rsq64(d0);
        const double l10 = a10 * is0;
        const double d1 = a11 - l10 * l10;
        if (!(d1 > 0.0)) {
          bad = true;
          break;
        }
        const double is1 = rsq64(d1);
        const int j = p + 2 + (lane & 31), jc = min(j, k - 1);
        const double lj0 = ws.a[jc][p] * is0;
        const double lj1 = (ws.a[jc][p + 1] - lj0 * l10) * is1;
        const int m = k - p - 2;   // trailing rows
        for (int q0 = 0; 2 * q0 < m; q0 += kChunk) {
          double li0[kChunk], li1[kChunk], aij[kChunk];
#pragma unroll
          for (int q = 0; q < kChunk; ++q) {
            const int ic = min(p + 2 + 2 * (q0 + q) + ho, k - 1);
            li0[q] = ws.a[ic][p] * is0;
            li1[q] = (ws.a[ic][p + 1] - li0[q] * l10) * is1;
            aij[q] = ws.a[ic][jc];
          }
#pragma unroll
          for (int q = 0; q < kChunk; ++q) {
            const int i = p + 2 + 2 * (q0 + q) + ho;
            if (i < k && j <= i) ws.a[i][j] = (aij[q] - li0[q] * lj0) - li1[q] * lj1;
          }
        }
        if (lane == 0) {
          ws.a[p][p] = d0 * is0;
          ws.a[p + 1][p] = l10;
          ws.a[p + 1][p + 1] = d1 * is1;
          ws.ip[p] = is0;
          ws.ip[p + 1] = is1;
        }
        if (ho == 0 && j < k) {
          ws.a[j][p] = lj0;
          ws.a[j][p + 1] = lj1;
        }
        __builtin_amdgcn_wave_barrier();
      }
      if (!bad && p < k) {   // the last column of an odd k
        const double d = lane_d(ws.a[p][p], 0);
        if (!(d > 0.0)) {
          bad = true;
        } else if (lane == 0) {
          const double is = rsq64(d);
          ws.a[p][p] = d * is;
          ws.ip[p] = is;
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
    const long long pix = (long long)(sys % (unsigned)g.plane);
    const int gap = (int)(sys / (unsigned)g.plane);
    const long long base = (long long)gap * g.plane + pix;   // the column in the lower slice
    if (bad) {
      if (lane == 0) atomicAdd(&ctr->bad_pivot, 1ull);
      for (int t = 1 + lane; t <= nt; t += 64) {
        const long long o = ((long long)gap * g.f + t) * g.plane + pix;
        volume[o] = __builtin_nanf("");
        if (variance) variance[o] = __builtin_nanf("");
      }
      if (lane == 0 && flags) flags[sys] = kFlagBadPivot;
      continue;
    }
    // data values of the kept candidates (a kept candidate lies in the image)
    const double z0 = keep0 ? (double)slices[base + off0] : 0.0;
    const double z1 = keep1 ? (double)slices[base + off1] : 0.0;
    // right-hand sides of a group: r = 0 the ones, r = 1..3 targets t0..t0+2
    // (the last repeated), and with the slice predictor r = 4 the slices
    constexpr int NR = DRIFT ? 5 : 4;
    for (int t0 = 1; t0 <= nt; t0 += 3) {
      int tr[NR];
      tr[0] = 0;
#pragma unroll
      for (int r = 1; r < 4; ++r) tr[r] = min(t0 + r - 1, nt);
      if (DRIFT) tr[NR - 1] = kMaxUpsample - 1;
      // y_r in lane-row form (row i = lane < k): u_r at the dropped candidates
      double yv[NR];
      const int di = lane < k ? ws.dl[lane] : 0;
#pragma unroll
      for (int r = 0; r < NR; ++r) yv[r] = lane < k ? U[tr[r] * kMaxCand + di] : 0.0;
      // forward: L y' = u_D; four steps' pivots and factor entries read
      // ahead of their chains (indices clamped to the factor)
      for (int p0 = 0; p0 < k; p0 += 4) {
        double ipp[4], lip[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int pc = min(p0 + u, k - 1);
          ipp[u] = ws.ip[pc];
          lip[u] = ws.a[min(lane, k - 1)][pc];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int p = p0 + u;
          if (p >= k) break;
          const double l = (lane > p && lane < k) ? lip[u] : 0.0;
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const double yp = lane_d(yv[r], p) * ipp[u];
            yv[r] = lane == p ? yp : yv[r] - l * yp;
          }
        }
      }
      // backward: L^T y = y'
      for (int p0 = k - 1; p0 >= 0; p0 -= 4) {
        double ipp[4], lpi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int pc = max(p0 - u, 0);
          ipp[u] = ws.ip[pc];
          lpi[u] = ws.a[pc][min(lane, kMaxDrop - 1)];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int p = p0 - u;
          if (p < 0) break;
          const double l = lane < p ? lpi[u] : 0.0;
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const double yp = lane_d(yv[r], p) * ipp[u];
            yv[r] = lane == p ? yp : yv[r] - l * yp;
          }
        }
      }
      // x_r at the lane's candidates: u_r - sum_j G[d_j][c] y_r[j] (G symmetric)
      double x0[NR], x1[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        x0[r] = in0 ? U[tr[r] * kMaxCand + lane] : 0.0;
        x1[r] = in1 ? U[tr[r] * kMaxCand + lane + 64] : 0.0;
      }
      // the solutions to LDS, read back as broadcasts
      if (lane < kMaxDrop) {
#pragma unroll
        for (int r = 0; r < NR; ++r) ws.y[lane][r] = yv[r];
      }
      __builtin_amdgcn_wave_barrier();
      // eight rows of G in flight at a time; rows past k reread row d_{k-1}
      // and take y = 0 (rows k..31 of y hold the zeros of lanes >= k, and a
      // row index past 31 occurs only for k < 32, where row 31 is such a row)
      const int c0i = in0 ? lane : 0, c1i = in1 ? lane + 64 : 0;
      for (int jb = 0; jb < k; jb += 8) {
        double g0[8], g1[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double* grow = G + ws.dl[min(jb + u, k - 1)] * kMaxCand;
          g0[u] = grow[c0i];
          g1[u] = grow[c1i];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const double yj = ws.y[min(jb + u, kMaxDrop - 1)][r];
            x0[r] -= g0[u] * yj;
            x1[r] -= g1[u] * yj;
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
      // kept candidates only from here on
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        x0[r] = keep0 ? x0[r] : 0.0;
        x1[r] = keep1 ? x1[r] : 0.0;
      }
      // the Lagrange multipliers of each target from sums over the kept
      // candidates, then w_t'z and w_t'c0_t, each set of sums reduced together
      double r2[6], lagr[3];
      double wt0[3], wt1[3];
      if (!DRIFT) {
        // mu_t = (1'x_t - 1) / 1'x_0, w_t = x_t - mu_t x_0
        double r1[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) r1[r] = x0[r] + x1[r];
        wave_sums_k<4>(r1);
#pragma unroll
        for (int r = 1; r < 4; ++r) {
          lagr[r - 1] = (r1[r] - 1.0) / r1[0];
          wt0[r - 1] = x0[r] - lagr[r - 1] * x0[0];
          wt1[r - 1] = x1[r] - lagr[r - 1] * x1[0];
        }
      } else {
        // with the slice s as second predictor (x_s = x[4]): the 2 x 2 system
        // [[1'x_1, 1'x_s], [1'x_s, s'x_s]] (p1, ps) = (1'x_t - 1, s'x_t - t/f),
        // w_t = x_t - p1 x_1 - ps x_s, multiplier term p1 + ps t/f
        double r1[9];
        r1[0] = x0[0] + x1[0];
        r1[1] = x0[NR - 1] + x1[NR - 1];
        r1[2] = sl0 * x0[NR - 1] + sl1 * x1[NR - 1];
#pragma unroll
        for (int r = 1; r < 4; ++r) {
          r1[2 + r] = x0[r] + x1[r];
          r1[5 + r] = sl0 * x0[r] + sl1 * x1[r];
        }
        wave_sums_k<9>(r1);
        const double g11 = r1[0], g12 = r1[1], g22 = r1[2];
        const double det = g11 * g22 - g12 * g12;
#pragma unroll
        for (int r = 1; r < 4; ++r) {
          const double qt = (double)tr[r] / g.f;
          const double e1 = r1[2 + r] - 1.0, e2 = r1[5 + r] - qt;
          const double p1 = (g22 * e1 - g12 * e2) / det, ps = (g11 * e2 - g12 * e1) / det;
          lagr[r - 1] = p1 + ps * qt;
          wt0[r - 1] = x0[r] - p1 * x0[0] - ps * x0[NR - 1];
          wt1[r - 1] = x1[r] - p1 * x1[0] - ps * x1[NR - 1];
        }
      }
#pragma unroll
      for (int r = 1; r < 4; ++r) {
        const double c00 = in0 ? C0[(tr[r] - 1) * kMaxCand + lane] : 0.0;
        const double c01 = in1 ? C0[(tr[r] - 1) * kMaxCand + lane + 64] : 0.0;
        r2[r - 1] = wt0[r - 1] * z0 + wt1[r - 1] * z1;
        r2[r + 2] = wt0[r - 1] * c00 + wt1[r - 1] * c01;
      }
      wave_sums_k<6>(r2);
      if (lane == 0) {
#pragma unroll
        for (int r = 1; r < 4; ++r) {
          const int t = t0 + r - 1;
          if (t > nt) break;
          const long long o = ((long long)gap * g.f + t) * g.plane + pix;
          volume[o] = (float)r2[r - 1];
          if (variance) variance[o] = (float)(sill - r2[r + 2] - lagr[r - 1]);
        }
      }
    }
    if (lane == 0 && flags) flags[sys] = 0;
    __builtin_amdgcn_wave_barrier();
  }
}

}  // namespace

hipError_t launch_points(const Vario& v, long long nsys, const int32_t* count,
                         const int64_t* offset, const float* xyz, const float* val,
                         const float* txyz, float* est, float* var, float* weights,
                         DevCounters* c, int grid, hipStream_t s) {
  if (nsys <= 0) return hipSuccess;
  const long long g = nsys < grid ? nsys : grid;
  hipLaunchKernelGGL(points_kernel, dim3((unsigned)g), dim3(64), 0, s, v, nsys, count, offset,
                     xyz, val, txyz, est, var, weights, c);
  return hipGetLastError();
}

}  // namespace okr

namespace okr {

int pattern_downdate_floor(const Geometry& g) {
  const int nb = g.f + 1 + g.drift;
  for (int NB = 1; NB <= kMaxBlocks; ++NB) {
    const int lo = std::max(1, 16 * (NB - 1) - nb + 1);
    if (lo <= g.ncand - 1 && lo >= g.ncand - kMaxDrop) return lo;
  }
  return g.ncand;
}

hipError_t launch_pattern(const float* slices, const uint8_t* count, DevCounters* c,
                          const Geometry& g, const Vario& v, double* pat, float* volume,
                          float* variance, uint8_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(pattern_weights_kernel, dim3(1), dim3(1024), 0, s, v, g, pat, c);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (g.nslices < 2) return hipSuccess;
  const double* W = pat + kPatW;
  const double* wvar = pat + kPatVar;
  dim3 tiles((g.nx + kPTX - 1) / kPTX, (g.ny + kPTY - 1) / kPTY, g.nslices - 1);
  switch (g.r) {
#define OKR_PATTERN_R(RR)                                                                      \
  case RR:                                                                                     \
    hipLaunchKernelGGL(pattern_apply_kernel<RR>, tiles, dim3(256), 0, s, slices, count, g, W,  \
                       wvar, volume, variance, flags);                                         \
    break;
    OKR_PATTERN_R(0)
    OKR_PATTERN_R(1)
    OKR_PATTERN_R(2)
    OKR_PATTERN_R(3)
#undef OKR_PATTERN_R
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_pattern_downdate(const float* slices, const uint64_t* bits,
                                   const uint8_t* count, const uint32_t* perm, DevCounters* c,
                                   const Geometry& g, const Vario& v, const double* pat, int nlo,
                                   float* volume, float* variance, uint8_t* flags, int grid,
                                   hipStream_t s) {
  if (g.nslices < 2 || nlo >= g.ncand) return hipSuccess;
  if (nlo < 1 || g.ncand - nlo > kMaxDrop || g.f + g.drift > kMaxUpsample)
    return hipErrorInvalidValue;
  if (g.drift)
    hipLaunchKernelGGL(pattern_downdate_kernel<true>, dim3(std::max(grid, 1)),
                       dim3(64 * kDdWaves), 0, s, slices, bits, count, perm, c, g, v.sill, pat,
                       nlo, volume, variance, flags);
  else
    hipLaunchKernelGGL(pattern_downdate_kernel<false>, dim3(std::max(grid, 1)),
                       dim3(64 * kDdWaves), 0, s, slices, bits, count, perm, c, g, v.sill, pat,
                       nlo, volume, variance, flags);
  return hipGetLastError();
}

}  // namespace okr
