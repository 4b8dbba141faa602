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

__global__ __launch_bounds__(64) void pattern_weights_kernel(Vario v, Geometry g, double* W,
                                                             double* wvar, DevCounters* ctr) {
  __shared__ double A[kPtMax * kPtLd];
  const int lane = threadIdx.x;
  const int n = g.ncand;
  for (int i = lane; i < n; i += 64) {
    int dxi, dyi, si;
    cand_xyz(i, g, &dxi, &dyi, &si);
    for (int j = 0; j <= i; ++j) {
      int dxj, dyj, sj;
      cand_xyz(j, g, &dxj, &dyj, &sj);
      const double ddx = dxi - dxj, ddy = dyi - dyj, ddz = (double)(si - sj) * g.f;
      A[i * kPtLd + j] = i == j ? v.sill : cov_d(v, sqrt(ddx * ddx + ddy * ddy + ddz * ddz));
    }
  }
  __builtin_amdgcn_wave_barrier();
  if (chol_lds(A, n)) {
    if (lane == 0) atomicAdd(&ctr->bad_pivot, 1ull);
    for (int t = 0; t < g.f - 1; ++t) {
      for (int i = lane; i < n; i += 64) W[t * kMaxCand + i] = __builtin_nan("");
      if (lane == 0) wvar[t] = __builtin_nan("");
    }
    return;
  }
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
  }
  for (int t = 1; t < g.f; ++t) {
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

// One thread per full-window system of the size-sorted list (the bucket of
// n = ncand): gathers its values and applies the cached weights in FP64. The
// weights sit in LDS in a 7 x 7 layout per slice (zero outside the window), so
// every window row is one unrolled group of seven loads (slots outside the
// window reload an in-window value and take a zero weight) instead of a
// loop of dependent loads.
__global__ __launch_bounds__(256) void pattern_apply_kernel(const float* __restrict__ slices,
                                                            const uint32_t* __restrict__ perm,
                                                            const DevCounters* __restrict__ ctr,
                                                            Geometry g, const double* __restrict__ W,
                                                            const double* __restrict__ wvar,
                                                            float* __restrict__ volume,
                                                            float* __restrict__ variance,
                                                            uint8_t* __restrict__ flags) {
  constexpr int kPad = kMaxWin * kMaxWin;   // slots per slice
  __shared__ double ws[(kMaxUpsample - 1) * 2 * kPad];
  __shared__ double vs[kMaxUpsample];
  const int n = g.ncand, nt = g.f - 1, Wn = g.W;
  for (int i = threadIdx.x; i < nt * 2 * kPad; i += blockDim.x) ws[i] = 0.0;
  for (int i = threadIdx.x; i < nt; i += blockDim.x) vs[i] = wvar[i];
  __syncthreads();
  for (int i = threadIdx.x; i < nt * n; i += blockDim.x) {
    const int t = i / n, c = i - t * n;
    int dx, dy, s;
    cand_xyz(c, g, &dx, &dy, &s);
    ws[t * 2 * kPad + s * kPad + (dy + g.r) * kMaxWin + (dx + g.r)] = W[t * kMaxCand + c];
  }
  __syncthreads();
  const unsigned long long start = ctr->offsets[n];
  const unsigned long long cnt = ctr->hist[n];
  for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < cnt;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    const unsigned sys = perm[start + i];
    const unsigned gap = sys / (unsigned)g.plane;
    const unsigned pix = sys - gap * (unsigned)g.plane;
    const int y = (int)(pix / (unsigned)g.nx), x = (int)(pix - (unsigned)y * (unsigned)g.nx);
    // a kept full window lies inside the image; checked, not assumed
    if (x < g.r || y < g.r || x + g.r >= g.nx || y + g.r >= g.ny) continue;
    const float* base = slices + (long long)gap * g.plane + pix - g.r - (long long)g.r * g.nx;
    double acc[kMaxUpsample - 1];
#pragma unroll
    for (int t = 0; t < kMaxUpsample - 1; ++t) acc[t] = 0.0;
    for (int s = 0; s < 2; ++s) {
      for (int yy = 0; yy < Wn; ++yy) {
        const float* row = base + (long long)s * g.plane + (long long)yy * g.nx;
        double z[kMaxWin];
#pragma unroll
        for (int xx = 0; xx < kMaxWin; ++xx) z[xx] = (double)row[xx < Wn ? xx : Wn - 1];
        const double* wrow = ws + s * kPad + yy * kMaxWin;
#pragma unroll
        for (int t = 0; t < kMaxUpsample - 1; ++t) {
          if (t < nt) {
#pragma unroll
            for (int xx = 0; xx < kMaxWin; ++xx) acc[t] += wrow[t * 2 * kPad + xx] * z[xx];
          }
        }
      }
    }
    for (int t = 0; t < nt; ++t) {
      const long long o = ((long long)gap * g.f + t + 1) * g.plane + pix;
      volume[o] = (float)acc[t];
      if (variance) variance[o] = (float)vs[t];
    }
    if (flags) flags[sys] = 0;
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

hipError_t launch_pattern(const float* slices, const uint32_t* perm, DevCounters* c,
                          const Geometry& g, const Vario& v, double* W, double* wvar,
                          float* volume, float* variance, uint8_t* flags, int grid, hipStream_t s) {
  hipLaunchKernelGGL(pattern_weights_kernel, dim3(1), dim3(64), 0, s, v, g, W, wvar, c);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pattern_apply_kernel, dim3(grid), dim3(256), 0, s, slices, perm, c, g, W,
                     wvar, volume, variance, flags);
  return hipGetLastError();
}

}  // namespace okr
