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
    // right-looking Cholesky, C = L L^T in the lower triangle
    bool bad = false;
    for (int k = 0; k < n; ++k) {
      const double d = A[k * kPtLd + k];
      if (!(d > 0.0)) {
        bad = true;
        break;
      }
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
    // two right-hand sides: b = 1 and b = c0; forward then back substitution
    double b1[2], bc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      b1[h] = lane + 64 * h < n ? 1.0 : 0.0;
      bc[h] = c0[h];
    }
    for (int k = 0; k < n; ++k) {
      const double lkk = A[k * kPtLd + k];
      const int hk = k >> 6, lk = k & 63;
      const double y1 = (hk ? lane_d(b1[1], lk) : lane_d(b1[0], lk)) / lkk;
      const double yc = (hk ? lane_d(bc[1], lk) : lane_d(bc[0], lk)) / lkk;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        if (i == k) {
          b1[h] = y1;
          bc[h] = yc;
        } else if (i > k && i < n) {
          const double lik = A[i * kPtLd + k];
          b1[h] -= lik * y1;
          bc[h] -= lik * yc;
        }
      }
    }
    for (int k = n - 1; k >= 0; --k) {
      const double lkk = A[k * kPtLd + k];
      const int hk = k >> 6, lk = k & 63;
      const double x1 = (hk ? lane_d(b1[1], lk) : lane_d(b1[0], lk)) / lkk;
      const double xc = (hk ? lane_d(bc[1], lk) : lane_d(bc[0], lk)) / lkk;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        if (i == k) {
          b1[h] = x1;
          bc[h] = xc;
        } else if (i < k) {
          const double lki = A[k * kPtLd + i];
          b1[h] -= lki * x1;
          bc[h] -= lki * xc;
        }
      }
    }
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
