// Plain per-voxel kriging: the straightforward GPU form of the method, one
// wavefront per missing voxel, used as the comparison kernel.
//
// For every kriged voxel the wave selects its neighbours (same edge rule and
// floor as the batched path, evaluated here directly from the edge mask),
// builds the covariance matrix C of its n points and their covariances c0 with
// the target from the FP64 covariance tables (indexed by point offset),
// factors C = L L^T by Cholesky in LDS (packed lower triangle, FP32), solves
// x1 = C^{-1} 1 and xc = C^{-1} c0, and forms the solution of the bordered
// system of Appendix A, [[C, 1], [1^T, 0]] [w; mu] = [c0; 1]:
//   mu = (1'xc - 1) / 1'x1,  w = xc - mu x1.
// With refinement (refine_max = 1) one step of iterative refinement follows:
// the FP64 residual [r_w; r_mu] = [c0 - C w - mu 1; 1 - 1'w] of the bordered
// system, its correction from the same factor (t = C^{-1} r_w,
// d_mu = (1't - r_mu) / 1'x1, d_w = t - d_mu x1), added in FP64. Then
// z_hat = sum w_i z_i and sigma^2 = sill - w'c0 - mu in FP64. Nothing is shared
// between voxels: the f-1 targets of a column each factor the same matrix.
#include "solver_core.h"

namespace okr {
namespace {

constexpr int kPN = kMaxCand;
constexpr int kPack = kPN * (kPN + 1) / 2;

struct PlainLds {
  float L[kPack];        // packed lower triangle, row i from i(i+1)/2
  int desc[kPN];         // kept points' candidate descriptors (cand_desc)
  float z[kPN];          // their values
  double c0[kPN];        // their covariances with the target
  float y1[kPN], yc[kPN];  // forward-substitution results
  double w[kPN];         // weights (FP64 after refinement)
};

__device__ __forceinline__ int prow(int i) { return (i * (i + 1)) >> 1; }

__device__ __forceinline__ float plain_sum(float x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ double plain_sum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Forward substitution L y = b for two right-hand sides (row by row; the
// partial sums of each row over its columns are spread over the lanes).
__device__ __forceinline__ void forward2(const PlainLds& ps, int n, const float* b1, const float* b2,
                                         float* y1, float* y2) {
  const int lane = threadIdx.x & 63;
  for (int i = 0; i < n; ++i) {
    const int ri = prow(i);
    float s1 = 0.0f, s2 = 0.0f;
    for (int j = lane; j < i; j += 64) {
      const float l = ps.L[ri + j];
      s1 += l * y1[j];
      s2 += l * y2[j];
    }
    s1 = plain_sum(s1);
    s2 = plain_sum(s2);
    const float d = ps.L[ri + i];
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
      y1[i] = (b1[i] - s1) / d;
      y2[i] = (b2[i] - s2) / d;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Back substitution L^T x = y in place (column by column: x_j is final once
// the rows below it have been subtracted; lane i holds entries i, i + 64).
__device__ __forceinline__ void backward(const PlainLds& ps, int n, float* y) {
  const int lane = threadIdx.x & 63;
  float v0 = lane < n ? y[lane] : 0.0f;
  float v1 = lane + 64 < n ? y[lane + 64] : 0.0f;
  for (int j = n - 1; j >= 0; --j) {
    const int rj = prow(j);
    const float yj = __shfl(j < 64 ? v0 : v1, j & 63, 64);
    const float xj = yj / ps.L[rj + j];
    if (lane < j) v0 -= ps.L[rj + lane] * xj;
    if (lane + 64 < j) v1 -= ps.L[rj + lane + 64] * xj;
    if (lane == (j & 63)) {
      if (j < 64) v0 = xj;
      else v1 = xj;
    }
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < n) y[lane] = v0;
  if (lane + 64 < n) y[lane + 64] = v1;
  __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(64) void plain_kernel(const float* __restrict__ slices,
                                                   const uint8_t* __restrict__ edge,
                                                   float* __restrict__ volume,
                                                   float* __restrict__ variance, Geometry geo,
                                                   SelectRule rule, double sill, TableSet tab,
                                                   int refine, long long nvox) {
  __shared__ PlainLds ps;
  const int lane = threadIdx.x;
  const int nc = geo.ncand;
  const int r = geo.r, W = geo.W, W2 = geo.W2, f = geo.f;
  const int centre = r * W + r;
  const long long per_gap = (long long)(f - 1) * geo.plane;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (long long vox = blockIdx.x; vox < nvox; vox += gridDim.x) {
    const long long gap = vox / per_gap;
    long long rem = vox - gap * per_gap;
    const int t = 1 + (int)(rem / geo.plane);
    rem -= (long long)(t - 1) * geo.plane;
    const int y = (int)(rem / geo.nx), x = (int)(rem - (long long)y * geo.nx);
    // --- neighbour selection ---
    bool keep[2], inimg[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = lane + 64 * h;
      keep[h] = inimg[h] = false;
      if (c < nc) {
        const int s = c >= W2;
        const int o = c - s * W2;
        const int a = o / W, b = o - a * W;
        const int yy = y + a - r, xx = x + b - r;
        inimg[h] = yy >= 0 && yy < geo.ny && xx >= 0 && xx < geo.nx;
        bool k = inimg[h];
        if (k && o != centre && edge) {
          uint64_t p = rule.path[o];
          const uint8_t* e = edge + (gap + s) * geo.plane;
          while (p) {
            const int cell = __ffsll((long long)p) - 1;
            p &= p - 1;
            const int pa = cell / W, pb = cell - pa * W;
            if (e[(long long)(y + pa - r) * geo.nx + (x + pb - r)]) {
              k = false;
              break;
            }
          }
        }
        keep[h] = k;
      }
    }
    uint64_t klo = __ballot(keep[0]), khi = __ballot(keep[1]);
    int n = __popcll(klo) + __popcll(khi);
    if (n < geo.min_points) {
      const uint64_t ilo = __ballot(inimg[0]), ihi = __ballot(inimg[1]);
      for (int i = 0; i < nc && n < geo.min_points; ++i) {
        const int c = rule.floor_order[i];
        const uint64_t bit = 1ull << (c & 63);
        if (c < 64) {
          if ((ilo & bit) && !(klo & bit)) {
            klo |= bit;
            ++n;
          }
        } else if ((ihi & bit) && !(khi & bit)) {
          khi |= bit;
          ++n;
        }
      }
    }
    const int n0 = __popcll(klo);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = lane + 64 * h;
      const uint64_t word = h ? khi : klo;
      if (c < nc && ((word >> lane) & 1ull)) {
        const int pos = (h ? n0 : 0) + __popcll(word & below);
        const int d = cand_desc(c, r, W, W2);
        const int cc = (d >> 8) & 0xff;
        const int s = (cc >> 6) & 1, a = (cc >> 3) & 7, b = cc & 7;
        ps.desc[pos] = d;
        ps.z[pos] = slices[(gap + s) * geo.plane + (long long)(y + a - r) * geo.nx + (x + b - r)];
        ps.c0[pos] = tab.t0_d[(t - 1) * kT0Stride + (d >> 16)];
      }
    }
    __builtin_amdgcn_wave_barrier();
    // --- covariance matrix (packed lower triangle, FP32 from the FP64 table) ---
    for (int i = 0; i < n; ++i) {
      const int di = ps.desc[i];
      for (int j = lane; j <= i; j += 64) ps.L[prow(i) + j] = (float)tab.tc_d[pair_class(di, ps.desc[j])];
    }
    __builtin_amdgcn_wave_barrier();
    // --- Cholesky, right-looking; lane owns trailing columns k+1+lane, k+65+lane ---
    for (int k = 0; k < n; ++k) {
      const float d = ps.L[prow(k) + k];
      const float piv = sqrtf(d > 0.0f ? d : 1.0f);
      const float inv = 1.0f / piv;
      __builtin_amdgcn_wave_barrier();
      for (int i = k + 1 + lane; i < n; i += 64) ps.L[prow(i) + k] *= inv;
      if (lane == 0) ps.L[prow(k) + k] = piv;
      __builtin_amdgcn_wave_barrier();
      const int j0 = k + 1 + lane, j1 = j0 + 64;
      const float l0 = j0 < n ? ps.L[prow(j0) + k] : 0.0f;
      const float l1 = j1 < n ? ps.L[prow(j1) + k] : 0.0f;
      for (int i = k + 1; i < n; ++i) {
        const int ri = prow(i);
        const float lik = ps.L[ri + k];
        if (j0 <= i) ps.L[ri + j0] -= lik * l0;
        if (j1 <= i) ps.L[ri + j1] -= lik * l1;
      }
      __builtin_amdgcn_wave_barrier();
    }
    // --- x1 = C^{-1} 1, xc = C^{-1} c0 ---
    for (int i = lane; i < n; i += 64) {   // right-hand sides, solved in place
      ps.y1[i] = 1.0f;
      ps.yc[i] = (float)ps.c0[i];
    }
    __builtin_amdgcn_wave_barrier();
    forward2(ps, n, ps.y1, ps.yc, ps.y1, ps.yc);
    backward(ps, n, ps.y1);
    backward(ps, n, ps.yc);
    // --- bordered solution ---
    float s1 = 0.0f, sc = 0.0f;
    for (int i = lane; i < n; i += 64) {
      s1 += ps.y1[i];
      sc += ps.yc[i];
    }
    s1 = plain_sum(s1);
    sc = plain_sum(sc);
    double mu = ((double)sc - 1.0) / (double)s1;
    for (int i = lane; i < n; i += 64) ps.w[i] = (double)ps.yc[i] - mu * (double)ps.y1[i];
    __builtin_amdgcn_wave_barrier();
    if (refine) {
      // FP64 residual of the bordered system
      double rm = 0.0;
      for (int i = lane; i < n; i += 64) rm += ps.w[i];
      rm = 1.0 - plain_sum(rm);
      float rv[2] = {0.0f, 0.0f};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int p = lane + 64 * h;
        if (p < n) {
          const int dp = ps.desc[p];
          double acc = 0.0;
          for (int q = 0; q < n; ++q) acc += tab.tc_d[pair_class(dp, ps.desc[q])] * ps.w[q];
          rv[h] = (float)(ps.c0[p] - acc - mu);
        }
      }
      __builtin_amdgcn_wave_barrier();
      if (lane < n) ps.yc[lane] = rv[0];
      if (lane + 64 < n) ps.yc[lane + 64] = rv[1];
      __builtin_amdgcn_wave_barrier();
      // t = C^{-1} r_w (forward on the residual alone; y1 holds x1 and stays)
      for (int i = 0; i < n; ++i) {
        const int ri = prow(i);
        float s = 0.0f;
        for (int j = lane; j < i; j += 64) s += ps.L[ri + j] * ps.yc[j];
        s = plain_sum(s);
        const float d = ps.L[ri + i];
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) ps.yc[i] = (ps.yc[i] - s) / d;
        __builtin_amdgcn_wave_barrier();
      }
      backward(ps, n, ps.yc);
      float st = 0.0f;
      for (int i = lane; i < n; i += 64) st += ps.yc[i];
      st = plain_sum(st);
      const double dmu = ((double)st - rm) / (double)s1;
      for (int i = lane; i < n; i += 64) ps.w[i] += (double)ps.yc[i] - dmu * (double)ps.y1[i];
      mu += dmu;
      __builtin_amdgcn_wave_barrier();
    }
    double ez = 0.0, wc = 0.0;
    for (int i = lane; i < n; i += 64) {
      ez += ps.w[i] * (double)ps.z[i];
      wc += ps.w[i] * ps.c0[i];
    }
    ez = plain_sum(ez);
    wc = plain_sum(wc);
    if (lane == 0) {
      const long long o = (gap * f + t) * geo.plane + (long long)y * geo.nx + x;
      volume[o] = (float)ez;
      if (variance) variance[o] = (float)(sill - wc - mu);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

}  // namespace

hipError_t launch_plain(const float* slices, const uint8_t* edge, float* volume, float* variance,
                        const Geometry& g, const SelectRule& rule, const Vario& v, TableSet tab,
                        int refine, int num_cu, hipStream_t s) {
  const long long nvox = (long long)(g.nslices - 1) * (g.f - 1) * g.plane;
  if (nvox <= 0) return hipSuccess;
  const long long cap = (long long)num_cu * 8;
  const long long grid = nvox < cap ? nvox : cap;
  hipLaunchKernelGGL(plain_kernel, dim3((unsigned)grid), dim3(64), 0, s, slices, edge, volume,
                     variance, g, rule, v.sill, tab, refine, nvox);
  return hipGetLastError();
}

}  // namespace okr
