// Plain per-voxel kriging: the straightforward GPU form of the method, one
// wavefront per missing voxel, used as the comparison kernel.
//
// For every kriged voxel the wave selects its neighbours (same edge rule and
// floor as the batched path, evaluated here directly from the edge mask),
// evaluates the covariance of every pair directly from the variogram, builds
// the bordered ordinary-kriging system of Appendix A,
//   [[C, 1], [1^T, 0]] [w; mu] = [c0; 1],
// and solves it by Gaussian elimination with partial pivoting in LDS, then
// forms z_hat = w^T z and sigma^2 = sill - w^T c0 - mu. Nothing is shared
// between voxels: the factorisation is repeated for each of the f-1 targets
// of a column.
#include "okrig_internal.h"

namespace okr {
namespace {

__device__ __forceinline__ float cov_f(const Vario& v, float h) {
  if (h == 0.0f) return (float)v.sill;
  const float a = (float)v.range;
  float rho;
  if (v.model == 0) {
    const float q = h / a;
    rho = q < 1.0f ? 1.0f - 1.5f * q + 0.5f * q * q * q : 0.0f;
  } else if (v.model == 1) {
    rho = expf(-3.0f * h / a);
  } else {
    const float q = h / a;
    rho = expf(-3.0f * q * q);
  }
  return (float)(v.sill - v.nugget) * rho;
}

__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__global__ __launch_bounds__(64) void plain_kernel(const float* __restrict__ slices,
                                                   const uint8_t* __restrict__ edge,
                                                   float* __restrict__ volume,
                                                   float* __restrict__ variance, Geometry geo,
                                                   SelectRule rule, Vario vg, long long nvox) {
  extern __shared__ float sm[];
  const int lane = threadIdx.x;
  const int nc = geo.ncand;
  const int ld = nc + 3;                 // row stride: up to nc+1 unknowns + rhs
  float* A = sm;                         // [(nc+1)][ld]
  float* pxs = A + (nc + 1) * ld;        // point coordinates and values
  float* pys = pxs + nc;
  float* pzs = pys + nc;
  float* pvs = pzs + nc;
  float* c0s = pvs + nc;
  const int r = geo.r, W = geo.W, W2 = geo.W2, f = geo.f;
  const int centre = r * W + r;
  const long long per_gap = (long long)(f - 1) * geo.plane;
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
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = lane + 64 * h;
      const uint64_t word = h ? khi : klo;
      if (c < nc && ((word >> lane) & 1ull)) {
        const int pos = (h ? n0 : 0) + __popcll(word & below);
        const int s = c >= W2;
        const int o = c - s * W2;
        const int a = o / W, b = o - a * W;
        pxs[pos] = (float)(b - r);
        pys[pos] = (float)(a - r);
        pzs[pos] = s ? (float)f : 0.0f;
        pvs[pos] = slices[(gap + s) * geo.plane + (long long)(y + a - r) * geo.nx + (x + b - r)];
      }
    }
    __syncthreads();
    // --- bordered system with direct covariance evaluation ---
    const int N = n + 1;
    for (int idx = lane; idx < N * N; idx += 64) {
      const int i = idx / N, j = idx - i * N;
      float val;
      if (i < n && j < n) {
        const float dx = pxs[i] - pxs[j], dy = pys[i] - pys[j], dz = pzs[i] - pzs[j];
        val = cov_f(vg, sqrtf(dx * dx + dy * dy + dz * dz));
      } else {
        val = (i == n && j == n) ? 0.0f : 1.0f;
      }
      A[i * ld + j] = val;
    }
    for (int i = lane; i < N; i += 64) {
      float val = 1.0f;
      if (i < n) {
        const float dz = pzs[i] - (float)t;
        val = cov_f(vg, sqrtf(pxs[i] * pxs[i] + pys[i] * pys[i] + dz * dz));
      }
      A[i * ld + N] = val;
      c0s[i] = val;
    }
    __syncthreads();
    // --- Gaussian elimination with partial pivoting ---
    for (int k = 0; k < N; ++k) {
      float best = -1.0f;
      int bi = k;
      for (int i = k + lane; i < N; i += 64) {
        const float a = fabsf(A[i * ld + k]);
        if (a > best) {
          best = a;
          bi = i;
        }
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const float ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (bi != k) {
        for (int j = k + lane; j <= N; j += 64) {
          const float tmp = A[k * ld + j];
          A[k * ld + j] = A[bi * ld + j];
          A[bi * ld + j] = tmp;
        }
      }
      __syncthreads();
      const float inv = 1.0f / A[k * ld + k];
      for (int i = k + 1 + lane; i < N; i += 64) A[i * ld + k] *= inv;
      __syncthreads();
      for (int j = k + 1 + lane; j <= N; j += 64) {
        const float akj = A[k * ld + j];
        for (int i = k + 1; i < N; ++i) A[i * ld + j] -= A[i * ld + k] * akj;
      }
      __syncthreads();
    }
    // --- back substitution (column oriented) ---
    for (int i = N - 1; i >= 0; --i) {
      const float xi = A[i * ld + N] / A[i * ld + i];
      __syncthreads();
      if (lane == 0) A[i * ld + N] = xi;
      for (int q = lane; q < i; q += 64) A[q * ld + N] -= A[q * ld + i] * xi;
      __syncthreads();
    }
    float ez = 0.0f, wc = 0.0f;
    for (int i = lane; i < n; i += 64) {
      const float w = A[i * ld + N];
      ez += w * pvs[i];
      wc += w * c0s[i];
    }
    ez = wave_sum(ez);
    wc = wave_sum(wc);
    if (lane == 0) {
      const float mu = A[n * ld + N];
      const long long o = (gap * f + t) * geo.plane + (long long)y * geo.nx + x;
      volume[o] = ez;
      if (variance) variance[o] = (float)vg.sill - wc - mu;
    }
    __syncthreads();
  }
}

}  // namespace

size_t plain_shared_bytes(const Geometry& g) {
  const int nc = g.ncand;
  const int ld = nc + 3;
  return sizeof(float) * ((size_t)(nc + 1) * ld + 5 * nc + 1);
}

hipError_t launch_plain(const float* slices, const uint8_t* edge, float* volume, float* variance,
                        const Geometry& g, const SelectRule& rule, const Vario& v, hipStream_t s) {
  const long long nvox = (long long)(g.nslices - 1) * (g.f - 1) * g.plane;
  if (nvox <= 0) return hipSuccess;
  long long grid = nvox < 256LL * 16 ? nvox : 256LL * 16;
  hipLaunchKernelGGL(plain_kernel, dim3((unsigned)grid), dim3(64), plain_shared_bytes(g), s, slices,
                     edge, volume, variance, g, rule, v, nvox);
  return hipGetLastError();
}

}  // namespace okr
