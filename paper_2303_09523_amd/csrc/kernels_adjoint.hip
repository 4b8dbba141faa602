// Leave-one-slice-out loss of a variogram and its adjoint gradient.
//
// Every known slice s in 1..n-2 is predicted from slices s-1 and s+1 (the
// geometry of a gap of two with the target half-way) with the same edge rule
// and floor as the volume path; the loss is the mean of (z_hat - z)^2 over
// all held-out voxels. Forward: one refined solve per (column, held-out
// slice) system (FP32 factorisation, FP64-corrected estimate), residual
// stored per system. Backward: the same solve recomputed (no factor is
// stored), then with e = 2 (z_hat - z) / N, the weights w and the adjoint
// vector nu = K^{-1} [e z; 0] of the extended system K = [[C, Q], [Q', 0]]
// (Q = 1, or [1 s] with the slice predictor; Q does not depend on the
// variogram, so its derivative drops out),
//   dL/dtheta = nu_w' dc0/dtheta - nu_w' (dC/dtheta) w
// with dC/dtheta and dc0/dtheta from the FP64 derivative tables (FP64
// products). Per-system values are summed in a fixed order, so the loss and
// the gradient are bitwise reproducible.
#include "solver_refine.h"

namespace okr {
namespace {

struct AdjSmem {
  double dtc[3][kTcSize];
  double dt0[3][kT0Stride];
  double w[4][128];
};

template <int NB, bool BACKWARD>
__global__ __launch_bounds__(256) void loso_class_kernel(SolveArgs a) {
  __shared__ Smem<float> sm;
  __shared__ LosoSmem msm;
  __shared__ AdjSmem as;
  __shared__ WaveScratch<float> wsa[4];
  __shared__ MixedScratch msa[4];
  __shared__ f32x4 xsa[4 * area_vec4<NB>()];   // each wave's area (see area_vec4)
  const double tscale = 1.0 / a.sill;
  block_setup<float>(a, sm, tscale);
  mixed_setup(a, sm, msm, tscale);
  if (BACKWARD) {
    for (int i = threadIdx.x; i < 3 * kTcSize; i += blockDim.x)
      as.dtc[i / kTcSize][i % kTcSize] = a.tab.dtc_d[i];
    for (int i = threadIdx.x; i < 3 * kT0Stride; i += blockDim.x)
      as.dt0[i / kT0Stride][i % kT0Stride] = a.tab.dt0_d[(i / kT0Stride) * kT0Size + i % kT0Stride];
  }
  __syncthreads();
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  WaveScratch<float>& ws = wsa[wid];
  MixedScratch& mx = msa[wid];
  double* wv = as.w[wid];
  const int nb = a.nb;
  int nlo = 16 * (NB - 1) - nb + 1, nhi = 16 * NB - nb;
  if (nlo < 1) nlo = 1;
  if (nhi > kHist - 1) nhi = kHist - 1;
  if (nhi > a.nmax) nhi = a.nmax;
  if (nlo > nhi) return;
  const unsigned long long start = a.ctr->offsets[nhi];
  const unsigned long long end = a.ctr->offsets[nlo] + a.ctr->hist[nlo];
  ClassRange cr = class_range(a, NB, start, end, false);
  const int ncand = a.geo.ncand;
  const unsigned plane = (unsigned)a.geo.plane;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int d0 = sm.sdesc[lane];
  const int d1 = lane + 64 < ncand ? sm.sdesc[lane + 64] : 0;
  for (;;) {
    unsigned long long base = 0;
    int nk = 0;
    if (!next_chunk(cr, base, nk)) break;
    Pipe q;
    pipe_load(q, a, a.perm, base, nk);
    pipe_prefetch(q, a, 0, d0, d1, below);
    for (int k = 0; k < nk; ++k) {
      const unsigned sys = __builtin_amdgcn_readlane(q.msys, k);
      const unsigned long long lo = lane_u64(q.mlo, k), hi = lane_u64(q.mhi, k);
      const int n = __popcll(lo) + __popcll(hi);
      pipe_commit<float>(q, ws, d0, d1, n);
      if (k + 1 < nk) pipe_prefetch(q, a, k + 1, d0, d1, below);
      double est = 0.0, zscale = 1.0;
      float var = 0.0f, mn, mxp;
      bool bad;
      mixed_system<NB, 0, true, LosoSmem>(n, nb, ws, sm, mx, xsa + area_vec4<NB>() * wid, msm, ncand, 1, a.sill, 0.0, &est, &var, mn, mxp, bad,
                          BACKWARD ? wv : nullptr, &zscale);
      est = __shfl(est, 0, 64);
      const unsigned gap = sys / plane;
      const unsigned pix = sys - gap * plane;
      if (!BACKWARD) {
        if (lane == 0) {
          const double truth = (double)a.slices[(long long)(gap + 1) * a.geo.plane + pix];
          a.resid[sys] = est - truth;
        }
        if (lane == 0 && bad) atomicAdd(&a.ctr->bad_pivot, 1ull);
      } else {
        __builtin_amdgcn_wave_barrier();
        // nu_w of the unscaled system for the data e*z: the refined solve
        // returned nu'_w for (z - z_ref)/s and C/sill.
        const double e = 2.0 * a.resid[sys] * a.inv_count;
        const double fac = e * zscale / a.sill;
        const int p0 = lane, p1 = lane + 64;
        const int e0 = p0 < n ? ws.desc[p0] : 0, e1 = p1 < n ? ws.desc[p1] : 0;
        const double nu0 = p0 < n ? fac * area_nuc(xsa + area_vec4<NB>() * wid)[e0 & 0x7f] : 0.0;
        const double nu1 = p1 < n ? fac * area_nuc(xsa + area_vec4<NB>() * wid)[e1 & 0x7f] : 0.0;
        const uint8_t* row0 = msm.row(e0 & 0x7f);
        const uint8_t* row1 = msm.row(e1 & 0x7f);
        double dcw0[3] = {0, 0, 0}, dcw1[3] = {0, 0, 0};
        for (int qq = 0; qq < n; ++qq) {
          const int cq = ws.desc[qq] & 0x7f;
          const double wq = wv[qq];
          const int c0 = row0[cq], c1 = row1[cq];
#pragma unroll
          for (int kk = 0; kk < 3; ++kk) {
            dcw0[kk] += as.dtc[kk][c0] * wq;
            dcw1[kk] += as.dtc[kk][c1] * wq;
          }
        }
        double gk[3];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          const double t0 = p0 < n ? as.dt0[kk][e0 >> 16] : 0.0;
          const double t1 = p1 < n ? as.dt0[kk][e1 >> 16] : 0.0;
          gk[kk] = nu0 * (t0 - dcw0[kk]) + nu1 * (t1 - dcw1[kk]);
        }
        wave_sums(gk);
        if (lane < 3) a.gpart[3ull * sys + lane] = lane == 0 ? gk[0] : (lane == 1 ? gk[1] : gk[2]);
      }
    }
  }
}

template <bool BACKWARD>
hipError_t launch_loso_classes(const SolveArgs& a, int grid, hipStream_t s) {
  const int nbmax = (a.geo.ncand + a.nb + 15) / 16;
#define OKR_CLS(K)                                                                            \
  if (nbmax >= K) {                                                                           \
    hipLaunchKernelGGL((loso_class_kernel<K, BACKWARD>), dim3(grid), dim3(256), 0, s, a);     \
    hipError_t e = hipGetLastError();                                                         \
    if (e != hipSuccess) return e;                                                            \
  }
  OKR_CLS(8) OKR_CLS(7) OKR_CLS(6) OKR_CLS(5) OKR_CLS(4) OKR_CLS(3) OKR_CLS(2) OKR_CLS(1)
#undef OKR_CLS
  return hipSuccess;
}

constexpr int kRedBlocks = 256;

// Pass 1: block b sums a contiguous range in index order (tree within the
// block in a fixed shape); pass 2: one block sums the partials the same way.
__global__ __launch_bounds__(256) void reduce_pass1(const double* __restrict__ x, long long n,
                                                    int ncomp, bool square,
                                                    double* __restrict__ partial) {
  __shared__ double red[256];
  const long long per = (n + kRedBlocks - 1) / kRedBlocks;
  const long long lo = blockIdx.x * per;
  const long long hi = lo + per < n ? lo + per : n;
  for (int c = 0; c < ncomp; ++c) {
    double acc = 0.0;
    for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x) {
      const double v = x[i * ncomp + c];
      acc += square ? v * v : v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int sft = 128; sft > 0; sft >>= 1) {
      if ((int)threadIdx.x < sft) red[threadIdx.x] += red[threadIdx.x + sft];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x * ncomp + c] = red[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void reduce_pass2(const double* __restrict__ partial, int ncomp,
                                                    double scale, double* __restrict__ out) {
  __shared__ double red[256];
  for (int c = 0; c < ncomp; ++c) {
    red[threadIdx.x] = partial[threadIdx.x * ncomp + c];
    __syncthreads();
    for (int sft = 128; sft > 0; sft >>= 1) {
      if ((int)threadIdx.x < sft) red[threadIdx.x] += red[threadIdx.x + sft];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0] * scale;
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_loso_forward(const SolveArgs& a, int grid, hipStream_t s) {
  return launch_loso_classes<false>(a, grid, s);
}

hipError_t launch_loso_backward(const SolveArgs& a, int grid, hipStream_t s) {
  return launch_loso_classes<true>(a, grid, s);
}

hipError_t launch_reduce(const double* x, long long n, int ncomp, double scale, double* partial,
                         double* out, bool square, hipStream_t s) {
  hipLaunchKernelGGL(reduce_pass1, dim3(kRedBlocks), dim3(256), 0, s, x, n, ncomp, square, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_pass2, dim3(1), dim3(256), 0, s, partial, ncomp, scale, out);
  return hipGetLastError();
}

}  // namespace okr
