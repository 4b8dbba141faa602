// Mixed-precision batched kriging with an FP64 residual correction.
//
// Per system (one wavefront):
//   1. The data values are shifted by a reference value z_ref (the first kept
//      point) and divided by a power of two s that bounds their spread, and the
//      covariances are divided by the sill. Ordinary kriging is affine in the
//      data and invariant to a common scale of C and c0, so
//      z_hat = z_ref + s * z_hat' and sigma^2 = sill * sigma'^2, while every
//      low-precision operand stays O(1).
//   2. Left-looking factorisation of [[C, B], [B^T, 0]] with FP32 diagonal
//      tiles and split FP16 (or BF16) MFMA trailing updates (hi*hi + hi*lo +
//      lo*hi, FP32 accumulation); the off-diagonal solves are FP32, or split
//      FP16 products as well in the FP16 read-out.
//   3. Back-substitution gives x_1 = C^{-1} 1, x_z = C^{-1} z, x_t = C^{-1} c0_t,
//      hence the weights w_t = x_t - mu_t x_1 (mu_t = (1'x_t - 1) / 1'x_1) and
//      the adjoint vector nu_w = x_z - (1'x_z / 1'x_1) x_1 with
//      nu_mu = 1'x_z / 1'x_1 of the bordered system K = [[C, 1], [1', 0]].
//   4. FP64 correction with the residual r_t - K lambda_t of the FP64 system:
//        z_hat_t = z' w_t + nu' r_t - (K nu)' lambda_t
//      which is exact up to the product of the errors of nu and lambda_t, so
//      the estimate reaches FP64-level accuracy from a low-precision factor.
//      The one FP64 matrix-vector product C nu_w per system uses a per-block
//      FP64 table of every candidate pair's covariance.
// Steps 3-4 run when the correction is enabled (a launch-time choice) and the
// system's pivot-ratio condition estimate exceeds a threshold; otherwise the
// estimate is the Schur read-out of step 2 in the normalised units.
// The kriging variance comes from the factorisation's Schur block (FP32).
// Systems with a non-positive pivot are queued for the FP64 re-solve.
#include "solver_refine.h"

namespace okr {
namespace {

// Without the correction the kernel holds only the factorisation's live tiles;
// it runs eight waves per workgroup, which share one copy of the block tables,
// so that two workgroups fit a CU's LDS and each SIMD holds four waves (128
// VGPRs; the few values spilled at NB >= 7 cost less than the latency the
// fourth wave hides). The corrected form keeps every L tile and runs one wave
// per SIMD in workgroups of four.
template <bool CORR> constexpr int mixed_waves() { return CORR ? 4 : 8; }

template <int NB, int UPD, bool CORR>
__global__ __launch_bounds__(64 * mixed_waves<CORR>())
__attribute__((amdgpu_waves_per_eu(CORR ? 2 : 4)))
void mixed_class_kernel(SolveArgs a) {
  constexpr int W = mixed_waves<CORR>();
  __shared__ Smem<float> sm;
  __shared__ MixedSmem msm;
  __shared__ WaveScratch<float> wsa[W];
  __shared__ ChunkStage csa[W];
  __shared__ MixedScratch msa[W];
  __shared__ f32x4 xsa[CORR ? W * area_vec4<NB>() : 1];   // each wave's area (see area_vec4)
  const double tscale = 1.0 / a.sill;
  block_setup<float>(a, sm, tscale);
  mixed_setup(a, sm, msm, tscale);
  __syncthreads();
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  WaveScratch<float>& ws = wsa[wid];
  ChunkStage& cst = csa[wid];
  MixedScratch& mx = msa[wid];
  const int nb = a.nb;
  int nlo = 16 * (NB - 1) - nb + 1, nhi = 16 * NB - nb;
  if (nlo < 1) nlo = 1;
  if (nhi > kHist - 1) nhi = kHist - 1;
  if (nhi > a.nmax) nhi = a.nmax;
  if (nlo > nhi) return;
  const unsigned long long start = a.ctr->offsets[nhi];
  const unsigned long long end = a.ctr->offsets[nlo] + a.ctr->hist[nlo];
  ClassRange cr = class_range(a, NB, start, end, true);
  const int ntgt = a.geo.f - 1, ncand = a.geo.ncand;
  const double zfloor = 0.01 * (double)__uint_as_float(a.ctr->zmax_bits);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int d0 = sm.sdesc[lane];
  const int d1 = lane + 64 < ncand ? sm.sdesc[lane + 64] : 0;
  Tally tally;
  unsigned long long refined = 0;
  for (;;) {
    unsigned long long base = 0;
    int nk = 0;
    if (!next_chunk(cr, base, nk)) break;
    Pipe q;
    pipe_load(q, a, a.perm, base, nk);
    unsigned sg = 0, sy = 0, sx = 0;
    const bool staged = stage_chunk(q, a, nk, cst, sg, sy, sx);
    if (staged)
      pipe_prefetch_staged(q, cst, 0, d0, d1, below, ncand);
    else
      pipe_prefetch(q, a, 0, d0, d1, below);
    for (int k = 0; k < nk; ++k) {
      const unsigned sys = __builtin_amdgcn_readlane(q.msys, k);
      const unsigned long long lo = lane_u64(q.mlo, k), hi = lane_u64(q.mhi, k);
      const int cnt = __builtin_amdgcn_readlane(q.mcnt, k);
      const int n = __popcll(lo) + __popcll(hi);
      pipe_commit<float>(q, ws, d0, d1, n);
      if (k + 1 < nk) {
        if (staged)
          pipe_prefetch_staged(q, cst, k + 1, d0, d1, below, ncand);
        else
          pipe_prefetch(q, a, k + 1, d0, d1, below);
      }
      // nb is fixed for the launch; hidden from loop-invariant code motion so that
      // the tests on it inside the factorisation stay scalar compares per system
      // instead of lane masks held (and spilled) across the whole loop
      int nbs = nb;
      asm volatile("" : "+s"(nbs));
      double est = 0.0;
      float var = 0.0f, mn, mxp;
      bool bad;
      double scale = 1.0, readout = 0.0, bound = 0.0;
      const bool check = CORR && a.refine_tol > 0.0;
      const bool corr = mixed_system<NB, UPD, CORR>(n, nbs, ws, sm, mx, xsa + area_vec4<NB>() * wid, msm, ncand, ntgt, a.sill,
                                                    a.refine_kappa, &est, &var, mn, mxp, bad,
                                                    nullptr, &scale, &readout,
                                                    check ? &bound : nullptr);
      bool route = false;
      uint8_t extra = 0;
      if (!CORR && a.route_tol > 0.0) {
        // error indicator of the read-out per target: kappa_w u s / max(|z_hat|, 0.01 Zmax)
        // (kappa_w bounds the system's condition number, u is the factorisation's
        // unit roundoff, s the power of two bounding the data spread)
        const double den = fmax(fabs(est), zfloor);
        const double ind = (lane < ntgt && den > 0.0) ? a.route_scale * scale / den : 0.0;
        route = __any(ind > a.route_tol);
      }
      if (check && corr) {
        // convergence: the error the correction leaves is at most the weights'
        // relative error (rho_hat, from kappa_w and the factorisation's unit
        // roundoff) times the bound mixed_system reports; the move of the
        // estimate from the read-out, scaled the same way, is included as well
        const double den = fmax(fabs(est), zfloor);
        const double c = (lane < ntgt && den > 0.0)
                             ? a.rho_hat * fmax(bound, fabs(est - readout)) / den : 0.0;
        if (__any(c > a.refine_tol)) {
          route = true;
          extra = kFlagUnconverged;
          tally.unconv += 1;
        }
      }
      finish_system<float>(a, 0, sys, cnt, (float)est, var, mn, mxp, bad, tally, route, extra,
                           staged ? &cst : nullptr, k);
      if (lane == 0 && a.flags && corr && !bad) a.flags[sys] |= kFlagRefined;
      refined += (corr && !bad) ? 1 : 0;
    }
    if (staged) flush_chunk(a, cst, nk, sg, sy, sx);
  }
  flush_tally(a, tally);
  if (lane == 0 && refined) atomicAdd(&a.ctr->refined, refined);
}

template <int UPD, bool CORR>
hipError_t launch_mixed_classes(const SolveArgs& a, int grid, hipStream_t s) {
  const int nbmax = (a.geo.ncand + a.nb + 15) / 16;
#define OKR_CLS(K)                                                                            \
  if (nbmax >= K) {                                                                           \
    hipLaunchKernelGGL((mixed_class_kernel<K, UPD, CORR>), dim3(grid),                         \
                       dim3(64 * mixed_waves<CORR>()), 0, s, a);                              \
    hipError_t e = hipGetLastError();                                                         \
    if (e != hipSuccess) return e;                                                            \
  }
  OKR_CLS(8) OKR_CLS(7) OKR_CLS(6) OKR_CLS(5) OKR_CLS(4) OKR_CLS(3) OKR_CLS(2) OKR_CLS(1)
#undef OKR_CLS
  return hipSuccess;
}

}  // namespace

hipError_t launch_solve_mixed(const SolveArgs& a, int grid, hipStream_t s) {
  if (a.upd == 2)
    return a.refine ? launch_mixed_classes<2, true>(a, grid, s) : launch_mixed_classes<2, false>(a, grid, s);
  if (a.upd == 0)
    return a.refine ? launch_mixed_classes<0, true>(a, grid, s) : launch_mixed_classes<0, false>(a, grid, s);
  return a.refine ? launch_mixed_classes<1, true>(a, grid, s) : launch_mixed_classes<1, false>(a, grid, s);
}

}  // namespace okr
