// Batched ordinary-kriging solver: one wavefront per (column, gap) system.
//
// Each system's extended covariance matrix (Appendix A with one constant
// predictor) is augmented by the right-hand sides of all its targets,
//
//        M = [[C, B], [B^T, 0]],   B = [1 | z | c0_1 ... c0_{f-1}],
//
// padded with identity rows between C and B to N = 16*NB rows, and held in
// registers as lower 16x16 tiles. Eliminating the C (and padding) columns by
// Cholesky leaves, in the B x B corner, -G with G = B^T C^{-1} B, the Gram
// matrix of L^{-1} B. Every estimate and kriging variance follows from G:
//
//   z_hat_t  = G[z][t] + (1 - G[1][t]) G[1][z] / G[1][1]
//   sigma2_t = sill - G[t][t] + (1 - G[1][t])^2 / G[1][1]
//
// which is the bordered solution [w; mu] = K^{-1} [c0; 1] with the Lagrange
// multiplier eliminated (the weights are never formed).
//
// Register layout of a tile T ("lane-row"): lane l = 16 g + r holds
// T[r][col(g, v)] in element v, where col(g, v) = 4g + v for FP32 tiles and
// 4v + g for FP64 tiles (the row order of the two instructions' accumulators).
// With A-operand P and B-operand Q taken element by element from two such
// tiles, four 16x16x4 MFMAs accumulate T += Q P^T in the same layout, so the
// updates S_ij += L_ik L_jk^T and the off-diagonal solve L_ik = M_ik L_kk^{-T}
// need no data movement. The matrix is stored negated (S = -M) so every
// update is an accumulation.
//
// The factorisation is left-looking: block column j is assembled from the
// covariance tables only when it is reached, receives the updates of the
// finished columns, and its L tiles stay live only while later columns need
// them, so about NB^2/4 tiles are live at once instead of NB(NB+1)/2.
//
// A diagonal tile is factored column by column: the pivot is read with
// readlane, the scaled column is fed to one MFMA as a rank-1 update of the
// tile, and a second MFMA applies the same row operation to the transpose of
// an identity tile, which yields L_kk^{-T} for the off-diagonal solves.
//
// Work distribution: persistent waves take chunks of 64 systems from the
// size-sorted permutation (largest first); lane i loads system i's metadata,
// and the neighbour values of the next system are loaded while the current
// one is factored.
#include "solver_core.h"

namespace okr {
namespace {

// One persistent launch per 16-wide size class: every system of the class has
// NB blocks, so the kernel holds exactly that class's register footprint. The
// class is a contiguous range of the size-sorted permutation.
// FP32 classes run eight waves per workgroup sharing one copy of the block
// tables (two workgroups per CU, four waves per SIMD at 128 VGPRs); FP64
// classes (twice the tile registers) run two waves per SIMD in workgroups of four.
template <typename T> constexpr int class_waves() { return sizeof(T) == 4 ? 8 : 4; }

template <typename T, int NB>
__global__ __launch_bounds__(64 * class_waves<T>())
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
void solve_class_kernel(SolveArgs a) {
  __shared__ Smem<T> sm;
  __shared__ WaveScratch<T> wsa[class_waves<T>()];
  __shared__ ChunkStage csa[class_waves<T>()];
  block_setup<T>(a, sm);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  WaveScratch<T>& ws = wsa[wid];
  ChunkStage& cst = csa[wid];
  const int nb = a.nb;
  int nlo = 16 * (NB - 1) - nb + 1, nhi = 16 * NB - nb;
  if (nlo < 1) nlo = 1;
  if (nhi > kHist - 1) nhi = kHist - 1;
  if (nhi > a.nmax) nhi = a.nmax;
  if (nlo > nhi) return;
  const unsigned long long start = a.ctr->offsets[nhi];
  const unsigned long long end = a.ctr->offsets[nlo] + a.ctr->hist[nlo];
  ClassRange cr = class_range(a, NB, start, end, false);
  const T sill = T(a.sill);
  const int ntgt = a.geo.f - 1, ncand = a.geo.ncand;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int d0 = sm.sdesc[lane];
  const int d1 = lane + 64 < ncand ? sm.sdesc[lane + 64] : 0;
  Tally tally;
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
      pipe_commit<T>(q, ws, d0, d1, n);
      if (k + 1 < nk) {
        if (staged)
          pipe_prefetch_staged(q, cst, k + 1, d0, d1, below, ncand);
        else
          pipe_prefetch(q, a, k + 1, d0, d1, below);
      }
      T est = 0, var = 0, mn, mx;
      bool bad;
      // nb is fixed for the launch: kept out of loop-invariant code motion, as in
      // the mixed kernel, so its tests stay per-system scalar compares
      int nbs = nb;
      asm volatile("" : "+s"(nbs));
      solve_system<T, NB>(n, nbs, ws, sm, ncand, ws.buf, sill, ntgt, &est, &var, mn, mx, bad);
      finish_system<T>(a, 0, sys, cnt, est, var, mn, mx, bad, tally, false, 0,
                       staged ? &cst : nullptr, k);
    }
    if (staged) flush_chunk(a, cst, nk, sg, sy, sx);
  }
  flush_tally(a, tally);
}

// FP64 re-solve of the queued systems (any size class).
template <typename T, int NBMAX>
__global__ __launch_bounds__(256) void solve_list_kernel(SolveArgs a) {
  __shared__ Smem<T> sm;
  __shared__ WaveScratch<T> wsa[4];
  block_setup<T>(a, sm);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  WaveScratch<T>& ws = wsa[wid];
  const unsigned long long total = a.ctr->n_fallback_list;
  const T sill = T(a.sill);
  const int ntgt = a.geo.f - 1, ncand = a.geo.ncand;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int d0 = sm.sdesc[lane];
  const int d1 = lane + 64 < ncand ? sm.sdesc[lane + 64] : 0;
  Tally tally;
  for (;;) {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(&a.ctr->next2, (unsigned long long)kChunk);
    base = uniform64(base);
    if (base >= total) break;
    const int nk = (int)((total - base) < (unsigned long long)kChunk ? (total - base) : kChunk);
    Pipe q;
    pipe_load(q, a, a.fallback, base, nk);
    pipe_prefetch(q, a, 0, d0, d1, below);
    for (int k = 0; k < nk; ++k) {
      const unsigned sys = __builtin_amdgcn_readlane(q.msys, k);
      const unsigned long long lo = lane_u64(q.mlo, k), hi = lane_u64(q.mhi, k);
      const int cnt = __builtin_amdgcn_readlane(q.mcnt, k);
      const int n = __popcll(lo) + __popcll(hi);
      pipe_commit<T>(q, ws, d0, d1, n);
      if (k + 1 < nk) pipe_prefetch(q, a, k + 1, d0, d1, below);
      const int NB = (n + a.nb + 15) >> 4;
      T est = 0, var = 0, mn, mx;
      bool bad;
      dispatch<T, NBMAX>(NB, n, a.nb, ws, sm, ncand, ws.buf, sill, ntgt, &est, &var, mn, mx, bad);
      finish_system<T>(a, 1, sys, cnt, est, var, mn, mx, bad, tally);
    }
  }
  flush_tally(a, tally);
}

template <typename T>
hipError_t launch_classes(const SolveArgs& a, int grid, hipStream_t s) {
  const int nbmax = (a.geo.ncand + a.nb + 15) / 16;
#define OKR_CLS(K)                                                                          \
  if (nbmax >= K) {                                                                         \
    hipLaunchKernelGGL((solve_class_kernel<T, K>), dim3(grid), dim3(64 * class_waves<T>()), \
                       0, s, a);                                                            \
    hipError_t e = hipGetLastError();                                                       \
    if (e != hipSuccess) return e;                                                          \
  }
  OKR_CLS(8) OKR_CLS(7) OKR_CLS(6) OKR_CLS(5) OKR_CLS(4) OKR_CLS(3) OKR_CLS(2) OKR_CLS(1)
#undef OKR_CLS
  return hipSuccess;
}

template <typename T>
hipError_t launch_list(const SolveArgs& a, int grid, hipStream_t s) {
  const int nbmax = (a.geo.ncand + a.nb + 15) / 16;
  switch (nbmax) {
#define OKR_CASE(K) \
  case K: hipLaunchKernelGGL((solve_list_kernel<T, K>), dim3(grid), dim3(256), 0, s, a); break;
    OKR_CASE(1) OKR_CASE(2) OKR_CASE(3) OKR_CASE(4) OKR_CASE(5) OKR_CASE(6) OKR_CASE(7) OKR_CASE(8)
#undef OKR_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

int solve_blocks_needed(const Geometry& g) {
  (void)g;
  return 256 * 3;
}

hipError_t launch_solve(const SolveArgs& a, int grid, hipStream_t s) {
  if (a.precision == 3) return launch_classes<double>(a, grid, s);
  return launch_classes<float>(a, grid, s);
}

hipError_t launch_solve_fallback(const SolveArgs& a, int grid, hipStream_t s) {
  return launch_list<double>(a, grid, s);
}

}  // namespace okr
