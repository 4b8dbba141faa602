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
#include "okrig_internal.h"

namespace okr {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct VecOf;
template <> struct VecOf<float> { using type = f32x4; };
template <> struct VecOf<double> { using type = f64x4; };

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// T += Q P^T, all three in lane-row layout.
template <typename V>
__device__ __forceinline__ V acc_qpt(V c, const V& q, const V& p) {
  c = mfma4(p[0], q[0], c);
  c = mfma4(p[1], q[1], c);
  c = mfma4(p[2], q[2], c);
  c = mfma4(p[3], q[3], c);
  return c;
}

__device__ __forceinline__ float lane_value(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
__device__ __forceinline__ double lane_value(double x, int lane) {
  long long b = __double_as_longlong(x);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), lane);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ unsigned long long lane_u64(unsigned long long x, int lane) {
  unsigned lo = __builtin_amdgcn_readlane((unsigned)(x & 0xffffffffu), lane);
  unsigned hi = __builtin_amdgcn_readlane((unsigned)(x >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned long long uniform64(unsigned long long x) {
  unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(x & 0xffffffffu));
  unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(x >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

constexpr int tix(int i, int j) { return i * (i + 1) / 2 + j; }

// Tile column held by element v of lane group g (see the layout note above).
template <typename T> __device__ __forceinline__ constexpr int colmap(int g, int v);
template <> __device__ __forceinline__ constexpr int colmap<float>(int g, int v) { return 4 * g + v; }
template <> __device__ __forceinline__ constexpr int colmap<double>(int g, int v) { return 4 * v + g; }
// Lane group and element holding tile column c.
template <typename T> __device__ __forceinline__ constexpr int colgroup(int c) {
  return sizeof(T) == 4 ? (c >> 2) : (c & 3);
}
template <typename T> __device__ __forceinline__ constexpr int colelem(int c) {
  return sizeof(T) == 4 ? (c & 3) : (c >> 2);
}

constexpr int kWaves = 4;
constexpr int kChunk = 64;

template <typename T>
struct WaveScratch {
  int desc[128];      // point descriptors in system order
  float val[128];     // point values
  T buf[16 * 17];     // tile transposes and the read-out
};

template <typename T> struct Smem {
  T tc[kTcSize];
  T t0[kT0Size];
  int sdesc[128];
  WaveScratch<T> ws[kWaves];
};
// FP32 blocks also keep the covariance of every candidate pair, so a matrix
// entry is a single LDS read.
template <> struct Smem<float> {
  float tc[kTcSize];
  float t0[kT0Size];
  int sdesc[128];
  WaveScratch<float> ws[kWaves];
  float cc[kMaxCand * kMaxCand];
};

// Candidate descriptor: bits 0..6 candidate index; bits 8..15
// (s<<6)|((dy+r)<<3)|(dx+r); bits 16..20 target-table column s*16+|dy|*4+|dx|.
__device__ __forceinline__ int cand_desc(int c, int r, int W, int W2) {
  int s = c >= W2;
  int o = c - s * W2;
  int a = o / W, b = o - a * W;
  int ady = a > r ? a - r : r - a;
  int adx = b > r ? b - r : r - b;
  return c | (((s << 6) | (a << 3) | b) << 8) | ((s * 16 + ady * 4 + adx) << 16);
}

__device__ __forceinline__ int pair_class(int dp, int dq) {
  const int cp = (dp >> 8) & 0xff, cq = (dq >> 8) & 0xff;
  const int ddy = ((cp >> 3) & 7) - ((cq >> 3) & 7);
  const int ddx = (cp & 7) - (cq & 7);
  return ((cp ^ cq) & 64) | ((ddy < 0 ? -ddy : ddy) << 3) | (ddx < 0 ? -ddx : ddx);
}

template <typename T>
__device__ __forceinline__ T cov_pair(int dp, int dq, const Smem<T>& sm, int ncand);
template <>
__device__ __forceinline__ float cov_pair<float>(int dp, int dq, const Smem<float>& sm, int ncand) {
  return sm.cc[(dp & 0x7f) * ncand + (dq & 0x7f)];
}
template <>
__device__ __forceinline__ double cov_pair<double>(int dp, int dq, const Smem<double>& sm, int) {
  return sm.tc[pair_class(dp, dq)];
}

// Entry M[p][q] of the augmented matrix from the two indices' descriptors:
//   >= 0: data point, -1: identity padding, <= -2: border row b = -2 - d.
template <typename T>
__device__ __forceinline__ T entry(int dp, int dq, float vp, float vq, bool same,
                                   const Smem<T>& sm, int ncand) {
  if (dp >= 0 && dq >= 0) return cov_pair<T>(dp, dq, sm, ncand);
  if (dp == -1 || dq == -1) return same ? T(1) : T(0);
  if (dp < -1 && dq < -1) return T(0);
  int b, d;
  float v;
  if (dp < -1) {
    b = -2 - dp; d = dq; v = vq;
  } else {
    b = -2 - dq; d = dp; v = vp;
  }
  if (b == 0) return T(1);
  if (b == 1) return T(v);
  return sm.t0[(b - 2) * kT0Stride + (d >> 16)];
}

// Left-looking factorisation of one system with NB blocks; leaves the last
// diagonal tile (holding G in its border corner) in buf.
template <typename T, int NB>
__device__ __forceinline__ void factor_system(int n, int nb, const WaveScratch<T>& ws,
                                              const Smem<T>& sm, int ncand, T* buf, T& minpiv,
                                              T& maxpiv, bool& bad) {
  using V = typename VecOf<T>::type;
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  constexpr int N = 16 * NB;
  const int bstart = N - nb;
  V L[NB * (NB + 1) / 2];
  int rd[NB];
  float rv[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int p = 16 * i + r;
    rd[i] = p < n ? ws.desc[p] : (p < bstart ? -1 : -2 - (p - bstart));
    rv[i] = p < n ? ws.val[p] : 0.0f;
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    // ---- assemble block column j (negated) ----
    int cd[4];
    float cv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = 16 * j + colmap<T>(g, v);
      cd[v] = q < n ? ws.desc[q] : (q < bstart ? -1 : -2 - (q - bstart));
      cv[v] = q < n ? ws.val[q] : 0.0f;
    }
    const bool colC = 16 * j + 16 <= n;
#pragma unroll
    for (int i = j; i < NB; ++i) {
      V t;
      if (colC && 16 * i + 16 <= n) {
#pragma unroll
        for (int v = 0; v < 4; ++v) t[v] = -cov_pair<T>(rd[i], cd[v], sm, ncand);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool same = (i == j) && (r == colmap<T>(g, v));
          t[v] = -entry<T>(rd[i], cd[v], rv[i], cv[v], same, sm, ncand);
        }
      }
      L[tix(i, j)] = t;
    }
    // ---- updates from the finished columns: S_ij += L_ik L_jk^T ----
#pragma unroll
    for (int k = 0; k < j; ++k) {
#pragma unroll
      for (int i = j; i < NB; ++i) L[tix(i, j)] = acc_qpt(L[tix(i, j)], L[tix(i, k)], L[tix(j, k)]);
    }
    // ---- diagonal tile ----
    const int ne = (j == NB - 1) ? 16 - nb : 16;
    V X;
#pragma unroll
    for (int v = 0; v < 4; ++v) X[v] = (r == colmap<T>(g, v)) ? T(1) : T(0);
    V D = L[tix(j, j)];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      if (c < ne) {
        const int g0 = colgroup<T>(c), v0 = colelem<T>(c);
        T piv = -lane_value(D[v0], 16 * g0 + c);
        if (!(piv > T(0)) || !isfinite(piv)) {
          bad = true;
          piv = T(1);
        }
        minpiv = piv < minpiv ? piv : minpiv;
        maxpiv = piv > maxpiv ? piv : maxpiv;
        const T sq = sqrt(piv);
        const T is = T(1) / sq;
        const bool mine = (g == g0);
        const T u = (mine && r > c) ? -D[v0] * is : T(0);
        X[v0] = mine ? X[v0] * is : X[v0];
        const T w = mine ? X[v0] : T(0);
        D = mfma4(u, u, D);
        X = mfma4(-u, w, X);
      }
    }
    L[tix(j, j)] = D;
    if (j < NB - 1) {
      // Inv = transpose(X) through LDS, negated
#pragma unroll
      for (int v = 0; v < 4; ++v) buf[r * 17 + colmap<T>(g, v)] = X[v];
      __builtin_amdgcn_wave_barrier();
      V NI;
#pragma unroll
      for (int v = 0; v < 4; ++v) NI[v] = -buf[colmap<T>(g, v) * 17 + r];
      __builtin_amdgcn_wave_barrier();
      // off-diagonal solve: L_ij = M_ij L_jj^{-T} = S_ij (-Inv)^T
#pragma unroll
      for (int i = j + 1; i < NB; ++i) {
        V z = {T(0), T(0), T(0), T(0)};
        L[tix(i, j)] = acc_qpt(z, L[tix(i, j)], NI);
      }
    }
  }
  const V& Lz = L[tix(NB - 1, NB - 1)];
#pragma unroll
  for (int v = 0; v < 4; ++v) buf[r * 17 + colmap<T>(g, v)] = Lz[v];
  __builtin_amdgcn_wave_barrier();
}

template <typename T, int NB>
__device__ void solve_system(int n, int nb, const WaveScratch<T>& ws, const Smem<T>& sm, int ncand,
                             T* buf, T sill, int ntgt, T* est, T* var, T& minpiv, T& maxpiv,
                             bool& bad) {
  minpiv = T(3.0e38);
  maxpiv = T(0);
  bad = false;
  factor_system<T, NB>(n, nb, ws, sm, ncand, buf, minpiv, maxpiv, bad);
  const int lane = threadIdx.x & 63;
  const int ne = 16 - nb;
  if (lane < ntgt) {
    const int t = lane + 1;
    const T g11 = buf[ne * 17 + ne];
    const T g1z = buf[ne * 17 + ne + 1];
    const T g1t = buf[ne * 17 + ne + 1 + t];
    const T gzt = buf[(ne + 1) * 17 + ne + 1 + t];
    const T gtt = buf[(ne + 1 + t) * 17 + ne + 1 + t];
    const T m = (T(1) - g1t) / g11;
    *est = gzt + m * g1z;
    *var = sill - gtt + (T(1) - g1t) * m;
  }
  __builtin_amdgcn_wave_barrier();
}

template <typename T, int NBMAX>
__device__ __forceinline__ void dispatch(int NB, int n, int nb, const WaveScratch<T>& ws,
                                         const Smem<T>& sm, int ncand, T* buf, T sill, int ntgt,
                                         T* est, T* var, T& mn, T& mx, bool& bad) {
  switch (NB) {
#define OKR_NB(K)                                                                      \
  case K:                                                                              \
    if constexpr (NBMAX >= K)                                                          \
      solve_system<T, K>(n, nb, ws, sm, ncand, buf, sill, ntgt, est, var, mn, mx, bad); \
    break;
    OKR_NB(1) OKR_NB(2) OKR_NB(3) OKR_NB(4) OKR_NB(5) OKR_NB(6) OKR_NB(7) OKR_NB(8)
#undef OKR_NB
    default: break;
  }
}

template <typename T>
__device__ void init_block(const SolveArgs& a, Smem<T>& sm) {
  const double* tcs = a.tab.tc_d;
  const double* t0s = a.tab.t0_d;
  for (int i = threadIdx.x; i < kTcSize; i += blockDim.x) sm.tc[i] = T(tcs[i]);
  for (int i = threadIdx.x; i < kT0Size; i += blockDim.x) sm.t0[i] = T(t0s[i]);
  for (int i = threadIdx.x; i < 128; i += blockDim.x)
    sm.sdesc[i] = i < a.geo.ncand ? cand_desc(i, a.geo.r, a.geo.W, a.geo.W2) : 0;
}

__device__ __forceinline__ void atomic_max_float(unsigned int* addr, float v) {
  if (v > 0.0f && isfinite(v)) atomicMax(addr, __float_as_uint(v));
}

// Persistent batched solve over the size-sorted permutation (largest n first).
// mode 0: all systems; mode 1: the FP64 re-solve list.
template <typename T, int NBMAX>
__global__ __launch_bounds__(256) void solve_kernel(SolveArgs a, int mode) {
  __shared__ Smem<T> sm;
  init_block<T>(a, sm);
  __syncthreads();
  if constexpr (sizeof(T) == 4) {
    // covariance of every candidate pair, rounded once from the FP64 table
    const int nc = a.geo.ncand;
    for (int i = threadIdx.x; i < nc * nc; i += blockDim.x) {
      const int p = i / nc, q = i - p * nc;
      sm.cc[i] = (float)a.tab.tc_d[pair_class(sm.sdesc[p], sm.sdesc[q])];
    }
    __syncthreads();
  }
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  WaveScratch<T>& ws = sm.ws[wid];
  const Geometry& geo = a.geo;
  const unsigned long long total =
      mode == 0 ? (unsigned long long)geo.nsys : a.ctr->n_fallback_list;
  unsigned long long* cursor = mode == 0 ? &a.ctr->next : &a.ctr->next2;
  const uint32_t* list = mode == 0 ? a.perm : a.fallback;
  const int ntgt = geo.f - 1;
  const int ncand = geo.ncand;
  const T sill = T(a.sill);
  const unsigned plane = (unsigned)geo.plane;
  const unsigned nx = (unsigned)geo.nx;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int d0 = sm.sdesc[lane];
  const int d1 = lane + 64 < ncand ? sm.sdesc[lane + 64] : 0;
  for (;;) {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(cursor, (unsigned long long)kChunk);
    base = uniform64(base);
    if (base >= total) break;
    const int nk = (int)((total - base) < (unsigned long long)kChunk ? (total - base) : kChunk);
    unsigned int msys = 0;
    unsigned long long mlo = 0, mhi = 0;
    int mcnt = 0;
    if (lane < nk) {
      msys = list[base + lane];
      mlo = a.bits[2ull * msys];
      mhi = a.bits[2ull * msys + 1];
      mcnt = a.count[msys];
    }
    // values of the next system, loaded ahead of its factorisation
    float pv0 = 0.0f, pv1 = 0.0f;
    int pp0 = -1, pp1 = -1;
    auto prefetch = [&](int k) {
      const unsigned sys = __builtin_amdgcn_readlane(msys, k);
      const unsigned long long lo = lane_u64(mlo, k), hi = lane_u64(mhi, k);
      const unsigned gap = sys / plane;
      const unsigned pix = sys - gap * plane;
      const unsigned y = pix / nx, x = pix - y * nx;
      const int n0 = __popcll(lo);
      pp0 = ((lo >> lane) & 1ull) ? __popcll(lo & below) : -1;
      pp1 = (lane + 64 < ncand && ((hi >> lane) & 1ull)) ? n0 + __popcll(hi & below) : -1;
      if (pp0 >= 0) {
        const int c = (d0 >> 8) & 0xff;
        const long long src = (long long)(gap + ((c >> 6) & 1)) * geo.plane +
                              (long long)((int)y + ((c >> 3) & 7) - geo.r) * geo.nx +
                              ((int)x + (c & 7) - geo.r);
        pv0 = a.slices[src];
      }
      if (pp1 >= 0) {
        const int c = (d1 >> 8) & 0xff;
        const long long src = (long long)(gap + ((c >> 6) & 1)) * geo.plane +
                              (long long)((int)y + ((c >> 3) & 7) - geo.r) * geo.nx +
                              ((int)x + (c & 7) - geo.r);
        pv1 = a.slices[src];
      }
    };
    prefetch(0);
    for (int k = 0; k < nk; ++k) {
      const unsigned sys = __builtin_amdgcn_readlane(msys, k);
      const unsigned long long lo = lane_u64(mlo, k), hi = lane_u64(mhi, k);
      const int cnt = __builtin_amdgcn_readlane(mcnt, k);
      if (pp0 >= 0) {
        ws.desc[pp0] = d0;
        ws.val[pp0] = pv0;
      }
      if (pp1 >= 0) {
        ws.desc[pp1] = d1;
        ws.val[pp1] = pv1;
      }
      __builtin_amdgcn_wave_barrier();
      if (k + 1 < nk) prefetch(k + 1);
      const int n = __popcll(lo) + __popcll(hi);
      const int NB = (n + a.nb + 15) >> 4;
      T est = 0, var = 0, mn, mx;
      bool bad;
      dispatch<T, NBMAX>(NB, n, a.nb, ws, sm, ncand, ws.buf, sill, ntgt, &est, &var, mn, mx, bad);
      const T kappa = mx / mn;
      const bool fallback = mode == 0 && a.fallback && (bad || (double)kappa > a.kappa_limit);
      const unsigned gap = sys / plane;
      const unsigned pix = sys - gap * plane;
      if (fallback) {
        if (lane == 0) {
          const unsigned long long slot = atomicAdd(&a.ctr->n_fallback_list, 1ull);
          a.fallback[slot] = sys;
        }
      } else if (lane < ntgt) {
        const long long o = ((long long)gap * geo.f + lane + 1) * geo.plane + pix;
        a.volume[o] = (float)est;
        if (a.variance) a.variance[o] = (float)var;
      }
      if (lane == 0) {
        uint8_t fl = (cnt & kFloorBit) ? kFlagFloor : 0;
        if (mode == 1) fl |= kFlagFp64;
        if (bad && mode == 0) fl |= kFlagBadPivot;
        if (a.flags) {
          if (mode == 0) a.flags[sys] = fl;
          else a.flags[sys] |= fl;
        }
        if (bad && mode == 0) atomicAdd(&a.ctr->bad_pivot, 1ull);
        if (mode == 1) atomicAdd(&a.ctr->fp64_fallback, 1ull);
        atomic_max_float(&a.ctr->max_kappa_bits, (float)kappa);
      }
    }
  }
}

template <typename T>
hipError_t launch_nbmax(const SolveArgs& a, int grid, int mode, hipStream_t s) {
  const int nbmax = (a.geo.ncand + a.nb + 15) / 16;
  switch (nbmax) {
#define OKR_CASE(K) \
  case K: hipLaunchKernelGGL((solve_kernel<T, K>), dim3(grid), dim3(256), 0, s, a, mode); break;
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
  if (a.precision == 3) return launch_nbmax<double>(a, grid, 0, s);
  return launch_nbmax<float>(a, grid, 0, s);
}

hipError_t launch_solve_fallback(const SolveArgs& a, int grid, hipStream_t s) {
  return launch_nbmax<double>(a, grid, 1, s);
}

}  // namespace okr
