// Explicit solutions and FP64 corrections on top of the batched factorisation.
//
// The read-out of kernels_solve.hip never forms the kriging weights. The
// refined paths need them: after the factorisation (whose L tiles are kept),
// a block back-substitution gives X = C^{-1} [1 | z | c0_1 ... c0_{f-1}], from
// which the weights w_t = x_{c0_t} - mu_t x_1 and the adjoint vector
// nu_w = x_z - (1'x_z / 1'x_1) x_1 of the bordered system follow.
//
// Trailing-update precisions (UPD):
//   0  FP32 MFMA (16x16x4)
//   1  split FP16: each L tile is kept as hi + lo halves and a product is
//      hi*hi + hi*lo + lo*hi on 16x16x16 MFMAs with FP32 accumulation
//   2  split BF16: the same with bfloat16 halves
// The diagonal tiles and the back-substitution are FP32 in every case, the
// off-diagonal solves too except in the FP16 read-out (split products there).
#pragma once

#include "solver_core.h"

namespace okr {
namespace {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef __bf16 b4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma_k16(h4 a, h4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_k16(b4 a, b4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Storage of finished L tiles for the trailing updates: the tiles of block
// columns 2m and 2m+1 of one block row are kept together (h = 0, 1), each as
// the operand of the 16x16x16 (or, FP32, 16x16x4) MFMAs of its products.
template <int UPD> struct PairStore;

template <> struct PairStore<0> {
  f32x4 t[2];
  __device__ __forceinline__ void put(int h, const f32x4& x) { t[h] = x; }
  __device__ __forceinline__ f32x4 get(int h) const { return t[h]; }
};

typedef float f32x2 __attribute__((ext_vector_type(2)));

template <typename E, typename V4> struct SplitPair {
  typedef E V2 __attribute__((ext_vector_type(2)));
  V4 hi[2], lo[2];   // whole 4-element halves; concatenated at each use
  // hi = round(x), lo = round(x - hi), two elements per packed conversion
  __device__ __forceinline__ void put(int h, const f32x4& x) {
    const f32x2 a = {x[0], x[1]}, b = {x[2], x[3]};
    const V2 ha = __builtin_convertvector(a, V2), hb = __builtin_convertvector(b, V2);
    const V2 la = __builtin_convertvector(a - __builtin_convertvector(ha, f32x2), V2);
    const V2 lb = __builtin_convertvector(b - __builtin_convertvector(hb, f32x2), V2);
    hi[h] = __builtin_shufflevector(ha, hb, 0, 1, 2, 3);
    lo[h] = __builtin_shufflevector(la, lb, 0, 1, 2, 3);
  }
  __device__ __forceinline__ f32x4 get(int h) const {
    f32x4 x;
#pragma unroll
    for (int v = 0; v < 4; ++v) x[v] = (float)hi[h][v] + (float)lo[h][v];
    return x;
  }
};
template <> struct PairStore<1> : SplitPair<_Float16, h4> {};
template <> struct PairStore<2> : SplitPair<__bf16, b4> {};

// c += Q P^T summed over both block columns of a pair.
template <int UPD>
__device__ __forceinline__ f32x4 acc_pair(f32x4 c, const PairStore<UPD>& q, const PairStore<UPD>& p) {
  if constexpr (UPD == 0) {
    c = acc_qpt(c, q.t[0], p.t[0]);
    return acc_qpt(c, q.t[1], p.t[1]);
  } else {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      c = mfma_k16(p.lo[h], q.hi[h], c);
      c = mfma_k16(p.hi[h], q.lo[h], c);
      c = mfma_k16(p.hi[h], q.hi[h], c);
    }
    return c;
  }
}

// c += Q P^T over the first block column of a pair only.
template <int UPD>
__device__ __forceinline__ f32x4 acc_first(f32x4 c, const PairStore<UPD>& q, const PairStore<UPD>& p) {
  if constexpr (UPD == 0) {
    return acc_qpt(c, q.t[0], p.t[0]);
  } else {
    c = mfma_k16(p.lo[0], q.hi[0], c);
    c = mfma_k16(p.hi[0], q.lo[0], c);
    return mfma_k16(p.hi[0], q.hi[0], c);
  }
}

// Lane-row transpose of a tile through the wave's LDS buffer, negated.
__device__ __forceinline__ f32x4 neg_transpose(const f32x4& x, float* buf) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) buf[r * 17 + 4 * g + v] = x[v];
  __builtin_amdgcn_wave_barrier();
  f32x4 t;
#pragma unroll
  for (int v = 0; v < 4; ++v) t[v] = -buf[(4 * g + v) * 17 + r];
  __builtin_amdgcn_wave_barrier();
  return t;
}

// Left-looking factorisation (FP32 diagonal / off-diagonal solves, UPD trailing
// updates) keeping every L tile in registers. With LAST_X (the back-substitution
// follows) every diagonal L^{-T} tile, the last one included, goes to the wave's
// LDS area xs (tile j at xs[64 j + lane]). Leaves the last diagonal tile (with
// G in its border corner) in buf.
template <int NB, int UPD, bool LAST_X>
__device__ __forceinline__ void factor_keep(int n, int nb, const WaveScratch<float>& ws,
                                            const Smem<float>& sm, int ncand, float* buf,
                                            float& minpiv, float& maxpiv, bool& bad,
                                            PairStore<UPD> (&Ls)[NB][(NB + 1) / 2],
                                            f32x4* xs) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  constexpr int N = 16 * NB;
  const int bstart = N - nb;
  int rb[NB], sh;
  float vrow;
  f32_rows<NB>(n, bstart, sm.bz, ncand, ws, rb, sh, vrow);
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    __builtin_amdgcn_sched_barrier(0);
    int ofs[4];
    float cv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = 16 * j + 4 * g + v;
      ofs[v] = ws.ofs[q];
      cv[v] = ws.val[q];
    }
    f32x4 S[NB];
#pragma unroll
    for (int i = j; i < NB; ++i) S[i] = tile_f32<NB>(i, j, n, bstart, rb, sh, vrow, ofs, cv, sm);
    // updates from the finished block columns, two at a time
#pragma unroll
    for (int m = 0; 2 * m + 1 < j; ++m) {
#pragma unroll
      for (int i = j; i < NB; ++i) S[i] = acc_pair<UPD>(S[i], Ls[i][m], Ls[j][m]);
    }
    if (j & 1) {
#pragma unroll
      for (int i = j; i < NB; ++i) S[i] = acc_first<UPD>(S[i], Ls[i][j / 2], Ls[j][j / 2]);
    }
    // diagonal tile
    const int ne = (j == NB - 1) ? 16 - nb : 16;
    f32x4 X;
    f32x4 D = S[j];
    diag_factor(D, X, ne, buf, minpiv, maxpiv, bad, j < NB - 1 || LAST_X);
    if constexpr (LAST_X) xs[64 * j + lane] = X;
    if (j < NB - 1) {
      const f32x4 NI = neg_transpose(X, buf);
      // FP16 halves: the off-diagonal solves as split products too (three
      // 16-cycle MFMAs instead of four 32-cycle FP32 ones). Kept in FP32 for
      // BF16 halves (too few bits for the explicit inverse).
      if constexpr (UPD != 1) {
#pragma unroll
        for (int i = j + 1; i < NB; ++i) {
          const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
          Ls[i][j / 2].put(j & 1, acc_qpt(z, S[i], NI));
        }
      } else {
        PairStore<UPD> ns;
        ns.put(0, NI);
#pragma unroll
        for (int i = j + 1; i < NB; ++i) {
          PairStore<UPD> ss;
          ss.put(0, S[i]);
          f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
          z = mfma_k16(ns.lo[0], ss.hi[0], z);
          z = mfma_k16(ns.hi[0], ss.lo[0], z);
          z = mfma_k16(ns.hi[0], ss.hi[0], z);
          Ls[i][j / 2].put(j & 1, z);
        }
      }
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) buf[r * 17 + 4 * g + v] = D[v];
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// Back-substitution in transposed form: with Z_I the (border rows) x (block I)
// tile of X^T, Z_I = (Y_I - sum_{K>I} Z_K L_KI) L_II^{-1}, Y the border rows of
// L. For the last block, Z is minus the border rows of its partial inverse.
// Row ne + b of the Z tiles holds x_b (b = 0: C^{-1} 1, 1: C^{-1} z,
// 1 + t: C^{-1} c0_t); write_rows copies them to LDS.
template <int NB, int UPD>
__device__ __forceinline__ void back_substitute(int nb, const PairStore<UPD> (&Ls)[NB][(NB + 1) / 2],
                                                const f32x4* xs, float* buf, f32x4 (&Z)[NB]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int ne = 16 - nb;
  {
    const f32x4 NI = neg_transpose(xs[64 * (NB - 1) + lane], buf);
#pragma unroll
    for (int v = 0; v < 4; ++v) Z[NB - 1][v] = (r >= ne && 4 * g + v < ne) ? NI[v] : 0.0f;
  }
#pragma unroll
  for (int I = NB - 2; I >= 0; --I) {
    const f32x4 yl = Ls[NB - 1][I / 2].get(I & 1);
    // two accumulators (even and odd K), so that consecutive products do not
    // wait on each other's MFMA results
    f32x4 acc, acc2 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = r >= ne ? yl[v] : 0.0f;
#pragma unroll
    for (int K = I + 1; K < NB; ++K) {
      const f32x4 P = neg_transpose(Ls[K][I / 2].get(I & 1), buf);
      if ((K - I) & 1)
        acc = acc_qpt(acc, Z[K], P);
      else
        acc2 = acc_qpt(acc2, Z[K], P);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] += acc2[v];
    const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
    Z[I] = acc_qpt(z, acc, xs[64 * I + lane]);
  }
}

// Rows row0 .. row0 + count - 1 of the Z tiles (one value per point) to slots
// slot0 .. slot0 + count - 1 of x.
template <int NB>
__device__ __forceinline__ void write_rows(const f32x4 (&Z)[NB], int row0, int count, int slot0,
                                           float (*x)[128]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int k = r - row0;
  if (k >= 0 && k < count) {
    float* dst = x[slot0 + k];
#pragma unroll
    for (int I = 0; I < NB; ++I) {
#pragma unroll
      for (int v = 0; v < 4; ++v) dst[16 * I + 4 * g + v] = Z[I][v];
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// ---- wave-wide reductions in a fixed order (the results are uniform) ----
// DPP controls: quad_perm [1,0,3,2] and [2,3,0,1], row_ror:4 and row_ror:8
// give every lane its 16-lane row's sum r0..r3; row_bcast:15 (rows 1 and 3
// take the last lane of the row before) and row_bcast:31 (rows 2 and 3 take
// lane 31) then leave (r2 + r3) + (r0 + r1) in lane 63, which is read once.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}
// Row broadcasts into the rows of ROWS only; the other rows get 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double bcast_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float bcast_f(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xf, false));
}
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

template <int K>
__device__ __forceinline__ void wave_sums(double (&x)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += dpp_d<0xB1>(x[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += dpp_d<0x4E>(x[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += dpp_d<0x124>(x[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += dpp_d<0x128>(x[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += bcast_d<kRowBcast15, 0xa>(x[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += bcast_d<kRowBcast31, 0xc>(x[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] = lane_value(x[k], 63);
}

template <int K>
__device__ __forceinline__ void wave_sums_f(float (&x)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += dpp_f<0xB1>(x[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += dpp_f<0x4E>(x[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += dpp_f<0x124>(x[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += dpp_f<0x128>(x[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += bcast_f<kRowBcast15, 0xa>(x[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += bcast_f<kRowBcast31, 0xc>(x[k]);
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] = lane_value(x[k], 63);
}

__device__ __forceinline__ double wave_sum_d(double x) {
  double s[1] = {x};
  wave_sums(s);
  return s[0];
}

__device__ __forceinline__ float wave_max_abs(float x) {
  x = fabsf(x);
  x = fmaxf(x, dpp_f<0xB1>(x));
  x = fmaxf(x, dpp_f<0x4E>(x));
  x = fmaxf(x, dpp_f<0x124>(x));
  x = fmaxf(x, dpp_f<0x128>(x));
  return fmaxf(fmaxf(lane_value(x, 0), lane_value(x, 16)), fmaxf(lane_value(x, 32), lane_value(x, 48)));
}

// One system with the FP64-corrected estimate (see kernels_mixed.hip).
constexpr int kRowTargets = 3;   // targets whose solution rows are staged at once
constexpr int kSlotXs = 2 + kRowTargets;
constexpr int kXRows = 3 + kRowTargets;
struct MixedScratch {
  float zr[128];                   // raw data values
};
// Each wave's LDS area holds the diagonal L^{-T} tiles (64 f32x4 per block)
// during the factorisation and the back-substitution, and afterwards, in the
// same bytes, the solution rows x[kXRows][128] (x_1, x_z, x_t of up to
// kRowTargets targets, x_s) and nu_w by candidate index (double[128], 0 for
// dropped candidates).
template <int NB> constexpr int area_vec4() {
  return NB * 64 > (kXRows * 128 * 4 + 128 * 8) / 16 ? NB * 64 : (kXRows * 128 * 4 + 128 * 8) / 16;
}
__device__ __forceinline__ float (*area_x(f32x4* area))[128] {
  return reinterpret_cast<float (*)[128]>(area);
}
__device__ __forceinline__ double* area_nuc(f32x4* area) {
  return reinterpret_cast<double*>(reinterpret_cast<float*>(area) + kXRows * 128);
}

// FP64 tables shared by the refined kernels' blocks.
struct MixedTables {
  double tc64[kTcSize];
  double t064[kT0Size];
};

// Refined estimates: the FP64 covariance of every point offset (layout of
// conv_row / conv_col), so an entry of the FP64 matrix-vector product is one
// LDS read.
struct MixedSmem : MixedTables {
  double cc64[kConvSize];
  // Slot of a point in the vector the offset mat-vec reads: the window laid
  // out 7 wide and 7 high per slice whatever the radius (slots outside the
  // window stay zero), so the mat-vec's inner loop has a fixed length.
  __device__ __forceinline__ static int vslot(int d) {
    const int c = (d >> 8) & 0xff;
    return (c >> 6) * (kMaxWin * kMaxWin) + ((c >> 3) & 7) * kMaxWin + (c & 7);
  }
};

// Leave-one-slice-out blocks also need the pair class (for the derivative
// tables), so they keep a byte class table instead.
struct LosoSmem : MixedTables {
  uint8_t cls8[kMaxCand * kMaxCand];
  int stride;
  __device__ __forceinline__ const uint8_t* row(int c) const { return cls8 + c * stride; }
  __device__ __forceinline__ double at(const uint8_t* row, int cq) const { return tc64[row[cq]]; }
  __device__ __forceinline__ static int vslot(int d) { return d & 0x7f; }   // candidate index
};

__device__ __forceinline__ void mixed_tables(const SolveArgs& a, MixedTables& mt, double tscale) {
  for (int i = threadIdx.x; i < kTcSize; i += blockDim.x) mt.tc64[i] = a.tab.tc_d[i] * tscale;
  for (int i = threadIdx.x; i < kT0Size; i += blockDim.x) mt.t064[i] = a.tab.t0_d[i] * tscale;
}

// Block set-up of the refined kernels (covariances times tscale). Needs the
// block's candidate descriptors.
__device__ __forceinline__ void mixed_setup(const SolveArgs& a, const Smem<float>&, MixedSmem& msm,
                                            double tscale) {
  mixed_tables(a, msm, tscale);
  for (int i = threadIdx.x; i < kConvSize; i += blockDim.x)
    msm.cc64[i] = a.tab.tc_d[conv_class(i)] * tscale;
}
__device__ __forceinline__ void mixed_setup(const SolveArgs& a, const Smem<float>& sm, LosoSmem& msm,
                                            double tscale) {
  mixed_tables(a, msm, tscale);
  const int nc = a.geo.ncand;
  if (threadIdx.x == 0) msm.stride = nc;
  for (int i = threadIdx.x; i < nc * nc; i += blockDim.x) {
    const int p = i / nc, q = i - p * nc;
    msm.cls8[i] = (uint8_t)pair_class(sm.sdesc[p], sm.sdesc[q]);
  }
}

// (C v)_p for the lane's points p = lane, lane + 64, in FP64. v is indexed by
// MixedSmem::vslot (zero for dropped candidates and for slots outside the
// window), so the loop runs over the whole 7-wide window rows with fixed
// offsets from each lane's row: no index loads and no branches inside a row,
// so a row's table and vector reads are issued together. Slots outside the
// window add exact zeros. The second point's sums only run when a system has
// more than 64 points.
template <bool TWO>
__device__ __forceinline__ void matvec64_rows(int W, const double* row0, const double* row1,
                                              const double* vc, double (&a0)[4],
                                              double (&a1)[4]) {
  for (int s = 0; s < 2; ++s) {
    for (int y = 0; y < W; ++y) {
      const int k = s * kConvSub + y * kConvQ;
      const double* v = vc + s * (kMaxWin * kMaxWin) + y * kMaxWin;
      // the row's reads first, then its products
      double vq[kMaxWin], c0[kMaxWin], c1[kMaxWin];
#pragma unroll
      for (int x = 0; x < kMaxWin; ++x) {
        vq[x] = v[x];
        c0[x] = row0[k + x];
        c1[x] = TWO ? row1[k + x] : 0.0;
      }
#pragma unroll
      for (int x = 0; x < kMaxWin; ++x) {
        a0[x & 3] += c0[x] * vq[x];
        if (TWO) a1[x & 3] += c1[x] * vq[x];
      }
    }
  }
}

__device__ __forceinline__ void matvec64(int n, int ncand, const int* desc, const double* vc,
                                         const MixedSmem& ms, double& out0, double& out1) {
  const int lane = threadIdx.x & 63;
  const double* row0 = ms.cc64 + conv_row(lane < n ? desc[lane] : 0);
  const double* row1 = ms.cc64 + conv_row(lane + 64 < n ? desc[lane + 64] : 0);
  // ncand = 2 W^2
  int W = 1;
  while (2 * W * W < ncand) ++W;
  double a0[4] = {0.0, 0.0, 0.0, 0.0}, a1[4] = {0.0, 0.0, 0.0, 0.0};
  if (n > 64)
    matvec64_rows<true>(W, row0, row1, vc, a0, a1);
  else
    matvec64_rows<false>(W, row0, row1, vc, a0, a1);
  out0 = lane < n ? (a0[0] + a0[1]) + (a0[2] + a0[3]) : 0.0;
  out1 = lane + 64 < n ? (a1[0] + a1[1]) + (a1[2] + a1[3]) : 0.0;
}

// The same over the class-indexed pair table of the leave-one-slice-out blocks.
template <typename MS>
__device__ __forceinline__ void matvec64(int n, int ncand, const int* desc, const double* vc,
                                         const MS& ms, double& out0, double& out1) {
  const int lane = threadIdx.x & 63;
  const auto row0 = ms.row(lane < n ? (desc[lane] & 0x7f) : 0);
  const auto row1 = ms.row(lane + 64 < n ? (desc[lane + 64] & 0x7f) : 0);
  double a0[4] = {0.0, 0.0, 0.0, 0.0}, a1[4] = {0.0, 0.0, 0.0, 0.0};
  int c = 0;
  for (; c + 4 <= ncand; c += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double vq = vc[c + u];
      a0[u] += ms.at(row0, c + u) * vq;
      a1[u] += ms.at(row1, c + u) * vq;
    }
  }
  for (; c < ncand; ++c) {
    const double vq = vc[c];
    a0[0] += ms.at(row0, c) * vq;
    a1[0] += ms.at(row1, c) * vq;
  }
  out0 = lane < n ? (a0[0] + a0[1]) + (a0[2] + a0[3]) : 0.0;
  out1 = lane + 64 < n ? (a1[0] + a1[1]) + (a1[2] + a1[3]) : 0.0;
}

// Returns whether the FP64 correction ran: it does when CORR is set and the
// pivot-ratio condition estimate exceeds refine_kappa; otherwise the estimate
// is the factorisation's Schur read-out in the normalised units.
template <int NB, int UPD, bool CORR, typename MS>
__device__ __forceinline__ bool mixed_system(int n, int nb, WaveScratch<float>& ws, const Smem<float>& sm,
                                             MixedScratch& mx, f32x4* xs, const MS& ms, int ncand,
                                             int ntgt, double sill, double refine_kappa,
                                             double* est_out, float* var_out, float& mn,
                                             float& mxp, bool& bad, double* w_out = nullptr,
                                             double* nu_scale = nullptr,
                                             double* readout_out = nullptr,
                                             double* bound_out = nullptr) {
  const int lane = threadIdx.x & 63;
  const int p0 = lane, p1 = lane + 64;
  // ---- 1. normalise the data ----
  const float zref = ws.val[0];
  const float a0 = p0 < n ? ws.val[p0] : zref;
  const float a1 = p1 < n ? ws.val[p1] : zref;
  const float spread = wave_max_abs(fmaxf(fabsf(a0 - zref), fabsf(a1 - zref)));
  const int ex = spread > 0.0f ? ilogbf(spread) + 1 : 0;   // s = 2^ex > spread
  const float inv_s = ldexpf(1.0f, -ex);
  if (p0 < n) {
    mx.zr[p0] = a0;
    ws.val[p0] = (a0 - zref) * inv_s;
  }
  if (p1 < n) {
    mx.zr[p1] = a1;
    ws.val[p1] = (a1 - zref) * inv_s;
  }
  __builtin_amdgcn_wave_barrier();
  // ---- 2. factorisation ----
  PairStore<UPD> Ls[NB][(NB + 1) / 2];
  mn = 3.0e38f;
  mxp = 0.0f;
  bad = false;
  factor_keep<NB, UPD, CORR>(n, nb, ws, sm, ncand, ws.buf, mn, mxp, bad, Ls, xs);
  const int ne = 16 - nb;
  float est_r = 0.0f;
  if (lane < ntgt) {
    float var_r;
    schur_readout<float>(ws.buf, ne, lane + 1, sm.bz - 1, ntgt + 1, 1.0f, est_r, var_r);
    *var_out = (float)(sill * (double)var_r);
    if (readout_out) *readout_out = (double)zref + ldexp((double)est_r, ex);
  }
  __builtin_amdgcn_wave_barrier();
  if (!CORR || !((double)mxp > refine_kappa * (double)mn)) {
    if (lane < ntgt) *est_out = (double)zref + ldexp((double)est_r, ex);
    if (nu_scale) *nu_scale = ldexp(1.0, ex);
    __builtin_amdgcn_wave_barrier();
    return false;
  }
  // ---- 3. explicit solutions x_1 = C^{-1} 1, x_z = C^{-1} z' (x_s = C^{-1} s) ----
  // Slots of x: 0 x_1, 1 x_z, 2.. the staged targets' x_t, kSlotXs x_s (in the area
  // of the diagonal tiles, which the back-substitution has finished reading).
  float (*const xrow)[128] = area_x(xs);
  double* const nuc = area_nuc(xs);
  __builtin_amdgcn_wave_barrier();
  f32x4 Z[NB];
  back_substitute<NB, UPD>(nb, Ls, xs, ws.buf, Z);
  const int dr = sm.bz - 1;   // 1 with the slice predictor (border rows 1, s, z, c0...)
  const int tcnt0 = ntgt < kRowTargets ? ntgt : kRowTargets;
  if (!dr) {
    write_rows<NB>(Z, ne, 2 + tcnt0, 0, xrow);
  } else {
    write_rows<NB>(Z, ne, 1, 0, xrow);
    write_rows<NB>(Z, ne + 1, 1, kSlotXs, xrow);
    write_rows<NB>(Z, ne + 2, 1 + tcnt0, 1, xrow);
  }
  const double x1_0 = p0 < n ? (double)xrow[0][p0] : 0.0, x1_1 = p1 < n ? (double)xrow[0][p1] : 0.0;
  const double xz_0 = p0 < n ? (double)xrow[1][p0] : 0.0, xz_1 = p1 < n ? (double)xrow[1][p1] : 0.0;
  const double xs_0 = (dr && p0 < n) ? (double)xrow[kSlotXs][p0] : 0.0;
  const double xs_1 = (dr && p1 < n) ? (double)xrow[kSlotXs][p1] : 0.0;
  const double sl_0 = (dr && p0 < n) ? (double)((ws.desc[p0] >> 14) & 1) : 0.0;
  const double sl_1 = (dr && p1 < n) ? (double)((ws.desc[p1] >> 14) & 1) : 0.0;
  // multipliers of the adjoint system: OK nu_mu = 1'x_z / 1'x_1; with the
  // slice predictor G (nu_1, nu_s) = (1'x_z, s'x_z), G = Q'C^-1 Q. These and
  // the multipliers of the targets below are sums of FP32 solution entries,
  // summed in FP32: the corrected estimate is exact for any approximate nu
  // (the residual absorbs it) and second order in the weights' error.
  float gf[5] = {(float)x1_0 + (float)x1_1, (float)xz_0 + (float)xz_1, (float)xs_0 + (float)xs_1,
                 (float)(sl_0 * xs_0) + (float)(sl_1 * xs_1), (float)(sl_0 * xz_0) + (float)(sl_1 * xz_1)};
  wave_sums_f(gf);
  const double g[5] = {(double)gf[0], (double)gf[1], (double)gf[2], (double)gf[3], (double)gf[4]};
  const double g11 = g[0], g1s = g[2], gss = g[3];
  const double det = g11 * gss - g1s * g1s;
  double nu_1, nu_s = 0.0;
  if (!dr) {
    nu_1 = g[1] / g11;
  } else {
    nu_1 = (gss * g[1] - g1s * g[4]) / det;
    nu_s = (g11 * g[4] - g1s * g[1]) / det;
  }
  const double nu0 = xz_0 - nu_1 * x1_0 - nu_s * xs_0, nu1 = xz_1 - nu_1 * x1_1 - nu_s * xs_1;
  nuc[lane] = 0.0;
  nuc[lane + 64] = 0.0;
  __builtin_amdgcn_wave_barrier();
  if (p0 < n) nuc[MS::vslot(ws.desc[p0])] = nu0;
  if (p1 < n) nuc[MS::vslot(ws.desc[p1])] = nu1;
  __builtin_amdgcn_wave_barrier();
  // ---- 4. FP64 correction ----
  // With h = z' - C nu_w - Q nu_phi (the FP64 residual of the adjoint system)
  // and w_t = x_t - x_Q phi_t, z'w_t + nu'(r_t - K lambda_t) equals
  //   A_t - phi_t'B + nu_phi'q0_t,  A_t = h'x_t + nu_w'c0_t,  B = x_Q'h + Q'nu_w
  // (OK: Q = 1, phi_t = mu_t; with the slice predictor Q = [1 s], q0_t = (1, t/f)).
  double cn0, cn1;
  matvec64(n, ncand, ws.desc, nuc, ms, cn0, cn1);
  const double zd = (double)zref;
  const double sd = ldexp(1.0, ex);
  const double isd = ldexp(1.0, -ex);
  const double h0 = p0 < n ? ((double)mx.zr[p0] - zd) * isd - cn0 - nu_1 - nu_s * sl_0 : 0.0;
  const double h1 = p1 < n ? ((double)mx.zr[p1] - zd) * isd - cn1 - nu_1 - nu_s * sl_1 : 0.0;
  const int d0 = p0 < n ? ws.desc[p0] : 0, d1 = p1 < n ? ws.desc[p1] : 0;
  double B1 = 0.0, Bs = 0.0;
  // For the error bound: |h_w|, |1'nu_w| and |s'nu_w| (the residual's border
  // components are -Q'nu_w).
  float hn = 0.0f, snu = 0.0f, ssnu = 0.0f;
  if (bound_out) {
    float nr[3] = {(float)(h0 * h0 + h1 * h1), (float)(nu0 + nu1), (float)(sl_0 * nu0 + sl_1 * nu1)};
    wave_sums_f(nr);
    hn = sqrtf(nr[0]);
    snu = fabsf(nr[1]);
    ssnu = fabsf(nr[2]);
  }
  for (int t0 = 1; t0 <= ntgt; t0 += kRowTargets) {
    const int cnt = (ntgt - t0 + 1) < kRowTargets ? (ntgt - t0 + 1) : kRowTargets;
    if (t0 > 1) write_rows<NB>(Z, ne + sm.bz + t0, cnt, 2, xrow);
    // sf: 1'x_t, s'x_t (FP32); sv: A_t, then B (FP64)
    float sf[2 * kRowTargets];
    double sv[kRowTargets + 2];
#pragma unroll
    for (int k = 0; k < kRowTargets; ++k) {
      sf[2 * k] = 0.0f;
      sf[2 * k + 1] = 0.0f;
      sv[k] = 0.0;
      if (k < cnt) {
        const int t = t0 + k;
        const float xf0 = p0 < n ? xrow[2 + k][p0] : 0.0f;
        const float xf1 = p1 < n ? xrow[2 + k][p1] : 0.0f;
        const double xt0 = (double)xf0, xt1 = (double)xf1;
        const double c00 = p0 < n ? ms.t064[(t - 1) * kT0Stride + (d0 >> 16)] : 0.0;
        const double c01 = p1 < n ? ms.t064[(t - 1) * kT0Stride + (d1 >> 16)] : 0.0;
        sf[2 * k] = xf0 + xf1;
        sv[k] = (h0 * xt0 + h1 * xt1) + (nu0 * c00 + nu1 * c01);
        sf[2 * k + 1] = (float)sl_0 * xf0 + (float)sl_1 * xf1;
      }
    }
    sv[kRowTargets] = t0 == 1 ? (h0 * x1_0 + h1 * x1_1) + (nu0 + nu1) : 0.0;
    sv[kRowTargets + 1] = (t0 == 1 && dr) ? (h0 * xs_0 + h1 * xs_1) + (sl_0 * nu0 + sl_1 * nu1)
                                          : 0.0;
    wave_sums_f(sf);
    wave_sums(sv);
    double s[3 * kRowTargets];
#pragma unroll
    for (int k = 0; k < kRowTargets; ++k) {
      s[3 * k] = (double)sf[2 * k];
      s[3 * k + 1] = sv[k];
      s[3 * k + 2] = (double)sf[2 * k + 1];
    }
    if (t0 == 1) {
      B1 = sv[kRowTargets];
      Bs = sv[kRowTargets + 1];
    }
    double p1k[kRowTargets], psk[kRowTargets];
#pragma unroll
    for (int k = 0; k < kRowTargets; ++k) {
      p1k[k] = 0.0;
      psk[k] = 0.0;
      if (k < cnt) {
        const int t = t0 + k;
        double p1c, psc = 0.0, corr;
        if (!dr) {
          p1c = (s[3 * k] - 1.0) / g11;
          corr = s[3 * k + 1] - p1c * B1 + nu_1;
        } else {
          const double qt = (double)t / (ntgt + 1);
          const double r1 = s[3 * k] - 1.0, r2 = s[3 * k + 2] - qt;
          p1c = (gss * r1 - g1s * r2) / det;
          psc = (g11 * r2 - g1s * r1) / det;
          corr = s[3 * k + 1] - p1c * B1 - psc * Bs + nu_1 + nu_s * qt;
        }
        if (lane == t - 1) *est_out = zd + sd * corr;
        if (w_out && t == 1) {
          if (p0 < n) w_out[p0] = (double)xrow[2][p0] - p1c * x1_0 - psc * xs_0;
          if (p1 < n) w_out[p1] = (double)xrow[2][p1] - p1c * x1_1 - psc * xs_1;
        }
        p1k[k] = p1c;
        psk[k] = psc;
      }
    }
    if (bound_out) {
      // The estimate above is exact up to (lambda - lambda~)'h, with lambda~ =
      // (w_t, phi_t) the computed weights and multipliers: bounded by
      // |w_t| |h_w| + |phi_t| |Q'nu_w| times their relative error, which the
      // caller supplies. Reported here without that factor, in data units.
      float ww[kRowTargets];
#pragma unroll
      for (int k = 0; k < kRowTargets; ++k) {
        ww[k] = 0.0f;
        if (k < cnt) {
          const float a0w = p0 < n ? (float)((double)xrow[2 + k][p0] - p1k[k] * x1_0 - psk[k] * xs_0) : 0.0f;
          const float a1w = p1 < n ? (float)((double)xrow[2 + k][p1] - p1k[k] * x1_1 - psk[k] * xs_1) : 0.0f;
          ww[k] = a0w * a0w + a1w * a1w;
        }
      }
      wave_sums_f(ww);
#pragma unroll
      for (int k = 0; k < kRowTargets; ++k) {
        if (k < cnt && lane == t0 + k - 1)
          *bound_out = sd * ((double)sqrtf(ww[k]) * (double)hn + fabs(p1k[k]) * (double)snu +
                             fabs(psk[k]) * (double)ssnu);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (nu_scale) *nu_scale = sd;
  __builtin_amdgcn_wave_barrier();
  return true;
}

}  // namespace
}  // namespace okr
