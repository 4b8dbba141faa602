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
//      hi*hi + hi*lo + lo*hi on 16x16x32 MFMAs with FP32 accumulation
//   2  split BF16: the same with bfloat16 halves
// The diagonal tiles, the off-diagonal solves and the back-substitution are
// FP32 in every case.
#pragma once

#include "solver_core.h"

namespace okr {
namespace {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b4 __attribute__((ext_vector_type(4)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mfma_k32(h8 a, h8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_k32(b8 a, b8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_k16(h4 a, h4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_k16(b4 a, b4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Storage of finished L tiles for the trailing updates: the tiles of block
// columns 2m and 2m+1 of one block row are kept together, already in the
// operand form of one K=32 MFMA (elements 0..3: column 2m, 4..7: column 2m+1).
template <int UPD> struct PairStore;

template <> struct PairStore<0> {
  f32x4 t[2];
  __device__ __forceinline__ void put(int h, const f32x4& x) { t[h] = x; }
  __device__ __forceinline__ f32x4 get(int h) const { return t[h]; }
};

template <typename E, typename V4, typename V8> struct SplitPair {
  V4 hi[2], lo[2];   // whole 4-element halves; concatenated at each use
  __device__ __forceinline__ void put(int h, const f32x4& x) {
    V4 vh, vl;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const E e = (E)x[v];
      vh[v] = e;
      vl[v] = (E)(x[v] - (float)e);
    }
    hi[h] = vh;
    lo[h] = vl;
  }
  __device__ __forceinline__ f32x4 get(int h) const {
    f32x4 x;
#pragma unroll
    for (int v = 0; v < 4; ++v) x[v] = (float)hi[h][v] + (float)lo[h][v];
    return x;
  }
  __device__ __forceinline__ V8 hi8() const {
    return __builtin_shufflevector(hi[0], hi[1], 0, 1, 2, 3, 4, 5, 6, 7);
  }
  __device__ __forceinline__ V8 lo8() const {
    return __builtin_shufflevector(lo[0], lo[1], 0, 1, 2, 3, 4, 5, 6, 7);
  }
};
template <> struct PairStore<1> : SplitPair<_Float16, h4, h8> {};
template <> struct PairStore<2> : SplitPair<__bf16, b4, b8> {};

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
// updates) keeping every L tile and every diagonal L^{-T} tile (Xs). Leaves
// the last diagonal tile (with G in its border corner) in buf.
template <int NB, int UPD>
__device__ __forceinline__ void factor_keep(int n, int nb, const WaveScratch<float>& ws,
                                            const Smem<float>& sm, int ncand, float* buf,
                                            float& minpiv, float& maxpiv, bool& bad,
                                            PairStore<UPD> (&Ls)[NB][(NB + 1) / 2],
                                            f32x4 (&Xs)[NB]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  constexpr int N = 16 * NB;
  const int bstart = N - nb;
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
    __builtin_amdgcn_sched_barrier(0);
    int cd[4];
    float cv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = 16 * j + 4 * g + v;
      cd[v] = q < n ? ws.desc[q] : (q < bstart ? -1 : -2 - (q - bstart));
      cv[v] = q < n ? ws.val[q] : 0.0f;
    }
    const bool colC = 16 * j + 16 <= n;
    f32x4 S[NB];
#pragma unroll
    for (int i = j; i < NB; ++i) {
      if (colC && 16 * i + 16 <= n) {
#pragma unroll
        for (int v = 0; v < 4; ++v) S[i][v] = -cov_pair<float>(rd[i], cd[v], sm, ncand);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool same = (i == j) && (r == 4 * g + v);
          S[i][v] = -entry<float>(rd[i], cd[v], rv[i], cv[v], same, sm, ncand);
        }
      }
    }
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
    diag_factor(D, X, ne, buf, minpiv, maxpiv, bad);
    Xs[j] = X;
    if (j < NB - 1) {
      const f32x4 NI = neg_transpose(X, buf);
#pragma unroll
      for (int i = j + 1; i < NB; ++i) {
        const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
        Ls[i][j / 2].put(j & 1, acc_qpt(z, S[i], NI));
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
// 1 + t: C^{-1} c0_t); write_row copies one of them to LDS.
template <int NB, int UPD>
__device__ __forceinline__ void back_substitute(int nb, const PairStore<UPD> (&Ls)[NB][(NB + 1) / 2],
                                                const f32x4 (&Xs)[NB], float* buf, f32x4 (&Z)[NB]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int ne = 16 - nb;
  {
    const f32x4 NI = neg_transpose(Xs[NB - 1], buf);
#pragma unroll
    for (int v = 0; v < 4; ++v) Z[NB - 1][v] = (r >= ne && 4 * g + v < ne) ? NI[v] : 0.0f;
  }
#pragma unroll
  for (int I = NB - 2; I >= 0; --I) {
    const f32x4 yl = Ls[NB - 1][I / 2].get(I & 1);
    f32x4 acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] = r >= ne ? yl[v] : 0.0f;
#pragma unroll
    for (int K = I + 1; K < NB; ++K) {
      const f32x4 P = neg_transpose(Ls[K][I / 2].get(I & 1), buf);
      acc = acc_qpt(acc, Z[K], P);
    }
    const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
    Z[I] = acc_qpt(z, acc, Xs[I]);
  }
}

template <int NB>
__device__ __forceinline__ void write_row(const f32x4 (&Z)[NB], int row, float* dst) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  if (r == row) {
#pragma unroll
    for (int I = 0; I < NB; ++I) {
#pragma unroll
      for (int v = 0; v < 4; ++v) dst[16 * I + 4 * g + v] = Z[I][v];
    }
  }
  __builtin_amdgcn_wave_barrier();
}

// ---- FP64 helpers (wave-wide) ----
__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// FP64 covariance of a pair from the pair-class table.
__device__ __forceinline__ double cov64(int dp, int dq, const double* tc64) {
  return tc64[pair_class(dp, dq)];
}

// (C v)_p for the lane's points p = lane, lane + 64 (FP64; C from the FP64
// class table; v in LDS).
__device__ __forceinline__ void matvec64(int n, const int* desc, const double* v, const double* tc64,
                                         double& out0, double& out1) {
  const int lane = threadIdx.x & 63;
  const int d0 = lane < n ? desc[lane] : 0;
  const int d1 = lane + 64 < n ? desc[lane + 64] : 0;
  double a0 = 0.0, a1 = 0.0;
  for (int q = 0; q < n; ++q) {
    const int dq = desc[q];
    const double vq = v[q];
    a0 += cov64(d0, dq, tc64) * vq;
    a1 += cov64(d1, dq, tc64) * vq;
  }
  out0 = lane < n ? a0 : 0.0;
  out1 = lane + 64 < n ? a1 : 0.0;
}

// One system with the FP64-corrected estimate (see kernels_mixed.hip).
struct MixedScratch {
  float xa[128];    // x_1
  float xb[128];    // x_z
  float xc[128];    // x_t (one target at a time)
  float zr[128];    // raw data values
  double nu[128];   // nu_w
};

struct MixedSmem {
  double tc64[kTcSize];
  double t064[kT0Size];
  MixedScratch ms[4];
};

__device__ __forceinline__ float wave_max_abs(float x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
  return x;
}

template <int NB, int UPD>
__device__ __forceinline__ void mixed_system(int n, int nb, WaveScratch<float>& ws, const Smem<float>& sm,
                                             MixedScratch& mx, const MixedSmem& ms, int ncand,
                                             int ntgt, double sill, double* est_out,
                                             float* var_out, float& mn, float& mxp, bool& bad,
                                             double* w_out = nullptr, double* nu_scale = nullptr) {
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
  f32x4 Xs[NB];
  mn = 3.0e38f;
  mxp = 0.0f;
  bad = false;
  factor_keep<NB, UPD>(n, nb, ws, sm, ncand, ws.buf, mn, mxp, bad, Ls, Xs);
  const int ne = 16 - nb;
  if (lane < ntgt) {
    const int t = lane + 1;
    const float g11 = ws.buf[ne * 17 + ne];
    const float g1t = ws.buf[(ne + 1 + t) * 17 + ne];
    const float gtt = ws.buf[(ne + 1 + t) * 17 + ne + 1 + t];
    const float m = (1.0f - g1t) / g11;
    *var_out = (float)(sill * (double)(1.0f - gtt + (1.0f - g1t) * m));
  }
  __builtin_amdgcn_wave_barrier();
  // ---- 3. explicit solutions ----
  f32x4 Z[NB];
  back_substitute<NB, UPD>(nb, Ls, Xs, ws.buf, Z);
  write_row<NB>(Z, ne, mx.xa);
  write_row<NB>(Z, ne + 1, mx.xb);
  const double x1_0 = p0 < n ? (double)mx.xa[p0] : 0.0, x1_1 = p1 < n ? (double)mx.xa[p1] : 0.0;
  const double xz_0 = p0 < n ? (double)mx.xb[p0] : 0.0, xz_1 = p1 < n ? (double)mx.xb[p1] : 0.0;
  const double g11 = wave_sum_d(x1_0 + x1_1);
  const double g1z = wave_sum_d(xz_0 + xz_1);
  const double nu_mu = g1z / g11;
  const double nu0 = xz_0 - nu_mu * x1_0, nu1 = xz_1 - nu_mu * x1_1;
  if (p0 < n) mx.nu[p0] = nu0;
  if (p1 < n) mx.nu[p1] = nu1;
  __builtin_amdgcn_wave_barrier();
  // ---- 4. FP64 correction ----
  double cn0, cn1;
  matvec64(n, ws.desc, mx.nu, ms.tc64, cn0, cn1);
  const double sum_nu = wave_sum_d(nu0 + nu1);
  const double zd = (double)zref;
  const double sd = ldexp(1.0, ex);
  const double isd = ldexp(1.0, -ex);
  const double zp0 = p0 < n ? ((double)mx.zr[p0] - zd) * isd : 0.0;
  const double zp1 = p1 < n ? ((double)mx.zr[p1] - zd) * isd : 0.0;
  const int d0 = p0 < n ? ws.desc[p0] : 0, d1 = p1 < n ? ws.desc[p1] : 0;
  for (int t = 1; t <= ntgt; ++t) {
    write_row<NB>(Z, ne + 1 + t, mx.xc);
    const double xc0 = p0 < n ? (double)mx.xc[p0] : 0.0, xc1 = p1 < n ? (double)mx.xc[p1] : 0.0;
    const double g1t = wave_sum_d(xc0 + xc1);
    const double mu = (g1t - 1.0) / g11;
    const double w0 = xc0 - mu * x1_0, w1 = xc1 - mu * x1_1;
    const double c00 = p0 < n ? ms.t064[(t - 1) * kT0Stride + (d0 >> 16)] : 0.0;
    const double c01 = p1 < n ? ms.t064[(t - 1) * kT0Stride + (d1 >> 16)] : 0.0;
    const double zw = wave_sum_d(zp0 * w0 + zp1 * w1);
    const double s_nc = wave_sum_d(nu0 * c00 + nu1 * c01);
    const double s_cw = wave_sum_d(cn0 * w0 + cn1 * w1);
    const double s_w = wave_sum_d(w0 + w1);
    const double delta = s_nc + nu_mu - s_cw - nu_mu * s_w - sum_nu * mu;
    if (lane == t - 1) *est_out = zd + sd * (zw + delta);
    if (w_out && t == 1) {
      if (p0 < n) w_out[p0] = w0;
      if (p1 < n) w_out[p1] = w1;
    }
  }
  if (nu_scale) *nu_scale = sd;
  __builtin_amdgcn_wave_barrier();
}

}  // namespace
}  // namespace okr
