// Device-side building blocks of the batched kriging solvers (included by the
// solver translation units; everything here is inlined into their kernels).
//
// See kernels_solve.hip for the method: the augmented matrix [[C, B], [B^T, 0]]
// of one (column, gap) system in 16x16 register tiles, left-looking Cholesky
// with MFMA updates, and the Schur read-out.
#pragma once

#include <cstddef>
#include <type_traits>

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

// 1/sqrt(x): the hardware reciprocal square root in FP32 (about 1 ulp, well
// inside the FP32 factorisation error). In FP64 the hardware estimate (relative
// error about 5e-8) takes one second-order Newton step in residual form,
// y = y0 + y0 e (1/2 + 3e/8) with e = 1 - x y0^2, which leaves about 1.3 ulp.
__device__ __forceinline__ float inv_sqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double inv_sqrt(double x) {
  const double y0 = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y0, y0, 1.0);
  return fma(y0 * e, fma(0.375, e, 0.5), y0);
}

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

constexpr int kChunk = 16;

template <typename T>
struct WaveScratch {
  int desc[128];      // point descriptors in system order
  float val[128];     // point values (0 past the last point)
  int ofs[128];       // FP32 assembly: pair-table offset | class-table offset << 16
  T buf[16 * 17];     // tile transposes and the read-out
};

// FP32 class-indexed rows (predictors, target covariances) hold the 32 pair
// classes and a zero at index 32, which columns that are not data points read.
constexpr int kT0StrideF = kT0Stride + 1;

// Covariance of two window points by their offset. The covariance depends only
// on the offset of the two points (translation invariance), so one table over
// every in-plane offset (-2R..2R per axis, R the largest radius), for each
// pair of slices, replaces a table over candidate pairs: 676 entries instead
// of 98 x 98. The entry of row point p and column point q sits at
// conv_row(p) + conv_col(q), layout [s_p][s_q][dy + 2R][dx + 2R] with
// (dy, dx) the offset of q from p.
constexpr int kConvHalf = 2 * kMaxRadius;
constexpr int kConvQ = 2 * kConvHalf + 1;
constexpr int kConvSub = kConvQ * kConvQ;
constexpr int kConvSize = 4 * kConvSub;

// From a candidate descriptor (bits 8..15: (s<<6)|((dy+r)<<3)|(dx+r)).
__device__ __forceinline__ int conv_row(int d) {
  const int c = (d >> 8) & 0xff;
  return (c >> 6) * (2 * kConvSub) + (kConvHalf - ((c >> 3) & 7)) * kConvQ + (kConvHalf - (c & 7));
}
__device__ __forceinline__ int conv_col(int d) {
  const int c = (d >> 8) & 0xff;
  return (c >> 6) * kConvSub + ((c >> 3) & 7) * kConvQ + (c & 7);
}
// Pair class ((ds<<6)|(|dy|<<3)|(|dx|)) of offset-table entry i.
__device__ __forceinline__ int conv_class(int i) {
  const int sr = i / (2 * kConvSub);
  const int rem = i - sr * (2 * kConvSub);
  const int sc = rem / kConvSub;
  const int k = rem - sc * kConvSub;
  const int dy = k / kConvQ - kConvHalf, dx = k % kConvQ - kConvHalf;
  return ((sr ^ sc) << 6) | ((dy < 0 ? -dy : dy) << 3) | (dx < 0 ? -dx : dx);
}

// Per-workgroup tables (each kernel declares its waves' WaveScratch beside
// them). Every covariance table holds NEGATED values (the factorisation works
// on S = -M), so an assembled entry needs no sign flip.
template <typename T> struct Smem {
  T tc[kTcSize];      // -Cov by pair class
  T t0[kT0Size];      // -c0 by (target, class)
  int sdesc[128];
  int bz;             // border row of the data values (1, or 2 with the slice predictor)
  uint8_t cls[kMaxCand * kMaxCand];   // pair class of every candidate pair
};
// FP32 blocks also keep the (negated) covariance of every candidate pair, so a
// matrix entry is a single LDS read.
template <> struct Smem<float> {
  float tc[kTcSize];
  float t0[kMaxUpsample * kT0StrideF];
  float bt[2 * kT0StrideF];  // class-indexed rows of the predictors: -1, -slice
  float zr[128];             // zeros: the row read by padding rows and the value row
  int sdesc[128];
  int bz;
  float cc[kConvSize];       // -Cov by offset (conv_row / conv_col)
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

// -Cov of two data points (FP64 path): the class table through the pair-class
// byte table (offsets from cc_row / cc_col). FP32 blocks assemble their
// entries with tile_f32 below.
template <typename T>
__device__ __forceinline__ T neg_cov_pair(int dp, int dq, int rbase, int col, const Smem<T>& sm);
template <>
__device__ __forceinline__ double neg_cov_pair<double>(int, int, int rbase, int col,
                                                       const Smem<double>& sm) {
  return sm.tc[sm.cls[rbase + col]];
}

// Offsets of a descriptor's row and column in the pair-class byte table (0
// for rows and columns that are not data points, which never read them).
template <typename T> __device__ __forceinline__ int cc_row(int d, int ncand) {
  return d >= 0 ? (d & 0x7f) * ncand : 0;
}
template <typename T> __device__ __forceinline__ int cc_col(int d) {
  return d >= 0 ? (d & 0x7f) : 0;
}

// ---- FP32 entries without branches ----
// Every row of the augmented matrix reads one LDS row of the block's tables:
// a data row its row of the pair table cc, a border row a class-indexed row
// (bt for the constant and slice predictors, t0 for the target covariances),
// padding rows and the data-value row the zero row zr. A column supplies an
// offset into either kind of row (ofs: candidate in the low half, pair class
// in the high half; columns past the last point select the zero of the class
// rows), and the value row adds the column's data value. Only the lower
// triangle is assembled this way; the factorisation never reads entries above
// the diagonal.
constexpr int kOffT0 = offsetof(Smem<float>, t0);
constexpr int kOffBt = offsetof(Smem<float>, bt);
constexpr int kOffZr = offsetof(Smem<float>, zr);
constexpr int kOffCc = offsetof(Smem<float>, cc);
constexpr int kTailOfs = (4 * kT0Stride) << 16;

// Column offsets of a candidate descriptor: its offset-table column (bytes)
// in the low half, its target-table class (bits 16..20, bytes) in the high half.
__device__ __forceinline__ int f32_ofs(int d) {
  return (conv_col(d) << 2) | (((d >> 16) & 31) << 18);
}

__device__ __forceinline__ float lds_at(const Smem<float>& sm, int off) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(&sm) + off);
}

// Row offsets of one system: rb[i] for the lane's row in block i; for the last
// block also the half of ofs the row uses (sh) and whether it is the value row.
template <int NB>
__device__ __forceinline__ void f32_rows(int n, int bstart, int bz, int ncand,
                                         const WaveScratch<float>& ws, int (&rb)[NB], int& sh,
                                         float& vrow) {
  const int r = threadIdx.x & 15;
#pragma unroll
  for (int i = 0; i < NB - 1; ++i) {   // data or padding (border rows are in the last block)
    const int p = 16 * i + r;
    rb[i] = p < n ? kOffCc + 4 * conv_row(ws.desc[p]) : kOffZr;
  }
  const int p = 16 * (NB - 1) + r;
  const int b = p - bstart;
  int o;
  if (p < n) o = kOffCc + 4 * conv_row(ws.desc[p]);
  else if (b < 0 || b == bz) o = kOffZr;
  else if (b == 0) o = kOffBt;
  else if (b < bz) o = kOffBt + 4 * kT0StrideF;
  else o = kOffT0 + (b - bz - 1) * 4 * kT0StrideF;
  rb[NB - 1] = o;
  sh = (b >= 0 && b != bz) ? 16 : 0;
  vrow = b == bz ? 1.0f : 0.0f;
}

// Tile (i, j) of -M in lane-row layout from the row offsets and the block
// column's offsets ofs and values cv (n data points, border from bstart).
template <int NB>
__device__ __forceinline__ f32x4 tile_f32(int i, int j, int n, int bstart, const int (&rb)[NB],
                                          int sh, float vrow, const int (&ofs)[4],
                                          const float (&cv)[4], const Smem<float>& sm) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  f32x4 t;
  if (i < NB - 1) {
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = lds_at(sm, rb[i] + (ofs[v] & 0xffff));
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v)
      t[v] = fmaf(vrow, -cv[v], lds_at(sm, rb[i] + (int)__builtin_amdgcn_ubfe(ofs[v], sh, 16)));
  }
  if (i == j && 16 * i + 16 > n) {
    const int p = 16 * i + r;
    const bool pad = p >= n && p < bstart;
#pragma unroll
    for (int v = 0; v < 4; ++v) t[v] = (pad && r == 4 * g + v) ? -1.0f : t[v];
  }
  return t;
}

// Entry -M[p][q] of the augmented matrix (FP64 path) from the two indices'
// descriptors:
//   >= 0: data point, -1: identity padding, <= -2: border row b = -2 - d.
// Border rows: b = 0 the constant predictor, 0 < b < bz the point's slice
// (0 lower, 1 upper; with the drift), b = bz the data values, b > bz the
// covariances with target b - bz.
template <typename T>
__device__ __forceinline__ T neg_entry(int dp, int dq, int rbase, int col, float vp, float vq,
                                       bool same, const Smem<T>& sm) {
  if (dp >= 0 && dq >= 0) return neg_cov_pair<T>(dp, dq, rbase, col, sm);
  if (dp == -1 || dq == -1) return same ? T(-1) : T(0);
  if (dp < -1 && dq < -1) return T(0);
  int b, d;
  float v;
  if (dp < -1) {
    b = -2 - dp; d = dq; v = vq;
  } else {
    b = -2 - dq; d = dp; v = vp;
  }
  const int bz = sm.bz;
  if (b == 0) return T(-1);
  if (b < bz) return T(-((d >> 14) & 1));
  if (b == bz) return T(-v);
  return sm.t0[(b - bz - 1) * kT0Stride + (d >> 16)];
}

// Estimate and variance of target t (1-based) from the Schur block G = B'C^-1 B
// left in buf (lower triangle, border rows from ne: 1, [slice], z, c0_1, ...).
// Ordinary kriging: nu = (G_1t - 1) / G_11. With the slice predictor the two
// Lagrange multipliers solve G_QQ nu = G_Qt - q0, q0 = (1, t/f). Then
//   z_hat = G_zt - G_zQ nu,  sigma^2 = sill - G_tt + G_tQ nu - nu' q0.
template <typename T>
__device__ __forceinline__ void schur_readout(const T* buf, int ne, int t, int drift, int f, T sill,
                                              T& est, T& var) {
  auto G = [&](int i, int j) { return buf[(ne + i) * 17 + ne + j]; };   // i >= j
  if (!drift) {
    const T g11 = G(0, 0), g1z = G(1, 0), g1t = G(1 + t, 0), gzt = G(1 + t, 1);
    const T gtt = G(1 + t, 1 + t);
    const T m = (T(1) - g1t) / g11;
    est = gzt + m * g1z;
    var = sill - gtt + (T(1) - g1t) * m;
  } else {
    const int it = 2 + t;
    const T a = G(0, 0), b = G(1, 0), c = G(1, 1);
    const T qt = T(t) / T(f);
    const T r1 = G(it, 0) - T(1), r2 = G(it, 1) - qt;
    const T det = a * c - b * b;
    const T n1 = (c * r1 - b * r2) / det, n2 = (a * r2 - b * r1) / det;
    est = G(it, 2) - G(2, 0) * n1 - G(2, 1) * n2;
    var = sill - G(it, it) + G(it, 0) * n1 + G(it, 1) * n2 - n1 - n2 * qt;
  }
}

// Cholesky of one diagonal tile over its first ne columns, in four panels of
// four columns. D is the negated tile (-A); on return its lower triangle holds
// the trailing Schur complement (negated) of the columns >= ne, and X holds
// L^{-T} in the lane-row layout (for ne < 16: the partial inverse of the
// eliminated columns applied to the rest). Inside a panel the columns are
// eliminated one by one on the vector ALUs; the rest of the tile then takes
// the panel's rank-4 update with one MFMA (and one more for X), instead of
// four rank-1 MFMAs. Entries above the diagonal are not kept up to date.
// The range of the pivots is recorded, and a pivot that is not positive (NaN
// included) is replaced by 1 and the system flagged; inputs are finite
// (checked at placement) and scaled, so a pivot cannot overflow.
//
// FP32 pivots are uniform values; positive finite floats order like their bit
// patterns, so the check and the running range run on the scalar unit.
// A pivot with bits b is accepted when b - 1 < 0x7f7fffff (0 < piv < +inf; NaN
// and -0 excluded), so the largest b - 1 seen (chkb) tells whether any failed.
__device__ __forceinline__ float take_pivot_bits(unsigned b, unsigned& minb, unsigned& maxb,
                                                 unsigned& chkb) {
  const unsigned m = b - 1u;
  chkb = m > chkb ? m : chkb;
  b = m < 0x7f7fffffu ? b : 0x3f800000u;   // 1.0f
  minb = b < minb ? b : minb;
  maxb = b > maxb ? b : maxb;
  // Settle the running values here, in scalar registers. Left free, the
  // compiler sinks these reductions to their single use after the last tile and
  // keeps every pivot live until then (spilled to VGPR lanes).
  asm volatile("" : "+s"(minb), "+s"(maxb), "+s"(chkb));
  return __uint_as_float(b);
}

// FP32 layout: the panel's four columns sit in one lane group (elements 0..3),
// so the in-panel work is lane-local and the MFMA operand (column k of the
// panel in lane group k) goes through LDS. With want_x false (the last tile
// of a read-out, whose L^{-T} nothing uses) X is left untouched.
__device__ __forceinline__ void diag_factor(f32x4& D, f32x4& X, int ne, float* buf, float& minpiv,
                                            float& maxpiv, bool& bad, bool want_x = true) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  // the range is uniform; say so, for the scalar-register pin in take_pivot_bits
  unsigned minb = __builtin_amdgcn_readfirstlane(__float_as_uint(minpiv));
  unsigned maxb = __builtin_amdgcn_readfirstlane(__float_as_uint(maxpiv));
  unsigned chkb = 0;
  if (want_x) {
#pragma unroll
    for (int v = 0; v < 4; ++v) X[v] = (r == 4 * g + v) ? 1.0f : 0.0f;
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    if (4 * p < ne) {
      const bool mine = (g == p);
      f32x4 P;
#pragma unroll
      for (int v0 = 0; v0 < 4; ++v0) {
        const int c = 4 * p + v0;
        if (c < ne) {
          // pivot -D[c][c]: the sign flip on the bits keeps the check on the scalar unit
          const unsigned nb = __builtin_amdgcn_readlane(__float_as_uint(D[v0]), 16 * p + c);
          const float piv = take_pivot_bits(nb ^ 0x80000000u, minb, maxb, chkb);
          const float is = inv_sqrt(piv);
          // column c of L in the panel's lanes, 0 elsewhere, so the in-panel
          // updates below leave the other lane groups' columns unchanged. Rows
          // r <= c hold no L entry: what they get only reaches entries above
          // the diagonal, and the MFMA operand masks them.
          const float l = mine ? -D[v0] * is : 0.0f;
          P[v0] = l;
          float xm = 0.0f;
          if (want_x) {
            X[v0] *= mine ? is : 1.0f;
            xm = mine ? X[v0] : 0.0f;
          }
#pragma unroll
          for (int v1 = v0 + 1; v1 < 4; ++v1) {
            const float s = lane_value(l, 16 * p + 4 * p + v1);   // L[c1][c]
            D[v1] += l * s;
            if (want_x) X[v1] -= xm * s;
          }
        } else {
          P[v0] = 0.0f;
        }
      }
      if (p < 3) {
        if (mine) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            buf[r * 4 + v] = P[v];
            if (want_x) buf[64 + r * 4 + v] = X[v];
          }
        }
        __builtin_amdgcn_wave_barrier();
        const float u = (r >= 4 * p + 4) ? buf[r * 4 + g] : 0.0f;   // L[r][4p+g]
        const float xw = want_x ? buf[64 + r * 4 + g] : 0.0f;        // X[r][4p+g]
        __builtin_amdgcn_wave_barrier();
        D = mfma4(u, u, D);
        if (want_x) X = mfma4(-u, xw, X);
      }
    }
  }
  minpiv = __uint_as_float(minb);
  maxpiv = __uint_as_float(maxb);
  bad = bad || chkb >= 0x7f7fffffu;
}

// FP64 pivots: the same on the high word (sign, exponent and 20 mantissa bits,
// enough for the pivot range); a pivot below 2^-1022 counts as non-positive.
__device__ __forceinline__ double take_pivot_hi(double piv, double& minpiv, double& maxpiv,
                                                bool& bad) {
  const long long b = __double_as_longlong(piv);
  const unsigned hi = (unsigned)(b >> 32);
  const bool ok = (hi - 1u) < 0x7fefffffu;   // 2^-1022 <= piv < +inf
  const double p = ok ? piv : 1.0;
  bad = bad || !ok;
  const unsigned ph = ok ? hi : 0x3ff00000u;
  const unsigned mn = (unsigned)(__double_as_longlong(minpiv) >> 32);
  const unsigned mx = (unsigned)(__double_as_longlong(maxpiv) >> 32);
  if (ph < mn) minpiv = p;
  if (ph > mx) maxpiv = p;
  return p;
}

// FP64 layout: the panel's columns 4p+k sit in element p of lane group k, which
// is already the MFMA operand layout. The panel (and the same columns of X) is
// copied through LDS so that every lane group holds all four columns of its
// row; the in-panel elimination then runs lane-locally (redundantly in the
// four groups) and each group takes its own column back.
__device__ __forceinline__ void diag_factor(f64x4& D, f64x4& X, int ne, double* buf, double& minpiv,
                                            double& maxpiv, bool& bad, bool = true) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) X[v] = (r == 4 * v + g) ? 1.0 : 0.0;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    if (4 * p < ne) {
      buf[r * 8 + g] = D[p];
      buf[r * 8 + 4 + g] = X[p];
      __builtin_amdgcn_wave_barrier();
      double dl[4], xl[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        dl[k] = buf[r * 8 + k];
        xl[k] = buf[r * 8 + 4 + k];
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int k0 = 0; k0 < 4; ++k0) {
        const int c = 4 * p + k0;
        if (c < ne) {
          const double piv = take_pivot_hi(-lane_value(dl[k0], c), minpiv, maxpiv, bad);
          const double is = inv_sqrt(piv);
          const double l = (r > c) ? -dl[k0] * is : 0.0;   // L[r][c]
          dl[k0] = l;
          xl[k0] *= is;
#pragma unroll
          for (int k1 = k0 + 1; k1 < 4; ++k1) {
            const double s = lane_value(l, 4 * p + k1);   // L[c1][c]
            dl[k1] += l * s;
            xl[k1] -= xl[k0] * s;
          }
        }
      }
      const double dg = g == 0 ? dl[0] : (g == 1 ? dl[1] : (g == 2 ? dl[2] : dl[3]));
      const double xg = g == 0 ? xl[0] : (g == 1 ? xl[1] : (g == 2 ? xl[2] : xl[3]));
      D[p] = dg;
      X[p] = xg;
      if (p < 3) {
        const double u = (4 * p + g < ne && r >= 4 * p + 4) ? dg : 0.0;
        D = mfma4(u, u, D);
        X = mfma4(-u, xg, X);
      }
    }
  }
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
  constexpr bool F32 = sizeof(T) == 4;
  // FP32: row offsets for tile_f32; FP64: descriptors, values and class-table
  // offsets for neg_entry
  int rd[NB], rb[NB];
  float rv[NB];
  int sh = 0;
  float vrow = 0.0f;
  if constexpr (F32) {
    f32_rows<NB>(n, bstart, sm.bz, ncand, ws, rb, sh, vrow);
  } else {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int p = 16 * i + r;
      rd[i] = p < n ? ws.desc[p] : (p < bstart ? -1 : -2 - (p - bstart));
      rv[i] = p < n ? ws.val[p] : 0.0f;
      rb[i] = cc_row<T>(rd[i], ncand);
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    // keep each column's loads and updates together: hoisting later columns'
    // table reads would hold them in registers for the whole factorisation
    __builtin_amdgcn_sched_barrier(0);
    // ---- assemble block column j (negated) ----
    int cd[4], cb[4], ofs[4];
    float cv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = 16 * j + colmap<T>(g, v);
      if constexpr (F32) {
        ofs[v] = ws.ofs[q];
        cv[v] = ws.val[q];
      } else {
        cd[v] = q < n ? ws.desc[q] : (q < bstart ? -1 : -2 - (q - bstart));
        cv[v] = q < n ? ws.val[q] : 0.0f;
        cb[v] = cc_col<T>(cd[v]);
      }
    }
    const bool colC = 16 * j + 16 <= n;
#pragma unroll
    for (int i = j; i < NB; ++i) {
      V t;
      if constexpr (F32) {
        t = tile_f32<NB>(i, j, n, bstart, rb, sh, vrow, ofs, cv, sm);
      } else if (colC && 16 * i + 16 <= n) {
#pragma unroll
        for (int v = 0; v < 4; ++v) t[v] = neg_cov_pair<T>(rd[i], cd[v], rb[i], cb[v], sm);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool same = (i == j) && (r == colmap<T>(g, v));
          t[v] = neg_entry<T>(rd[i], cd[v], rb[i], cb[v], rv[i], cv[v], same, sm);
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
    V D = L[tix(j, j)];
    diag_factor(D, X, ne, buf, minpiv, maxpiv, bad, j < NB - 1);
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
__device__ __forceinline__ void solve_system(int n, int nb, const WaveScratch<T>& ws, const Smem<T>& sm, int ncand,
                             T* buf, T sill, int ntgt, T* est, T* var, T& minpiv, T& maxpiv,
                             bool& bad) {
  minpiv = T(3.0e38);
  maxpiv = T(0);
  bad = false;
  factor_system<T, NB>(n, nb, ws, sm, ncand, buf, minpiv, maxpiv, bad);
  const int lane = threadIdx.x & 63;
  const int ne = 16 - nb;
  if (lane < ntgt) schur_readout<T>(buf, ne, lane + 1, sm.bz - 1, ntgt + 1, sill, *est, *var);
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
__device__ void init_block(const SolveArgs& a, Smem<T>& sm, double tscale) {
  const double* tcs = a.tab.tc_d;
  const double* t0s = a.tab.t0_d;
  for (int i = threadIdx.x; i < kTcSize; i += blockDim.x) sm.tc[i] = T(-(tcs[i] * tscale));
  if constexpr (sizeof(T) == 4) {
    // class-indexed rows with a trailing zero: the targets' covariances, the
    // constant predictor -1 and the slice predictor -s (s = 1 for the upper
    // slice, class indices 16..31)
    for (int i = threadIdx.x; i < kMaxUpsample * kT0StrideF; i += blockDim.x) {
      const int t = i / kT0StrideF, c = i - t * kT0StrideF;
      sm.t0[i] = c < kT0Stride ? (float)(-(t0s[t * kT0Stride + c] * tscale)) : 0.0f;
    }
    for (int i = threadIdx.x; i < 2 * kT0StrideF; i += blockDim.x) {
      const int c = i < kT0StrideF ? i : i - kT0StrideF;
      sm.bt[i] = c == kT0Stride ? 0.0f : ((i < kT0StrideF || c >= 16) ? -1.0f : 0.0f);
    }
    for (int i = threadIdx.x; i < 128; i += blockDim.x) sm.zr[i] = 0.0f;
  } else {
    for (int i = threadIdx.x; i < kT0Size; i += blockDim.x) sm.t0[i] = T(-(t0s[i] * tscale));
  }
  for (int i = threadIdx.x; i < 128; i += blockDim.x)
    sm.sdesc[i] = i < a.geo.ncand ? cand_desc(i, a.geo.r, a.geo.W, a.geo.W2) : 0;
  if (threadIdx.x == 0) sm.bz = 1 + a.geo.drift;
}

__device__ __forceinline__ void atomic_max_float(unsigned int* addr, float v) {
  if (v > 0.0f && isfinite(v)) atomicMax(addr, __float_as_uint(v));
}


// Metadata of up to kChunk systems (one per lane) and the one-system-ahead
// prefetch of neighbour values.
struct Pipe {
  unsigned int msys = 0;
  unsigned long long mlo = 0, mhi = 0;
  int mcnt = 0;
  float pv0 = 0.0f, pv1 = 0.0f;
  int pp0 = -1, pp1 = -1;
};

__device__ __forceinline__ void pipe_load(Pipe& q, const SolveArgs& a, const uint32_t* list,
                                          unsigned long long base, int nk) {
  const int lane = threadIdx.x & 63;
  if (lane < nk) {
    q.msys = list[base + lane];
    q.mlo = a.bits[2ull * q.msys];
    q.mhi = a.bits[2ull * q.msys + 1];
    q.mcnt = a.count[q.msys];
  }
}

__device__ __forceinline__ void pipe_prefetch(Pipe& q, const SolveArgs& a, int k, int d0, int d1,
                                              uint64_t below) {
  const int lane = threadIdx.x & 63;
  const Geometry& geo = a.geo;
  const unsigned plane = (unsigned)geo.plane, nx = (unsigned)geo.nx;
  const unsigned sys = __builtin_amdgcn_readlane(q.msys, k);
  const unsigned long long lo = lane_u64(q.mlo, k), hi = lane_u64(q.mhi, k);
  const unsigned gap = sys / plane;
  const unsigned pix = sys - gap * plane;
  const unsigned y = pix / nx, x = pix - y * nx;
  const int n0 = __popcll(lo);
  q.pp0 = ((lo >> lane) & 1ull) ? __popcll(lo & below) : -1;
  q.pp1 = (lane + 64 < geo.ncand && ((hi >> lane) & 1ull)) ? n0 + __popcll(hi & below) : -1;
  if (q.pp0 >= 0) {
    const int c = (d0 >> 8) & 0xff;
    q.pv0 = a.slices[(long long)(gap + ((c >> 6) & 1) * a.step) * geo.plane +
                     (long long)((int)y + ((c >> 3) & 7) - geo.r) * geo.nx +
                     ((int)x + (c & 7) - geo.r)];
  }
  if (q.pp1 >= 0) {
    const int c = (d1 >> 8) & 0xff;
    q.pv1 = a.slices[(long long)(gap + ((c >> 6) & 1) * a.step) * geo.plane +
                     (long long)((int)y + ((c >> 3) & 7) - geo.r) * geo.nx +
                     ((int)x + (c & 7) - geo.r)];
  }
}

// ---- chunk staging ----
// When a chunk's systems are consecutive columns of one row of one gap (the
// common case in the size-sorted order, whose buckets keep system order), the
// window rows of both slices they read are loaded once into LDS with
// contiguous row loads, each system's values are then read from there, and
// their estimates and variances are collected in LDS and written as one
// contiguous row segment per target plane when the chunk is done.
constexpr int kTileW = kChunk + 2 * kMaxRadius;
struct ChunkStage {
  float tile[2 * kMaxWin * kTileW];      // [slice][window row][column from x0 - r]
  float est[kMaxUpsample - 1][kChunk];   // [target][system of the chunk]
  float var[kMaxUpsample - 1][kChunk];
};

// Whether the chunk's nk systems (lane i holds system i) are one row run;
// if so, loads the tile (coordinates clamped to the image: out-of-image
// candidates are never kept, so those entries are never read) and returns the
// run's gap, row and first column.
__device__ __forceinline__ bool stage_chunk(const Pipe& q, const SolveArgs& a, int nk,
                                            ChunkStage& cs, unsigned& gap, unsigned& y,
                                            unsigned& x0) {
  const int lane = threadIdx.x & 63;
  const Geometry& geo = a.geo;
  const unsigned sys0 = __builtin_amdgcn_readfirstlane(q.msys);
  const unsigned plane = (unsigned)geo.plane, nx = (unsigned)geo.nx;
  gap = sys0 / plane;
  const unsigned pix = sys0 - gap * plane;
  y = pix / nx;
  x0 = pix - y * nx;
  const bool mine = lane >= nk || q.msys == sys0 + (unsigned)lane;
  if (!__all(mine) || x0 + (unsigned)nk > nx) return false;
  const int r = geo.r, W = geo.W, cols = nk + 2 * r, per = W * cols;
  for (int i = lane; i < 2 * per; i += 64) {
    const int sl = i >= per;
    const int rem = i - sl * per;
    const int row = rem / cols, c = rem - row * cols;
    int yy = (int)y + row - r, xx = (int)x0 + c - r;
    yy = yy < 0 ? 0 : (yy >= geo.ny ? geo.ny - 1 : yy);
    xx = xx < 0 ? 0 : (xx >= geo.nx ? geo.nx - 1 : xx);
    cs.tile[(sl * kMaxWin + row) * kTileW + c] =
        a.slices[(long long)(gap + sl * a.step) * geo.plane + (long long)yy * geo.nx + xx];
  }
  __builtin_amdgcn_wave_barrier();
  return true;
}

// pipe_prefetch of system k of a staged chunk: the values come from the tile.
__device__ __forceinline__ void pipe_prefetch_staged(Pipe& q, const ChunkStage& cs, int k, int d0,
                                                     int d1, uint64_t below, int ncand) {
  const int lane = threadIdx.x & 63;
  const unsigned long long lo = lane_u64(q.mlo, k), hi = lane_u64(q.mhi, k);
  const int n0 = __popcll(lo);
  q.pp0 = ((lo >> lane) & 1ull) ? __popcll(lo & below) : -1;
  q.pp1 = (lane + 64 < ncand && ((hi >> lane) & 1ull)) ? n0 + __popcll(hi & below) : -1;
  if (q.pp0 >= 0) {
    const int c = (d0 >> 8) & 0xff;
    q.pv0 = cs.tile[(((c >> 6) & 1) * kMaxWin + ((c >> 3) & 7)) * kTileW + k + (c & 7)];
  }
  if (q.pp1 >= 0) {
    const int c = (d1 >> 8) & 0xff;
    q.pv1 = cs.tile[(((c >> 6) & 1) * kMaxWin + ((c >> 3) & 7)) * kTileW + k + (c & 7)];
  }
}

// The staged chunk's outputs, one contiguous row segment per target plane.
__device__ __forceinline__ void flush_chunk(const SolveArgs& a, const ChunkStage& cs, int nk,
                                            unsigned gap, unsigned y, unsigned x0) {
  const int lane = threadIdx.x & 63;
  const Geometry& geo = a.geo;
  const int ntgt = geo.f - 1;
  __builtin_amdgcn_wave_barrier();
  for (int i = lane; i < ntgt * nk; i += 64) {
    const int t = i / nk, k = i - t * nk;
    const long long o = ((long long)gap * geo.f + t + 1) * geo.plane + (long long)y * geo.nx + x0 + k;
    a.volume[o] = cs.est[t][k];
    if (a.variance) a.variance[o] = cs.var[t][k];
  }
  __builtin_amdgcn_wave_barrier();
}

// Writes the system's points (n of them) in system order; the slots past the
// last point get value 0 and the column offsets of a non-point.
template <typename T>
__device__ __forceinline__ void pipe_commit(const Pipe& q, WaveScratch<T>& ws, int d0, int d1,
                                            int n) {
  const int lane = threadIdx.x & 63;
  if (q.pp0 >= 0) {
    ws.desc[q.pp0] = d0;
    ws.val[q.pp0] = q.pv0;
    ws.ofs[q.pp0] = f32_ofs(d0);
  }
  if (q.pp1 >= 0) {
    ws.desc[q.pp1] = d1;
    ws.val[q.pp1] = q.pv1;
    ws.ofs[q.pp1] = f32_ofs(d1);
  }
  if (lane >= n) {
    ws.val[lane] = 0.0f;
    ws.ofs[lane] = kTailOfs;
  }
  if (lane + 64 >= n) {
    ws.val[lane + 64] = 0.0f;
    ws.ofs[lane + 64] = kTailOfs;
  }
  __builtin_amdgcn_wave_barrier();
}

// Shared tables of a workgroup; covariances are multiplied by tscale (1, or
// 1/sill for the scaled mixed-precision systems).
template <typename T>
__device__ __forceinline__ void block_setup(const SolveArgs& a, Smem<T>& sm, double tscale = 1.0) {
  init_block<T>(a, sm, tscale);
  __syncthreads();
  if constexpr (sizeof(T) == 8) {
    const int nc = a.geo.ncand;
    for (int i = threadIdx.x; i < nc * nc; i += blockDim.x) {
      const int p = i / nc, q = i - p * nc;
      sm.cls[i] = (uint8_t)pair_class(sm.sdesc[p], sm.sdesc[q]);
    }
    __syncthreads();
  }
  if constexpr (sizeof(T) == 4) {
    // (negated) covariance of every offset, rounded once from the FP64 table
    for (int i = threadIdx.x; i < kConvSize; i += blockDim.x)
      sm.cc[i] = (float)(-(a.tab.tc_d[conv_class(i)] * tscale));
    __syncthreads();
  }
}


// Work ranges by XCD: workgroups are dispatched to the eight XCDs in turn, so
// the persistent workgroups of one XCD (blockIdx.x modulo the parts) take
// chunks from their own contiguous part of a size class's range first, and
// neighbouring columns are solved under one L2; a wave whose part is used up
// moves on to the next parts, so no XCD idles while another has work. Classes
// of fewer than 8 x 4096 systems (and grids of fewer than 8 workgroups) keep
// one part: there the spread of reads matters less than the extra claims.
// Used by the refined kernels, whose solve traffic it cuts by two thirds at
// the same speed; the FP32 and FP64 classes, faster per system, ran up to
// 11 % slower split and keep one part (split = false).
struct ClassRange {
  unsigned long long start, len;
  unsigned long long* cursors;   // one per part
  unsigned parts, home, visited;
};
__device__ __forceinline__ ClassRange class_range(const SolveArgs& a, int NB,
                                                  unsigned long long start,
                                                  unsigned long long end, bool split) {
  ClassRange r;
  r.parts = (split && gridDim.x >= 8u && end > start && end - start >= 8ull * 4096ull) ? 8u : 1u;
  r.home = blockIdx.x % r.parts;
  r.visited = 0;
  r.start = start;
  r.len = end > start ? end - start : 0ull;
  r.cursors = &a.ctr->cls_next[NB][0];
  return r;
}
// Claims the next chunk of up to kChunk systems: [base, base + nk). Uniform.
__device__ __forceinline__ bool next_chunk(ClassRange& r, unsigned long long& base, int& nk) {
  const int lane = threadIdx.x & 63;
  while (r.visited < r.parts) {
    const unsigned x = (r.home + r.visited) % r.parts;
    const unsigned long long lo = r.start + r.len * x / r.parts;
    const unsigned long long hi = r.start + r.len * (x + 1) / r.parts;
    unsigned long long b = 0;
    if (lane == 0) b = lo + atomicAdd(&r.cursors[x], (unsigned long long)kChunk);
    b = uniform64(b);
    if (b < hi) {
      base = b;
      nk = (int)((hi - b) < (unsigned long long)kChunk ? (hi - b) : kChunk);
      return true;
    }
    ++r.visited;
  }
  return false;
}

// Per-wave tallies of the finished systems, flushed to the counters once per
// wave (one atomic per wave instead of one per system).
struct Tally {
  float kmax = 0.0f;
  unsigned bad = 0, fp64 = 0, failed = 0, unconv = 0;
};

__device__ __forceinline__ void flush_tally(const SolveArgs& a, const Tally& t) {
  if ((threadIdx.x & 63) == 0) {
    if (t.bad) atomicAdd(&a.ctr->bad_pivot, (unsigned long long)t.bad);
    if (t.fp64) atomicAdd(&a.ctr->fp64_fallback, (unsigned long long)t.fp64);
    if (t.failed) atomicAdd(&a.ctr->failed, (unsigned long long)t.failed);
    if (t.unconv) atomicAdd(&a.ctr->unconverged, (unsigned long long)t.unconv);
    atomic_max_float(&a.ctr->max_kappa_bits, t.kmax);
  }
}

// Writes the estimates and variances of one system, or queues it for the
// FP64 pass; updates flags and the wave's tallies.
template <typename T>
__device__ __forceinline__ void finish_system(const SolveArgs& a, int mode, unsigned sys, int cnt,
                                              T est, T var, T mn, T mx, bool bad, Tally& tally,
                                              bool route = false, uint8_t extra_flags = 0,
                                              ChunkStage* cs = nullptr, int k = 0) {
  const int lane = threadIdx.x & 63;
  const Geometry& geo = a.geo;
  const int ntgt = geo.f - 1;
  const T kappa = mx / mn;
  const bool fallback =
      mode == 0 && a.fallback && (bad || route || (double)kappa > a.kappa_limit);
  const unsigned plane = (unsigned)geo.plane;
  const unsigned gap = sys / plane;
  const unsigned pix = sys - gap * plane;
  if (fallback) {
    if (lane == 0) {
      const unsigned long long slot = atomicAdd(&a.ctr->n_fallback_list, 1ull);
      a.fallback[slot] = sys;
    }
  } else if (lane < ntgt) {
    if (cs) {   // written with the rest of the staged chunk
      cs->est[lane][k] = (float)est;
      cs->var[lane][k] = (float)var;
    } else {
      const long long o = ((long long)gap * geo.f + lane + 1) * geo.plane + pix;
      a.volume[o] = (float)est;
      if (a.variance) a.variance[o] = (float)var;
    }
  }
  // re-solved in FP64: the re-solve pass, or an FP64 launch standing in for it
  const bool resolved = mode == 1 || a.as_resolve;
  if (lane == 0 && a.flags) {
    uint8_t fl = ((cnt & kFloorBit) ? kFlagFloor : 0) | extra_flags;
    if (resolved) fl |= kFlagFp64;
    if (resolved && bad) fl |= kFlagFailed;
    if (bad && !resolved) fl |= kFlagBadPivot;
    if (mode == 0) a.flags[sys] = fl;
    else a.flags[sys] |= fl;
  }
  if (bad && !resolved) tally.bad += 1;
  if (resolved) tally.fp64 += 1;
  if (resolved && bad) tally.failed += 1;
  const float kf = (float)kappa;
  if (kf > tally.kmax && isfinite(kf)) tally.kmax = kf;
}

}  // namespace
}  // namespace okr
