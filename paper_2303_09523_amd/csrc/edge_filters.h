// Discrete shearlet filters of the edge post-pass (Appendix B), evaluated at
// compile time so that every tap is a constant of the kernel and zero taps
// cost nothing.
//
// System: psi_{a,s,t}(x) = a^{-3/4} psi(A_a^{-1} S_s^{-1} (x - t)) with
// A_a = diag(a, sqrt a), S_s = [[1, -s], [0, 1]], at the single scale a = 1/4
// (a^{-3/4} = 2 sqrt 2, 1/a = 4, 1/sqrt a = 2). The mother shearlet is
// separable, psi(u1, u2) = psi1(u1) phi(u2), with the compactly supported
// odd wavelet psi1(u) = -u (1 - (u/10)^2)^2 and window
// phi(u) = (1 - (u/10)^2)^2 on |u| < 10 (zero elsewhere). Taps are sampled at
// integer offsets |d1|, |d2| <= 4 of the image axes x1 = y (columns) and
// x2 = z (rows). Eight orientations: the horizontal cone
// psi1(4 (d1 + s d2)) phi(2 d2), s = -1, -1/2, 0, 1/2, then the vertical cone
// psi1(4 (d2 + s d1)) phi(2 d1), s = 1, 1/2, 0, -1/2; their edge normals lie
// at -45, -26.6, 0, 26.6, 45, 63.4, 90 and 116.6 degrees from x1 toward x2.
//
// Each tap is a short chain of correctly rounded operations on exact binary
// fractions (the division by 10 rounds once), written below in one fixed
// order and evaluated by the compiler's constant evaluator, which rounds
// every operation separately.
#pragma once

namespace okr {
namespace edge {

constexpr int kR = 4;               // taps at |d| <= kR
constexpr int kTaps = 2 * kR + 1;   // 9 x 9
constexpr int kOrient = 8;
constexpr double kSupport = 10.0;
// sqrt(2) rounded to the nearest double (the library checks it against
// the host's sqrt when it first runs the pass)
constexpr double kSqrt2 = 0x1.6a09e667f3bcdp+0;

struct Shear {
  int cone;   // 0: horizontal, 1: vertical
  double s;   // shear
};
constexpr Shear kShears[kOrient] = {{0, -1.0}, {0, -0.5}, {0, 0.0}, {0, 0.5},
                                    {1, 1.0},  {1, 0.5},  {1, 0.0}, {1, -0.5}};

constexpr double psi1(double u) {
  if (u <= -kSupport || u >= kSupport) return 0.0;
  const double q = 1.0 - (u / kSupport) * (u / kSupport);
  return -u * (q * q);
}

constexpr double phi(double u) {
  if (u <= -kSupport || u >= kSupport) return 0.0;
  const double q = 1.0 - (u / kSupport) * (u / kSupport);
  return q * q;
}

constexpr double tap(int k, int i2, int i1) {
  const double d1 = i1 - kR, d2 = i2 - kR;
  double u = 0.0, v = 0.0;
  if (kShears[k].cone == 0) {
    u = d1 + kShears[k].s * d2;
    v = d2;
  } else {
    u = d2 + kShears[k].s * d1;
    v = d1;
  }
  return (2.0 * kSqrt2) * (psi1(u * 4.0) * phi(v * 2.0));
}

struct TapTable {
  double v[kOrient][kTaps][kTaps];   // [k][d2 + kR][d1 + kR]
};

constexpr TapTable make_taps() {
  TapTable t{};
  for (int k = 0; k < kOrient; ++k)
    for (int i2 = 0; i2 < kTaps; ++i2)
      for (int i1 = 0; i1 < kTaps; ++i1) t.v[k][i2][i1] = tap(k, i2, i1);
  return t;
}

constexpr TapTable kTapTable = make_taps();

// Clockwise neighbour order with x1 = y to the right and x2 = z downward:
// E, SE, S, SW, W, NW, N, NE, as (d1, d2) = (column, row) offsets.
constexpr int kCwD1[8] = {1, 1, 0, -1, -1, -1, 0, 1};
constexpr int kCwD2[8] = {0, 1, 1, 1, 0, -1, -1, -1};

// The same offsets packed two bits per direction (offset + 1), so device code
// can look them up in a register instead of a table in memory.
constexpr unsigned pack_offsets(const int (&d)[8]) {
  unsigned v = 0;
  for (int i = 0; i < 8; ++i) v |= (unsigned)(d[i] + 1) << (2 * i);
  return v;
}
constexpr unsigned kCwPack1 = pack_offsets(kCwD1);
constexpr unsigned kCwPack2 = pack_offsets(kCwD2);

}  // namespace edge
}  // namespace okr
