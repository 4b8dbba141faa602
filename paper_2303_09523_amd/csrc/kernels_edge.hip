// Edge post-pass on the reconstructed volume (Section 4.1.2, Algorithm 2;
// Appendix B), on every YZ image I_x(z, y) = V[z][y][x]:
//
//   edge_shear_kernel  FP64 shearlet coefficients of the eight orientations,
//                      M = max_k |SH_k| and theta = its first argmax; lanes
//                      run along x, so every tap is one coalesced load of 64
//                      images and the eight accumulators stay in registers.
//   edge_nms_kernel    edge = M >= tau and M not below its two neighbours
//                      along the rounded normal; writes the byte edge map and
//                      one bit per pixel into per-image bitmaps.
//   edge_trace_kernel  one wave per image: scans its bitmap (held in LDS when
//                      it fits) row by row for chain starts, follows each
//                      chain clockwise, and checks every full window of 16
//                      chain pixels; a noisy window is re-routed along the
//                      edge tangent and the three pixels on each side of every
//                      new edge pixel take their median.
//
// The coefficient sums are taken in the fixed tap order (d2 outer, d1 inner,
// each product rounded before it is added), so the coefficients, and with
// them every threshold and argmax decision, are reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "edge_filters.h"
#include "edge_internal.h"

namespace okr {
namespace {

using edge::kR;
using edge::kTaps;
using edge::kOrient;

constexpr int kShearRows = 4;   // output rows (z) per thread of the shearlet kernel
constexpr int kShearWaves = 4;  // waves per workgroup (consecutive y)
constexpr int kWindow = 16;     // chain pixels per window
constexpr int kMinChanges = 4;  // orientation changes that make a window noisy

#pragma clang fp contract(off)

// rounded edge normal (d1, d2) of orientation k
__device__ __forceinline__ int normal1(const EdgeArgs& a, int k) {
  return (int)((a.n1 >> (4 * k)) & 15u) - 1;
}
__device__ __forceinline__ int normal2(const EdgeArgs& a, int k) {
  return (int)((a.n2 >> (4 * k)) & 15u) - 1;
}

// clockwise neighbour offsets (d1, d2) of direction d in 0..7
__device__ __forceinline__ int cw_d1(int d) { return (int)((edge::kCwPack1 >> (2 * d)) & 3u) - 1; }
__device__ __forceinline__ int cw_d2(int d) { return (int)((edge::kCwPack2 >> (2 * d)) & 3u) - 1; }

// acc[k] += tap(k, I2, I1) * x for every orientation whose tap is nonzero.
// Zero taps are skipped: for finite inputs adding a signed zero to a sum that
// starts at +0 never changes it.
template <int I2, int I1, int K>
__device__ __forceinline__ void tap_k(double* acc, double x) {
  if constexpr (I2 >= 0 && I2 < kTaps) {
    constexpr double t = edge::kTapTable.v[K][I2][I1];
    if constexpr (t != 0.0) acc[K] = acc[K] + t * x;
  }
  if constexpr (K + 1 < kOrient) tap_k<I2, I1, K + 1>(acc, x);
}

// Pixel of input row RHO (output row J sees it at tap row RHO - J) and
// column I1, added to every output row of the thread.
template <int RHO, int I1, int J>
__device__ __forceinline__ void tap_j(double (&acc)[kShearRows][kOrient], double x) {
  tap_k<RHO - J, I1, 0>(acc[J], x);
  if constexpr (J + 1 < kShearRows) tap_j<RHO, I1, J + 1>(acc, x);
}

// Input rows in order, and within a row the columns in order: for each output
// row this visits its taps with d2 outer and d1 inner.
template <int RHO, int I1>
__device__ __forceinline__ void tap_rc(double (&acc)[kShearRows][kOrient], const float* vol,
                                       unsigned xs, const long long* rowoff,
                                       const long long* coloff) {
  // wave-uniform row pointer plus the lane's 32-bit byte offset
  const char* row = reinterpret_cast<const char*>(vol + (rowoff[RHO] + coloff[I1]));
  const double x = (double)*reinterpret_cast<const float*>(row + xs);
  tap_j<RHO, I1, 0>(acc, x);
  if constexpr (I1 + 1 < kTaps) {
    tap_rc<RHO, I1 + 1>(acc, vol, xs, rowoff, coloff);
  } else if constexpr (RHO + 1 < kShearRows + 2 * kR) {
    // Finish each row before the next: the sums are pinned here (otherwise
    // the compiler sinks all arithmetic below the bounds checks of the stores
    // and issues every row's loads first, holding all pixels of the thread in
    // registers at once).
#pragma unroll
    for (int j = 0; j < kShearRows; ++j)
#pragma unroll
      for (int k = 0; k < kOrient; ++k) asm volatile("" : "+v"(acc[j][k]));
    tap_rc<RHO + 1, 0>(acc, vol, xs, rowoff, coloff);
  }
}

__global__ __launch_bounds__(64 * kShearWaves) void edge_shear_kernel(EdgeArgs a) {
  const int lane = threadIdx.x & 63;
  const int x = blockIdx.x * 64 + lane;
  const int y = __builtin_amdgcn_readfirstlane(blockIdx.y * kShearWaves + (threadIdx.x >> 6));
  const int z0 = __builtin_amdgcn_readfirstlane(blockIdx.z * kShearRows);
  if (y >= a.ny) return;
  const long long nx = a.nx, plane = (long long)a.ny * a.nx;
  // byte offset of the lane's image; lanes past the edge load a valid pixel
  const unsigned xs = 4u * (unsigned)(x < a.nx ? x : a.nx - 1);
  // border replicated: clamped row and column offsets
  long long rowoff[kShearRows + 2 * kR], coloff[kTaps];
#pragma unroll
  for (int r = 0; r < kShearRows + 2 * kR; ++r) {
    int z = z0 - kR + r;
    z = z < 0 ? 0 : (z >= a.nz ? a.nz - 1 : z);
    rowoff[r] = (long long)z * plane;
  }
#pragma unroll
  for (int c = 0; c < kTaps; ++c) {
    int yy = y - kR + c;
    yy = yy < 0 ? 0 : (yy >= a.ny ? a.ny - 1 : yy);
    coloff[c] = (long long)yy * nx;
  }
  double acc[kShearRows][kOrient];
#pragma unroll
  for (int j = 0; j < kShearRows; ++j)
#pragma unroll
    for (int k = 0; k < kOrient; ++k) acc[j][k] = 0.0;
  tap_rc<0, 0>(acc, a.volume, xs, rowoff, coloff);
  if (x >= a.nx) return;
#pragma unroll
  for (int j = 0; j < kShearRows; ++j) {
    const int z = z0 + j;
    if (z >= a.nz) break;
    double m = fabs(acc[j][0]);
    int th = 0;
#pragma unroll
    for (int k = 1; k < kOrient; ++k) {
      const double v = fabs(acc[j][k]);
      if (v > m) {
        m = v;
        th = k;
      }
    }
    const long long i = (long long)z * plane + (long long)y * nx + x;
    a.mag[i] = m;
    a.theta[i] = (uint8_t)th;
    if (a.orient_out) a.orient_out[i] = (uint8_t)th;
  }
}

// One thread per (image x, padded row, bitmap word): 32 pixels of one row.
// Bitmap layout bits[(row * wr + word) * nx + x], padded row = z + 1, padded
// column bit = y + 1; the padding rows and bits stay zero, so the tracer needs
// no bounds checks.
__global__ __launch_bounds__(256) void edge_nms_kernel(EdgeArgs a) {
  const int x = blockIdx.y * 64 + (threadIdx.x & 63);
  const long long task = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (x >= a.nx || task >= (long long)(a.nz + 2) * a.wr) return;
  const int row = (int)(task / a.wr), w = (int)(task % a.wr);
  const long long nx = a.nx, plane = (long long)a.ny * a.nx;
  uint32_t word = 0;
  if (row >= 1 && row <= a.nz) {
    const int z = row - 1;
    for (int b = 0; b < 32; ++b) {
      const int y = w * 32 + b - 1;
      if (y < 0 || y >= a.ny) continue;
      const long long i = (long long)z * plane + (long long)y * nx + x;
      const double m = a.mag[i];
      bool e = m >= a.tau;
      if (e) {
        const int th = a.theta[i];
        const int n1 = normal1(a, th), n2 = normal2(a, th);
#pragma unroll
        for (int sgn = 1; sgn >= -1; sgn -= 2) {
          const int zz = z + sgn * n2, yy = y + sgn * n1;
          if (zz >= 0 && zz < a.nz && yy >= 0 && yy < a.ny &&
              a.mag[(long long)zz * plane + (long long)yy * nx + x] > m)
            e = false;
        }
      }
      if (e) word |= 1u << b;
      if (a.edge_out) a.edge_out[i] = e ? 1 : 0;
    }
  }
  a.bits[task * nx + x] = word;
}

// Bitmap of one image: in LDS, or in place in the global bitmaps.
template <bool kLds>
struct Bitmap {
  uint32_t* lds;
  uint32_t* g;   // bits + x
  long long nx;
  __device__ uint32_t word(long long i) const { return kLds ? lds[i] : g[i * nx]; }
  __device__ void clear(long long i, int b) const {
    if (kLds)
      atomicAnd(&lds[i], ~(1u << b));
    else
      atomicAnd(&g[i * nx], ~(1u << b));
  }
};

// Full windows wait in a queue in LDS (pixel index z * ny + y of each of
// their 16 pixels) and are checked kQueue at a time, one lane per window,
// with all orientation loads in flight together. Windows only read the
// orientations of the shearlet pass and change the output volume and maps,
// never the bitmap the chains follow, so checking them after the chains that
// produced them, in queue order, gives the same result as checking each as
// soon as it is complete.
constexpr int kQueue = 64;

struct WindowQueue {
  uint32_t pix[kQueue][kWindow];
  uint8_t th[kQueue][kWindow];
};

__device__ __forceinline__ float median3(float a, float b, float c) {
  // insertion sort with strict comparisons: equal values keep their order
  float t;
  if (b < a) { t = a; a = b; b = t; }
  if (c < b) {
    t = b; b = c; c = t;
    if (b < a) { t = a; a = b; b = t; }
  }
  return b;
}

// Steps 4 and 5 on noisy window q of the queue (one lane).
__device__ void reroute_window(const EdgeArgs& a, int x, const WindowQueue& wq, int q) {
  const long long nx = a.nx;
  const int H = a.nz, Wd = a.ny;
  const uint32_t* pix = wq.pix[q];
  const uint8_t* th = wq.th[q];
  // representative orientation: the most frequent, ties to the one seen first
  int best = -1, rep = 0;
  for (int i = 0; i < kWindow; ++i) {
    int c = 0;
    for (int j = 0; j < kWindow; ++j) c += th[j] == th[i];
    if (c > best) {
      best = c;
      rep = th[i];
    }
  }
  // edge tangent: the rounded normal turned by 90 degrees, pointing from the
  // window's first pixel toward its last
  int t1 = -normal2(a, rep), t2 = normal1(a, rep);
  const int z0 = (int)(pix[0] / (uint32_t)Wd), y0 = (int)(pix[0] % (uint32_t)Wd);
  const int zl = (int)(pix[kWindow - 1] / (uint32_t)Wd), yl = (int)(pix[kWindow - 1] % (uint32_t)Wd);
  if (t1 * (yl - y0) + t2 * (zl - z0) < 0) {
    t1 = -t1;
    t2 = -t2;
  }
  // the 3 neighbours on each side of the tangent (cross product t x d > 0,
  // then < 0), in clockwise order; the two sides are disjoint, so both
  // medians read values the other does not write
  int o1[6], o2[6], ns0 = 0, ns1 = 3;
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    const int d1 = cw_d1(d), d2 = cw_d2(d);
    const int cr = t1 * d2 - t2 * d1;
    if (cr > 0) {
      o1[ns0] = d1;
      o2[ns0] = d2;
      ++ns0;
    } else if (cr < 0) {
      o1[ns1] = d1;
      o2[ns1] = d2;
      ++ns1;
    }
  }
  int qz = z0, qy = y0;
  for (int m = 1; m < kWindow - 1; ++m) {
    const int pz = (int)(pix[m] / (uint32_t)Wd), py = (int)(pix[m] % (uint32_t)Wd);
    const long long ip = (long long)pix[m] * nx + x;
    const int nz_ = qz + t2, ny_ = qy + t1;
    if (th[m] == rep || nz_ < 0 || nz_ >= H || ny_ < 0 || ny_ >= Wd) {
      qz = pz;
      qy = py;
      if (a.orient_out) a.orient_out[ip] = (uint8_t)rep;
      continue;
    }
    const long long in = ((long long)nz_ * Wd + ny_) * nx + x;
    if (a.edge_out) {
      a.edge_out[ip] = 0;
      a.edge_out[in] = 1;
    }
    if (a.orient_out) a.orient_out[in] = (uint8_t)rep;
    qz = nz_;
    qy = ny_;
    long long idx[6];
    bool inside[2] = {true, true};
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int zz = nz_ + o2[j], yy = ny_ + o1[j];
      const bool ok = zz >= 0 && zz < H && yy >= 0 && yy < Wd;
      inside[j / 3] = inside[j / 3] && ok;
      idx[j] = ok ? ((long long)zz * Wd + yy) * nx + x : in;
    }
    float v[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) v[j] = a.out[idx[j]];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (!inside[side]) continue;
      const float med = median3(v[3 * side], v[3 * side + 1], v[3 * side + 2]);
#pragma unroll
      for (int j = 0; j < 3; ++j) a.out[idx[3 * side + j]] = med;
    }
  }
}

// Check the nq queued windows: lane w loads window w's orientations and
// counts their changes; noisy windows are then re-routed in queue order.
__device__ void flush_windows(const EdgeArgs& a, int x, int lane, WindowQueue& wq, int nq) {
  bool noisy = false;
  if (lane < nq) {
    int t[kWindow];
#pragma unroll
    for (int i = 0; i < kWindow; ++i) t[i] = a.theta[(long long)wq.pix[lane][i] * a.nx + x];
    int changes = 0;
#pragma unroll
    for (int i = 0; i < kWindow; ++i) {
      wq.th[lane][i] = (uint8_t)t[i];
      if (i > 0) changes += t[i] != t[i - 1];
    }
    noisy = changes >= kMinChanges;
  }
  unsigned long long mask = __ballot(noisy);
  __syncthreads();
  while (mask) {
    const int q = __ffsll((long long)mask) - 1;
    mask &= mask - 1;
    if (lane == 0) reroute_window(a, x, wq, q);
  }
  __syncthreads();
}

template <bool kLds>
__global__ __launch_bounds__(64) void edge_trace_kernel(EdgeArgs a) {
  extern __shared__ uint32_t lds_bits[];
  __shared__ WindowQueue wq;
  const int x = blockIdx.x, lane = threadIdx.x;
  const long long wr = a.wr, nwords = (long long)(a.nz + 2) * wr;
  const long long last_word = (long long)(a.nz + 1) * wr;   // end of padded row nz
  const Bitmap<kLds> bm{lds_bits, a.bits + x, a.nx};
  if (kLds) {
#pragma unroll 8
    for (long long i = lane; i < nwords; i += 64) lds_bits[i] = a.bits[i * a.nx + x];
    __syncthreads();
  }
  uint32_t wpix = 0;    // pixel (z * ny + y) of window slot `lane`
  int nq = 0;           // windows queued
  long long scan = wr;  // first word of padded row 1
  for (;;) {
    // next chain start: the first remaining edge pixel in row-major order
    long long wi = -1;
    uint32_t wv = 0;
    while (scan < last_word) {
      const long long i = scan + lane;
      const uint32_t v = i < last_word ? bm.word(i) : 0u;
      const unsigned long long bal = __ballot(v != 0u);
      if (bal) {
        const int l = __ffsll((long long)bal) - 1;
        wi = scan + l;
        wv = (uint32_t)__shfl((int)v, l);
        break;
      }
      scan += 64;
    }
    if (wi < 0) break;
    scan = wi;   // earlier bits of this word are already zero
    int row = (int)(wi / wr);
    int cb = (int)(wi % wr) * 32 + (__ffs((int)wv) - 1);
    if (lane == 0) bm.clear(wi, cb & 31);
    if (lane == 0) wpix = (uint32_t)(row - 1) * (uint32_t)a.ny + (uint32_t)(cb - 1);
    int slot = 1;
    int last = -1;
    for (;;) {
      // first remaining neighbour clockwise, starting three steps
      // counter-clockwise of the last move (east for the first move)
      const int start = last < 0 ? 0 : (last + 5) & 7;
      const int dir = (start + lane) & 7;
      bool av = false;
      if (lane < 8) {
        const int nr = row + cw_d2(dir), nc = cb + cw_d1(dir);
        av = (bm.word((long long)nr * wr + (nc >> 5)) >> (nc & 31)) & 1u;
      }
      const unsigned long long bal = __ballot(av);
      if (!bal) break;
      const int d = (start + __ffsll((long long)bal) - 1) & 7;
      row += cw_d2(d);
      cb += cw_d1(d);
      last = d;
      if (lane == 0) bm.clear((long long)row * wr + (cb >> 5), cb & 31);
      if (lane == slot) wpix = (uint32_t)(row - 1) * (uint32_t)a.ny + (uint32_t)(cb - 1);
      if (++slot == kWindow) {
        if (lane < kWindow) wq.pix[nq][lane] = wpix;
        slot = 0;
        if (++nq == kQueue) {
          __syncthreads();
          flush_windows(a, x, lane, wq, nq);
          nq = 0;
        }
      }
    }
  }
  if (nq > 0) {
    __syncthreads();
    flush_windows(a, x, lane, wq, nq);
  }
}

}  // namespace

int edge_words_per_row(int ny) { return (ny + 2 + 31) / 32; }

hipError_t launch_edge_shear(const EdgeArgs& a, hipStream_t s) {
  dim3 grid((a.nx + 63) / 64, (a.ny + kShearWaves - 1) / kShearWaves,
            (a.nz + kShearRows - 1) / kShearRows);
  hipLaunchKernelGGL(edge_shear_kernel, grid, dim3(64 * kShearWaves), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_edge_nms(const EdgeArgs& a, hipStream_t s) {
  const long long tasks = (long long)(a.nz + 2) * a.wr;
  dim3 grid((unsigned)((tasks + 3) / 4), (a.nx + 63) / 64);
  hipLaunchKernelGGL(edge_nms_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

bool launch_edge_trace(const EdgeArgs& a, int lds_limit, hipStream_t s, hipError_t* err) {
  // the bitmap of one image in LDS when it fits in 64 KB (and the device's
  // limit) beside the window queue, else traced in place in global memory
  const size_t bitmap = sizeof(uint32_t) * (size_t)(a.nz + 2) * (size_t)a.wr;
  const size_t cap = lds_limit < 65536 ? (size_t)lds_limit : 65536;
  const bool in_lds = bitmap + sizeof(WindowQueue) + 256 <= cap;
  if (in_lds)
    hipLaunchKernelGGL(edge_trace_kernel<true>, dim3(a.nx), dim3(64), bitmap, s, a);
  else
    hipLaunchKernelGGL(edge_trace_kernel<false>, dim3(a.nx), dim3(64), 0, s, a);
  *err = hipGetLastError();
  return in_lds;
}

}  // namespace okr
