// Tables, placement, neighbour selection and size bucketing.
//
//  * tables:  FP64 covariance tables (and their derivatives) indexed by offset
//             class, so the solver assembles each kriging system by table
//             lookups (Appendix A's extended covariance matrix and vector).
//  * place:   known slice s -> output plane z = s*f, variance 0 there
//             (Algorithm 1, step 3).
//  * select:  per (column, gap) the kept candidates of the (2r+1)^2 x 2 window
//             under the edge rule and the floor (Section 4.1.2), staged through
//             an LDS tile of both slices' edge masks.
//  * bucket:  counting sort of the systems by neighbour count, largest first.
#include "okrig_internal.h"
#include "variogram.h"

namespace okr {
namespace {

__global__ void tables_kernel(Vario v, int f, int r, TableSet t) {
  for (int i = threadIdx.x; i < kTcSize; i += blockDim.x) {
    int ds = i >> 6, ady = (i >> 3) & 7, adx = i & 7;
    double c = 0, dn = 0, dsl = 0, da = 0;
    if (ady <= 2 * r && adx <= 2 * r) {
      double dz = ds ? (double)f : 0.0;
      double h = sqrt((double)(adx * adx + ady * ady) + dz * dz);
      cov_and_grad(v, h, &c, &dn, &dsl, &da);
    }
    t.tc_d[i] = c;
    t.tc_f[i] = (float)c;
    t.dtc_d[i] = dn;
    t.dtc_d[kTcSize + i] = dsl;
    t.dtc_d[2 * kTcSize + i] = da;
  }
  for (int i = threadIdx.x; i < kT0Size; i += blockDim.x) {
    int tt = i / kT0Stride, rem = i % kT0Stride;
    int s = rem >> 4, ady = (rem >> 2) & 3, adx = rem & 3;
    double c = 0, dn = 0, dsl = 0, da = 0;
    if (tt < f - 1 && ady <= r && adx <= r) {
      int t1 = tt + 1;
      double dz = s ? (double)(f - t1) : (double)t1;
      double h = sqrt((double)(adx * adx + ady * ady) + dz * dz);
      cov_and_grad(v, h, &c, &dn, &dsl, &da);
    }
    t.t0_d[i] = c;
    t.t0_f[i] = (float)c;
    t.dt0_d[i] = dn;
    t.dt0_d[kT0Size + i] = dsl;
    t.dt0_d[2 * kT0Size + i] = da;
  }
}

__global__ void reset_kernel(DevCounters* c) {
  int i = threadIdx.x;
  for (int k = i; k < (kMaxBlocks + 1) * 8; k += blockDim.x) (&c->cls_next[0][0])[k] = 0;
  if (i < kHist) {
    c->hist[i] = 0;
    c->cursor[i] = 0;
    c->offsets[i] = 0;
  }
  if (i == 0) {
    c->next = 0;
    c->next2 = 0;
    c->floor_filled = 0;
    c->refined = 0;
    c->unconverged = 0;
    c->fp64_fallback = 0;
    c->bad_pivot = 0;
    c->failed = 0;
    c->max_kappa_bits = 0;
    c->zmax_bits = 0;
    c->nonfinite = 0;
    c->bad_input = 0;
    c->offsets[kHist] = 0;
    c->n_fallback_list = 0;
  }
}

__global__ void reset_cursors_kernel(DevCounters* c) {
  int i = threadIdx.x;
  for (int k = i; k < (kMaxBlocks + 1) * 8; k += blockDim.x) (&c->cls_next[0][0])[k] = 0;
  if (i == 0) {
    c->next = 0;
    c->next2 = 0;
  }
}

// Known slice s -> plane s*f of the volume; variance 0 there. Also latches
// non-finite inputs and records the largest |known voxel| (the floor of the
// per-voxel error measure of the mixed path's routing). Grid (x, slice); one
// flag and one maximum per block go to the counters.
__global__ __launch_bounds__(256) void place_kernel(const float* __restrict__ slices,
                                                    float* __restrict__ volume,
                                                    float* __restrict__ variance, long long plane,
                                                    int f, DevCounters* ctr) {
  __shared__ float wmax[4];
  __shared__ unsigned wbad[4];
  const long long s = blockIdx.y;
  const float* src = slices + s * plane;
  float* dst = volume + s * f * plane;
  float* dvar = variance ? variance + s * f * plane : nullptr;
  bool bad = false;
  float amax = 0.0f;
  for (long long p = blockIdx.x * 256ll + threadIdx.x; p < plane; p += (long long)gridDim.x * 256) {
    const float v = src[p];
    const bool fin = isfinite(v);
    bad |= !fin;
    amax = fin ? fmaxf(amax, fabsf(v)) : amax;
    dst[p] = v;
    if (dvar) dvar[p] = 0.0f;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
  const bool wb = __any(bad);
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    wmax[wid] = amax;
    wbad[wid] = wb ? 1u : 0u;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const float m = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
    if (wbad[0] | wbad[1] | wbad[2] | wbad[3]) atomicOr(&ctr->nonfinite, 1u);
    if (m > 0.0f) atomicMax(&ctr->zmax_bits, __float_as_uint(m));
  }
}

constexpr int kSelTile = 16;

// One thread per (column, gap). Systems of gap g use slices g (lower) and
// g + step (upper).
__global__ __launch_bounds__(256) void select_kernel(const uint8_t* __restrict__ edge, Geometry geo,
                                                     int step, SelectRule rule,
                                                     uint64_t* __restrict__ bits,
                                                     uint8_t* __restrict__ count,
                                                     DevCounters* __restrict__ ctr) {
  constexpr int TW = kSelTile + 2 * kMaxRadius;
  __shared__ uint8_t tile[2][TW][TW + 1];
  __shared__ unsigned int lhist[kHist];
  __shared__ unsigned int lfloor;
  const int r = geo.r, W = geo.W, W2 = geo.W2;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kSelTile + tx;
  const int x0 = blockIdx.x * kSelTile, y0 = blockIdx.y * kSelTile, gap = blockIdx.z;
  const int tw = kSelTile + 2 * r;
  for (int i = tid; i < kHist; i += 256) lhist[i] = 0;
  if (tid == 0) lfloor = 0;
  // stage both slices' masks (tile + halo), zero outside the image
  for (int i = tid; i < 2 * tw * tw; i += 256) {
    int s = i / (tw * tw), rem = i - s * tw * tw;
    int a = rem / tw, b = rem - a * tw;
    int yy = y0 - r + a, xx = x0 - r + b;
    uint8_t e = 0;
    if (edge && yy >= 0 && yy < geo.ny && xx >= 0 && xx < geo.nx)
      e = edge[(long long)(gap + s * step) * geo.plane + (long long)yy * geo.nx + xx] != 0;
    tile[s][a][b] = e;
  }
  __syncthreads();
  const int x = x0 + tx, y = y0 + ty;
  if (x < geo.nx && y < geo.ny) {
    uint64_t e0 = 0, e1 = 0, inimg = 0;
    for (int a = 0; a < W; ++a) {
      for (int b = 0; b < W; ++b) {
        const int cell = a * W + b;
        const int yy = y + a - r, xx = x + b - r;
        if (yy >= 0 && yy < geo.ny && xx >= 0 && xx < geo.nx) inimg |= 1ull << cell;
        e0 |= (uint64_t)tile[0][ty + a][tx + b] << cell;
        e1 |= (uint64_t)tile[1][ty + a][tx + b] << cell;
      }
    }
    const int centre = r * W + r;
    uint64_t k0 = 0, k1 = 0;
    for (int o = 0; o < W2; ++o) {
      if (!((inimg >> o) & 1)) continue;
      const uint64_t bit = 1ull << o;
      if (o == centre) {
        k0 |= bit;
        k1 |= bit;
        continue;
      }
      const uint64_t p = rule.path[o];
      if (!(e0 & p)) k0 |= bit;
      if (!(e1 & p)) k1 |= bit;
    }
    int n = __popcll(k0) + __popcll(k1);
    bool floored = false;
    if (n < geo.min_points) {
      for (int i = 0; i < geo.ncand && n < geo.min_points; ++i) {
        const int c = rule.floor_order[i];
        const int s = c >= W2;
        const int o = c - s * W2;
        const uint64_t bit = 1ull << o;
        if (!(inimg & bit)) continue;
        if (s) {
          if (k1 & bit) continue;
          k1 |= bit;
        } else {
          if (k0 & bit) continue;
          k0 |= bit;
        }
        ++n;
        floored = true;
      }
    }
    const uint64_t lo = k0 | (k1 << W2);
    const uint64_t hi = (W2 < 64) ? (k1 >> (64 - W2)) : 0;
    const long long sys = (long long)gap * geo.plane + (long long)y * geo.nx + x;
    bits[2 * sys] = lo;
    bits[2 * sys + 1] = hi;
    count[sys] = (uint8_t)(n | (floored ? kFloorBit : 0));
    atomicAdd(&lhist[n], 1u);
    if (floored) atomicAdd(&lfloor, 1u);
  }
  __syncthreads();
  for (int i = tid; i < kHist; i += 256)
    if (lhist[i]) atomicAdd(&ctr->hist[i], (unsigned long long)lhist[i]);
  if (tid == 0 && lfloor) atomicAdd(&ctr->floor_filled, (unsigned long long)lfloor);
}

// Bucket starts, largest n first (longest-processing-time order).
__global__ void scan_kernel(DevCounters* ctr) {
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int n = kHist - 1; n >= 0; --n) {
      ctr->offsets[n] = run;
      ctr->cursor[n] = 0;
      run += ctr->hist[n];
    }
    ctr->offsets[kHist] = run;
  }
}

// Each block ranks kScatterPer x 256 systems in an LDS histogram, claims its
// range of every bucket with one global atomic per bucket, and writes the
// systems' slots of the size-sorted permutation. Systems are bucketed by the
// key of their neighbour count: every count of one size class shares the
// class's bucket (the full window keeps its own), so within a class the
// systems keep the order of their columns and neighbouring columns are solved
// close together in time.
constexpr int kScatterPer = 16;

struct BucketKeys {
  uint8_t key[kHist];   // bucket of neighbour count n: the largest n of its class
};

__global__ __launch_bounds__(256) void scatter_kernel(const uint8_t* __restrict__ count,
                                                      long long nsys, uint32_t* __restrict__ perm,
                                                      DevCounters* __restrict__ ctr,
                                                      BucketKeys keys) {
  __shared__ unsigned int lh[kHist];
  __shared__ unsigned long long base[kHist];
  const int tid = threadIdx.x;
  for (int i = tid; i < kHist; i += 256) lh[i] = 0;
  __syncthreads();
  const long long b0 = blockIdx.x * (256ll * kScatterPer) + tid;
  int nn[kScatterPer];
  unsigned int rank[kScatterPer];
#pragma unroll
  for (int k = 0; k < kScatterPer; ++k) {
    const long long sys = b0 + 256ll * k;
    nn[k] = 0;
    rank[k] = 0;
    if (sys < nsys) {
      nn[k] = keys.key[count[sys] & 0x7f];
      rank[k] = atomicAdd(&lh[nn[k]], 1u);
    }
  }
  __syncthreads();
  for (int i = tid; i < kHist; i += 256)
    if (lh[i]) base[i] = ctr->offsets[i] + atomicAdd(&ctr->cursor[i], (unsigned long long)lh[i]);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScatterPer; ++k) {
    const long long sys = b0 + 256ll * k;
    if (sys < nsys) perm[base[nn[k]] + rank[k]] = (uint32_t)sys;
  }
}

}  // namespace

hipError_t launch_tables(const Vario& v, const Geometry& g, TableSet t, hipStream_t s) {
  hipLaunchKernelGGL(tables_kernel, dim3(1), dim3(256), 0, s, v, g.f, g.r, t);
  return hipGetLastError();
}

// Device-detected status of the last execute on these counters, as an
// okr_status value: non-finite input, then (strict) an FP64 re-solve that met a
// non-positive pivot.
__global__ void status_kernel(const DevCounters* c, int strict, int32_t* out) {
  if (threadIdx.x == 0) *out = c->nonfinite ? 3 : ((strict && c->failed) ? 7 : 0);
}

hipError_t launch_status(const DevCounters* c, int strict, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(status_kernel, dim3(1), dim3(64), 0, s, c, strict, out);
  return hipGetLastError();
}

hipError_t launch_reset(DevCounters* c, hipStream_t s) {
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(kHist), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_reset_cursors(DevCounters* c, hipStream_t s) {
  hipLaunchKernelGGL(reset_cursors_kernel, dim3(1), dim3(64), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_place(const float* slices, float* volume, float* variance, const Geometry& g,
                        DevCounters* c, hipStream_t s) {
  if (g.nslices < 1 || g.plane < 1) return hipSuccess;
  // about 2048 blocks in all, at most one thread per voxel of a plane
  long long gx = (g.plane + 255) / 256;
  const long long want = (2048 + g.nslices - 1) / g.nslices;
  if (gx > want) gx = want;
  if (gx < 1) gx = 1;
  hipLaunchKernelGGL(place_kernel, dim3((unsigned)gx, (unsigned)g.nslices), dim3(256), 0, s, slices,
                     volume, variance, g.plane, g.f, c);
  return hipGetLastError();
}

hipError_t launch_select_step(const uint8_t* edge, const Geometry& g, int step, int ngaps,
                              const SelectRule& rule, uint64_t* bits, uint8_t* count,
                              DevCounters* c, hipStream_t s) {
  dim3 grid((g.nx + kSelTile - 1) / kSelTile, (g.ny + kSelTile - 1) / kSelTile, ngaps);
  hipLaunchKernelGGL(select_kernel, grid, dim3(kSelTile, kSelTile), 0, s, edge, g, step, rule,
                     bits, count, c);
  return hipGetLastError();
}

hipError_t launch_select(const uint8_t* edge, const Geometry& g, const SelectRule& rule,
                         uint64_t* bits, uint8_t* count, DevCounters* c, hipStream_t s) {
  return launch_select_step(edge, g, 1, g.nslices - 1, rule, bits, count, c, s);
}

hipError_t launch_bucket(const uint8_t* count, const Geometry& g, int nb, uint32_t* perm,
                         DevCounters* c,
                         hipStream_t s) {
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(64), 0, s, c);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (g.nsys < 1) return hipSuccess;
  const long long per = 256ll * kScatterPer;
  const long long blocks = (g.nsys + per - 1) / per;
  // the size classes of the solve kernels: 16 (NB - 1) - nb < n <= 16 NB - nb
  BucketKeys keys;
  for (int n = 0; n < kHist; ++n) {
    const int NB = (n + nb + 15) / 16;
    int hi = 16 * NB - nb;
    if (hi > kHist - 1) hi = kHist - 1;
    if (n < g.ncand && hi >= g.ncand) hi = g.ncand - 1;
    keys.key[n] = (uint8_t)(n == g.ncand ? n : hi);
  }
  hipLaunchKernelGGL(scatter_kernel, dim3((unsigned)blocks), dim3(256), 0, s, count, g.nsys, perm,
                     c, keys);
  return hipGetLastError();
}

}  // namespace okr
