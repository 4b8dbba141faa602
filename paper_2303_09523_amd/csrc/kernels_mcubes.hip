// Marching cubes on a float32 volume [nz][ny][nx] (Appendix C): the case
// table (mcubes_table.cpp) gives each corner configuration's triangles as
// cube-edge triples; crossing points are interpolated on their edges.
//
// HBM-bound. Three launches: count (triangles per workgroup), scan (one
// workgroup turns the counts into output offsets) and emit (recounts, ranks
// the cubes of the workgroup in index order and writes the triangles). A
// workgroup takes a run of up to kMcRun cubes of one (z, y) row, four per
// thread, so its eight corner loads per cube are four coalesced row reads,
// and the output keeps the cube order without storing per-cube counts.
#include "okrig_internal.h"

namespace okr {
namespace {

constexpr int kMcThreads = 256;
constexpr int kMcPer = kMcRun / kMcThreads;

struct McRow {
  const float* r00;   // (z, y)
  const float* r01;   // (z, y + 1)
  const float* r10;   // (z + 1, y)
  const float* r11;   // (z + 1, y + 1)
  int z, y, x0;
};

__device__ __forceinline__ McRow mc_row(const float* vol, int nx, int ny, int nseg) {
  const long long b = blockIdx.x;
  const long long row = b / nseg;
  McRow m;
  m.x0 = (int)(b - row * nseg) * kMcRun;
  m.z = (int)(row / (ny - 1));
  m.y = (int)(row - (long long)m.z * (ny - 1));
  const long long plane = (long long)nx * ny;
  m.r00 = vol + m.z * plane + (long long)m.y * nx;
  m.r01 = m.r00 + nx;
  m.r10 = m.r00 + plane;
  m.r11 = m.r10 + nx;
  return m;
}

// Corner values (c = x + 2y + 4z) of the cube at x and its configuration
// (bit c set when corner c is inside: value >= iso; NaN is outside).
__device__ __forceinline__ int mc_config(const McRow& m, int x, float iso, float (&v)[8]) {
  v[0] = m.r00[x];
  v[1] = m.r00[x + 1];
  v[2] = m.r01[x];
  v[3] = m.r01[x + 1];
  v[4] = m.r10[x];
  v[5] = m.r10[x + 1];
  v[6] = m.r11[x];
  v[7] = m.r11[x + 1];
  int cfg = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) cfg |= (v[c] >= iso) ? (1 << c) : 0;
  return cfg;
}

__device__ __forceinline__ unsigned block_sum(unsigned x, unsigned* red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wid] = x;
  __syncthreads();
  const unsigned s = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return s;
}

__global__ __launch_bounds__(kMcThreads) void mc_count_kernel(const float* __restrict__ vol, int nx,
                                                              int ny, int nseg, float iso,
                                                              const McTable* __restrict__ table,
                                                              uint32_t* __restrict__ block_tris) {
  __shared__ uint8_t ntri[256];
  __shared__ unsigned red[4];
  ntri[threadIdx.x] = table->ntri[threadIdx.x];
  __syncthreads();
  const McRow m = mc_row(vol, nx, ny, nseg);
  unsigned cnt = 0;
#pragma unroll
  for (int k = 0; k < kMcPer; ++k) {
    const int x = m.x0 + k * kMcThreads + (int)threadIdx.x;
    if (x < nx - 1) {
      float v[8];
      cnt += ntri[mc_config(m, x, iso, v)];
    }
  }
  const unsigned s = block_sum(cnt, red);
  if (threadIdx.x == 0) block_tris[blockIdx.x] = s;
}

// Exclusive prefix sums of the per-workgroup counts (one workgroup of 1024
// threads, each summing a contiguous chunk); off[nblk] is the total.
__global__ __launch_bounds__(1024) void mc_scan_kernel(const uint32_t* __restrict__ block_tris,
                                                       long long nblk,
                                                       unsigned long long* __restrict__ off) {
  __shared__ unsigned long long part[1024];
  const long long chunk = (nblk + 1023) / 1024;
  const long long b0 = threadIdx.x * chunk;
  const long long b1 = b0 + chunk < nblk ? b0 + chunk : nblk;
  unsigned long long s = 0;
  for (long long b = b0; b < b1; ++b) s += block_tris[b];
  part[threadIdx.x] = s;
  __syncthreads();
  // inclusive scan of the 1024 chunk sums (Hillis-Steele in LDS)
  for (int d = 1; d < 1024; d <<= 1) {
    const unsigned long long add = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0ull;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  unsigned long long run = threadIdx.x ? part[threadIdx.x - 1] : 0ull;
  for (long long b = b0; b < b1; ++b) {
    off[b] = run;
    run += block_tris[b];
  }
  if (threadIdx.x == 1023) off[nblk] = part[1023];
}

__global__ __launch_bounds__(kMcThreads) void mc_emit_kernel(
    const float* __restrict__ vol, int nx, int ny, int nseg, float iso,
    const McTable* __restrict__ table, const unsigned long long* __restrict__ off,
    float* __restrict__ tris, long long* __restrict__ cube_id, long long max_tris) {
  __shared__ McTable tab;
  __shared__ unsigned wsum[4];
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(table);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&tab);
    for (int i = threadIdx.x; i < (int)(sizeof(McTable) / 4); i += kMcThreads) dst[i] = src[i];
  }
  __syncthreads();
  const McRow m = mc_row(vol, nx, ny, nseg);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  unsigned long long base = off[blockIdx.x];
  const long long rowbase = ((long long)m.z * (ny - 1) + m.y) * (nx - 1);
#pragma unroll 1
  for (int k = 0; k < kMcPer; ++k) {
    const int x = m.x0 + k * kMcThreads + (int)threadIdx.x;
    float v[8];
    int cfg = 0, n = 0;
    if (x < nx - 1) {
      cfg = mc_config(m, x, iso, v);
      n = tab.ntri[cfg];
    }
    // rank among the workgroup's cubes of this pass, in x order
    unsigned inc = (unsigned)n;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned t = __shfl_up(inc, o, 64);
      if (lane >= o) inc += t;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    unsigned before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      before += w < wid ? wsum[w] : 0u;
      total += wsum[w];
    }
    __syncthreads();
    const unsigned long long first = base + before + inc - (unsigned)n;
    for (int j = 0; j < n; ++j) {
      const long long o = (long long)(first + j);
      if (o >= max_tris) break;
      float* t = tris + 9 * o;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int e = tab.tri[cfg][3 * j + q];
        const int axis = e >> 2;
        // lower corner of the edge: bit `axis` clear, the edge's (u, w) on
        // the other two axes
        const int b0 = axis == 0 ? 1 : 0, b1 = axis == 2 ? 1 : 2;
        const int lo = ((e & 1) << b0) | (((e >> 1) & 1) << b1);
        const int hi = lo | (1 << axis);
        const float A = v[lo], B = v[hi];
        const float tt = __fdiv_rn(iso - A, B - A);
        float p[3] = {(float)(x + (lo & 1)), (float)(m.y + ((lo >> 1) & 1)),
                      (float)(m.z + ((lo >> 2) & 1))};
        p[axis] = p[axis] + tt;
        t[3 * q + 0] = p[0];
        t[3 * q + 1] = p[1];
        t[3 * q + 2] = p[2];
      }
      if (cube_id) cube_id[o] = rowbase + x;
    }
    base += total;
  }
}

}  // namespace

hipError_t launch_mc_count(const float* vol, int nx, int ny, long long nblk, int nseg, float iso,
                           const McTable* table, uint32_t* block_tris, hipStream_t s) {
  hipLaunchKernelGGL(mc_count_kernel, dim3((unsigned)nblk), dim3(kMcThreads), 0, s, vol, nx, ny,
                     nseg, iso, table, block_tris);
  return hipGetLastError();
}

hipError_t launch_mc_scan(const uint32_t* block_tris, long long nblk, unsigned long long* off,
                          hipStream_t s) {
  hipLaunchKernelGGL(mc_scan_kernel, dim3(1), dim3(1024), 0, s, block_tris, nblk, off);
  return hipGetLastError();
}

hipError_t launch_mc_emit(const float* vol, int nx, int ny, long long nblk, int nseg, float iso,
                          const McTable* table, const unsigned long long* off, float* tris,
                          long long* cube_id, long long max_tris, hipStream_t s) {
  hipLaunchKernelGGL(mc_emit_kernel, dim3((unsigned)nblk), dim3(kMcThreads), 0, s, vol, nx, ny,
                     nseg, iso, table, off, tris, cube_id, max_tris);
  return hipGetLastError();
}

}  // namespace okr
