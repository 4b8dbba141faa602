// Marching cubes on a float32 volume [nz][ny][nx] (Appendix C): the case
// table (mcubes_table.cpp) gives each corner configuration's triangles as
// cube-edge triples; crossing points are interpolated on their edges.
//
// Four launches: count, two scan levels, emit. A wave takes a strip of 64
// cubes of one z-slab over kMcRows rows and slides down y, classifying each
// row's four corners once (a cube's configuration joins the patterns of its
// two rows), so each cube loads only its new row (two coalesced reads per
// z-level). Counts are kept per (row, strip): count and emit need no
// workgroup barrier, the scans turn them into output offsets that keep the
// cube order, and the emit pass visits only the (row, strip) pairs whose
// count is not zero.
#include "okrig_internal.h"

namespace okr {
namespace {

// One wave's strip of cubes: z-slab z, rows [y0, y1), columns x = x0 + lane.
struct McStrip {
  const float* p0;    // plane z
  const float* p1;    // plane z + 1
  int x, y0, y1, z;
  long long strip, nstrip;
};

__device__ __forceinline__ McStrip mc_strip(const float* vol, int nx, int ny, int nstrip,
                                            int nych) {
  const long long wave = blockIdx.x * 4ll + (threadIdx.x >> 6);
  McStrip m;
  m.nstrip = nstrip;
  m.strip = wave % nstrip;
  const long long t = wave / nstrip;
  const int ych = (int)(t % nych);
  m.z = (int)(t / nych);
  m.x = (int)m.strip * 64 + (int)(threadIdx.x & 63);
  m.y0 = ych * kMcRows;
  m.y1 = m.y0 + kMcRows < ny - 1 ? m.y0 + kMcRows : ny - 1;
  const long long plane = (long long)nx * ny;
  m.p0 = vol + m.z * plane;
  m.p1 = m.p0 + plane;
  return m;
}

// Corner values of row y at column x: (x, z), (x+1, z), (x, z+1), (x+1, z+1).
struct McPair {
  float a, b, c, d;
};

__device__ __forceinline__ McPair mc_load(const McStrip& m, int nx, int y) {
  const long long o = (long long)y * nx + m.x;
  return {m.p0[o], m.p0[o + 1], m.p1[o], m.p1[o + 1]};
}

// Corners c = x + 2y + 4z of the cube between rows y (lo) and y + 1 (hi);
// bit c of the configuration set when corner c is inside (value >= iso,
// NaN outside).
// A row's four corners classified once: bits 0, 1, 4, 5 (x and x + 1 at z,
// then at z + 1); the cube between rows y and y + 1 has configuration
// nib(y) | nib(y + 1) << 2.
__device__ __forceinline__ int mc_nib(const McPair& r, float iso) {
  return (r.a >= iso ? 1 : 0) | (r.b >= iso ? 2 : 0) | (r.c >= iso ? 16 : 0) |
         (r.d >= iso ? 32 : 0);
}

// Rows y + 1 .. y + kMcGroup (those before m.y1) of the strip.
__device__ __forceinline__ void mc_load_group(const McStrip& m, int nx, int y, bool valid,
                                              McPair (&g)[kMcGroup]) {
#pragma unroll
  for (int k = 0; k < kMcGroup; ++k)
    g[k] = (valid && y + k < m.y1) ? mc_load(m, nx, y + k + 1) : McPair{0, 0, 0, 0};
}

// Triangle counts are 0..5: three bits. The wave's total and each lane's
// exclusive prefix come from one ballot per bit (popcounts on the scalar unit,
// lane-masked counts with mbcnt), without a shuffle through LDS.
struct McBits {
  uint64_t b0, b1, b2;
};

__device__ __forceinline__ McBits mc_bits(unsigned n) {
  return {__ballot(n & 1u), __ballot(n & 2u), __ballot(n & 4u)};
}

__device__ __forceinline__ unsigned mc_total(const McBits& b) {
  return (unsigned)(__popcll(b.b0) + 2 * __popcll(b.b1) + 4 * __popcll(b.b2));
}

__device__ __forceinline__ unsigned mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ unsigned mc_prefix(const McBits& b) {
  return mbcnt64(b.b0) + 2u * mbcnt64(b.b1) + 4u * mbcnt64(b.b2);
}

// count of (row, strip) at index row * nstrip + strip, row = z * (ny-1) + y
__global__ __launch_bounds__(256) void mc_count_kernel(const float* __restrict__ vol, int nx,
                                                       int ny, int nstrip, int nych,
                                                       long long nwaves, float iso,
                                                       const McTable* __restrict__ table,
                                                       uint32_t* __restrict__ cnt) {
  __shared__ uint8_t ntri[256];
  ntri[threadIdx.x] = table->ntri[threadIdx.x];
  __syncthreads();
  if (blockIdx.x * 4ll + (threadIdx.x >> 6) >= nwaves) return;
  const McStrip m = mc_strip(vol, nx, ny, nstrip, nych);
  const bool valid = m.x < nx - 1;
  int nlo = valid ? mc_nib(mc_load(m, nx, m.y0), iso) : 0;
  // rows in groups of kMcGroup; the next group's loads are issued before the
  // current group is classified, for memory-level parallelism
  McPair cur[kMcGroup], nxt[kMcGroup];
  mc_load_group(m, nx, m.y0, valid, cur);
  for (int y = m.y0; y < m.y1; y += kMcGroup) {
    mc_load_group(m, nx, y + kMcGroup, valid, nxt);
#pragma unroll
    for (int k = 0; k < kMcGroup; ++k) {
      if (y + k < m.y1) {
        const int nhi = mc_nib(cur[k], iso);
        const unsigned n = valid ? ntri[nlo | (nhi << 2)] : 0u;
        const unsigned tot = mc_total(mc_bits(n));
        if ((threadIdx.x & 63) == 0)
          cnt[((long long)m.z * (ny - 1) + y + k) * m.nstrip + m.strip] = tot;
        nlo = nhi;
      }
    }
#pragma unroll
    for (int k = 0; k < kMcGroup; ++k) cur[k] = nxt[k];
  }
}

// Level 1: each workgroup turns 1024 counts into offsets within the tile (in
// place) and records the tile's total.
__global__ __launch_bounds__(1024) void mc_scan_tiles_kernel(uint32_t* __restrict__ cnt,
                                                             long long ncnt,
                                                             unsigned long long* __restrict__ tile_sum) {
  __shared__ unsigned wtot[16];
  const long long i = blockIdx.x * 1024ll + threadIdx.x;
  const unsigned c = i < ncnt ? cnt[i] : 0u;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  unsigned inc = c;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wtot[wid] = inc;
  __syncthreads();
  unsigned before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < 16; ++w) {
    before += w < wid ? wtot[w] : 0u;
    total += wtot[w];
  }
  if (i < ncnt) cnt[i] = before + inc - c;
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// Level 2 (one workgroup): exclusive offsets of the tiles, in place;
// tile_sum[ntile] receives the total.
__global__ __launch_bounds__(1024) void mc_scan_top_kernel(unsigned long long* __restrict__ tile_sum,
                                                           long long ntile) {
  __shared__ unsigned long long wtot[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  unsigned long long carry = 0;
  for (long long base = 0; base < ntile; base += 1024) {
    const long long i = base + threadIdx.x;
    const unsigned long long c = i < ntile ? tile_sum[i] : 0ull;
    unsigned long long inc = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long t = __shfl_up(inc, o, 64);
      if (lane >= o) inc += t;
    }
    if (lane == 63) wtot[wid] = inc;
    __syncthreads();
    unsigned long long before = 0, total = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      before += w < wid ? wtot[w] : 0ull;
      total += wtot[w];
    }
    __syncthreads();
    if (i < ntile) tile_sum[i] = carry + before + inc - c;
    carry += total;
  }
  if (threadIdx.x == 0) tile_sum[ntile] = carry;
}

// Per-wave queue of the emit pass: the cubes that have triangles (first
// output slot, column, row and configuration in one 16-byte record) and one
// task per triangle (cube slot << 3 | triangle); the corner values are read
// again (from cache) when the triangles are computed. Rows are appended until
// 64 or more triangles wait; the wave then computes them, two per lane at a
// time, so consecutive lanes write consecutive triangles. Capacity: fewer
// than 64 waiting plus one row's at most 5 x 64.
constexpr int kMcQCubes = 128;
constexpr int kMcQTris = 64 + 5 * 64;
struct McCube {
  unsigned long long first;
  int x;
  int ycfg;   // row | configuration << 24
};
struct McQueue {
  McCube cube[kMcQCubes];
  unsigned task[kMcQTris];
};

// v[c] for a lane-varying corner c: a select tree on the bits of c.
__device__ __forceinline__ float mc_pick(const float (&v)[8], int c) {
  const bool b0 = c & 1, b1 = c & 2, b2 = c & 4;
  const float q0 = b0 ? v[1] : v[0], q1 = b0 ? v[3] : v[2];
  const float q2 = b0 ? v[5] : v[4], q3 = b0 ? v[7] : v[6];
  const float r0 = b1 ? q1 : q0, r1 = b1 ? q3 : q2;
  return b2 ? r1 : r0;
}

// Triangle j of a queued cube: three vertices and the cube id.
__device__ __forceinline__ void mc_triangle(const McCube& c, int j, const McTable& tab,
                                            const McStrip& m, int nx, int ny, float iso,
                                            float* __restrict__ tris,
                                            long long* __restrict__ cube_id, long long max_tris) {
  const long long o = (long long)(c.first + j);
  if (o >= max_tris) return;
  const int cfg = (int)((unsigned)c.ycfg >> 24), y = c.ycfg & 0xffffff, x = c.x;
  const long long r0 = (long long)y * nx + x, r1 = r0 + nx;
  const float v[8] = {m.p0[r0], m.p0[r0 + 1], m.p0[r1], m.p0[r1 + 1],
                      m.p1[r0], m.p1[r0 + 1], m.p1[r1], m.p1[r1 + 1]};
  float out[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int ed = tab.tri[cfg][3 * j + k];
    const int axis = ed >> 2;
    // lower corner of the edge: bit `axis` clear, the edge's (u, w) on the
    // other two axes
    const int b0 = axis == 0 ? 1 : 0, b1 = axis == 2 ? 1 : 2;
    const int lc = ((ed & 1) << b0) | (((ed >> 1) & 1) << b1);
    const int hc = lc | (1 << axis);
    const float A = mc_pick(v, lc), B = mc_pick(v, hc);
    const float tt = __fdiv_rn(iso - A, B - A);
    float p[3] = {(float)(x + (lc & 1)), (float)(y + ((lc >> 1) & 1)),
                  (float)(m.z + ((lc >> 2) & 1))};
    p[axis] = p[axis] + tt;
    out[3 * k + 0] = p[0];
    out[3 * k + 1] = p[1];
    out[3 * k + 2] = p[2];
  }
  float* dst = tris + 9 * o;
#pragma unroll
  for (int k = 0; k < 9; ++k) dst[k] = out[k];
  if (cube_id) cube_id[o] = ((long long)m.z * (ny - 1) + y) * (nx - 1) + x;
}

__device__ __forceinline__ void mc_flush(const McQueue& q, int ntask, const McTable& tab,
                                      const McStrip& m, int nx, int ny, float iso,
                                      float* __restrict__ tris,
                                      long long* __restrict__ cube_id, long long max_tris) {
  const int lane = threadIdx.x & 63;
  for (int t = lane; t < ntask; t += 128) {
    // two tasks per lane: their loads overlap
    const bool two = t + 64 < ntask;
    const unsigned ta = q.task[t], tb = two ? q.task[t + 64] : 0u;
    const McCube ca = q.cube[ta >> 3];
    const McCube cb = q.cube[tb >> 3];
    mc_triangle(ca, (int)(ta & 7), tab, m, nx, ny, iso, tris, cube_id, max_tris);
    if (two) mc_triangle(cb, (int)(tb & 7), tab, m, nx, ny, iso, tris, cube_id, max_tris);
  }
}

__global__ __launch_bounds__(256) void mc_emit_kernel(
    const float* __restrict__ vol, int nx, int ny, int nstrip, int nych, long long nwaves,
    long long ncnt, long long ntile, float iso, const McTable* __restrict__ table,
    const uint32_t* __restrict__ off_local, const unsigned long long* __restrict__ tile_off,
    float* __restrict__ tris, long long* __restrict__ cube_id, long long max_tris) {
  __shared__ McTable tab;
  __shared__ McQueue queues[4];
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(table);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&tab);
    for (int i = threadIdx.x; i < (int)(sizeof(McTable) / 4); i += 256) dst[i] = src[i];
  }
  __syncthreads();
  if (blockIdx.x * 4ll + (threadIdx.x >> 6) >= nwaves) return;
  McQueue& q = queues[threadIdx.x >> 6];
  const McStrip m = mc_strip(vol, nx, ny, nstrip, nych);
  const bool valid = m.x < nx - 1;
  const int lane = threadIdx.x & 63;
  // output offsets of the strip's rows, one row per lane (kMcRows <= 64); a
  // row whose offset equals the next (row, strip)'s has no triangle in this
  // strip and is skipped
  unsigned long long row_off = 0;
  bool row_has = false;
  if (m.y0 + lane < m.y1) {
    const long long e = ((long long)m.z * (ny - 1) + m.y0 + lane) * m.nstrip + m.strip;
    row_off = tile_off[e >> 10] + off_local[e];
    const long long e1 = e + 1;
    const unsigned long long next = e1 < ncnt ? tile_off[e1 >> 10] + off_local[e1] : tile_off[ntile];
    row_has = next > row_off;
  }
  uint64_t act = __ballot(row_has);
  if (act == 0) return;
  // the rows with triangles in order; the next one's corner rows are loaded
  // while the current one is queued (a row shared by consecutive cubes' rows
  // is loaded once); one flush site keeps the kernel small
  int y = m.y0 + (int)__builtin_ctzll(act);
  act &= act - 1;
  McPair lo = valid ? mc_load(m, nx, y) : McPair{0, 0, 0, 0};
  McPair hi = valid ? mc_load(m, nx, y + 1) : McPair{0, 0, 0, 0};
  int ncube = 0, ntask = 0;
#pragma unroll 1
  for (;;) {
    const bool more = act != 0;
    const int yn = more ? m.y0 + (int)__builtin_ctzll(act) : y;
    McPair nlo = hi, nhi = hi;
    if (more) {
      if (yn != y + 1) nlo = valid ? mc_load(m, nx, yn) : McPair{0, 0, 0, 0};
      nhi = valid ? mc_load(m, nx, yn + 1) : McPair{0, 0, 0, 0};
    }
    const int cfg = valid ? (mc_nib(lo, iso) | (mc_nib(hi, iso) << 2)) : 0;
    const int n = valid ? tab.ntri[cfg] : 0;
    const McBits bits = mc_bits((unsigned)n);
    const unsigned pre = mc_prefix(bits), total = mc_total(bits);
    const unsigned r_lo = __builtin_amdgcn_readlane((unsigned)(row_off & 0xffffffffu), y - m.y0);
    const unsigned r_hi = __builtin_amdgcn_readlane((unsigned)(row_off >> 32), y - m.y0);
    const unsigned long long rbase = ((unsigned long long)r_hi << 32) | r_lo;
    const uint64_t has = __ballot(n > 0);
    if (n > 0) {
      const int slot = ncube + (int)mbcnt64(has);
      q.cube[slot] = McCube{rbase + pre, m.x, y | (cfg << 24)};
      for (int j = 0; j < n; ++j) q.task[ntask + pre + j] = ((unsigned)slot << 3) | (unsigned)j;
    }
    ncube += __popcll(has);
    ntask += (int)total;
    if (ntask >= 64 || (!more && ntask > 0)) {
      __builtin_amdgcn_wave_barrier();
      mc_flush(q, ntask, tab, m, nx, ny, iso, tris, cube_id, max_tris);
      __builtin_amdgcn_wave_barrier();
      ncube = 0;
      ntask = 0;
    }
    if (!more) break;
    act &= act - 1;
    y = yn;
    lo = nlo;
    hi = nhi;
  }
}

}  // namespace

McGrid mc_grid(long long nz, long long ny, long long nx) {
  McGrid g;
  g.nstrip = (nx - 1 + 63) / 64;
  g.nych = (ny - 1 + kMcRows - 1) / kMcRows;
  g.nwaves = (nz - 1) * g.nych * g.nstrip;
  g.ncnt = (nz - 1) * (ny - 1) * g.nstrip;
  g.ntile = (g.ncnt + 1023) / 1024;
  return g;
}

hipError_t launch_mc_count(const float* vol, int nx, int ny, const McGrid& g, float iso,
                           const McTable* table, uint32_t* cnt, hipStream_t s) {
  hipLaunchKernelGGL(mc_count_kernel, dim3((unsigned)((g.nwaves + 3) / 4)), dim3(256), 0, s, vol,
                     nx, ny, (int)g.nstrip, (int)g.nych, g.nwaves, iso, table, cnt);
  return hipGetLastError();
}

hipError_t launch_mc_scan(uint32_t* cnt, const McGrid& g, unsigned long long* tile,
                          hipStream_t s) {
  hipLaunchKernelGGL(mc_scan_tiles_kernel, dim3((unsigned)g.ntile), dim3(1024), 0, s, cnt, g.ncnt,
                     tile);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mc_scan_top_kernel, dim3(1), dim3(1024), 0, s, tile, g.ntile);
  return hipGetLastError();
}

hipError_t launch_mc_emit(const float* vol, int nx, int ny, const McGrid& g, float iso,
                          const McTable* table, const uint32_t* off_local,
                          const unsigned long long* tile_off, float* tris, long long* cube_id,
                          long long max_tris, hipStream_t s) {
  hipLaunchKernelGGL(mc_emit_kernel, dim3((unsigned)((g.nwaves + 3) / 4)), dim3(256), 0, s, vol,
                     nx, ny, (int)g.nstrip, (int)g.nych, g.nwaves, g.ncnt, g.ntile, iso, table,
                     off_local, tile_off, tris, cube_id, max_tris);
  return hipGetLastError();
}

}  // namespace okr
