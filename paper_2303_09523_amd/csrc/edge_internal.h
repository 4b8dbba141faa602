// Internal declarations of the edge post-pass shared by the host library and
// its kernels (kernels_edge.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace okr {

struct EdgeArgs {
  const float* volume;  // input volume [nz][ny][nx]
  float* out;           // adjusted volume: a copy of the input, or the input itself
  double* mag;          // M = max_k |SH_k| [nz][ny][nx]
  uint8_t* theta;       // first argmax orientation [nz][ny][nx]
  uint32_t* bits;       // per-image edge bitmaps [(nz + 2) * wr][nx]
  uint8_t* edge_out;    // edge map [nz][ny][nx] (nullable)
  uint8_t* orient_out;  // orientation map [nz][ny][nx] (nullable)
  double tau;           // edge threshold on M
  int nz, ny, nx;
  int wr;               // bitmap words per padded row
  uint32_t n1, n2;      // rounded normal of orientation k: 4-bit field k holds n + 1
};

int edge_words_per_row(int ny);
hipError_t launch_edge_shear(const EdgeArgs& a, hipStream_t s);
hipError_t launch_edge_nms(const EdgeArgs& a, hipStream_t s);
// Traces every image: its bitmap in LDS when it fits below min(lds_limit,
// 64 KB) beside the window queue (returns true), else in place in the global
// bitmaps. *err receives the launch status.
bool launch_edge_trace(const EdgeArgs& a, int lds_limit, hipStream_t s, hipError_t* err);

}  // namespace okr
