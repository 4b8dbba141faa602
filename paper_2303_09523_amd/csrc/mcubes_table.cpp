// Case table of marching cubes (Appendix C): for each of the 256 corner
// configurations, the triangles as triples of cube edges, built once on the
// host from the rules below and copied to each plan's device memory.
//
//   corner c = x + 2y + 4z; edge e = 4a + u + 2w runs along axis a from the
//   corner with bit a clear to the one with it set, (u, w) being its position
//   on the other two axes in increasing axis order.
//   On every face the crossing edges are paired into segments; a face with
//   four crossings (diagonal corners alike) pairs the two crossings next to
//   each inside corner, so both cubes that share the face pair it the same way.
//   Segments chain into cycles. A cycle is oriented so that the vector area of
//   the polygon through its edges' midpoints points the way its edges go from
//   inside to outside, and is triangulated as a fan from its lowest edge id;
//   cycles are listed by lowest edge id.
#include <algorithm>
#include <array>
#include <cstdint>
#include <mutex>
#include <vector>

#include "okrig_internal.h"

namespace okr {
namespace {

struct Vec3 {
  double v[3];
};

void other_axes(int a, int& b0, int& b1) {
  b0 = a == 0 ? 1 : 0;
  b1 = a == 2 ? 1 : 2;
}

int edge_id(int c0, int c1) {
  const int d = c0 ^ c1;
  const int a = d == 1 ? 0 : (d == 2 ? 1 : 2);
  const int lo = std::min(c0, c1);
  int b0, b1;
  other_axes(a, b0, b1);
  return 4 * a + ((lo >> b0) & 1) + 2 * ((lo >> b1) & 1);
}

// lower corner and axis of an edge
void edge_ends(int e, int& lo, int& axis) {
  axis = e / 4;
  int b0, b1;
  other_axes(axis, b0, b1);
  lo = ((e & 1) << b0) | (((e >> 1) & 1) << b1);
}

Vec3 edge_mid(int e) {
  int lo, a;
  edge_ends(e, lo, a);
  Vec3 m{{double(lo & 1), double((lo >> 1) & 1), double((lo >> 2) & 1)}};
  m.v[a] += 0.5;
  return m;
}

void build_case(int cfg, uint8_t& ntri, uint8_t* out) {
  auto in = [cfg](int c) { return (cfg >> c) & 1; };
  std::array<std::vector<int>, 12> nb;
  for (int a = 0; a < 3; ++a) {
    int b0, b1;
    other_axes(a, b0, b1);
    for (int s = 0; s < 2; ++s) {
      const int ring[4] = {s << a, (s << a) | (1 << b0), (s << a) | (1 << b0) | (1 << b1),
                           (s << a) | (1 << b1)};
      int pos[4], eid[4], n = 0;
      for (int i = 0; i < 4; ++i) {
        const int c0 = ring[i], c1 = ring[(i + 1) & 3];
        if (in(c0) != in(c1)) {
          pos[n] = i;
          eid[n] = edge_id(c0, c1);
          ++n;
        }
      }
      auto link = [&nb](int e0, int e1) {
        nb[e0].push_back(e1);
        nb[e1].push_back(e0);
      };
      if (n == 2) {
        link(eid[0], eid[1]);
      } else if (n == 4) {
        // ring edges 0..3 all cross; consecutive ones meet at ring[i + 1]
        for (int j = 0; j < 4; ++j)
          if (in(ring[(pos[j] + 1) & 3])) link(eid[j], eid[(j + 1) & 3]);
      }
    }
  }
  ntri = 0;
  bool used[12] = {false};
  for (int start = 0; start < 12; ++start) {
    if (used[start] || nb[start].empty()) continue;
    std::vector<int> cyc{start};
    used[start] = true;
    int prev = -1, cur = start;
    for (;;) {
      const int nxt = nb[cur][0] == prev ? nb[cur][1] : nb[cur][0];
      if (nxt == start) break;
      cyc.push_back(nxt);
      used[nxt] = true;
      prev = cur;
      cur = nxt;
    }
    double area[3] = {0, 0, 0}, dir[3] = {0, 0, 0};
    const size_t k = cyc.size();
    for (size_t i = 0; i < k; ++i) {
      const Vec3 p = edge_mid(cyc[i]), q = edge_mid(cyc[(i + 1) % k]);
      area[0] += p.v[1] * q.v[2] - p.v[2] * q.v[1];
      area[1] += p.v[2] * q.v[0] - p.v[0] * q.v[2];
      area[2] += p.v[0] * q.v[1] - p.v[1] * q.v[0];
      int lo, ax;
      edge_ends(cyc[i], lo, ax);
      dir[ax] += in(lo) ? 1.0 : -1.0;
    }
    if (area[0] * dir[0] + area[1] * dir[1] + area[2] * dir[2] < 0.0)
      std::reverse(cyc.begin() + 1, cyc.end());
    for (size_t i = 1; i + 1 < k; ++i) {
      uint8_t* t = out + 3 * ntri;
      t[0] = (uint8_t)cyc[0];
      t[1] = (uint8_t)cyc[i];
      t[2] = (uint8_t)cyc[i + 1];
      ++ntri;
    }
  }
}

}  // namespace

const McTable& mc_table() {
  static McTable table;
  static std::once_flag once;
  std::call_once(once, [] {
    for (int cfg = 0; cfg < 256; ++cfg) {
      std::fill(table.tri[cfg], table.tri[cfg] + kMcMaxTri * 3, (uint8_t)0);
      build_case(cfg, table.ntri[cfg], table.tri[cfg]);
    }
  });
  return table;
}

}  // namespace okr
