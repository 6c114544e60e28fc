// Marching-cubes case table, generated at load time from a rule (the paper
// runs marching cubes on the reconstructed corners, Sec. IV-D, without fixing
// a table).
//
// Rule: corner i is inside iff its value is below the iso-value.  On each of
// the six faces, traversed counter-clockwise about its outward normal, an edge
// crossed from an outside corner to an inside one opens a run of inside
// corners and the next edge crossed from inside to outside closes it; the
// surface crosses the face on a segment from the opening edge to the closing
// edge.  (On a face with two diagonal inside corners this cuts each inside
// corner off separately, so neighbouring cells agree on the shared face.)
// Every crossed edge closes a run on one of its two faces and opens one on the
// other, so the segments link into closed loops.  Each loop is listed from its
// lowest-numbered edge, loops in order of that edge, and each is fanned from
// its first vertex; the resulting triangles face the larger values.
#include <cstring>

#include "isx_internal.h"

namespace isx {

namespace {

// edge -> (lower corner, upper corner)
constexpr unsigned char kEdge[12][2] = {{0, 1}, {1, 2}, {3, 2}, {0, 3}, {4, 5}, {5, 6},
                                        {7, 6}, {4, 7}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};

// faces, corners in counter-clockwise order about the outward normal
// (x=0, x=1, y=0, y=1, z=0, z=1)
constexpr unsigned char kFace[6][4] = {{0, 4, 7, 3}, {1, 2, 6, 5}, {0, 1, 5, 4},
                                       {3, 7, 6, 2}, {0, 3, 2, 1}, {4, 5, 6, 7}};

int edge_between(int a, int b) {
  for (int e = 0; e < 12; ++e)
    if ((kEdge[e][0] == a && kEdge[e][1] == b) || (kEdge[e][0] == b && kEdge[e][1] == a)) return e;
  return -1;
}

McTable build() {
  McTable t;
  std::memset(&t, 0, sizeof(t));
  std::memset(t.edges, -1, sizeof(t.edges));
  for (int cs = 0; cs < 256; ++cs) {
    int link[12];
    for (int e = 0; e < 12; ++e) link[e] = -1;
    for (int f = 0; f < 6; ++f) {
      // crossings around the face: +1 opening (out -> in), -1 closing (in -> out)
      int kind[4], edge[4], n = 0;
      for (int s = 0; s < 4; ++s) {
        const int a = kFace[f][s], b = kFace[f][(s + 1) & 3];
        const int ia = (cs >> a) & 1, ib = (cs >> b) & 1;
        if (ia != ib) {
          kind[n] = ib ? +1 : -1;
          edge[n] = edge_between(a, b);
          ++n;
        }
      }
      for (int i = 0; i < n; ++i) {
        if (kind[i] != +1) continue;
        for (int d = 1; d < n; ++d) {
          const int j = (i + d) % n;
          if (kind[j] == -1) {
            link[edge[i]] = edge[j];
            break;
          }
        }
      }
    }
    bool used[12] = {};
    int ntri = 0;
    for (int e0 = 0; e0 < 12; ++e0) {
      if (link[e0] < 0 || used[e0]) continue;
      int loop[12], len = 0;
      int e = e0;
      do {
        used[e] = true;
        loop[len++] = e;
        e = link[e];
      } while (e != e0 && len < 12);
      for (int i = 1; i + 1 < len && ntri < 5; ++i) {
        t.edges[cs][3 * ntri + 0] = (int8_t)loop[0];
        t.edges[cs][3 * ntri + 1] = (int8_t)loop[i];
        t.edges[cs][3 * ntri + 2] = (int8_t)loop[i + 1];
        ++ntri;
      }
    }
    t.count[cs] = (uint8_t)ntri;
  }
  return t;
}

}  // namespace

const McTable& mc_table() {
  static const McTable table = build();
  return table;
}

}  // namespace isx
