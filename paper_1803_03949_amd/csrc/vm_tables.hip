// Marching-cubes tables of the library, generated on the host when a volume
// is created (Sec. V-B: the table T maps the 8-bit cube type to the edges
// that carry vertices and the triangles joining them; the paper prints no
// table).
//
// Rule (a face-consistent marching cubes): each of the six cube faces is
// walked counter-clockwise as seen from outside the cube.  Going around the
// face, an edge where the walk passes from an outside corner (d >= 0) to an
// inside corner (d < 0) is an entry, the reverse an exit; each entry is
// joined to the next exit.  On a face with four crossings this cuts off each
// inside corner on its own, so two cubes sharing the face always agree.  The
// joined segments close into polygons, oriented so that their normals point
// to the outside region; every polygon is fanned from its lowest-numbered
// edge, and polygons are listed by that edge.
#include <stdint.h>
#include <string.h>

namespace vm {

// Cube corners: 0 (0,0,0) 1 (1,0,0) 2 (1,1,0) 3 (0,1,0) 4 (0,0,1) 5 (1,0,1)
// 6 (1,1,1) 7 (0,1,1).  Edges 0-3 ring z=0, 4-7 ring z=1, 8-11 pillars.
static const int kEdgeCorners[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6},
                                        {6, 7}, {7, 4}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};

// Each face's corners in counter-clockwise order seen from outside:
// z=0, z=1, y=0, y=1, x=0, x=1.
static const int kFaceLoop[6][4] = {{0, 3, 2, 1}, {4, 5, 6, 7}, {0, 1, 5, 4},
                                    {3, 7, 6, 2}, {0, 4, 7, 3}, {1, 2, 6, 5}};

// tri[t*16]: number of triangles n, then 3n cube-edge ids (0xFF padding).
// uses[t*12 + e]: number of the type's triangles that use edge e.
void build_mc_tables(uint8_t* tri, uint8_t* uses) {
  int edge_between[8][8];
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b) edge_between[a][b] = -1;
  for (int e = 0; e < 12; ++e) {
    edge_between[kEdgeCorners[e][0]][kEdgeCorners[e][1]] = e;
    edge_between[kEdgeCorners[e][1]][kEdgeCorners[e][0]] = e;
  }
  memset(tri, 0xFF, 256 * 16);
  memset(uses, 0, 256 * 12);
  for (int t = 0; t < 256; ++t) {
    int next[12];
    for (int e = 0; e < 12; ++e) next[e] = -1;
    for (int f = 0; f < 6; ++f) {
      int kind[4], edge[4];  // kind: +1 entry, -1 exit, 0 no crossing
      for (int i = 0; i < 4; ++i) {
        int a = kFaceLoop[f][i], b = kFaceLoop[f][(i + 1) & 3];
        int ina = (t >> a) & 1, inb = (t >> b) & 1;
        edge[i] = edge_between[a][b];
        kind[i] = (!ina && inb) ? 1 : (ina && !inb) ? -1 : 0;
      }
      for (int i = 0; i < 4; ++i) {
        if (kind[i] != 1) continue;
        for (int k = 1; k < 4; ++k) {
          int j = (i + k) & 3;
          if (kind[j] == -1) {
            next[edge[i]] = edge[j];
            break;
          }
        }
      }
    }
    int n = 0;
    bool done[12] = {false};
    for (int e0 = 0; e0 < 12; ++e0) {
      if (next[e0] < 0 || done[e0]) continue;
      int loop[12], len = 0;
      for (int e = e0; !done[e]; e = next[e]) {
        done[e] = true;
        loop[len++] = e;
      }
      for (int i = 1; i + 1 < len; ++i) {
        uint8_t* out = tri + t * 16 + 1 + 3 * n;
        out[0] = (uint8_t)loop[0];
        out[1] = (uint8_t)loop[i];
        out[2] = (uint8_t)loop[i + 1];
        for (int j = 0; j < 3; ++j) uses[t * 12 + out[j]]++;
        ++n;
      }
    }
    tri[t * 16] = (uint8_t)n;
  }
}

}  // namespace vm
