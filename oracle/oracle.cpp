// CPU oracle for incremental volumetric meshing over a spatially hashed TSDF
// (Dong, Shi, Tang, Wang, Zha: "An Efficient Volumetric Mesh Representation
// for Real-time Scene Reconstruction using Spatial Hashing", arXiv 1803.03949).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
// reference the GPU library is checked against.  It shares no code, header,
// table or constant generator with the GPU path; only the test suite, the
// smoke check and the CPU-baseline leg of the benchmark may load it.
//
// Everything here is scalar and single threaded.  Containers are ordered
// std::map/std::set (no hash table of our own).  Floating point follows the
// operation order written in each comment; the library is built with
// -ffp-contract=off and without fast-math so every product and sum is rounded
// separately, which is what makes cube signs reproducible bit for bit.
//
// Readings of points the paper leaves open are marked READING and listed in
// the design notes of the repository.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Lattice conventions (Sec. IV, Fig. "cube"): a voxel is a lattice corner
// g in Z^3 at world position g*s; its TSDF value lives at the corner.  A block
// is 8x8x8 voxels.  The cube anchored at corner c has its eight corners in
// the cyclic order below (READING of the missing bit-order figure of
// Sec. V-F: under this numbering the six printed regular types are exactly
// the six axis-aligned half-cube splits).
// ---------------------------------------------------------------------------
const int kCorner[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                           {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
// The twelve cube edges as pairs of corners: bottom ring, top ring, pillars.
const int kEdgeEnds[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6},
                              {6, 7}, {7, 4}, {0, 4}, {1, 5}, {2, 6}, {3, 7}};
// The regular cube types of Sec. V-F, written as the paper prints them
// (most significant bit first).
const char* kRegularPrinted[6] = {"11001100", "00110011", "10011001",
                                  "01100110", "11110000", "00001111"};

struct I3 {
  int x, y, z;
  bool operator<(const I3& o) const {
    if (x != o.x) return x < o.x;
    if (y != o.y) return y < o.y;
    return z < o.z;
  }
  bool operator==(const I3& o) const { return x == o.x && y == o.y && z == o.z; }
};

// An edge of the lattice: it starts at voxel g and runs one step along axis
// (0=x, 1=y, 2=z).  The voxel g "owns" it (Sec. IV: each corner keeps the
// three edges e_x, e_y, e_z that start from it).
struct EdgeKey {
  int x, y, z, axis;
  bool operator<(const EdgeKey& o) const {
    if (x != o.x) return x < o.x;
    if (y != o.y) return y < o.y;
    if (z != o.z) return z < o.z;
    return axis < o.axis;
  }
  bool operator==(const EdgeKey& o) const {
    return x == o.x && y == o.y && z == o.z && axis == o.axis;
  }
};

struct Tri {
  EdgeKey e[3];
};

struct Block {
  float d[512];          // TSDF in voxel units
  float w[512];          // fusion weight
  uint8_t prev[512];     // cube type t_{i-1}
  uint8_t cur[512];      // cube type t_i (the type whose triangles exist)
};

struct Vertex {
  float t;   // edge parameter: position = owner + t * axis (voxel units)
  int ref;   // reference count = number of triangles using the vertex
  int born = 0;       // frame of the pass at whose end the count last became positive
  bool live = false;  // count positive at the end of the last pass
};

// Per-voxel record of the last fusion, kept for the backward pass.
struct FuseRec {
  double d0, w0;  // TSDF and weight before the update
  double zc;      // camera-space depth of the voxel (FP32 value promoted)
  int pixel;      // index v*W+u of the pixel the voxel projected to
  int clamped;    // 1 when the truncation at +mu was active
};

int floor_div8(int g) { return g >= 0 ? g / 8 : -((-g + 7) / 8); }

int local_index(int lx, int ly, int lz) { return lx + 8 * ly + 64 * lz; }

const int kKeyMin = -8192, kKeyMax = 8191;  // representable block coordinates

int popcount8(unsigned v) {
  int n = 0;
  for (int k = 0; k < 8; ++k) n += (v >> k) & 1u;
  return n;
}

unsigned parse_printed_type(const char* s) {
  unsigned v = 0;
  for (int i = 0; i < 8; ++i) v = (v << 1) | (unsigned)(s[i] == '1');
  return v;
}

// ---------------------------------------------------------------------------
// Marching-cubes polygons of one cube type (Sec. V-B, after Lorensen & Cline).
// The paper prints no table and no rule for ambiguous faces.  READING: each
// cube face is handled on its own.  The crossing edges of a face are joined
// by segments; on a face whose corner signs alternate, each inside corner is
// cut off by its own segment.  Every segment is directed so that, seen from
// outside the cube, the inside corner lies to its right; the segments then
// chain into closed polygons whose normals point to the outside (d > 0)
// region.  Each polygon is fanned from its lowest-numbered edge.  Because two
// cubes that share a face see the same four corner signs on it, neighbouring
// polygons meet edge for edge (no cracks).
// Built per call, on purpose: no cached table.
// ---------------------------------------------------------------------------
void edge_midpoint(int e, double m[3]) {
  for (int i = 0; i < 3; ++i)
    m[i] = 0.5 * (kCorner[kEdgeEnds[e][0]][i] + kCorner[kEdgeEnds[e][1]][i]);
}

bool edge_crosses(unsigned type, int e) {
  return ((type >> kEdgeEnds[e][0]) & 1u) != ((type >> kEdgeEnds[e][1]) & 1u);
}

// Returns false if the segments do not chain into cycles (never expected).
bool cube_polygons(unsigned type, std::vector<std::vector<int>>& polys) {
  polys.clear();
  int next[12], indeg[12];
  for (int e = 0; e < 12; ++e) next[e] = -1, indeg[e] = 0;
  for (int axis = 0; axis < 3; ++axis) {
    for (int side = 0; side < 2; ++side) {
      double n[3] = {0, 0, 0};
      n[axis] = side ? 1.0 : -1.0;  // outward normal of the face
      std::vector<int> fcorners, fedges, fcross;
      for (int k = 0; k < 8; ++k)
        if (kCorner[k][axis] == side) fcorners.push_back(k);
      for (int e = 0; e < 12; ++e)
        if (kCorner[kEdgeEnds[e][0]][axis] == side &&
            kCorner[kEdgeEnds[e][1]][axis] == side)
          fedges.push_back(e);
      for (int e : fedges)
        if (edge_crosses(type, e)) fcross.push_back(e);
      // Each segment: two face edges plus an inside corner on its inside side.
      std::vector<std::array<int, 3>> segs;
      if (fcross.size() == 2) {
        int inside = -1;
        for (int k : fcorners)
          if ((type >> k) & 1u) { inside = k; break; }
        segs.push_back({fcross[0], fcross[1], inside});
      } else if (fcross.size() == 4) {
        for (int k : fcorners) {
          if (!((type >> k) & 1u)) continue;
          int ab[2], na = 0;
          for (int e : fedges)
            if (kEdgeEnds[e][0] == k || kEdgeEnds[e][1] == k) ab[na++] = e;
          segs.push_back({ab[0], ab[1], k});
        }
      } else if (!fcross.empty()) {
        return false;
      }
      for (auto& sg : segs) {
        double a[3], b[3], x[3], u[3], v[3], c[3];
        edge_midpoint(sg[0], a);
        edge_midpoint(sg[1], b);
        for (int i = 0; i < 3; ++i) {
          x[i] = kCorner[sg[2]][i];
          u[i] = b[i] - a[i];
          v[i] = x[i] - a[i];
        }
        c[0] = u[1] * v[2] - u[2] * v[1];
        c[1] = u[2] * v[0] - u[0] * v[2];
        c[2] = u[0] * v[1] - u[1] * v[0];
        double side_of = c[0] * n[0] + c[1] * n[1] + c[2] * n[2];
        int from = side_of < 0 ? sg[0] : sg[1];
        int to = side_of < 0 ? sg[1] : sg[0];
        if (next[from] != -1) return false;
        next[from] = to;
        indeg[to]++;
      }
    }
  }
  bool seen[12] = {false};
  for (int e = 0; e < 12; ++e) {
    bool cr = edge_crosses(type, e);
    if (cr != (next[e] != -1) || cr != (indeg[e] == 1)) return false;
  }
  for (int e = 0; e < 12; ++e) {
    if (!edge_crosses(type, e) || seen[e]) continue;
    std::vector<int> poly;
    int cur = e;
    do {
      poly.push_back(cur);
      seen[cur] = true;
      cur = next[cur];
    } while (cur != e && (int)poly.size() <= 12);
    if (cur != e) return false;
    polys.push_back(poly);
  }
  return true;
}

// Triangles of a cube type as triples of cube-edge numbers.
void cube_triangles(unsigned type, std::vector<std::array<int, 3>>& tris) {
  tris.clear();
  std::vector<std::vector<int>> polys;
  cube_polygons(type, polys);
  for (auto& p : polys)
    for (size_t i = 1; i + 1 < p.size(); ++i) tris.push_back({p[0], p[i], p[i + 1]});
}

// The lattice edge a cube edge lies on: its owner is the endpoint with the
// smaller coordinate along the edge (Sec. IV: 3 edges in the cube itself,
// 9 in adjacent cubes).
EdgeKey cube_edge_key(const I3& c, int e) {
  const int* p = kCorner[kEdgeEnds[e][0]];
  const int* q = kCorner[kEdgeEnds[e][1]];
  EdgeKey k;
  int axis = 0;
  for (int i = 0; i < 3; ++i)
    if (p[i] != q[i]) axis = i;
  k.x = c.x + std::min(p[0], q[0]);
  k.y = c.y + std::min(p[1], q[1]);
  k.z = c.z + std::min(p[2], q[2]);
  k.axis = axis;
  return k;
}

// Hamming-distance refinement, Eqs. (3)-(5) of Sec. V-F.
// READINGS: t_{i-1} is the type applied at the cube's previous extraction (0
// for a cube never extracted); when several regular types qualify, keep the
// previous type if it is one of them, else take the nearest, ties broken by
// the order in which the paper lists them.
unsigned refine_type(unsigned t, unsigned prev, const float dcorner[8], float eps) {
  if (popcount8(t ^ prev) > 3) return t;
  int best = -1, best_dist = 99;
  bool prev_ok = false;
  for (int j = 0; j < 6; ++j) {
    unsigned r = parse_printed_type(kRegularPrinted[j]);
    unsigned diff = t ^ r;
    int dist = popcount8(diff);
    if (dist > 3) continue;
    bool small = true;
    for (int k = 0; k < 8; ++k)
      if (((diff >> k) & 1u) && !(std::fabs(dcorner[k]) < eps)) small = false;
    if (!small) continue;
    if (r == prev) prev_ok = true;
    if (dist < best_dist) best = j, best_dist = dist;
  }
  if (best < 0) return t;
  if (prev_ok) return prev;
  return parse_printed_type(kRegularPrinted[best]);
}

// Vertex position along its edge (Sec. V-C): linear interpolation of the
// endpoint TSDF values, which extrapolates when refinement forces a type
// whose edge endpoints share a sign.  READING: equal endpoint values give the
// edge midpoint.
template <typename T>
T edge_param(T da, T db) {
  if (da == db) return T(0.5);
  return da / (da - db);
}

// ---------------------------------------------------------------------------
// The volume.
// ---------------------------------------------------------------------------
struct Volume {
  float s;          // voxel size in metres
  float mu_v;       // truncation in voxel units
  float mu_m;       // truncation in metres, (float)(trunc_vox * s) in FP64
  float inv_s;      // (float)(1/s) in FP64
  float inv_block;  // (float)(1/(8 s)) in FP64
  float eps;        // refinement threshold in voxel units

  std::map<I3, Block> blocks;
  std::map<EdgeKey, Vertex> verts;
  std::map<I3, std::vector<Tri>> cube_tris;  // triangles held by each cube

  std::set<I3> frame_touched;    // blocks collected by the last integration
  std::set<I3> pending_touched;  // blocks touched since the last extraction
  std::set<I3> last_dirty;       // blocks processed by the last extraction

  // Optional restriction of collection to a fixed set of blocks (empty: no
  // restriction).  A block's collection and fusion depend only on the depth
  // frame and on the block's own voxels, so a restricted run computes
  // exactly what a full run computes for those blocks, at a fraction of the
  // cost: used to check sampled blocks of long sequences.
  std::set<I3> only;

  // Kept from the last integration for the backward pass.
  std::map<I3, FuseRec> fuse;
  std::vector<float> last_depth;
  int W = 0, H = 0;
  float fx = 0, fy = 0, cx = 0, cy = 0, dmin = 0, dmax = 0;
  int frame = 0;  // integrations and imports so far (the first is frame 1)

  // Threads for the loops over blocks (and pixel rows) below.  Every such
  // loop computes per block what the single-threaded loop computes, and
  // the shared maps (vertices, triangles, fusion records) are updated
  // afterwards in one thread, in the same order, so the result does not
  // depend on the thread count.
  int threads = 1;
  // Keep per-voxel fusion records for the backward pass (off: the forward
  // steps alone, for long sequences).
  bool keep_fuse = true;
};

Block* find_block(Volume& v, const I3& b) {
  auto it = v.blocks.find(b);
  return it == v.blocks.end() ? nullptr : &it->second;
}

Block* new_block(Volume& v, const I3& b) {
  Block& blk = v.blocks[b];
  for (int i = 0; i < 512; ++i) blk.d[i] = 0.f, blk.w[i] = 0.f, blk.prev[i] = 0, blk.cur[i] = 0;
  return &blk;
}

// Voxel accessor: returns false when the voxel's block is not allocated.
bool voxel(Volume& v, int gx, int gy, int gz, float& d, float& w) {
  I3 b{floor_div8(gx), floor_div8(gy), floor_div8(gz)};
  Block* blk = find_block(v, b);
  if (!blk) return false;
  int l = local_index(gx - 8 * b.x, gy - 8 * b.y, gz - 8 * b.z);
  d = blk->d[l];
  w = blk->w[l];
  return true;
}

bool depth_valid(float D, float dmin, float dmax) {
  return std::isfinite(D) && D > 0.f && D >= dmin && D <= dmax;
}

// Cube type (Sec. V-B): bit k is set when d(c_k) < 0.  READING: the cube is
// meshed only when all eight corners lie in allocated blocks and carry
// positive weight; otherwise its type is 0.
bool classify(Volume& v, const I3& c, unsigned& type, float dc[8]) {
  type = 0;
  for (int k = 0; k < 8; ++k) {
    float d, w;
    if (!voxel(v, c.x + kCorner[k][0], c.y + kCorner[k][1], c.z + kCorner[k][2], d, w))
      return false;
    if (!(w > 0.f)) return false;
    dc[k] = d;
    if (d < 0.f) type |= 1u << k;
  }
  return true;
}

float edge_t_of(Volume& v, const EdgeKey& e) {
  float da = 0, db = 0, w;
  voxel(v, e.x, e.y, e.z, da, w);
  voxel(v, e.x + (e.axis == 0), e.y + (e.axis == 1), e.z + (e.axis == 2), db, w);
  return edge_param<float>(da, db);
}

// Lazy vertex initialisation / update (Sec. V-C) for every edge the cube's
// applied type uses: the edges and their t (appended to out), then the map
// update, which creates a vertex on first use and otherwise rewrites its t.
void cube_vertices(Volume& v, const I3& c, unsigned type,
                   std::vector<std::pair<EdgeKey, float>>& out) {
  for (int e = 0; e < 12; ++e) {
    if (!edge_crosses(type, e)) continue;
    EdgeKey k = cube_edge_key(c, e);
    out.push_back({k, edge_t_of(v, k)});
  }
}

void apply_vertices(Volume& v, const std::vector<std::pair<EdgeKey, float>>& edges) {
  for (auto& kt : edges) {
    auto it = v.verts.find(kt.first);
    if (it == v.verts.end())
      v.verts[kt.first] = Vertex{kt.second, 0, 0, false};
    else
      it->second.t = kt.second;
  }
}

void touch_vertices(Volume& v, const I3& c, unsigned type) {
  std::vector<std::pair<EdgeKey, float>> edges;
  cube_vertices(v, c, type, edges);
  apply_vertices(v, edges);
}

// The triangles of a cube of the given type, as edge keys.
std::vector<Tri> cube_tri_keys(const I3& c, unsigned type) {
  std::vector<Tri> out;
  if (type == 0 || type == 255) return out;
  std::vector<std::array<int, 3>> tris;
  cube_triangles(type, tris);
  for (auto& t3 : tris) {
    Tri tr;
    for (int i = 0; i < 3; ++i) tr.e[i] = cube_edge_key(c, t3[i]);
    out.push_back(tr);
  }
  return out;
}

// Triangulation with reference counting (Sec. V-D, V-E): clear the cube's
// old triangles (-1 on their vertices) and create the new ones (+1).
void retriangulate(Volume& v, const I3& c, const std::vector<Tri>& fresh) {
  auto it = v.cube_tris.find(c);
  if (it != v.cube_tris.end()) {
    for (auto& tr : it->second)
      for (int i = 0; i < 3; ++i) v.verts[tr.e[i]].ref -= 1;
    v.cube_tris.erase(it);
  }
  if (fresh.empty()) return;
  std::vector<Tri>& out = v.cube_tris[c];
  for (const Tri& tr : fresh) {
    for (int i = 0; i < 3; ++i) v.verts[tr.e[i]].ref += 1;
    out.push_back(tr);
  }
}

void retriangulate(Volume& v, const I3& c, unsigned type) {
  retriangulate(v, c, cube_tri_keys(c, type));
}

// Birth frames (READING: the paper shows how long each vertex has been held,
// Fig. 1, without defining it): at the end of every extraction or
// refinement, a vertex whose count is positive but was not at the end of
// the previous pass (or that did not exist) is stamped with the current
// frame.  Counts are judged at pass ends only; within a pass they move
// triangle by triangle.
void stamp_births(Volume& v) {
  for (auto& kv : v.verts) {
    Vertex& x = kv.second;
    if (x.ref > 0 && !x.live) x.born = v.frame;
    x.live = x.ref > 0;
  }
}

// Extraction over a set of blocks: cube types, then vertices, then
// triangles, in the paper's order (Sec. V-B to V-D).  With refine, each new
// type goes through the Hamming refinement (Eqs. 3-5, against the type it
// replaces) before the vertices and triangles are made from it: Sec. V-F
// applies the regular type before marching cubes.  The per-block work of
// each step (types; edge keys and t of the vertices to create or update;
// triangles of changed cubes) runs over blocks in parallel, and the
// vertex and triangle maps are then updated in one thread in block, cube
// and edge order.
void extract_blocks(Volume& v, const std::set<I3>& dirty, bool refine) {
  const std::vector<I3> list(dirty.begin(), dirty.end());
  const long n = (long)list.size();
#pragma omp parallel for schedule(dynamic, 4) num_threads(v.threads)
  for (long i = 0; i < n; ++i) {
    const I3& b = list[i];
    Block* blk = find_block(v, b);
    for (int l = 0; l < 512; ++l) {
      I3 c{8 * b.x + (l & 7), 8 * b.y + ((l >> 3) & 7), 8 * b.z + (l >> 6)};
      unsigned type;
      float dc[8];
      bool valid = classify(v, c, type, dc);
      blk->prev[l] = blk->cur[l];
      if (valid && refine) type = refine_type(type, blk->prev[l], dc, v.eps);
      blk->cur[l] = valid ? (uint8_t)type : 0;
    }
  }
  // vertices of every meshed cube: (edge, t) per block, then the map
  std::vector<std::vector<std::pair<EdgeKey, float>>> touch(list.size());
#pragma omp parallel for schedule(dynamic, 4) num_threads(v.threads)
  for (long i = 0; i < n; ++i) {
    const I3& b = list[i];
    Block* blk = find_block(v, b);
    for (int l = 0; l < 512; ++l) {
      if (!blk->cur[l]) continue;
      I3 c{8 * b.x + (l & 7), 8 * b.y + ((l >> 3) & 7), 8 * b.z + (l >> 6)};
      cube_vertices(v, c, blk->cur[l], touch[i]);
    }
  }
  for (auto& per_block : touch) apply_vertices(v, per_block);
  // triangles of cubes whose type changed (t_i != t_{i-1}); the others keep
  // theirs
  std::vector<std::vector<std::pair<I3, std::vector<Tri>>>> tris(list.size());
#pragma omp parallel for schedule(dynamic, 4) num_threads(v.threads)
  for (long i = 0; i < n; ++i) {
    const I3& b = list[i];
    Block* blk = find_block(v, b);
    for (int l = 0; l < 512; ++l) {
      if (blk->cur[l] == blk->prev[l]) continue;  // t_i == t_{i-1}: keep
      I3 c{8 * b.x + (l & 7), 8 * b.y + ((l >> 3) & 7), 8 * b.z + (l >> 6)};
      tris[i].push_back({c, cube_tri_keys(c, blk->cur[l])});
    }
  }
  for (auto& per_block : tris)
    for (auto& ct : per_block) retriangulate(v, ct.first, ct.second);
  v.last_dirty = dirty;
}

void check_block_keys(const I3& b, bool& ok) {
  ok = b.x >= kKeyMin && b.x <= kKeyMax && b.y >= kKeyMin && b.y <= kKeyMax &&
       b.z >= kKeyMin && b.z <= kKeyMax;
}

}  // namespace

// ===========================================================================
// C interface (loaded by the tests through ctypes).
// ===========================================================================
extern "C" {

void* orc_create(float voxel_m, float trunc_vox, float refine_eps_vox) {
  Volume* v = new Volume();
  v->s = voxel_m;
  v->mu_v = trunc_vox;
  v->mu_m = (float)((double)trunc_vox * (double)voxel_m);
  v->inv_s = (float)(1.0 / (double)voxel_m);
  v->inv_block = (float)(1.0 / (8.0 * (double)voxel_m));
  v->eps = refine_eps_vox;
  return v;
}

void orc_destroy(void* h) { delete (Volume*)h; }

// Threads of the loops over blocks (1: single-threaded; results do not depend
// on it) and whether fusion keeps per-voxel records for the backward pass.
void orc_set_threads(void* h, int n) { ((Volume*)h)->threads = n < 1 ? 1 : n; }
void orc_keep_fusion(void* h, int on) { ((Volume*)h)->keep_fuse = on != 0; }

// Block collection (Eq. 1) and TSDF fusion (Eq. 2) of one depth frame.
// depth: H*W metres, row-major; cam_to_world: 4x4 row-major FP32 pose.
// READINGS: the band lambda in [1-delta, 1+delta] is taken as camera depth
// z in [D-mu, D+mu]; every block in the integer box spanned by the two band
// end points is collected.  Fusion follows the running weighted average of
// KinectFusion with unit weight per observation, the nearest pixel, the
// projective distance, skip behind -mu and clamp at +mu.
// Returns the number of collected blocks.
int orc_integrate(void* h, const float* depth, int W, int H, float fx, float fy,
                  float cx, float cy, float dmin, float dmax, const float* T) {
  Volume& v = *(Volume*)h;
  ++v.frame;
  float Rcw[3][3], tcw[3], Rwc[3][3], twc[3];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) Rcw[i][j] = T[4 * i + j];
    tcw[i] = T[4 * i + 3];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Rwc[i][j] = Rcw[j][i];
  for (int i = 0; i < 3; ++i) {
    double acc = (double)Rcw[0][i] * (double)tcw[0];
    acc = acc + (double)Rcw[1][i] * (double)tcw[1];
    acc = acc + (double)Rcw[2][i] * (double)tcw[2];
    twc[i] = (float)(-acc);
  }
  v.W = W, v.H = H, v.fx = fx, v.fy = fy, v.cx = cx, v.cy = cy, v.dmin = dmin, v.dmax = dmax;
  v.last_depth.assign(depth, depth + (size_t)W * H);

  // --- block collection (pixel rows in parallel, each into its own set) ---
  std::set<I3> touched;
#pragma omp parallel num_threads(v.threads)
  {
    std::set<I3> mine;
#pragma omp for schedule(static)
    for (int py = 0; py < H; ++py) {
      for (int px = 0; px < W; ++px) {
        float D = depth[(size_t)py * W + px];
        if (!depth_valid(D, dmin, dmax)) continue;
        float xn = ((float)px - cx) / fx;
        float yn = ((float)py - cy) / fy;
        int bmin[3], bmax[3];
        bool in_range = true;
        for (int end = 0; end < 2; ++end) {
          float z = end == 0 ? D - v.mu_m : D + v.mu_m;
          float p[3] = {xn * z, yn * z, z};
          for (int i = 0; i < 3; ++i) {
            float P = Rcw[i][0] * p[0];
            P = P + Rcw[i][1] * p[1];
            P = P + Rcw[i][2] * p[2];
            P = P + tcw[i];
            float fb = std::floor(P * v.inv_block);
            if (!(fb >= (float)kKeyMin && fb <= (float)kKeyMax)) { in_range = false; break; }
            int b = (int)fb;
            if (end == 0) bmin[i] = bmax[i] = b;
            else bmin[i] = std::min(bmin[i], b), bmax[i] = std::max(bmax[i], b);
          }
          if (!in_range) break;
        }
        if (!in_range) continue;
        for (int bz = bmin[2]; bz <= bmax[2]; ++bz)
          for (int by = bmin[1]; by <= bmax[1]; ++by)
            for (int bx = bmin[0]; bx <= bmax[0]; ++bx) {
              const I3 b{bx, by, bz};
              if (v.only.empty() || v.only.count(b)) mine.insert(b);
            }
      }
    }
#pragma omp critical
    touched.insert(mine.begin(), mine.end());
  }
  for (const I3& b : touched)
    if (!find_block(v, b)) new_block(v, b);

  // --- fusion (blocks in parallel; each voxel's update is its own) ---
  v.fuse.clear();
  const std::vector<I3> list(touched.begin(), touched.end());
  const long n = (long)list.size();
  std::vector<std::vector<std::pair<I3, FuseRec>>> recs(v.keep_fuse ? list.size() : 0);
#pragma omp parallel for schedule(dynamic, 4) num_threads(v.threads)
  for (long i = 0; i < n; ++i) {
    const I3& b = list[i];
    Block* blk = find_block(v, b);
    for (int l = 0; l < 512; ++l) {
      int gx = 8 * b.x + (l & 7), gy = 8 * b.y + ((l >> 3) & 7), gz = 8 * b.z + (l >> 6);
      float X = (float)gx * v.s, Y = (float)gy * v.s, Z = (float)gz * v.s;
      float xc[3];
      for (int j = 0; j < 3; ++j) {
        float a = Rwc[j][0] * X;
        a = a + Rwc[j][1] * Y;
        a = a + Rwc[j][2] * Z;
        a = a + twc[j];
        xc[j] = a;
      }
      if (!(xc[2] > 0.f)) continue;
      float u = fx * (xc[0] / xc[2]) + cx;
      float vv = fy * (xc[1] / xc[2]) + cy;
      float fu = std::floor(u + 0.5f), fv = std::floor(vv + 0.5f);
      if (!(fu >= 0.f && fu < (float)W && fv >= 0.f && fv < (float)H)) continue;
      int ui = (int)fu, vi = (int)fv;
      float D = depth[(size_t)vi * W + ui];
      if (!depth_valid(D, dmin, dmax)) continue;
      float sdf = (D - xc[2]) * v.inv_s;
      if (sdf < -v.mu_v) continue;
      float dt = std::fmin(sdf, v.mu_v);
      if (v.keep_fuse)
        recs[i].push_back({I3{gx, gy, gz}, FuseRec{(double)blk->d[l], (double)blk->w[l],
                                                   (double)xc[2], vi * W + ui,
                                                   sdf >= v.mu_v ? 1 : 0}});
      float num = blk->d[l] * blk->w[l];
      num = num + dt;
      float den = blk->w[l] + 1.0f;
      blk->d[l] = num / den;
      blk->w[l] = den;
    }
  }
  for (auto& per_block : recs)
    for (auto& r : per_block) v.fuse[r.first] = r.second;
  v.frame_touched = touched;
  v.pending_touched.insert(touched.begin(), touched.end());
  return (int)touched.size();
}

// Restrict block collection of later integrations to the n given blocks
// (n = 0 lifts the restriction).
void orc_restrict_blocks(void* h, const int* coords, int n) {
  Volume& v = *(Volume*)h;
  v.only.clear();
  for (int i = 0; i < n; ++i) v.only.insert(I3{coords[3 * i], coords[3 * i + 1], coords[3 * i + 2]});
}

// Allocate blocks and set their TSDF/weights directly (used for synthetic
// volumes that are sampled rather than fused).  coords: n*3 block coordinates;
// d, w: n*512 values in local order x + 8y + 64z.  The blocks count as
// touched for the next extraction.
int orc_import_blocks(void* h, const int* coords, const float* d, const float* w, int n) {
  Volume& v = *(Volume*)h;
  ++v.frame;
  std::set<I3> touched;
  for (int i = 0; i < n; ++i) {
    I3 b{coords[3 * i], coords[3 * i + 1], coords[3 * i + 2]};
    bool ok;
    check_block_keys(b, ok);
    if (!ok) return -1;
    Block* blk = find_block(v, b);
    if (!blk) blk = new_block(v, b);
    for (int l = 0; l < 512; ++l) blk->d[l] = d[(size_t)i * 512 + l], blk->w[l] = w[(size_t)i * 512 + l];
    touched.insert(b);
  }
  v.frame_touched = touched;
  v.pending_touched.insert(touched.begin(), touched.end());
  v.fuse.clear();
  return n;
}

// Mesh extraction.  scope 0: the blocks touched since the last extraction
// (by integrations or imports) plus their allocated neighbours in the -x/-y/-z directions (the
// cubes whose corners moved); scope 1: every allocated block.
static int extract_scope(Volume& v, int scope, bool refine) {
  std::set<I3> dirty;
  if (scope == 1) {
    for (auto& kv : v.blocks) dirty.insert(kv.first);
  } else {
    for (const I3& b : v.pending_touched)
      for (int dz = -1; dz <= 0; ++dz)
        for (int dy = -1; dy <= 0; ++dy)
          for (int dx = -1; dx <= 0; ++dx) {
            I3 nb{b.x + dx, b.y + dy, b.z + dz};
            if (find_block(v, nb)) dirty.insert(nb);
          }
  }
  extract_blocks(v, dirty, refine);
  v.pending_touched.clear();
  stamp_births(v);
  return (int)dirty.size();
}

int orc_extract(void* h, int scope) { return extract_scope(*(Volume*)h, scope, false); }

// Extraction with the refinement applied to each new type before its
// vertices and triangles are made (Sec. V-F).  Types, vertices, t and
// triangles end as after orc_extract followed by orc_refine; a vertex the
// unrefined types would have dropped and the refined ones keep is never
// dropped, so it keeps its birth frame.
int orc_extract_refine(void* h, int scope) { return extract_scope(*(Volume*)h, scope, true); }

// Hamming refinement (Eqs. 3-5) over the cubes of the last extraction.
// Returns the number of cubes whose type changed.
int orc_refine(void* h) {
  Volume& v = *(Volume*)h;
  // the applied types of the last extraction's cubes, blocks in parallel
  const std::vector<I3> list(v.last_dirty.begin(), v.last_dirty.end());
  const long n = (long)list.size();
  std::vector<std::vector<std::pair<I3, unsigned>>> per_block(list.size());
#pragma omp parallel for schedule(dynamic, 4) num_threads(v.threads)
  for (long i = 0; i < n; ++i) {
    const I3& b = list[i];
    Block* blk = find_block(v, b);
    for (int l = 0; l < 512; ++l) {
      I3 c{8 * b.x + (l & 7), 8 * b.y + ((l >> 3) & 7), 8 * b.z + (l >> 6)};
      unsigned raw;
      float dc[8];
      if (!classify(v, c, raw, dc)) continue;
      unsigned a = refine_type(blk->cur[l], blk->prev[l], dc, v.eps);
      if (a != blk->cur[l]) per_block[i].push_back({c, a});
    }
  }
  std::vector<std::pair<I3, unsigned>> changed;
  for (auto& pb : per_block) changed.insert(changed.end(), pb.begin(), pb.end());
  for (auto& ca : changed) touch_vertices(v, ca.first, ca.second);
  for (auto& ca : changed) {
    const I3& c = ca.first;
    I3 b{floor_div8(c.x), floor_div8(c.y), floor_div8(c.z)};
    Block* blk = find_block(v, b);
    blk->cur[local_index(c.x - 8 * b.x, c.y - 8 * b.y, c.z - 8 * b.z)] = (uint8_t)ca.second;
    retriangulate(v, c, ca.second);
  }
  stamp_births(v);
  return (int)changed.size();
}

void orc_export_births(void* h, int* out) {
  Volume& v = *(Volume*)h;
  size_t i = 0;
  for (auto& kv : v.verts)
    if (kv.second.ref > 0) out[i++] = kv.second.born;
}

// Garbage collection (Sec. V-E): vertices no triangle references are freed.
int orc_gc(void* h) {
  Volume& v = *(Volume*)h;
  int freed = 0;
  for (auto it = v.verts.begin(); it != v.verts.end();) {
    if (it->second.ref == 0) {
      it = v.verts.erase(it);
      ++freed;
    } else {
      ++it;
    }
  }
  return freed;
}

// ----- inspection ----------------------------------------------------------
int orc_num_blocks(void* h) { return (int)((Volume*)h)->blocks.size(); }

void orc_export_blocks(void* h, int* coords, float* d, float* w, uint8_t* prev, uint8_t* cur) {
  Volume& v = *(Volume*)h;
  size_t i = 0;
  for (auto& kv : v.blocks) {
    coords[3 * i] = kv.first.x, coords[3 * i + 1] = kv.first.y, coords[3 * i + 2] = kv.first.z;
    if (d) std::memcpy(d + 512 * i, kv.second.d, sizeof(float) * 512);
    if (w) std::memcpy(w + 512 * i, kv.second.w, sizeof(float) * 512);
    if (prev) std::memcpy(prev + 512 * i, kv.second.prev, 512);
    if (cur) std::memcpy(cur + 512 * i, kv.second.cur, 512);
    ++i;
  }
}

// which: 0 = blocks collected by the last integration, 1 = blocks processed
// by the last extraction, 2 = blocks touched since the last extraction.
const std::set<I3>& block_set(Volume& v, int which) {
  return which == 0 ? v.frame_touched : which == 1 ? v.last_dirty : v.pending_touched;
}

int orc_num_set(void* h, int which) { return (int)block_set(*(Volume*)h, which).size(); }

void orc_export_set(void* h, int which, int* coords) {
  Volume& v = *(Volume*)h;
  const std::set<I3>& s = block_set(v, which);
  size_t i = 0;
  for (const I3& b : s) coords[3 * i] = b.x, coords[3 * i + 1] = b.y, coords[3 * i + 2] = b.z, ++i;
}

// live_only: 1 = vertices with a positive reference count.
int orc_num_vertices(void* h, int live_only) {
  Volume& v = *(Volume*)h;
  int n = 0;
  for (auto& kv : v.verts) n += (!live_only || kv.second.ref > 0);
  return n;
}

void orc_export_vertices(void* h, int live_only, int* keys, float* t, int* ref) {
  Volume& v = *(Volume*)h;
  size_t i = 0;
  for (auto& kv : v.verts) {
    if (live_only && kv.second.ref <= 0) continue;
    keys[4 * i] = kv.first.x, keys[4 * i + 1] = kv.first.y, keys[4 * i + 2] = kv.first.z,
    keys[4 * i + 3] = kv.first.axis;
    t[i] = kv.second.t;
    ref[i] = kv.second.ref;
    ++i;
  }
}

int orc_num_triangles(void* h) {
  Volume& v = *(Volume*)h;
  size_t n = 0;
  for (auto& kv : v.cube_tris) n += kv.second.size();
  return (int)n;
}

// Triangles as triples of edge keys (n*3*4 ints), cube by cube.
void orc_export_triangles(void* h, int* keys) {
  Volume& v = *(Volume*)h;
  size_t i = 0;
  for (auto& kv : v.cube_tris)
    for (auto& tr : kv.second) {
      for (int j = 0; j < 3; ++j) {
        int* k = keys + 12 * i + 4 * j;
        k[0] = tr.e[j].x, k[1] = tr.e[j].y, k[2] = tr.e[j].z, k[3] = tr.e[j].axis;
      }
      ++i;
    }
}

// Mesh download (vertices in metres, triangles as indices into them), the
// live vertices in edge-key order.
void orc_download(void* h, float* verts, int* tris) {
  Volume& v = *(Volume*)h;
  std::map<EdgeKey, int> index;
  int n = 0;
  for (auto& kv : v.verts) {
    if (kv.second.ref <= 0) continue;
    const EdgeKey& k = kv.first;
    int g[3] = {k.x, k.y, k.z};
    for (int i = 0; i < 3; ++i) {
      float c = (float)g[i];
      if (i == k.axis) c = c + kv.second.t;
      verts[3 * n + i] = c * v.s;
    }
    index[k] = n++;
  }
  size_t i = 0;
  for (auto& kv : v.cube_tris)
    for (auto& tr : kv.second) {
      for (int j = 0; j < 3; ++j) tris[3 * i + j] = index[tr.e[j]];
      ++i;
    }
}

// Triangles of one cube type as cube-edge numbers (up to 5 x 3 ints).
// Returns the triangle count, or -1 when the face segments do not close.
int orc_cube_triangles(int type, int* out) {
  std::vector<std::vector<int>> polys;
  if (!cube_polygons((unsigned)type, polys)) return -1;
  std::vector<std::array<int, 3>> tris;
  cube_triangles((unsigned)type, tris);
  for (size_t i = 0; i < tris.size(); ++i)
    for (int j = 0; j < 3; ++j) out[3 * i + j] = tris[i][j];
  return (int)tris.size();
}

// Polygons of one cube type: sizes[i] edges each, concatenated in `edges`
// (at most 12 entries).  Returns the polygon count.
int orc_cube_polygons(int type, int* sizes, int* edges) {
  std::vector<std::vector<int>> polys;
  if (!cube_polygons((unsigned)type, polys)) return -1;
  int n = 0;
  for (size_t i = 0; i < polys.size(); ++i) {
    sizes[i] = (int)polys[i].size();
    for (int e : polys[i]) edges[n++] = e;
  }
  return (int)polys.size();
}

// Polygon sizes of one cube type (up to 4 polygons); returns their count.
int orc_cube_polygon_sizes(int type, int* sizes) {
  std::vector<std::vector<int>> polys;
  if (!cube_polygons((unsigned)type, polys)) return -1;
  for (size_t i = 0; i < polys.size(); ++i) sizes[i] = (int)polys[i].size();
  return (int)polys.size();
}

int orc_refine_type(int t, int prev, const float* dcorner, float eps) {
  return (int)refine_type((unsigned)t, (unsigned)prev, dcorner, eps);
}

int orc_regular_type(int j) { return (int)parse_printed_type(kRegularPrinted[j]); }

void orc_corner_offsets(int* out) {
  for (int k = 0; k < 8; ++k)
    for (int i = 0; i < 3; ++i) out[3 * k + i] = kCorner[k][i];
}

void orc_edge_ends(int* out) {
  for (int e = 0; e < 12; ++e) out[2 * e] = kEdgeEnds[e][0], out[2 * e + 1] = kEdgeEnds[e][1];
}

// ----- FP64 twin for gradients (connectivity held fixed) --------------------
// Voxels are addressed through the block export order; a voxel outside the
// allocated blocks reads as 0.

// Analytic dL/dd at every voxel of every block (export order, n*512),
// given dL/dv for the live vertices (export order, n_live*3, metres).
// dv/dt = s * axis; dt/dd_a = -d_b/(d_a-d_b)^2, dt/dd_b = d_a/(d_a-d_b)^2.
void orc_grad_tsdf64(void* h, const double* dL_dv, double* out) {
  Volume& v = *(Volume*)h;
  std::map<I3, size_t> bidx;
  size_t nb = 0;
  for (auto& kv : v.blocks) bidx[kv.first] = nb++;
  std::memset(out, 0, sizeof(double) * 512 * nb);
  auto add = [&](int gx, int gy, int gz, double val) {
    I3 b{floor_div8(gx), floor_div8(gy), floor_div8(gz)};
    auto it = bidx.find(b);
    if (it == bidx.end()) return;
    out[512 * it->second + local_index(gx - 8 * b.x, gy - 8 * b.y, gz - 8 * b.z)] += val;
  };
  size_t i = 0;
  for (auto& kv : v.verts) {
    if (kv.second.ref <= 0) continue;
    const EdgeKey& k = kv.first;
    float fa = 0, fb = 0, w;
    int ox = k.axis == 0, oy = k.axis == 1, oz = k.axis == 2;
    voxel(v, k.x, k.y, k.z, fa, w);
    voxel(v, k.x + ox, k.y + oy, k.z + oz, fb, w);
    double da = fa, db = fb;
    double g = dL_dv[3 * i + k.axis] * (double)v.s;
    if (da != db) {
      double den = (da - db) * (da - db);
      add(k.x, k.y, k.z, g * (-db / den));
      add(k.x + ox, k.y + oy, k.z + oz, g * (da / den));
    }
    ++i;
  }
}

// FP64 positions (metres, n_live*3) of the live vertices with the TSDF at
// voxel (gx,gy,gz) shifted by delta voxel units.
void orc_positions64(void* h, int gx, int gy, int gz, double delta, double* pos) {
  Volume& v = *(Volume*)h;
  size_t i = 0;
  for (auto& kv : v.verts) {
    if (kv.second.ref <= 0) continue;
    const EdgeKey& k = kv.first;
    int ox = k.axis == 0, oy = k.axis == 1, oz = k.axis == 2;
    float fa = 0, fb = 0, w;
    voxel(v, k.x, k.y, k.z, fa, w);
    voxel(v, k.x + ox, k.y + oy, k.z + oz, fb, w);
    double da = fa, db = fb;
    if (k.x == gx && k.y == gy && k.z == gz) da += delta;
    if (k.x + ox == gx && k.y + oy == gy && k.z + oz == gz) db += delta;
    double t = edge_param<double>(da, db);
    int g[3] = {k.x, k.y, k.z};
    for (int j = 0; j < 3; ++j) pos[3 * i + j] = ((double)g[j] + (j == k.axis ? t : 0.0)) * (double)v.s;
    ++i;
  }
}

// Vertex normals.  READING: Sec. IV keeps a normal in every vertex record
// but does not say how it is formed.  Here: the TSDF gradient at a voxel by
// central differences over observed neighbours (allocated block, weight >
// 0), per axis (d(x+e) - d(x-e)) / 2, one-sided d(x+e) - d(x) or
// d(x) - d(x-e) when only one neighbour is observed, 0 when neither is; the
// gradient is interpolated along the vertex's edge at its parameter t (the
// stored FP32 value) and normalised, 0 when it vanishes.  It points to
// increasing TSDF, the outside of the surface.  out: n_live*3, key order;
// len: the length before normalisation, n_live.
static void tsdf_gradient64(Volume& v, int gx, int gy, int gz, double g[3]) {
  float d0 = 0, w0 = 0;
  voxel(v, gx, gy, gz, d0, w0);
  for (int i = 0; i < 3; ++i) {
    const int ex = i == 0, ey = i == 1, ez = i == 2;
    float dp = 0, wp = 0, dm = 0, wm = 0;
    const bool hp = voxel(v, gx + ex, gy + ey, gz + ez, dp, wp) && wp > 0.f;
    const bool hm = voxel(v, gx - ex, gy - ey, gz - ez, dm, wm) && wm > 0.f;
    if (hp && hm) g[i] = ((double)dp - (double)dm) / 2.0;
    else if (hp) g[i] = (double)dp - (double)d0;
    else if (hm) g[i] = (double)d0 - (double)dm;
    else g[i] = 0.0;
  }
}

void orc_normals64(void* h, double* out, double* len) {
  Volume& v = *(Volume*)h;
  size_t i = 0;
  for (auto& kv : v.verts) {
    if (kv.second.ref <= 0) continue;
    const EdgeKey& k = kv.first;
    const int ox = k.axis == 0, oy = k.axis == 1, oz = k.axis == 2;
    double g0[3], g1[3], n[3];
    tsdf_gradient64(v, k.x, k.y, k.z, g0);
    tsdf_gradient64(v, k.x + ox, k.y + oy, k.z + oz, g1);
    const double t = kv.second.t;
    for (int j = 0; j < 3; ++j) n[j] = (1.0 - t) * g0[j] + t * g1[j];
    const double l = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int j = 0; j < 3; ++j) out[3 * i + j] = l > 0.0 ? n[j] / l : 0.0;
    len[i] = l;
    ++i;
  }
}

// Backward of the last fusion (Eq. 2), all branches held fixed.
// dL_dd1: dL/d(fused TSDF), block export order (n*512).  Writes dL/d(TSDF
// before fusion) in the same order and dL/dD for every pixel (H*W).
// Updated voxel: d1 = (d0*W0 + dt)/(W0+1); unclamped dt = (D - z)/s.
void orc_grad_fusion64(void* h, const double* dL_dd1, double* dL_dd0, double* dL_dD) {
  Volume& v = *(Volume*)h;
  std::memset(dL_dD, 0, sizeof(double) * (size_t)v.W * v.H);
  size_t bi = 0;
  double inv_s = 1.0 / (double)v.s;
  for (auto& kv : v.blocks) {
    const I3& b = kv.first;
    for (int l = 0; l < 512; ++l) {
      size_t idx = 512 * bi + l;
      I3 g{8 * b.x + (l & 7), 8 * b.y + ((l >> 3) & 7), 8 * b.z + (l >> 6)};
      auto it = v.fuse.find(g);
      if (it == v.fuse.end()) {
        dL_dd0[idx] = dL_dd1[idx];
        continue;
      }
      const FuseRec& r = it->second;
      dL_dd0[idx] = dL_dd1[idx] * (r.w0 / (r.w0 + 1.0));
      if (!r.clamped) dL_dD[r.pixel] += dL_dd1[idx] * (inv_s / (r.w0 + 1.0));
    }
    ++bi;
  }
}

// FP64 positions of the live vertices with depth pixel `pixel` of the last
// fused frame shifted by delta metres; the TSDF of every voxel that fused
// this pixel is recomputed in FP64 with its branches held fixed.
void orc_positions64_depth(void* h, int pixel, double delta, double* pos) {
  Volume& v = *(Volume*)h;
  auto dval = [&](int gx, int gy, int gz) -> double {
    float d = 0, w;
    voxel(v, gx, gy, gz, d, w);
    auto it = v.fuse.find(I3{gx, gy, gz});
    if (it == v.fuse.end() || it->second.pixel != pixel) return (double)d;
    const FuseRec& r = it->second;
    double D = (double)v.last_depth[pixel] + delta;
    double dt = r.clamped ? (double)v.mu_v : (D - r.zc) / (double)v.s;
    return (r.d0 * r.w0 + dt) / (r.w0 + 1.0);
  };
  size_t i = 0;
  for (auto& kv : v.verts) {
    if (kv.second.ref <= 0) continue;
    const EdgeKey& k = kv.first;
    int ox = k.axis == 0, oy = k.axis == 1, oz = k.axis == 2;
    double da = dval(k.x, k.y, k.z), db = dval(k.x + ox, k.y + oy, k.z + oz);
    double t = edge_param<double>(da, db);
    int g[3] = {k.x, k.y, k.z};
    for (int j = 0; j < 3; ++j) pos[3 * i + j] = ((double)g[j] + (j == k.axis ? t : 0.0)) * (double)v.s;
    ++i;
  }
}

// Fusion records of the last integration: n voxels, each (gx,gy,gz,pixel,
// clamped) plus (d0, w0).
int orc_num_fused(void* h) { return (int)((Volume*)h)->fuse.size(); }

void orc_export_fused(void* h, int* ints, double* vals) {
  Volume& v = *(Volume*)h;
  size_t i = 0;
  for (auto& kv : v.fuse) {
    int* p = ints + 5 * i;
    p[0] = kv.first.x, p[1] = kv.first.y, p[2] = kv.first.z, p[3] = kv.second.pixel,
    p[4] = kv.second.clamped;
    vals[2 * i] = kv.second.d0, vals[2 * i + 1] = kv.second.w0;
    ++i;
  }
}

}  // extern "C"
