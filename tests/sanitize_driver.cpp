// Test driver for the oracle under AddressSanitizer and UndefinedBehavior-
// Sanitizer (CPU only).  It is compiled together with oracle/oracle.cpp by
// tests/test_oracle_sanitizers.py and runs every C entry point of the oracle
// on small synthetic inputs made here: a sampled sphere TSDF imported as
// blocks, a depth frame of a tilted plane fused twice from two poses (one
// thread, then eight), extraction, refinement, garbage collection, the
// exports, the FP64 gradients and the table helpers.  Any sanitizer report
// ends the run with a nonzero status.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
void* orc_create(float voxel_m, float trunc_vox, float refine_eps_vox);
void orc_destroy(void* h);
void orc_set_threads(void* h, int n);
void orc_keep_fusion(void* h, int on);
int orc_integrate(void* h, const float* depth, int W, int H, float fx, float fy, float cx,
                  float cy, float dmin, float dmax, const float* T);
void orc_restrict_blocks(void* h, const int* coords, int n);
int orc_import_blocks(void* h, const int* coords, const float* d, const float* w, int n);
int orc_extract(void* h, int scope);
int orc_refine(void* h);
int orc_gc(void* h);
void orc_export_births(void* h, int* out);
int orc_num_blocks(void* h);
void orc_export_blocks(void* h, int* coords, float* d, float* w, uint8_t* prev, uint8_t* cur);
int orc_num_set(void* h, int which);
void orc_export_set(void* h, int which, int* coords);
int orc_num_vertices(void* h, int live_only);
void orc_export_vertices(void* h, int live_only, int* keys, float* t, int* ref);
int orc_num_triangles(void* h);
void orc_export_triangles(void* h, int* keys);
void orc_download(void* h, float* verts, int* tris);
int orc_cube_triangles(int type, int* out);
int orc_cube_polygons(int type, int* sizes, int* edges);
int orc_cube_polygon_sizes(int type, int* sizes);
int orc_refine_type(int t, int prev, const float* dcorner, float eps);
int orc_regular_type(int j);
void orc_corner_offsets(int* out);
void orc_edge_ends(int* out);
void orc_grad_tsdf64(void* h, const double* dL_dv, double* out);
void orc_positions64(void* h, int gx, int gy, int gz, double delta, double* pos);
void orc_normals64(void* h, double* out, double* len);
void orc_grad_fusion64(void* h, const double* dL_dd1, double* dL_dd0, double* dL_dD);
void orc_positions64_depth(void* h, int pixel, double delta, double* pos);
int orc_num_fused(void* h);
void orc_export_fused(void* h, int* ints, double* vals);
}

namespace {

int fail(const char* what) {
  std::fprintf(stderr, "sanitize driver: %s\n", what);
  return 1;
}

// Every export of a volume, into buffers of exactly the reported sizes.
int exercise_exports(void* h) {
  const int nb = orc_num_blocks(h);
  std::vector<int> coords(3 * (size_t)nb);
  std::vector<float> d(512 * (size_t)nb), w(512 * (size_t)nb);
  std::vector<uint8_t> prev(512 * (size_t)nb), cur(512 * (size_t)nb);
  orc_export_blocks(h, coords.data(), d.data(), w.data(), prev.data(), cur.data());
  for (int which = 0; which < 3; ++which) {
    std::vector<int> s(3 * (size_t)orc_num_set(h, which) + 1);
    orc_export_set(h, which, s.data());
  }
  for (int live = 0; live < 2; ++live) {
    const int nv = orc_num_vertices(h, live);
    std::vector<int> keys(4 * (size_t)nv + 1), ref((size_t)nv + 1);
    std::vector<float> t((size_t)nv + 1);
    orc_export_vertices(h, live, keys.data(), t.data(), ref.data());
  }
  const int nv = orc_num_vertices(h, 1), nt = orc_num_triangles(h);
  std::vector<int> tkeys(12 * (size_t)nt + 1), tris(3 * (size_t)nt + 1), births((size_t)nv + 1);
  std::vector<float> verts(3 * (size_t)nv + 1);
  orc_export_triangles(h, tkeys.data());
  orc_download(h, verts.data(), tris.data());
  orc_export_births(h, births.data());
  for (int i = 0; i < 3 * nt; ++i)
    if (tris[i] < 0 || tris[i] >= nv) return fail("triangle index out of range");
  std::vector<double> n3(3 * (size_t)nv + 1), len((size_t)nv + 1), p3(3 * (size_t)nv + 1);
  orc_normals64(h, n3.data(), len.data());
  std::vector<double> g(3 * (size_t)nv + 1, 1.0), out(512 * (size_t)nb + 1);
  orc_grad_tsdf64(h, g.data(), out.data());
  orc_positions64(h, 0, 0, 0, 1e-6, p3.data());
  return 0;
}

int sphere_import(int threads) {
  void* h = orc_create(0.02f, 4.f, 0.5f);
  orc_set_threads(h, threads);
  const int nb = 3;
  std::vector<int> coords;
  std::vector<float> d, w;
  for (int bz = 0; bz < nb; ++bz)
    for (int by = 0; by < nb; ++by)
      for (int bx = 0; bx < nb; ++bx) {
        coords.insert(coords.end(), {bx, by, bz});
        for (int l = 0; l < 512; ++l) {
          const double x = 8 * bx + (l & 7) - 11.3, y = 8 * by + ((l >> 3) & 7) - 12.1,
                       z = 8 * bz + (l >> 6) - 11.7;
          const double s = std::sqrt(x * x + y * y + z * z) - 7.5;
          d.push_back((float)std::fmax(-4.0, std::fmin(4.0, s)));
          w.push_back((l % 97) == 5 ? 0.f : 1.f);  // a few unobserved voxels
        }
      }
  if (orc_import_blocks(h, coords.data(), d.data(), w.data(), nb * nb * nb) < 0)
    return fail("import");
  orc_extract(h, 1);
  orc_refine(h);
  orc_gc(h);
  if (orc_num_triangles(h) == 0) return fail("no triangles");
  int r = exercise_exports(h);
  // a second import over part of the volume, then an incremental pass
  for (float& x : d) x = -x;
  if (orc_import_blocks(h, coords.data(), d.data(), w.data(), 5) < 0) return fail("import 2");
  orc_extract(h, 0);
  orc_gc(h);
  r |= exercise_exports(h);
  orc_destroy(h);
  return r;
}

int plane_fusion(int threads) {
  const int W = 64, H = 48;
  const float fx = 50.f, fy = 50.f, cx = 31.5f, cy = 23.5f;
  void* h = orc_create(0.02f, 4.f, 0.5f);
  orc_set_threads(h, threads);
  std::vector<float> depth((size_t)W * H);
  for (int frame = 0; frame < 2; ++frame) {
    for (int v = 0; v < H; ++v)
      for (int u = 0; u < W; ++u) {
        float z = 0.8f + 0.004f * (float)u + 0.002f * (float)v + 0.01f * (float)frame;
        if ((u * 7 + v * 3) % 29 == 0) z = 0.f;  // holes
        depth[(size_t)v * W + u] = z;
      }
    const float T[16] = {1, 0, 0, 0.01f * (float)frame, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
    orc_integrate(h, depth.data(), W, H, fx, fy, cx, cy, 0.1f, 5.f, T);
    const int nf = orc_num_fused(h);
    std::vector<int> ints(5 * (size_t)nf + 1);
    std::vector<double> vals(2 * (size_t)nf + 1);
    orc_export_fused(h, ints.data(), vals.data());
    orc_extract(h, 0);
    orc_refine(h);
    orc_gc(h);
  }
  if (orc_num_vertices(h, 1) == 0) return fail("plane: no vertices");
  int r = exercise_exports(h);
  const int nb = orc_num_blocks(h), nv = orc_num_vertices(h, 1);
  std::vector<double> g1(512 * (size_t)nb, 1.0), g0(512 * (size_t)nb), gD((size_t)W * H);
  orc_grad_fusion64(h, g1.data(), g0.data(), gD.data());
  std::vector<double> pos(3 * (size_t)nv + 1);
  orc_positions64_depth(h, (H / 2) * W + W / 2, 1e-7, pos.data());
  // restricted collection of a few blocks
  std::vector<int> only = {0, 0, 2, 1, 0, 2};
  orc_restrict_blocks(h, only.data(), 2);
  const float T[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
  orc_integrate(h, depth.data(), W, H, fx, fy, cx, cy, 0.1f, 5.f, T);
  orc_restrict_blocks(h, nullptr, 0);
  orc_extract(h, 0);
  orc_gc(h);
  r |= exercise_exports(h);
  orc_destroy(h);
  return r;
}

int tables() {
  int out[15], sizes[8], edges[12], co[24], ee[24];
  for (int t = 0; t < 256; ++t) {
    if (orc_cube_triangles(t, out) < 0) return fail("cube triangles");
    if (orc_cube_polygons(t, sizes, edges) < 0) return fail("cube polygons");
    if (orc_cube_polygon_sizes(t, sizes) < 0) return fail("polygon sizes");
    const float dc[8] = {0.1f, -0.2f, 0.3f, -0.05f, 0.2f, -0.3f, 0.04f, -0.1f};
    orc_refine_type(t, (t * 37) & 255, dc, 0.5f);
  }
  for (int j = 0; j < 6; ++j) orc_regular_type(j);
  orc_corner_offsets(co);
  orc_edge_ends(ee);
  return 0;
}

}  // namespace

int main() {
  int r = tables();
  r |= sphere_import(1);
  r |= sphere_import(8);
  r |= plane_fusion(1);
  r |= plane_fusion(8);
  if (r == 0) std::printf("sanitize driver: ok\n");
  return r;
}
