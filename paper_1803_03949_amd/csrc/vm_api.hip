// C-ABI of the voxmesh library: argument checks, workspace layout, pose
// inversion and the kernel sequence of each call.  No device allocation:
// every byte lives in the caller's buffer.
#include <math.h>
#include <stddef.h>
#include <string.h>

#include <hip/hip_ext.h>

#include <mutex>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include "voxmesh.h"
#include "vm_internal.h"

namespace vm {
void build_mc_tables(uint8_t* tri, uint8_t* uses);
}

using namespace vm;

struct vm_volume {
  struct ProfRec {
    int kid;
    hipEvent_t a, b;
  };
  // A captured phase of vm_extract_batch with what it was captured for,
  // and the host-side state the captured forward left.
  struct BatchGraph {
    hipGraphExec_t exec = nullptr;
    vm_batch_io io;
    vm_launch launch;
    const float* d;
    const float* w;
    uint32_t frame, epoch, pass, xcount, vcount, xsel, vsel, dev_frame;
  };
  vm_config cfg;
  char* mem;
  size_t bytes;
  VolDev dev;
  float* own_d;     // the workspace's TSDF and weight arrays (d, w when unbound)
  float* own_w;
  uint32_t frame;   // last frame number handed to the device
  uint32_t epoch;   // extraction epoch (pending-list stamps)
  uint32_t pass;    // dirty / vertex-list stamps
  uint32_t xcount;  // extractions so far (parity selects the dirty-list length)
  int64_t dl_nv;    // vertices of the last download (-1: none since the mesh changed)
  uint32_t vcount;  // extractions and refinements so far (vertex-list length)
  FrameParams last_fp;
  bool have_fp;
  bool last_refine = false;  // the last extraction-side call was a refinement
  int cus;          // compute units of the device
  vm_launch launch; // workgroup mapping (see vm_set_launch)
  int grid_blocks;  // workgroups of per-block kernels
  int grid_items;   // workgroups of per-item kernels
  int grid_waves;   // workgroups of wave-per-block kernels
  uint32_t prof;    // bit k: bracket launches of kernel k with events
  std::vector<hipEvent_t> ev_free;
  std::vector<ProfRec> recs;
  int scratch_dev = -1;  // device whose static workspace holds the volume, -1 if the caller's
  BatchGraph bgraph[2];  // vm_extract_batch: forward, backward
};

namespace {

uint8_t g_tri[256 * 16];
uint8_t g_uses[256 * 12];
uint32_t g_roles[4 * 256];
std::once_flag g_tables_once;

// The vertex pass's edge-use table: for each cube type, by the cube's place
// around a voxel (role 0: cube (x, y), 1: (x, y-1), 2: (x-1, y), 3:
// (x-1, y-1), all in the voxel's layer), how many of the type's triangles
// use the voxel's x, y and z edge (6-bit fields at bits 0, 6, 12) and the x
// and y edge of the voxel one layer up (bits 18, 24), which the same cube
// also touches.  The cube edges follow the cyclic numbering: a voxel's x
// edge is e0 of cube (x, y), e2 of (x, y-1), e4 and e6 of those one layer
// down; its y edge e3 of (x, y), e1 of (x-1, y), e7 and e5 one layer down;
// its z edge e8, e11, e9, e10 of (x, y), (x, y-1), (x-1, y), (x-1, y-1).
void build_roles(const uint8_t* uses, uint32_t* roles) {
  for (int t = 0; t < 256; ++t) {
    const uint8_t* u = uses + 12 * t;
    roles[t] = u[0] | u[3] << 6 | u[8] << 12 | u[4] << 18 | u[7] << 24;
    roles[256 + t] = u[2] | u[11] << 12 | u[6] << 18;
    roles[512 + t] = u[1] << 6 | u[9] << 12 | u[5] << 24;
    roles[768 + t] = u[10] << 12;
  }
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

bool config_ok(const vm_config* c) {
  return c && c->voxel_m > 0.f && isfinite(c->voxel_m) && c->trunc_vox > 0.f &&
         isfinite(c->trunc_vox) && c->refine_eps_vox >= 0.f && c->hash_log2 >= 10 &&
         c->hash_log2 <= 28 && c->max_blocks >= 1 && c->max_blocks <= kMaxBlocks &&
         c->max_vertices >= 1 && c->max_vertices <= (1 << 30) &&
         (c->hash_mode == 0 || c->hash_mode == 1) &&
         c->batch_volumes >= 0 && c->batch_volumes <= kMaxSlots;
}

bool launch_ok(const vm_launch* l) {
  return l && (l->wave_group_size == 2 || l->wave_group_size == 4 || l->wave_group_size == 8) &&
         l->wave_groups_per_cu >= 1 && l->wave_groups_per_cu <= 32 &&
         l->block_groups_per_cu >= 1 && l->block_groups_per_cu <= 16 &&
         l->item_groups_per_cu >= 1 && l->item_groups_per_cu <= 32 &&
         l->block_order >= 0 && l->block_order <= 3;
}

void apply_launch(vm_volume* vol, const vm_launch& l) {
  vol->launch = l;
  vol->grid_blocks = vol->cus * l.block_groups_per_cu;
  vol->grid_items = vol->cus * l.item_groups_per_cu;
  vol->grid_waves = vol->cus * l.wave_groups_per_cu;
  vol->dev.order = (uint32_t)l.block_order;
}

// Carve the workspace; with base == nullptr only the size is computed.
size_t carve(const vm_config& c, char* base, VolDev* v) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? (void*)(base + off) : nullptr;
    off = align_up(off + bytes);
    return p;
  };
  const size_t H = (size_t)1 << c.hash_log2, B = (size_t)c.max_blocks,
               V = (size_t)c.max_vertices, C = B * kVox;
  // download parts, or three counts per import part
  const size_t scan = (V > C ? V : C) / 1024 + 2 + 3 * (B / kImportRows + 1);
  v->cnt = (Counters*)take(sizeof(Counters));
  v->vseg = (Seg*)take(sizeof(Seg) * kSegs);
  v->cseg = (Seg*)take(sizeof(Seg) * kSegs);
  v->tri_table = (const uint8_t*)take(256 * 16);
  v->edge_uses = (const uint8_t*)take(256 * 12);
  v->edge_roles = (const uint32_t*)take(4 * 4 * 256);
  v->slots = (unsigned long long*)take(8 * H);
  v->slot_stamp = (uint32_t*)take(4 * H);
  v->slot_src = (uint32_t*)take(4 * H);
  v->block_key = (uint64_t*)take(8 * B);
  v->nbr = (int32_t*)take(4 * 27 * B);
  v->d = (float*)take(4 * kVox * B);
  v->w = (float*)take(4 * kVox * B);
  v->tprev = (uint8_t*)take(kVox * B);
  v->tcur = (uint8_t*)take(kVox * B);
  v->evtx = (int32_t*)take(4 * 3 * kVox * B);
  v->et = (float*)take(4 * 3 * kVox * B);
  v->emask = (uint32_t*)take(4 * 64 * B);
  v->wmask = (uint64_t*)take(8 * 8 * B);
  v->smask = (uint64_t*)take(8 * 8 * B);
  v->nmask = (uint64_t*)take(8 * 8 * B);
  v->st_pending = (uint32_t*)take(4 * B);
  v->st_dirty = (uint32_t*)take(4 * B);
  v->st_vtx = (uint32_t*)take(4 * B);
  v->st_frame = (uint32_t*)take(4 * B);
  v->frame_list = (uint32_t*)take(4 * B);
  v->frame_src = (uint32_t*)take(4 * B);
  v->frame_key = (uint64_t*)take(8 * B);
  v->row_slot = (uint32_t*)take(4 * B);
  v->pending = (uint32_t*)take(4 * B);
  v->dirty = (uint32_t*)take(4 * B);
  v->vcand = (uint32_t*)take(4 * 8 * B);
  v->vblocks = (uint32_t*)take(4 * B);
  v->vowner = (uint32_t*)take(4 * V);
  v->vring = (uint32_t*)take(4 * V);
  v->vdl = (int32_t*)take(4 * V);
  v->vbirth = (uint32_t*)take(4 * V);
  v->scan = (uint32_t*)take(4 * scan);
  v->scan_cap = (uint32_t)scan;
  v->max_blocks = (uint32_t)B;
  v->max_vertices = (uint32_t)V;
  // one segment per 256 blocks of capacity, at most kSegs
  const size_t nseg = B / 256 < 1 ? 1 : (B / 256 > (size_t)kSegs ? (size_t)kSegs : B / 256);
  v->nseg = (uint32_t)nseg;
  v->vseg_cap = (uint32_t)((V + nseg - 1) / nseg);
  v->hash_mask = (uint32_t)(H - 1);
  v->hash_mode = c.hash_mode;
  return off;
}

int hip_status(hipError_t e) { return e == hipSuccess ? VM_OK : VM_ERR_HIP; }

int launched() { return hip_status(hipGetLastError()); }

// Fill n 32-bit words with a value: a kernel rather than a memset node, so
// that a reset can sit inside a captured graph.
void fill(void* p, uint32_t value, size_t bytes, hipStream_t stream) {
  const uint64_t n = bytes / 4;
  uint64_t g = (n + 255) / 256;
  g = g < 1 ? 1 : (g > 2048 ? 2048 : g);
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, stream, (uint32_t*)p, value, n);
}

// Empty the volume.  full = true (creation) also clears the running totals
// and uploads the marching-cubes tables.
int clear_state(vm_volume* vol, hipStream_t stream, bool full) {
  const VolDev& v = vol->dev;
  const size_t H = (size_t)v.hash_mask + 1, B = v.max_blocks;
  fill(v.cnt, 0, full ? sizeof(Counters) : offsetof(Counters, acc), stream);
  fill(v.vseg, 0, sizeof(Seg) * kSegs, stream);
  fill(v.cseg, 0, sizeof(Seg) * kSegs, stream);
  fill(v.slots, 0xFFFFFFFFu, 8 * H, stream);
  fill(v.slot_stamp, 0, 4 * H, stream);
  fill(v.st_pending, 0, 4 * B, stream);
  fill(v.st_dirty, 0, 4 * B, stream);
  fill(v.st_vtx, 0, 4 * B, stream);
  fill(v.st_frame, 0, 4 * B, stream);
  hipError_t e = hipGetLastError();
  if (full) {
    if (e == hipSuccess)
      e = hipMemcpyAsync((void*)v.tri_table, g_tri, sizeof(g_tri), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync((void*)v.edge_uses, g_uses, sizeof(g_uses), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync((void*)v.edge_roles, g_roles, sizeof(g_roles), hipMemcpyHostToDevice,
                         stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
  }
  vol->frame = 0;
  vol->epoch = 1;
  vol->pass = 0;
  vol->last_refine = false;
  vol->have_fp = false;
  vol->dl_nv = -1;
  return hip_status(e);
}

int read_counters(vm_volume* vol, Counters* c, hipStream_t stream) {
  hipError_t e = hipMemcpyAsync(c, vol->dev.cnt, sizeof(Counters), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  return hip_status(e);
}

int error_code(uint32_t bits) {
  for (int k = 0; k < 16; ++k)
    if (bits & (1u << k)) return -(k + 2);
  return VM_OK;
}

// Two events for timing a launch of kernel kid while it is profiled (not
// on a stream under capture: such launches run untimed).
bool prof_pair(vm_volume* vol, int kid, hipStream_t s, hipEvent_t* a, hipEvent_t* b) {
  if (!((vol->prof >> kid) & 1u)) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (s != nullptr && (hipStreamIsCapturing(s, &cs) != hipSuccess ||
                       cs != hipStreamCaptureStatusNone))
    return false;
  hipEvent_t e[2] = {nullptr, nullptr};
  for (hipEvent_t& x : e) {
    if (!vol->ev_free.empty()) {
      x = vol->ev_free.back();
      vol->ev_free.pop_back();
    } else if (hipEventCreate(&x) != hipSuccess) {
      x = nullptr;
    }
  }
  if (!e[0] || !e[1]) {
    for (hipEvent_t x : e)
      if (x) vol->ev_free.push_back(x);
    return false;
  }
  *a = e[0], *b = e[1];
  return true;
}

// A launch whose start and end the launch itself records in two events
// (hipExtLaunchKernel): no marker packets between kernels, and the time is
// the kernel's own.  The arguments are converted to the kernel's parameter
// types first.
template <typename... P, typename... A, size_t... I>
hipError_t launch_timed_at(void (*k)(P...), dim3 g, dim3 b, hipStream_t s, hipEvent_t e0,
                           hipEvent_t e1, std::index_sequence<I...>, A&&... a) {
  std::tuple<P...> t(std::forward<A>(a)...);
  void* args[] = {(void*)&std::get<I>(t)...};
  return hipExtLaunchKernel((const void*)k, g, b, args, 0, s, e0, e1, 0);
}
template <typename... P, typename... A>
hipError_t launch_timed(void (*k)(P...), dim3 g, dim3 b, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1, A&&... a) {
  return launch_timed_at(k, g, b, s, e0, e1, std::index_sequence_for<P...>{},
                         std::forward<A>(a)...);
}

// Launch a kernel; while it is profiled, the launch records its start and
// end (a timed launch that fails is made again untimed, so that timing
// never drops a kernel).
#define VM_LAUNCH(vol, kid, kernel, grid, block, stream, ...)                                \
  do {                                                                                     \
    hipEvent_t vm_a_ = nullptr, vm_b_ = nullptr;                                           \
    bool vm_done_ = false;                                                                 \
    if (prof_pair((vol), (kid), (stream), &vm_a_, &vm_b_)) {                               \
      if (launch_timed(kernel, grid, block, stream, vm_a_, vm_b_, __VA_ARGS__) == hipSuccess) { \
        (vol)->recs.push_back({(kid), vm_a_, vm_b_});                                      \
        vm_done_ = true;                                                                   \
      } else {                                                                             \
        (vol)->ev_free.push_back(vm_a_), (vol)->ev_free.push_back(vm_b_);                  \
        (void)hipGetLastError();                                                           \
      }                                                                                    \
    }                                                                                      \
    if (!vm_done_) hipLaunchKernelGGL(kernel, grid, block, 0, stream, __VA_ARGS__);        \
  } while (0)

// Launch a wave-per-block kernel instantiated for the volume's group size.
#define VM_LAUNCH_W(vol, kid, kernel, stream, ...)                                          \
  do {                                                                                  \
    const dim3 vm_g_((vol)->grid_waves);                                                \
    switch ((vol)->launch.wave_group_size) {                                            \
      case 2: VM_LAUNCH(vol, kid, kernel<2>, vm_g_, dim3(128), stream, __VA_ARGS__); break; \
      case 8: VM_LAUNCH(vol, kid, kernel<8>, vm_g_, dim3(512), stream, __VA_ARGS__); break; \
      default: VM_LAUNCH(vol, kid, kernel<4>, vm_g_, dim3(256), stream, __VA_ARGS__); break; \
    }                                                                                   \
  } while (0)

// The same for kernels with a second, compile-time mode argument.
#define VM_LAUNCH_WM(vol, kid, kernel, mode, stream, ...)                                     \
  do {                                                                                      \
    const dim3 vm_g_((vol)->grid_waves);                                                    \
    switch ((vol)->launch.wave_group_size) {                                                \
      case 2: VM_LAUNCH(vol, kid, (kernel<2, mode>), vm_g_, dim3(128), stream, __VA_ARGS__); break; \
      case 8: VM_LAUNCH(vol, kid, (kernel<8, mode>), vm_g_, dim3(512), stream, __VA_ARGS__); break; \
      default: VM_LAUNCH(vol, kid, (kernel<4, mode>), vm_g_, dim3(256), stream, __VA_ARGS__); break; \
    }                                                                                       \
  } while (0)

void prep(vm_volume* vol, int op, hipStream_t s) {
  VM_LAUNCH(vol, VM_K_COUNTERS, k_prep, dim3(1), dim3(64), s, vol->dev, op, 0u);
}

// Host copy of the counters and both segment tables.
struct Snapshot {
  Counters c;
  Seg vseg[kSegs], cseg[kSegs];
};

int read_snapshot(vm_volume* vol, Snapshot* s, hipStream_t stream) {
  hipError_t e = hipMemcpyAsync(&s->c, vol->dev.cnt, sizeof(Counters), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->vseg, vol->dev.vseg, sizeof(s->vseg), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->cseg, vol->dev.cseg, sizeof(s->cseg), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  return hip_status(e);
}

// One phase of vm_extract_batch as plain launches (0 forward, 1 backward).
int batch_enqueue(vm_volume* vol, const vm_batch_io& io, int ph, hipStream_t s) {
  if (ph == 1)
    return vm_extract_backward_slots(vol, io.dL_dpos, io.rows, io.n, io.dL_dtsdf, s);
  int r = vm_reset_volume(vol, s);
  if (r == VM_OK)
    r = vm_import_batch(vol, io.slots, io.coords, io.tsdf, io.weight, io.n, io.rows, s);
  if (r == VM_OK) r = vm_extract_mesh(vol, VM_SCOPE_ALL, s);
  if (r == VM_OK) r = vm_export_positions(vol, io.pos, io.slot_of, io.pos_cap, s);
  return r;
}

// Host-side state of a volume that its calls advance.
void save_host_state(const vm_volume* vol, vm_volume::BatchGraph& g) {
  g.frame = vol->frame, g.epoch = vol->epoch, g.pass = vol->pass;
  g.xcount = vol->xcount, g.vcount = vol->vcount;
  g.xsel = vol->dev.xsel, g.vsel = vol->dev.vsel, g.dev_frame = vol->dev.frame;
}

void load_host_state(vm_volume* vol, const vm_volume::BatchGraph& g) {
  vol->frame = g.frame, vol->epoch = g.epoch, vol->pass = g.pass;
  vol->xcount = g.xcount, vol->vcount = g.vcount;
  vol->dev.xsel = g.xsel, vol->dev.vsel = g.vsel, vol->dev.frame = g.dev_frame;
  vol->have_fp = false;
  vol->dl_nv = -1;
}

// One phase of vm_extract_batch: replay its graph, capturing it first when
// there is none for these arguments; plain launches where a graph cannot
// be captured (a stream under capture already, the legacy default stream)
// or would hold profiling events.
int batch_phase(vm_volume* vol, const vm_batch_io& io, int ph, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (s != nullptr && hipStreamIsCapturing(s, &cs) != hipSuccess) return VM_ERR_HIP;
  if (s == nullptr || cs != hipStreamCaptureStatusNone || vol->prof != 0)
    return batch_enqueue(vol, io, ph, s);
  vm_volume::BatchGraph& g = vol->bgraph[ph];
  const bool same = g.exec && memcmp(&g.io, &io, sizeof(io)) == 0 &&
                    memcmp(&g.launch, &vol->launch, sizeof(vm_launch)) == 0 &&
                    g.d == vol->dev.d && g.w == vol->dev.w;
  if (!same) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g.exec = nullptr;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return VM_ERR_HIP;
    const int r = batch_enqueue(vol, io, ph, s);
    const hipError_t e = hipStreamEndCapture(s, &graph);
    if (r != VM_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return r != VM_OK ? r : VM_ERR_HIP;
    }
    const hipError_t ei = hipGraphInstantiateWithFlags(&g.exec, graph, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      g.exec = nullptr;
      return VM_ERR_HIP;
    }
    g.io = io;
    g.launch = vol->launch;
    g.d = vol->dev.d;
    g.w = vol->dev.w;
    save_host_state(vol, g);
  }
  const hipError_t e = hipGraphLaunch(g.exec, s);
  if (e != hipSuccess) return VM_ERR_HIP;
  if (ph == 0) load_host_state(vol, g);
  return VM_OK;
}

// Set up a volume handle over the workspace mem (bytes long, already
// checked against the configuration) and clear the workspace on `stream`.
int init_volume(vm_volume* vol, const vm_config* cfg, char* mem, size_t bytes,
                hipStream_t stream) {
  std::call_once(g_tables_once, [] {
    build_mc_tables(g_tri, g_uses);
    build_roles(g_uses, g_roles);
  });
  vol->cfg = *cfg;
  vol->mem = mem;
  vol->bytes = bytes;
  VolDev& v = vol->dev;
  carve(*cfg, vol->mem, &v);
  v.s = cfg->voxel_m;
  v.inv_s = (float)(1.0 / (double)cfg->voxel_m);
  v.inv_block = (float)(1.0 / (8.0 * (double)cfg->voxel_m));
  v.mu_m = (float)((double)cfg->trunc_vox * (double)cfg->voxel_m);
  v.mu_v = cfg->trunc_vox;
  v.eps = cfg->refine_eps_vox;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    return VM_ERR_HIP;
  v.batch = (uint32_t)cfg->batch_volumes;
  v.bound = 0;
  vol->own_d = v.d;
  vol->own_w = v.w;
  vol->cus = cus;
  apply_launch(vol, vm_launch{4, 16, 8, 8, 0});
  vol->prof = 0;
  return clear_state(vol, stream, true);
}

// Workspace of vm_create_volume_noalloc: one per device, held until the
// process ends.  Host code never passes the array's name to a kernel or a
// copy: it takes the device address from hipGetSymbolAddress, once per
// device, and uses that.
constexpr size_t kScratchBytes = (size_t)VM_NOALLOC_MAX_BYTES;
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kScratchDevices];
bool g_scratch_used[kScratchDevices];
alignas(vm_volume) unsigned char g_scratch_vol_mem[kScratchDevices][sizeof(vm_volume)];
vm_volume* const g_scratch_vol = reinterpret_cast<vm_volume*>(g_scratch_vol_mem);

}  // namespace

static __device__ __align__(256) unsigned char scratch[VM_NOALLOC_MAX_BYTES];

extern "C" {

int vm_volume_bytes(const vm_config* cfg, size_t* bytes) {
  if (!config_ok(cfg) || !bytes) return VM_ERR_ARG;
  VolDev v;
  *bytes = carve(*cfg, nullptr, &v);
  return VM_OK;
}

int vm_create_volume(const vm_config* cfg, void* dev_mem, size_t bytes, hipStream_t stream,
                     vm_volume** out) {
  if (!config_ok(cfg) || !dev_mem || !out || ((uintptr_t)dev_mem & 255)) return VM_ERR_ARG;
  VolDev probe;
  if (bytes < carve(*cfg, nullptr, &probe)) return VM_ERR_ARG;
  vm_volume* vol = new (std::nothrow) vm_volume();
  if (!vol) return VM_ERR_ARG;
  const int r = init_volume(vol, cfg, (char*)dev_mem, bytes, stream);
  if (r != VM_OK) {
    delete vol;
    return r;
  }
  *out = vol;
  return VM_OK;
}

int vm_create_volume_noalloc(const vm_config* cfg, hipStream_t stream, vm_volume** out) {
  if (!config_ok(cfg) || !out) return VM_ERR_ARG;
  VolDev probe;
  const size_t need = carve(*cfg, nullptr, &probe);
  if (need > kScratchBytes) return VM_ERR_CAPACITY;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return VM_ERR_HIP;
  if (dev < 0 || dev >= kScratchDevices) return VM_ERR_ARG;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    // the array's device address on this device (the name itself is only
    // a host-side stand-in)
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return VM_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  if (g_scratch_used[dev]) return VM_ERR_ARG;  // one volume per device at a time
  vm_volume* vol = new (&g_scratch_vol[dev]) vm_volume();
  const int r = init_volume(vol, cfg, (char*)g_scratch_ptr[dev], kScratchBytes, stream);
  if (r != VM_OK) {
    vol->~vm_volume();
    return r;
  }
  vol->scratch_dev = dev;
  g_scratch_used[dev] = true;
  *out = vol;
  return VM_OK;
}

int vm_destroy_volume(vm_volume* vol) {
  if (!vol) return VM_ERR_ARG;
  for (auto& g : vol->bgraph)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  for (auto& r : vol->recs) vol->ev_free.push_back(r.a), vol->ev_free.push_back(r.b);
  for (hipEvent_t e : vol->ev_free) (void)hipEventDestroy(e);
  const int sdev = vol->scratch_dev;
  if (sdev < 0) {
    delete vol;
    return VM_OK;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  vol->~vm_volume();
  g_scratch_used[sdev] = false;
  return VM_OK;
}

int vm_reset_volume(vm_volume* vol, hipStream_t stream) {
  if (!vol) return VM_ERR_ARG;
  prep(vol, VM_OP_RESET, stream);
  int r = launched();
  if (r != VM_OK) return r;
  return clear_state(vol, stream, false);
}

int vm_integrate_depth(vm_volume* vol, const float* depth, const vm_intrinsics* K,
                       const float cam_to_world[16], hipStream_t stream) {
  if (!vol || !depth || !K || !cam_to_world || K->width <= 0 || K->height <= 0 ||
      (int64_t)K->width * K->height > (1 << 28) || !(K->fx != 0.f) || !(K->fy != 0.f) ||
      vol->dev.batch)
    return VM_ERR_ARG;
  FrameParams fp;
  const float* T = cam_to_world;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) {
      fp.Rcw[3 * i + j] = T[4 * i + j];
      fp.Rwc[3 * j + i] = T[4 * i + j];
    }
    fp.tcw[i] = T[4 * i + 3];
  }
  // world -> sensor translation: -R^T t in FP64, rounded once
  for (int i = 0; i < 3; ++i) {
    double acc = (double)fp.Rcw[0 * 3 + i] * (double)fp.tcw[0];
    acc = acc + (double)fp.Rcw[1 * 3 + i] * (double)fp.tcw[1];
    acc = acc + (double)fp.Rcw[2 * 3 + i] * (double)fp.tcw[2];
    fp.twc[i] = (float)(-acc);
  }
  fp.fx = K->fx, fp.fy = K->fy, fp.cx = K->cx, fp.cy = K->cy;
  fp.dmin = K->min_depth_m, fp.dmax = K->max_depth_m;
  fp.W = K->width, fp.H = K->height;
  fp.frame = ++vol->frame;
  vol->dl_nv = -1;
  const VolDev& v = vol->dev;
  // one workgroup per 32 x 16 pixel tile
  const unsigned tiles = (unsigned)((K->width + 31) / 32) * (unsigned)((K->height + 15) / 16);
  VM_LAUNCH(vol, VM_K_COLLECT, k_collect, dim3(tiles), dim3(512), stream, v, fp, depth,
            vol->epoch);
  VM_LAUNCH_W(vol, VM_K_FUSE, k_fuse, stream, v, fp, depth, vol->epoch);
  vol->last_fp = fp;
  vol->have_fp = true;
  return launched();
}

int vm_import_blocks(vm_volume* vol, const int32_t* coords, const float* tsdf,
                     const float* weight, int64_t n, hipStream_t stream) {
  if (!vol || vol->dev.batch) return VM_ERR_ARG;
  return vm_import_batch(vol, nullptr, coords, tsdf, weight, n, nullptr, stream);
}

int vm_import_batch(vm_volume* vol, const int32_t* slots, const int32_t* coords,
                    const float* tsdf, const float* weight, int64_t n, int32_t* rows,
                    hipStream_t stream) {
  if (!vol || n < 0 || n > (int64_t)vol->dev.max_blocks ||
      (n > 0 && (!coords || !tsdf || !weight)) || (vol->dev.batch != 0) != (slots != nullptr) ||
      (vol->dev.bound && n > 0 && (tsdf != vol->dev.d || weight != vol->dev.w)))
    return VM_ERR_ARG;
  if (n == 0) return VM_OK;
  const VolDev& v = vol->dev;
  const uint32_t frame = ++vol->frame;
  vol->dl_nv = -1;
  // blocks are listed, and new ones numbered, in row order: a caller's
  // spatially ordered rows give a spatially ordered pool
  const uint32_t nparts = (uint32_t)((n + kImportRows - 1) / kImportRows);
  VM_LAUNCH(vol, VM_K_IMPORT, k_import_insert, dim3((unsigned)((n + 255) / 256)), dim3(256), stream,
            v, slots, coords, (uint32_t)n, frame);
  VM_LAUNCH(vol, VM_K_ASSIGN, k_import_count, dim3(nparts), dim3(kImportRows), stream, v,
            (uint32_t)n, vol->epoch);
  VM_LAUNCH(vol, VM_K_ASSIGN, k_import_scan, dim3(1), dim3(1024), stream, v, nparts, frame,
            vol->epoch);
  VM_LAUNCH(vol, VM_K_ASSIGN, k_import_assign, dim3(nparts), dim3(kImportRows), stream, v,
            (uint32_t)n, nparts, vol->epoch);
  VM_LAUNCH_W(vol, VM_K_IMPORT, k_import_copy, stream, v, tsdf, weight, frame, rows);
  vol->have_fp = false;
  return launched();
}

int vm_bind_tsdf(vm_volume* vol, float* tsdf, float* weight) {
  if (!vol || (tsdf == nullptr) != (weight == nullptr) || ((uintptr_t)tsdf & 3) ||
      ((uintptr_t)weight & 3))
    return VM_ERR_ARG;
  VolDev& v = vol->dev;
  v.d = tsdf ? tsdf : vol->own_d;
  v.w = weight ? weight : vol->own_w;
  v.bound = tsdf ? 1u : 0u;
  return VM_OK;
}

int vm_extract_mesh(vm_volume* vol, int scope, hipStream_t stream) {
  const bool refine = (scope & VM_EXTRACT_REFINE) != 0;
  scope &= ~VM_EXTRACT_REFINE;
  if (!vol || (scope != VM_SCOPE_DIRTY && scope != VM_SCOPE_ALL)) return VM_ERR_ARG;
  const uint32_t pass = ++vol->pass;
  vol->dl_nv = -1;
  // the first kernel starts the call (segments, statistics, list lengths)
  vol->dev.xsel = ++vol->xcount & 1u;
  vol->dev.frame = vol->frame;
  vol->dev.vsel = ++vol->vcount & 1u;
  const VolDev& v = vol->dev;
  // the vertex pass re-places the vertices whose end points' blocks were
  // fused or imported since the last extraction (every block for ALL)
  const uint32_t moved = scope == VM_SCOPE_ALL ? kMovedAll : vol->epoch;
  if (scope == VM_SCOPE_ALL)
    VM_LAUNCH(vol, VM_K_DIRTY, k_dirty_all, dim3(vol->grid_items), dim3(256), stream, v, pass);
  else
    VM_LAUNCH(vol, VM_K_DIRTY, k_dirty, dim3(vol->grid_items), dim3(256), stream, v, pass,
              vol->epoch);
  ++vol->epoch;
  if (refine)
    VM_LAUNCH_WM(vol, VM_K_CLASSIFY, k_classify, kExtractRefined, stream, v, pass);
  else
    VM_LAUNCH_WM(vol, VM_K_CLASSIFY, k_classify, kExtract, stream, v, pass);
  VM_LAUNCH_W(vol, VM_K_VERTICES, k_vertices, stream, v, moved, 1);
  vol->last_refine = false;
  return launched();
}

int vm_refine_mesh(vm_volume* vol, hipStream_t stream) {
  if (!vol) return VM_ERR_ARG;
  const uint32_t pass = ++vol->pass;
  vol->dl_nv = -1;
  vol->dev.vsel = ++vol->vcount & 1u;
  vol->dev.frame = vol->frame;
  const VolDev& v = vol->dev;
  prep(vol, VM_OP_REFINE, stream);
  VM_LAUNCH_WM(vol, VM_K_REFINE, k_classify, kRefine, stream, v, pass);
  VM_LAUNCH(vol, VM_K_DIRTY, k_vblock_compact, dim3(vol->grid_items), dim3(256), stream, v);
  // refinement changes types only: the end points that moved are those in
  // blocks fused or imported since the last extraction (normally none)
  VM_LAUNCH_W(vol, VM_K_VERTICES, k_vertices, stream, v, vol->epoch, 0);
  vol->last_refine = true;
  return launched();
}

int vm_gc(vm_volume* vol, hipStream_t stream) {
  if (!vol) return VM_ERR_ARG;
  // nothing to launch: the vertex pass already freed every vertex whose
  // count dropped to zero (its edge forgot it, its slot went to the
  // segment's recycle ring), and the next extraction or refinement closes
  // the rings before it allocates
  (void)stream;
  return VM_OK;
}

int vm_download_mesh(vm_volume* vol, float* verts, uint64_t* edge_keys, int32_t* tris,
                     int64_t vcap, int64_t tcap, int64_t* nv, int64_t* nt, hipStream_t stream) {
  if (!vol || !nv || !nt || vcap < 0 || tcap < 0 || (vcap > 0 && !verts) || (tcap > 0 && !tris))
    return VM_ERR_ARG;
  const VolDev& v = vol->dev;
  prep(vol, VM_OP_FINALISE, stream);
  int r = launched();
  if (r != VM_OK) return r;
  Counters c;
  const uint32_t pv = (v.max_vertices + 1023) / 1024,
                 pt = (uint32_t)(((uint64_t)v.max_blocks * kVox + 1023) / 1024);
  const uint32_t vc = (uint32_t)(vcap > 0xFFFFFFFFll ? 0xFFFFFFFFll : vcap);
  const uint32_t tc = (uint32_t)(tcap > 0xFFFFFFFFll ? 0xFFFFFFFFll : tcap);
  VM_LAUNCH(vol, VM_K_DOWNLOAD, k_dl_count, dim3(pv), dim3(256), stream, v, 0);
  VM_LAUNCH(vol, VM_K_DOWNLOAD, k_dl_scan, dim3(1), dim3(1024), stream, v, 0, pv);
  VM_LAUNCH(vol, VM_K_DOWNLOAD, k_dl_write_vertices, dim3(pv), dim3(256), stream, v, verts, edge_keys,
            vc);
  VM_LAUNCH(vol, VM_K_DOWNLOAD, k_dl_count, dim3(pt), dim3(256), stream, v, 1);
  VM_LAUNCH(vol, VM_K_DOWNLOAD, k_dl_scan, dim3(1), dim3(1024), stream, v, 1, pt);
  VM_LAUNCH(vol, VM_K_DOWNLOAD, k_dl_write_triangles, dim3(pt), dim3(256), stream, v, tris, tc);
  r = launched();
  if (r != VM_OK) return r;
  r = read_counters(vol, &c, stream);
  if (r != VM_OK) return r;
  *nv = c.dl_nv;
  *nt = c.dl_nt;
  vol->dl_nv = c.dl_nv;
  if (c.error) return error_code(c.error);
  if ((int64_t)c.dl_nv > vcap || (int64_t)c.dl_nt > tcap) return VM_ERR_CAPACITY;
  return VM_OK;
}

int vm_download_normals(vm_volume* vol, float* normals, int64_t cap, hipStream_t stream) {
  if (!vol || (cap > 0 && !normals) || cap < 0) return VM_ERR_ARG;
  if (vol->dl_nv < 0) return VM_ERR_ARG;
  if (cap < vol->dl_nv) return VM_ERR_CAPACITY;
  VM_LAUNCH(vol, VM_K_DOWNLOAD, k_dl_normals, dim3(vol->grid_items), dim3(256), stream, vol->dev,
            normals);
  return launched();
}

int vm_download_births(vm_volume* vol, uint32_t* births, int64_t cap, hipStream_t stream) {
  if (!vol || (cap > 0 && !births) || cap < 0) return VM_ERR_ARG;
  if (vol->dl_nv < 0) return VM_ERR_ARG;
  if (cap < vol->dl_nv) return VM_ERR_CAPACITY;
  VM_LAUNCH(vol, VM_K_DOWNLOAD, k_dl_births, dim3(vol->grid_items), dim3(256), stream, vol->dev,
            births);
  return launched();
}

int vm_sharing_ablation(vm_volume* vol, int scheme, int32_t* edge_slot, float* edge_t,
                        uint32_t* counter, hipStream_t stream) {
  if (!vol || !edge_slot || !edge_t || !counter || (scheme != 0 && scheme != 1))
    return VM_ERR_ARG;
  const dim3 g(vol->grid_items), b(256);
  if (scheme == 0) {
    VM_LAUNCH(vol, VM_K_ABLATION, k_share_lock, g, b, stream, vol->dev, edge_slot, edge_t,
              counter);
  } else {
    for (int group = 0; group < 4; ++group)
      VM_LAUNCH(vol, VM_K_ABLATION, k_share_free, g, b, stream, vol->dev, group, edge_slot,
                edge_t, counter);
  }
  return launched();
}

int vm_extract_backward(vm_volume* vol, const float* dL_dverts, float* dL_dtsdf,
                        hipStream_t stream) {
  if (!vol || !dL_dtsdf) return VM_ERR_ARG;
  VM_LAUNCH_W(vol, VM_K_BACKWARD, k_bwd_tsdf, stream, vol->dev, dL_dverts, 0, nullptr, 0u,
              dL_dtsdf);
  return launched();
}

int vm_extract_backward_slots(vm_volume* vol, const float* dL_dpos, const int32_t* rows,
                              int64_t n_rows, float* dL_dtsdf, hipStream_t stream) {
  if (!vol || !dL_dpos || !dL_dtsdf || (rows && (n_rows < 0 || n_rows > (int64_t)kMaxBlocks)))
    return VM_ERR_ARG;
  VM_LAUNCH_W(vol, VM_K_BACKWARD, k_bwd_tsdf, stream, vol->dev, dL_dpos, 1, rows,
              (uint32_t)(rows ? n_rows : 0), dL_dtsdf);
  return launched();
}

int vm_export_positions(vm_volume* vol, float* pos, int32_t* slot_of, int64_t cap,
                        hipStream_t stream) {
  if (!vol || !pos) return VM_ERR_ARG;
  if (cap < (int64_t)vol->dev.max_vertices) return VM_ERR_CAPACITY;
  prep(vol, VM_OP_FINALISE, stream);
  VM_LAUNCH(vol, VM_K_POSITIONS, k_positions, dim3(vol->grid_items), dim3(256), stream, vol->dev,
            pos, slot_of);
  return launched();
}

int vm_set_launch(vm_volume* vol, const vm_launch* launch) {
  if (!vol || !launch_ok(launch)) return VM_ERR_ARG;
  apply_launch(vol, *launch);
  return VM_OK;
}

int vm_get_launch(vm_volume* vol, vm_launch* launch) {
  if (!vol || !launch) return VM_ERR_ARG;
  *launch = vol->launch;
  return VM_OK;
}

int vm_integrate_backward(vm_volume* vol, const float* depth, const float* dL_dtsdf1,
                          float* dL_dtsdf0, float* dL_ddepth, hipStream_t stream) {
  if (!vol || !depth || !dL_dtsdf1 || !dL_dtsdf0 || !dL_ddepth || !vol->have_fp) return VM_ERR_ARG;
  const FrameParams& fp = vol->last_fp;
  VM_LAUNCH(vol, VM_K_BACKWARD, k_zero_f32, dim3(256), dim3(256), stream, dL_ddepth,
            (uint64_t)fp.W * (uint64_t)fp.H);
  VM_LAUNCH(vol, VM_K_BACKWARD, k_bwd_fusion, dim3(vol->grid_blocks), dim3(512), stream, vol->dev,
            fp, depth, dL_dtsdf1, dL_dtsdf0, dL_ddepth);
  return launched();
}

int vm_get_status(vm_volume* vol, vm_status* out, hipStream_t stream) {
  if (!vol || !out) return VM_ERR_ARG;
  prep(vol, VM_OP_FINALISE, stream);
  int r = launched();
  if (r != VM_OK) return r;
  Snapshot sn;
  r = read_snapshot(vol, &sn, stream);
  if (r != VM_OK) return r;
  const Counters& c = sn.c;
  const uint32_t B = vol->dev.max_blocks;
  uint32_t st_new = 0, st_upd = 0, st_freed = 0, st_chg = 0, st_ref = 0;
  int64_t vh = 0, vf = 0, tris = 0, tcubes = 0, seg_live = 0;
  for (int k = 0; k < kSegs; ++k) {
    st_new += sn.vseg[k].st_new, st_upd += sn.vseg[k].st_upd, st_freed += sn.vseg[k].st_freed;
    st_chg += sn.cseg[k].st_chg, st_ref += sn.cseg[k].st_ref;
    vh += sn.vseg[k].hwm, vf += sn.vseg[k].count;
    tris += (int64_t)sn.cseg[k].st_fnew - (int64_t)sn.cseg[k].st_fold;
    tcubes += (int64_t)sn.cseg[k].st_cnew - (int64_t)sn.cseg[k].st_cold;
    const int64_t live = (int64_t)sn.vseg[k].hwm - (int64_t)sn.vseg[k].count;
    seg_live = live > seg_live ? live : seg_live;
  }
  memset(out, 0, sizeof(*out));
  out->error = error_code(c.error);
  out->error_bits = c.error;
  out->blocks = c.n_blocks < B ? c.n_blocks : B;
  const uint32_t nf = c.n_frame[vol->frame & 1];
  out->frame_blocks = nf < B ? nf : B;
  out->pending_blocks = c.n_pending[vol->epoch & 1];
  out->dirty_blocks = c.n_dirty[vol->dev.xsel];
  out->vertex_blocks = c.n_vblocks[vol->dev.vsel] + (vol->last_refine ? 0u : c.n_dirty[vol->dev.xsel]);
  out->changed_cubes = st_chg - c.base_chg;
  out->vertex_slots = vh;
  out->free_vertex_slots = vf;
  out->triangles = tris;
  out->tri_cubes = tcubes;
  out->new_vertices = st_new - c.base_new;
  out->updated_vertices = st_upd - c.base_upd;
  out->freed_vertices = st_freed - c.base_freed;
  out->refined_cubes = st_ref - c.base_ref;
  out->vertex_segments = vol->dev.nseg;
  out->segment_capacity = vol->dev.vseg_cap;
  out->max_segment_live = seg_live;
  return out->error;
}

int vm_export_blocks(vm_volume* vol, int32_t* coords, float* tsdf, float* weight,
                     uint8_t* type_prev, uint8_t* type_cur, int64_t cap, int64_t* n,
                     hipStream_t stream) {
  if (!vol || !n || cap < 0 || (cap > 0 && !coords)) return VM_ERR_ARG;
  Counters c;
  int r = read_counters(vol, &c, stream);
  if (r != VM_OK) return r;
  const VolDev& v = vol->dev;
  const size_t nb = c.n_blocks < v.max_blocks ? c.n_blocks : v.max_blocks;
  *n = (int64_t)nb;
  const size_t m = (size_t)cap < nb ? (size_t)cap : nb;
  if (m == 0) return VM_OK;
  std::vector<uint64_t> keys(m);
  hipError_t e = hipMemcpyAsync(keys.data(), v.block_key, 8 * m, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && tsdf)
    e = hipMemcpyAsync(tsdf, v.d, 4 * kVox * m, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess && weight)
    e = hipMemcpyAsync(weight, v.w, 4 * kVox * m, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess && type_prev)
    e = hipMemcpyAsync(type_prev, v.tprev, kVox * m, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess && type_cur)
    e = hipMemcpyAsync(type_cur, v.tcur, kVox * m, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return VM_ERR_HIP;
  for (size_t i = 0; i < m; ++i) unpack_key(keys[i], coords[3 * i], coords[3 * i + 1], coords[3 * i + 2]);
  return VM_OK;
}

int vm_export_vertices(vm_volume* vol, uint64_t* edge_keys, float* t, int32_t* refcount,
                       int64_t cap, int64_t* n, hipStream_t stream) {
  if (!vol || !n || cap < 0 || (cap > 0 && (!edge_keys || !t || !refcount))) return VM_ERR_ARG;
  prep(vol, VM_OP_FINALISE, stream);
  int r = launched();
  if (r != VM_OK) return r;
  *n = vol->dev.max_vertices;
  const uint32_t m = (uint32_t)((int64_t)vol->dev.max_vertices < cap ? vol->dev.max_vertices : cap);
  if (m == 0) return hip_status(hipStreamSynchronize(stream));
  hipLaunchKernelGGL(k_export_vertices, dim3((m + 255) / 256), dim3(256), 0, stream, vol->dev,
                     edge_keys, t, refcount, m);
  r = launched();
  if (r != VM_OK) return r;
  return hip_status(hipStreamSynchronize(stream));
}

int vm_export_block_list(vm_volume* vol, int which, int32_t* coords, int64_t cap, int64_t* n,
                         hipStream_t stream) {
  if (!vol || !n || which < 0 || which > 2 || cap < 0 || (cap > 0 && !coords)) return VM_ERR_ARG;
  Counters c;
  int r = read_counters(vol, &c, stream);
  if (r != VM_OK) return r;
  const VolDev& v = vol->dev;
  const uint32_t len = which == 0 ? c.n_frame[vol->frame & 1] : which == 1 ? c.n_dirty[vol->dev.xsel] : c.n_pending[vol->epoch & 1];
  const size_t cnt = len < v.max_blocks ? len : v.max_blocks;
  *n = (int64_t)cnt;
  const size_t m = (size_t)cap < cnt ? (size_t)cap : cnt;
  if (m == 0) return VM_OK;
  const uint32_t* list = which == 0 ? v.frame_list : which == 1 ? v.dirty : v.pending;
  const size_t nb = c.n_blocks < v.max_blocks ? c.n_blocks : v.max_blocks;
  std::vector<uint32_t> idx(m);
  std::vector<uint64_t> keys(nb);
  hipError_t e = hipMemcpyAsync(idx.data(), list, 4 * m, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess && nb)
    e = hipMemcpyAsync(keys.data(), v.block_key, 8 * nb, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return VM_ERR_HIP;
  size_t k = 0;
  for (size_t i = 0; i < m; ++i) {
    if (idx[i] == kNone) continue;
    const uint32_t b = idx[i] & ~kNewFlag;
    if (b >= nb) continue;
    unpack_key(keys[b], coords[3 * k], coords[3 * k + 1], coords[3 * k + 2]);
    ++k;
  }
  *n = (int64_t)k;
  return VM_OK;
}

int vm_lookup_blocks(vm_volume* vol, const int32_t* coords, int32_t* idx, int64_t n,
                     hipStream_t stream) {
  if (!vol || n < 0 || n > 0x7FFFFFFF || (n > 0 && (!coords || !idx))) return VM_ERR_ARG;
  if (n == 0) return VM_OK;
  const uint32_t m = (uint32_t)n;
  hipLaunchKernelGGL(k_lookup, dim3((m + 255) / 256 < 65535 ? (m + 255) / 256 : 65535), dim3(256), 0,
                     stream, vol->dev, coords, idx, m);
  return launched();
}

int vm_get_totals(vm_volume* vol, int64_t* out, int n, hipStream_t stream) {
  if (!vol || !out || n < 0 || n > VM_TOTAL_COUNT) return VM_ERR_ARG;
  Snapshot sn;
  int r = read_snapshot(vol, &sn, stream);
  if (r != VM_OK) return r;
  unsigned long long t[VM_TOTAL_COUNT];
  for (int i = 0; i < VM_TOTAL_COUNT; ++i) t[i] = sn.c.acc[i];
  for (int k = 0; k < kSegs; ++k) {
    t[VM_TOTAL_NEW_VERTICES] += sn.vseg[k].st_new;
    t[VM_TOTAL_UPDATED_VERTICES] += sn.vseg[k].st_upd;
    t[VM_TOTAL_MOVED_VERTICES] += sn.vseg[k].st_mov;
    t[VM_TOTAL_FREED_VERTICES] += sn.vseg[k].st_freed;
    t[VM_TOTAL_CHANGED_CUBES] += sn.cseg[k].st_chg;
    t[VM_TOTAL_REFINED_CUBES] += sn.cseg[k].st_ref;
    t[VM_TOTAL_NEW_TRIANGLES] += sn.cseg[k].st_fnew;
    t[VM_TOTAL_DROPPED_TRIANGLES] += sn.cseg[k].st_fold;
  }
  for (int i = 0; i < n; ++i) out[i] = (int64_t)t[i];
  return VM_OK;
}

int vm_extract_batch(vm_volume* vol, const vm_batch_io* io, int phase, hipStream_t stream) {
  if (!vol || !io || (phase != VM_BATCH_FORWARD && phase != VM_BATCH_BACKWARD) || io->n < 1 ||
      io->n > (int64_t)vol->dev.max_blocks || !io->coords || !io->tsdf || !io->weight ||
      !io->rows || (vol->dev.batch != 0) != (io->slots != nullptr))
    return VM_ERR_ARG;
  if (phase == VM_BATCH_FORWARD && !io->pos) return VM_ERR_ARG;
  if (phase == VM_BATCH_BACKWARD && (!io->dL_dpos || !io->dL_dtsdf)) return VM_ERR_ARG;
  if (io->pos_cap < (int64_t)vol->dev.max_vertices) return VM_ERR_CAPACITY;
  return batch_phase(vol, *io, phase == VM_BATCH_FORWARD ? 0 : 1, stream);
}

int vm_profile_mask(vm_volume* vol, uint32_t mask) {
  if (!vol || (mask >> VM_K_COUNT)) return VM_ERR_ARG;
  if (mask) {
    for (auto& r : vol->recs) vol->ev_free.push_back(r.a), vol->ev_free.push_back(r.b);
    vol->recs.clear();
  }
  vol->prof = mask;
  return VM_OK;
}

int vm_profile(vm_volume* vol, int enable) {
  return vm_profile_mask(vol, enable ? (1u << VM_K_COUNT) - 1u : 0u);
}

int vm_profile_read(vm_volume* vol, int64_t* launches, double* ms) {
  if (!vol || !launches || !ms) return VM_ERR_ARG;
  for (int k = 0; k < VM_K_COUNT; ++k) launches[k] = 0, ms[k] = 0.0;
  if (!vol->recs.empty() && hipEventSynchronize(vol->recs.back().b) != hipSuccess) return VM_ERR_HIP;
  for (auto& r : vol->recs) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return VM_ERR_HIP;
    launches[r.kid] += 1;
    ms[r.kid] += (double)t;
  }
  return VM_OK;
}

}  // extern "C"
