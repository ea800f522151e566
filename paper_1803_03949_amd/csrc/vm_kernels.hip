// HIP kernels of the voxmesh library for gfx950 (wave64).
//
// Work that is per block (fusion, classification, vertex update, backward)
// runs one 512-lane workgroup per 8^3 block, one lane per voxel/cube, with
// the block and its one-voxel halo staged in LDS.  Work lists live on the
// device, so every kernel loops over its list with a grid stride and the
// host never waits for a count.  Allocation in the pools uses one atomic
// per wave (ballot + popcount ranks) or per workgroup.
#include "vm_internal.h"

namespace vm {

// ============================================================================
// counters
// ============================================================================
__global__ void k_counters(VolDev v, int op, uint32_t arg) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Counters* c = v.cnt;
  switch (op) {
    case VM_OP_BEGIN_FRAME:
      c->n_frame = 0;
      break;
    case VM_OP_END_FRAME:
      c->last_frame_list = min(c->n_frame, v.max_blocks);
      break;
    case VM_OP_BEGIN_EXTRACT:
      c->n_dirty = 0;
      c->n_vblocks = 0;
      c->n_changed = 0;
      c->st_new_vtx = 0;
      c->st_upd_vtx = 0;
      c->st_refined = 0;
      break;
    case VM_OP_BEGIN_REFINE:
      c->n_vblocks = 0;
      c->n_changed = 0;
      c->st_new_vtx = 0;
      c->st_upd_vtx = 0;
      c->st_refined = 0;
      break;
    case VM_OP_END_PENDING:
      c->n_pending = 0;
      break;
    case VM_OP_FIN_VERTICES: {
      uint32_t avail = c->vtx_tail - c->vtx_head;
      uint32_t used = c->vtx_ticket;
      uint32_t from_ring = min(used, avail);
      c->vtx_head += from_ring;
      uint64_t hwm = (uint64_t)c->vtx_hwm + (used - from_ring);
      c->vtx_hwm = hwm > v.max_vertices ? v.max_vertices : (uint32_t)hwm;
      c->vtx_ticket = 0;
      break;
    }
    case VM_OP_FIN_TRIANGLES: {
      uint32_t avail = c->chk_tail - c->chk_head;
      uint32_t used = c->chk_ticket;
      uint32_t from_ring = min(used, avail);
      c->chk_head += from_ring;
      uint64_t hwm = (uint64_t)c->chk_hwm + (used - from_ring);
      c->chk_hwm = hwm > v.max_chunks ? v.max_chunks : (uint32_t)hwm;
      c->chk_tail += c->chk_push;
      c->chk_ticket = 0;
      c->chk_push = 0;
      break;
    }
    case VM_OP_BEGIN_GC:
      c->vtx_push = 0;
      break;
    case VM_OP_FIN_GC:
      c->vtx_tail += c->vtx_push;
      c->st_freed = c->vtx_push;
      c->vtx_push = 0;
      break;
    default:
      break;
  }
  (void)arg;
}

// ============================================================================
// block collection (Eq. 1)
// ============================================================================

// Mark one block key as collected by this frame: insert it if absent and
// list its hash slot once per frame.
__device__ static void collect_key(const VolDev& v, uint64_t key, uint32_t frame, uint32_t src) {
  bool inserted;
  int64_t s = hash_insert(v, key, &inserted);
  if (s < 0) {
    atomicOr(&v.cnt->error, kErrHash);
    return;
  }
  uint32_t* st = &v.slot_stamp[s];
  if (__hip_atomic_load(st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == frame) return;
  if (atomicMax(st, frame) >= frame) return;
  uint32_t pos = atomicAdd(&v.cnt->n_frame, 1u);
  if (pos < v.max_blocks) {
    v.frame_slots[pos] = (uint32_t)s;
    v.frame_src[pos] = src;
  } else {
    atomicOr(&v.cnt->error, kErrBlocks);
  }
}

// One lane per pixel.  Each valid pixel spans the integer box of blocks
// between its ray points at camera depth D - mu and D + mu; lanes of a wave
// that name the same block are merged before touching the hash.
__global__ __launch_bounds__(256) void k_collect(VolDev v, FrameParams fp,
                                                 const float* __restrict__ depth) {
  const int npix = fp.W * fp.H;
  const int pix = blockIdx.x * blockDim.x + threadIdx.x;
  int lo[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
  int nbox = 0;
  if (pix < npix) {
    const int px = pix % fp.W, py = pix / fp.W;
    const float D = depth[pix];
    if (depth_ok(D, fp.dmin, fp.dmax)) {
      const float xn = ((float)px - fp.cx) / fp.fx;
      const float yn = ((float)py - fp.cy) / fp.fy;
      int b[2][3];
      bool ok = true;
#pragma unroll
      for (int end = 0; end < 2; ++end) {
        const float z = end == 0 ? D - v.mu_m : D + v.mu_m;
        const float p0 = xn * z, p1 = yn * z;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          float P = fp.Rcw[3 * i] * p0;
          P = P + fp.Rcw[3 * i + 1] * p1;
          P = P + fp.Rcw[3 * i + 2] * z;
          P = P + fp.tcw[i];
          const float fb = floorf(P * v.inv_block);
          ok = ok && (fb >= -8192.f && fb <= 8191.f);
          b[end][i] = ok ? (int)fb : 0;
        }
      }
      if (ok) {
        nbox = 1;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          lo[i] = min(b[0][i], b[1][i]);
          ext[i] = abs(b[1][i] - b[0][i]) + 1;
          nbox *= ext[i];
        }
      }
    }
  }
  for (int j = 0; __ballot(j < nbox); ++j) {
    bool has = j < nbox;
    uint64_t key = 0;
    if (has) {
      const int cx = j % ext[0], cy = (j / ext[0]) % ext[1], cz = j / (ext[0] * ext[1]);
      key = pack_key(lo[0] + cx, lo[1] + cy, lo[2] + cz);
    }
    uint64_t todo = __ballot(has);
    while (todo) {
      const int leader = __ffsll((unsigned long long)todo) - 1;
      const uint32_t klo = __shfl((uint32_t)key, leader);
      const uint32_t khi = __shfl((uint32_t)(key >> 32), leader);
      const uint64_t lk = ((uint64_t)khi << 32) | klo;
      const bool same = has && key == lk;
      todo &= ~__ballot(same);
      if (same) has = false;
      if ((int)__lane_id() == leader) collect_key(v, lk, fp.frame, 0);
    }
  }
}

__global__ void k_import_insert(VolDev v, const int32_t* __restrict__ coords, uint32_t n,
                                uint32_t frame) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int x = coords[3 * i], y = coords[3 * i + 1], z = coords[3 * i + 2];
  if (!key_in_range(x, y, z)) {
    atomicOr(&v.cnt->error, kErrRange);
    return;
  }
  collect_key(v, pack_key(x, y, z), frame, i);
}

// Give every newly inserted key of the frame a pool index (one atomic per
// wave), publish it in the hash slot and list the block as pending for the
// next extraction.
__global__ __launch_bounds__(256) void k_assign(VolDev v, uint32_t epoch) {
  const uint32_t n = min(v.cnt->n_frame, v.max_blocks);
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
    const uint32_t i = base + threadIdx.x;
    const bool act = i < n;
    uint32_t s = 0, idx = kNone;
    uint64_t key = 0;
    if (act) {
      s = v.frame_slots[i];
      const unsigned long long val = load_slot(&v.slots[s]);
      key = val >> kIdxBits;
      idx = (uint32_t)(val & kIdxMask);
    }
    const bool isnew = act && idx == kPending;
    const uint32_t t = wave_ticket(&v.cnt->n_blocks, isnew);
    if (isnew) {
      if (t < v.max_blocks) {
        idx = t;
        v.slots[s] = ((unsigned long long)key << kIdxBits) | idx;
        v.block_key[idx] = key;
        int32_t* nb = v.nbr + (size_t)idx * 27;
        for (int d = 0; d < 27; ++d) nb[d] = d == kSelf ? (int32_t)idx : -1;
        v.frame_list[i] = idx | kNewFlag;
      } else {
        atomicOr(&v.cnt->error, kErrBlocks);
        v.frame_list[i] = kNone;
        idx = kNone;
      }
    } else if (act) {
      v.frame_list[i] = idx;
    }
    const bool pend = act && idx != kNone && v.st_pending[idx] != epoch;
    if (pend) v.st_pending[idx] = epoch;
    const uint32_t p = wave_ticket(&v.cnt->n_pending, pend);
    if (pend) {
      if (p < v.max_blocks) v.pending[p] = idx;
      else atomicOr(&v.cnt->error, kErrBlocks);
    }
  }
}

// Link each new block with its 26 neighbours in both directions.
__global__ __launch_bounds__(256) void k_link(VolDev v) {
  const uint32_t n = min(v.cnt->n_frame, v.max_blocks);
  const uint32_t total = n * 27u;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    const uint32_t i = t / 27u, dir = t % 27u;
    if (dir == (uint32_t)kSelf) continue;
    const uint32_t e = v.frame_list[i];
    if (e == kNone || !(e & kNewFlag)) continue;
    const uint32_t idx = e & ~kNewFlag;
    int x, y, z;
    unpack_key(v.block_key[idx], x, y, z);
    const int nx = x + (int)(dir % 3) - 1, ny = y + (int)((dir / 3) % 3) - 1, nz = z + (int)(dir / 9) - 1;
    if (!key_in_range(nx, ny, nz)) continue;
    const int32_t nb = hash_find(v, pack_key(nx, ny, nz));
    if (nb < 0) continue;
    v.nbr[(size_t)idx * 27 + dir] = nb;
    v.nbr[(size_t)nb * 27 + (26 - dir)] = (int32_t)idx;
  }
}

// ============================================================================
// fusion (Eq. 2) and import
// ============================================================================
__device__ inline void init_cube(const VolDev& v, uint32_t idx, int l) {
  const size_t o = (size_t)idx * kVox + l;
  v.tprev[o] = 0;
  v.tcur[o] = 0;
  v.cchunk[o] = -1;
  v.evtx[((size_t)idx * 3 + 0) * kVox + l] = -1;
  v.evtx[((size_t)idx * 3 + 1) * kVox + l] = -1;
  v.evtx[((size_t)idx * 3 + 2) * kVox + l] = -1;
}

__global__ __launch_bounds__(512) void k_fuse(VolDev v, FrameParams fp,
                                              const float* __restrict__ depth) {
  const uint32_t n = min(v.cnt->n_frame, v.max_blocks);
  const int l = threadIdx.x, lx = l & 7, ly = (l >> 3) & 7, lz = l >> 6;
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const uint32_t e = v.frame_list[i];
    if (e == kNone) continue;
    const uint32_t idx = e & ~kNewFlag;
    const bool isnew = (e & kNewFlag) != 0;
    int bx, by, bz;
    unpack_key(v.block_key[idx], bx, by, bz);
    const size_t o = (size_t)idx * kVox + l;
    float d = 0.f, w = 0.f;
    if (isnew) init_cube(v, idx, l);
    else d = v.d[o], w = v.w[o];
    const FuseSample fs = fuse_sample(v, fp, depth, 8 * bx + lx, 8 * by + ly, 8 * bz + lz);
    if (fs.upd) {
      float num = d * w;
      num = num + fs.dt;
      const float den = w + 1.0f;
      d = num / den;
      w = den;
    }
    if (fs.upd || isnew) {
      v.d[o] = d;
      v.w[o] = w;
    }
    if (l == 0) v.st_frame[idx] = fp.frame;
  }
}

__global__ __launch_bounds__(512) void k_import_copy(VolDev v, const float* __restrict__ tsdf,
                                                     const float* __restrict__ weight,
                                                     uint32_t frame) {
  const uint32_t n = min(v.cnt->n_frame, v.max_blocks);
  const int l = threadIdx.x;
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const uint32_t e = v.frame_list[i];
    if (e == kNone) continue;
    const uint32_t idx = e & ~kNewFlag;
    if (e & kNewFlag) init_cube(v, idx, l);
    const size_t src = (size_t)v.frame_src[i] * kVox + l;
    const size_t o = (size_t)idx * kVox + l;
    v.d[o] = tsdf[src];
    v.w[o] = weight[src];
    if (l == 0) v.st_frame[idx] = frame;
  }
}

// ============================================================================
// extraction: dirty set, classification (+ refinement), vertices, triangles
// ============================================================================

// Dirty = pending blocks and their allocated neighbours at offsets {-1,0}^3.
__global__ __launch_bounds__(256) void k_dirty(VolDev v, uint32_t pass) {
  const uint32_t n = min(v.cnt->n_pending, v.max_blocks);
  const uint32_t total = n * 8u;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < total; base += stride) {
    const uint32_t t = base + threadIdx.x;
    bool claim = false;
    int32_t nb = -1;
    if (t < total) {
      const uint32_t idx = v.pending[t >> 3], o = t & 7u;
      nb = v.nbr[(size_t)idx * 27 + nbr_dir(-(int)(o & 1), -(int)((o >> 1) & 1), -(int)(o >> 2))];
      if (nb >= 0 && v.st_dirty[nb] != pass) claim = atomicMax(&v.st_dirty[nb], pass) < pass;
    }
    const uint32_t p = wave_ticket(&v.cnt->n_dirty, claim);
    if (claim) v.dirty[p] = (uint32_t)nb;
  }
}

__global__ __launch_bounds__(256) void k_dirty_all(VolDev v, uint32_t pass) {
  const uint32_t n = min(v.cnt->n_blocks, v.max_blocks);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    v.dirty[i] = i;
    v.st_dirty[i] = pass;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) v.cnt->n_dirty = n;
}

__device__ inline uint32_t refine_type(uint32_t t, uint32_t prev, const float dc[8], float eps) {
  // Eqs. (3)-(5); regular types in the order the paper lists them.
  const uint32_t kRegular[6] = {0xCCu, 0x33u, 0x99u, 0x66u, 0xF0u, 0x0Fu};
  if (__popc(t ^ prev) > 3) return t;
  int best = -1, best_d = 9;
  bool keep_prev = false;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const uint32_t x = t ^ kRegular[j];
    const int dist = __popc(x);
    if (dist > 3) continue;
    bool near = true;
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (((x >> k) & 1u) && !(fabsf(dc[k]) < eps)) near = false;
    if (!near) continue;
    if (kRegular[j] == prev) keep_prev = true;
    if (dist < best_d) best_d = dist, best = j;
  }
  if (best < 0) return t;
  return keep_prev ? prev : kRegular[best];
}

// One workgroup per dirty block, one lane per cube.  The block's 8^3 corners
// plus the +x/+y/+z halo layer (9^3) are staged in LDS.  refine = 0: new
// cube types from the signs (Sec. V-B), previous type saved.  refine = 1:
// Eqs. (3)-(5) applied to the current types (Sec. V-F).
__global__ __launch_bounds__(512) void k_classify(VolDev v, uint32_t pass, int refine) {
  __shared__ float sd[729];
  __shared__ uint8_t sok[729];
  __shared__ int32_t snb[8];
  __shared__ uint32_t sflags, srefined;
  const uint32_t n = min(v.cnt->n_dirty, v.max_blocks);
  const int l = threadIdx.x, lx = l & 7, ly = (l >> 3) & 7, lz = l >> 6;
  const int coff[8] = {0, 1, 1 + 9, 9, 81, 1 + 81, 1 + 9 + 81, 9 + 81};
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const uint32_t idx = v.dirty[i];
    if (l < 8) snb[l] = v.nbr[(size_t)idx * 27 + nbr_dir(l & 1, (l >> 1) & 1, l >> 2)];
    if (l == 0) sflags = 0, srefined = 0;
    __syncthreads();
    for (int j = l; j < 729; j += 512) {
      const int x = j % 9, y = (j / 9) % 9, z = j / 81;
      const int nb = snb[(x >> 3) | ((y >> 3) << 1) | ((z >> 3) << 2)];
      float dv = 0.f;
      uint8_t ok = 0;
      if (nb >= 0) {
        const size_t o = (size_t)nb * kVox + (x & 7) + 8 * (y & 7) + 64 * (z & 7);
        dv = v.d[o];
        ok = v.w[o] > 0.f;
      }
      sd[j] = dv;
      sok[j] = ok;
    }
    __syncthreads();
    const int base = lx + 9 * ly + 81 * lz;
    bool valid = true;
    uint32_t t = 0;
    float dc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      valid = valid && sok[base + coff[k]];
      dc[k] = sd[base + coff[k]];
      t |= (uint32_t)(dc[k] < 0.f) << k;
    }
    if (!valid) t = 0;
    const size_t o = (size_t)idx * kVox + l;
    const uint32_t old = v.tcur[o];
    uint32_t nt;
    if (!refine) {
      v.tprev[o] = (uint8_t)old;
      nt = t;
    } else {
      nt = valid ? refine_type(old, v.tprev[o], dc, v.eps) : old;
    }
    if (nt != old) v.tcur[o] = (uint8_t)nt;
    const bool tri_change = nt != old && (v.tri_table[old * 16] || v.tri_table[nt * 16]);
    const uint32_t p = wave_ticket(&v.cnt->n_changed, tri_change);
    if (tri_change) {
      if (p < v.max_changed) v.changed[p] = (idx << 9) | (uint32_t)l;
      else atomicOr(&v.cnt->error, kErrTris);
      // owners of this cube's edges: this block and, on its +x/+y/+z
      // faces, the neighbours (never the +x+y+z corner one)
      const bool ex = lx == 7, ey = ly == 7, ez = lz == 7;
      uint32_t f = 1u | (ex ? 2u : 0u) | (ey ? 4u : 0u) | (ez ? 16u : 0u) | (ex && ey ? 8u : 0u) |
                   (ex && ez ? 32u : 0u) | (ey && ez ? 64u : 0u);
      atomicOr(&sflags, f);
      if (refine) atomicAdd(&srefined, 1u);
    }
    __syncthreads();
    if (l < 64) {
      // extraction recomputes every dirty block's vertices (their end
      // points may have moved); refinement only blocks with changed cubes
      const uint32_t flags = sflags | (refine ? 0u : 1u);
      int32_t nb = -1;
      bool claim = false;
      if (l < 8 && ((flags >> l) & 1u)) {
        nb = l == 0 ? (int32_t)idx : snb[l];
        if (nb >= 0 && v.st_vtx[nb] != pass) claim = atomicMax(&v.st_vtx[nb], pass) < pass;
      }
      const uint32_t q = wave_ticket(&v.cnt->n_vblocks, claim);
      if (claim) v.vblocks[q] = (uint32_t)nb;
      if (l == 0 && srefined) atomicAdd(&v.cnt->st_refined, srefined);
    }
    __syncthreads();
  }
}

// One workgroup per listed block, one lane per voxel.  Each voxel owns the
// edges from it along +x, +y, +z.  The reference count of an edge is the
// number of triangles, over the four cubes around it, that use it; a
// positive count needs a vertex (created here on first use), whose
// parameter t is rewritten from the end point TSDF values.  The counts come
// from cube types staged in LDS with the -x/-y/-z halo, so no atomics and no
// per-triangle increments are needed.
__global__ __launch_bounds__(512) void k_vertices(VolDev v) {
  __shared__ uint8_t suses[256 * 12];
  __shared__ uint8_t st[729];   // cube types at local -1..7
  __shared__ float sd[729];     // TSDF at local 0..8
  __shared__ int32_t snb[27];
  __shared__ uint32_t swave[8];
  __shared__ uint32_t sbase, snew, supd;
  const int l = threadIdx.x, lx = l & 7, ly = (l >> 3) & 7, lz = l >> 6;
  {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(v.edge_uses);
    uint32_t* dst = reinterpret_cast<uint32_t*>(suses);
    for (int j = l; j < 256 * 12 / 4; j += 512) dst[j] = src[j];
  }
  const uint32_t n = min(v.cnt->n_vblocks, v.max_blocks);
  const uint32_t head = v.cnt->vtx_head, tail = v.cnt->vtx_tail, hwm = v.cnt->vtx_hwm;
  const int wave = l >> 6;
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const uint32_t idx = v.vblocks[i];
    if (l < 27) snb[l] = v.nbr[(size_t)idx * 27 + l];
    if (l == 0) snew = 0, supd = 0;
    __syncthreads();
    for (int j = l; j < 729; j += 512) {
      const int x = j % 9, y = (j / 9) % 9, z = j / 81;
      const int cx = x - 1, cy = y - 1, cz = z - 1;
      const int nb = snb[nbr_dir(cx < 0 ? -1 : 0, cy < 0 ? -1 : 0, cz < 0 ? -1 : 0)];
      st[j] = nb >= 0 ? v.tcur[(size_t)nb * kVox + (cx & 7) + 8 * (cy & 7) + 64 * (cz & 7)] : 0;
      const int nb2 = snb[nbr_dir(x >> 3, y >> 3, z >> 3)];
      sd[j] = nb2 >= 0 ? v.d[(size_t)nb2 * kVox + (x & 7) + 8 * (y & 7) + 64 * (z & 7)] : 0.f;
    }
    __syncthreads();
    const int tb = (lx + 1) + 9 * (ly + 1) + 81 * (lz + 1);
#define USES(c, e) ((uint32_t)suses[(uint32_t)st[c] * 12 + (e)])
    uint32_t ref[3];
    ref[0] = USES(tb, 0) + USES(tb - 9, 2) + USES(tb - 81, 4) + USES(tb - 90, 6);
    ref[1] = USES(tb, 3) + USES(tb - 1, 1) + USES(tb - 81, 7) + USES(tb - 82, 5);
    ref[2] = USES(tb, 8) + USES(tb - 1, 9) + USES(tb - 10, 10) + USES(tb - 9, 11);
#undef USES
    size_t eo[3];
    int32_t slot[3];
    bool need[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      eo[a] = ((size_t)idx * 3 + a) * kVox + l;
      slot[a] = v.evtx[eo[a]];
      need[a] = ref[a] > 0 && slot[a] < 0;
    }
    const uint64_t m0 = __ballot(need[0]), m1 = __ballot(need[1]), m2 = __ballot(need[2]);
    const uint32_t c0 = __popcll(m0), c1 = __popcll(m1), c2 = __popcll(m2);
    const uint64_t lt = lanes_below();
    uint32_t rank[3];
    rank[0] = __popcll(m0 & lt);
    rank[1] = c0 + __popcll(m1 & lt);
    rank[2] = c0 + c1 + __popcll(m2 & lt);
    if (__lane_id() == 0) swave[wave] = c0 + c1 + c2;
    __syncthreads();
    if (l == 0) {
      uint32_t acc = 0;
      for (int w = 0; w < 8; ++w) {
        const uint32_t c = swave[w];
        swave[w] = acc;
        acc += c;
      }
      sbase = acc ? atomicAdd(&v.cnt->vtx_ticket, acc) : 0u;
    }
    __syncthreads();
    const uint32_t tk = sbase + swave[wave];
    const int sdb = lx + 9 * ly + 81 * lz;
    const int step[3] = {1, 9, 81};
    uint32_t nnew = 0, nupd = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (ref[a] > 0) {
        int32_t s = slot[a];
        if (s < 0) {
          const uint32_t ns = ticket_slot(tk + rank[a], v.vring, head, tail, hwm, v.max_vertices);
          if (ns == kNone) {
            atomicOr(&v.cnt->error, kErrVertices);
            continue;
          }
          s = (int32_t)ns;
          v.evtx[eo[a]] = s;
          v.vowner[s] = (uint32_t)eo[a];
          ++nnew;
        } else {
          ++nupd;
        }
        v.vt[s] = edge_param(sd[sdb], sd[sdb + step[a]]);
        v.vref[s] = (int32_t)ref[a];
      } else if (slot[a] >= 0) {
        v.vref[slot[a]] = 0;
      }
    }
    if (nnew) atomicAdd(&snew, nnew);
    if (nupd) atomicAdd(&supd, nupd);
    __syncthreads();
    if (l == 0) {
      if (snew) atomicAdd(&v.cnt->st_new_vtx, snew);
      if (supd) atomicAdd(&v.cnt->st_upd_vtx, supd);
    }
  }
}

// Owner of each cube edge: offset from the cube's anchor voxel and axis,
// packed as ox | oy << 1 | oz << 2 | axis << 3.
// e0 (000,x) e1 (100,y) e2 (010,x) e3 (000,y) e4 (001,x) e5 (101,y)
// e6 (011,x) e7 (001,y) e8 (000,z) e9 (100,z) e10 (110,z) e11 (010,z)
__device__ inline void edge_owner(int e, int& ox, int& oy, int& oz, int& axis) {
  static constexpr uint8_t kOwn[12] = {0, 9, 2, 8, 4, 13, 6, 12, 16, 17, 19, 18};
  const uint32_t p = kOwn[e];
  ox = (int)(p & 1u);
  oy = (int)((p >> 1) & 1u);
  oz = (int)((p >> 2) & 1u);
  axis = (int)(p >> 3);
}

// One lane per cube whose triangles changed: (re)write its triangle chunk
// as vertex slots of the owning edges, or recycle the chunk when the cube's
// new type has no triangles (Sec. V-D).  Unchanged cubes keep theirs.
__global__ __launch_bounds__(256) void k_triangles(VolDev v) {
  const uint32_t n = min(v.cnt->n_changed, v.max_changed);
  const uint32_t head = v.cnt->chk_head, tail = v.cnt->chk_tail, hwm = v.cnt->chk_hwm;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
    const uint32_t i = base + threadIdx.x;
    const bool act = i < n;
    uint32_t idx = 0, l = 0, type = 0, ntri = 0;
    int32_t chunk = -1;
    if (act) {
      const uint32_t e = v.changed[i];
      idx = e >> 9;
      l = e & 511u;
      type = v.tcur[(size_t)idx * kVox + l];
      ntri = v.tri_table[type * 16];
      chunk = v.cchunk[(size_t)idx * kVox + l];
    }
    const bool want_alloc = act && ntri > 0 && chunk < 0;
    const bool want_free = act && ntri == 0 && chunk >= 0;
    const uint32_t ta = wave_ticket(&v.cnt->chk_ticket, want_alloc);
    const uint32_t tf = wave_ticket(&v.cnt->chk_push, want_free);
    if (want_free) {
      v.chunks[(size_t)chunk * kChunkWords] = kNone;
      v.cring[(uint32_t)(((uint64_t)tail + tf) % v.max_chunks)] = (uint32_t)chunk;
      v.cchunk[(size_t)idx * kVox + l] = -1;
    }
    if (!act || ntri == 0) continue;
    if (chunk < 0) {
      const uint32_t ns = ticket_slot(ta, v.cring, head, tail, hwm, v.max_chunks);
      if (ns == kNone) {
        atomicOr(&v.cnt->error, kErrTris);
        continue;
      }
      chunk = (int32_t)ns;
      v.cchunk[(size_t)idx * kVox + l] = chunk;
    }
    uint32_t* c = v.chunks + (size_t)chunk * kChunkWords;
    c[0] = (idx << 9) | l;
    const int lx = l & 7, ly = (l >> 3) & 7, lz = l >> 6;
    const uint8_t* tt = v.tri_table + type * 16 + 1;
    for (int k = 0; k < 15; ++k) {
      uint32_t slot = kNone;
      if (k < (int)(3 * ntri)) {
        int ox, oy, oz, axis;
        edge_owner(tt[k], ox, oy, oz, axis);
        const int x = lx + ox, y = ly + oy, z = lz + oz;
        const int dir = nbr_dir(x >> 3, y >> 3, z >> 3);
        const int32_t nb = dir == kSelf ? (int32_t)idx : v.nbr[(size_t)idx * 27 + dir];
        if (nb >= 0) {
          const int32_t s = v.evtx[((size_t)nb * 3 + axis) * kVox + (x & 7) + 8 * (y & 7) + 64 * (z & 7)];
          slot = s >= 0 ? (uint32_t)s : kNone;
        }
      }
      c[1 + k] = slot;
    }
  }
}

// ============================================================================
// garbage collection (Sec. V-E)
// ============================================================================
__global__ __launch_bounds__(256) void k_gc(VolDev v) {
  const uint32_t n = v.cnt->vtx_hwm;
  const uint32_t tail = v.cnt->vtx_tail;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += stride) {
    const uint32_t i = base + threadIdx.x;
    const bool dead = i < n && v.vref[i] == 0;
    const uint32_t p = wave_ticket(&v.cnt->vtx_push, dead);
    if (dead) {
      v.evtx[v.vowner[i]] = -1;
      v.vref[i] = -1;
      v.vring[(uint32_t)(((uint64_t)tail + p) % v.max_vertices)] = i;
    }
  }
}

// ============================================================================
// download: two-level exclusive scans over the vertex and triangle pools
// ============================================================================
constexpr int kScanItems = 1024;  // items per workgroup (256 lanes x 4)

__device__ inline uint32_t item_count(const VolDev& v, int what, uint32_t i, uint32_t n) {
  if (i >= n) return 0;
  if (what == 0) return v.vref[i] > 0 ? 1u : 0u;
  const uint32_t* c = v.chunks + (size_t)i * kChunkWords;
  if (c[0] == kNone) return 0;
  uint32_t k = 0;
  for (int t = 0; t < 5; ++t) k += c[1 + 3 * t] != kNone;
  return k;
}

// Exclusive scan of one value per lane across a 256-lane workgroup.
__device__ inline uint32_t wg_exclusive_scan(uint32_t x, uint32_t* swave, uint32_t* total) {
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  uint32_t incl = x;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  if (lane == 63) swave[wave] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < wave) before += swave[w];
    all += swave[w];
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

__global__ __launch_bounds__(256) void k_dl_count(VolDev v, int what) {
  __shared__ uint32_t swave[4];
  const uint32_t n = what == 0 ? v.cnt->vtx_hwm : v.cnt->chk_hwm;
  const uint32_t i0 = blockIdx.x * kScanItems + threadIdx.x * 4;
  uint32_t c = 0;
  for (int k = 0; k < 4; ++k) c += item_count(v, what, i0 + k, n);
  uint32_t total;
  wg_exclusive_scan(c, swave, &total);
  if (threadIdx.x == 0) v.scan[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_dl_scan(VolDev v, int what, uint32_t nparts) {
  __shared__ uint32_t sw[16];
  __shared__ uint32_t carry;
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < nparts; base += 1024) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t x = i < nparts ? v.scan[i] : 0u;
    uint32_t incl = x;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(incl, off);
      if (lane >= off) incl += y;
    }
    if (lane == 63) sw[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < 16; ++w) {
      if (w < wave) before += sw[w];
      all += sw[w];
    }
    if (i < nparts) v.scan[i] = carry + before + incl - x;
    __syncthreads();
    if (threadIdx.x == 0) carry += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (what == 0) v.cnt->dl_nv = carry;
    else v.cnt->dl_nt = carry;
  }
}

__global__ __launch_bounds__(256) void k_dl_write_vertices(VolDev v, float* __restrict__ verts,
                                                           uint64_t* __restrict__ keys,
                                                           uint32_t vcap) {
  __shared__ uint32_t swave[4];
  const uint32_t n = v.cnt->vtx_hwm;
  const uint32_t i0 = blockIdx.x * kScanItems + threadIdx.x * 4;
  uint32_t live[4], c = 0;
  for (int k = 0; k < 4; ++k) c += (live[k] = item_count(v, 0, i0 + k, n));
  uint32_t total;
  uint32_t j = v.scan[blockIdx.x] + wg_exclusive_scan(c, swave, &total);
  for (int k = 0; k < 4; ++k) {
    const uint32_t i = i0 + k;
    if (i >= n) break;
    if (!live[k]) {
      v.vdl[i] = -1;
      continue;
    }
    v.vdl[i] = (int32_t)j;
    if (j < vcap) {
      const uint32_t owner = v.vowner[i];
      const uint32_t blk = owner / (3 * kVox), rem = owner % (3 * kVox);
      const int axis = (int)(rem / kVox), local = (int)(rem % kVox);
      const uint64_t bkey = v.block_key[blk];
      int bx, by, bz;
      unpack_key(bkey, bx, by, bz);
      const int g[3] = {8 * bx + (local & 7), 8 * by + ((local >> 3) & 7), 8 * bz + (local >> 6)};
      const float t = v.vt[i];
      for (int a = 0; a < 3; ++a) {
        float p = (float)g[a];
        if (a == axis) p = p + t;
        verts[3 * (size_t)j + a] = p * v.s;
      }
      if (keys) keys[j] = edge_key(bkey, local, axis);
    }
    ++j;
  }
}

__global__ __launch_bounds__(256) void k_dl_write_triangles(VolDev v, int32_t* __restrict__ tris,
                                                            uint32_t tcap) {
  __shared__ uint32_t swave[4];
  const uint32_t n = v.cnt->chk_hwm;
  const uint32_t i0 = blockIdx.x * kScanItems + threadIdx.x * 4;
  uint32_t c = 0;
  for (int k = 0; k < 4; ++k) c += item_count(v, 1, i0 + k, n);
  uint32_t total;
  uint32_t j = v.scan[blockIdx.x] + wg_exclusive_scan(c, swave, &total);
  for (int k = 0; k < 4; ++k) {
    const uint32_t i = i0 + k;
    if (i >= n) break;
    const uint32_t* ch = v.chunks + (size_t)i * kChunkWords;
    if (ch[0] == kNone) continue;
    for (int t = 0; t < 5; ++t) {
      if (ch[1 + 3 * t] == kNone) continue;
      if (j < tcap) {
        for (int q = 0; q < 3; ++q) {
          const uint32_t s = ch[1 + 3 * t + q];
          tris[3 * (size_t)j + q] = s == kNone ? -1 : v.vdl[s];
        }
      }
      ++j;
    }
  }
}

// ============================================================================
// backward passes
// ============================================================================

// dL/d(TSDF) at every voxel of every block: gather over the at most six
// edges incident to the voxel (its own three, and the three owned by its
// -x/-y/-z neighbours), in a fixed order.
__global__ __launch_bounds__(512) void k_bwd_tsdf(VolDev v, const float* __restrict__ dL_dv,
                                                  float* __restrict__ out) {
  __shared__ float sd[1000];  // TSDF at local -1..8
  __shared__ int32_t snb[27];
  const uint32_t n = min(v.cnt->n_blocks, v.max_blocks);
  const uint32_t nv = v.cnt->dl_nv;
  const int l = threadIdx.x, lx = l & 7, ly = (l >> 3) & 7, lz = l >> 6;
  const int lc[3] = {lx, ly, lz};
  for (uint32_t idx = blockIdx.x; idx < n; idx += gridDim.x) {
    if (l < 27) snb[l] = v.nbr[(size_t)idx * 27 + l];
    __syncthreads();
    for (int j = l; j < 1000; j += 512) {
      const int x = j % 10 - 1, y = (j / 10) % 10 - 1, z = j / 100 - 1;
      const int nb = snb[nbr_dir(x < 0 ? -1 : (x > 7 ? 1 : 0), y < 0 ? -1 : (y > 7 ? 1 : 0),
                                 z < 0 ? -1 : (z > 7 ? 1 : 0))];
      sd[j] = nb >= 0 ? v.d[(size_t)nb * kVox + (x & 7) + 8 * (y & 7) + 64 * (z & 7)] : 0.f;
    }
    __syncthreads();
    const int c = (lx + 1) + 10 * (ly + 1) + 100 * (lz + 1);
    const int step[3] = {1, 10, 100};
    float acc = 0.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      // the edge this voxel owns: it is the first end point
      int32_t s = v.evtx[((size_t)idx * 3 + a) * kVox + l];
      if (s >= 0 && v.vref[s] > 0) {
        const int32_t r = v.vdl[s];
        if (r >= 0 && (uint32_t)r < nv) {
          const float da = sd[c], db = sd[c + step[a]];
          if (da != db) {
            const float g = dL_dv[3 * (size_t)r + a] * v.s;
            const float den = (da - db) * (da - db);
            acc = acc + g * (-db / den);
          }
        }
      }
      // the edge its -a neighbour owns: it is the second end point
      const int back = lc[a] - 1;
      const int dir = nbr_dir(a == 0 && back < 0 ? -1 : 0, a == 1 && back < 0 ? -1 : 0,
                              a == 2 && back < 0 ? -1 : 0);
      const int32_t nb = snb[dir];
      if (nb >= 0) {
        // local index of the owner: one step back along a, wrapping into
        // the -a neighbour block when this voxel is on the block's face
        const int lstep = a == 0 ? 1 : a == 1 ? 8 : 64;
        const int ol = back < 0 ? l + 7 * lstep : l - lstep;
        s = v.evtx[((size_t)nb * 3 + a) * kVox + ol];
        if (s >= 0 && v.vref[s] > 0) {
          const int32_t r = v.vdl[s];
          if (r >= 0 && (uint32_t)r < nv) {
            const float da = sd[c - step[a]], db = sd[c];
            if (da != db) {
              const float g = dL_dv[3 * (size_t)r + a] * v.s;
              const float den = (da - db) * (da - db);
              acc = acc + g * (da / den);
            }
          }
        }
      }
    }
    out[(size_t)idx * kVox + l] = acc;
    __syncthreads();
  }
}

// Backward of the last fusion (Eq. 2) with its branches fixed.
__global__ __launch_bounds__(512) void k_bwd_fusion(VolDev v, FrameParams fp,
                                                    const float* __restrict__ depth,
                                                    const float* __restrict__ g1,
                                                    float* __restrict__ g0,
                                                    float* __restrict__ gD) {
  const uint32_t n = min(v.cnt->n_blocks, v.max_blocks);
  const int l = threadIdx.x, lx = l & 7, ly = (l >> 3) & 7, lz = l >> 6;
  for (uint32_t idx = blockIdx.x; idx < n; idx += gridDim.x) {
    const size_t o = (size_t)idx * kVox + l;
    const float g = g1[o];
    float out = g;
    if (v.st_frame[idx] == fp.frame) {
      int bx, by, bz;
      unpack_key(v.block_key[idx], bx, by, bz);
      const FuseSample fs = fuse_sample(v, fp, depth, 8 * bx + lx, 8 * by + ly, 8 * bz + lz);
      if (fs.upd) {
        const float W1 = v.w[o];
        const float W0 = W1 - 1.0f;
        out = g * (W0 / W1);
        if (!fs.clamped && g != 0.f) unsafeAtomicAdd(&gD[fs.pixel], g * (v.inv_s / W1));
      }
    }
    g0[o] = out;
  }
}

__global__ void k_zero_f32(float* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

// ============================================================================
// inspection
// ============================================================================
__global__ void k_export_vertices(VolDev v, uint64_t* keys, float* t, int32_t* ref, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int32_t r = v.vref[i];
    ref[i] = r;
    t[i] = v.vt[i];
    uint64_t k = ~0ull;
    if (r >= 0) {
      const uint32_t owner = v.vowner[i];
      const uint32_t blk = owner / (3 * kVox), rem = owner % (3 * kVox);
      k = edge_key(v.block_key[blk], (int)(rem % kVox), (int)(rem / kVox));
    }
    keys[i] = k;
  }
}

}  // namespace vm
