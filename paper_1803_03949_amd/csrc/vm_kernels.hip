// HIP kernels of the voxmesh library for gfx950 (wave64).
//
// Per-block work (fusion, import, classification, vertices, the TSDF
// backward) gives each 8^3 block one wave: lane q owns the column of eight
// voxels or cubes at (q & 7, q >> 3), and the block's halo is staged in the
// wave's own LDS, so waves of a workgroup never wait for each other.  Work
// lists live on the device and every kernel loops over its list on a grid
// sized to the device, so the host never waits for a count.  Lists are
// appended to with at most one atomic per workgroup (per wave for the short
// list of extra vertex blocks); pool allocations take one atomic per block
// on the block's pool segment.
#include "voxmesh.h"
#include "vm_internal.h"

namespace vm {

// ============================================================================
// bookkeeping
// ============================================================================
// Close a vertex pool segment after an allocating pass: the ring entries
// taken are consumed, bumped slots raise the high-water mark, and the slots
// pushed by frees join the ring.  A free only returns a slot that was in use,
// so ring entries plus pushes never exceed the segment size.
__device__ inline void finalise_seg(Seg& g, uint32_t size) {
  const uint32_t from_ring = min(g.ticket, g.count);
  g.head = ring_pos(g.head, from_ring, size);
  const uint64_t hwm = (uint64_t)g.hwm + (g.ticket - from_ring);
  g.hwm = hwm > size ? size : (uint32_t)hwm;
  g.count = g.count - from_ring + g.push;
  g.ticket = 0;
  g.push = 0;
}

// Segment statistics summed over all segments (running counts, modulo 2^32).
struct SegSums {
  uint32_t nw, upd, freed, mov, chg, ref, fnew, fold;
};

// One full wave closes every vertex pool segment (lane q takes segments q,
// q + 64, ...: slots freed by earlier passes become available) and sums the
// segment statistics; every lane receives the sums.
__device__ inline SegSums close_segments(const VolDev& v) {
  static_assert(kSegs % 64 == 0, "whole waves of segments");
  constexpr int kPer = kSegs / 64;
  SegSums r{0, 0, 0, 0, 0, 0, 0, 0};
  // every lane's segments are read before any is written back
  Seg g[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int s = __lane_id() + 64 * j;
    g[j] = v.vseg[s];
    const Seg& cs = v.cseg[s];
    r.chg += cs.st_chg, r.ref += cs.st_ref, r.fnew += cs.st_fnew, r.fold += cs.st_fold;
  }
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int s = __lane_id() + 64 * j;
    r.nw += g[j].st_new, r.upd += g[j].st_upd, r.freed += g[j].st_freed, r.mov += g[j].st_mov;
    finalise_seg(g[j], seg_size(s, v.vseg_cap, v.max_vertices));
    Seg& vs = v.vseg[s];
    vs.hwm = g[j].hwm, vs.head = g[j].head, vs.count = g[j].count;
    vs.ticket = 0, vs.push = 0;
  }
  r.nw = wave_sum(r.nw), r.upd = wave_sum(r.upd), r.freed = wave_sum(r.freed);
  r.mov = wave_sum(r.mov), r.chg = wave_sum(r.chg), r.ref = wave_sum(r.ref);
  r.fnew = wave_sum(r.fnew), r.fold = wave_sum(r.fold);
  return r;
}

// Start of an extraction (refine = false) or refinement, done by one full
// wave while nothing else touches the segments: the segments are closed,
// and lane 0 records the statistics the call reports per call and clears
// the list lengths of the next call.
__device__ inline void begin_call(const VolDev& v, bool refine) {
  const SegSums m = close_segments(v);
  const uint32_t sum_new = m.nw, sum_upd = m.upd, sum_freed = m.freed, sum_chg = m.chg,
                 sum_ref = m.ref;
  if (__lane_id() != 0) return;
  Counters* c = v.cnt;
  if (!refine) c->n_dirty[v.xsel ^ 1u] = 0;
  c->n_vblocks[v.vsel ^ 1u] = 0;
  c->base_new = sum_new;
  c->base_upd = sum_upd;
  c->base_freed = sum_freed;
  c->base_chg = sum_chg;
  c->base_ref = sum_ref;
}

// One wave: the segments are closed and their statistics summed, then lane
// 0 does the operation's resets and snapshots.
__global__ __launch_bounds__(64) void k_prep(VolDev v, int op, uint32_t arg) {
  if (op == VM_OP_REFINE) {
    begin_call(v, true);
    return;
  }
  const SegSums m = close_segments(v);
  if (threadIdx.x != 0) return;
  Counters* c = v.cnt;
  switch (op) {
    case VM_OP_RESET:
      c->acc[VM_TOTAL_NEW_TRIANGLES] += m.fnew;
      c->acc[VM_TOTAL_DROPPED_TRIANGLES] += m.fold;
      c->acc[VM_TOTAL_NEW_VERTICES] += m.nw;
      c->acc[VM_TOTAL_UPDATED_VERTICES] += m.upd;
      c->acc[VM_TOTAL_MOVED_VERTICES] += m.mov;
      c->acc[VM_TOTAL_FREED_VERTICES] += m.freed;
      c->acc[VM_TOTAL_CHANGED_CUBES] += m.chg;
      c->acc[VM_TOTAL_REFINED_CUBES] += m.ref;
      break;
    default:
      break;
  }
  (void)arg;
}

// ============================================================================
// block collection (Eq. 1)
// ============================================================================

// One lane per pixel, one wave per 8 x 8 tile of pixels, a workgroup per
// 32 x 16 tile.  Each valid pixel spans the integer box of blocks between
// its ray points at camera depth D - mu and D + mu.  Neighbouring pixels
// span nearly the same blocks, so the wave first forms the union of its
// pixels' boxes as a bit mask over a 4 x 4 x 4 window of blocks placed at
// one pixel's box (an OR over the wave), and its lanes then take the
// distinct blocks one each; a pixel whose box leaves the window (a depth
// edge inside the tile) has its blocks agreed on by a slower ballot loop.
// The lanes holding distinct blocks insert them into the hash and claim the
// slot for this frame (exchange of the slot's frame stamp): the one claim
// that wins lists the block.  The workgroup gathers its claims in LDS and
// appends them with one atomic per list: the frame list, the pending list
// (blocks touched since the last extraction) and, for blocks new to the
// hash, pool indices, given here with their neighbour tables cleared.  The
// three appends are one packed 64-bit atomic (one per workgroup): atomics
// on one address from every workgroup are what limits this kernel.
constexpr int kTileW = 32, kTileH = 16;  // pixels per workgroup (8 waves of 8 x 8)
constexpr int kClaimCap = 512;   // claims per workgroup gathered in LDS
constexpr int kWaveKeys = 128;   // keys a wave gathers in its slow loop before claiming them

// List a claimed block: frame list entry, pending list entry (once per
// extraction epoch) and, for a block new to the hash, its pool index (slot
// value and key record updated, neighbour table cleared).  fpos, ppos and
// bidx are the positions the caller reserved.
__device__ inline void list_claim(const VolDev& v, uint32_t s, unsigned long long seen,
                                  bool pend, uint32_t fpos, uint32_t ppos, uint32_t bidx,
                                  uint32_t epoch) {
  uint32_t idx = (uint32_t)(seen & kIdxMask), entry = idx;
  if (idx == kPending) {
    if (bidx < v.max_blocks) {
      idx = bidx;
      const uint64_t key = seen >> kIdxBits;
      v.slots[s] = (key << kIdxBits) | idx;
      v.block_key[idx] = key;
      int32_t* nb = v.nbr + (size_t)idx * 27;
      for (int d = 0; d < 27; ++d) nb[d] = d == kSelf ? (int32_t)idx : -1;
      entry = idx | kNewFlag;
    } else {
      atomicOr(&v.cnt->error, kErrBlocks);
      idx = kNone;
      entry = kNone;
    }
  }
  if (fpos < v.max_blocks) {
    v.frame_list[fpos] = entry;
    v.frame_key[fpos] = seen >> kIdxBits;
  } else {
    atomicOr(&v.cnt->error, kErrBlocks);
  }
  if (pend) {
    if (idx != kNone) v.st_pending[idx] = epoch;
    if (ppos < v.max_blocks) v.pending[ppos] = idx;
    else atomicOr(&v.cnt->error, kErrBlocks);
  }
}

__global__ __launch_bounds__(512) void k_collect(VolDev v, FrameParams fp,
                                                const float* __restrict__ depth, uint32_t epoch) {
  __shared__ unsigned long long sseen[kClaimCap];  // slot contents seen by the claim
  __shared__ uint32_t sslot[kClaimCap];            // slot | pending << 31
  __shared__ unsigned long long skeys_all[8][kWaveKeys];  // each wave's slow-loop keys
  __shared__ uint8_t sunion_all[8][64];                   // each wave's union, as cells
  __shared__ uint32_t nclaim;
  __shared__ uint32_t swave[8];
  __shared__ uint32_t sbase[3];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), q = __lane_id();
  const int tiles_x = (fp.W + kTileW - 1) / kTileW;
  const int px = (int)(blockIdx.x % tiles_x) * kTileW + (wave & 3) * 8 + (q & 7);
  const int py = (int)(blockIdx.x / tiles_x) * kTileH + (wave >> 2) * 8 + (q >> 3);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // the other parity's list and appends are the next frame's
    v.cnt->n_frame[(fp.frame + 1) & 1] = 0;
    v.cnt->collect_acc[(fp.frame + 1) & 1] = 0;
    v.cnt->acc[VM_TOTAL_FRAMES] += 1;
  }
  // the lists this frame appends to: the frame list starts empty, the
  // pending list and the pool continue from where they stand (nothing else
  // changes them during this kernel)
  unsigned long long* acc = &v.cnt->collect_acc[fp.frame & 1];
  const uint32_t pend_base = v.cnt->n_pending[epoch & 1], blk_base = v.cnt->n_blocks;
  // cleared here, first used after the barrier below
  if (threadIdx.x == 0) nclaim = 0;
  int lo[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
  int nbox = 0;
  if (px < fp.W && py < fp.H) {
    const float D = depth[py * fp.W + px];
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
  // Claim one key per lane (has: the lane holds one): insert it, take the
  // slot's frame stamp, and gather the winners in the workgroup's list with
  // whether each must join the pending list.
  auto claim = [&](bool has, uint64_t key) {
    unsigned long long seen = 0;
    int64_t s = -1;
    if (has) {
      s = hash_insert_seen(v, key, &seen);
      if (s < 0) atomicOr(&v.cnt->error, kErrHash);
    }
    // one claim per block and frame wins (an exchange of the slot's frame
    // stamp); the block's pending stamp is requested with it (only the
    // winner of this frame's claim writes it)
    bool won = false, pend = false;
    if (s >= 0) {
      const uint32_t idx = (uint32_t)(seen & kIdxMask);
      const uint32_t pst = idx != kPending ? v.st_pending[idx] : 0u;
      won = atomicExch(&v.slot_stamp[s], fp.frame) != fp.frame;
      pend = won && (idx == kPending || pst != epoch);
    }
    const uint64_t bw = __ballot(won);
    if (bw == 0ull) return;
    uint32_t c0 = 0;
    if (q == 0) c0 = atomicAdd(&nclaim, (uint32_t)__popcll(bw));
    const uint32_t c = uniform(c0) + mask_rank(bw);
    if (!won) return;
    if (c < (uint32_t)kClaimCap) {
      sslot[c] = (uint32_t)s | (pend ? 0x80000000u : 0u);
      sseen[c] = seen;
    } else {
      // more claims than the workgroup gathers: list this one alone
      const bool isnew = (uint32_t)(seen & kIdxMask) == kPending;
      const uint64_t p = atomicAdd(acc, (unsigned long long)collect_pack(1u, pend, isnew));
      list_claim(v, (uint32_t)s, seen, pend, collect_frame(p), pend_base + collect_pend(p),
                 blk_base + collect_new(p), epoch);
    }
  };
  // the union of the boxes that fit the window, over the wave
  const uint64_t act = __ballot(nbox > 0);
  bool fits = true;
  int w0 = 0, w1 = 0, w2 = 0, cell = -1;
  if (act) {
    const int lead = __builtin_ctzll(act);
    w0 = __builtin_amdgcn_readlane(lo[0], lead) - 1;
    w1 = __builtin_amdgcn_readlane(lo[1], lead) - 1;
    w2 = __builtin_amdgcn_readlane(lo[2], lead) - 1;
    const int ox = lo[0] - w0, oy = lo[1] - w1, oz = lo[2] - w2;
    uint64_t m = 0;
    if (nbox > 0) {
      fits = ox >= 0 && oy >= 0 && oz >= 0 && ox + ext[0] <= 4 && oy + ext[1] <= 4 &&
             oz + ext[2] <= 4;
      if (fits) {
        // the box's rows along x as runs of bits
        const uint64_t row = ((1ull << ext[0]) - 1ull) << ox;
        for (int z = 0; z < ext[2]; ++z)
          for (int y = 0; y < ext[1]; ++y) m |= row << (4 * (oy + y) + 16 * (oz + z));
      }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) m |= shfl64(m, q ^ off);
    // lane k takes the union's k-th block: lane c, for a cell c in the
    // union, places it at its rank among the union's cells
    const uint64_t u = ((uint64_t)uniform((uint32_t)(m >> 32)) << 32) | uniform((uint32_t)m);
    uint8_t* sunion = sunion_all[wave];
    if ((u >> q) & 1ull) sunion[mask_rank(u)] = (uint8_t)q;
    wave_sync();
    if (q < __popcll(u)) cell = sunion[q];
  }
  __syncthreads();  // the claim count is cleared
  if (act)
    claim(cell >= 0, cell >= 0 ? pack_key(w0 + (cell & 3), w1 + ((cell >> 2) & 3), w2 + (cell >> 4))
                               : 0ull);
  // boxes that leave the window: the wave agrees on their distinct keys per
  // box position (duplicates between positions are left to the claim) and
  // claims them kWaveKeys at a time
  if (__ballot(!fits) != 0ull) {
    unsigned long long* skeys = skeys_all[wave];
    uint32_t nkeys = 0;
    auto claim_keys = [&]() {
      wave_sync();
      for (uint32_t i0 = 0; i0 < nkeys; i0 += 64) {
        const uint32_t i = i0 + (uint32_t)q;
        claim(i < nkeys, i < nkeys ? skeys[i] : 0ull);
      }
      nkeys = 0;
      wave_sync();
    };
    const int nslow = fits ? 0 : nbox;
    int cx = 0, cy = 0, cz = 0;
    const uint64_t below = lanes_below();
    for (int j = 0; __ballot(j < nslow); ++j) {
      bool has = j < nslow;
      uint64_t key = 0;
      if (has) {
        key = pack_key(lo[0] + cx, lo[1] + cy, lo[2] + cz);
        if (++cx == ext[0]) {
          cx = 0;
          if (++cy == ext[1]) cy = 0, ++cz;
        }
      }
      bool mine = false;  // this lane holds the first copy of its key
      uint64_t todo = __ballot(has);
      while (todo) {
        // the leader is wave-uniform: its key is read lane to scalar
        const int leader = __builtin_ctzll(todo);
        const uint32_t klo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)key, leader);
        const uint32_t khi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(key >> 32), leader);
        const uint64_t lk = ((uint64_t)khi << 32) | klo;
        const bool same = has && key == lk;
        todo &= ~__ballot(same);
        if (q == leader) mine = true;
        if (same) has = false;
      }
      const uint64_t bm = __ballot(mine);
      const uint32_t nm = (uint32_t)__popcll(bm);
      if (nkeys + nm > (uint32_t)kWaveKeys) claim_keys();
      if (mine) skeys[nkeys + (uint32_t)__popcll(bm & below)] = key;
      nkeys += nm;
    }
    claim_keys();
  }
  __syncthreads();
  // one claim per thread: the three lists' positions from one workgroup
  // scan of packed counts (fields of 10 bits, at most 512 each)
  const uint32_t nc = min(nclaim, (uint32_t)kClaimCap);
  const uint32_t c = threadIdx.x;
  const bool hit = c < nc;
  unsigned long long seen = 0;
  uint32_t slot = 0;
  bool isnew = false, pend = false;
  if (hit) {
    seen = sseen[c];
    slot = sslot[c];
    pend = (slot >> 31) != 0u;
    slot &= 0x7FFFFFFFu;
    isnew = (uint32_t)(seen & kIdxMask) == kPending;
  }
  const uint64_t bh = __ballot(hit), bn = __ballot(isnew), bp = __ballot(pend);
  if (q == 0)
    swave[wave] = (uint32_t)__popcll(bh) | (uint32_t)__popcll(bn) << 10 |
                  (uint32_t)__popcll(bp) << 20;
  __syncthreads();
  uint32_t before = 0, all = 0;
  const int nwave = (int)(blockDim.x >> 6);
  for (int w = 0; w < nwave; ++w) {
    const uint32_t cw = swave[w];
    if (w < wave) before += cw;
    all += cw;
  }
  if (threadIdx.x == 0 && (all & 1023u)) {
    const uint64_t p = atomicAdd(
        acc, (unsigned long long)collect_pack(all & 1023u, all >> 20, (all >> 10) & 1023u));
    sbase[0] = collect_frame(p);
    sbase[1] = blk_base + collect_new(p);
    sbase[2] = pend_base + collect_pend(p);
  }
  __syncthreads();
  if (hit)
    list_claim(v, slot, seen, pend, sbase[0] + (before & 1023u) + mask_rank(bh),
               sbase[2] + (before >> 20) + mask_rank(bp),
               sbase[1] + ((before >> 10) & 1023u) + mask_rank(bn), epoch);
}

__global__ void k_import_insert(VolDev v, const int32_t* __restrict__ slots,
                                const int32_t* __restrict__ coords, uint32_t n, uint32_t frame) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    // this import's list starts empty, and so does the next frame's: an
    // integration appends to its own parity's list (and packed appends)
    // without clearing them
    v.cnt->n_frame[frame & 1] = 0;
    v.cnt->n_frame[(frame + 1) & 1] = 0;
    v.cnt->collect_acc[0] = 0;
    v.cnt->collect_acc[1] = 0;
    v.cnt->acc[VM_TOTAL_FRAMES] += 1;
  }
  if (i >= n) return;
  v.row_slot[i] = kNone;  // until the row's key is in the table
  int x = coords[3 * i];
  const int y = coords[3 * i + 1], z = coords[3 * i + 2];
  if (slots) {
    const int k = slots[i];
    if (k < 0 || (uint32_t)k >= v.batch || x < 0 || x > kSlotSpan - 2) {
      atomicOr(&v.cnt->error, kErrRange);
      return;
    }
    x += kSlotSpan * k - kKeyBias;
  }
  if (!key_in_range(x, y, z)) {
    atomicOr(&v.cnt->error, kErrRange);
    return;
  }
  const int64_t s = hash_insert(v, pack_key(x, y, z));
  if (s < 0) {
    atomicOr(&v.cnt->error, kErrHash);
    return;
  }
  v.slot_stamp[s] = frame;
  v.slot_src[s] = i;
  v.row_slot[i] = (uint32_t)s;
}

// Row-order compaction of an import.  Of the rows naming one key, the row
// recorded last in its slot speaks for it.  Such a row lists its block in
// the frame list, numbers it when it is new and adds it to the pending list
// once per extraction epoch, all in row order: counts per part of
// kImportRows rows, one workgroup's scan over the parts, then the writes.
struct ImportRow {
  uint32_t s;       // hash slot
  uint32_t idx;     // pool index, kPending when new
  bool hit, fresh, pend;
};
__device__ inline ImportRow import_row(const VolDev& v, uint32_t i, uint32_t n, uint32_t epoch) {
  ImportRow r{kNone, kNone, false, false, false};
  if (i >= n) return r;
  r.s = v.row_slot[i];
  if (r.s == kNone || v.slot_src[r.s] != i) return r;
  r.hit = true;
  r.idx = (uint32_t)(v.slots[r.s] & kIdxMask);
  r.fresh = r.idx == kPending;
  r.pend = r.fresh || v.st_pending[r.idx] != epoch;
  return r;
}

__global__ __launch_bounds__(kImportRows) void k_import_count(VolDev v, uint32_t n,
                                                               uint32_t epoch) {
  __shared__ uint32_t swave[16];
  const ImportRow r = import_row(v, blockIdx.x * kImportRows + threadIdx.x, n, epoch);
  uint32_t t_hit, t_new, t_pend;
  wg_scan_bits<1>(r.hit, swave, &t_hit);
  wg_scan_bits<1>(r.fresh, swave, &t_new);
  wg_scan_bits<1>(r.pend, swave, &t_pend);
  if (threadIdx.x == 0) {
    v.scan[3 * blockIdx.x] = t_hit;
    v.scan[3 * blockIdx.x + 1] = t_new;
    v.scan[3 * blockIdx.x + 2] = t_pend;
  }
}

// Exclusive scans of the three per-part counts, offset by the list lengths
// and the pool high-water mark, which then grow by the totals.
__global__ __launch_bounds__(1024) void k_import_scan(VolDev v, uint32_t nparts, uint32_t frame,
                                                      uint32_t epoch) {
  __shared__ uint32_t swave[16];
  __shared__ uint32_t carry[3];
  uint32_t* len[3] = {&v.cnt->n_frame[frame & 1], &v.cnt->n_blocks, &v.cnt->n_pending[epoch & 1]};
  if (threadIdx.x < 3) carry[threadIdx.x] = *len[threadIdx.x];
  __syncthreads();
  if (threadIdx.x == 0) v.cnt->import_base = carry[1];
  for (uint32_t base = 0; base < nparts; base += 1024) {
    const uint32_t p = base + threadIdx.x;
    for (int k = 0; k < 3; ++k) {
      const uint32_t x = p < nparts ? v.scan[3 * p + k] : 0u;
      uint32_t all;
      const uint32_t before = wg_scan(x, swave, &all);
      if (p < nparts) v.scan[3 * p + k] = carry[k] + before;
      __syncthreads();
      if (threadIdx.x == 0) carry[k] += all;
      __syncthreads();
    }
  }
  if (threadIdx.x < 3) *len[threadIdx.x] = carry[threadIdx.x];
}

__global__ __launch_bounds__(kImportRows) void k_import_assign(VolDev v, uint32_t n,
                                                                uint32_t nparts, uint32_t epoch) {
  __shared__ uint32_t swave[16];
  const uint32_t i = blockIdx.x * kImportRows + threadIdx.x;
  const ImportRow r = import_row(v, i, n, epoch);
  uint32_t t_hit, t_new, t_pend;
  const uint32_t pos = v.scan[3 * blockIdx.x] + wg_scan_bits<1>(r.hit, swave, &t_hit);
  const uint32_t t = v.scan[3 * blockIdx.x + 1] + wg_scan_bits<1>(r.fresh, swave, &t_new);
  const uint32_t p = v.scan[3 * blockIdx.x + 2] + wg_scan_bits<1>(r.pend, swave, &t_pend);
  if (!r.hit) return;
  uint32_t idx = r.idx, entry = r.idx;
  if (r.fresh) {
    if (t < v.max_blocks) {
      idx = t;
      const uint64_t key = v.slots[r.s] >> kIdxBits;
      v.slots[r.s] = (key << kIdxBits) | idx;
      v.block_key[idx] = key;
      int32_t* nb = v.nbr + (size_t)idx * 27;
      for (int d = 0; d < 27; ++d) nb[d] = d == kSelf ? (int32_t)idx : -1;
      entry = idx | kNewFlag;
    } else {
      atomicOr(&v.cnt->error, kErrBlocks);
      idx = kNone;
      entry = kNone;
    }
  }
  if (pos < v.max_blocks) {
    v.frame_list[pos] = entry;
    v.frame_src[pos] = i;
  } else {
    atomicOr(&v.cnt->error, kErrBlocks);
  }
  if (r.pend) {
    if (idx != kNone) v.st_pending[idx] = epoch;
    if (p < v.max_blocks) v.pending[p] = idx;
    else atomicOr(&v.cnt->error, kErrBlocks);
  }
}

// Link a new block with its 26 neighbours in both directions (lanes 0..26
// of the workgroup handling it).  With forward_only, only the 13 neighbours
// after it (l > kSelf) are looked up: enough when every block present is
// new in the same call, as each pair is then linked by its first block.
__device__ inline void link_block(const VolDev& v, uint32_t idx, int l, bool forward_only = false) {
  if (l >= 27 || l == kSelf || (forward_only && l < kSelf)) return;
  int x, y, z;
  unpack_key(v.block_key[idx], x, y, z);
  const int nx = x + l % 3 - 1, ny = y + (l / 3) % 3 - 1, nz = z + l / 9 - 1;
  if (!key_in_range(nx, ny, nz)) return;
  const int32_t nb = hash_find(v, pack_key(nx, ny, nz));
  if (nb < 0) return;
  v.nbr[(size_t)idx * 27 + l] = nb;
  v.nbr[(size_t)nb * 27 + (26 - l)] = (int32_t)idx;
}

// A new block's column q of cubes: no type, and none of the column's edges
// holds a vertex (an edge's slot is meaningful only under its set bit, so
// the slots are not written).
__device__ inline void init_column(const VolDev& v, uint32_t idx, int q) {
#pragma unroll
  for (int lz = 0; lz < 8; ++lz) {
    const size_t o = (size_t)idx * kVox + q + 64 * lz;
    v.tprev[o] = 0;
    v.tcur[o] = 0;
  }
  v.emask[(size_t)idx * 64 + q] = 0;
}

// ============================================================================
// fusion (Eq. 2) and import
// ============================================================================
// One wave per collected block, eight voxels per lane (one column of the
// block), so that many blocks are in flight per CU.  The list entry and
// block key of the wave's next block are requested one block ahead, so a
// block waits only for its TSDF, weights and depth samples; with the
// strided mapping a wave's first item does not depend on the list length,
// and its entry and key are requested together with it (an entry past the
// length is ignored).
template <int W>
__global__ __launch_bounds__(64 * W) void k_fuse(VolDev v, FrameParams fp,
                                                 const float* __restrict__ depth, uint32_t epoch) {
  // the collection's appends: its frame list length, and (one thread) the
  // lengths the later kernels read
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const bool strided = (v.order & 3u) == 0u;
  const uint32_t i0 = blockIdx.x * W + (uint32_t)wave;
  uint32_t e0 = kNone;
  uint64_t k0 = 0;
  if (strided && i0 < v.max_blocks) e0 = v.frame_list[i0], k0 = v.frame_key[i0];
  const uint64_t app = v.cnt->collect_acc[fp.frame & 1];
  const uint32_t n = min(collect_frame(app), v.max_blocks);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    v.cnt->acc[VM_TOTAL_FRAME_BLOCKS] += n;
    v.cnt->n_frame[fp.frame & 1] = collect_frame(app);
    v.cnt->n_pending[epoch & 1] += collect_pend(app);
    v.cnt->n_blocks += collect_new(app);
  }
  ItemLoop it = item_loop(v, n, W, wave);
  auto entry = [&](uint32_t i) -> uint32_t { return i < it.end ? v.frame_list[i] : kNone; };
  auto key_at = [&](uint32_t i) -> uint64_t { return i < it.end ? v.frame_key[i] : 0ull; };
  // this block's entry and key
  uint32_t e1 = strided ? (it.i < it.end ? e0 : kNone) : entry(it.i);
  uint64_t k1 = strided ? k0 : key_at(it.i);
  for (; it.i < it.end; it.i += it.step) {
    const uint32_t e = uniform(e1);
    const uint64_t key = ((uint64_t)uniform((uint32_t)(k1 >> 32)) << 32) | uniform((uint32_t)k1);
    e1 = entry(it.i + it.step);
    k1 = key_at(it.i + it.step);
    if (e == kNone) continue;
    const int q = fresh_lane(), lx = q & 7, ly = q >> 3;
    const uint32_t idx = e & ~kNewFlag;
    const bool isnew = (e & kNewFlag) != 0;
    int bx, by, bz;
    unpack_key(key, bx, by, bz);
    float d[8], w[8];
    if (isnew) {
      init_column(v, idx, q);
#pragma unroll
      for (int lz = 0; lz < 8; ++lz) d[lz] = 0.f, w[lz] = 0.f;
      link_block(v, idx, q);
    } else {
#pragma unroll
      for (int lz = 0; lz < 8; ++lz) {
        d[lz] = v.d[(size_t)idx * kVox + q + 64 * lz];
        w[lz] = v.w[(size_t)idx * kVox + q + 64 * lz];
      }
    }
    // every voxel's depth sample is requested before any is used (a voxel
    // that projects nowhere reads pixel 0 and ignores it)
    FuseProj pr[8];
    float D[8];
#pragma unroll
    for (int lz = 0; lz < 8; ++lz) {
      pr[lz] = fuse_project(v, fp, 8 * bx + lx, 8 * by + ly, 8 * bz + lz);
      D[lz] = depth[pr[lz].pix >= 0 ? pr[lz].pix : 0];
    }
    // lane lz < 8 keeps the observed, negative-TSDF and near-zero (|TSDF| <
    // eps, the refinement's test) masks of layer lz
    uint64_t mine = 0, mneg = 0, mnear = 0;
#pragma unroll
    for (int lz = 0; lz < 8; ++lz) {
      const FuseSample fs = fuse_finish(v, fp, pr[lz], D[lz]);
      const size_t o = (size_t)idx * kVox + q + 64 * lz;
      float dn = d[lz];
      if (fs.upd) {
        float num = d[lz] * w[lz];
        num = num + fs.dt;
        const float den = w[lz] + 1.0f;
        dn = num / den;
        v.d[o] = dn;
        v.w[o] = den;
      } else if (isnew) {
        v.d[o] = d[lz];
        v.w[o] = w[lz];
      }
      const uint64_t m = __ballot(fs.upd || w[lz] > 0.f), mn = __ballot(dn < 0.f);
      const uint64_t mz = __ballot(fabsf(dn) < v.eps);
      if (q == lz) mine = m, mneg = mn, mnear = mz;
    }
    if (q < 8) {
      v.wmask[(size_t)idx * 8 + q] = mine;
      v.smask[(size_t)idx * 8 + q] = mneg;
      v.nmask[(size_t)idx * 8 + q] = mnear;
    }
    if (q == 0) v.st_frame[idx] = fp.frame;
  }
}

// One wave per imported block, eight voxels per lane: the caller's rows are
// read first, then the new block is initialised and linked while they
// arrive.  With bound arrays (the caller's rows are the volume's TSDF and
// weights) a block must land on its own row, and nothing is copied: the
// rows are read only for the observed-voxel and negative-TSDF masks.
template <int W>
__global__ __launch_bounds__(64 * W) void k_import_copy(VolDev v, const float* __restrict__ tsdf,
                                                        const float* __restrict__ weight,
                                                        uint32_t frame, int32_t* __restrict__ rows) {
  const uint32_t n = min(v.cnt->n_frame[frame & 1], v.max_blocks);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (blockIdx.x == 0 && threadIdx.x == 0) v.cnt->acc[VM_TOTAL_FRAME_BLOCKS] += n;
  // into an empty pool every neighbour is new too: link forward only
  const bool forward_only = v.cnt->import_base == 0;
  for (ItemLoop it = item_loop(v, n, W, wave); it.i < it.end; it.i += it.step) {
    const uint32_t e = uniform(v.frame_list[it.i]);
    const uint32_t row = uniform(v.frame_src[it.i]);
    if (e == kNone) continue;
    const int q = fresh_lane();
    const uint32_t idx = e & ~kNewFlag;
    if (v.bound && idx != row) {
      if (q == 0) atomicOr(&v.cnt->error, kErrRange);
      continue;
    }
    float d[8], w[8];
#pragma unroll
    for (int lz = 0; lz < 8; ++lz) {
      d[lz] = tsdf[(size_t)row * kVox + q + 64 * lz];
      w[lz] = weight[(size_t)row * kVox + q + 64 * lz];
    }
    if (e & kNewFlag) {
      init_column(v, idx, q);
      link_block(v, idx, q, forward_only);
    }
#pragma unroll
    for (int lz = 0; lz < 8; ++lz) {
      if (!v.bound) {
        v.d[(size_t)idx * kVox + q + 64 * lz] = d[lz];
        v.w[(size_t)idx * kVox + q + 64 * lz] = w[lz];
      }
      const uint64_t m = __ballot(w[lz] > 0.f), mn = __ballot(d[lz] < 0.f);
      const uint64_t mz = __ballot(fabsf(d[lz]) < v.eps);
      if (q == 0) {
        v.wmask[(size_t)idx * 8 + lz] = m;
        v.smask[(size_t)idx * 8 + lz] = mn;
        v.nmask[(size_t)idx * 8 + lz] = mz;
      }
    }
    if (q == 0) {
      v.st_frame[idx] = frame;
      if (rows) rows[row] = (int32_t)idx;
    }
  }
}

// ============================================================================
// extraction: dirty set, classification (+ refinement), vertices, triangles
// ============================================================================

// Dirty = pending blocks and their allocated neighbours at offsets {-1,0}^3.
// Candidates (8 per pending block) are claimed through a per-block pass
// stamp and compacted tile by tile, one atomic per tile.
// The last workgroup's first wave also starts the extraction (segments,
// statistics, next list lengths): nothing else in this kernel touches them,
// and the last workgroup has the fewest candidates (usually none), so the
// chain of dependent accesses this takes runs beside the claims.
__global__ __launch_bounds__(256) void k_dirty(VolDev v, uint32_t pass, uint32_t epoch) {
  __shared__ uint32_t swave[16];
  __shared__ uint32_t sbase;
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x < 64) begin_call(v, false);
  const uint32_t np = min(v.cnt->n_pending[epoch & 1], v.max_blocks);
  if (blockIdx.x == 0 && threadIdx.x == 0) v.cnt->n_pending[(epoch + 1) & 1] = 0;
  const uint32_t total = np * 8u;
  for (uint32_t t0 = blockIdx.x * kTile; t0 < total; t0 += gridDim.x * kTile) {
    int32_t got[kTilePer];
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < kTilePer; ++k) {
      const uint32_t t = t0 + threadIdx.x * kTilePer + k;
      got[k] = -1;
      if (t >= total) continue;
      const uint32_t idx = v.pending[t >> 3], o = t & 7u;
      if (idx == kNone) continue;
      const int32_t nb =
          v.nbr[(size_t)idx * 27 + nbr_dir(-(int)(o & 1), -(int)((o >> 1) & 1), -(int)(o >> 2))];
      if (nb >= 0 && atomicMax(&v.st_dirty[nb], pass) < pass) {
        got[k] = nb;
        ++cnt;
      }
    }
    uint32_t tot;
    uint32_t r = wg_scan_bits<kTileBits>(cnt, swave, &tot);  // cnt <= kTilePer
    if (tot == 0) continue;
    if (threadIdx.x == 0) sbase = atomicAdd(&v.cnt->n_dirty[v.xsel], tot);
    __syncthreads();
    r += sbase;
#pragma unroll
    for (int k = 0; k < kTilePer; ++k)
      if (got[k] >= 0) v.dirty[r++] = (uint32_t)got[k];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_dirty_all(VolDev v, uint32_t pass) {
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x < 64) begin_call(v, false);
  const uint32_t n = min(v.cnt->n_blocks, v.max_blocks);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    v.dirty[i] = i;
    v.st_dirty[i] = pass;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    v.cnt->n_dirty[v.xsel] = n;
    v.cnt->n_pending[0] = 0;
    v.cnt->n_pending[1] = 0;
  }
}

// One wave per dirty block, four blocks per workgroup, no workgroup
// barriers: per-block work is a chain of dependent memory round trips, and
// many independent waves hide it better than one wide workgroup.  Lane q
// owns the column (q & 7, q >> 3) of cubes, z = 0..7.  What the cubes need
// of their corners, the block's and its +x/+y/+z halo layer (9^3), is one
// bit each, read from per-block masks that fusion and import keep and
// staged in the wave's LDS: the sign, whether the corner is observed and,
// for refinement, whether |TSDF| < eps; the TSDF itself is never read.
// Mode, fixed at compile time so that each keeps only its own code:
// kExtract: new cube types from the signs (Sec. V-B), previous type saved;
// kExtractRefined: the same, each new type refined by Eqs. (3)-(5) against
// the type it replaces before it is written (Sec. V-F applies the regular
// type before marching cubes); kRefine: Eqs. (3)-(5) applied to the current
// types (Sec. V-F).
// Writing a cube's new type replaces its triangles (Sec. V-D): the type
// names them and the edges they use, and a cube whose type is unchanged
// keeps them.  The blocks whose vertices must be recomputed: on extraction
// every dirty block (its edges' end points may have moved) and the
// neighbours, not dirty themselves, that own edges of changed cubes on its
// +x/+y/+z faces, appended to a short list; on refinement the owners of the
// edges of changed cubes (this block and neighbours), claimed once per pass
// and written as candidates at fixed positions 8i..8i+7 for compaction.
template <int W, int refine>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(8))) void k_classify(VolDev v, uint32_t pass) {
  __shared__ uint32_t smk_all[W][3 * 128];  // the eight blocks' masks, in 32-bit halves
  __shared__ uint32_t srow_all[W][2 * 81];  // corner rows: signs | observed << 16, near
  __shared__ int32_t snb_all[W][8];
  // per cube type: its triangles, and in bit 8 whether it has any; for
  // refinement its regular-type candidates
  __shared__ uint16_t sntri[256];
  __shared__ uint32_t scand_lo[refine ? 256 : 1], scand_hi[refine ? 256 : 1];
  // with the strided mapping the wave's first block is requested at once,
  // before the list length (an entry past the length is ignored)
  const bool strided = (v.order & 3u) == 0u;
  const uint32_t i0 = blockIdx.x * W + (threadIdx.x >> 6);
  const uint32_t d0 = strided && i0 < v.max_blocks ? v.dirty[i0] : kNone;
  for (int j = threadIdx.x; j < 256; j += blockDim.x) {
    const uint32_t nt = v.tri_table[j * 16];
    sntri[j] = (uint16_t)(nt | (nt ? 256u : 0u));
    if (refine) {
      const uint64_t c = refine_candidates((uint32_t)j);
      scand_lo[j] = (uint32_t)c;
      scand_hi[j] = (uint32_t)(c >> 32);
    }
  }
  __syncthreads();
  auto refined = [&](uint32_t t, uint32_t prev, uint32_t near8) -> uint32_t {
    const uint64_t cand = (uint64_t)scand_hi[t] << 32 | scand_lo[t];
    return refine_type(t, prev, (scand_hi[prev] >> 31) != 0u, near8, cand);
  };
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t* smk = smk_all[wave];
  uint32_t* srow = srow_all[wave];
  uint32_t* nrow = srow_all[wave] + 81;
  int32_t* snb = snb_all[wave];
  const uint32_t n = min(v.cnt->n_dirty[v.xsel], v.max_blocks);
  if (blockIdx.x == 0 && threadIdx.x == 0) v.cnt->acc[VM_TOTAL_DIRTY_BLOCKS] += n;
  for (ItemLoop it = item_loop(v, n, W, wave); it.i < it.end; it.i += it.step) {
    // lane addressing is formed again per block (fewer registers)
    const int q = fresh_lane(), lx = q & 7, ly = q >> 3;
    const uint32_t i = it.i;
    const uint32_t idx = uniform(strided && i == i0 ? d0 : v.dirty[i]);
    const int32_t mynb = q < 8 ? v.nbr[(size_t)idx * 27 + nbr_dir(q & 1, (q >> 1) & 1, q >> 2)] : -1;
    // the block's own types, independent of the halo: load them now (the
    // previous applied types only for refinement)
    uint32_t old[8], prev[8];
#pragma unroll
    for (int lz = 0; lz < 8; ++lz) {
      old[lz] = v.tcur[(size_t)idx * kVox + q + 64 * lz];
      prev[lz] = refine == 1 ? v.tprev[(size_t)idx * kVox + q + 64 * lz] : 0u;
    }
    if (q < 8) snb[q] = mynb;
    wave_sync();
    // The corners' bits as rows: row (y, z) of the 9 x 9 x 9 corners holds
    // x = 0..8 in bits 0..8: whether TSDF < 0, and from bit 16 whether the
    // corner is observed; for refinement also whether |TSDF| < eps (Eq. 5).
    // They come from the eight blocks' masks (64 bytes each per block and
    // kind, kept by fusion and import): lane q requests layer q & 7 of block
    // q >> 3 (x | y << 1 | z << 2) and stages it in LDS; then lane j forms
    // row j (and j + 64), bits 0..7 from the block of its y and z, bit 8
    // from the +x one.
    {
      const int32_t nb = snb[q >> 3];
      uint64_t sn = 0, ob = 0, nz = 0;
      if (nb >= 0) {
        sn = v.smask[(size_t)nb * 8 + (q & 7)];
        ob = v.wmask[(size_t)nb * 8 + (q & 7)];
        if (refine) nz = v.nmask[(size_t)nb * 8 + (q & 7)];
      }
      smk[2 * q] = (uint32_t)sn;
      smk[2 * q + 1] = (uint32_t)(sn >> 32);
      smk[128 + 2 * q] = (uint32_t)ob;
      smk[128 + 2 * q + 1] = (uint32_t)(ob >> 32);
      smk[256 + 2 * q] = (uint32_t)nz;
      smk[256 + 2 * q + 1] = (uint32_t)(nz >> 32);
    }
    wave_sync();
    for (int j = q; j < 81; j += 64) {
      const int y = j % 9, z = j / 9;
      const int w0 = (((y >> 3) << 1 | (z >> 3) << 2) << 3) + (z & 7), w1 = w0 + 8;
      const uint32_t sh = 8u * (uint32_t)(y & 7), h = sh >> 5, b = sh & 31u;
      auto row = [&](int kind) -> uint32_t {
        const uint32_t* m = smk + 128 * kind;
        return ((m[2 * w0 + h] >> b) & 255u) | ((m[2 * w1 + h] >> b) & 1u) << 8;
      };
      srow[j] = row(0) | row(1) << 16;
      if (refine) nrow[j] = row(2);
    }
    wave_sync();
    uint32_t flags = 0, nchanged = 0, nrefined = 0;
    // triangles (bits 0..7) and triangle-carrying cubes (from bit 8) of the
    // changed cubes' new and old types
    uint32_t fnew = 0, fold = 0;
    // the lane's column of cubes shares corner faces between layers: face
    // z holds the signs of corners (x, y), (x+1, y), (x+1, y+1), (x, y+1) at
    // height z in bits 0..3 (the cyclic corner order) and, in bit 4, whether
    // all four are observed; cube z is faces z and z+1
    auto face = [&](int z) -> uint32_t {
      const uint32_t r0 = srow[ly + 9 * z] >> lx, r1 = srow[ly + 1 + 9 * z] >> lx;
      return (r0 & 3u) | ((r1 & 2u) << 1) | ((r1 & 1u) << 3) |
             ((((r0 & r1) >> 16) & 3u) == 3u ? 16u : 0u);
    };
    // the same corners' near-zero bits (refinement)
    auto near_face = [&](int z) -> uint32_t {
      const uint32_t r0 = nrow[ly + 9 * z] >> lx, r1 = nrow[ly + 1 + 9 * z] >> lx;
      return (r0 & 3u) | ((r1 & 2u) << 1) | ((r1 & 1u) << 3);
    };
    uint32_t f_lo = face(0), n_lo = refine ? near_face(0) : 0u;
#pragma unroll
    for (int lz = 0; lz < 8; ++lz) {
      const uint32_t f_hi = face(lz + 1), n_hi = refine ? near_face(lz + 1) : 0u;
      const bool valid = (f_lo & f_hi & 16u) != 0;
      const uint32_t t = valid ? (f_lo & 15u) | ((f_hi & 15u) << 4) : 0u;
      const uint32_t near8 = n_lo | n_hi << 4;
      f_lo = f_hi;
      n_lo = n_hi;
      const size_t o = (size_t)idx * kVox + q + 64 * lz;
      uint32_t nt;
      if (refine != 1) {
        v.tprev[o] = (uint8_t)old[lz];
        nt = t;
        // types 0 and 255 are at distance 4 from every regular type, so a
        // layer with no other type has nothing to refine
        if (refine == 2 && __ballot(valid && t - 1u < 254u)) {
          if (valid) nt = refined(t, old[lz], near8);
          nrefined += (uint32_t)__popcll(__ballot(nt != t));
        }
      } else {
        nt = old[lz];
        if (__ballot(valid && old[lz] - 1u < 254u) && valid) nt = refined(old[lz], prev[lz], near8);
      }
      if (nt != old[lz]) v.tcur[o] = (uint8_t)nt;
      // an unchanged cube keeps its triangles: only changed ones count
      const uint32_t tri_old = sntri[old[lz]], tri_new = sntri[nt];
      const bool tri_change = nt != old[lz] && (tri_old | tri_new) != 0u;
      if (tri_change) fnew += tri_new, fold += tri_old;
      nchanged += (uint32_t)__popcll(__ballot(tri_change));
      if (tri_change) {
        // owners of this cube's edges: this block and, on its +x/+y/+z
        // faces, the neighbours (never the +x+y+z corner one)
        const bool ex = lx == 7, ey = ly == 7, ez = lz == 7;
        flags |= 1u | (ex ? 2u : 0u) | (ey ? 4u : 0u) | (ez ? 16u : 0u) | (ex && ey ? 8u : 0u) |
                 (ex && ez ? 32u : 0u) | (ey && ez ? 64u : 0u);
      }
    }
    // wave-wide OR of the owner flags
    uint32_t wflags = refine == 1 ? 0u : 1u;
    for (int b = 0; b < 7; ++b)
      if (__ballot((flags >> b) & 1u)) wflags |= 1u << b;
    if (refine != 1) {
      // extraction: the vertex pass walks every dirty block, this one
      // included; a +x/+y/+z neighbour that owns edges of changed cubes and
      // is not dirty itself joins as an extra block, claimed once per pass
      // and appended with one atomic per wave
      bool extra = false;
      if (q >= 1 && q < 8 && ((wflags >> q) & 1u) && mynb >= 0)
        extra = v.st_dirty[mynb] != pass && v.st_vtx[mynb] != pass &&
                atomicMax(&v.st_vtx[mynb], pass) < pass;
      const uint64_t be = __ballot(extra);
      if (be) {
        uint32_t b0 = 0;
        if (q == 0) b0 = atomicAdd(&v.cnt->n_vblocks[v.vsel], (uint32_t)__popcll(be));
        const uint32_t pos = uniform(b0) + mask_rank(be);
        if (extra) {
          if (pos < v.max_blocks) v.vblocks[pos] = (uint32_t)mynb;
          else atomicOr(&v.cnt->error, kErrBlocks);
        }
      }
    } else if (q < 8) {
      uint32_t out = kNone;
      if ((wflags >> q) & 1u) {
        const int32_t nb = q == 0 ? (int32_t)idx : mynb;
        if (nb >= 0 && v.st_vtx[nb] != pass && atomicMax(&v.st_vtx[nb], pass) < pass)
          out = (uint32_t)nb;
      }
      v.vcand[(size_t)i * 8 + q] = out;
    }
    // per lane at most 40 triangles (5 in 8 cubes) and 8 cubes each
    const uint32_t cnew = wave_sum_bits<4>(fnew >> 8), cold = wave_sum_bits<4>(fold >> 8);
    fnew = wave_sum_bits<6>(fnew & 255u);
    fold = wave_sum_bits<6>(fold & 255u);
    if (q == 0 && (nchanged | nrefined)) {
      Seg& cs = v.cseg[idx % v.nseg];
      auto add2 = [](uint32_t* lo, uint32_t a, uint32_t b) {
        atomicAdd(reinterpret_cast<unsigned long long*>(lo),
                  (unsigned long long)a | (unsigned long long)b << 32);
      };
      add2(&cs.st_chg, nchanged, refine == 1 ? nchanged : nrefined);
      if (cnew | cold) add2(&cs.st_cnew, cnew, cold);
      if (fnew | fold) add2(&cs.st_fnew, fnew, fold);
    }
    wave_sync();
  }
}

// Compact the vertex-block candidates a refinement wrote (8 per dirty
// block, already claimed), one atomic per tile.
// The candidate list is 8 entries per dirty block and mostly empty, and
// can be long (every block of a large import), so each lane takes 8 entries
// (coalesced: entry k of a lane sits k * 256 past the first) and a tile of
// 2048 entries costs one atomic on the list length.
constexpr int kVbPer = 8;
__global__ __launch_bounds__(256) void k_vblock_compact(VolDev v) {
  __shared__ uint32_t swave[16];
  __shared__ uint32_t sbase;
  const uint32_t n = min(v.cnt->n_dirty[v.xsel], v.max_blocks);
  const uint32_t total = n * 8u;
  constexpr uint32_t kT = 256 * kVbPer;
  for (uint32_t t0 = blockIdx.x * kT; t0 < total; t0 += gridDim.x * kT) {
    uint32_t got[kVbPer], cnt = 0;
#pragma unroll
    for (int k = 0; k < kVbPer; ++k) {
      const uint32_t t = t0 + k * 256 + threadIdx.x;
      got[k] = t < total ? v.vcand[t] : kNone;
      cnt += got[k] != kNone;
    }
    uint32_t tot;
    uint32_t r = wg_scan_bits<count_bits(kVbPer)>(cnt, swave, &tot);
    if (tot == 0) continue;
    if (threadIdx.x == 0) sbase = atomicAdd(&v.cnt->n_vblocks[v.vsel], tot);
    __syncthreads();
    r += sbase;
#pragma unroll
    for (int k = 0; k < kVbPer; ++k)
      if (got[k] != kNone) v.vblocks[r++] = got[k];
    __syncthreads();
  }
}

// One wave per listed block.  Each voxel owns the edges from it along +x,
// +y, +z.  The reference count of an edge is the number of triangles, over
// the four cubes around it, that use it; a positive count needs a vertex
// (created here on first use, Sec. V-C), whose parameter t is rewritten
// from the end point TSDF values when either end point may have changed
// since the last extraction.  Counts are formed, never stored: the cube
// types are staged in LDS with the -x/-y/-z halo, and a per-type table of
// edge uses packed by the cube's place around the voxel (four roles, three
// 6-bit counts each, plus the counts the cube gives the voxel one layer up)
// gives a lane the three counts of a voxel from four table reads, walking
// up its column.  Which edges hold a vertex is one 24-bit word per lane
// (bit 8a + lz), read at the start and written back when it changes.  New
// vertices take slots from the block's pool segment, one atomic per block,
// and the recycled slots it takes are fetched in one batch.  The edges with
// work (a vertex to create, to free, or to move) are listed in LDS lane by
// lane, each lane's place from a prefix sum of the lanes' counts; the
// write pass runs over that list, 64 edges per step, in chunks of kWorkCap
// edges.  Each chunk first requests everything it reads, the freed
// vertices' slots and the end point TSDF values of the others, and only
// then stores: on this hardware a load issued after stores waits for them
// too.  A block with no vertex and no cube with triangles around its edges
// (one in free space) stops after the type staging.
constexpr int kRingBatch = 256;  // recycled slots fetched per block at once
constexpr int kWorkCap = 512;    // listed edges per chunk of the write pass

template <int W>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(6))) void k_vertices(VolDev v, uint32_t moved, int walk_dirty) {
  __shared__ uint32_t srole[4 * 256];  // edge uses by role, per cube type
  __shared__ uint32_t st_all[W][kRingBatch];  // cube types at local -1..7, then slots
  __shared__ uint32_t swork_all[W][kWorkCap]; // edge 64k + q | count > 0 << 11 | has vertex << 12
  __shared__ int32_t snb_all[W][27];
  static_assert(kRingBatch * 4 >= 732, "type staging fits the slot batch");
  // the blocks: after an extraction the dirty list and then the extra
  // blocks classification appended; after a refinement the compacted list
  const uint32_t nd = walk_dirty ? min(v.cnt->n_dirty[v.xsel], v.max_blocks) : 0u;
  const uint32_t n = nd + min(v.cnt->n_vblocks[v.vsel], v.max_blocks);
  if (blockIdx.x == 0 && threadIdx.x == 0) v.cnt->acc[VM_TOTAL_VERTEX_BLOCKS] += n;
  {
    // a workgroup whose first wave has no block has none at all
    const ItemLoop first = item_loop(v, n, W, 0);
    if (first.i >= first.end) return;
  }
  for (int j = threadIdx.x; j < 4 * 256; j += blockDim.x) srole[j] = v.edge_roles[j];
  __syncthreads();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint8_t* st = reinterpret_cast<uint8_t*>(st_all[wave]);
  uint32_t* sring = st_all[wave];
  uint32_t* swork = swork_all[wave];
  int32_t* snb = snb_all[wave];
  for (ItemLoop it = item_loop(v, n, W, wave); it.i < it.end; it.i += it.step) {
    // lane addressing is formed again per block rather than held in
    // registers across the loop
    const int q = fresh_lane(), lx = q & 7, ly = q >> 3;
    const uint32_t idx = uniform(it.i < nd ? v.dirty[it.i] : v.vblocks[it.i - nd]);
    const uint32_t sg = uniform(idx % v.nseg);
    // the block's edge arrays, addressed by block-local edge a * 512 + l;
    // pool arrays by 32-bit byte offsets from their bases (every index here
    // is below 2^30 entries of 4 bytes)
    const size_t eb = (size_t)idx * (3 * kVox);
    int32_t* evtx_b = v.evtx + eb;
    float* et_b = v.et + eb;
    auto pool32 = [](uint32_t* base, uint32_t s) -> uint32_t& {
      return *reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(base) + s * 4u);
    };
    // requested at once: the neighbour table, which edges hold a vertex,
    // the block's cube types and its pool segment (fixed during this kernel)
    const int32_t mynb = q < 27 ? v.nbr[(size_t)idx * 27 + q] : -1;
    const uint32_t has = v.emask[(size_t)idx * 64 + q];
    uint32_t tv[8];
#pragma unroll
    for (int lz = 0; lz < 8; ++lz) tv[lz] = v.tcur[(size_t)idx * kVox + q + 64 * lz];
    const Seg& g = v.vseg[sg];
    const uint32_t head = g.head, count = g.count, hwm = g.hwm;
    if (q < 27) snb[q] = mynb;
    wave_sync();
    // the -x/-y/-z halo of types (217 cells): the three faces, one cell per
    // lane each, then the three edges and the corner (lanes 0..24); and,
    // after an extraction of pending blocks, which of this block and its
    // +x/+y/+z neighbours were pending
    const uint8_t* tcur = v.tcur;
    const int32_t bnx = snb[nbr_dir(-1, 0, 0)], bny = snb[nbr_dir(0, -1, 0)],
                  bnz = snb[nbr_dir(0, 0, -1)];
    const uint32_t hx = bnx >= 0 ? tcur[(uint32_t)bnx * 512u + 7u + 8u * (uint32_t)q] : 0u;
    const uint32_t hy = bny >= 0 ? tcur[(uint32_t)bny * 512u + 56u + (uint32_t)(lx + 64 * ly)] : 0u;
    const uint32_t hz = bnz >= 0 ? tcur[(uint32_t)bnz * 512u + 448u + (uint32_t)q] : 0u;
    uint32_t he = 0;
    int hcell = -1;
    {
      int dir = -1;
      uint32_t off = 0;
      if (q < 8) dir = nbr_dir(-1, -1, 0), off = 63u + 64u * (uint32_t)q, hcell = 81 * (q + 1);
      else if (q < 16) dir = nbr_dir(-1, 0, -1), off = 7u + 8u * (uint32_t)(q - 8) + 448u, hcell = 9 * (q - 7);
      else if (q < 24) dir = nbr_dir(0, -1, -1), off = (uint32_t)(q - 16) + 504u, hcell = q - 15;
      else if (q == 24) dir = nbr_dir(-1, -1, -1), off = 511u, hcell = 0;
      const int32_t nb = dir >= 0 ? snb[dir] : -1;
      if (nb >= 0) he = tcur[(uint32_t)nb * 512u + off];
    }
    uint32_t mv = 0xFFFFFFu;  // edges whose end points may have moved (bit 8a + lz)
    if (moved != kMovedAll) {
      const bool pend = q < 27 && mynb >= 0 && v.st_pending[mynb] == moved;
      const uint64_t pm = __ballot(pend);
      if (!((pm >> kSelf) & 1u)) {
        mv = (lx == 7 && ((pm >> nbr_dir(1, 0, 0)) & 1u) ? 0xFFu : 0u) |
             (ly == 7 && ((pm >> nbr_dir(0, 1, 0)) & 1u) ? 0xFF00u : 0u) |
             (((pm >> nbr_dir(0, 0, 1)) & 1u) ? 0x800000u : 0u);
      }
    }
    // types into LDS (local -1..7 per axis); whether a staged cube has
    // triangles (a type other than 0 and 255)
    uint32_t surf = 0;
#pragma unroll
    for (int lz = 0; lz < 8; ++lz) {
      st[(lx + 1) + 9 * (ly + 1) + 81 * (lz + 1)] = (uint8_t)tv[lz];
      surf |= (uint32_t)(tv[lz] - 1u < 254u);
    }
    st[9 * (lx + 1) + 81 * (ly + 1)] = (uint8_t)hx;      // (-1, y, z), y = q & 7
    st[(lx + 1) + 81 * (ly + 1)] = (uint8_t)hy;          // (x, -1, z)
    st[(lx + 1) + 9 * (ly + 1)] = (uint8_t)hz;           // (x, y, -1)
    if (hcell >= 0) st[hcell] = (uint8_t)he;
    surf |= (uint32_t)(hx - 1u < 254u) | (uint32_t)(hy - 1u < 254u) | (uint32_t)(hz - 1u < 254u) |
            (uint32_t)(he - 1u < 254u);
    // no cube around the block's edges has triangles and no edge holds a
    // vertex: every count stays zero and there is nothing to write (about a
    // third of the blocks of a frame of the room sequence lie in free space)
    if (__ballot(has != 0u || surf != 0u) == 0ull) {
      wave_sync();
      continue;
    }
    wave_sync();
    // counts, layer by layer up the lane's column.  A table entry holds,
    // for a cube in its role, the uses of the x, y, z edges of the voxel in
    // bits 0, 6, 12 and, from bit 18, those of the x and y edges of the
    // voxel one layer up; no 6-bit field can overflow (at most 4 x 7).
    const int cb = (lx + 1) + 9 * (ly + 1);
    auto cell_sum = [&](int b) -> uint32_t {
      return srole[st[b]] + srole[256 + st[b - 9]] + srole[512 + st[b - 1]] +
             srole[768 + st[b - 10]];
    };
    uint32_t carry = cell_sum(cb) >> 18;  // the layer below the block
    uint32_t R = 0;  // edges with a positive count, bit 8a + lz
#pragma unroll
    for (int lz = 0; lz < 8; ++lz) {
      const uint32_t sum = cell_sum(cb + 81 * (lz + 1));
      const uint32_t r = (sum & 0x3FFFFu) + carry;
      carry = sum >> 18;
      // bit 5 of each field of r + 31 is set iff the count is nonzero;
      // times 0x15 places the three bits at 5, 13 and 21 (no carries)
      const uint32_t nz = ((r + 0x1F7DFu) & 0x20820u) * 0x15u & 0x202020u;
      R |= lz <= 5 ? nz >> (5 - lz) : nz << (lz - 5);
    }
    const uint32_t need = R & ~has, freed = has & ~R, kept = R & has;
    const uint32_t work = need | freed | (kept & mv);
    // one allocation and one recycling atomic per block, issued together;
    // a vertex whose count dropped to zero goes back to the segment's ring
    // at once (Sec. V-E), where it can be taken again once the ring is
    // closed, never by this pass
    // per lane at most 24 of each (its three edges in eight layers)
    const uint32_t total = wave_sum_bits<5>((uint32_t)__popc(need));
    const uint32_t tfree = wave_sum_bits<5>((uint32_t)__popc(freed));
    uint32_t nwork;
    const uint32_t wpos = wave_prefix_bits<5>((uint32_t)__popc(work), &nwork);
    uint32_t base = 0, fbase = 0;
    if (q == 0) {
      if (total) base = atomicAdd(&v.vseg[sg].ticket, total);
      if (tfree) fbase = atomicAdd(&v.vseg[sg].push, tfree);
    }
    base = uniform(base);
    fbase = uniform(fbase);
    const uint32_t gbase = sg * v.vseg_cap, gsize = seg_size(sg, v.vseg_cap, v.max_vertices);
    const uint32_t rtail = ring_pos(head, count, gsize);  // where pushes start
    // the slots of the first kRingBatch allocations, fetched together (the
    // type staging is no longer needed: the batch reuses its LDS)
    wave_sync();
    const uint32_t batch = min(total, (uint32_t)kRingBatch);
    for (uint32_t k = q; k < batch; k += 64)
      sring[k] = seg_slot(head, count, hwm, base + k, v.vring, gbase, gsize);
    // slot of allocation k of this block (k counted from 0)
    auto new_slot = [&](uint32_t k) -> uint32_t {
      return k < batch ? sring[k] : seg_slot(head, count, hwm, base + k, v.vring, gbase, gsize);
    };
    // the edge's vertex is no longer used: back to the ring (k-th free of
    // this block).  A slot of -1 (the edge's allocation had failed) goes in
    // as kNone, which whoever takes it reports as a full segment.
    auto free_vertex = [&](int32_t s, uint32_t k) {
      pool32(v.vring, gbase + ring_pos(rtail, fbase + k, gsize)) = (uint32_t)s;
      if (s >= 0) pool32(v.vowner, (uint32_t)s) = kNone;
    };
    uint32_t nnew = 0, nmov = 0, knew = 0, kfree = 0;
    // the blocks with the longest write pass finish last and so set the
    // kernel's end: their waves take issue priority over the others on the
    // SIMD until their writes are done
    if (nwork > 128u) __builtin_amdgcn_s_setprio(2);
    for (uint32_t c0 = 0; c0 < nwork; c0 += kWorkCap) {
      // the lane's items of this chunk, at its place in the list
      wave_sync();
      {
        uint32_t p = wpos - c0, rem = work;
        while (rem) {
          const uint32_t k = (uint32_t)__builtin_ctz(rem);
          rem &= rem - 1u;
          if (p < (uint32_t)kWorkCap)
            swork[p] = (k << 6 | (uint32_t)q) | ((R >> k) & 1u) << 11 | ((has >> k) & 1u) << 12;
          ++p;
        }
      }
      wave_sync();
      const uint32_t m = min(nwork - c0, (uint32_t)kWorkCap);
      // the chunk's loads: per item of the lane, the slot of the vertex it
      // frees, or the TSDF at its edge's two end points (the far one in the
      // +axis neighbour when the owner sits on the block's +axis face)
      constexpr int kSteps = kWorkCap / 64;
      int32_t fslot[kSteps];
      float da[kSteps], db[kSteps];
#pragma unroll
      for (int k = 0; k < kSteps; ++k) {
        fslot[k] = -1;
        da[k] = 0.f;
        db[k] = 0.f;
        const uint32_t i = (uint32_t)(64 * k + q);
        if (i < m) {
          const uint32_t item = swork[i];
          const uint32_t e = item & 2047u;
          if (!((item >> 11) & 1u)) {
            fslot[k] = evtx_b[e];
          } else {
            const uint32_t a = e >> 9, l = e & 511u;
            const uint32_t c = a == 0 ? (l & 7u) : (a == 1 ? ((l >> 3) & 7u) : (l >> 6));
            const uint32_t stp = a == 0 ? 1u : (a == 1 ? 8u : 64u);
            int32_t fb = (int32_t)idx;
            uint32_t fl = l + stp;
            if (c == 7u) {
              fb = snb[nbr_dir(a == 0, a == 1, a == 2)];
              fl = l - 7u * stp;
            }
            da[k] = v.d[(size_t)idx * kVox + l];
            db[k] = fb >= 0 ? v.d[(size_t)fb * kVox + fl] : 0.f;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < kSteps; ++k) {
        const uint32_t i0 = 64u * (uint32_t)k;
        if (i0 >= m) break;
        const bool act = i0 + q < m;
        const uint32_t item = act ? swork[i0 + q] : 0u;
        const uint32_t e = item & 2047u;
        const bool cnt = (item >> 11) & 1u, hv = (item >> 12) & 1u;
        const bool is_new = act && cnt && !hv, is_free = act && !cnt;
        const uint64_t bn = __ballot(is_new), bf = __ballot(is_free);
        const uint32_t myk = mask_rank(bn, knew), myf = mask_rank(bf, kfree);
        knew += (uint32_t)__popcll(bn);
        kfree += (uint32_t)__popcll(bf);
        if (!act) continue;
        if (cnt) {
          if (!hv) {
            const uint32_t ns = new_slot(myk);
            if (ns == kNone) {
              // pool exhausted: the edge stays without a vertex, and its
              // triangles will reference none
              atomicOr(&v.cnt->error, kErrVertices);
              evtx_b[e] = -1;
              continue;
            }
            evtx_b[e] = (int32_t)ns;
            pool32(v.vowner, ns) = (uint32_t)eb + e;
            pool32(v.vbirth, ns) = v.frame;
            ++nnew;
          } else {
            ++nmov;
          }
          et_b[e] = edge_param(da[k], db[k]);
        } else {
          free_vertex(fslot[k], myf);
        }
      }
    }
    __builtin_amdgcn_s_setprio(0);
    if (R != has) v.emask[(size_t)idx * 64 + q] = R;
    nnew = wave_sum_bits<5>(nnew);
    nmov = wave_sum_bits<5>(nmov);
    const uint32_t nupd = wave_sum_bits<5>((uint32_t)__popc(kept));
    if (q == 0) {
      if (nnew | nupd)
        atomicAdd(reinterpret_cast<unsigned long long*>(&v.vseg[sg].st_new),
                  (unsigned long long)nnew | (unsigned long long)nupd << 32);
      if (nmov | tfree)
        atomicAdd(reinterpret_cast<unsigned long long*>(&v.vseg[sg].st_mov),
                  (unsigned long long)nmov | (unsigned long long)tfree << 32);
    }
    wave_sync();
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

// ============================================================================
// ablation: the paper's two ways of sharing vertices between cubes
// ============================================================================
// Sec. V-C gives two GPU schemes that initialise each vertex once while the
// cubes around its edge run in parallel, and Sec. VI-A times them against
// each other.  These kernels reproduce both, for measurement beside edge
// ownership, on the cubes of the last extraction's dirty blocks, one lane
// per cube: for every edge its type uses, a vertex is allocated (one atomic
// on a global counter, as from a heap) if the edge has none, and the edge
// parameter t is written.  The state is the caller's: slot[e] (-1: none) and
// t[e], e = (block * 3 + axis) * 512 + voxel, kept across calls.

// Index of the owner edge of cube-edge e of cube l in block idx, -1 when the
// owner block is not allocated; t receives its parameter.
__device__ inline int64_t cube_edge_slot_index(const VolDev& v, uint32_t idx, int l, int e,
                                               float& t) {
  int ox, oy, oz, axis;
  edge_owner(e, ox, oy, oz, axis);
  const int x = (l & 7) + ox, y = ((l >> 3) & 7) + oy, z = (l >> 6) + oz;
  const int32_t nb = v.nbr[(size_t)idx * 27 + nbr_dir(x >> 3, y >> 3, z >> 3)];
  const int fx = x + (axis == 0), fy = y + (axis == 1), fz = z + (axis == 2);
  const int32_t fb = v.nbr[(size_t)idx * 27 + nbr_dir(fx >> 3, fy >> 3, fz >> 3)];
  if (nb < 0 || fb < 0) return -1;
  const int ol = (x & 7) + 8 * (y & 7) + 64 * (z & 7);
  t = edge_param(v.d[(size_t)nb * kVox + ol],
                 v.d[(size_t)fb * kVox + (fx & 7) + 8 * (fy & 7) + 64 * (fz & 7)]);
  return ((int64_t)nb * 3 + axis) * kVox + ol;
}

// Lock-based: the first lane to take an edge (compare-and-swap from -1)
// allocates its vertex; every lane using the edge writes the same t.
__global__ __launch_bounds__(256) void k_share_lock(VolDev v, int32_t* __restrict__ slot,
                                                    float* __restrict__ tv,
                                                    uint32_t* __restrict__ counter) {
  const uint32_t n = min(v.cnt->n_dirty[v.xsel], v.max_blocks) * kVox;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t idx = v.dirty[i / kVox];
    const int l = (int)(i % kVox);
    const uint32_t type = v.tcur[(size_t)idx * kVox + l];
    if (v.tri_table[type * 16] == 0) continue;
    for (int e = 0; e < 12; ++e) {
      if (!v.edge_uses[type * 12 + e]) continue;
      float t;
      const int64_t eo = cube_edge_slot_index(v, idx, l, e, t);
      if (eo < 0) continue;
      if (atomicCAS(&slot[eo], -1, -2) == -1) slot[eo] = (int32_t)atomicAdd(counter, 1u);
      tv[eo] = t;
    }
  }
}

// Lock-free: the cubes of each 2x2x2 cell form four groups of two at
// opposite corners (parities 000/111, 100/011, 010/101, 001/110); no two
// cubes of a group share an edge, so within one launch a lane allocates
// without any claim.  The four groups are four launches.
__global__ __launch_bounds__(256) void k_share_free(VolDev v, int group,
                                                    int32_t* __restrict__ slot,
                                                    float* __restrict__ tv,
                                                    uint32_t* __restrict__ counter) {
  const uint32_t n = min(v.cnt->n_dirty[v.xsel], v.max_blocks) * 128u;
  const int first = group == 0 ? 0 : (1 << (group - 1));  // parity x | y << 1 | z << 2
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t idx = v.dirty[i / 128u];
    const int k = (int)(i % 128u), cell = k & 63;
    const int p = (k >> 6) ? first ^ 7 : first;
    const int x = 2 * (cell & 3) + (p & 1), y = 2 * ((cell >> 2) & 3) + ((p >> 1) & 1),
              z = 2 * (cell >> 4) + (p >> 2);
    const int l = x + 8 * y + 64 * z;
    const uint32_t type = v.tcur[(size_t)idx * kVox + l];
    if (v.tri_table[type * 16] == 0) continue;
    for (int e = 0; e < 12; ++e) {
      if (!v.edge_uses[type * 12 + e]) continue;
      float t;
      const int64_t eo = cube_edge_slot_index(v, idx, l, e, t);
      if (eo < 0) continue;
      if (slot[eo] < 0) slot[eo] = (int32_t)atomicAdd(counter, 1u);
      tv[eo] = t;
    }
  }
}

// ============================================================================
// download: two-level exclusive scans over the vertex and triangle pools
// ============================================================================
constexpr int kScanItems = 1024;  // items per workgroup (256 lanes x 4)

__device__ inline bool slot_in_use(const Seg* seg, uint32_t cap, uint32_t i) {
  const uint32_t s = i / cap;
  return i - s * cap < seg[s].hwm;
}

__device__ inline uint32_t item_count(const VolDev& v, int what, uint32_t i) {
  if (what == 0) {
    if (i >= v.max_vertices || !slot_in_use(v.vseg, v.vseg_cap, i)) return 0;
    return v.vowner[i] != kNone ? 1u : 0u;
  }
  // cube i of the block pool: its type's triangles
  if (i / kVox >= min(v.cnt->n_blocks, v.max_blocks)) return 0;
  return v.tri_table[(uint32_t)v.tcur[i] * 16];
}

// Position in metres of the vertex in pool entry i, in the frame of its
// volume (the slot's own frame in a batch): owner voxel g, plus t along the
// edge's axis.  Returns the slot; *key receives the edge key when non-NULL.
__device__ inline int vertex_position(const VolDev& v, uint32_t i, float p[3], uint64_t* key) {
  const uint32_t owner = v.vowner[i];
  const uint32_t blk = owner / (3 * kVox), rem = owner % (3 * kVox);
  const int axis = (int)(rem / kVox), local = (int)(rem % kVox);
  const uint64_t bkey = v.block_key[blk];
  int bx, by, bz, slot;
  unpack_key(bkey, bx, by, bz);
  block_frame(v, bx, slot);
  const int g[3] = {8 * bx + (local & 7), 8 * by + ((local >> 3) & 7), 8 * bz + (local >> 6)};
  const float t = v.et[owner];
  for (int a = 0; a < 3; ++a) {
    float c = (float)g[a];
    if (a == axis) c = c + t;
    p[a] = c * v.s;
  }
  if (key) *key = edge_key(bkey, local, axis);
  return slot;
}

__global__ __launch_bounds__(256) void k_dl_count(VolDev v, int what) {
  __shared__ uint32_t swave[16];
  const uint32_t i0 = blockIdx.x * kScanItems + threadIdx.x * 4;
  uint32_t c = 0;
  for (int k = 0; k < 4; ++k) c += item_count(v, what, i0 + k);
  uint32_t total;
  wg_scan(c, swave, &total);
  if (threadIdx.x == 0) v.scan[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_dl_scan(VolDev v, int what, uint32_t nparts) {
  __shared__ uint32_t swave[16];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t base = 0; base < nparts; base += 1024) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t x = i < nparts ? v.scan[i] : 0u;
    uint32_t all;
    const uint32_t before = wg_scan(x, swave, &all);
    if (i < nparts) v.scan[i] = carry + before;
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
  __shared__ uint32_t swave[16];
  const uint32_t i0 = blockIdx.x * kScanItems + threadIdx.x * 4;
  uint32_t live[4], c = 0;
  for (int k = 0; k < 4; ++k) c += (live[k] = item_count(v, 0, i0 + k));
  uint32_t total;
  uint32_t j = v.scan[blockIdx.x] + wg_scan(c, swave, &total);
  for (int k = 0; k < 4; ++k) {
    const uint32_t i = i0 + k;
    if (i >= v.max_vertices) break;
    if (!live[k]) {
      v.vdl[i] = -1;
      continue;
    }
    v.vdl[i] = (int32_t)j;
    if (j < vcap) {
      float p[3];
      uint64_t key;
      vertex_position(v, i, p, &key);
      for (int a = 0; a < 3; ++a) verts[3 * (size_t)j + a] = p[a];
      if (keys) keys[j] = key;
    }
    ++j;
  }
}

// Every vertex pool entry's position (0 and slot -1 for entries without a
// live vertex): no compaction, so no host round trip.
__global__ __launch_bounds__(256) void k_positions(VolDev v, float* __restrict__ pos,
                                                   int32_t* __restrict__ slot_of) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < v.max_vertices;
       i += gridDim.x * blockDim.x) {
    float p[3] = {0.f, 0.f, 0.f};
    int slot = -1;
    if (item_count(v, 0, i)) slot = vertex_position(v, i, p, nullptr);
    pos[3 * (size_t)i] = p[0];
    pos[3 * (size_t)i + 1] = p[1];
    pos[3 * (size_t)i + 2] = p[2];
    if (slot_of) slot_of[i] = slot;
  }
}

// Triangles of every cube, in pool order: the cube's type lists its
// triangles as cube edges, each edge is resolved to the vertex its owner
// voxel holds (the owner block through the cube's neighbour table), and the
// vertex to its row in this download.
__global__ __launch_bounds__(256) void k_dl_write_triangles(VolDev v, int32_t* __restrict__ tris,
                                                            uint32_t tcap) {
  __shared__ uint32_t swave[16];
  const uint32_t i0 = blockIdx.x * kScanItems + threadIdx.x * 4;
  uint32_t c = 0;
  for (int k = 0; k < 4; ++k) c += item_count(v, 1, i0 + k);
  uint32_t total;
  uint32_t j = v.scan[blockIdx.x] + wg_scan(c, swave, &total);
  for (int k = 0; k < 4; ++k) {
    const uint32_t i = i0 + k;
    const uint32_t ntri = item_count(v, 1, i);
    if (ntri == 0) continue;
    const uint32_t idx = i / kVox, l = i % kVox, type = v.tcur[i];
    const uint8_t* edges = v.tri_table + type * 16 + 1;
    for (uint32_t t = 0; t < ntri; ++t, ++j) {
      if (j >= tcap) continue;
      for (int q = 0; q < 3; ++q) {
        int ox, oy, oz, axis;
        edge_owner(edges[3 * t + q], ox, oy, oz, axis);
        const int x = (int)(l & 7u) + ox, y = (int)((l >> 3) & 7u) + oy, z = (int)(l >> 6) + oz;
        const int32_t nb = v.nbr[(size_t)idx * 27 + nbr_dir(x >> 3, y >> 3, z >> 3)];
        int32_t s = -1;
        if (nb >= 0)
          s = v.evtx[((size_t)nb * 3 + axis) * kVox + (x & 7) + 8 * (y & 7) + 64 * (z & 7)];
        tris[3 * (size_t)j + q] = s < 0 ? -1 : v.vdl[s];
      }
    }
  }
}

// TSDF at voxel (x, y, z) local to block idx, coordinates in [-1, 9]; false
// when the voxel is not observed (block not allocated, or weight 0).
__device__ inline bool observed_tsdf(const VolDev& v, uint32_t idx, int x, int y, int z,
                                     float& d) {
  const int32_t nb = v.nbr[(size_t)idx * 27 + nbr_dir(x >> 3, y >> 3, z >> 3)];
  if (nb < 0) return false;
  const size_t o = (size_t)nb * kVox + (x & 7) + 8 * (y & 7) + 64 * (z & 7);
  d = v.d[o];
  return v.w[o] > 0.f;
}

// TSDF gradient at a voxel: per axis the central difference over its two
// neighbours, one-sided when only one is observed, 0 when neither is.
__device__ inline void tsdf_gradient(const VolDev& v, uint32_t idx, int x, int y, int z,
                                     float g[3]) {
  float d0 = 0.f;
  observed_tsdf(v, idx, x, y, z, d0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int ex = i == 0, ey = i == 1, ez = i == 2;
    float dp = 0.f, dm = 0.f;
    const bool hp = observed_tsdf(v, idx, x + ex, y + ey, z + ez, dp);
    const bool hm = observed_tsdf(v, idx, x - ex, y - ey, z - ez, dm);
    g[i] = hp && hm ? (dp - dm) * 0.5f : (hp ? dp - d0 : (hm ? d0 - dm : 0.f));
  }
}

// Unit normals of the vertices of the last download, in its row order (the
// paper keeps a normal in every vertex, Sec. IV): the TSDF gradient at the
// edge's two end points, interpolated at t and normalised, (0, 0, 0) when it
// vanishes; it points to increasing TSDF.  One lane per pool slot.
__global__ __launch_bounds__(256) void k_dl_normals(VolDev v, float* __restrict__ normals) {
  const uint32_t nv = v.cnt->dl_nv;
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < v.max_vertices;
       s += gridDim.x * blockDim.x) {
    if (!item_count(v, 0, s)) continue;
    const int32_t row = v.vdl[s];
    if (row < 0 || (uint32_t)row >= nv) continue;
    const uint32_t eo = v.vowner[s];
    const uint32_t idx = eo / (3 * kVox), a = (eo / kVox) % 3, l = eo % kVox;
    const int x = (int)(l & 7u), y = (int)((l >> 3) & 7u), z = (int)(l >> 6);
    const float t = v.et[eo];
    float g0[3], g1[3], n[3];
    tsdf_gradient(v, idx, x, y, z, g0);
    tsdf_gradient(v, idx, x + (a == 0), y + (a == 1), z + (a == 2), g1);
#pragma unroll
    for (int j = 0; j < 3; ++j) n[j] = (1.f - t) * g0[j] + t * g1[j];
    const float len = sqrtf(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
#pragma unroll
    for (int j = 0; j < 3; ++j) normals[3 * (size_t)row + j] = len > 0.f ? n[j] / len : 0.f;
  }
}

// Birth frames of the vertices of the last download, in its row order: the
// frame (integration or import count) of the pass in which the vertex's
// count last became positive.
__global__ __launch_bounds__(256) void k_dl_births(VolDev v, uint32_t* __restrict__ births) {
  const uint32_t nv = v.cnt->dl_nv;
  for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < v.max_vertices;
       s += gridDim.x * blockDim.x) {
    if (!item_count(v, 0, s)) continue;
    const int32_t row = v.vdl[s];
    if (row >= 0 && (uint32_t)row < nv) births[row] = v.vbirth[s];
  }
}

// ============================================================================
// backward passes
// ============================================================================

// dL/d(TSDF) of every voxel of the listed blocks, one wave per block and
// eight voxels per lane.  A voxel's gradient sums, in a fixed order, the
// contributions of the at most six edges incident to it: per axis its own
// edge (the voxel is the first end point), then the edge owned by the voxel
// one step back (the voxel is the second); each contribution is the vertex
// gradient along the axis times s times dt/dd.  Only edges that carry a
// vertex contribute, about one in a hundred: which edges hold a vertex
// comes from the block's edge masks (one word per lane), its neighbours'
// lanes and the three back faces' words, the (voxel, edge) pairs with a
// vertex are listed, and slots, end-point TSDF values and upstream
// gradients are fetched for the listed pairs alone.  The list is worked
// through layer by layer when it would overflow (dense sign fields).
constexpr int kGradCap = 384;  // listed pairs per step; one layer has at most 6 * 64

template <int W>
__global__ __launch_bounds__(64 * W) void k_bwd_tsdf(VolDev v, const float* __restrict__ dL_dv,
                                                     int by_slot, const int32_t* __restrict__ rows,
                                                     uint32_t n_rows, float* __restrict__ out) {
  __shared__ uint16_t slist_all[W][kGradCap];  // lane | lz << 6 | k << 9 (k = 2a + back)
  __shared__ float sc_all[W][kGradCap];        // contribution of each listed pair
  __shared__ uint8_t sf_all[W][kGradCap];      // whether it contributes
  __shared__ int32_t snb_all[W][27];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint16_t* slist = slist_all[wave];
  float* sc = sc_all[wave];
  uint8_t* sf = sf_all[wave];
  int32_t* snb = snb_all[wave];
  const uint32_t nb_all = min(v.cnt->n_blocks, v.max_blocks);
  const uint32_t n = rows ? n_rows : nb_all;
  const uint32_t nv = v.cnt->dl_nv;
  const uint64_t below = lanes_below();
  for (ItemLoop it = item_loop(v, n, W, wave); it.i < it.end; it.i += it.step) {
    const int q = fresh_lane(), lx = q & 7, ly = q >> 3;
    const int32_t idx = rows ? (int32_t)uniform((uint32_t)rows[it.i]) : (int32_t)it.i;
    float* o = out + (size_t)it.i * kVox;
    if (idx < 0 || (uint32_t)idx >= nb_all) {
#pragma unroll
      for (int lz = 0; lz < 8; ++lz) o[q + 64 * lz] = 0.f;
      continue;
    }
    // the block's edge masks (lane q: the edges of its column, bit 8a +
    // lz) and its neighbours; an edge ending at a voxel from behind is
    // owned by the voxel one step back: the lane at x - 1 (y - 1) of this
    // block or, on the block's back face, the -x (-y) neighbour's lane at
    // x = 7 (y = 7); along z, the layer below or the -z neighbour's top
    const int32_t mynb = q < 27 ? v.nbr[(size_t)idx * 27 + q] : -1;
    const uint32_t hm = v.emask[(size_t)idx * 64 + q];
    if (q < 27) snb[q] = mynb;
    wave_sync();
    const int32_t bnx = snb[nbr_dir(-1, 0, 0)], bny = snb[nbr_dir(0, -1, 0)],
                  bnz = snb[nbr_dir(0, 0, -1)];
    const uint32_t fx = bnx >= 0 ? v.emask[(size_t)bnx * 64 + (q | 7)] : 0u;
    const uint32_t fy = bny >= 0 ? v.emask[(size_t)bny * 64 + (q | 56)] : 0u;
    const uint32_t fz = bnz >= 0 ? v.emask[(size_t)bnz * 64 + q] : 0u;
    const uint32_t hx = __shfl(hm, (q - 1) & 63), hy = __shfl(hm, (q - 8) & 63);
    const uint32_t bxm = lx > 0 ? hx : fx, bym = ly > 0 ? hy : fy;
    // which incident edges of the lane's eight voxels carry a vertex
    uint64_t act = 0;  // bit 6 * lz + k
#pragma unroll
    for (int lz = 0; lz < 8; ++lz) {
      const uint32_t b2 = lz > 0 ? (hm >> (15 + lz)) & 1u : (fz >> 23) & 1u;
      const uint64_t m = (uint64_t)((hm >> lz) & 1u) | (uint64_t)((bxm >> lz) & 1u) << 1 |
                         (uint64_t)((hm >> (8 + lz)) & 1u) << 2 |
                         (uint64_t)((bym >> (8 + lz)) & 1u) << 3 |
                         (uint64_t)((hm >> (16 + lz)) & 1u) << 4 | (uint64_t)b2 << 5;
      act |= m << (6 * lz);
    }
    if (__ballot(act != 0ull) == 0ull) {
      // no incident edge of the block carries a vertex
#pragma unroll
      for (int lz = 0; lz < 8; ++lz) o[q + 64 * lz] = 0.f;
      continue;
    }
    uint32_t cnt = 0;
    int lz0 = 0;
    // contributions of the listed pairs, then the sums of layers [lz0, lz1)
    auto flush = [&](int lz1) {
      wave_sync();
      for (uint32_t i0 = 0; i0 < cnt; i0 += 64) {
        const uint32_t i = i0 + q;
        if (i >= cnt) continue;
        const uint32_t e = slist[i];
        const int p = (int)(e & 63u), pz = (int)((e >> 6) & 7u), k = (int)(e >> 9);
        const int a = k >> 1, back = k & 1;
        const int pc = a == 0 ? (p & 7) : (a == 1 ? (p >> 3) : pz);
        const int lstep = a == 0 ? 1 : (a == 1 ? 8 : 64);
        const int l = p + 64 * pz;
        // owner voxel (block ob, local ol) and far end point (fb, fl)
        int32_t ob = idx, fb = idx;
        int ol = l, fl = l;
        if (!back) {
          if (pc < 7) fl = l + lstep;
          else fb = snb[nbr_dir(a == 0, a == 1, a == 2)], fl = l - 7 * lstep;
        } else {
          if (pc > 0) ol = l - lstep;
          else ob = snb[nbr_dir(-(a == 0), -(a == 1), -(a == 2))], ol = l + 7 * lstep;
        }
        bool ok = false;
        float cval = 0.f;
        if (ob >= 0 && fb >= 0) {
          const int32_t s = v.evtx[((size_t)ob * 3 + a) * kVox + ol];
          const float da = v.d[(size_t)ob * kVox + ol], db = v.d[(size_t)fb * kVox + fl];
          int32_t r = -1;
          if (s >= 0) {
            if (by_slot) {
              r = s;
            } else {
              r = v.vdl[s];
              if (!(r >= 0 && (uint32_t)r < nv)) r = -1;
            }
          }
          if (r >= 0 && da != db) {
            const float g = dL_dv[3 * (size_t)r + a] * v.s;
            const float den = (da - db) * (da - db);
            cval = back ? g * (da / den) : g * (-db / den);
            ok = true;
          }
        }
        sc[i] = cval;
        sf[i] = ok;
      }
      wave_sync();
      uint32_t pos = 0;  // the list order, replayed
      for (int lz = lz0; lz < lz1; ++lz) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const bool on = (act >> (6 * lz + k)) & 1u;
          const uint64_t b = __ballot(on);
          if (on) {
            const uint32_t i = pos + (uint32_t)__popcll(b & below);
            if (sf[i]) acc = acc + sc[i];
          }
          pos += (uint32_t)__popcll(b);
        }
        o[q + 64 * lz] = acc;
      }
      wave_sync();
    };
    for (int lz = 0; lz < 8; ++lz) {
      uint64_t bk[6];
      uint32_t lc = 0;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        bk[k] = __ballot((act >> (6 * lz + k)) & 1u);
        lc += (uint32_t)__popcll(bk[k]);
      }
      if (cnt + lc > (uint32_t)kGradCap) {
        flush(lz);
        cnt = 0;
        lz0 = lz;
      }
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        if ((bk[k] >> q) & 1u)
          slist[cnt + (uint32_t)__popcll(bk[k] & below)] = (uint16_t)(q | lz << 6 | k << 9);
        cnt += (uint32_t)__popcll(bk[k]);
      }
    }
    flush(8);
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
  for (ItemLoop it = item_loop(v, n, 1, 0); it.i < it.end; it.i += it.step) {
    const uint32_t idx = it.i;
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

__global__ void k_fill_u32(uint32_t* p, uint32_t value, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_zero_f32(float* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

// ============================================================================
// inspection
// ============================================================================
// Reference count of edge (axis a, voxel l) of block blk, formed from the
// applied types of the four cubes around it (in this block or its -x/-y/-z
// neighbours; a missing block's cubes have no type).
__device__ inline int32_t edge_count(const VolDev& v, uint32_t blk, int a, int l) {
  // per axis, the four cubes as offsets from the voxel and the cube edge
  // that is this edge in each: x (0,0,0) e0, (0,-1,0) e2, (0,0,-1) e4,
  // (0,-1,-1) e6; y (0,0,0) e3, (-1,0,0) e1, (0,0,-1) e7, (-1,0,-1) e5;
  // z (0,0,0) e8, (-1,0,0) e9, (-1,-1,0) e10, (0,-1,0) e11
  const int8_t off[3][4][4] = {{{0, 0, 0, 0}, {0, -1, 0, 2}, {0, 0, -1, 4}, {0, -1, -1, 6}},
                               {{0, 0, 0, 3}, {-1, 0, 0, 1}, {0, 0, -1, 7}, {-1, 0, -1, 5}},
                               {{0, 0, 0, 8}, {-1, 0, 0, 9}, {-1, -1, 0, 10}, {0, -1, 0, 11}}};
  const int x = l & 7, y = (l >> 3) & 7, z = l >> 6;
  int32_t c = 0;
  for (int j = 0; j < 4; ++j) {
    const int cx = x + off[a][j][0], cy = y + off[a][j][1], cz = z + off[a][j][2];
    const int32_t b = v.nbr[(size_t)blk * 27 + nbr_dir(cx < 0 ? -1 : 0, cy < 0 ? -1 : 0, cz < 0 ? -1 : 0)];
    if (b < 0) continue;
    const uint32_t t = v.tcur[(size_t)b * kVox + (cx & 7) + 8 * (cy & 7) + 64 * (cz & 7)];
    c += v.edge_uses[t * 12 + off[a][j][3]];
  }
  return c;
}

__global__ void k_export_vertices(VolDev v, uint64_t* keys, float* t, int32_t* ref, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t owner = slot_in_use(v.vseg, v.vseg_cap, i) ? v.vowner[i] : kNone;
    uint64_t k = ~0ull;
    int32_t r = -1;
    if (owner != kNone) {
      const uint32_t blk = owner / (3 * kVox), rem = owner % (3 * kVox);
      k = edge_key(v.block_key[blk], (int)(rem % kVox), (int)(rem / kVox));
      r = edge_count(v, blk, (int)(rem / kVox), (int)(rem % kVox));
    }
    keys[i] = k;
    ref[i] = r;
    t[i] = owner != kNone ? v.et[owner] : 0.f;
  }
}

__global__ void k_lookup(VolDev v, const int32_t* __restrict__ coords, int32_t* __restrict__ idx,
                         uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int x = coords[3 * i], y = coords[3 * i + 1], z = coords[3 * i + 2];
    idx[i] = key_in_range(x, y, z) ? hash_find(v, pack_key(x, y, z)) : -1;
  }
}

#define VM_CLASSIFY_MODES(W)                                      \
  template __global__ void k_classify<W, kExtract>(VolDev, uint32_t); \
  template __global__ void k_classify<W, kRefine>(VolDev, uint32_t);  \
  template __global__ void k_classify<W, kExtractRefined>(VolDev, uint32_t);
VM_CLASSIFY_MODES(2)
VM_CLASSIFY_MODES(4)
VM_CLASSIFY_MODES(8)
template __global__ void k_vertices<2>(VolDev, uint32_t, int);
template __global__ void k_vertices<4>(VolDev, uint32_t, int);
template __global__ void k_vertices<8>(VolDev, uint32_t, int);
template __global__ void k_fuse<2>(VolDev, FrameParams, const float*, uint32_t);
template __global__ void k_fuse<4>(VolDev, FrameParams, const float*, uint32_t);
template __global__ void k_fuse<8>(VolDev, FrameParams, const float*, uint32_t);
template __global__ void k_import_copy<2>(VolDev, const float*, const float*, uint32_t, int32_t*);
template __global__ void k_import_copy<4>(VolDev, const float*, const float*, uint32_t, int32_t*);
template __global__ void k_import_copy<8>(VolDev, const float*, const float*, uint32_t, int32_t*);
template __global__ void k_bwd_tsdf<2>(VolDev, const float*, int, const int32_t*, uint32_t, float*);
template __global__ void k_bwd_tsdf<4>(VolDev, const float*, int, const int32_t*, uint32_t, float*);
template __global__ void k_bwd_tsdf<8>(VolDev, const float*, int, const int32_t*, uint32_t, float*);

}  // namespace vm
