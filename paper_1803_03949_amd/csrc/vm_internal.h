// Internal device-side layout and helpers of the voxmesh library (gfx950).
//
// Volume state lives in one workspace buffer, carved into structure-of-arrays
// regions (block-major, voxel-minor): the kernels that give each 8^3 block
// one wave (eight voxels or cubes per lane, one column of 8 along z) read
// and write a block's rows as coalesced 2 KiB runs.
//   hash      u64 slot = (42-bit block key << 22) | 22-bit pool index,
//             all-ones = empty; open addressing with linear probing and
//             64-bit compare-and-swap inserts, no deletion; a per-slot frame
//             stamp marks the blocks a frame collected.
//   blocks    key u64, 27-neighbour index table, TSDF f32[512],
//             weight f32[512], previous/current cube type u8[512],
//             per owned edge (three per voxel): vertex slot i32 and the
//             vertex's t f32; which owned edges hold a vertex, one 32-bit
//             word per column of voxels (u32[64]); observed-voxel
//             (weight > 0), negative-TSDF and near-zero (|TSDF| < eps)
//             bitmasks u64[8] each; pass stamps.  Reference counts are not stored: a cube's type
//             fixes how many of its triangles use each of its edges, so an
//             edge's count is formed from the four cubes around it.
//   vertices  per pool slot: owner edge (index into the edge arrays, kNone
//             when free), recycle ring, download row, birth frame.
//   triangles no storage of their own: a cube's applied type names its
//             triangles and each triangle's three edges, and each edge
//             holds its one vertex, so the types are the triangle records;
//             a download resolves them to vertex rows.
//
// Contention on single counters is what limits a GPU here, not bytes: every
// list is built with at most one atomic per workgroup, and the vertex pool
// is split into up to kSegs independent segments (a block's
// allocations go to segment block % nseg; small volumes use fewer segments
// so that each still averages over many blocks), each with its own 128-byte
// counter line, bump pointer and recycle ring.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace vm {

constexpr int kVox = 512;                    // voxels (cubes) per block
constexpr uint64_t kEmpty = ~0ull;           // empty hash slot
constexpr uint32_t kIdxBits = 22;
constexpr uint32_t kIdxMask = (1u << kIdxBits) - 1;
// Key inserted, pool index not yet assigned.  Never all-ones, so that no
// occupied slot can read as empty.
constexpr uint32_t kPending = kIdxMask - 1;
constexpr int kKeyBias = 8192;               // block coords in [-8192, 8191]
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kNewFlag = 0x80000000u;   // frame-list entry: block is new
constexpr int kMaxBlocks = 1 << 21;
constexpr int kSegs = 256;                   // pool segments
constexpr int kTile = 512;                   // list items per compaction workgroup (256 lanes)
constexpr int kTilePer = kTile / 256;        // items per lane
// bits that hold a count in [0, n]
constexpr int count_bits(int n) { return n < 2 ? 1 : (n < 4 ? 2 : (n < 8 ? 3 : 4)); }
constexpr int kTileBits = count_bits(kTilePer);  // bits of a lane's count

// Which blocks' TSDF may have changed since the vertices were last placed,
// for the vertex pass: kMovedAll (every block: extraction of everything),
// or else an extraction epoch (epochs start at 1): the blocks stamped
// pending with it, i.e. fused or imported since the last extraction.
constexpr uint32_t kMovedAll = 0u;

// Error bits (bit k <-> VM error code -(k+2)).
constexpr uint32_t kErrHash = 1u << 0;
constexpr uint32_t kErrBlocks = 1u << 1;
constexpr uint32_t kErrVertices = 1u << 2;
constexpr uint32_t kErrRange = 1u << 6;

// One pool segment: slots [base, base + size) of the pool, with its own
// bump pointer, recycle ring (same index range of the ring array) and
// running statistics.  128 bytes, so that segments never share a line.
struct Seg {
  uint32_t hwm;      // slots handed out by bumping, relative to base
  uint32_t head;     // ring read position, in [0, segment size)
  uint32_t count;    // free slots in the ring, from head on (wrapping)
  uint32_t ticket;   // allocations taken since the last finalise
  uint32_t push;     // frees pushed since the last finalise
  uint32_t pad0;
  // the vertex pass adds to each pair with one 64-bit atomic
  uint32_t st_new;   // running count of allocations
  uint32_t st_upd;   // running count of kept vertices
  uint32_t st_mov;   // running count of kept vertices whose t was rewritten
  uint32_t st_freed; // running count of frees
  // classification adds to each pair with one 64-bit atomic; a segment's
  // triangles are st_fnew - st_fold, its cubes with triangles st_cnew - st_cold
  uint32_t st_chg;   // running count of cubes whose triangles changed
  uint32_t st_ref;   // running count of cubes re-typed by refinement
  uint32_t st_cnew;  // running count of changed cubes whose new type has triangles
  uint32_t st_cold;  // running count of changed cubes whose old type had triangles
  uint32_t st_fnew;  // running count of triangles of changed cubes' new types
  uint32_t st_fold;  // running count of triangles of changed cubes' old types
  uint32_t pad[16];
};
static_assert(sizeof(Seg) == 128, "segment record size");

// Device counters (one 256-byte record at the start of the workspace).
struct Counters {
  uint32_t n_blocks;       // pool high-water mark (may exceed capacity on error)
  uint32_t n_frame[2];     // entries of the frame list of frames of each parity
  uint32_t n_pending[2];   // blocks touched since the last extraction (by epoch parity)
  // list lengths, one slot per call parity: a call appends to its own slot
  // and clears the other one, which the next call then uses
  uint32_t n_dirty[2];     // dirty blocks, by extraction parity
  uint32_t n_vblocks[2];   // blocks whose owned edges get recomputed, by
                           // extraction / refinement parity
  uint32_t error;
  uint32_t dl_nv, dl_nt;
  uint32_t n_refined;      // cubes re-typed by the last refinement
  // segment totals when the last extract / refine started
  uint32_t base_new, base_upd, base_freed, base_chg, base_ref;
  uint32_t import_base;    // blocks in the pool before the last import
  uint32_t pad0;
  // collection's appends, by frame parity, packed so that a workgroup
  // reserves its places in all three lists with one atomic (fields below);
  // the fusion that follows folds them into n_frame, n_pending, n_blocks
  unsigned long long collect_acc[2];
  uint32_t pad[8];
  // running totals since the volume was created (not cleared by a reset)
  unsigned long long acc[12];
  unsigned long long pad2[4];
};
static_assert(sizeof(Counters) == 256, "counter record size");
static_assert(offsetof(Counters, collect_acc) < offsetof(Counters, acc), "cleared by a reset");

// Fields of a collection append: frame-list entries (bits 0..20),
// pending-list entries (21..41), new blocks (42..63).  A frame's counts
// stay below 2^21 while it has fewer claims than that; a larger frame
// exceeds the block capacity (at most 2^21) first, and that is reported.
__host__ __device__ inline uint64_t collect_pack(uint32_t frame, uint32_t pend, uint32_t fresh) {
  return (uint64_t)frame | (uint64_t)pend << 21 | (uint64_t)fresh << 42;
}
__host__ __device__ inline uint32_t collect_frame(uint64_t p) { return (uint32_t)(p & 0x1FFFFFu); }
__host__ __device__ inline uint32_t collect_pend(uint64_t p) { return (uint32_t)((p >> 21) & 0x1FFFFFu); }
__host__ __device__ inline uint32_t collect_new(uint64_t p) { return (uint32_t)(p >> 42); }

// Everything a kernel needs, passed by value.
struct VolDev {
  float s, inv_s, inv_block, mu_m, mu_v, eps;
  uint32_t hash_mask;
  int32_t hash_mode;
  uint32_t max_blocks, max_vertices;
  uint32_t xsel;              // parity of the current extraction (dirty list)
  uint32_t frame;             // frames (integrations, imports) since the last reset
  uint32_t vsel;              // parity of the current extraction / refinement (vertex list)
  uint32_t nseg;              // pool segments in use (1..kSegs)
  uint32_t vseg_cap;            // vertex slots per segment
  Counters* cnt;
  Seg* vseg;                  // [kSegs] vertex pool segments
  Seg* cseg;                  // [kSegs] cube statistics (changed, refined, triangles)
  const uint8_t* tri_table;   // [256][16]: count, then 15 cube-edge ids
  const uint8_t* edge_uses;   // [256][12]: triangles of the type using the edge
  const uint32_t* edge_roles; // [4][256]: the same counts packed by role (vertex pass)
  unsigned long long* slots;  // [hash]
  uint32_t* slot_stamp;       // [hash] frame that last collected the slot
  uint32_t* slot_src;         // [hash] import: source row of the slot's block
  uint64_t* block_key;        // [B]
  int32_t* nbr;               // [B][27]
  float* d;                   // [B][512]
  float* w;                   // [B][512]
  uint8_t* tprev;             // [B][512]
  uint8_t* tcur;              // [B][512]
  int32_t* evtx;              // [B][3][512] vertex slot of the edge: valid where the
                              // edge's emask bit is set (-1 after a failed
                              // allocation), stale elsewhere
  float* et;                  // [B][3][512] t of the edge's vertex
  uint32_t* emask;            // [B][64] word q: edges (a, q + 64 lz) that hold a
                              // vertex, bit 8a + lz
  uint64_t* wmask;            // [B][8] per z layer: voxels with weight > 0 (bit x + 8y)
  uint64_t* smask;            // [B][8] per z layer: voxels with TSDF < 0 (bit x + 8y)
  uint64_t* nmask;            // [B][8] per z layer: voxels with |TSDF| < eps (bit x + 8y)
  uint32_t* st_pending;       // [B] extraction epoch that listed the block
  uint32_t* st_dirty;         // [B] pass that listed the block as dirty
  uint32_t* st_vtx;           // [B] pass that listed the block for vertices
  uint32_t* st_frame;         // [B] last frame that fused the block
  uint32_t* frame_list;       // [B] pool index | kNewFlag
  uint32_t* frame_src;        // [B] import: source row of each entry
  uint64_t* frame_key;        // [B] collection: block key of each entry
  uint32_t* row_slot;         // [B] import: hash slot of each source row (kNone if refused)
  uint32_t* pending;          // [B]
  uint32_t* dirty;            // [B]
  uint32_t* vcand;            // [8B] vertex-block candidates of each dirty block
  uint32_t* vblocks;          // [B] vertex pass: after a refinement its blocks, after an
                              // extraction the extra ones beyond the dirty list
  uint32_t* vowner;           // [V] index into the edge arrays, kNone if free
  uint32_t* vring;            // [V]
  int32_t* vdl;               // [V] row in the last download, -1 if none
  uint32_t* vbirth;           // [V] frame in which the vertex last became used
  uint32_t* scan;             // [scan_cap] download partial sums
  uint32_t scan_cap;
  uint32_t batch;             // number of volume slots, 0 for a plain volume
  uint32_t bound;             // d and w are the caller's arrays (vm_bind_tsdf)
  uint32_t order;             // 0: strided block-to-workgroup mapping, 1: runs
};

// Batched volumes: slot k's block x lies in [0, kSlotSpan - 2] and is stored
// at x + kSlotSpan * k - kKeyBias, so slots never touch.
constexpr int kSlotSpan = 64;
constexpr int kMaxSlots = 16384 / kSlotSpan;

// Block position in the frame its positions are reported in: the world for a
// plain volume, the slot's own frame (and the slot index) for a batch.
__device__ inline void block_frame(const VolDev& v, int& bx, int& slot) {
  slot = 0;
  if (v.batch) {
    slot = (bx + kKeyBias) / kSlotSpan;
    bx = (bx + kKeyBias) % kSlotSpan;
  }
}

// Items of a loop shared by `lanes` workers per workgroup (waves or whole
// workgroups, lanes = 1).  Order bit 0: strided (item i to workgroup
// i / lanes mod grid) or contiguous runs of about n / grid items per
// workgroup.  Bit 1: the list is first cut into 8 equal contiguous ranges,
// one per XCD (workgroup b runs on XCD b mod 8, and each XCD has an L2 of
// its own), which that XCD's workgroups then share as bit 0 says; so
// neighbouring list entries are handled under one L2.
struct ItemLoop {
  uint32_t i, end, step;
};
__device__ inline ItemLoop item_loop(const VolDev& v, uint32_t n, uint32_t lanes, uint32_t lane) {
  uint32_t lo = 0, hi = n, wg = blockIdx.x, groups = gridDim.x;
  if ((v.order & 2u) && gridDim.x >= 8) {
    const uint32_t x = blockIdx.x & 7u;
    lo = (uint32_t)((uint64_t)n * x / 8);
    hi = (uint32_t)((uint64_t)n * (x + 1) / 8);
    wg = blockIdx.x >> 3;
    groups = (gridDim.x >> 3) + (x < (gridDim.x & 7u) ? 1u : 0u);
  }
  if ((v.order & 1u) == 0) return {lo + wg * lanes + lane, hi, groups * lanes};
  const uint32_t per = (hi - lo + groups - 1) / groups;
  const uint32_t b = min(hi, lo + wg * per);
  return {b + lane, min(hi, b + per), lanes};
}

// Per-frame camera parameters, passed by value.
struct FrameParams {
  float Rcw[9], tcw[3];   // sensor -> world
  float Rwc[9], twc[3];   // world -> sensor (inverted on the host in FP64)
  float fx, fy, cx, cy, dmin, dmax;
  int32_t W, H;
  uint32_t frame;
};

// ---- block keys ------------------------------------------------------------
__host__ __device__ inline uint64_t pack_key(int x, int y, int z) {
  return ((uint64_t)(uint32_t)(x + kKeyBias) << 28) | ((uint64_t)(uint32_t)(y + kKeyBias) << 14) |
         (uint64_t)(uint32_t)(z + kKeyBias);
}
__host__ __device__ inline void unpack_key(uint64_t k, int& x, int& y, int& z) {
  x = (int)((k >> 28) & 0x3FFF) - kKeyBias;
  y = (int)((k >> 14) & 0x3FFF) - kKeyBias;
  z = (int)(k & 0x3FFF) - kKeyBias;
}
__host__ __device__ inline bool key_in_range(int x, int y, int z) {
  return x >= -kKeyBias && x < kKeyBias && y >= -kKeyBias && y < kKeyBias && z >= -kKeyBias &&
         z < kKeyBias;
}
// Public edge key: block coords (14 bits each), local voxel (9), axis (2).
__host__ __device__ inline uint64_t edge_key(uint64_t bkey, int local, int axis) {
  return (bkey << 11) | ((uint64_t)local << 2) | (uint64_t)axis;
}

__device__ inline uint32_t hash_home(uint64_t key, uint32_t mask, int mode) {
  if (mode == 1) return 0;
  uint64_t h = key + 0x9E3779B97F4A7C15ull;  // splitmix64 finaliser
  h = (h ^ (h >> 30)) * 0xBF58476D1CE4E5B9ull;
  h = (h ^ (h >> 27)) * 0x94D049BB133111EBull;
  h ^= h >> 31;
  return (uint32_t)h & mask;
}

__device__ inline unsigned long long load_slot(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Find-or-insert a block key.  Returns the slot, or -1 when the table is
// full.  A new entry's pool index is kPending until the compaction pass.
// Probes use plain (cacheable) loads: a slot's key never changes once set,
// so a stale read can only show an empty slot, and the compare-and-swap
// that follows returns the slot's true content.
// Insert (if absent) and also return the slot's contents as this lane saw
// them with the key in place: key | kPending for a key new to the table in
// the current kernel, key | pool index otherwise.
__device__ inline int64_t hash_insert_seen(const VolDev& v, uint64_t key,
                                           unsigned long long* seen) {
  uint32_t h = hash_home(key, v.hash_mask, v.hash_mode);
  for (uint32_t probe = 0; probe <= v.hash_mask; ++probe) {
    uint32_t s = (h + probe) & v.hash_mask;
    unsigned long long cur = v.slots[s];
    if (cur == kEmpty) {
      unsigned long long want = ((unsigned long long)key << kIdxBits) | kPending;
      unsigned long long prev = atomicCAS(&v.slots[s], (unsigned long long)kEmpty, want);
      if (prev == kEmpty) {
        *seen = want;
        return s;
      }
      cur = prev;
    }
    if ((cur >> kIdxBits) == key) {
      *seen = cur;
      return s;
    }
  }
  return -1;
}

__device__ inline int64_t hash_insert(const VolDev& v, uint64_t key) {
  uint32_t h = hash_home(key, v.hash_mask, v.hash_mode);
  for (uint32_t probe = 0; probe <= v.hash_mask; ++probe) {
    uint32_t s = (h + probe) & v.hash_mask;
    unsigned long long cur = v.slots[s];
    if (cur == kEmpty) {
      unsigned long long want = ((unsigned long long)key << kIdxBits) | kPending;
      unsigned long long prev = atomicCAS(&v.slots[s], (unsigned long long)kEmpty, want);
      if (prev == kEmpty) return s;
      cur = prev;
    }
    if ((cur >> kIdxBits) == key) return s;
  }
  return -1;
}

// Pool index of a key, or -1 if absent (or not yet assigned).  For use
// after the kernel that assigned the indices has completed.
__device__ inline int32_t hash_find(const VolDev& v, uint64_t key) {
  uint32_t h = hash_home(key, v.hash_mask, v.hash_mode);
  for (uint32_t probe = 0; probe <= v.hash_mask; ++probe) {
    uint32_t s = (h + probe) & v.hash_mask;
    unsigned long long cur = v.slots[s];
    if (cur == kEmpty) return -1;
    if ((cur >> kIdxBits) == key) {
      uint32_t idx = (uint32_t)(cur & kIdxMask);
      return idx == kPending ? -1 : (int32_t)idx;
    }
  }
  return -1;
}

// ---- neighbour directions --------------------------------------------------
__host__ __device__ inline int nbr_dir(int dx, int dy, int dz) {
  return (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
}
constexpr int kSelf = 13;

// ---- wave and workgroup helpers (wave64) ------------------------------------
__device__ inline uint64_t lanes_below() {
  return (1ull << __lane_id()) - 1ull;
}

// Make a wave's LDS writes visible to the other lanes of the same wave (no
// workgroup barrier: waves that own separate LDS regions run independently).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A value every lane of the wave holds alike (a list entry read at a
// wave-uniform index), moved to a scalar register so that the addressing
// derived from it is scalar.
__device__ inline uint32_t uniform(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

// The lane index, opaque to loop-invariant code motion: values derived from
// it inside a loop are recomputed each trip instead of occupying registers
// for the whole loop.
__device__ inline int fresh_lane() {
  int q = __lane_id();
  asm volatile("" : "+v"(q));
  return q;
}

// Exclusive prefix of x over the wave and the wave's total.
__device__ inline uint32_t wave_scan(uint32_t x, uint32_t* total) {
  const int lane = __lane_id();
  uint32_t incl = x;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  *total = __shfl(incl, 63);
  return incl - x;
}

__device__ inline uint32_t wave_sum(uint32_t x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// Sum over the wave of per-lane values in [0, 2^B): one ballot per bit,
// counted in scalar registers, so there is no chain of cross-lane moves.
template <int B>
__device__ inline uint32_t wave_sum_bits(uint32_t x) {
  uint32_t s = 0;
#pragma unroll
  for (int b = 0; b < B; ++b) s += (uint32_t)__popcll(__ballot((x >> b) & 1u)) << b;
  return s;
}

// Lanes below this one whose bit is set in the wave mask m, plus acc.
__device__ inline uint32_t mask_rank(uint64_t m, uint32_t acc = 0) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, acc));
}

// Exclusive prefix over the wave of per-lane values in [0, 2^B), and the
// wave's total: one ballot per bit.
template <int B>
__device__ inline uint32_t wave_prefix_bits(uint32_t x, uint32_t* total) {
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const uint64_t m = __ballot((x >> b) & 1u);
    pre += mask_rank(m) << b;
    tot += (uint32_t)__popcll(m) << b;
  }
  *total = tot;
  return pre;
}

__device__ inline uint64_t shfl64(uint64_t x, int src) {
  const uint32_t lo = __shfl((uint32_t)x, src), hi = __shfl((uint32_t)(x >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

// Exclusive prefix of x over the workgroup and its total, for workgroups of
// up to 16 waves.  Every lane must call; swave holds 16 words of LDS.
__device__ inline uint32_t wg_scan(uint32_t x, uint32_t* swave, uint32_t* total) {
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  const int nwave = (blockDim.x + 63) >> 6;
  uint32_t incl = x;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  if (lane == 63) swave[wave] = incl;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int w = 0; w < nwave; ++w) {
    const uint32_t c = swave[w];
    if (w < wave) before += c;
    all += c;
  }
  __syncthreads();
  *total = all;
  return before + incl - x;
}

// wg_scan for per-lane values in [0, 2^B): the wave prefix comes from one
// ballot per bit (lane-masked popcounts), the wave totals go through LDS.
template <int B>
__device__ inline uint32_t wg_scan_bits(uint32_t x, uint32_t* swave, uint32_t* total) {
  const int wave = threadIdx.x >> 6;
  const int nwave = (blockDim.x + 63) >> 6;
  const uint64_t below = lanes_below();
  uint32_t pre = 0, wt = 0;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const uint64_t m = __ballot((x >> b) & 1u);
    pre += (uint32_t)__popcll(m & below) << b;
    wt += (uint32_t)__popcll(m) << b;
  }
  if (__lane_id() == 0) swave[wave] = wt;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int w = 0; w < nwave; ++w) {
    const uint32_t c = swave[w];
    if (w < wave) before += c;
    all += c;
  }
  __syncthreads();
  *total = all;
  return before + pre;
}

// Segment bounds.
__device__ inline uint32_t seg_size(uint32_t s, uint32_t cap, uint32_t total) {
  const uint64_t b = (uint64_t)s * cap;
  return b >= total ? 0u : (uint32_t)((total - b) < cap ? (total - b) : cap);
}

// Ring position p + k for p < size and k <= size: one wrap at most, so no
// division.
__device__ inline uint32_t ring_pos(uint32_t p, uint32_t k, uint32_t size) {
  const uint32_t r = p + k;
  return r >= size ? r - size : r;
}

// Slot of allocation ticket k of a segment: from its recycle ring first,
// then by bumping; kNone when the segment is exhausted.  The segment's
// head/count/hwm are fixed for the duration of the allocating kernel.
__device__ inline uint32_t seg_slot(uint32_t head, uint32_t count, uint32_t hwm, uint32_t k,
                                    const uint32_t* ring, uint32_t base, uint32_t size) {
  if (k < count) return ring[base + ring_pos(head, k, size)];
  const uint64_t s = (uint64_t)hwm + (k - count);
  return s < size ? base + (uint32_t)s : kNone;
}

// The 217 cells of a 9^3 halo region that are not in the 8^3 block: those
// with some coordinate at the outer layer `edge` (8 for the +x/+y/+z halo,
// -1 for the -x/-y/-z one).  Faces x, y, z (64 each), then the three
// edges (8 each), then the corner.  Writes the cell's coordinates.
__device__ inline void halo_cell(int h, int edge, int& x, int& y, int& z) {
  const int a = h & 7, b = (h >> 3) & 7;
  if (h < 64) x = edge, y = a, z = b;
  else if (h < 128) x = a, y = edge, z = b;
  else if (h < 192) x = a, y = b, z = edge;
  else if (h < 200) x = edge, y = edge, z = a;
  else if (h < 208) x = edge, y = a, z = edge;
  else if (h < 216) x = a, y = edge, z = edge;
  else x = edge, y = edge, z = edge;
}

__device__ inline bool depth_ok(float D, float dmin, float dmax) {
  return isfinite(D) && D > 0.f && D >= dmin && D <= dmax;
}

// One voxel's fusion sample (Eq. 2): projection to the nearest pixel and
// the truncated projective distance.  Shared by the forward fusion and its
// backward pass so both take identical branches.
struct FuseSample {
  bool upd;
  bool clamped;
  int pixel;
  float dt;
};

// The voxel's nearest pixel (-1 when it is behind the camera or outside the
// image) and its camera depth z.
struct FuseProj {
  int pix;
  float z;
};

__device__ inline FuseProj fuse_project(const VolDev& v, const FrameParams& fp, int gx, int gy,
                                        int gz) {
  FuseProj r{-1, 0.f};
  float X = (float)gx * v.s, Y = (float)gy * v.s, Z = (float)gz * v.s;
  float xc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float a = fp.Rwc[3 * i] * X;
    a = a + fp.Rwc[3 * i + 1] * Y;
    a = a + fp.Rwc[3 * i + 2] * Z;
    a = a + fp.twc[i];
    xc[i] = a;
  }
  if (!(xc[2] > 0.f)) return r;
  float u = fp.fx * (xc[0] / xc[2]) + fp.cx;
  float vv = fp.fy * (xc[1] / xc[2]) + fp.cy;
  float fu = floorf(u + 0.5f), fv = floorf(vv + 0.5f);
  if (!(fu >= 0.f && fu < (float)fp.W && fv >= 0.f && fv < (float)fp.H)) return r;
  r.pix = (int)fv * fp.W + (int)fu;
  r.z = xc[2];
  return r;
}

// The fusion sample from the projection and the pixel's depth D.
__device__ inline FuseSample fuse_finish(const VolDev& v, const FrameParams& fp, FuseProj p,
                                         float D) {
  FuseSample r{false, false, -1, 0.f};
  if (p.pix < 0 || !depth_ok(D, fp.dmin, fp.dmax)) return r;
  float sdf = (D - p.z) * v.inv_s;
  if (sdf < -v.mu_v) return r;
  r.upd = true;
  r.clamped = sdf >= v.mu_v;
  r.pixel = p.pix;
  r.dt = fminf(sdf, v.mu_v);
  return r;
}

__device__ inline FuseSample fuse_sample(const VolDev& v, const FrameParams& fp,
                                         const float* __restrict__ depth, int gx, int gy,
                                         int gz) {
  const FuseProj p = fuse_project(v, fp, gx, gy, gz);
  return fuse_finish(v, fp, p, p.pix >= 0 ? depth[p.pix] : 0.f);
}

// Eqs. (3)-(5) in two halves.  The paper lists the regular types as three
// complementary pairs, 11001100/00110011, 10011001/01100110,
// 11110000/00001111: a type's distances to the two members of a pair add to
// 8, so at most one member is within 3.  Per type t, refine_candidates
// gives those members as corner flips x = t ^ r (bytes 0..2, nearest first,
// ties in the listed order) and, in the high word, bit 8k + 7 set when byte
// k holds one and bit 31 set when t is itself a regular type.
__host__ __device__ inline uint64_t refine_candidates(uint32_t t) {
  uint32_t xs[3] = {0u, 0u, 0u}, ds[3] = {0u, 0u, 0u};
  int n = 0;
  for (int j = 0; j < 3; ++j) {
    const uint32_t r = j == 0 ? 0xCCu : (j == 1 ? 0x99u : 0xF0u);
    uint32_t x = t ^ r, d = 0;
    for (int k = 0; k < 8; ++k) d += (x >> k) & 1u;
    if (d > 4u) x ^= 0xFFu, d = 8u - d;  // the complementary member
    if (d > 3u) continue;
    int i = n++;
    for (; i > 0 && ds[i - 1] > d; --i) xs[i] = xs[i - 1], ds[i] = ds[i - 1];  // stable
    xs[i] = x, ds[i] = d;
  }
  uint32_t lo = 0, hi = 0;
  for (int k = 0; k < n; ++k) lo |= xs[k] << (8 * k), hi |= 0x80u << (8 * k);
  if (n > 0 && ds[0] == 0u) hi |= 0x80000000u;
  return (uint64_t)hi << 32 | lo;
}

// The refined type of a valid cube of type t, previous type prev (whether
// that is a regular type: prev_regular), with near8 bit k set when corner
// k's |TSDF| < eps (Eq. 5), from t's candidates: prev if it is one whose
// flipped corners are all near zero, else the first such candidate, else t;
// t itself when d_H(t, prev) > 3.
__host__ __device__ inline uint32_t refine_type(uint32_t t, uint32_t prev, bool prev_regular,
                                                uint32_t near8, uint64_t cand) {
  // evaluated without branches: most lanes of a wave take every path
  const uint32_t xp = t ^ prev, far = ~near8 & 0xFFu;
  // bit 8k + 7 of bad: candidate k flips a corner that is not near zero
  const uint32_t m = (uint32_t)cand & far * 0x010101u;
  const uint32_t bad = (((m & 0x7F7F7Fu) + 0x7F7F7Fu) | m) & 0x808080u;
  const uint32_t ok = (uint32_t)(cand >> 32) & 0x808080u & ~bad;
  const uint32_t first = t ^ (((uint32_t)cand >> (__builtin_ctz(ok | 0x80000000u) & 0x18u)) & 0xFFu);
  const uint32_t r = prev_regular && !(xp & far) ? prev : (ok ? first : t);
  return __builtin_popcount(xp) > 3 ? t : r;
}

__device__ inline float edge_param(float da, float db) {
  if (da == db) return 0.5f;
  return da / (da - db);
}

}  // namespace vm

// ---- kernels (defined in vm_kernels.hip, launched from vm_api.hip) ----------
namespace vm {
__global__ void k_prep(VolDev v, int op, uint32_t arg);
__global__ void k_collect(VolDev v, FrameParams fp, const float* __restrict__ depth,
                          uint32_t epoch);
__global__ void k_import_insert(VolDev v, const int32_t* __restrict__ slots,
                                const int32_t* __restrict__ coords, uint32_t n,
                                uint32_t frame);
__global__ void k_import_count(VolDev v, uint32_t n, uint32_t epoch);
__global__ void k_import_scan(VolDev v, uint32_t nparts, uint32_t frame, uint32_t epoch);
__global__ void k_import_assign(VolDev v, uint32_t n, uint32_t nparts, uint32_t epoch);
constexpr int kImportRows = 256;  // import rows per workgroup of the row-order compaction
template <int W>
__global__ void k_fuse(VolDev v, FrameParams fp, const float* __restrict__ depth, uint32_t epoch);
template <int W>
__global__ void k_import_copy(VolDev v, const float* __restrict__ tsdf,
                              const float* __restrict__ weight, uint32_t frame,
                              int32_t* __restrict__ rows);
__global__ void k_dirty(VolDev v, uint32_t pass, uint32_t epoch);
__global__ void k_dirty_all(VolDev v, uint32_t pass);
// classification modes (k_classify's second template argument)
constexpr int kExtract = 0, kRefine = 1, kExtractRefined = 2;
template <int W, int mode>
__global__ void k_classify(VolDev v, uint32_t pass);
__global__ void k_vblock_compact(VolDev v);
template <int W>
__global__ void k_vertices(VolDev v, uint32_t moved, int walk_dirty);
__global__ void k_dl_count(VolDev v, int what);
__global__ void k_dl_scan(VolDev v, int what, uint32_t nparts);
__global__ void k_dl_write_vertices(VolDev v, float* __restrict__ verts,
                                    uint64_t* __restrict__ keys, uint32_t vcap);
__global__ void k_dl_write_triangles(VolDev v, int32_t* __restrict__ tris, uint32_t tcap);
__global__ void k_dl_normals(VolDev v, float* __restrict__ normals);
__global__ void k_dl_births(VolDev v, uint32_t* __restrict__ births);
__global__ void k_share_lock(VolDev v, int32_t* __restrict__ slot, float* __restrict__ tv,
                             uint32_t* __restrict__ counter);
__global__ void k_share_free(VolDev v, int group, int32_t* __restrict__ slot,
                             float* __restrict__ tv, uint32_t* __restrict__ counter);
template <int W>
__global__ void k_bwd_tsdf(VolDev v, const float* __restrict__ dL_dv, int by_slot,
                           const int32_t* __restrict__ rows, uint32_t n_rows,
                           float* __restrict__ out);
__global__ void k_positions(VolDev v, float* __restrict__ pos, int32_t* __restrict__ slot_of);
__global__ void k_fill_u32(uint32_t* p, uint32_t value, uint64_t n);
__global__ void k_bwd_fusion(VolDev v, FrameParams fp, const float* __restrict__ depth,
                             const float* __restrict__ g1, float* __restrict__ g0,
                             float* __restrict__ gD);
__global__ void k_zero_f32(float* p, uint64_t n);
__global__ void k_export_vertices(VolDev v, uint64_t* keys, float* t, int32_t* ref, uint32_t n);
__global__ void k_lookup(VolDev v, const int32_t* __restrict__ coords, int32_t* __restrict__ idx,
                         uint32_t n);
}  // namespace vm

// Bookkeeping operations of k_prep.  Every one of them first finalises the
// pool segments (recycled slots consumed, bump pointers advanced, frees
// made available), which is idempotent.
enum {
  VM_OP_REFINE = 2,     // before a refinement: snapshot, clear the next vertex list
  VM_OP_FINALISE = 4,   // segments only
  VM_OP_RESET = 5       // before a reset: fold segment statistics into the totals
};
