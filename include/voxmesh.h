/*
 * voxmesh -- incremental mesh extraction over a spatially hashed TSDF volume
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: Dong, Shi, Tang, Wang, Zha, "An Efficient Volumetric Mesh
 * Representation for Real-time Scene Reconstruction using Spatial Hashing",
 * arXiv 1803.03949.  Each depth frame is fused into 8x8x8-voxel blocks held in
 * a hash table (Sec. III, Eqs. 1-2); every cube gets its marching-cubes type
 * (Sec. V-B); each vertex lives exactly once, on the lattice edge that owns
 * it (Sec. IV, V-C); triangles reference vertices and reference counts drive
 * garbage collection (Sec. V-D, V-E); the Hamming-distance refinement snaps
 * disturbed cubes to regular types (Sec. V-F, Eqs. 3-5).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Return value: VM_OK (0) or a negative VM_ERR_* code.
 * - Every call is enqueued on the given HIP stream and returns without
 *   waiting, except vm_download_mesh, vm_get_status and the vm_export_*
 *   calls, which synchronise that stream.  A volume must be used from one
 *   stream at a time.
 * - The caller owns all device memory.  The library never allocates device
 *   memory: a volume lives in one caller buffer of vm_volume_bytes() bytes,
 *   and every input/output array is a caller pointer.  Pointers documented
 *   as "device" must be device (or managed) memory; "host" pointers are read
 *   before the call returns.
 * - Capacity overflow inside a kernel (hash table, block pool, vertex pool)
 *   sets a sticky error bit in the volume; the next
 *   synchronising call returns the matching VM_ERR_* code.  The volume is
 *   not usable for meshing after such an error (reset it).
 * - Lattice: voxel g (integer 3-vector) sits at world position g * voxel_m;
 *   its TSDF (voxel units) and weight live at that corner.  Block b holds the
 *   voxels 8b .. 8b+7 per axis, stored in local order x + 8y + 64z.  Block
 *   coordinates must lie in [-8192, 8191].
 * - Edge keys (vm_download_mesh, vm_export_vertices): the edge that starts
 *   at voxel g = 8b + l and runs one step along axis a (0 x, 1 y, 2 z) has
 *   key ((b.x+8192) << 39) | ((b.y+8192) << 25) | ((b.z+8192) << 11)
 *     | ((l.x + 8 l.y + 64 l.z) << 2) | a.
 * - Batches: a volume created with batch_volumes = m > 0 holds m independent
 *   volumes ("slots") in one hash table and one set of pools, so that every
 *   call processes all of them in the same kernel launches.  Block (x, y, z)
 *   of slot k, with 0 <= x <= 62, is stored at block coordinate
 *   (64k - 8192 + x, y, z): slots lie 64 blocks apart along x with at least
 *   one empty block between them, so no cube, edge or vertex spans two
 *   slots and each slot's mesh and gradients are exactly those of a plain
 *   volume holding only its blocks.  Edge keys carry the stored coordinate
 *   (key bits 39.. hold 64k + x); vertex positions are in the slot's frame.
 *   Blocks enter through vm_import_batch; vm_integrate_depth and
 *   vm_import_blocks reject a batch.
 * - Floating point: FP32 everywhere on the hot path, without contraction of
 *   products into fused multiply-adds and with correctly rounded division, so
 *   fusion and cube signs are reproducible bit for bit.
 */
#ifndef VOXMESH_H
#define VOXMESH_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  VM_OK = 0,
  VM_ERR_ARG = -1,             /* invalid argument or configuration */
  VM_ERR_HASH_FULL = -2,       /* hash table probe sequence exhausted */
  VM_ERR_BLOCK_POOL_FULL = -3, /* more blocks than max_blocks */
  VM_ERR_VERTEX_POOL_FULL = -4,/* a vertex pool segment is full (max_vertices) */
                               /* (-5 is not used: triangles take no pool) */
  VM_ERR_CAPACITY = -6,        /* caller output buffer or workspace too small */
  VM_ERR_HIP = -7,             /* a HIP runtime call failed */
  VM_ERR_RANGE = -8            /* a block coordinate outside [-8192, 8191] */
};

enum { VM_SCOPE_DIRTY = 0, VM_SCOPE_ALL = 1 };
/* Flag OR-ed into vm_extract_mesh's scope: refine each new type (Sec. V-F)
 * before its vertices and triangles are made. */
enum { VM_EXTRACT_REFINE = 0x100 };

/* Volume configuration.  Sizes are capacities of the caller buffer: per
 * block of max_blocks about 17.6 KiB (TSDF and weight 4 KiB, types 1 KiB,
 * vertex slot and t of its 1536 owned edges 12 KiB, one bit per edge for
 * whether it holds a vertex, 64-byte masks of its observed and of its
 * negative-TSDF voxels, lists and stamps), per vertex of max_vertices 16
 * bytes, plus 16 bytes per hash slot.  Triangles take no memory of their
 * own: a cube's type names them (see vm_extract_mesh). */
typedef struct vm_config {
  float voxel_m;        /* cube edge length s in metres (e.g. 0.008) */
  float trunc_vox;      /* truncation mu in voxel units (e.g. 4) */
  float refine_eps_vox; /* refinement threshold epsilon, voxel units (Eq. 5) */
  int32_t hash_log2;    /* hash table holds 2^hash_log2 slots, 10..28 */
  int32_t max_blocks;   /* block pool capacity, 1 .. 2^21 */
  int32_t max_vertices; /* vertex pool capacity, 1 .. 2^30, split into
                           n = clamp(max_blocks / 256, 1, 256) segments of
                           ceil(max_vertices / n) slots (the last one the
                           remainder): the block at pool
                           row b creates its vertices in segment b mod n
                           only (one allocation atomic per block and
                           segment), so VM_ERR_VERTEX_POOL_FULL is raised
                           when one segment's share is exhausted, which can
                           come before max_vertices live vertices when the
                           surface crowds the blocks of one segment
                           (vm_status reports the fullest segment) */
  int32_t hash_mode;    /* 0: mixing hash; 1: every key starts probing at
                           slot 0 (long probe chains, for testing only) */
  int32_t batch_volumes;/* 0: a plain volume; m in 1..256: a batch of m
                           independent volumes (see "Batches" below) */
} vm_config;

/* Pinhole camera, pixel (u, v) at column u, row v; depth in metres. */
typedef struct vm_intrinsics {
  float fx, fy, cx, cy;
  int32_t width, height;
  float min_depth_m, max_depth_m; /* depth outside this range is invalid */
} vm_intrinsics;

/* Counters and the sticky error, as of the last completed call. */
typedef struct vm_status {
  int32_t error;            /* VM_OK or the first VM_ERR_* raised on device */
  uint32_t error_bits;      /* bit k set: error code -(k+2) was raised */
  int64_t blocks;           /* allocated blocks */
  int64_t frame_blocks;     /* blocks collected by the last integrate/import */
  int64_t pending_blocks;   /* blocks touched since the last extraction */
  int64_t dirty_blocks;     /* blocks classified by the last extract/refine */
  int64_t vertex_blocks;    /* blocks whose owned edges were recomputed */
  int64_t changed_cubes;    /* cubes whose triangles changed */
  int64_t vertex_slots;     /* vertex pool high-water mark */
  int64_t free_vertex_slots;/* recycled vertex slots awaiting reuse */
  int64_t triangles;        /* triangles of the current mesh */
  int64_t tri_cubes;        /* cubes holding triangles */
  int64_t new_vertices;     /* vertices created by the last extract/refine */
  int64_t updated_vertices; /* vertices whose position was rewritten */
  int64_t freed_vertices;   /* vertices recycled by the last extract/refine */
  int64_t refined_cubes;    /* cubes the last extract/refine re-typed by Eqs. 3-5 */
  int64_t vertex_segments;  /* segments of the vertex pool (see max_vertices) */
  int64_t segment_capacity; /* vertex slots per segment */
  int64_t max_segment_live; /* live vertices of the fullest segment */
} vm_status;

/* Running totals of work done since the volume was created (kept across
 * vm_reset_volume), read with vm_get_totals.  Benchmarks turn them into
 * bytes moved per kernel. */
enum {
  VM_TOTAL_FRAMES = 0,          /* integrations and imports */
  VM_TOTAL_FRAME_BLOCKS = 1,    /* blocks collected over all of them */
  VM_TOTAL_DIRTY_BLOCKS = 2,    /* blocks classified (extract and refine) */
  VM_TOTAL_VERTEX_BLOCKS = 3,   /* blocks whose owned edges were recomputed */
  VM_TOTAL_NEW_VERTICES = 4,
  VM_TOTAL_UPDATED_VERTICES = 5, /* vertices of recomputed edges that stay */
  VM_TOTAL_CHANGED_CUBES = 6,   /* cubes whose triangles were replaced */
  VM_TOTAL_NEW_TRIANGLES = 7,   /* triangles of those cubes' new types */
  VM_TOTAL_FREED_VERTICES = 8,
  VM_TOTAL_REFINED_CUBES = 9,
  VM_TOTAL_DROPPED_TRIANGLES = 10, /* triangles of those cubes' old types */
  VM_TOTAL_MOVED_VERTICES = 11, /* updated vertices whose t was rewritten (an end
                                   point's block fused or imported since the last
                                   extraction); the others keep their t */
  VM_TOTAL_COUNT = 12
};

/* Kernels, for vm_profile_read. */
enum {
  VM_K_COLLECT = 0,      /* block collection along pixel rays (Eq. 1) */
  VM_K_ASSIGN = 1,       /* import: pool indices for new blocks, in row order */
  VM_K_FUSE = 2,         /* TSDF fusion (Eq. 2) */
  VM_K_IMPORT = 3,       /* import: hash inserts, block state and copies */
  VM_K_DIRTY = 4,        /* dirty block list, vertex block list */
  VM_K_CLASSIFY = 5,     /* cube types, which also replace triangles */
  VM_K_REFINE = 6,       /* cube types, refinement pass */
  VM_K_VERTICES = 7,     /* edge-owned vertices, reference counts, recycling */
  VM_K_DOWNLOAD = 8,     /* download compaction (all its kernels) */
  VM_K_BACKWARD = 9,     /* backward passes */
  VM_K_COUNTERS = 10,    /* single-wave bookkeeping kernels */
  VM_K_ABLATION = 11,    /* vm_sharing_ablation (the paper's sharing schemes) */
  VM_K_POSITIONS = 12,   /* vm_export_positions */
  VM_K_COUNT = 13
};

typedef struct vm_volume vm_volume;

/* Bytes of device memory a volume with this configuration needs.
 * Returns VM_ERR_ARG for an invalid configuration. */
int vm_volume_bytes(const vm_config* cfg, size_t* bytes);

/* Create a volume inside the caller's device buffer dev_mem (at least
 * vm_volume_bytes() bytes, 256-byte aligned) and clear it on `stream`.
 * *out receives a host-side handle; the buffer must outlive it.  The
 * volume starts empty (Sec. III: blocks are allocated only where depth
 * observations land). */
int vm_create_volume(const vm_config* cfg, void* dev_mem, size_t bytes,
                     hipStream_t stream, vm_volume** out);

/* Largest workspace (vm_volume_bytes) of a volume made by
 * vm_create_volume_noalloc: 64 MiB. */
#define VM_NOALLOC_MAX_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * vm_create_volume with the workspace taken from a static array of
 * VM_NOALLOC_MAX_BYTES that the library holds on every device it runs on
 * until the process ends, instead of a caller buffer.  The call allocates
 * nothing (no device memory, no events, no host heap): the handle lives in
 * static storage too.  The volume behaves as one made by vm_create_volume
 * and is released with vm_destroy_volume.  Returns VM_ERR_CAPACITY when
 * vm_volume_bytes(cfg) exceeds VM_NOALLOC_MAX_BYTES (checked before any HIP
 * call), VM_ERR_ARG for an invalid configuration or while another such
 * volume exists on the current device: all of them would share the one
 * array, so each device holds at most one at a time (calls that overlapped
 * on it would race).  The workspace keeps the last volume's contents;
 * creation clears everything a new volume reads before writing, as
 * vm_create_volume does.  Synchronises `stream` (the table upload). */
int vm_create_volume_noalloc(const vm_config* cfg, hipStream_t stream, vm_volume** out);

/* Release the host handle.  Never frees dev_mem. */
int vm_destroy_volume(vm_volume* vol);

/* Empty the volume again (blocks, mesh, errors), on `stream`. */
int vm_reset_volume(vm_volume* vol, hipStream_t stream);

/* Block collection (Eq. 1) and TSDF fusion (Eq. 2) of one depth frame.
 * depth: device, height*width FP32 metres, row-major, 0 or non-finite =
 * invalid.  cam_to_world: host, 4x4 row-major FP32 sensor-to-world pose
 * [R | t] (Sec. V-A); it is inverted on the host in FP64.
 * For every valid pixel, all blocks in the integer box spanned by the two
 * points of its ray at camera depth D - mu and D + mu are allocated; then
 * every voxel of those blocks that projects (nearest pixel) onto a valid
 * pixel with (D - z)/s >= -mu takes the running average with weight 1 of
 * min((D - z)/s, mu).  A pixel whose box leaves the block coordinate range
 * is skipped.  The depth buffer must stay valid until the stream reaches
 * this call. */
int vm_integrate_depth(vm_volume* vol, const float* depth,
                       const vm_intrinsics* K, const float cam_to_world[16],
                       hipStream_t stream);

/* Allocate the given blocks (if new) and overwrite their TSDF and weights:
 * for volumes sampled from an analytic field rather than fused.
 * coords: device, n*3 int32 block coordinates (distinct); tsdf, weight:
 * device, n*512 FP32 in local voxel order.  The blocks count as touched for
 * the next VM_SCOPE_DIRTY extraction.  New blocks take pool rows in input
 * order (into an empty volume, input row i becomes pool row i), so rows
 * given in a spatial order keep neighbouring blocks close in memory. */
int vm_import_blocks(vm_volume* vol, const int32_t* coords, const float* tsdf,
                     const float* weight, int64_t n, hipStream_t stream);

/* Mesh extraction (Sec. V-B..V-D).  VM_SCOPE_DIRTY: the blocks touched since
 * the last extraction plus their allocated neighbours at offsets in
 * {-1,0}^3 (all cubes with a corner in a touched block); VM_SCOPE_ALL: every
 * block.  For each such cube: type t with bit k = [d(c_k) < 0] over the
 * corners in cyclic order (0,0,0) (1,0,0) (1,1,0) (0,1,0) (0,0,1) (1,0,1)
 * (1,1,1) (0,1,1); a cube with a corner in a missing block or with weight 0
 * has type 0.  The previous type is kept (t_{i-1}).  A cube's triangles are
 * those its type names, each as three cube edges: writing a changed type
 * replaces them, an unchanged cube keeps them (Sec. V-D), and they are
 * resolved to vertex indices only by a download.  Every edge used by some
 * cube's triangles holds one vertex at t = d(g)/(d(g) - d(g+a)) (0.5 if
 * equal), created on first use and updated when its end points move; each
 * vertex's reference count is the number of triangles using it.  With
 * VM_EXTRACT_REFINE in scope, each valid cube's new type t is first replaced
 * by the refinement of vm_refine_mesh against the type it replaces (the
 * paper applies the regular type before marching cubes, Sec. V-F): types,
 * vertices, t, counts and triangles end as after this extraction without
 * the flag followed by vm_refine_mesh, but no vertex is dropped and created
 * again between the two, so none is re-born.  Other scope bits:
 * VM_ERR_ARG. */
int vm_extract_mesh(vm_volume* vol, int scope, hipStream_t stream);

/* Hamming-distance refinement (Sec. V-F, Eqs. 3-5) of the cubes of the last
 * extraction: a valid cube with type t and previous type p is set to the
 * regular type r_j when d_H(t,p) <= 3, d_H(t,r_j) <= 3 and |d(c_k)| < eps
 * on every corner where t and r_j differ; among several qualifying r_j,
 * p is kept if it is one of them, else the nearest, ties in the order
 * 11001100, 00110011, 10011001, 01100110, 11110000, 00001111 (bit 7 first).
 * Triangles and vertices follow; vertex positions extrapolate where the
 * regular type puts a vertex on an edge without a sign change. */
int vm_refine_mesh(vm_volume* vol, hipStream_t stream);

/* Garbage collection (Sec. V-E).  A vertex no triangle uses any more is
 * freed by the extraction (or refinement) that drops its count to zero: its
 * edge forgets it at once, so it is in no download or export from then on,
 * and its slot goes to its pool segment's recycle ring, which the next
 * extraction or refinement opens for allocation before it allocates.  So
 * vm_gc has no device work left and launches nothing; it exists so that a
 * caller follows the method's steps, and returns VM_OK (VM_ERR_ARG for a
 * NULL volume). */
int vm_gc(vm_volume* vol, hipStream_t stream);

/* The mesh handed over as plain arrays, the step the paper times as
 * "compressing" the mesh for rendering (Sec. VI, Table I): live vertices
 * compacted in pool order, each cube's triangles resolved from its type
 * through the edges' owner voxels to vertex rows.  Caller buffers
 * (device): verts[vcap][3] FP32
 * metres (vertex on edge (g, a): g*s with (g_a + t)*s on axis a),
 * edge_keys[vcap] (may be NULL), tris[tcap][3] int32 indices into verts,
 * oriented counter-clockwise seen from the outside (d > 0).  *nv, *nt
 * (host) receive the mesh size; returns VM_ERR_CAPACITY (after filling
 * what fits) when it exceeds vcap or tcap.  Synchronises `stream`.  Also
 * records which output row each vertex went to, for vm_extract_backward. */
int vm_download_mesh(vm_volume* vol, float* verts, uint64_t* edge_keys,
                     int32_t* tris, int64_t vcap, int64_t tcap, int64_t* nv,
                     int64_t* nt, hipStream_t stream);

/* Unit normals of the vertices of the last vm_download_mesh, in its row
 * order: normals[cap][3] FP32 (device).  Sec. IV keeps a normal in every
 * vertex record without fixing how it is formed; here it is the TSDF
 * gradient interpolated along the vertex's edge at its parameter t and
 * normalised, pointing to increasing TSDF (the outside, the side the
 * triangles face).  The gradient at a voxel is, per axis, the central
 * difference over its two neighbours when both are observed (allocated
 * block, weight > 0), the one-sided difference when one is, 0 when neither
 * is; a vertex whose interpolated gradient vanishes gets (0, 0, 0).
 * Call after vm_download_mesh and before the volume changes
 * (VM_ERR_ARG otherwise, or for a NULL volume); VM_ERR_CAPACITY (nothing
 * written) when cap is below the downloaded vertex count.  Stream-ordered;
 * does not synchronise. */
int vm_download_normals(vm_volume* vol, float* normals, int64_t cap, hipStream_t stream);

/* Birth frames of the vertices of the last vm_download_mesh, in its row
 * order: births[cap] (device).  A volume counts frames (vm_integrate_depth
 * and import calls since creation or the last reset, the first being 1); a
 * vertex's birth frame is the frame of the extraction or refinement at the
 * end of which its reference count was positive while at the end of the
 * previous pass it was zero or the vertex did not exist, i.e. how long it has
 * been held (the paper visualises this duration, Fig. 1).  Call after
 * vm_download_mesh and before the volume changes (VM_ERR_ARG otherwise, or
 * for a NULL volume); VM_ERR_CAPACITY (nothing written) when cap is below
 * the downloaded vertex count.  Stream-ordered; does not synchronise. */
int vm_download_births(vm_volume* vol, uint32_t* births, int64_t cap, hipStream_t stream);

/* Ablation (not part of the method's path): the two GPU schemes Sec. V-C
 * gives for initialising each vertex once while the cubes around its edge
 * run in parallel, which Sec. VI-A times against each other, reproduced for
 * measurement beside edge ownership.  Over the cubes of the last
 * extraction's dirty blocks, one lane per cube: for every edge the cube's
 * current type uses, a vertex is allocated if the edge has none (an atomic
 * add on *counter, as from a heap) and the edge parameter t is written.
 * scheme 0, lock-based: the first lane to claim the edge (compare-and-swap)
 * allocates; one launch.  scheme 1, lock-free: the cubes of each 2x2x2 cell
 * in four groups of two at opposite corners, which share no edge; four
 * launches, one per group.  State (device, the caller's, kept across
 * calls): edge_slot and edge_t of max_blocks * 3 * 512 entries indexed
 * (block * 3 + axis) * 512 + voxel, edge_slot -1 for edges without a vertex
 * (the caller fills it before the first call); *counter the number of
 * vertices allocated.  Both schemes leave the same set of edges with a
 * vertex and the same t.  VM_ERR_ARG for NULL arguments or another scheme.
 * Stream-ordered. */
int vm_sharing_ablation(vm_volume* vol, int scheme, int32_t* edge_slot, float* edge_t,
                        uint32_t* counter, hipStream_t stream);

/* Gradient of a loss through the vertex positions of the last download to
 * the fused TSDF, with connectivity fixed: for the vertex on edge (g, a),
 * dv/dt = s * e_a, dt/dd(g) = -d(g+a)/(d(g)-d(g+a))^2 and
 * dt/dd(g+a) = d(g)/(d(g)-d(g+a))^2 (0 where the two are equal).
 * dL_dverts: device, nv*3 FP32 (rows as downloaded); dL_dtsdf: device,
 * blocks*512 FP32 in block pool order (see vm_export_blocks), overwritten.
 * Each voxel gathers its at most six incident edges in a fixed order, so
 * the result is deterministic. */
int vm_extract_backward(vm_volume* vol, const float* dL_dverts,
                        float* dL_dtsdf, hipStream_t stream);

/* Gradient through the last vm_integrate_depth (Eq. 2) with its branches
 * fixed: for a voxel that frame updated, dd1/dd0 = W0/(W0+1) and, unless
 * the truncation at +mu was active, dd1/dD(p) = (1/s)/(W0+1) for its pixel
 * p; other voxels pass dL/dd1 through unchanged.  depth: the same device
 * frame; dL_dtsdf1, dL_dtsdf0: device, blocks*512 FP32 pool order;
 * dL_ddepth: device height*width FP32, overwritten (accumulated with
 * atomics, so its summation order is not fixed). */
int vm_integrate_backward(vm_volume* vol, const float* depth,
                          const float* dL_dtsdf1, float* dL_dtsdf0,
                          float* dL_ddepth, hipStream_t stream);

/* Import with explicit slots and output rows.  slots: device int32 n, the
 * slot of each block (must be NULL for a plain volume, non-NULL for a
 * batch); coords: device n*3 int32 in the slot's frame; tsdf, weight as for
 * vm_import_blocks; rows: device int32 n or NULL, receives each block's
 * row in pool order (for vm_extract_backward_slots).  A slot outside
 * 0..m-1 or x outside 0..62 sets VM_ERR_RANGE and skips the block. */
int vm_import_batch(vm_volume* vol, const int32_t* slots, const int32_t* coords,
                    const float* tsdf, const float* weight, int64_t n,
                    int32_t* rows, hipStream_t stream);

/* Use caller memory as the volume's TSDF and weight storage, so that an
 * import does not copy them (many volumes imported again for every
 * forward + backward, as in a training loop).  tsdf, weight: device,
 * max_blocks*512 FP32 each, in pool row order (row r = the block at pool
 * row r), 4-byte aligned, owned by the caller, who keeps them alive and
 * does not write them while the volume uses them; both NULL returns the
 * volume to its own arrays (their contents are then undefined).  While
 * bound, vm_import_blocks / vm_import_batch must pass these same two
 * pointers (else VM_ERR_ARG), and every imported row must become the pool
 * row of the same number (import into an empty volume, distinct keys, see
 * vm_import_blocks); a row that does not sets VM_ERR_RANGE.  Fusion writes
 * the bound arrays.  Takes effect for calls made after it; kernels already
 * enqueued keep the arrays they were given. */
int vm_bind_tsdf(vm_volume* vol, float* tsdf, float* weight);

/* Positions of every vertex pool entry, uncompacted and without
 * synchronising (for graph capture): pos (device, cap*3 FP32 metres, slot
 * frame) and slot_of (device int32 cap, may be NULL) get, for each entry
 * holding a live vertex, its position and slot (0 for a plain volume), and
 * 0 / -1 for every other entry.  cap must be at least max_vertices
 * (VM_ERR_CAPACITY otherwise); entries from max_vertices on are not
 * written. */
int vm_export_positions(vm_volume* vol, float* pos, int32_t* slot_of,
                        int64_t cap, hipStream_t stream);

/* vm_extract_backward with the upstream gradient per vertex pool entry
 * (dL_dpos: device max_vertices*3 FP32, rows as vm_export_positions; rows
 * of entries without a live vertex are ignored) and the output in the
 * caller's block order: with rows (device int32 n_rows, pool rows e.g. from
 * vm_import_batch; -1 gives a zero row), dL_dtsdf (device n_rows*512 FP32)
 * row i is the gradient of block rows[i]; with rows == NULL it holds every
 * block in pool order.  Deterministic, as vm_extract_backward. */
int vm_extract_backward_slots(vm_volume* vol, const float* dL_dpos,
                              const int32_t* rows, int64_t n_rows,
                              float* dL_dtsdf, hipStream_t stream);

/* Arguments of vm_extract_batch: the blocks of every slot and the
 * forward's and backward's arrays (all device memory, owned by the caller,
 * kept alive and at the same addresses while their graphs are reused). */
typedef struct vm_batch_io {
  const int32_t* slots;  /* n: slot of each block (NULL for a plain volume) */
  const int32_t* coords; /* n*3: block coordinates in the slot's frame */
  const float* tsdf;     /* n*512: TSDF rows (the bound array when bound) */
  const float* weight;   /* n*512: weight rows (likewise) */
  int64_t n;             /* blocks, 1 .. max_blocks */
  int32_t* rows;         /* n, out: pool row of each block */
  float* pos;            /* pos_cap*3, out: position per vertex pool entry */
  int32_t* slot_of;      /* pos_cap, out (may be NULL): slot per entry, -1 none */
  int64_t pos_cap;       /* at least max_vertices */
  const float* dL_dpos;  /* pos_cap*3, in: gradient per vertex pool entry */
  float* dL_dtsdf;       /* n*512, out: gradient per block, input row order */
} vm_batch_io;

enum { VM_BATCH_FORWARD = 1, VM_BATCH_BACKWARD = 2 };

/* The batched forward and backward of many independent volumes (the slots
 * of a batch volume, or one plain volume), each phase one HIP graph that
 * the library captures on the first call and replays on later calls with
 * the same arguments, mapping and bound storage (anything else captures
 * again).  VM_BATCH_FORWARD: empty the volume, import the n blocks
 * (vm_import_batch, rows out), extract the mesh of every block
 * (vm_extract_mesh with VM_SCOPE_ALL) and write every vertex pool entry's
 * position (vm_export_positions).  VM_BATCH_BACKWARD: the TSDF gradient
 * from io->dL_dpos (vm_extract_backward_slots over io->rows), for the mesh
 * of the last forward; the caller computes dL_dpos from the forward's pos
 * in between.  One phase per call: a forward assigns pool entries in no
 * fixed order, so a dL_dpos exists only after it.  On a stream that is
 * being captured, on the
 * legacy default stream (which cannot be captured) and while profiling,
 * the phases are enqueued as plain launches instead.  After a replay the
 * volume's host-side state is what the captured forward left, so status,
 * download and export calls see the replayed mesh.  VM_ERR_ARG for invalid
 * arguments, a phase other than the two, or a volume that rejects the
 * import (see vm_import_batch);
 * VM_ERR_CAPACITY when pos_cap < max_vertices.  Stream-ordered. */
int vm_extract_batch(vm_volume* vol, const vm_batch_io* io, int phase, hipStream_t stream);

/* Workgroup mapping of the volume's kernels; results do not depend on it
 * (bit for bit), only speed does.  Defaults: {4, 16, 8, 8, 0} (the fastest
 * of a sweep on the 8 mm room sequence, MI355X). */
typedef struct vm_launch {
  int32_t wave_group_size;    /* waves per workgroup of the kernels that give
                                 each block one wave (classification,
                                 vertices, triangles): 2, 4 or 8 */
  int32_t wave_groups_per_cu; /* their workgroups per compute unit, 1..32 */
  int32_t block_groups_per_cu;/* workgroups per compute unit of the kernels
                                 that give each block a 512-lane workgroup
                                 (fusion, import, backward), 1..16 */
  int32_t item_groups_per_cu; /* workgroups per compute unit of the list
                                 kernels (256 lanes), 1..32 */
  int32_t block_order;        /* bit 0 clear: block i goes to workgroup
                                 i mod grid; set: each workgroup takes a
                                 contiguous run.  Bit 1 set: the list is
                                 first cut into 8 contiguous ranges, one
                                 per XCD (workgroup b runs on XCD b mod
                                 8), so that neighbouring list entries
                                 share an L2.  0..3 */
} vm_launch;

/* Set / read the mapping.  VM_ERR_ARG for values outside the ranges. */
int vm_set_launch(vm_volume* vol, const vm_launch* launch);
int vm_get_launch(vm_volume* vol, vm_launch* launch);

/* Pool indices of blocks by coordinate, one hash lookup each (the O(1)
 * access of Sec. IV).  coords: device n*3 int32; idx: device n int32,
 * receives the block's row in pool order (as in vm_export_blocks and the
 * gradient arrays) or -1 when the block is not allocated. */
int vm_lookup_blocks(vm_volume* vol, const int32_t* coords, int32_t* idx, int64_t n,
                     hipStream_t stream);

/* Synchronise `stream` and report counters and the sticky device error. */
int vm_get_status(vm_volume* vol, vm_status* out, hipStream_t stream);

/* Inspection (synchronising).  vm_export_blocks writes, for the first
 * min(cap, blocks) pool entries, their coordinates (coords: host int32
 * cap*3) and, when non-NULL, device arrays tsdf/weight (cap*512 FP32) and
 * type_prev/type_cur (cap*512 uint8).  *n receives the block count. */
int vm_export_blocks(vm_volume* vol, int32_t* coords, float* tsdf,
                     float* weight, uint8_t* type_prev, uint8_t* type_cur,
                     int64_t cap, int64_t* n, hipStream_t stream);

/* Raw vertex pool (device outputs, cap entries each): edge key, t and
 * reference count (-1 marks a recycled slot).  *n receives the pool's
 * high-water mark. */
int vm_export_vertices(vm_volume* vol, uint64_t* edge_keys, float* t,
                       int32_t* refcount, int64_t cap, int64_t* n,
                       hipStream_t stream);

/* Block lists (host int32 cap*3 coordinates): which = 0 blocks collected by
 * the last integrate/import, 1 blocks classified by the last
 * extraction/refinement, 2 blocks touched since the last extraction. */
int vm_export_block_list(vm_volume* vol, int which, int32_t* coords,
                         int64_t cap, int64_t* n, hipStream_t stream);

/* Running totals (see VM_TOTAL_*): out[n] receives the first n of them.
 * Synchronises `stream`. */
int vm_get_totals(vm_volume* vol, int64_t* out, int n, hipStream_t stream);

/* Kernel timing for benchmarks.  While enabled, each kernel launch of the
 * volume records its start and end in two HIP events on its stream, set by
 * the launch itself (hipExtLaunchKernel; events are created by the library
 * on first use and reused).  vm_profile(vol, 1) clears previous records;
 * vm_profile_read synchronises the recorded events and writes, per VM_K_*
 * kernel, the launch count and the summed start-to-end milliseconds
 * (arrays of VM_K_COUNT entries, host).  vm_profile_mask records only the
 * kernels whose bit (1 << VM_K_*) is set in mask (0 stops recording), so
 * that timing one kernel touches that kernel's launches alone.  Launches on
 * a stream under graph capture are not timed. */
int vm_profile(vm_volume* vol, int enable);
int vm_profile_mask(vm_volume* vol, uint32_t mask);
int vm_profile_read(vm_volume* vol, int64_t* launches, double* ms);

#ifdef __cplusplus
}
#endif

#endif /* VOXMESH_H */
