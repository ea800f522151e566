"""Benchmark: incremental hashed-TSDF meshing on one MI355X.

A step is one pass of the hot path over the depth-fusion workload: the
100-frame synthetic room sequence (640x480 depth, 8 mm voxels, 2^20 hash
slots) fused and meshed frame by frame (integrate + extract + gc) into a
volume that starts empty.  The reported value is fused frames per second
over the timed steps, with every depth frame already resident in HBM.

Prints one JSON line.  Beside the headline value it reports:
  - the roofline of the dominant kernel, timed with HIP events that its
    launches inside the timed region record at their start and end (the
    launch records them itself: hipExtLaunchKernel), on the bytes the method must
    move per unit of work (`algorithmic_bytes`), with the bytes the kernel
    itself reads and writes beside them;
  - the whole frame (fusion + extraction + garbage collection) against the
    same peak, and blocks meshed per second;
  - the single-sphere extraction (512 blocks, blocks meshed per second);
  - the 4 mm sequence with holes and refinement (frames per second);
  - differentiable extraction of the 128^3 scene (forward + backward time);
  - batched forward + backward over 64 sphere volumes in one graph launch
    (blocks per second) against the same steps volume by volume;
  - the CPU oracle timed on a bounded sample of the headline sequence.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0

# HBM bytes per launch from hardware counters (rocprofv3 --pmc FETCH_SIZE, then
# WRITE_SIZE, KiB per dispatch averaged over one pass of this workload; the
# summaries and commands are in profiles/).  FETCH_SIZE read 131088.19 KiB
# for a 256 MiB device copy, WRITE_SIZE 262144 KiB: the factors below scale
# the counters to bytes.  Each entry holds the hash of its kernel's source
# when the counters were taken; a kernel changed since reports no traffic.
COUNTER_SCALE = {"fetch": 262144 / 131088.1875, "write": 1.0}
MEASURED_TRAFFIC = {
    "collect": {"fetch_kib": 1525.4, "write_kib": 1606.5, "source_sha1": "ae25bb272f48"},
    "fuse": {"fetch_kib": 12003.7, "write_kib": 13602.3, "source_sha1": "2f4eb3ca2b89"},
    "classify": {"fetch_kib": 3633.4, "write_kib": 3249.7, "source_sha1": "45183c9ad8c4"},
    "vertices": {"fetch_kib": 8678.7, "write_kib": 8507.0, "source_sha1": "e9287b86bfa5"},
}


def kernel_source_sha1(kernel: str) -> str:
    """Hash of the text of kernel k_<kernel> in the library's kernel source."""
    import hashlib
    import re
    path = os.path.join(ROOT, "paper_1803_03949_amd", "csrc", "vm_kernels.hip")
    src = open(path).read()
    m = re.search(r"void k_" + kernel + r"\(", src)
    if m is None:
        return ""
    a = src.rfind("\n", 0, m.start()) + 1
    b = src.index("\n}\n", m.start()) + 3
    return hashlib.sha1(src[a:b].encode()).hexdigest()[:12]


def measured_traffic(kernel: str):
    """HBM bytes per launch of the kernel as counted, or None when the
    counters predate the kernel's current source."""
    m = MEASURED_TRAFFIC.get(kernel)
    if m is None or kernel_source_sha1(kernel) != m["source_sha1"]:
        return None
    return int(1024 * (m["fetch_kib"] * COUNTER_SCALE["fetch"] +
                       m["write_kib"] * COUNTER_SCALE["write"]))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def render_frames(seq, ks, workers):
    if workers <= 1:
        return [seq.frame(k) for k in ks]
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(workers) as ex:
        return list(ex.map(seq.frame, ks))


def algorithmic_bytes(tot, npix, refine=False):
    """Bytes the method must move for the work in `tot` (differences of the
    device's running totals), per kernel and per step, from per-unit
    figures: fusion 4*W*H per frame (the depth image, charged to
    collection, which reads it first) + 8192 per collected block (TSDF and
    weight read and written); extraction 4096 per dirty block (TSDF and
    weight) + 1024 (t_{i-1} and t_i read and written), 20 per new or updated
    vertex, 12 per new triangle and 8 per changed triangle (new or dropped:
    its reference counts move); garbage collection 8 per freed vertex.
    Halo re-reads, hash probes and list bookkeeping are excluded.  The
    triangle terms belong to no kernel here: a cube's type is its triangle
    record, so no kernel writes triangles; the step total keeps them, as
    the method's figure.  With refine, every extraction was followed by one
    refinement over the same dirty blocks, charged 3072 per block (TSDF read,
    types read and written) to the refinement pass."""
    dirty = tot["dirty_blocks"] // 2 if refine else tot["dirty_blocks"]
    kernels = {
        "collect": 4 * npix * tot["frames"],
        "fuse": 8192 * tot["frame_blocks"],
        "classify": 5120 * dirty,
        "vertices": 20 * (tot["new_vertices"] + tot["updated_vertices"])
        + 8 * tot["freed_vertices"],
    }
    if refine:
        kernels["refine"] = 3072 * dirty
    triangles = 12 * tot["new_triangles"] + 8 * (tot["new_triangles"] + tot["dropped_triangles"])
    return kernels, sum(kernels.values()) + triangles


def touched_bytes(tot, npix, refine=False):
    """Bytes each kernel reads and writes by design (its own inputs and
    outputs, once each, halo re-reads excluded), the figure a kernel's
    speed of light is judged by: the vertex pass, for one, reads the types,
    TSDF and edge-vertex bits of every block it recomputes (2816 bytes),
    which the method's figure charges to classification alone, and writes
    t only for the kept vertices whose end points moved.  With refine, half the dirty-block total is the
    refinement's (TSDF, observed mask, both types read, types written)."""
    dirty = tot["dirty_blocks"] // 2 if refine else tot["dirty_blocks"]
    out = {
        "collect": 4 * npix * tot["frames"],
        "fuse": 4 * npix * tot["frames"] + 8192 * tot["frame_blocks"],
        "classify": 5632 * dirty,
        "vertices": 2816 * tot["vertex_blocks"] + 4 * tot["moved_vertices"]
        + 16 * tot["new_vertices"] + 12 * tot["freed_vertices"],
    }
    if refine:
        out["refine"] = 3648 * dirty
    return out


def frac(nbytes, ms):
    return nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS


def median_ms(fn, reps, warm=2):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        out.append(a.elapsed_time(b))
    return float(np.median(out))


def room_fusion(args, dev):
    """Headline workload; returns (fields of the JSON line, frames, seq)."""
    import torch

    import scenes
    from paper_1803_03949_amd import Volume

    seq = scenes.room_sequence(seed=2, n_frames=args.frames, voxel_m=0.008)
    t0 = time.time()
    frames = render_frames(seq, range(args.frames), args.workers)
    log(f"rendered {args.frames} frames in {time.time() - t0:.1f}s")
    depth = torch.from_numpy(np.stack(frames)).to(dev)
    poses = list(seq.poses)
    vol = Volume(seq.voxel_m, hash_log2=20, max_blocks=1 << 17, max_vertices=1 << 23, device=dev)

    def step():
        vol.reset()
        for k in range(args.frames):
            vol.integrate(depth[k], scenes.K, poses[k], seq.min_depth, seq.max_depth)
            vol.extract()
            vol.gc()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    npix = depth.shape[1] * depth.shape[2]

    # profiling pass: every kernel timed, to find the dominant one
    tot0 = vol.totals()
    vol.profile(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    vol.profile(False)
    prof = vol.profile_read()
    tot = {k: v - tot0[k] for k, v in vol.totals().items()}
    algo, _ = algorithmic_bytes(tot, npix)
    touched = touched_bytes(tot, npix)
    kernels = {}
    for k, (n, ms) in prof.items():
        e = {"launches": n, "ms_total": round(ms, 4), "us_per_launch": round(1000 * ms / n, 3)}
        if k in algo and ms > 0:
            e["bytes_per_launch"] = algo[k] // max(n, 1)
            e["GBps"] = round(algo[k] / (ms * 1e-3) / 1e9, 2)
            e["frac"] = round(frac(algo[k], ms), 5)
            e["touched_bytes_per_launch"] = touched[k] // max(n, 1)
            e["touched_frac"] = round(frac(touched[k], ms), 5)
            e["hbm_bytes_per_launch"] = measured_traffic(k)
        kernels[k] = e
    dom = max((k for k in kernels if k in algo), key=lambda k: kernels[k]["ms_total"])

    # timed region: K steps, events around the dominant kernel's launches only
    tot0 = vol.totals()
    vol.profile(True, kernels=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    vol.profile(False)
    n_dom, ms_dom = vol.profile_read()[dom]
    tot = {k: v - tot0[k] for k, v in vol.totals().items()}
    algo, step_total = algorithmic_bytes(tot, npix)
    bytes_dom = algo[dom]
    achieved = bytes_dom / (ms_dom * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2),
                "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                "traffic": measured_traffic(dom), "bytes_per_launch": bytes_dom // max(n_dom, 1),
                "us_per_launch": round(1000 * ms_dom / n_dom, 3),
                "touched_bytes_per_launch": touched_bytes(tot, npix)[dom] // max(n_dom, 1),
                "touched_frac": frac(touched_bytes(tot, npix)[dom], ms_dom)}
    # the whole frame (fusion + extraction + GC) against the same peak
    frame = {"bytes_per_frame": step_total // (args.frames * args.steps),
             "us_per_frame": 1e6 * dt / (args.frames * args.steps),
             "frac": frac(step_total, 1e3 * dt)}
    fps = args.frames * args.steps / dt

    # the same steps without any event
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    fps_noev = args.frames * args.steps / (time.perf_counter() - t0)
    st = vol.status()
    log(f"{fps:.1f} frames/s ({fps_noev:.1f} without events), blocks {st['blocks']}")

    # the same step captured once as a HIP graph (poses and frame numbers
    # baked into its launches) and replayed: what launching costs per frame
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            step()
    torch.cuda.current_stream().wait_stream(side)
    graph.replay()
    torch.cuda.synchronize()
    st_g = vol.status()
    reps = max(args.steps, 3)
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    dt_g = time.perf_counter() - t0
    # the pool slots a block's vertices take depend on the order blocks were
    # numbered in, so compare blocks, triangles and live vertices
    same = (st_g["blocks"] == st["blocks"] and st_g["triangles"] == st["triangles"] and
            st_g["vertex_slots"] - st_g["free_vertex_slots"] ==
            st["vertex_slots"] - st["free_vertex_slots"])
    graph_fields = {"frames_per_s": args.frames * reps / dt_g,
                    "us_per_frame": 1e6 * dt_g / (args.frames * reps), "replays": reps,
                    "same_mesh_counts": same}
    log(f"graph replay: {graph_fields}")
    del graph
    for k, e in sorted(kernels.items(), key=lambda kv: -kv[1]["ms_total"]):
        log(f"  {k:10s} {e}")
    fields = {"value": fps, "ms_per_step": 1000.0 * dt / args.steps, "roofline": roofline,
              "frame": frame, "value_without_events": fps_noev, "graph_replay": graph_fields,
              "blocks": st["blocks"],
              "blocks_meshed_per_s": tot["dirty_blocks"] / dt,
              "totals_per_step": {k: v // args.steps for k, v in tot.items()},
              "kernels": kernels}
    del vol
    return fields, frames, seq


def mesh_memory(args, dev, frames, seq):
    """Mesh size over the 8 mm room sequence (Sec. VI-B, Table I): live
    vertices V and triangles F every 10 frames, against a triangle soup that
    stores three vertices per triangle (the comparison the paper draws), and
    the bytes per cube of this layout."""
    import ctypes

    import torch

    import scenes
    from paper_1803_03949_amd import Volume, binding

    depth = torch.from_numpy(np.stack(frames)).to(dev)
    vol = Volume(seq.voxel_m, hash_log2=20, max_blocks=1 << 17, max_vertices=1 << 23, device=dev)
    series = []
    for k in range(len(frames)):
        vol.integrate(depth[k], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        vol.extract()
        vol.gc()
        if (k + 1) % 10 == 0 or k + 1 == len(frames):
            st = vol.status()
            nv = st["vertex_slots"] - st["free_vertex_slots"]
            series.append({"frame": k + 1, "blocks": st["blocks"], "vertices": nv,
                           "triangles": st["triangles"], "soup_vertices": 3 * st["triangles"]})

    # bytes per block and per vertex of capacity, from the workspace sizing
    def ws(**kw):
        c = dict(voxel_m=0.008, trunc_vox=4.0, refine_eps_vox=0.5, hash_log2=20,
                 max_blocks=1 << 17, max_vertices=1 << 23, hash_mode=0, batch_volumes=0)
        c.update(kw)
        n = ctypes.c_size_t()
        binding.lib().vm_volume_bytes(ctypes.byref(binding.vm_config(**c)), ctypes.byref(n))
        return n.value
    per_block = (ws(max_blocks=(1 << 17) + 4096) - ws()) / 4096
    per_vertex = (ws(max_vertices=(1 << 23) + 65536) - ws()) / 65536
    last = series[-1]
    in_use = last["blocks"] * per_block + last["vertices"] * per_vertex
    # vertex normals of the final mesh (download first: they follow its rows)
    verts, _, _ = vol.download(with_keys=False)
    normals_ms = median_ms(vol.download_normals, 20)
    assert len(vol.download_normals()) == len(verts)
    out = {"series": series, "vertices": last["vertices"], "triangles": last["triangles"],
           "soup_vertices": last["soup_vertices"],
           "soup_over_shared": last["soup_vertices"] / max(1, last["vertices"]),
           "triangles_per_vertex": last["triangles"] / max(1, last["vertices"]),
           "bytes_per_block": per_block, "bytes_per_cube": per_block / 512,
           "bytes_per_vertex": per_vertex, "in_use_MB": in_use / 1e6,
           "paper_bytes_per_cube": {"as_built": 56, "minimised": 24},
           "normals_ms": normals_ms, "normals_per_s": len(verts) / normals_ms * 1e3}
    log(f"mesh memory: V {last['vertices']}, F {last['triangles']}, soup 3F "
        f"{last['soup_vertices']} ({out['soup_over_shared']:.2f}x V), "
        f"{out['bytes_per_cube']:.1f} B per cube of capacity; normals of {len(verts)} vertices in "
        f"{normals_ms:.3f} ms")
    del vol, depth
    torch.cuda.empty_cache()
    return out


def sharing_ablation(args, dev, frames, seq, vertices_us):
    """The paper's two vertex-sharing schemes (Sec. V-C; compared in Sec. VI-A)
    over the 8 mm room sequence, each with its own vertex state kept across
    frames, timed per frame with events, beside edge ownership (the vertex
    pass of the headline, which also forms counts and frees vertices)."""
    import torch

    import scenes
    from paper_1803_03949_amd import Volume

    depth = torch.from_numpy(np.stack(frames)).to(dev)
    vol = Volume(seq.voxel_m, hash_log2=20, max_blocks=1 << 17, max_vertices=1 << 23, device=dev)
    n = (1 << 17) * 3 * 512
    states = [(torch.full((n,), -1, dtype=torch.int32, device=dev),
               torch.zeros(n, dtype=torch.float32, device=dev),
               torch.zeros(1, dtype=torch.int32, device=dev)) for _ in range(2)]
    ev = [[], []]
    for k in range(len(frames)):
        vol.integrate(depth[k], scenes.K, seq.poses[k], seq.min_depth, seq.max_depth)
        vol.extract()
        vol.gc()
        for scheme in (0, 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            vol.sharing_ablation(scheme, *states[scheme])
            b.record()
            ev[scheme].append((a, b))
    torch.cuda.synchronize()
    us = [1000.0 * float(np.mean([a.elapsed_time(b) for a, b in e])) for e in ev]
    (s0, t0, c0), (s1, t1, c1) = states
    same = bool(torch.equal(s0 >= 0, s1 >= 0)) and bool(torch.equal(t0[s0 >= 0], t1[s1 >= 0]))
    out = {"lock_based_us_per_frame": us[0], "lock_free_us_per_frame": us[1],
           "lock_free_over_lock_based": us[1] / us[0],
           "edge_ownership_vertex_pass_us": vertices_us,
           "vertices_initialised": int(c0.item()), "same_vertices_and_t": same}
    log(f"sharing ablation: lock-based {us[0]:.1f} us, lock-free {us[1]:.1f} us per frame "
        f"({us[1] / us[0]:.2f}x), edge ownership vertex pass {vertices_us:.1f} us; same {same}")
    del vol, depth, states
    torch.cuda.empty_cache()
    return out


def sphere_extract(dev):
    import torch

    import scenes
    from paper_1803_03949_amd import Volume

    sv = scenes.sphere_volume(seed=1)
    coords, d, w = sv.blocks()
    cdev = [torch.from_numpy(a).to(dev) for a in (coords, d, w)]
    vol = Volume(sv.voxel_m, hash_log2=16, max_blocks=1024, max_vertices=1 << 20, device=dev)
    times = []
    for rep in range(110):
        vol.reset()
        vol.import_blocks(*cdev)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        vol.extract(scope_all=True)
        b.record()
        torch.cuda.synchronize()
        if rep >= 10:
            times.append(a.elapsed_time(b))
    ms = float(np.median(times))
    return {"blocks_per_s": 512 / (ms / 1000.0), "extract_ms": ms}


def room_fine(args, dev):
    """4 mm, holes, refinement at every extraction: as a separate pass after
    it, and applied inside it to each new type."""
    import torch

    import scenes

    seq = scenes.room_sequence(seed=3, n_frames=args.fine_frames, voxel_m=0.004, holes=True)
    t0 = time.time()
    frames = render_frames(seq, range(args.fine_frames), args.workers)
    log(f"rendered {args.fine_frames} 4 mm frames in {time.time() - t0:.1f}s")
    depth = torch.from_numpy(np.stack(frames)).to(dev)
    poses = list(seq.poses)
    del frames
    out = fine_pass(args, seq, depth, poses, dev, fused=False)
    out["refining_extraction"] = fine_pass(args, seq, depth, poses, dev, fused=True)
    del depth
    torch.cuda.empty_cache()
    return out


def fine_pass(args, seq, depth, poses, dev, fused):
    """The 4 mm sequence on resident depth frames: each frame integrate,
    extract and gc, with a refinement pass after the extraction, or (fused)
    the refinement applied to each new type inside the extraction."""
    import torch

    import scenes
    from paper_1803_03949_amd import Volume

    vol = Volume(seq.voxel_m, hash_log2=22, max_blocks=1 << 19, max_vertices=1 << 24, device=dev)

    def step():
        vol.reset()
        for k in range(args.fine_frames):
            vol.integrate(depth[k], scenes.K, poses[k], seq.min_depth, seq.max_depth)
            vol.extract(refine=fused)
            if not fused:
                vol.refine()
            vol.gc()

    step()
    torch.cuda.synchronize()
    tot0 = vol.totals()
    t0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tot = {k: v - tot0[k] for k, v in vol.totals().items()}
    st = vol.status()
    # one more pass with every kernel timed: per-kernel rates
    # against algorithmic bytes
    vol.profile(True)
    step()
    torch.cuda.synchronize()
    vol.profile(False)
    prof = vol.profile_read()
    npix = depth.shape[1] * depth.shape[2]
    algo, step_total = algorithmic_bytes(tot, npix, refine=not fused)
    touched = touched_bytes(tot, npix, refine=not fused)
    kernels = {}
    for k, (n, ms) in prof.items():
        e = {"launches": n, "us_per_launch": round(1000 * ms / n, 3)}
        if k in algo and ms > 0:
            e["bytes_per_launch"] = algo[k] // max(n, 1)
            e["GBps"] = round(algo[k] / (ms * 1e-3) / 1e9, 2)
            e["frac"] = round(frac(algo[k], ms), 5)
            e["touched_bytes_per_launch"] = touched[k] // max(n, 1)
            e["touched_frac"] = round(frac(touched[k], ms), 5)
        kernels[k] = e
    out = {"frames_per_s": args.fine_frames / dt, "ms_per_frame": 1000 * dt / args.fine_frames,
           "frames": args.fine_frames, "blocks": st["blocks"],
           "blocks_meshed_per_s": (tot["dirty_blocks"] if fused else tot["dirty_blocks"] // 2) / dt,
           "refined_cubes": tot["refined_cubes"], "totals": tot,
           "frame": {"bytes_per_frame": step_total // args.fine_frames,
                     "us_per_frame": 1e6 * dt / args.fine_frames,
                     "frac": frac(step_total, 1e3 * dt)},
           "kernels": kernels}
    what = "refining extraction" if fused else "extraction + refinement pass"
    log(f"4 mm, {what}: {out['frames_per_s']:.1f} frames/s, blocks {st['blocks']}")
    for k, e in sorted(kernels.items(), key=lambda kv: -kv[1]["us_per_launch"] * kv[1]["launches"]):
        log(f"  {k:10s} {e}")
    del vol
    torch.cuda.empty_cache()
    return out


def grad_scene_fwd_bwd(dev):
    import torch

    import scenes
    from paper_1803_03949_amd import Volume
    from paper_1803_03949_amd.autograd import FusedMesh

    gs = scenes.grad_scene(seed=4)
    coords, d, w = gs.volume.blocks()
    vol = Volume(gs.volume.voxel_m, hash_log2=16, max_blocks=1 << 14, max_vertices=1 << 21, device=dev)
    cd, td, wd = (torch.from_numpy(a).to(dev) for a in (coords, d, w))
    dd = torch.from_numpy(gs.depth).to(dev)
    (c0, r0) = gs.target.spheres[0]
    c0 = torch.tensor(c0, device=dev, dtype=torch.float32)

    def fwd_bwd():
        dt_ = dd.clone().requires_grad_(True)
        t_ = td.clone().requires_grad_(True)
        verts, tris, keys = FusedMesh.apply(dt_, t_, wd, cd, vol, scenes.K, gs.pose, 0.1, 10.0)
        L = ((torch.linalg.norm(verts - c0, dim=1) - r0) ** 2).sum()
        L.backward()
        return verts.shape[0]

    nv = fwd_bwd()
    ms = median_ms(fwd_bwd, 20)
    return {"fwd_bwd_ms": ms, "blocks": int(len(coords)), "vertices": int(nv),
            "note": "includes the host synchronisation of the mesh download"}


def batch_workload(dev):
    """The 64 sphere volumes of the batched workload, on the device."""
    import torch

    import scenes

    t0 = time.time()
    vols = scenes.batch_volumes(seed=5, n=64, voxel_m=0.008)
    coords, ds, ws = [], [], []
    for v in vols:
        c, d, w = v.blocks()
        coords.append(c)
        ds.append(d)
        ws.append(w)
    sizes = [len(c) for c in coords]
    tsdf = torch.from_numpy(np.concatenate(ds)).to(dev)
    weight = torch.from_numpy(np.concatenate(ws)).to(dev)
    del ds, ws
    centers = torch.tensor(np.stack([v.meta["center"] for v in vols]), dtype=torch.float32,
                           device=dev)
    radii = torch.tensor([v.meta["target_radius"] for v in vols], dtype=torch.float32,
                         device=dev)
    log(f"64 volumes, {sum(sizes)} blocks (sizes {min(sizes)}..{max(sizes)}), built in "
        f"{time.time() - t0:.1f}s")
    return coords, tsdf, weight, centers, radii


def batch_step_bytes(tot):
    """Bytes the batched forward + backward must move per step, from
    per-unit figures: the extraction of every block (as for a
    frame) and the backward, 12 per vertex (dL/dv) + 4096 per block (TSDF
    and edge reads) + 2048 per block (dL/dTSDF written)."""
    f_new, f_drop = tot["new_triangles"], tot["dropped_triangles"]
    extract = (5120 * tot["dirty_blocks"] + 20 * (tot["new_vertices"] + tot["updated_vertices"])
               + 12 * f_new + 8 * (f_new + f_drop) + 8 * tot["freed_vertices"])
    backward = 12 * tot["new_vertices"] + 6144 * tot["frame_blocks"]
    return extract + backward


def batched(args, dev):
    import torch

    from paper_1803_03949_amd.batch import (BatchMesher, PlainMesher, autotune,
                                            default_space, sphere_loss_grad)

    coords, tsdf, weight, centers, radii = batch_workload(dev)
    sizes = [len(c) for c in coords]
    N = int(sum(sizes))
    b = BatchMesher(0.008, coords, tsdf, weight, sphere_loss_grad(centers, radii))
    space = default_space() if args.tune_full else \
        [p for p in default_space() if p["block_groups_per_cu"] == 8]
    tune = autotune(b, space=space, reps=5, log=log)
    tot0 = b.vol.totals()
    batch_ms = median_ms(b.replay, args.batch_reps)
    tot = {k: (v - tot0[k]) // (args.batch_reps + 2) for k, v in b.vol.totals().items()}
    step_bytes = batch_step_bytes(tot)
    # the library's own graphs (vm_extract_batch), the loss between them
    lib_ms = median_ms(b.step, args.batch_reps)
    default_launch = dict(wave_group_size=4, wave_groups_per_cu=16, block_groups_per_cu=8,
                          item_groups_per_cu=8, block_order=0)
    b.set_launch(**default_launch)
    b.capture()
    default_ms = median_ms(b.replay, args.batch_reps)
    b.set_launch(**tune["launch"])
    b.capture()
    b.replay()
    torch.cuda.synchronize()
    grad_b = b.grad.clone()

    p = PlainMesher(0.008, coords, tsdf, weight,
                    [sphere_loss_grad(centers[i:i + 1], radii[i:i + 1]) for i in range(64)])
    plain_ms = median_ms(p.run, args.batch_reps)
    identical = bool(torch.equal(p.grad(), grad_b))
    # the per-volume sequence captured in one graph too (launch overhead removed)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        p.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        p.run()
    plain_graph_ms = median_ms(g.replay, args.batch_reps)
    out = {
        "volumes": 64, "blocks": N, "sizes": sizes,
        "batched_blocks_per_s": N / (batch_ms / 1000), "batched_ms": batch_ms,
        "library_graphs_ms": lib_ms,
        "batched_default_mapping_ms": default_ms,
        "plain_blocks_per_s": N / (plain_ms / 1000), "plain_ms": plain_ms,
        "plain_graph_ms": plain_graph_ms,
        "speedup_vs_plain": plain_ms / batch_ms,
        "speedup_vs_plain_graph": plain_graph_ms / batch_ms,
        "identical_to_plain": identical,
        "tuned_launch": tune["launch"], "tune_points": tune.get("points"),
        "tune_cached": tune.get("cached"), "replays_timed": args.batch_reps,
        "step": {"bytes_per_step": step_bytes, "frac": frac(step_bytes, batch_ms),
                 "vertices": tot["new_vertices"]},
    }
    log(f"batched fwd+bwd {batch_ms:.3f} ms ({out['batched_blocks_per_s']:.3e} blocks/s; "
        f"{lib_ms:.3f} ms with the library's graphs), "
        f"plain {plain_ms:.3f} ms, plain graph {plain_graph_ms:.3f} ms, identical {identical}")
    del b, p, g
    torch.cuda.empty_cache()
    return out


def batched_replays(args, dev):
    """The batched step alone (default mapping, graph replays), for profiling."""
    import torch

    from paper_1803_03949_amd.batch import BatchMesher, sphere_loss_grad

    coords, tsdf, weight, centers, radii = batch_workload(dev)
    b = BatchMesher(0.008, coords, tsdf, weight, sphere_loss_grad(centers, radii))
    b.capture()
    ms = median_ms(b.replay, args.batch_reps)
    n = int(sum(len(c) for c in coords))
    log(f"batched fwd+bwd {ms:.3f} ms ({n / ms * 1e3:.3e} blocks/s), default mapping")
    return {"batched_ms": ms, "blocks": n, "batched_blocks_per_s": n / ms * 1e3}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(frames, seq, budget_s=20.0, single_budget_s=12.0):
    """The oracle on the host cores over the headline sequence from its first
    frame, integrate + extract + gc per frame, until a time budget is spent:
    threads over blocks on every core the host gives (at most 16), then a
    single thread.  The oracle's results do not depend on its thread
    count."""
    import oracle
    import scenes

    threads = min(16, os.cpu_count() or 1)
    legs = {}
    for name, thr, budget in (("threads", threads, budget_s), ("single", 1, single_budget_s)):
        o = oracle.OracleVolume(seq.voxel_m, threads=thr, keep_fusion=False)
        n = 0
        c0 = time.perf_counter()
        while n < len(frames) and time.perf_counter() - c0 < budget:
            o.integrate(frames[n], scenes.K, seq.poses[n], seq.min_depth, seq.max_depth)
            o.extract()
            o.gc()
            n += 1
        cdt = time.perf_counter() - c0
        legs[name] = {"frames": n, "seconds": round(cdt, 3), "frames_per_s": n / cdt,
                      "threads": thr}
        log(f"cpu oracle, {thr} threads: {n} frames in {cdt:.1f}s ({n / cdt:.3f} frames/s)")
        del o
    t = legs["threads"]
    return {"value": t["frames_per_s"], "unit": "frames/s", "cores": threads, "kind": "oracle",
            "sample": f"first {t['frames']} frames of the same 8 mm room sequence, integrate + "
                      f"extract + gc per frame, {threads} threads (about {budget_s:.0f} s of "
                      "work)",
            "single_thread": legs["single"], "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--frames", type=int, default=100)
    ap.add_argument("--fine-frames", type=int, default=500)
    ap.add_argument("--batch-reps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline workload only (for profiling runs)")
    ap.add_argument("--tune-full", action="store_true")
    ap.add_argument("--only", choices=["batch", "fine"],
                    help="profiling: run only this workload (batch: graph replays of the 64 "
                         "volumes with the default mapping; fine: the 4 mm sequence) and print "
                         "its figures")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a kernel of "
                         "known traffic, to calibrate hardware byte counters)")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the method has no multi-GPU path here "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "no GPU"
    dev = torch.device("cuda:0")
    if args.copy_probe_mib:
        n = args.copy_probe_mib << 18
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + written")
        del a, b
    if args.only == "batch":
        print(json.dumps(batched_replays(args, dev)))
        return
    if args.only == "fine":
        print(json.dumps(room_fine(args, dev)))
        return
    head, frames, seq = room_fusion(args, dev)
    extras = {}
    if not args.no_extras:
        extras["mesh_memory_8mm"] = mesh_memory(args, dev, frames, seq)
        extras["sharing_ablation_8mm"] = sharing_ablation(
            args, dev, frames, seq, head["kernels"]["vertices"]["us_per_launch"])
        extras["sphere_512_blocks"] = sphere_extract(dev)
        log(f"sphere: {extras['sphere_512_blocks']}")
        extras["grad_scene_128"] = grad_scene_fwd_bwd(dev)
        log(f"grad scene: {extras['grad_scene_128']}")
        extras["batched_64_volumes"] = batched(args, dev)
        extras["room_4mm_holes_refine"] = room_fine(args, dev)
    cpu = None if args.no_cpu_baseline else cpu_baseline(frames, seq)

    out = {
        "metric": "fused frames/s @8mm (integrate + extract + gc per frame)",
        "value": head["value"],
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"room sequence, {args.frames} frames 640x480, 8 mm voxels, "
                               "8^3 blocks, 2^20 hash slots, integrate+extract+gc per frame"},
        "roofline": head["roofline"],
        "frame": head["frame"],
        "blocks_meshed_per_s": head["blocks_meshed_per_s"],
        "batched": ({k: extras["batched_64_volumes"][k] for k in
                     ("batched_blocks_per_s", "plain_blocks_per_s", "speedup_vs_plain", "step")}
                    if "batched_64_volumes" in extras else None),
        "cpu_baseline": cpu,
        "value_without_events": head["value_without_events"],
        "graph_replay": head["graph_replay"],
        "blocks": head["blocks"],
        "totals_per_step": head["totals_per_step"],
        "kernels": head["kernels"],
        "extras": extras,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
