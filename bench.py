"""Throughput benchmark of the MLS immersed-boundary transfer on one MI355X.

A step is one pass of the whole hot path over all markers of all bodies:
jitter (<= 0.1 h, counter-based) -> transfer-function build (exact MLS by
default) -> interpolation of u, v, w -> direct forcing F = (V_b - U)/dt ->
conservative spreading into the forcing fields.  Default workload: 10,000
bodies of 320/1280/5120 surface markers (22.66 M markers) in a periodic
1024^3 staggered grid, one launch per phase over all bodies, the step
captured once as a HIP graph and replayed.

Prints ONE JSON line on stdout (progress goes to stderr):
  value     markers/s over the timed graph replays (inputs resident in HBM)
  roofline  dominant kernel: algorithmic bytes per launch / average duration
            (HIP events around each launch in a timed eager pass)
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same markers
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash():
    """SHA-256 over the HIP sources and headers of the library (the counter
    summaries under profiles/ name the sources they were measured on)."""
    from paper_1805_01113_amd import build
    return build.source_sha256()


def measured_traffic(kernel, workload, step):
    """HBM bytes per launch of `kernel` from the rocprofv3 counter summary in
    profiles/ (FETCH_SIZE and WRITE_SIZE scaled by the factors a plain device
    copy reads for them), or None if there is none for the current sources,
    this workload and this step (method and transfer-function form: the same
    timing label covers different kernels in other steps)."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_sha256") != source_hash() or d.get("workload") != workload or d.get("step") != step:
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else int(k["traffic_bytes_per_launch"])


def make_workload(name):
    from paper_1805_01113_amd import workloads as W
    if name == "uneven":
        return W.uneven_bodies()
    if name == "ellipsoids":
        return W.ellipsoids()
    if name == "stretched":
        return W.stretched_channel()
    if name == "sphere":
        return W.single_sphere()
    if name == "contact":
        return W.contact_pairs()
    raise SystemExit("unknown workload %s" % name)


def touched_nodes(torch, ctx, home, n, footprint=None):
    """Unique (component, node) pairs in the supports of all markers (for the
    algorithmic bytes of interpolation and spreading).  If footprint is a
    dict, it also receives the unique 32-byte sectors, 64-byte and 128-byte
    lines of the FP32 component fields that hold those nodes: the least a
    gather (or a read-modify-write) of the touched values moves at each
    memory access granularity."""
    from paper_1805_01113_amd import mls
    h = mls.unblock(home, n)[:, :, 0].to(torch.int64) & 0xFFFFFFFF
    total = 0
    sect = {32: 0, 64: 0, 128: 0}
    for c in range(3):
        nx, ny, nz = ctx.dims(c)
        mask = torch.zeros(nx * ny * nz, dtype=torch.bool, device=home.device)
        i = h[c] & 0x7FF
        j = (h[c] >> 11) & 0x7FF
        k = h[c] >> 22
        for dz in (-1, 0, 1):
            kk = (k + dz) % nz if ctx.periodic[2] else k + dz
            for dy in (-1, 0, 1):
                jj = (j + dy) % ny if ctx.periodic[1] else j + dy
                for dx in (-1, 0, 1):
                    ii = (i + dx) % nx if ctx.periodic[0] else i + dx
                    mask[(kk * ny + jj) * nx + ii] = True
        total += int(mask.sum().item())
        if footprint is not None:
            for b in sect:
                per = b // 4
                m = mask
                if m.numel() % per:
                    m = torch.cat([m, torch.zeros(per - m.numel() % per, dtype=torch.bool, device=m.device)])
                sect[b] += int(m.view(-1, per).any(dim=1).sum().item())
        del mask
    if footprint is not None:
        footprint.update({"nodes": total, "sectors_32B": sect[32], "lines_64B": sect[64], "lines_128B": sect[128]})
    return total


def cpu_baseline(wl, fields_dev, target_s):
    """The FP64 oracle (build + interp + spread, three components) on the first
    markers of the workload, sized to take about target_s seconds."""
    from oracle import oracle as orc
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(threads))
    orc.build()
    g = orc.Grid(wl.grid.faces, wl.grid.periodic)
    fields = [f.cpu().numpy() for f in fields_dev]

    def run(m):
        x, y, z = wl.x[:m], wl.y[:m], wl.z[:m]
        t0 = time.perf_counter()
        refs = [orc.build_exact(g, c, x, y, z) for c in range(3)]
        t1 = time.perf_counter()
        for c in range(3):
            orc.interp(g, c, refs[c]["home"], refs[c]["phi"], fields[c])
        t2 = time.perf_counter()
        for c in range(3):
            f = np.zeros(wl.grid.shape(c))       # pages touched lazily
            orc.spread(g, c, refs[c]["home"], refs[c]["phi"], wl.area[:m], wl.force[c, :m], f)
            del f
        t3 = time.perf_counter()
        return t3 - t0, (t1 - t0, t2 - t1, t3 - t2)

    m = min(wl.n, 20000)
    t, _ = run(m)
    # fixed costs weigh more on the small pilot, so the sample is sized again
    # from the first sized run when that one falls well short of the target
    for _ in range(2):
        m = int(min(wl.n, max(m, m * target_s / max(t, 1e-3))))
        t, parts = run(m)
        if t >= 0.6 * target_s or m == wl.n:
            break
    return {"value": m / t, "unit": "markers/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of %d markers (whole bodies in generation order), build+interp+spread, "
                      "3 components, FP64; build %.1fs interp %.1fs spread %.1fs" % (m, wl.n, *parts)}


METHODS = {"exact": 0, "fast": 1, "learned": 2, "fast_linear": 3}


def load_network(ctx, path):
    """Load the trained surrogate into ctx; None if no checkpoint is available."""
    from paper_1805_01113_amd import train_mlp
    path = path or train_mlp.DEFAULT_WEIGHTS
    if not os.path.exists(path):
        log("no surrogate checkpoint at %s: learned method skipped" % path)
        return None
    p, q, meta = train_mlp.load_weights(path)
    ctx.mlp_load(p, q)
    return {"path": os.path.relpath(path, ROOT), "trained": meta["config"], "held_out": meta["end"]}


def per_body_rate(torch, ctx, wl, bufs, fields, forcing, x0, y0, z0, area, method, jitter, seed, stream, sub):
    """markers/s of one mls_step per body (a host loop over bodies), same kernels."""
    import ctypes
    from paper_1805_01113_amd import mls
    offs = wl.body_offsets
    torch.cuda.synchronize()
    t_a = time.perf_counter()
    for b in range(sub):
        s, e = int(offs[b]), int(offs[b + 1])
        sb = mls._StepBuf()
        sb.n = e - s
        for key, t in (("x0", x0), ("y0", y0), ("z0", z0), ("x", bufs.x), ("y", bufs.y), ("z", bufs.z),
                       ("area", area)):
            setattr(sb, key, t.data_ptr() + 4 * s)
        sb.home = bufs.home.data_ptr()
        sb.phi = bufs.phi.data_ptr()
        sb.U = bufs.U.data_ptr()
        sb.F = bufs.F.data_ptr()
        sb.u, sb.v, sb.w = [f.data_ptr() for f in fields]
        sb.fx, sb.fy, sb.fz = [f.data_ptr() for f in forcing]
        d = mls._desc(method, 1.0, jitter, seed)
        st = ctx._lib.mls_step(ctx.h, ctypes.byref(d), ctypes.byref(sb), stream.cuda_stream)
        assert st == 0
    torch.cuda.synchronize()
    t_b = time.perf_counter()
    ctx.sync()
    return int(offs[sub]) / (t_b - t_a)


def byte_models(method, compact, nf, t_per, jitter_kernel):
    """Algorithmic bytes per marker of each timed kernel, two ways.

    contract: the hot-path contract's figures (transfer functions stored as 27
    FP32 values and read back): build 12 + 12 + 324 = 348, interpolation
    336 + 12 + 4T, spreading 336 + 12 + 4 + 8T (T = touched (component, node)
    pairs per marker); a fused kernel carries the sum of the phases it does.
    own: what this implementation's kernel has to move at least once (compact
    rows of nf floats for an exact step, c_l F_l by row, U and F by marker)."""
    tf = 4.0 * 3 * (nf if compact else 27)
    contract = {
        "build_exact": 348.0, "build_fast": 348.0,
        # the learned build of a time step interpolates and forces as well
        "build_learned": 348 + 336 + 12 + 4.0 * t_per,
        "interp": 336 + 12 + 4.0 * t_per,
        "build_interp": 348 + 336 + 12 + 4.0 * t_per,
        "fast_interp": 348 + 336 + 12 + 4.0 * t_per,
        "spread_tiles": 336 + 12 + 4 + 8.0 * t_per,
    }
    own = {
        "jitter": 24.0,
        "build_exact": 12 + 12 + 324.0, "build_fast": 12 + 12 + 324.0,
        # positions and area, homes, full rows, touched field values, U and F
        # by marker, c_l F_l by row
        "build_learned": 16 + 12 + 324 + 4.0 * t_per + 12 + 12 + 12,
        "interp": 12 + 324 + 12 + 4.0 * t_per,
        # positions and area, homes, transfer functions, touched field values,
        # U and F by marker, c_l F_l by row
        "build_interp": 16 + 12 + tf + 4.0 * t_per + 12 + 12 + 12,
        "fast_interp": 16 + 12 + 324 + 4.0 * t_per + 12 + 12 + 12,
        "force": 24.0,
        # homes, transfer functions, c_l F_l by row, read-modify-write of the
        # touched field values
        "spread_tiles": 12 + (tf if method == 0 else 324) + 12 + 8.0 * t_per,
        # positions (and the jitter's read and write when the binning does it)
        # the tile of each marker, the sorted marker list
        "spread_bin": (24.0 if jitter_kernel else 36.0) + 8.0,
    }
    return contract, own


def compare_methods(torch, ctx, wl, bufs, fields, forcing, x0, y0, z0, area, jitter, seed, args, ms_main,
                    main_method):
    """{per-body, batched} x {exact, fast, learned}: markers/s, and the
    interpolated velocity of each method against exact MLS on the same
    jittered positions (normwise: max |U - U_exact| / max |U_exact|)."""
    from paper_1805_01113_amd import mls
    stream = torch.cuda.current_stream()
    n = wl.n
    names = ["exact", "fast", "fast_linear"] + (["learned"] if ctx.mlp_loaded else [])
    sub = int(min(len(wl.body_offsets) - 1, 2000))
    # reference velocities: exact MLS at a fixed jitter counter
    probe_step = 1 << 20
    ref = None
    out = {}
    for name in names:
        m = METHODS[name]
        mls.step_counter_set(ctx, probe_step)
        ctx.stats_reset()
        mls.step(ctx, bufs, method=m, dt=1.0, jitter=jitter, seed=seed)
        ctx.sync()
        st = ctx.stats()
        U = bufs.U.clone()
        if ref is None:
            ref = U
        err = float((U - ref).abs().max().item() / ref.abs().max().item())
        row = {"interp_err_vs_exact": err}
        if m == mls.MLS_LEARNED:
            tot = st["learned"] + st["fallbacks"]
            row["fallback_rate"] = st["fallbacks"] / max(1, tot)
            row["network_kept"] = st["learned"]
        saved = None
        if m == main_method:
            ms = ms_main
        else:
            if not args.no_tune:
                # each method with the launch shapes tuned for it
                saved = ctx.tune_get()
                ctx.autotune(bufs, method=m, cache_path=args.tune_cache)
                row["autotune"] = {k: v for k, v in ctx.tune_get().items()}
            g2 = mls.StepGraph(ctx, bufs, method=m, dt=1.0, jitter=jitter, seed=seed)
            g2.launch(args.warmup)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            g2.launch(args.steps)
            e1.record(stream)
            torch.cuda.synchronize()
            ctx.sync()
            ms = e0.elapsed_time(e1) / max(args.steps, 1)
            g2.close()
        row["batched"] = {"ms_per_step": round(ms, 4), "markers_per_s": round(n / (ms * 1e-3), 1)}
        rate = per_body_rate(torch, ctx, wl, bufs, fields, forcing, x0, y0, z0, area, m, jitter, seed, stream, sub)
        row["per_body"] = {"markers_per_s": round(rate, 1), "bodies_timed": sub}
        if saved is not None:
            ctx.tune_set(**{k: saved[k] for k in ("spread_tile", "spread_blocks_per_cu", "build_blocks_per_cu",
                                                 "interp_blocks_per_cu", "spread_threads")})
        log("%s: batched %.3f ms/step (%.3e markers/s), per-body %.3e markers/s, interp err vs exact %.2e%s"
            % (name, ms, n / (ms * 1e-3), rate, err,
               (", fallback rate %.4f" % row["fallback_rate"]) if "fallback_rate" in row else ""))
        out[name] = row
    return out


def config_matrix(torch, args, names=("sphere", "ellipsoids", "stretched")):
    """The other workloads of the hot path (one sphere on 64^3; 1,000
    ellipsoids on 512^3; 2,000 spheres in the tanh-stretched 512x512x768
    channel): every method's batched step (graph replays, autotuned shapes),
    its interpolation error against exact MLS on the same jittered positions,
    the learned method's fallback rate, and the dominant kernel's HBM
    fraction on the contract's bytes."""
    from paper_1805_01113_amd import mls
    from paper_1805_01113_amd import workloads as W
    out = {}
    stream = torch.cuda.current_stream()
    for name in names:
        t0 = time.time()
        wl = make_workload(name)
        n = wl.n
        x0, y0, z0 = [torch.from_numpy(a).cuda() for a in (wl.x, wl.y, wl.z)]
        area = torch.from_numpy(wl.area).cuda()
        fields = [W.fourier_field(wl.grid, c, wl.modes[c], wl.lengths, device="cuda") for c in range(3)]
        forcing = [torch.zeros(wl.grid.shape(c), dtype=torch.float32, device="cuda") for c in range(3)]
        ctx = mls.Context(wl.grid.faces, wl.grid.periodic)
        ctx.reserve(n)
        net = load_network(ctx, args.weights)
        bufs = mls.StepBuffers(ctx, x0, y0, z0, area, fields, forcing)
        nf = 7 if all(wl.grid.uniform_axis(d) for d in range(3)) else 13
        jitter = 0.1 * wl.grid.h_min
        seed = 20180503
        row = {"markers": n, "bodies": int(len(wl.body_offsets) - 1), "grid": list(wl.grid.n), "methods": {}}
        ref = None
        t_per = None
        names_m = ["exact", "fast", "fast_linear"] + (["learned"] if net is not None else [])
        for mname in names_m:
            m = METHODS[mname]
            compact = m == mls.MLS_EXACT
            if not args.no_tune:
                ctx.autotune(bufs, method=m, cache_path=args.tune_cache, compact=compact)
            # interpolation error against exact MLS at a fixed jitter counter
            mls.step_counter_set(ctx, 1 << 20)
            ctx.stats_reset()
            mls.step(ctx, bufs, method=m, dt=1.0, jitter=jitter, seed=seed, compact=compact)
            ctx.sync()
            U = bufs.U.clone()
            if ref is None:
                ref = U
                t_per = touched_nodes(torch, ctx, bufs.home, n) / n
            r = {"interp_err_vs_exact": float((U - ref).abs().max().item() / ref.abs().max().item())}
            if m == mls.MLS_LEARNED:
                st = ctx.stats()
                r["fallback_rate"] = st["fallbacks"] / max(1, st["learned"] + st["fallbacks"])
            g = mls.StepGraph(ctx, bufs, method=m, dt=1.0, jitter=jitter, seed=seed, compact=compact)
            g.launch(args.warmup)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            g.launch(args.steps)
            e1.record(stream)
            torch.cuda.synchronize()
            ctx.sync()
            ms = e0.elapsed_time(e1) / max(args.steps, 1)
            g.close()
            r["batched"] = {"ms_per_step": round(ms, 4), "markers_per_s": round(n / (ms * 1e-3), 1)}
            # per-kernel times of eager steps: the dominant kernel's roofline
            mls.timing_enable(ctx, True)
            mls.timing_get(ctx, reset=True)
            for _ in range(args.steps):
                mls.step(ctx, bufs, method=m, dt=1.0, jitter=jitter, seed=seed, compact=compact)
            torch.cuda.synchronize()
            kt = mls.timing_get(ctx, reset=True)
            mls.timing_enable(ctx, False)
            ctx.sync()
            contract, _ = byte_models(m, compact, nf, t_per, "jitter" in kt)
            times = {k: v[0] / v[1] for k, v in kt.items()}
            dom = max((k for k in times if contract.get(k)), key=lambda k: times[k])
            gbs = contract[dom] * n / (times[dom] * 1e-3) / 1e9
            r["kernels_ms"] = {k: round(v, 4) for k, v in times.items()}
            r["roofline"] = {"kernel": dom, "achieved": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                             "alg_bytes_per_marker": round(contract[dom], 1)}
            row["methods"][mname] = r
            log("%s %s: %.3f ms/step (%.3e markers/s), err vs exact %.2e, dominant %s %.1f%% of HBM"
                % (name, mname, ms, n / (ms * 1e-3), r["interp_err_vs_exact"], dom, 100 * gbs / HBM_PEAK_GBS))
        row["touched_nodes_per_marker"] = round(t_per, 3)
        row["seconds"] = round(time.time() - t0, 1)
        out[wl.name] = row
        ctx.close()
        del bufs, fields, forcing, x0, y0, z0, area, ref, U
        torch.cuda.empty_cache()
    return out


def collision_cost(torch, ctx, wl, x, y, z, steps, ms_step):
    """Coarse-grained collision detection on the step's markers: time of the
    detection (cell ids + flags) and of the O(n) clear that readies the cell
    array for the next step, against the step time."""
    from paper_1805_01113_amd import mls
    from paper_1805_01113_amd import workloads as W
    n = wl.n
    body = torch.from_numpy(W.body_ids(wl.body_offsets)).cuda()
    coll = torch.zeros(ctx.cell_shape(), dtype=torch.int32, device="cuda")
    flags = torch.empty(n, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    ctx.collide(x, y, z, body, coll, flags)
    cells = int(torch.count_nonzero(coll))
    shared = int((coll == -1).sum())
    ctx.collide_clear(x, y, z, coll)
    ctx.sync()
    mls.timing_enable(ctx, True)
    mls.timing_get(ctx, reset=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        ctx.collide(x, y, z, body, coll, flags)
        ctx.collide_clear(x, y, z, coll)
    e1.record(stream)
    torch.cuda.synchronize()
    ctx.sync()
    kt = mls.timing_get(ctx, reset=True)
    mls.timing_enable(ctx, False)
    ms = e0.elapsed_time(e1) / max(steps, 1)
    flagged = int(flags.sum())
    c = cells / n
    alg = {"collide": 12 + 4 + 8 * c + 12 + 4 * c + 1, "collide_clear": 12 + 4 * c}
    kern = {}
    for k, (t, cnt) in kt.items():
        avg = t / cnt
        kern[k] = {"avg_ms": round(avg, 4), "alg_bytes_per_marker": round(alg[k], 2),
                   "GBs": round(alg[k] * n / (avg * 1e-3) / 1e9, 1)}
    del coll
    return {"workload": wl.name, "ms_detect_and_clear": round(ms, 4), "markers_per_s": round(n / (ms * 1e-3), 1),
            "overhead_vs_step": round(ms / ms_step, 4), "flagged_markers": flagged, "occupied_cells": cells,
            "shared_cells": shared, "kernels": kern}


def refinement_cost(torch, ctx, wl, steps):
    """Adaptive Lagrangian refinement of the workload's base meshes (one
    triangle per marker): time per call, markers out, level histogram."""
    from paper_1805_01113_amd import mls
    from paper_1805_01113_amd import workloads as W
    v, t = W.body_mesh(wl)
    tri = torch.from_numpy(t).cuda()
    xv, yv, zv = (torch.from_numpy(np.ascontiguousarray(v[:, d])).cuda() for d in range(3))
    r = ctx.refine(tri, xv, yv, zv)
    ctx.sync()
    m = r["count"]
    hist = torch.bincount(r["level"].long(), minlength=4).tolist()
    del r
    mls.timing_enable(ctx, True)
    mls.timing_get(ctx, reset=True)
    for _ in range(steps):
        ctx.refine(tri, xv, yv, zv, sync=False)
    torch.cuda.synchronize()
    ctx.sync()
    kt = mls.timing_get(ctx, reset=True)
    mls.timing_enable(ctx, False)
    ms = kt["refine"][0] / kt["refine"][1]
    T = len(t)
    # per triangle, in each of the two passes: indices 12 B and 3 vertices
    # 36 B; the level byte written once and read once; per marker 32 B written
    alg = T * (2 * (12 + 36) + 2) + m * 32
    return {"triangles": T, "markers_out": m, "levels": hist, "ms": round(ms, 4),
            "triangles_per_s": round(T / (ms * 1e-3), 1), "alg_GBs": round(alg / (ms * 1e-3) / 1e9, 1)}


def gradient_cost(torch, ctx, wl, x, y, z, fields, steps, t_per):
    """Fused velocity values and gradients at the markers (derivative shape
    functions, no Phi stored): time per call and throughput."""
    from paper_1805_01113_amd import mls
    n = wl.n
    out = ctx.interp_grad(x, y, z, *fields)
    ctx.sync()
    del out
    mls.timing_enable(ctx, True)
    mls.timing_get(ctx, reset=True)
    for _ in range(steps):
        ctx.interp_grad(x, y, z, *fields)
    torch.cuda.synchronize()
    ctx.sync()
    kt = mls.timing_get(ctx, reset=True)
    mls.timing_enable(ctx, False)
    ms = kt["interp_grad"][0] / kt["interp_grad"][1]
    alg = 12 + 4.0 * t_per + 12 + 36     # positions, touched field values, U and G
    return {"ms": round(ms, 4), "markers_per_s": round(n / (ms * 1e-3), 1),
            "alg_bytes_per_marker": round(alg, 1), "alg_GBs": round(alg * n / (ms * 1e-3) / 1e9, 1),
            "outputs": "U [3][n], G [9][n] (d u_c / d x_d)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="uneven", choices=["uneven", "ellipsoids", "stretched", "sphere", "contact"])
    ap.add_argument("--method", default="exact", choices=["exact", "fast", "learned", "fast_linear"])
    ap.add_argument("--weights", default=None, help="surrogate checkpoint (default: the packaged one)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (JSON lines)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--full-phi", action="store_true",
                    help="exact steps store all 27 shape-function values per row instead of the compact form")
    ap.add_argument("--no-extra", action="store_true", help="skip the eager / per-body / fast comparisons")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads' method matrix")
    ap.add_argument("--copy-gib", type=float, default=0.0,
                    help="only run a plain device-to-device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.copy_gib > 0:
        import torch
        nbytes = int(args.copy_gib * (1 << 30))
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": nbytes, "launches": 3}), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1805_01113_amd import mls

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    mls.load()
    lib_version = mls.version()
    if not lib_version.endswith(source_hash()):
        log("warning: libmls_hip.so was not built from the current sources (%s)" % lib_version)
    t0 = time.time()
    wl = make_workload(args.workload)
    log("workload %s: %d markers, %d bodies, generated in %.1fs" % (wl.name, wl.n, len(wl.body_offsets) - 1,
                                                                     time.time() - t0))
    dev = "cuda"
    n = wl.n
    h_min = wl.grid.h_min
    x0, y0, z0 = [torch.from_numpy(a).to(dev) for a in (wl.x, wl.y, wl.z)]
    area = torch.from_numpy(wl.area).to(dev)
    from paper_1805_01113_amd import workloads as W
    fields = []
    for c in range(3):
        fields.append(W.fourier_field(wl.grid, c, wl.modes[c], wl.lengths, device=dev))
        torch.cuda.synchronize()
        log("velocity component %d ready" % c)
    forcing = [torch.zeros(wl.grid.shape(c), dtype=torch.float32, device=dev) for c in range(3)]
    torch.cuda.synchronize()
    log("fields ready (%.1f GB velocity + %.1f GB forcing)" % (sum(f.numel() for f in fields) * 4e-9,
                                                                 sum(f.numel() for f in forcing) * 4e-9))
    method = METHODS[args.method]
    ctx = mls.Context(wl.grid.faces, wl.grid.periodic)
    ctx.reserve(n)
    net_meta = load_network(ctx, args.weights)
    if method == mls.MLS_LEARNED and net_meta is None:
        raise SystemExit("--method learned needs the surrogate checkpoint")
    bufs = mls.StepBuffers(ctx, x0, y0, z0, area, fields, forcing)
    # exact steps keep the transfer functions compact (gamma and the support
    # offsets) unless --full-phi: the same U, F and forcing, fewer bytes
    compact = method == mls.MLS_EXACT and not args.full_phi
    nf = 7 if all(wl.grid.uniform_axis(d) for d in range(3)) else 13
    step_cfg = {"method": args.method,
                "transfer_function": ("compact, %d floats per row" % nf) if compact else "27 floats per row"}
    tune = None
    if not args.no_tune:
        t_a = time.time()
        tune = ctx.autotune(bufs, method=method, cache_path=args.tune_cache, compact=compact)
        for f in forcing:
            f.zero_()
        torch.cuda.synchronize()
        log("autotune (%.1fs): %s" % (time.time() - t_a, json.dumps(tune)))
    jitter = 0.1 * h_min
    seed = 20180503
    graph = mls.StepGraph(ctx, bufs, method=method, dt=1.0, jitter=jitter, seed=seed, compact=compact)
    stream = torch.cuda.current_stream()

    # ---- timed region: graph replays ------------------------------------------
    graph.launch(args.warmup)
    ctx.sync()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    graph.launch(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ctx.sync()
    ms_graph = e0.elapsed_time(e1) / max(args.steps, 1)
    value = n / (ms_graph * 1e-3)
    log("graph: %.3f ms/step, %.3e markers/s" % (ms_graph, value))

    # ---- per-kernel timing (eager steps, HIP events around each launch) -------
    mls.timing_enable(ctx, True)
    mls.timing_get(ctx, reset=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        mls.step(ctx, bufs, method=method, dt=1.0, jitter=jitter, seed=seed, compact=compact)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_eager = e0.elapsed_time(e1) / max(args.steps, 1)
    kt = mls.timing_get(ctx, reset=True)
    mls.timing_enable(ctx, False)
    ctx.sync()
    fp = {}
    T = touched_nodes(torch, ctx, bufs.home, n, fp)
    t_per = T / n
    contract, own = byte_models(method, compact, nf, t_per, "jitter" in kt)
    kernels = {}
    for k, (ms, cnt) in kt.items():
        avg = ms / cnt
        kernels[k] = {"avg_ms": round(avg, 4), "launches": cnt}
        if contract.get(k):
            kernels[k]["contract_bytes_per_marker"] = round(contract[k], 1)
            kernels[k]["GBs_contract_bytes"] = round(contract[k] * n / (avg * 1e-3) / 1e9, 1)
        if own.get(k):
            kernels[k]["kernel_bytes_per_marker"] = round(own[k], 1)
            kernels[k]["GBs_kernel_bytes"] = round(own[k] * n / (avg * 1e-3) / 1e9, 1)
    dom = max(((k, v) for k, v in kernels.items() if contract.get(k)), key=lambda kv: kv[1]["avg_ms"])
    step_contract = sum(contract.get(k, 0.0) for k in kernels) * n
    step_own = sum(own.get(k, 0.0) for k in kernels) * n
    log("eager: %.3f ms/step; kernels: %s" % (ms_eager, json.dumps(kernels)))
    traffic = measured_traffic(dom[0], wl.name, step_cfg)
    achieved = dom[1]["GBs_contract_bytes"]
    roof = {"bound": "hbm", "kernel": dom[0], "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "alg_bytes_per_marker": round(contract[dom[0]], 1), "markers_per_launch": n,
            "bytes_basis": "the hot-path contract's bytes per marker (Phi stored and read, 27 floats)",
            "frac_kernel_bytes": round(dom[1].get("GBs_kernel_bytes", 0.0) / HBM_PEAK_GBS, 4),
            "kernel_bytes_per_marker": round(own.get(dom[0], 0.0), 1),
            "frac_counter_bytes": (round(traffic / (dom[1]["avg_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                   if traffic else None)}

    extra = {"library": lib_version, "ms_per_step_eager": round(ms_eager, 4), "kernels": kernels, "autotune": tune,
             "touched_nodes_per_marker": round(t_per, 3),
             # bytes per marker of the touched field values at 4 B, and at
             # the 32 B sector, 64 B and 128 B line granularity of the memory
             # system (one read each; the spreading reads and writes them)
             "touched_field_bytes_per_marker": {
                 "values_4B": round(4.0 * fp["nodes"] / n, 2), "sectors_32B": round(32.0 * fp["sectors_32B"] / n, 2),
                 "lines_64B": round(64.0 * fp["lines_64B"] / n, 2),
                 "lines_128B": round(128.0 * fp["lines_128B"] / n, 2)},
             "step_contract_bytes_per_marker": round(step_contract / n, 1),
             "step_hbm_frac_contract_bytes": round(step_contract / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "step_kernel_bytes_per_marker": round(step_own / n, 1),
             "step_hbm_frac_kernel_bytes": round(step_own / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    if not args.no_extra:
        extra["methods"] = compare_methods(torch, ctx, wl, bufs, fields, forcing, x0, y0, z0, area, jitter, seed,
                                           args, ms_graph, method)
        mt = extra["methods"]
        if "learned" in mt and "exact" in mt:
            # the target's status: the learned, batched step against the exact one
            extra["learned_vs_exact"] = {
                "speed_ratio": round(mt["learned"]["batched"]["markers_per_s"] /
                                     mt["exact"]["batched"]["markers_per_s"], 4),
                "interp_err_vs_exact": mt["learned"]["interp_err_vs_exact"],
                "fallback_rate": mt["learned"].get("fallback_rate")}

        extra["collision"] = collision_cost(torch, ctx, wl, x0, y0, z0, args.steps, ms_graph)
        log("collision detection: %s" % json.dumps(extra["collision"]))
        extra["velocity_gradients"] = gradient_cost(torch, ctx, wl, x0, y0, z0, fields, args.steps, t_per)
        log("velocity gradients: %s" % json.dumps(extra["velocity_gradients"]))
        if "centres" in wl.meta:
            extra["refinement"] = refinement_cost(torch, ctx, wl, args.steps)
            log("refinement: %s" % json.dumps(extra["refinement"]))

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(wl, fields, args.cpu_seconds)
        log("cpu baseline: %.3e markers/s on %d threads" % (cpu["value"], cpu["cores"]))

    if not args.no_extra and not args.no_configs:
        # the main workload's buffers are released first (25.8 GB of fields)
        graph.close()
        ctx.close()
        del bufs, fields, forcing, x0, y0, z0, area
        torch.cuda.empty_cache()
        extra["configs"] = config_matrix(torch, args)
        graph = ctx = None

    out = {
        "metric": "markers/s build+interp+spread: learned/batched vs exact MLS, 1 GPU, ≤1e-4 err",
        "value": round(value, 1),
        "unit": "markers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_graph, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "markers": n, "bodies": int(len(wl.body_offsets) - 1),
                   "grid": list(wl.grid.n), "method": args.method, "execution": "hipgraph_batched",
                   "step": "jitter+build+interp+force+spread",
                   "transfer_function": step_cfg["transfer_function"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    if net_meta is not None:
        extra["surrogate"] = net_meta
    print(json.dumps(out), flush=True)
    if graph is not None:
        graph.close()
        ctx.close()


if __name__ == "__main__":
    main()
