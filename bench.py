"""Benchmark: splatted points per second for forward+backward trilinear point splatting.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-batched]
                [--no-coarser] [--no-optim] [--no-8m] [--no-decoder] [--no-extras]
                [--opt-iters N]

Headline workload (one step = the whole hot path once): 2M points drawn from 64 anisotropic
Gaussian clusters plus 30% on planar patches, one 1920x1080 pinhole view, 8 pyramid layers,
4-channel float32 descriptors, upstream pyramid gradient N(0, 1); forward (projection,
layer pair, trilinear write, per-texel depth sort, top-16, blend) then backward (gradients
for positions, world sizes, opacities and descriptors).  Synthetic, seeded inputs resident
in HBM before the timed region.

The timed step is the forward + backward launch sequence, timed both captured once in a HIP
graph and replayed, and launched directly; the faster is the headline (`step_mode`).  Also
reported: per-kernel durations (eager steps with HIP events around every launch, on its
stream); the roofline of the dominant kernel in the method's own byte units (per fragment,
kept fragment, texel and point) beside the implementation's byte model; the whole step's
fraction of HBM peak; a plain device copy's bandwidth; the forward alone at the same size;
the 4096-point 256x256 forward latency; the same cloud in Morton order of position (a
spatially coherent input order) instead of shuffled; the reconstruction network (Sec. 3.3) on the rendered
pyramid, with its matrix-core roofline; the same workload with coarser-layer inclusion; the
batched multi-view form (16 views of mixed resolution over 4M points, autotuned launch shape)
against 16 single-view launch sequences; 8M points at 1080p; the optimisation loop (8M
points, 8 views of 2560x1440, D = 8, 100 iterations of fwd + bwd + Adam against targets the
CPU oracle renders); and the CPU oracle on the host's cores beside each.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "splatted points/sec fwd+bwd at 1080p (+ % HBM roofline), batched vs per-view"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
PARAMS = ("x", "y", "z", "sw", "alpha", "desc")
FINE_E = 256  # tiles with at most this many entries are rendered whole (the fine path)
SIDE_STREAM = ("fwd_fine", "bwd_fine")  # launched on a second stream beside the work items


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------------------
# Byte counts.

def method_bytes(stage, w):
    """The method's own algorithmic bytes (per point, fragment, kept fragment, texel) that
    one launch of `stage` moves, the whole-step count split over the kernels that do each
    part: points read for projection (20 B per point: 16 in the count pass, the opacity in
    the scatter), fragments written (8 B each, scatter) and read back (8 B each, by the tile
    kernels that sort them), kept ids saved (4 B, forward) and reloaded (4 B, backward),
    pyramid written and upstream gradient read (4D B per texel), descriptors read per
    visible point (4D B, forward and backward, split between the tile kernels in proportion
    to their kept fragments), points re-read in backward (20 B per visible point) and
    gradients written (4 (5 + D) B per point).  Kernels with no part (the scans, the merge
    of partial lists) count zero; the parts sum to step_bytes()."""
    N, D, Nv, P = w["N"], w["D"], w["Nv"], w["P"]
    F, Fc, Ff, K, Kc, Kf = w["F"], w["F_c"], w["F_f"], w["K"], w["K_c"], w["K_f"]
    Pc, Pf = w["P_c"], w["P_f"]
    share_c = Kc / K if K else 0.0
    share_f = Kf / K if K else 0.0
    table = {
        "count": 16 * N,
        "colscan": 0,
        "binscan": 0,
        "scatter": 4 * N + 8 * F,
        "fwd_items": 8 * Fc + 4 * Kc + 4 * D * Pc + 4 * D * Nv * share_c,
        "fwd_fine": 8 * Ff + 4 * Kf + 4 * D * Pf + 4 * D * Nv * share_f,
        "fwd_merge": 0,
        "bwd_pixels": 4 * Kc + 4 * D * Pc + 4 * D * Nv * share_c,
        "bwd_items": 0,
        "bwd_fine": 4 * Kf + 4 * D * Pf + 4 * D * Nv * share_f,
        "bwd_points": 20 * Nv + 4 * (5 + D) * N,
    }
    return table.get(stage)


def impl_bytes(stage, w):
    """The implementation's own byte model of one launch (reads + writes of its data
    structures: 20-byte tile entries, 32-byte rows, 16-bit per-block histograms and their
    32-bit prefixes, kept keys and gammas), for comparison with the method's bytes and the
    counters."""
    N, D, E, Ef, K, Kf, Nv = w["N"], w["D"], w["E"], w["E_f"], w["K"], w["K_f"], w["Nv"]
    NB, NBf, Ic, Pc, Pf, nblk = w["NB"], w["NB_f"], w["I_c"], w["P_c"], w["P_f"], w["nblk"]
    Ec, Kc, NBc = E - Ef, K - Kf, NB - NBf
    row = 4 * (4 + D)
    table = {
        "count": 16 * N + 2 * nblk * NB,
        "colscan": 6 * nblk * NB + 4 * NB,
        "scatter": 20 * N + 4 * nblk * NB + 4 * NB + 20 * E + 32 * Nv,
        "fwd_items": 20 * Ec + (4 * D + 12) * Kc + 4 * 256 * NBc + 4 * D * Pc,
        "fwd_fine": (24 + 4 * D) * Ef + 12 * Kf + 4 * 256 * NBf + 4 * D * Pf,
        "bwd_pixels": 4 * 256 * NBc + (12 + 4 * D + 8) * Kc + 4 * D * Pc,
        "bwd_items": (20 + row) * Ec + 16 * Kc + Ic * 256 * (4 + 4 * D),
        "bwd_fine": (24 + 4 * D + row) * Ef + 4 * 256 * NBf + 4 * D * Pf,
        "bwd_points": 20 * N + 32 * Nv + row * E + 4 * (5 + D) * N,
    }
    return table.get(stage)


def step_bytes(N, Nv, D, F, K, P):
    """Whole-step algorithmic bytes of the method (one view, fwd+bwd, fragment lists
    materialised once): point reads, descriptor reads of visible points, fragment write and
    read, kept ids saved and reloaded, pyramid write and upstream-gradient read, point
    re-read in backward, gradient write."""
    return N * 20 + Nv * 4 * D + 16 * F + 8 * K + 8 * D * P + Nv * (20 + 4 * D) + N * (20 + 4 * D)


def forward_bytes(N, Nv, D, F, P):
    """Forward alone, nothing saved: point reads, descriptor reads, fragment write and read,
    pyramid write."""
    return N * 20 + Nv * 4 * D + 16 * F + 4 * D * P


def measured_traffic(kernel, field="bytes_per_launch"):
    """HBM bytes per launch of `kernel` from the committed counter summary (read and write
    requests to memory by size, two passes), or, with field="step_bytes", those of every
    kernel of one step; None when no summary was taken on the current kernel source."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_2401_06003_amd", "csrc", "trips.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.md"))):
        for line in open(f):
            if line.startswith("traffic-json: "):
                d = json.loads(line[len("traffic-json: "):])
                if d.get("kernel") == kernel and d.get("source_sha256") == h:
                    return d.get(field)
    return None


# ---------------------------------------------------------------------------------------
# Workload counts.

def texel_bins(cams, nl, tile_w=16):
    """Tile (bin) of every texel of the pyramid of `cams`, in pyramid order; bins are
    numbered view, layer, tile row, tile column (256-texel tiles of width tile_w)."""
    import numpy as np
    th = 256 // tile_w
    out, base = [], 0
    for c in cams:
        for L in range(nl):
            W = -(-int(c["W"]) // (1 << L))
            H = -(-int(c["H"]) // (1 << L))
            tx = -(-W // tile_w)
            j, i = np.divmod(np.arange(W * H, dtype=np.int64), W)
            out.append(base + (j // th) * tx + (i // tile_w))
            base += tx * (-(-H // th))
    return np.concatenate(out)


def workload_counts(tp, r, cams, nl, N, D, item_e=8192, tile_w=16):
    """Counts of the last forward call of renderer r (synchronises)."""
    import numpy as np
    import torch
    st = r.stats()
    counts, _ids = r.export_fragments()
    c = counts.to(torch.int64).cpu().numpy()
    kept = np.minimum(c, tp.KEEP)
    tile_e, tile_k = r.tile_stats()
    fine = tile_e <= FINE_E
    bins = texel_bins(cams, nl, tile_w)
    tex_fine = fine[bins]
    F, K = int(c.sum()), int(kept.sum())
    return {"N": N, "D": D, "E": st["entries"], "E_f": int(tile_e[fine].sum()), "F": F,
            "F_f": int(c[tex_fine].sum()), "F_c": int(c[~tex_fine].sum()), "K": K,
            "K_f": int(kept[tex_fine].sum()), "K_c": int(kept[~tex_fine].sum()),
            "NB": st["bins"], "NB_f": int(fine.sum()),
            "I_c": int(((tile_e[~fine].astype(np.int64) + item_e - 1) // item_e).sum()),
            "P": r.texels, "P_f": int(tex_fine.sum()), "P_c": int((~tex_fine).sum()),
            "nblk": (N + 4095) // 4096, "Nv": st["visible"]}


# ---------------------------------------------------------------------------------------
# Timing helpers.

def timed(torch, fn, steps):
    """Mean milliseconds of `steps` calls of fn, HIP events on the current stream around
    the whole sequence, synchronised on both sides."""
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def stage_times(torch, tp, fn, steps):
    """Per-kernel mean milliseconds over `steps` calls of fn (HIP events on each launch's
    stream), and the mean step time of that run."""
    tp.timing_enable(True)
    ms = timed(torch, fn, steps)
    stages = tp.timing_read()
    tp.timing_enable(False)
    return {k: v[0] / max(v[1], 1) for k, v in stages.items() if v[1] > 0}, ms


# ---------------------------------------------------------------------------------------
# CPU oracle timings.

def median_time(fn, runs):
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), ts


def cpu_baseline(sc, G, runs=3):
    """The oracle on the headline workload (one forward + backward of all 2M points), on every
    host thread available (texel-interleaved sets, one unchanged oracle call each), median of
    `runs`; and once on one thread."""
    import numpy as np
    from oracle import oracle, parallel
    cam, nl = sc["cams"][0], sc["nlayers"]
    n = len(sc["points"]["x"])
    Gd = G.astype(np.float64).reshape(-1, sc["D"])
    workers = parallel.default_workers()

    def par():
        parallel.forward(sc["points"], cam, nl, workers=workers)
        parallel.backward(sc["points"], cam, nl, Gd, workers=workers)

    med, ts = median_time(par, runs)
    t0 = time.perf_counter()
    oracle.forward(sc["points"], cam, nl)
    oracle.backward(sc["points"], cam, nl, Gd)
    t1 = time.perf_counter() - t0
    return {"value": n / med, "unit": "points/s", "cores": workers, "kind": "oracle",
            "sample": "one forward+backward of the full workload (%d points, %dx%d, %d layers) "
                      "on %d threads, median of %d (%s s)" %
                      (n, cam["W"], cam["H"], nl, workers, runs,
                       ", ".join("%.2f" % t for t in ts)),
            "value_1core": n / t1, "seconds_1core": t1}


# ---------------------------------------------------------------------------------------
# GPU sections.

def run_small_latency(torch, tp, scenes, steps, dev):
    """4096 points in the unit cube, 256x256, 5 layers: forward alone and forward + backward
    latency (microseconds) of direct launches and of a captured graph's replays, the same
    with the autotuner's launch shape, and the oracle's forward on one and on every host
    thread (median of 3)."""
    import numpy as np
    from oracle import oracle, parallel
    sc = scenes.unit_cube(1)
    cam, nl, D = sc["cams"][0], sc["nlayers"], sc["D"]
    n = len(sc["points"]["x"])
    t = {k: torch.from_numpy(sc["points"][k]).to(dev) for k in PARAMS}
    args = [t[k] for k in PARAMS]
    r = tp.Renderer([cam], nl, D, n, device=dev)
    pyr = torch.empty(r.pyramid_numel(), device=dev)
    G = torch.from_numpy(scenes.upstream_gradient(1, r.pyramid_numel())).to(dev)
    grads = [torch.empty(n, device=dev) for _ in range(5)] + [torch.empty((n, D), device=dev)]
    for _ in range(5):
        r.forward(*args, out=pyr)
        r.backward(*args, G, outs=grads)
    fwd_ms = timed(torch, lambda: r.forward(*args, out=pyr), steps)
    fb_ms = timed(torch, lambda: (r.forward(*args, out=pyr), r.backward(*args, G, outs=grads)),
                  steps)
    # the same calls captured once in a HIP graph and replayed (no per-call host work)
    plan = tp.Plan(r, *args, pyr, G, grads)
    for _ in range(3):
        plan.launch(forward=True, backward=True)
    fwd_graph_ms = timed(torch, lambda: plan.launch(forward=True, backward=False), steps)
    fb_graph_ms = timed(torch, lambda: plan.launch(forward=True, backward=True), steps)
    del plan
    # the autotuner's launch shape for this workload: smaller binning blocks and work items
    # spread a few heavy tiles over more workgroups
    cand = [(tw, pb, ie) for tw in (8, 16) for pb in (512, 1024, 4096) for ie in (256, 512, 1024, 8192)]
    best, _ = tp.autotune([cam], nl, D, *args, candidates=cand, reps=5, device=dev)
    rt = tp.Renderer([cam], nl, D, n, tuning=best, device=dev)
    for _ in range(5):
        rt.forward(*args, out=pyr)
        rt.backward(*args, G, outs=grads)
    tfwd_ms = timed(torch, lambda: rt.forward(*args, out=pyr), steps)
    tfb_ms = timed(torch, lambda: (rt.forward(*args, out=pyr), rt.backward(*args, G, outs=grads)),
                   steps)
    del rt
    one, _ = median_time(lambda: oracle.forward(sc["points"], cam, nl), 3)
    workers = parallel.default_workers()
    par, _ = median_time(lambda: parallel.forward(sc["points"], cam, nl, workers=workers), 3)
    return {"workload": "unitcube4096_256x256_5layers_d4", "points": n,
            "forward_us": fwd_ms * 1e3, "fwd_bwd_us": fb_ms * 1e3,
            "forward_us_graph": fwd_graph_ms * 1e3, "fwd_bwd_us_graph": fb_graph_ms * 1e3,
            "tuned": {"tile_w": best.tile_w, "points_per_block": best.points_per_block,
                      "item_entries": best.item_entries, "forward_us": tfwd_ms * 1e3,
                      "fwd_bwd_us": tfb_ms * 1e3},
            "oracle_forward_us_1core": one * 1e6, "oracle_forward_us_all_cores": par * 1e6,
            "oracle_cores": workers}


def run_copy(torch, dev, mib=512, steps=10):
    """A plain device-to-device copy of `mib` MiB: bytes read + written per second, the
    bandwidth a streaming kernel reaches on this part."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    ms = timed(torch, lambda: dst.copy_(src), steps)
    gbs = 2 * n * 4 / (ms / 1e3) / 1e9
    return {"bytes_each_way": n * 4, "ms": ms, "gbps": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS}


def run_forward_only(torch, tp, r, pargs, pyr, w, steps, workers_sc=None):
    """The headline scene's forward pass alone (direct launches) and its effective fraction
    of HBM peak (forward bytes: points, descriptors, fragments written and read, pyramid)."""
    for _ in range(3):
        r.forward(*pargs, out=pyr)
    ms = timed(torch, lambda: r.forward(*pargs, out=pyr), steps)
    fb = forward_bytes(w["N"], w["Nv"], w["D"], w["F"], w["P"])
    out = {"workload": "clusters2m_1920x1080_8layers_d4_fwd", "ms": ms,
           "points_per_s": w["N"] / (ms / 1e3), "algorithmic_bytes": fb,
           "effective_hbm_frac": fb / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
    if workers_sc is not None:
        from oracle import parallel
        sc = workers_sc
        workers = parallel.default_workers()
        med, _ = median_time(lambda: parallel.forward(sc["points"], sc["cams"][0], sc["nlayers"],
                                                      workers=workers), 3)
        out["oracle_forward_s"] = med
        out["oracle_cores"] = workers
    return out


def run_coarser(torch, tp, sc, pargs, G, steps, warmup, dev, ms_plain):
    """The headline workload with coarser-layer inclusion: graph-replayed steps, then eager
    steps with per-kernel events.  The inclusion passes are charged the bytes of their own data
    structures (an implementation model: the paper gives the variant no byte count): forward,
    per texel the own kept fragments read (12 B), every blended item's descriptor gathered
    (4D B) and, above layer 0 (whose lists are rebuilt where read), written (12 B), plus the
    texel (4D B) and its count (4 B); backward, every blended item read (12 B) with its
    descriptor (4D B) and its totals written and read once more (8 (1 + D) B), plus the
    upstream gradient (4D B) and the count (4 B)."""
    cam, nl, D = sc["cams"][0], sc["nlayers"], sc["D"]
    N = len(sc["points"]["x"])
    r = tp.Renderer([cam], nl, D, N, device=dev, include_coarser=True)
    pyr = torch.empty(r.pyramid_numel(), device=dev)
    grads = [torch.empty(N, device=dev) for _ in range(5)] + [torch.empty((N, D), device=dev)]
    plan = tp.Plan(r, *pargs, pyr, G, grads)
    for _ in range(warmup):
        plan.launch(forward=True, backward=True)
    torch.cuda.synchronize()
    counts, ids = r.export_fragments()
    c64 = counts.to(torch.int64)
    K = int(torch.clamp(c64, max=tp.KEEP).sum().item())
    Fb = int((ids >= 0).sum().item())
    P = r.texels
    Fb0 = int((ids[:r.layouts[0][1][1]] >= 0).sum().item())  # blended items of layer 0

    def eager():
        r.forward(*pargs, out=pyr)
        r.backward(*pargs, G, outs=grads)

    ms_graph = timed(torch, lambda: plan.launch(forward=True, backward=True), steps)
    ms_eager = timed(torch, eager, steps)
    ms = min(ms_graph, ms_eager)
    stage_ms, _ = stage_times(torch, tp, eager, steps)
    ib = {"incl_fwd": 12 * K + 4 * D * Fb + 12 * (Fb - Fb0) + (4 * D + 4) * P,
          "incl_bwd": (12 + 4 * D + 8 * (1 + D)) * Fb + (4 * D + 4) * P}
    return {"workload": "clusters2m_1920x1080_8layers_d4_fwd_bwd_coarser_inclusion",
            "ms_per_step": ms, "ms_per_step_graph": ms_graph, "ms_per_step_eager": ms_eager,
            "inclusion_overhead_ms": ms - ms_plain,
            "points_per_s": N / (ms / 1e3), "blended_items": Fb,
            "blended_items_plain": K, "stage_ms": {k: round(v, 5) for k, v in stage_ms.items()},
            "incl_impl_gbps": {k: round(b / (stage_ms[k] / 1e3) / 1e9, 1) for k, b in ib.items()
                               if k in stage_ms}}


def run_points_8m(torch, tp, scenes, steps, warmup, dev):
    """The headline recipe with 8M points (1920x1080, 8 layers, D = 4, forward + backward),
    launched directly, with the whole step's effective fraction of HBM peak; then the same with
    the autotuner's launch shape for this size."""
    sc = scenes.cluster_scene(2, n=8_000_000)
    cam, nl, D = sc["cams"][0], sc["nlayers"], sc["D"]
    n = len(sc["points"]["x"])
    t = {k: torch.from_numpy(sc["points"][k]).to(dev) for k in PARAMS}
    args = [t[k] for k in PARAMS]
    r = tp.Renderer([cam], nl, D, n, device=dev)
    G = torch.from_numpy(scenes.upstream_gradient(3, r.pyramid_numel())).to(dev)
    pyr = torch.empty(r.pyramid_numel(), device=dev)
    grads = [torch.empty(n, device=dev) for _ in range(5)] + [torch.empty((n, D), device=dev)]

    def step():
        r.forward(*args, out=pyr)
        r.backward(*args, G, outs=grads)

    for _ in range(warmup):
        step()
    ms = timed(torch, step, steps)
    w = workload_counts(tp, r, [cam], nl, n, D)
    stage_ms, _ = stage_times(torch, tp, step, steps)
    sb = step_bytes(n, w["Nv"], D, w["F"], w["K"], w["P"])
    del r
    # the autotuner's launch shape for this size (four times the headline's entries per tile)
    cand = [(16, pb, ie) for pb in (4096, 8192) for ie in (8192, 16384, 32768)]
    best, _ = tp.autotune([cam], nl, D, *args, candidates=cand, reps=3, device=dev)
    rt = tp.Renderer([cam], nl, D, n, tuning=best, device=dev)

    def step_tuned():
        rt.forward(*args, out=pyr)
        rt.backward(*args, G, outs=grads)

    for _ in range(warmup):
        step_tuned()
    ms_t = timed(torch, step_tuned, steps)
    del rt
    return {"workload": "clusters8m_1920x1080_8layers_d4_fwd_bwd", "points": n,
            "ms_per_step": ms, "points_per_s": n / (ms / 1e3),
            "step_algorithmic_bytes": sb,
            "step_effective_hbm_frac": sb / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
            "fragments": w["F"], "kept_fragments": w["K"], "visible_points": w["Nv"],
            "tile_entries": w["E"],
            "stage_ms": {k: round(v, 5) for k, v in stage_ms.items()},
            "tuned": {"tile_w": best.tile_w, "points_per_block": best.points_per_block,
                      "item_entries": best.item_entries, "ms_per_step": ms_t,
                      "points_per_s": n / (ms_t / 1e3),
                      "step_effective_hbm_frac": sb / (ms_t / 1e3) / 1e9 / HBM_PEAK_GBS}}


def run_ordered(torch, tp, scenes, sc, G, steps, warmup, dev):
    """The headline cloud with its points in Morton order of position (a spatially coherent
    cloud, as a scan or a reconstruction delivers it) instead of shuffled: same fragments and
    results, a different order of the entries within every tile."""
    so = scenes.morton_sorted(sc)
    cam, nl, D = so["cams"][0], so["nlayers"], so["D"]
    n = len(so["points"]["x"])
    t = {k: torch.from_numpy(so["points"][k]).to(dev) for k in PARAMS}
    args = [t[k] for k in PARAMS]
    r = tp.Renderer([cam], nl, D, n, device=dev)
    pyr = torch.empty(r.pyramid_numel(), device=dev)
    grads = [torch.empty(n, device=dev) for _ in range(5)] + [torch.empty((n, D), device=dev)]

    def step():
        r.forward(*args, out=pyr)
        r.backward(*args, G, outs=grads)

    for _ in range(warmup):
        step()
    ms = timed(torch, step, steps)
    stage_ms, _ = stage_times(torch, tp, step, steps)
    return {"workload": "clusters2m_1920x1080_8layers_d4_fwd_bwd_morton_order", "points": n,
            "ms_per_step": ms, "points_per_s": n / (ms / 1e3),
            "stage_ms": {k: round(v, 5) for k, v in stage_ms.items()}}


def run_batched(torch, tp, scenes, steps, warmup, dev, cpu_views=0):
    """16 views of mixed resolution over 4M points.  The launch shape is picked by the
    autotuner (forward + backward of the whole batch timed per candidate); then one batched
    forward+backward per step (as a graph launch and as direct launches; the faster counts)
    against 16 single-view forward+backward sequences on the same stream, both with that
    shape.  The method's point traffic a batched call shares across views (projection read,
    backward re-read, gradient write once per call instead of once per view) is reported
    beside the times.  cpu_views: time the oracle's forward + backward of that many views
    (the largest and the smallest first) on every host thread."""
    import numpy as np
    sc = scenes.multiview_scene(4, n=4_000_000, views=16, nlayers=8)
    n, nl, D, cams = len(sc["points"]["x"]), sc["nlayers"], sc["D"], sc["cams"]
    t = {k: torch.from_numpy(sc["points"][k]).to(dev) for k in PARAMS}
    args = [t[k] for k in PARAMS]
    t0 = time.perf_counter()
    best, tune_ms = tp.autotune(cams, nl, D, *args, reps=2, device=dev)
    tune_s = time.perf_counter() - t0
    rb = tp.Renderer(cams, nl, D, n, device=dev, tuning=best)
    G = torch.from_numpy(scenes.upstream_gradient(4, rb.pyramid_numel())).to(dev)
    pyr = torch.empty(rb.pyramid_numel(), device=dev)
    grads = [torch.empty(n, device=dev) for _ in range(5)] + [torch.empty((n, D), device=dev)]
    plan = tp.Plan(rb, *args, pyr, G, grads)
    singles, offs, o = [], [], 0
    big = max(range(16), key=lambda v: cams[v]["W"] * cams[v]["H"])
    first = tp.Renderer([cams[big]], nl, D, n, device=dev, tuning=best)
    for cam in cams:
        # the single-view calls run one after another: they share the largest buffers
        r = tp.Renderer([cam], nl, D, n, device=dev, tuning=best, share_buffers_with=first)
        singles.append(r)
        offs.append((o, o + r.pyramid_numel()))
        o += r.pyramid_numel()
    Gs = [G[a:b].contiguous() for (a, b) in offs]

    def per_view():
        for r, g in zip(singles, Gs):
            r.forward(*args)
            r.backward(*args, g)

    def batched():
        plan.launch(forward=True, backward=True)

    def batched_eager():
        rb.forward(*args, out=pyr)
        rb.backward(*args, G, outs=grads)

    res = {}
    for name, fn in (("per_view", per_view), ("batched", batched), ("batched_eager", batched_eager)):
        for _ in range(warmup):
            fn()
        res[name] = timed(torch, fn, steps)
    # the method's bytes: per view, and the point traffic shared by a batched call
    rb.forward(*args, out=pyr)
    torch.cuda.synchronize()
    counts, _ = rb.export_fragments()
    c = counts.to(torch.int64).cpu().numpy()
    st = rb.stats()
    F, K, P = int(c.sum()), int(np.minimum(c, tp.KEEP).sum()), rb.texels
    Nv = st["visible"]  # (point, view) pairs with fragments, summed over views
    per_view_bytes = (16 * (20 * n + (20 + 4 * D) * n) + 16 * F + 8 * K + 8 * D * P
                      + (20 + 8 * D) * Nv)
    batched_bytes = per_view_bytes - 15 * (20 * n + (20 + 4 * D) * n)
    best_ms = min(res["batched"], res["batched_eager"])
    out = {"workload": "clusters4m_16views_mixed_640x480_to_1920x1080_fwd_bwd", "points": n,
           "views": 16, "steps": steps,
           "tuning": {"tile_w": best.tile_w, "points_per_block": best.points_per_block,
                      "item_entries": best.item_entries},
           "autotune_s": tune_s, "autotune_candidates": len(tune_ms),
           "per_view_ms": res["per_view"],
           "batched_graph_ms": res["batched"], "batched_eager_ms": res["batched_eager"],
           "speedup": res["per_view"] / best_ms,
           "batched_points_per_s": n * 16 / (best_ms / 1e3),
           "per_view_points_per_s": n * 16 / (res["per_view"] / 1e3),
           "visible_point_views": Nv, "fragments": F, "kept_fragments": K,
           "algorithmic_bytes_per_view_sum": per_view_bytes,
           "algorithmic_bytes_batched": batched_bytes,
           "shared_point_bytes_saved": per_view_bytes - batched_bytes,
           "batched_effective_hbm_frac": batched_bytes / (best_ms / 1e3) / 1e9 / HBM_PEAK_GBS}
    if cpu_views:
        from oracle import parallel
        workers = parallel.default_workers()
        order = sorted(range(16), key=lambda v: -cams[v]["W"] * cams[v]["H"])
        pick = [order[0], order[-1]][:cpu_views]
        secs = []
        for v in pick:
            gv = G[offs[v][0]:offs[v][1]].cpu().numpy().astype(np.float64).reshape(-1, D)
            t0 = time.perf_counter()
            parallel.forward(sc["points"], cams[v], nl, workers=workers)
            parallel.backward(sc["points"], cams[v], nl, gv, workers=workers)
            secs.append(time.perf_counter() - t0)
        out["oracle_views"] = {"views": pick, "seconds": secs, "cores": workers,
                               "point_views_per_s": n * len(pick) / sum(secs)}
    return out


def run_optimisation(torch, tp, scenes, iters, warmup, dev):
    """The optimisation workload: 8M points, 8 views of 2560x1440 in one batched call, 8
    layers, D = 8.  Targets: the CPU oracle renders the 8 views of a perturbed copy of the
    scene (positions + N(0, 0.01^2), world sizes x U[0.5, 2]) on every host thread (timed:
    the oracle's side of this workload).  Each iteration renders the unperturbed starting
    scene's parameters through the autograd function, takes the squared error summed over
    layers, each normalised by W_L H_L D, back-propagates and steps Adam on positions,
    log-sizes, opacities and descriptors; `iters` iterations are timed, and the loss's
    final/initial ratio is reported."""
    import numpy as np
    from oracle import parallel
    sc = scenes.ring_scene(5)
    pts, cams, nl, D = sc["points"], sc["cams"], sc["nlayers"], sc["D"]
    n = len(pts["x"])
    truth = scenes.perturbed(pts, seed=55)
    workers = parallel.default_workers()
    t0 = time.perf_counter()
    tg = [parallel.forward(truth, c, nl, workers=workers)["pyr"].astype(np.float32).reshape(-1)
          for c in cams]
    oracle_s = time.perf_counter() - t0
    target = torch.from_numpy(np.concatenate(tg)).to(dev)
    del tg
    r = tp.Renderer(cams, nl, D, n, device=dev)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    wts = []
    for c in cams:
        dims, _ = tp.layer_layout(c, nl)
        for (w, h) in dims:
            wts.append(torch.full((w * h * D,), 1.0 / (w * h * D), device=dev))
    wts = torch.cat(wts)
    xyz = [dv(pts[k]).requires_grad_(True) for k in ("x", "y", "z")]
    log_sw = torch.log(dv(pts["sw"])).requires_grad_(True)
    alpha = dv(pts["alpha"]).requires_grad_(True)
    desc = dv(pts["desc"]).requires_grad_(True)
    params = [*xyz, log_sw, alpha, desc]
    init = [p.detach().clone() for p in params]

    def make_opt():
        return torch.optim.Adam([{"params": xyz, "lr": 1e-4}, {"params": [log_sw], "lr": 1e-2},
                                 {"params": [desc], "lr": 1e-2}, {"params": [alpha], "lr": 1e-2}],
                                betas=(0.9, 0.999))

    def step(opt):
        opt.zero_grad()
        out = tp.render(*xyz, torch.exp(log_sw), alpha, desc, r)
        loss = ((out - target) ** 2 * wts).sum()
        loss.backward()
        opt.step()
        with torch.no_grad():
            alpha.clamp_(0.0, 1.0)
        return loss

    opt = make_opt()
    for _ in range(warmup):
        step(opt)
    with torch.no_grad():  # the timed run starts from the unperturbed scene again
        for p, v in zip(params, init):
            p.copy_(v)
    opt = make_opt()
    losses = []
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        losses.append(step(opt).detach())
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    losses = [float(v) for v in torch.stack(losses).cpu()]
    return {"workload": "ring8m_8views_2560x1440_8layers_d8_fwd_bwd_adam", "points": n,
            "views": len(cams), "iterations": iters, "ms_per_iteration": ms,
            "point_views_per_s": n * len(cams) / (ms / 1e3),
            "loss_first": losses[0], "loss_last": losses[-1],
            "loss_ratio": losses[-1] / losses[0],
            "loss_monotone_smoothed": bool(np.all(np.diff(
                np.convolve(losses, np.ones(5) / 5, mode="valid")) <= 0)),
            "targets": "CPU oracle, %d views, %d threads, %.1f s" % (len(cams), workers, oracle_s),
            "oracle_targets_s": oracle_s, "oracle_cores": workers}


def decoder_flops(dims, D, out_dim, features=32):
    """Multiply-adds x 2 of the network on layer sizes `dims` [(W_L, H_L)], finest first: per
    texel of layer L a 3x3 convolution of C_in(L) channels (D for the coarsest layer, D + 32
    otherwise) to 64 outputs, and the 1x1 output layer on layer 0."""
    nl = len(dims)
    f = 0
    for L, (w, h) in enumerate(dims):
        cin = D if L == nl - 1 else D + features
        f += 2 * w * h * 9 * cin * 2 * features
    w0, h0 = dims[0]
    return f + 2 * w0 * h0 * features * out_dim


def run_decoder(torch, tp, scenes, pyr, cam, nl, D, steps, warmup, dev, cpu=True):
    """The reconstruction network (Sec. 3.3) on the headline view's rendered pyramid
    (1920x1080, 8 layers, D = 4, 3 output channels, seeded binary16 weights): whole-network
    time, the finest block alone, and the matrix-core roofline of the finest block (its
    algorithmic multiply-adds over its time, against the binary16 dense peak); the oracle's
    double-precision network on the host beside it."""
    import numpy as np
    W, H = cam["W"], cam["H"]
    wt = scenes.decoder_weights(61, nl, D)
    d = tp.Decoder(W, H, nl, D, wt, device=dev)
    img = torch.empty((H, W, 3), dtype=torch.float32, device=dev)
    for _ in range(warmup):
        d.forward(pyr, img)
    ms = timed(torch, lambda: d.forward(pyr, img), steps)
    # the finest block alone (block 1's output as its input, the output layer applied)
    W1, H1 = d.dims[1]
    h1 = torch.zeros((H1, W1, 32), dtype=torch.float16, device=dev)
    f0 = pyr[:W * H * D].view(H, W, D)
    ms0 = timed(torch, lambda: d.block(0, f0, h1, final=True), steps)
    fl = decoder_flops(d.dims, D, 3)
    fl0 = 2 * W * H * (9 * (D + 32) * 64 + 32 * 3)
    peak = 2500.0  # TFLOP/s, binary16 dense matrix cores
    out = {"workload": "decoder_1920x1080_8layers_d4_out3_fp16", "ms": ms,
           "frames_per_s": 1e3 / ms, "flops": fl, "tflops": fl / (ms / 1e3) / 1e12,
           "layer0_ms": ms0,
           "roofline": {"bound": "mfma", "kernel": "dec_block (layer 0)",
                        "achieved": fl0 / (ms0 / 1e3) / 1e12, "peak": peak, "unit": "TFLOP/s",
                        "frac": fl0 / (ms0 / 1e3) / 1e12 / peak, "flops_per_launch": fl0}}
    if cpu:
        from oracle import decoder as dec
        host = pyr.cpu().numpy().astype(np.float64)
        layers, o = [], 0
        for (w, h) in d.dims:
            layers.append(host[o:o + w * h * D].reshape(h, w, D))
            o += w * h * D
        t0 = time.perf_counter()
        dec.decode(layers, wt, fp16=True)
        sec = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1.0 / sec, "unit": "frames/s", "kind": "oracle",
                               "cores": torch.get_num_threads(),
                               "sample": "one 1920x1080 frame, 8 layers, double precision "
                                         "numpy (its matrix products on %d threads), %.1f s" %
                                         (torch.get_num_threads(), sec)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-coarser", action="store_true")
    ap.add_argument("--no-optim", action="store_true")
    ap.add_argument("--no-8m", action="store_true")
    ap.add_argument("--no-decoder", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the copy, forward-only and 4096-point sections (profiling runs)")
    ap.add_argument("--opt-iters", type=int, default=100)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (the reference for "
                         "scaling HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this renderer runs on one GPU; runs over several GPUs are not "
              "implemented (views would shard across GPUs with one gradient all-reduce).",
              flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": n * 4, "launches": 5}), flush=True)
        return

    import paper_2401_06003_amd as tp
    import scenes

    dev = torch.device("cuda:0")
    log("generating the 2M-point scene")
    sc = scenes.cluster_scene(2)
    cam, nl, D = sc["cams"][0], sc["nlayers"], sc["D"]
    N = len(sc["points"]["x"])
    t = {k: torch.from_numpy(sc["points"][k]).to(dev) for k in PARAMS}
    pargs = [t[k] for k in PARAMS]
    r = tp.Renderer([cam], nl, D, N, device=dev)
    Gnp = scenes.upstream_gradient(3, r.pyramid_numel())
    G = torch.from_numpy(Gnp).to(dev)
    pyr = torch.empty(r.pyramid_numel(), device=dev)
    grads = [torch.empty(N, device=dev) for _ in range(5)] + [torch.empty((N, D), device=dev)]

    def step():
        r.forward(*pargs, out=pyr)
        r.backward(*pargs, G, outs=grads)

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    w = workload_counts(tp, r, [cam], nl, N, D)

    # the step captured once in a HIP graph (forward then backward), replayed per step
    plan = tp.Plan(r, *pargs, pyr, G, grads)

    def step_graph():
        plan.launch(forward=True, backward=True)

    for _ in range(args.warmup):
        step_graph()
    log("timed %d graph steps" % args.steps)
    ms_graph = timed(torch, step_graph, args.steps)
    log("timed %d eager steps" % args.steps)
    ms_eager = timed(torch, step, args.steps)
    # the same launch sequence either way (the fine-tile kernels on a second stream beside the
    # work items, a graph branch when captured); the faster mode is the headline
    ms, mode = (ms_graph, "graph") if ms_graph <= ms_eager else (ms_eager, "eager")
    log("timed %d eager steps with per-kernel events" % args.steps)
    stage_ms, ms_events = stage_times(torch, tp, step, args.steps)
    # the dominant kernel: the longest on the launch stream (the fine-tile kernels run on a
    # second stream beside the work items, and their spans include waiting for the CUs the
    # items hold)
    dom = max((k for k in stage_ms if method_bytes(k, w) is not None and k not in SIDE_STREAM),
              key=lambda k: stage_ms[k])
    dom_bytes = method_bytes(dom, w)
    achieved = dom_bytes / (stage_ms[dom] / 1e3) / 1e9
    sbytes = step_bytes(N, w["Nv"], D, w["F"], w["K"], w["P"])
    assert abs(sum(method_bytes(k, w) for k in
                   ("count", "scatter", "fwd_items", "fwd_fine", "bwd_pixels", "bwd_fine",
                    "bwd_points")) - sbytes) <= 1e-6 * sbytes
    step_meas = measured_traffic(dom, "step_bytes")
    out = {
        "metric": METRIC, "value": N / (ms / 1e3), "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "clusters2m_1920x1080_8layers_d4_fwd_bwd", "points": N, "views": 1,
                   "width": cam["W"], "height": cam["H"], "layers": nl, "desc_dim": D},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom),
                     # the counters' HBM bytes over the same time: what the kernel moves, not
                     # what the method needs (a re-read counts twice here)
                     "traffic_frac": (measured_traffic(dom) / (stage_ms[dom] / 1e3) / 1e9
                                      / HBM_PEAK_GBS if measured_traffic(dom) else None),
                     "bytes_per_launch": dom_bytes, "ms_per_launch": stage_ms[dom],
                     "impl_bytes_per_launch": impl_bytes(dom, w),
                     "step_frac": sbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS},
        "step_mode": mode, "ms_per_step_graph": ms_graph, "ms_per_step_eager": ms_eager,
        "ms_per_step_eager_with_kernel_events": ms_events,
        "step_effective_hbm_frac": sbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
        "step_algorithmic_bytes": sbytes,
        "step_measured_hbm_bytes": step_meas,
        "step_measured_over_algorithmic": (step_meas / sbytes if step_meas else None),
        "step_counter_hbm_frac": (step_meas / (ms / 1e3) / 1e9 / HBM_PEAK_GBS if step_meas else None),
        "stage_ms": {k: round(v, 5) for k, v in stage_ms.items()},
        "stage_method_gbps": {k: round(method_bytes(k, w) / (v / 1e3) / 1e9, 1)
                              for k, v in stage_ms.items() if method_bytes(k, w)},
        "stage_impl_gbps": {k: round(impl_bytes(k, w) / (v / 1e3) / 1e9, 1)
                            for k, v in stage_ms.items() if impl_bytes(k, w)},
        "fragments": w["F"], "kept_fragments": w["K"], "tile_entries": w["E"], "tiles": w["NB"],
        "texels": w["P"], "visible_points": w["Nv"], "fine_tiles": w["NB_f"],
        "fine_tile_entries": w["E_f"], "fine_tile_fragments": w["F_f"],
        "fine_tile_kept": w["K_f"], "work_items": w["I_c"],
    }
    if not args.no_extras:
        log("plain device copy")
        out["copy"] = run_copy(torch, dev)
        log("forward alone")
        out["forward_only"] = run_forward_only(torch, tp, r, pargs, pyr, w, args.steps,
                                               None if args.no_cpu_baseline else sc)
        log("4096 points at 256x256")
        out["small"] = run_small_latency(torch, tp, scenes, args.steps, dev)
        log("the headline cloud in Morton order")
        out["ordered_input"] = run_ordered(torch, tp, scenes, sc, G, args.steps, args.warmup, dev)
    if not args.no_decoder:
        log("reconstruction network on the rendered pyramid")
        r.forward(*pargs, out=pyr)
        out["decoder"] = run_decoder(torch, tp, scenes, pyr, cam, nl, D, args.steps,
                                     args.warmup, dev, not args.no_cpu_baseline)
    if not args.no_coarser:
        log("coarser-layer inclusion on the same workload")
        out["coarser"] = run_coarser(torch, tp, sc, pargs, G, args.steps, args.warmup, dev, ms)
    del plan
    if not args.no_batched:
        log("batched vs per-view (16 views, 4M points, autotuned)")
        out["batched"] = run_batched(torch, tp, scenes, max(3, args.steps // 4),
                                     max(1, args.warmup // 2), dev,
                                     0 if args.no_cpu_baseline else 2)
        torch.cuda.empty_cache()
    if not args.no_8m:
        log("8M points at 1080p")
        out["points_8m"] = run_points_8m(torch, tp, scenes, max(3, args.steps // 2),
                                         max(1, args.warmup // 2), dev)
        torch.cuda.empty_cache()
    if not args.no_optim:
        log("optimisation loop (8M points, 8 views of 2560x1440, D = 8, oracle targets)")
        out["optimisation"] = run_optimisation(torch, tp, scenes, args.opt_iters,
                                               max(1, args.warmup // 2), dev)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, all host threads, median of 3; and one thread)")
        out["cpu_baseline"] = cpu_baseline(sc, Gnp)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
