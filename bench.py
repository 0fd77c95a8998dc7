#!/usr/bin/env python
"""Benchmark of the GAVIS visibility-field path on one MI355X.

One step = the whole hot path over one batch of synthetic input:
  vf_build over every training view (VF CONST), vf_query_views over every
  candidate view (VF QUERY), select_next_view (next-best view).
Metric: candidate-view uncertainty Mpix/s (candidate pixels / GPU time of
vf_query_views + select_next_view), with VF build ms and p50/p99 query
latency reported beside it.  Inputs are resident in HBM before timing.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU lane-operation slots per composited (pixel, Gaussian) pair, counted on
# the inner loops of the two blend kernels (a transcendental counts 4 slots).
# Algorithmic VALU issue slots per composited (pixel, Gaussian) pair.  The
# reported fraction counts a transcendental (exp2, log2) as 4 slots (quarter
# rate): VF CONST about 14 VALU ops + 1 exp = 18, VF QUERY about 20 VALU ops +
# exp + log = 28.  Itemised:
#   VF CONST: offsets 2, first factor 2, second factor 1, quadratic form 2,
#     overlap and termination tests 2, contribution select 1, alpha = o 2^-p
#     1 + exp, T update 1, sum of T 1, count 1                    = 14 + exp
#   VF QUERY: offsets to quadratic form 7, tests 2, alpha* = o' 2^-p + o0'
#     2 + exp, w* = alpha* T with select 2, x = v w* 1, log2 x with guard
#     1 + log, sum x log x 1, sums of x and w* 2, T update 1, count 1
#                                                                 = 20 + exp + log
VALU_SLOTS_PER_PAIR = {"raster_vis": 18.0, "raster_uq": 28.0}
# The same with transcendentals at the half rate measured on gfx950 (2 slots).
VALU_SLOTS_PER_PAIR_HALF_RATE_TRANS = {"raster_vis": 16.0, "raster_uq": 24.0}
# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz: VALU lane-operation issue rate.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def strip_comments(src: str) -> str:
    """C/C++ source without comments and blank space runs (string and
    character literals kept), so that comment edits leave the hash alone."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            i = src.find("\n", i)
            i = n if i < 0 else i
        elif src.startswith("/*", i):
            i = src.find("*/", i + 2)
            i = n if i < 0 else i + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """Hash of the library's sources, comments and spacing aside."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2605_30342_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            h.update(strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


TRAFFIC_PATH = ("profiles", "traffic.json")
# stages of a call, in launch order (the library's per-stage event names)
BINNING_STAGES = ("cull", "project", "sort_depth", "emit", "sort_tile", "ranges")
RADIX_KERNELS = ("k_radix_hist", "k_radix_scan", "k_radix_scatter")
SCAN_KERNELS = ("k_scan_reduce", "k_scan_blocks", "k_scan_down")


def _load_traffic():
    try:
        with open(os.path.join(ROOT, *TRAFFIC_PATH)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if not isinstance(t, dict) or t.get("source_hash") != kernel_source_hash():
        return None
    return t


def stage_traffic(workload: str, call: str):
    """HBM bytes per launch of every stage of one call ("build" or "query")
    of a workload, from the committed rocprofv3 counter summary, if it was
    taken on the current kernel sources; else None."""
    t = _load_traffic()
    if t is None:
        return None
    return t.get("workloads", {}).get(workload, {}).get(call)


def traffic_for(kernel: str):
    """HBM bytes per launch of a blend kernel on the room workload (the
    roofline kernel of the bench line), or None."""
    call = "build" if kernel == "raster_vis" else "query"
    st = stage_traffic("room", call)
    if not st or kernel not in st:
        return None
    e = st[kernel]
    return int(round((e["read"] + e["write"]) / max(e["launches"], 1)))


def _kernel_base(name: str) -> str:
    n = name.split("(")[0].split("<")[0].strip()
    n = n.split(" ")[-1]
    return n.split("::")[-1]


def label_stages(names):
    """Stage of every kernel of one call, from the launch order: the cull
    and its record scan, the projection, the depth sort, the instance scan
    and emission, the tile sort, the tile ranges, then the blend and what
    follows it."""
    out, state = [], "cull"
    for n in names:
        b = _kernel_base(n)
        if b == "k_project":
            state = "project"
        elif b in RADIX_KERNELS:
            state = "sort_depth" if state in ("project", "sort_depth") else "sort_tile"
        elif b in SCAN_KERNELS or b == "k_emit":
            if state not in ("cull",):
                state = "emit"
        elif b == "k_ranges":
            state = "ranges"
        elif b == "k_raster_vis":
            state = "raster_vis"
        elif b in ("k_vf_accum", "k_vis_logsum", "k_view_vis"):
            state = "vf_accum"
        elif b == "k_raster_uq":
            state = "raster_uq"
        elif b in ("k_scores", "k_argmax"):
            state = "scores"
        if b == "k_fill_u32" and state == "sort_depth":
            lab = "emit"            # the clear of the tile ranges
        elif b in ("k_fill_dev_u32", "k_convert", "__amd_rocclr_copyBuffer", "__amd_rocclr_fillBufferAligned"):
            lab = "other"
        else:
            lab = state
        out.append(lab)
    return out


def _read_csv(path, counter=None):
    import csv
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if counter is not None and r.get("Counter_Name") != counter:
                continue
            v = float(r["Counter_Value"]) if counter is not None else 0.0
            rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], v, int(r["Start_Timestamp"]),
                         int(r["End_Timestamp"])))
    rows.sort()
    return rows


def _last_calls(rows):
    """(build, query) dispatch slices: the last one-pass call that blends with
    k_raster_vis and the last that blends with k_raster_uq.  A call runs from
    the upload of its view table (the copy before its k_count) to the kernel
    before the next call's upload; a query's argmax, if any, belongs to it."""
    starts = []
    for i, r in enumerate(rows):
        if _kernel_base(r[1]) != "k_count":
            continue
        if i > 0 and _kernel_base(rows[i - 1][1]) == "k_fill_u32":     # the status words' clear
            i -= 1
        if i > 0 and "copyBuffer" in rows[i - 1][1]:                      # the view table's upload
            i -= 1
        starts.append(i)
    starts.append(len(rows))
    last = {}
    for j in range(len(starts) - 1):
        seg = rows[starts[j]:starts[j + 1]]
        while seg and not _kernel_base(seg[-1][1]).startswith("k_"):      # other work after the call
            seg = seg[:-1]
        names = {_kernel_base(r[1]) for r in seg}
        if "k_raster_vis" in names:
            last["build"] = seg
        elif "k_raster_uq" in names:
            # the timed form: not the variant that counts composited pairs
            # (k_raster_uq<batch, maps, count, ...>)
            uq = next(r[1] for r in seg if _kernel_base(r[1]) == "k_raster_uq")
            targs = uq.split("<", 1)[1].split(">", 1)[0].split(",") if "<" in uq else []
            if len(targs) < 3 or targs[2].strip() != "true":
                last["query"] = seg
    return last["build"], last["query"]


def summarize_counters(d: str, workload: str, copy_mib: int):
    """Per-stage HBM bytes of the last build and query of a profiled run:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch, two separate rocprofv3 --pmc
    runs) scaled so that the largest device copy of the run (copy_mib MiB)
    reads and writes copy_mib MiB, with the kernel-trace durations beside."""
    F = _read_csv(os.path.join(d, f"pmc_{workload}_FETCH_SIZE", "pm_counter_collection.csv"), "FETCH_SIZE")
    W = _read_csv(os.path.join(d, f"pmc_{workload}_WRITE_SIZE", "pm_counter_collection.csv"), "WRITE_SIZE")
    T = _read_csv(os.path.join(d, f"kt_{workload}", "kt_kernel_trace.csv"))
    cf = max(r[2] for r in F if "copyBuffer" in r[1])
    cw = max(r[2] for r in W if "copyBuffer" in r[1])
    fs, ws = copy_mib * 1024 / cf, copy_mib * 1024 / cw
    out = {"fetch_scale": round(fs, 4), "write_scale": round(ws, 4)}
    for call, f, w, t in zip(("build", "query"), _last_calls(F), _last_calls(W), _last_calls(T)):
        assert [_kernel_base(r[1]) for r in f] == [_kernel_base(r[1]) for r in w] == [_kernel_base(r[1]) for r in t]
        agg = {}
        for lab, rf, rw, rt in zip(label_stages([r[1] for r in f]), f, w, t):
            a = agg.setdefault(lab, {"read": 0.0, "write": 0.0, "launches": 0, "trace_ms": 0.0})
            a["read"] += rf[2] * 1024 * fs
            a["write"] += rw[2] * 1024 * ws
            a["trace_ms"] += (rt[4] - rt[3]) * 1e-6
            a["launches"] += 1
        for a in agg.values():
            a["read"], a["write"], a["trace_ms"] = int(a["read"]), int(a["write"]), round(a["trace_ms"], 4)
        out[call] = agg
    return out


def hbm_fractions(traffic, stage_ms):
    """Per stage and for the projection + binning stages together: bytes per
    call (counters) over the live per-call stage time, against 8 TB/s."""
    if not traffic:
        return None
    res, tb, tt = {}, 0.0, 0.0
    for k, e in traffic.items():
        if k not in stage_ms or not stage_ms[k]:
            continue
        b = e["read"] + e["write"]
        t = stage_ms[k] / 1e3
        res[k] = {"bytes": b, "ms": round(stage_ms[k], 4), "gb_s": round(b / t / 1e9, 1),
                  "frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}
        if k in BINNING_STAGES:
            tb += b
            tt += t
    if tt > 0:
        res["projection_and_binning"] = {"bytes": int(tb), "ms": round(tt * 1e3, 4), "gb_s": round(tb / tt / 1e9, 1),
                                         "frac": round(tb / tt / 1e9 / HBM_PEAK_GBS, 4)}
    return res


def query_valu(pairs, stages_q, query_ms):
    """VALU fraction of the query blend (its composited pairs at 28 slots each
    over its live launch time) and, time-weighted, of the whole query call
    (the same work over the call's time, projection and binning included)."""
    t = stages_q.get("raster_uq")
    if not t:
        return None
    a = pairs * VALU_SLOTS_PER_PAIR["raster_uq"] / (t / 1e3) / 1e12
    a2 = pairs * VALU_SLOTS_PER_PAIR_HALF_RATE_TRANS["raster_uq"] / (t / 1e3) / 1e12
    aw = pairs * VALU_SLOTS_PER_PAIR["raster_uq"] / (query_ms / 1e3) / 1e12
    return {"achieved": round(a, 3), "peak": round(VALU_PEAK_TOPS, 2), "frac": round(a / VALU_PEAK_TOPS, 4),
            "frac_transcendentals_at_half_rate": round(a2 / VALU_PEAK_TOPS, 4), "avg_launch_ms": round(t, 4),
            "pairs": int(pairs), "query_call_ms": round(query_ms, 4),
            "time_weighted_frac": round(aw / VALU_PEAK_TOPS, 4)}


def stage_times(ctx, fn, reps, torch):
    """Per-call live stage times (ms) of `fn` from the library's per-stage
    HIP events, recorded on the stream the kernels run on."""
    ctx.profile(True)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    st = ctx.profile_read()
    ctx.profile(False)
    return {k: ms / reps for k, (ms, n) in st.items() if n}


SERVING_SCENES = (   # name, Gaussians, rooms (x, y), storage
    ("s100k", 100_000, 1, 1, "f32"), ("room200k", 200_000, 1, 1, "f32"), ("s400k", 400_000, 1, 1, "bf16"),
    ("s700k", 700_000, 2, 1, "bf16"), ("s1m", 1_000_000, 2, 1, "f32"), ("s1500k", 1_500_000, 2, 1, "bf16"),
    ("s2m", 2_000_000, 2, 2, "f32"), ("s3m", 3_000_000, 2, 2, "bf16"))


def serving_bench(ctx, w, dsc, gamma, L, log, n_requests=300, rates=(50.0, 80.0, 300.0)):
    """Poisson stream of candidate-view requests over eight resident scenes
    (100k-3M Gaussians, FP32 and BF16 storage, prebuilt fields), each request
    16-512 views (log-uniform) of one class of 160x120 / 320x240 / 640x480:
    continuous batching (3 slots, same-scene merging, memory admission)
    against a plain queue (one slot, one request at a time), at Poisson rates
    below and above the device's capacity (about 150 requests/s here)."""
    import numpy as np
    import torch
    from paper_2605_30342_amd import scenes
    from paper_2605_30342_amd.api import DeviceScene
    from paper_2605_30342_amd.serve import GpuBackend, Server, replay
    resident, extents = {}, {}
    t0 = time.time()
    for i, (name, n, nx, ny, dt) in enumerate(SERVING_SCENES):
        if name == "room200k":
            resident[name] = (dsc, gamma, w.train.n)
            extents[name] = w.scene.extent
            continue
        sc = scenes.rooms_scene(n, nx, ny, seed=2100 + 100 * i)
        if dt != "f32":
            sc = scenes.subset_scene(sc, scenes.morton_order(sc))
        tr = scenes.ellipse_path_cameras(24, 2101 + 100 * i, 400, 400)
        d = DeviceScene(sc, dtype=dt)
        resident[name] = (d, ctx.vf_build(d, tr, L, gamma_dtype=dt), tr.n)
        extents[name] = sc.extent
    names = list(resident)
    classes = ((160, 120), (320, 240), (640, 480))
    pool = []
    rng = np.random.default_rng(77)
    for i in range(n_requests):
        nv = int(np.exp(rng.uniform(np.log(16), np.log(512))))
        wh = classes[int(rng.integers(0, 3))]
        sid = names[int(rng.integers(0, len(names)))]
        pool.append((sid, scenes.room_candidates(nv, 9000 + i, extents[sid], *wh)))
    torch.cuda.synchronize()
    budget = 48 << 30
    out = {"scenes": [f"{nm}:{n}:{dt}" for nm, n, _, _, dt in SERVING_SCENES], "requests": len(pool),
           "views": int(sum(c.n for _, c in pool)), "pixels": int(sum(c.pixels() for _, c in pool)),
           "memory_budget_gib": budget >> 30, "rates": {}}
    log(f"serving: {len(names)} scenes resident, {out['views']} views / {out['pixels'] / 1e6:.0f} Mpix in "
        f"{len(pool)} requests (setup {time.time() - t0:.1f}s)")
    backends = {}
    for label, slots in (("continuous_batching", 3), ("plain_queue", 1)):
        be = GpuBackend(ctx, n_slots=slots)
        for k, (d, g, nt) in resident.items():
            be.add_scene(k, d, g, L, nt)
        backends[label] = (be, slots)
    for rate in rates:                           # Poisson arrivals, requests per second
        rr = np.random.default_rng(int(rate))
        t, arrivals = 0.0, []
        for sid, cams in pool:
            t += rr.exponential(1.0 / rate)
            arrivals.append((t, sid, cams))
        res = {}
        for label, (be, slots) in backends.items():
            maxv = 512 if slots > 1 else 0
            replay(Server(be, memory_budget=budget, n_slots=slots, max_batch_views=maxv), arrivals[:8])
            torch.cuda.synchronize()
            s0, r0 = be.exact_sizings, be.relaunches
            st = replay(Server(be, memory_budget=budget, n_slots=slots, max_batch_views=maxv), arrivals,
                        timeout=600.0)
            st["exact_sizings"], st["overflow_relaunches"] = be.exact_sizings - s0, be.relaunches - r0
            st["offered_views_per_s"] = sum(c.n for _, _, c in arrivals) / arrivals[-1][0]
            res[label] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
            log(f"serving rate {rate:.0f}/s {label}: {res[label]}")
        out["rates"][str(int(rate))] = res
    return out


def _seen_counts(cams, means, znear=0.2):
    """Per camera, how many of the points project inside its image in front of
    the near plane."""
    import numpy as np
    out = []
    m = means.astype(np.float64)
    for i in range(cams.n):
        p = m @ cams.R[i].astype(np.float64).T + cams.t[i].astype(np.float64)
        z = p[:, 2]
        ok = z > znear
        u = cams.K[i, 0] * p[ok, 0] / z[ok] + cams.K[i, 2]
        v = cams.K[i, 1] * p[ok, 1] / z[ok] + cams.K[i, 3]
        out.append(int(np.sum((u >= 0) & (u < cams.wh[i, 0]) & (v >= 0) & (v < cams.wh[i, 1]))))
    return np.array(out)


def precision_subset_errors(ctx, w, L, log, n_sub=10_000, n_views=16, n_train=8):
    """Per-map error of the FP32, FP16 and BF16 storage paths against the FP64
    oracle on the original FP32 inputs (storage and arithmetic together) on
    a 10k-Gaussian spatial subset of the three-million-Gaussian scene: a run
    of the Morton-ordered scene (a compact patch), its field built by the
    oracle from the training views that see most of it, and the maps of the
    candidate views that see most of it.  Per map: the L1 error relative to
    the map's L1 norm, the largest pixel error relative to the map's largest
    value, and the score error; the median and the worst over the maps."""
    import numpy as np
    import torch
    import oracle
    from paper_2605_30342_amd import scenes
    from paper_2605_30342_amd.api import DeviceScene
    F = lambda x: float(np.float32(x))  # noqa: E731   the GPU's float32 parameters
    prm = oracle.Params(kappa=F(w.kappa), eps_T=F(1e-4), znear=F(0.2), lowpass=F(0.3), cut=F(9.0), beta=F(0.5),
                        o0=F(0.15))
    i0 = w.scene.n // 2 - n_sub // 2
    sub = scenes.subset_scene(w.scene, np.arange(i0, i0 + n_sub))
    tr = w.train.subset(list(np.argsort(-_seen_counts(w.train, sub.means), kind="stable")[:n_train]))
    seen = _seen_counts(w.cand, sub.means)
    order = np.argsort(-seen, kind="stable")[:n_views]
    cd = w.cand.subset(list(order))
    b = oracle.vf_build(sub, tr, L, prm)
    g32 = b["gamma"].astype(np.float32)
    q = oracle.vf_query(sub, g32.astype(np.float64), L, tr.n, cd, prm)
    ref, sizes = q["maps_flat"], [m.size for m in q["maps"]]
    out = {"subset": f"Gaussians {i0}..{i0 + n_sub - 1} of the Morton-ordered scene; field of {tr.n} training "
                     f"views; {cd.n} candidate views 320x240 seeing {int(seen[order].min())}-"
                     f"{int(seen[order].max())} of the subset's centres",
           "flagged_px": round(float(q["flags_flat"].mean()), 6)}
    for dt, td in (("f32", torch.float32), ("f16", torch.float16), ("bf16", torch.bfloat16)):
        d = DeviceScene(sub, dtype=dt)
        gt = torch.from_numpy(np.ascontiguousarray(g32.T)).to(td).cuda()
        sc, mp = ctx.vf_query_views(d, gt, L, tr.n, cd, want_maps=True)
        torch.cuda.synchronize()
        a, s_gpu = mp.double().cpu().numpy(), sc.double().cpu().numpy()
        l1, mx, off = [], [], 0
        for n in sizes:
            bb, aa = ref[off:off + n], a[off:off + n]
            l1.append(np.abs(aa - bb).sum() / max(np.abs(bb).sum(), 1e-300))
            mx.append(np.abs(aa - bb).max() / max(np.abs(bb).max(), 1e-300))
            off += n
        srel = np.abs(s_gpu - q["scores"]) / np.abs(q["scores"])
        out[dt] = {k: {"median": float(np.median(v)), "worst": float(np.max(v))}
                   for k, v in (("map_rel_l1", l1), ("map_max_err_over_max", mx), ("score_rel", srel))}
    log(f"precision per-map errors vs FP64 on the subset {out}")
    return out


def batched_bench(ctx, uprm, timed, log):
    """Batched workload at full size: 1M Gaussians in two rooms, VF build over
    300 training views 1280x720 (50 views per pass), and 256 candidates of
    mixed 160x120 / 320x240 / 640x480 queried one call per view, in one call
    and as one graph replay."""
    import torch
    from paper_2605_30342_amd import _lib, scenes
    from paper_2605_30342_amd.api import DeviceScene
    t0 = time.time()
    w = scenes.workload("batched")
    L = w.sh_degree
    from paper_2605_30342_amd.autotune import Autotuner
    saved = ctx.get_tuning()
    tuner = Autotuner(ctx)
    d = DeviceScene(w.scene)
    vp = _lib.default_vf_params(sh_degree=L, kappa=w.kappa, views_per_pass=50)
    wsb = ctx.build_workspace(d, w.train, vp)
    g = torch.empty(((L + 1) ** 2, w.scene.n), dtype=torch.float32, device="cuda")
    tuner.tune_build(d, w.train, vp, wsb, g, reps=1, rounds=2)
    build_ms = timed(lambda: ctx.vf_build(d, w.train, L, vp, wsb, g), reps=2)
    wsq = ctx.query_workspace(d, w.cand, uprm, L)
    sc = torch.empty(w.cand.n, dtype=torch.float32, device="cuda")
    tuner.tune_query(d, g, L, w.train.n, w.cand, uprm, wsq)
    q_ms = timed(lambda: ctx.vf_query_views(d, g, L, w.train.n, w.cand, uprm, wsq, scores=sc))
    gprm = _lib.default_uq_params(use_graph=1)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g_ms = timed(lambda: ctx.vf_query_views(d, g, L, w.train.n, w.cand, gprm, wsq, scores=sc))
    torch.cuda.synchronize()
    singles = [w.cand.subset([v]) for v in range(w.cand.n)]
    one = torch.empty(1, dtype=torch.float32, device="cuda")

    def plain():
        for c in singles:
            ctx.vf_query_views(d, g, L, w.train.n, c, uprm, wsq, scores=one)
    p_ms = timed(plain, reps=2)

    def plain_graph():       # one replay per view (one captured graph per image size)
        for c in singles:
            ctx.vf_query_views(d, g, L, w.train.n, c, gprm, wsq, scores=one)
    with torch.cuda.stream(side):
        pg_ms = timed(plain_graph, reps=2)
    torch.cuda.synchronize()
    st, _ = ctx.check_workspace(wsq)
    assert st == 0, "batched workload: query workspace overflow"
    stages = stage_times(ctx, lambda: ctx.vf_query_views(d, g, L, w.train.n, w.cand, uprm, wsq, scores=sc), 3, torch)
    ctx.vf_query_views(d, g, L, w.train.n, w.cand, _lib.default_uq_params(count_pairs=1), wsq, scores=sc)
    _, cnt = ctx.check_workspace(wsq)
    px = w.cand.pixels()
    out = {"workload": f"batched: {w.scene.n} Gaussians, {w.train.n} training views 1280x720, {w.cand.n} "
                       f"candidates of mixed 160x120/320x240/640x480 ({px} px), SH degree {L}",
           "vf_build_ms": round(build_ms, 3), "query_ms": round(q_ms, 4), "mpix_s": round(px / (q_ms / 1e3) / 1e6, 3),
           "graph_replay_ms": round(g_ms, 4), "plain_per_view_ms": round(p_ms, 4),
           "plain_per_view_graph_replay_ms": round(pg_ms, 4),
           "speedup_batched_vs_plain": round(p_ms / q_ms, 3), "speedup_graph_vs_plain": round(p_ms / g_ms, 3),
           "query_stages_ms": {k: round(v, 4) for k, v in stages.items()},
           "query_records": cnt[0], "query_instances": cnt[1],
           "raster_uq_roofline": query_valu(cnt[3], stages, q_ms),
           "hbm": hbm_fractions(stage_traffic("batched", "query"), stages),
           "schedules": {"tuning": ctx.get_tuning(), "table": tuner.table}}
    ctx.set_tuning(**saved)
    log(f"batched workload {out} (setup and runs {time.time() - t0:.1f}s)")
    del wsb, wsq, g, d
    torch.cuda.empty_cache()
    return out


def precision_bench(ctx, uprm, timed, log):
    """Precision workload at full size: 3M Gaussians (Morton ordered) in a 2x2
    grid of rooms, field built in FP32 from 300 training views 640x480, then
    512 candidates 320x240 queried with the scene and field stored in FP32,
    FP16 and BF16 (FP32 arithmetic, FP32 depth keys and 2D inversion)."""
    import torch
    from paper_2605_30342_amd import _lib, scenes
    from paper_2605_30342_amd.api import DeviceScene
    t0 = time.time()
    w = scenes.workload("precision")
    L = w.sh_degree
    d32 = DeviceScene(w.scene)
    vp = _lib.default_vf_params(sh_degree=L, kappa=w.kappa, views_per_pass=100)
    wsb = ctx.build_workspace(d32, w.train, vp)
    g32 = ctx.vf_build(d32, w.train, L, vp, wsb)
    del wsb
    px = w.cand.pixels()
    out = {"workload": f"precision: {w.scene.n} Gaussians, {w.train.n} training views 640x480, {w.cand.n} "
                       f"candidates 320x240 ({px} px), SH degree {L}"}
    ws = ctx.query_workspace(d32, w.cand, uprm, L)
    s32 = torch.empty(w.cand.n, dtype=torch.float32, device="cuda")
    from paper_2605_30342_amd.autotune import Autotuner
    saved = ctx.get_tuning()
    tuner = Autotuner(ctx)
    tuner.tune_query(d32, g32, L, w.train.n, w.cand, uprm, ws, reps=1, rounds=2)
    t32 = timed(lambda: ctx.vf_query_views(d32, g32, L, w.train.n, w.cand, uprm, ws, scores=s32))
    stages = stage_times(ctx, lambda: ctx.vf_query_views(d32, g32, L, w.train.n, w.cand, uprm, ws, scores=s32), 3,
                         torch)
    ctx.vf_query_views(d32, g32, L, w.train.n, w.cand, _lib.default_uq_params(count_pairs=1), ws, scores=s32)
    _, cnt = ctx.check_workspace(ws)
    ctx.vf_query_views(d32, g32, L, w.train.n, w.cand, uprm, ws, scores=s32)
    out["f32"] = {"query_ms": round(t32, 4), "mpix_s": round(px / (t32 / 1e3) / 1e6, 3),
                  "scene_bytes": d32.nbytes() + g32.numel() * 4,
                  "query_stages_ms": {k: round(v, 4) for k, v in stages.items()},
                  "query_records": cnt[0], "query_instances": cnt[1],
                  "raster_uq_roofline": query_valu(cnt[3], stages, t32),
                  "hbm": hbm_fractions(stage_traffic("precision", "query"), stages)}
    for dt in ("f16", "bf16"):
        dh = DeviceScene(w.scene, dtype=dt)
        gh = g32.to(torch.float16 if dt == "f16" else torch.bfloat16)
        wsh = ctx.query_workspace(dh, w.cand, uprm, L)
        sh = torch.empty_like(s32)
        t_ms = timed(lambda: ctx.vf_query_views(dh, gh, L, w.train.n, w.cand, uprm, wsh, scores=sh))
        torch.cuda.synchronize()
        rel = ((sh.double() - s32.double()).abs() / s32.double().abs())
        out[dt] = {"query_ms": round(t_ms, 4), "mpix_s": round(px / (t_ms / 1e3) / 1e6, 3),
                   "max_rel_score_diff_vs_f32": float(rel.max().item()),
                   "median_rel_score_diff_vs_f32": float(rel.median().item()),
                   "scene_bytes": dh.nbytes() + gh.numel() * gh.element_size()}
        # the view whose score moves most: its maps in both storages, to show
        # whether the score's change comes from the map or from cancellation
        # of positive and negative pixel terms in the sum
        v = int(torch.argmax(rel).item())
        one = w.cand.subset([v])
        ws1 = ctx.query_workspace(d32, one, uprm, L)
        _, m32 = ctx.vf_query_views(d32, g32, L, w.train.n, one, uprm, ws1, want_maps=True)
        ws1h = ctx.query_workspace(dh, one, uprm, L)
        _, mh = ctx.vf_query_views(dh, gh, L, w.train.n, one, uprm, ws1h, want_maps=True)
        # the same view with only the field in the half type, and with only
        # the Gaussian attributes in it: which storage moves the map
        _, mg = ctx.vf_query_views(d32, gh, L, w.train.n, one, uprm, ws1, want_maps=True)
        _, ma = ctx.vf_query_views(dh, g32, L, w.train.n, one, uprm, ws1h, want_maps=True)
        torch.cuda.synchronize()
        m32, mh, mg, ma = m32.double(), mh.double(), mg.double(), ma.double()
        l1 = lambda m: float(((m - m32).abs().sum() / m32.abs().sum()).item())  # noqa: E731
        out[dt]["worst_view"] = {"view": v, "score_rel_diff": float(rel[v].item()), "map_rel_l1_diff": l1(mh),
                                 "map_rel_l1_diff_field_only": l1(mg), "map_rel_l1_diff_attributes_only": l1(ma),
                                 "sum_abs_H_over_abs_score": float((m32.abs().sum() / m32.sum().abs()).item())}
        del dh, gh, wsh, ws1, ws1h, m32, mh, mg, ma
    out["schedules"] = {"tuning": ctx.get_tuning(), "table": tuner.table}
    ctx.set_tuning(**saved)
    out["per_map_error_vs_fp64"] = precision_subset_errors(ctx, w, L, log)
    log(f"precision workload {out} (setup and runs {time.time() - t0:.1f}s)")
    del ws, g32, d32
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="room")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-views", type=int, default=16, help="candidate views the CPU baseline runs")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-exact", action="store_true", help="skip the exact-visibility validation mode")
    ap.add_argument("--no-color", action="store_true", help="skip the per-Gaussian colour covariance query")
    ap.add_argument("--no-configs", action="store_true", help="skip the batched and precision workloads")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default blend batch sizes instead of tuning them on this workload")
    ap.add_argument("--profile-only", action="store_true",
                    help="only the timed steps (for counter collection): no batching/precision/serving sections")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a device copy of this size (HBM counter calibration under rocprofv3)")
    ap.add_argument("--serving-requests", type=int, default=300)
    ap.add_argument("--serving-rates", default="50,80,300", help="Poisson arrival rates, requests per second")
    ap.add_argument("--cpu-build-views", type=int, default=4, help="training views the CPU baseline's build runs")
    ap.add_argument("--counters-summary", metavar="DIR", default=None,
                    help="no GPU work: reduce rocprofv3 runs under DIR (kt_<w>/, pmc_<w>_FETCH_SIZE/, "
                         "pmc_<w>_WRITE_SIZE/ for each workload of --counters-workloads, each a --profile-only run "
                         "with --calib-copy-mib) to per-stage HBM bytes in profiles/traffic.json")
    ap.add_argument("--counters-workloads", default="room,batched,precision")
    args = ap.parse_args()
    if args.counters_summary:
        doc = {"_about": "HBM bytes per call and stage of the last build and query of a --profile-only run: "
                         "rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per dispatch, separate passes) scaled so that "
                         "the run's device copy of --calib-copy-mib MiB reads and writes that many bytes; "
                         "trace_ms from the kernel trace of the same command.  Valid for the kernel sources "
                         "whose hash (comments and spacing aside) is given; bench.py reports null otherwise.",
               "command": "cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --stats --output-format csv "
                          "-d DIR/kt_<w> -o kt -- python3 bench.py --workload <w> --steps 3 --warmup 1 "
                          "--profile-only --no-autotune; then for C in FETCH_SIZE WRITE_SIZE: "
                          "timeout -s KILL 300 rocprofv3 --pmc $C --output-format csv -d DIR/pmc_<w>_$C -o pm -- "
                          f"python3 bench.py --workload <w> --steps 2 --warmup 1 --profile-only --no-autotune "
                          f"--calib-copy-mib {args.calib_copy_mib or 256}; then python3 bench.py "
                          "--counters-summary DIR",
               "source_hash": kernel_source_hash(), "workloads": {}}
        for wl in [x for x in args.counters_workloads.split(",") if x]:
            if not os.path.isdir(os.path.join(args.counters_summary, f"kt_{wl}")):
                continue
            doc["workloads"][wl] = summarize_counters(args.counters_summary, wl, args.calib_copy_mib or 256)
        with open(os.path.join(ROOT, *TRAFFIC_PATH), "w") as f:
            json.dump(doc, f, indent=1)
        print(json.dumps({k: list(v) for k, v in doc["workloads"].items()}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(across GPUs the query would be split by candidate view and the build's fields summed)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2605_30342_amd import _lib, scenes
    from paper_2605_30342_amd.api import Context, DeviceScene

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    t_setup = time.time()
    w = scenes.workload(args.workload)
    L = w.sh_degree
    log(f"workload {w.name}: {w.scene.n} Gaussians, {w.train.n} training views {tuple(w.train.wh[0])}, "
        f"{w.cand.n} candidates, {w.cand.pixels()} candidate px, L={L}")
    ctx = Context(0)
    dsc = DeviceScene(w.scene)
    vprm = _lib.default_vf_params(sh_degree=L, kappa=w.kappa)
    uprm = _lib.default_uq_params()
    ws_b = ctx.build_workspace(dsc, w.train, vprm)
    ws_q = ctx.query_workspace(dsc, w.cand, uprm, L)
    K = (L + 1) ** 2
    gamma = torch.empty((K, w.scene.n), dtype=torch.float32, device="cuda")
    scores = torch.empty(w.cand.n, dtype=torch.float32, device="cuda")
    log(f"workspaces: build {ws_b.nbytes / 2**20:.1f} MiB (R={ws_b.plan.max_records}, "
        f"M={ws_b.plan.max_instances}); query {ws_q.nbytes / 2**20:.1f} MiB (R={ws_q.plan.max_records}, "
        f"M={ws_q.plan.max_instances}); setup {time.time() - t_setup:.1f}s")

    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    lat = []

    def step(i=None):
        if i is not None:
            ev[i][0].record(stream)
        ctx.vf_build(dsc, w.train, L, vprm, ws_b, gamma)
        if i is not None:
            ev[i][1].record(stream)
        ctx.vf_query_views(dsc, gamma, L, w.train.n, w.cand, uprm, ws_q, scores=scores)
        if i is not None:
            ev[i][2].record(stream)
        best = ctx.select_next_view(scores)      # device argmax, copy to the host, synchronise
        if i is not None:
            ev[i][3].record(stream)
        return best

    step()
    # batch sizes of the two blends, chosen by timing each candidate on this
    # workload (outputs checked equal across candidates)
    tuning = ctx.get_tuning()
    if not args.no_autotune:
        from paper_2605_30342_amd.autotune import Autotuner
        tuner = Autotuner(ctx)
        tuner.tune_build(dsc, w.train, vprm, ws_b, gamma)
        tuner.tune_query(dsc, gamma, L, w.train.n, w.cand, uprm, ws_q)
        tuning = ctx.get_tuning()
        log(f"autotuned blend batches: {tuning} ({tuner.table})")
    for _ in range(args.warmup):
        step()
    st, cnt_b = ctx.check_workspace(ws_b)
    assert st == 0, "build workspace overflow"
    st, cnt_q = ctx.check_workspace(ws_q)
    assert st == 0, "query workspace overflow"

    # timed region: whole steps, no per-stage events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        best = step(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # query latency of one request (all candidates of the workload): from the
    # call on an idle device to the selected view on the host
    for _ in range(max(20, args.steps)):
        torch.cuda.synchronize()
        tq = time.perf_counter()
        ctx.vf_query_views(dsc, gamma, L, w.train.n, w.cand, uprm, ws_q, scores=scores)
        ctx.select_next_view(scores)
        lat.append((time.perf_counter() - tq) * 1e3)
    # per-call stage times of the build and of the query: the same calls again
    # with HIP events around every stage, recorded on the stream the kernels
    # run on
    stages_b = stage_times(ctx, lambda: ctx.vf_build(dsc, w.train, L, vprm, ws_b, gamma), args.steps, torch)
    stages_q = stage_times(ctx, lambda: ctx.vf_query_views(dsc, gamma, L, w.train.n, w.cand, uprm, ws_q,
                                                           scores=scores), args.steps, torch)
    build_ms = [ev[i][0].elapsed_time(ev[i][1]) for i in range(args.steps)]
    query_ms = [ev[i][1].elapsed_time(ev[i][2]) for i in range(args.steps)]
    qsel_ms = [ev[i][1].elapsed_time(ev[i][3]) for i in range(args.steps)]
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    px = w.cand.pixels()
    # the headline rate: candidate pixels over the GPU time of the query and
    # the next-best-view selection (argmax on the device, index to the host)
    mpix_s = px * args.steps / (sum(qsel_ms) / 1e3) / 1e6
    log(f"step {ms_per_step:.3f} ms; build {np.median(build_ms):.3f} ms; query {np.median(query_ms):.3f} ms; "
        f"query + select {np.median(qsel_ms):.3f} ms; {mpix_s:.1f} Mpix/s; best view {best}")
    for nm, stg in (("build", stages_b), ("query", stages_q)):
        for k, ms in stg.items():
            log(f"  {nm} stage {k:11s} {ms:9.4f} ms per call")

    # algorithmic pair counts of the two blends
    pairs_vis = cnt_b[3]
    cprm = _lib.default_uq_params(count_pairs=1)
    ctx.vf_query_views(dsc, gamma, L, w.train.n, w.cand, cprm, ws_q, scores=scores)
    _, cnt_c = ctx.check_workspace(ws_q)
    pairs_uq = cnt_c[3]
    log(f"pairs: build {pairs_vis:.3e}, query {pairs_uq:.3e}")

    # dominant kernel of the step and its roofline (the build is one pass
    # here, so a call's stage time is one launch)
    per_call = {k: stages_b.get(k, 0.0) + stages_q.get(k, 0.0) for k in set(stages_b) | set(stages_q)}
    dom = max(per_call, key=per_call.get)
    roof = None
    if dom in VALU_SLOTS_PER_PAIR:
        pairs = pairs_vis if dom == "raster_vis" else pairs_uq
        t = per_call[dom] / 1e3
        achieved = pairs * VALU_SLOTS_PER_PAIR[dom] / t / 1e12
        roof = {"kernel": f"k_{dom}", "bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "TOP/s (VALU lane-ops)", "frac": round(achieved / VALU_PEAK_TOPS, 4),
                "traffic": traffic_for(dom), "avg_launch_ms": round(per_call[dom], 4),
                "units_per_launch": int(pairs), "per_unit": f"{VALU_SLOTS_PER_PAIR[dom]:.0f} VALU slots per pair",
                "frac_transcendentals_at_half_rate": round(
                    pairs * VALU_SLOTS_PER_PAIR_HALF_RATE_TRANS[dom] / t / 1e12 / VALU_PEAK_TOPS, 4)}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": None, "traffic": None, "avg_launch_ms": round(per_call[dom], 4)}
    # the query blend's own fraction (the query's roofline target is stated on it)
    # and the whole query's, with all its stages' time in the denominator
    uq_frac = query_valu(pairs_uq, stages_q, float(np.median(query_ms)))
    # HBM fractions of every stage and of projection + binning, per call
    hbm = {"build": hbm_fractions(stage_traffic(w.name, "build"), stages_b),
           "query": hbm_fractions(stage_traffic(w.name, "query"), stages_q)}

    # a plain device copy of known size, to scale HBM byte counters taken
    # under rocprofv3 (only when asked for)
    if args.calib_copy_mib:
        n = args.calib_copy_mib * 2**20 // 4
        a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
    if args.profile_only:
        print(json.dumps({"build_stages_ms": stages_b, "query_stages_ms": stages_q,
                          "pairs": [int(pairs_vis), int(pairs_uq)]}), flush=True)
        ctx.close()
        return

    # batching: the same candidates as one call per view (plain form), as one
    # call for all views, and as one replay of the captured graph
    def timed(fn, reps=5):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        cur = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(cur)
        for _ in range(reps):
            fn()
        e1.record(cur)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    singles = [w.cand.subset([v]) for v in range(w.cand.n)]
    one = torch.empty(1, dtype=torch.float32, device="cuda")

    def plain():
        for c in singles:
            ctx.vf_query_views(dsc, gamma, L, w.train.n, c, uprm, ws_q, scores=one)
    gprm = _lib.default_uq_params(use_graph=1)
    side = torch.cuda.Stream()
    plain_ms = timed(plain)
    batched_ms = timed(lambda: ctx.vf_query_views(dsc, gamma, L, w.train.n, w.cand, uprm, ws_q, scores=scores))

    def plain_graph():       # the per-view form, each call a replay (views differ only in pose)
        for c in singles:
            ctx.vf_query_views(dsc, gamma, L, w.train.n, c, gprm, ws_q, scores=one)
    with torch.cuda.stream(side):
        graph_ms = timed(lambda: ctx.vf_query_views(dsc, gamma, L, w.train.n, w.cand, gprm, ws_q, scores=scores))
        plain_graph_ms = timed(plain_graph)
    torch.cuda.synchronize()
    batching = {"plain_per_view_ms": round(plain_ms, 4), "batched_call_ms": round(batched_ms, 4),
                "graph_replay_ms": round(graph_ms, 4), "plain_per_view_graph_replay_ms": round(plain_graph_ms, 4),
                "speedup_batched_vs_plain": round(plain_ms / batched_ms, 3),
                "speedup_graph_vs_plain": round(plain_ms / graph_ms, 3),
                "speedup_per_view_graph_vs_plain": round(plain_ms / plain_graph_ms, 3)}
    log(f"batching {batching}")

    # the paper's image geometry: the same scene and field seen by 64
    # candidates of 512x512 (90 degrees), as one call and as one call per
    # view (the form in which uncertainty maps are timed per view)
    paper_geometry = None
    if not args.no_configs:
        wc = scenes.workload("ctx512")
        ws_c = ctx.query_workspace(dsc, wc.cand, uprm, L)
        s_c = torch.empty(wc.cand.n, dtype=torch.float32, device="cuda")
        c_ms = timed(lambda: ctx.vf_query_views(dsc, gamma, L, w.train.n, wc.cand, uprm, ws_c, scores=s_c))
        singles_c = [wc.cand.subset([v]) for v in range(wc.cand.n)]

        def plain_c():
            for c in singles_c:
                ctx.vf_query_views(dsc, gamma, L, w.train.n, c, uprm, ws_c, scores=one)
        pc_ms = timed(plain_c, reps=3)
        pxc = wc.cand.pixels()
        paper_geometry = {"workload": f"room scene and field, {wc.cand.n} candidates 512x512 (90 deg FOV)",
                          "query_ms": round(c_ms, 4), "mpix_s": round(pxc / (c_ms / 1e3) / 1e6, 3),
                          "views_per_s": round(wc.cand.n / (c_ms / 1e3), 1),
                          "one_call_per_view_ms": round(pc_ms, 4),
                          "views_per_s_one_call_per_view": round(wc.cand.n / (pc_ms / 1e3), 1),
                          "paper_reference": "uncertainty maps at about 200 views/s (192.6-251.5 FPS over its four "
                                             "datasets, one view per call) on an NVIDIA A40, scenes of other sizes"}
        del ws_c, s_c
        log(f"paper geometry {paper_geometry}")

    # the batched and precision workloads at full size (the launch
    # configurations of those workloads; figures reported beside the room line)
    batched_cfg = precision = None
    if not args.no_configs:
        batched_cfg = batched_bench(ctx, uprm, timed, log)
        precision = precision_bench(ctx, uprm, timed, log)

    # validation mode: the exact multi-view visibility (O(|P|) per record) in
    # place of the field's AM-GM query, and the score gap between the two
    exact = None
    if not args.no_exact:
        vis_v, centres = ctx.view_visibility(dsc, w.train, vprm, ws_b)
        vv_ms = timed(lambda: ctx.view_visibility(dsc, w.train, vprm, ws_b), reps=3)
        s_ex = torch.empty_like(scores)
        ex_ms = timed(lambda: ctx.vf_query_views_exact(dsc, vis_v, centres, w.kappa, w.cand, uprm, ws_q,
                                                       scores=s_ex), reps=3)
        ctx.vf_query_views(dsc, gamma, L, w.train.n, w.cand, uprm, ws_q, scores=scores)
        torch.cuda.synchronize()
        se, sq = s_ex.double().cpu().numpy(), scores.double().cpu().numpy()
        gap = np.abs(sq - se) / np.abs(se)
        b_sh, b_ex = int(np.argmax(sq)), int(np.argmax(se))
        exact = {"view_visibility_ms": round(vv_ms, 4), "exact_query_ms": round(ex_ms, 4),
                 "max_rel_score_gap_sh_vs_exact": float(gap.max()),
                 "median_rel_score_gap_sh_vs_exact": float(np.median(gap)),
                 "best_view_sh": b_sh, "best_view_exact": b_ex,
                 "exact_rank_of_sh_choice": int((se > se[b_sh]).sum()),
                 "exact_score_ratio_of_sh_choice": float(se[b_sh] / se[b_ex])}
        del vis_v, centres, s_ex
        log(f"exact validation {exact}")

    # per-Gaussian colour covariance from colour SH-coefficient variances
    # (degree 3, the 3DGS colour degree) in place of the constant Q_c
    color = None
    if not args.no_color:
        cvar = torch.from_numpy(scenes.color_sh_variances(w.scene.n, 3, 5001)).cuda()
        s_c = torch.empty_like(scores)
        c_ms = timed(lambda: ctx.vf_query_views_color(dsc, gamma, L, w.train.n, cvar, w.cand, uprm, ws_q,
                                                      scores=s_c))
        torch.cuda.synchronize()
        color = {"query_ms": round(c_ms, 4), "mpix_s": round(px / (c_ms / 1e3) / 1e6, 3),
                 "constant_covariance_query_ms": round(batched_ms, 4),
                 "best_view": int(torch.argmax(s_c).item()), "color_sh_degree": 3}
        # expected-depth maps beside the entropy maps (the depth eq. id's
        # correction takes), against the entropy maps alone
        mbuf = torch.empty(2 * px, dtype=torch.float32, device="cuda")
        m_ms = timed(lambda: ctx.vf_query_views(dsc, gamma, L, w.train.n, w.cand, uprm, ws_q, scores=s_c,
                                                want_maps=True, maps=mbuf))
        d_ms = timed(lambda: ctx.vf_query_views(dsc, gamma, L, w.train.n, w.cand, uprm, ws_q, scores=s_c,
                                                maps=mbuf, want_depth=True))
        uprm.write_maps, uprm.write_depth = 0, 0
        color["maps_query_ms"] = round(m_ms, 4)
        color["maps_and_depth_query_ms"] = round(d_ms, 4)
        del cvar, s_c, mbuf
        log(f"colour covariance / depth {color}")

    serving = None
    if not args.no_serving:
        serving = serving_bench(ctx, w, dsc, gamma, L, log, n_requests=args.serving_requests,
                                rates=tuple(float(x) for x in args.serving_rates.split(",")))


    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        prm = oracle.Params()
        nb = max(1, min(args.cpu_build_views, w.train.n))
        tr = w.train.subset([int(round(k * (w.train.n - 1) / max(nb - 1, 1))) for k in range(nb)])
        sub = w.cand.subset(list(range(min(args.cpu_views, w.cand.n))))
        # the oracle's own field (its input never comes from the GPU path) over
        # a few of the training views, timed as the VF build sample
        tc = time.perf_counter()
        bo = oracle.vf_build(w.scene, tr, L, prm)
        dt_b = time.perf_counter() - tc
        g = bo["gamma"]
        tc = time.perf_counter()
        qo = oracle.vf_query(w.scene, g, L, tr.n, sub, prm, want_maps=False)
        dt = time.perf_counter() - tc
        pairs_cpu = int(qo["stats"][0])
        cpu = {"value": round(sub.pixels() / dt / 1e6, 4), "unit": "Mpix/s", "cores": oracle.num_threads(),
               "kind": "oracle", "sample": f"VF QUERY of {sub.n} of the {w.cand.n} candidate views "
                                          f"({sub.pixels()} px, full scene, field of {tr.n} training views), "
                                          f"{dt:.1f} s; VF build over {tr.n} training views, {dt_b:.1f} s",
               "pairs": pairs_cpu, "pairs_per_s": round(pairs_cpu / dt, 1),
               "vf_build_sample_s": round(dt_b, 3), "vf_build_pairs": int(bo["stats"][0]),
               "vf_build_ms_extrapolated_to_all_views": round(dt_b / tr.n * w.train.n * 1e3, 1)}
        # the GPU on the same work: the same FP32-rounded field and views,
        # timed, with its composited pairs counted
        gdev = torch.from_numpy(np.ascontiguousarray(g.astype(np.float32).T)).cuda()
        ws_s = ctx.query_workspace(dsc, sub, uprm, L)
        s_b = torch.empty(sub.n, dtype=torch.float32, device="cuda")
        g_ms = timed(lambda: ctx.vf_query_views(dsc, gdev, L, tr.n, sub, uprm, ws_s, scores=s_b))
        ctx.vf_query_views(dsc, gdev, L, tr.n, sub, cprm, ws_s, scores=s_b)
        _, cnt_s = ctx.check_workspace(ws_s)
        torch.cuda.synchronize()
        rel = np.abs(s_b.double().cpu().numpy() - qo["scores"]) / np.abs(qo["scores"])
        cpu["gpu_same_work"] = {"query_ms": round(g_ms, 4), "mpix_s": round(sub.pixels() / (g_ms / 1e3) / 1e6, 1),
                                "pairs": int(cnt_s[3]), "pairs_per_s": round(cnt_s[3] / (g_ms / 1e3), 1),
                                "max_rel_score_error_vs_oracle": float(rel.max())}
        del ws_s, gdev
        log(f"cpu baseline {cpu}")

    out = {
        "metric": "candidate-view uncertainty Mpix/s + VF build ms; p50/p99 query latency",
        "value": round(mpix_s, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.scene.n} Gaussians, {w.train.n} training views "
                               f"{w.train.wh[0][0]}x{w.train.wh[0][1]} (VF build), {w.cand.n} candidate views "
                               f"{w.cand.wh[0][0]}x{w.cand.wh[0][1]}, SH degree {L}, kappa {w.kappa}",
                   "gaussians": w.scene.n, "train_views": w.train.n, "candidate_views": w.cand.n,
                   "candidate_pixels": px, "sh_degree": L, "blend_batches": tuning},
        "vf_build_ms": round(float(np.median(build_ms)), 4),
        "query_ms": round(float(np.median(query_ms)), 4),
        "p50_query_latency_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_query_latency_ms": round(float(np.percentile(lat, 99)), 4),
        "query_select_ms": round(float(np.median(qsel_ms)), 4),
        "build_stages_ms": {k: round(v, 4) for k, v in stages_b.items()},
        "query_stages_ms": {k: round(v, 4) for k, v in stages_q.items()},
        "hbm": hbm,
        "pairs": {"raster_vis": int(pairs_vis), "raster_uq": int(pairs_uq)},
        "records": {"build": cnt_b[0], "query": cnt_q[0]},
        "instances": {"build": cnt_b[1], "query": cnt_q[1]},
        "roofline": roof,
        "raster_uq_roofline": uq_frac,
        "batching": batching,
        "paper_geometry": paper_geometry,
        "batched_workload": batched_cfg,
        "precision": precision,
        "serving": serving,
        "exact_validation": exact,
        "color_covariance_and_depth": color,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
