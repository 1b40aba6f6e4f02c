#!/usr/bin/env python3
"""Labeling throughput on one MI355X.

One step = the whole labeling of one bond-percolation realization held in HBM:
init, the Algorithm-1 merge and the flatten (for the CSR path: the tile kernel,
the cross kernel and the flatten).  The headline workload is the periodic
triangle lattice L = 8192 (67,108,864 sites, 201,326,592 bonds) at p = 0.3473,
int32 half-CSR with a uint8 occupancy mask and int32 labels.

Prints ONE JSON line on stdout (everything else goes to stderr):
  value        labelled sites per second, Gsites/s (N / time per step)
  roofline     the dominant kernel's algorithmic bytes per launch / its mean
               launch time (HIP events on the launch stream), against 8 TB/s
  cpu_baseline the CPU oracle (sequential union-find, one core) on the same
               realization
  extra        the other workloads: honeycomb L=256, random 3-regular 2^24,
               the batched and per-instance schedules, serving latency.
"""
from __future__ import annotations

import argparse
import hashlib

import numpy as np
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "labelled sites/s (Gsites/s) + % HBM peak; batched vs per-launch; p99 latency"


# groups of extra measurements (--extras all runs them in this order)
EXTRA_GROUPS = ["probes", "slab", "fig7", "honeycomb", "batched", "serving", "monte_carlo", "rspan", "stats",
                "ell", "random3reg"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- bytes model
# Algorithmic bytes a kernel must move per launch (inputs read once, labels
# read / written once), independent of how many bytes the hardware moves.

def alg_bytes_csr(kernel: str, n: int, m: int) -> float:
    if kernel == "ccl_csr_tile":  # row_ptr + col + occ read, labels written
        return 4.0 * (n + 1) + 5.0 * m + 4.0 * n
    if kernel == "ccl_csr_cross":  # nothing the method itself must move
        return 0.0
    if kernel in ("ccl_flatten", "ccl_flatten_window", "ccl_flatten_grid"):  # labels read and written
        return 8.0 * n
    return 0.0


def alg_bytes_edges(kernel: str, n: int, m: int) -> float:
    if kernel == "ccl_init":
        return 4.0 * n
    if kernel == "ccl_merge_edges":  # src, dst, occ + one label read per site
        return 9.0 * m + 4.0 * n
    if kernel == "ccl_flatten":
        return 8.0 * n
    return 0.0


def path_bytes_csr(n: int, m: int) -> float:
    """Whole path: CSR inputs once + 16 B/site of label traffic."""
    return 4.0 * (n + 1) + 5.0 * m + 16.0 * n


def path_bytes_edges(n: int, m: int) -> float:
    return 9.0 * m + 16.0 * n


def kernel_source_hash() -> str:
    """Hash of what the CSR path's kernels are built from (csr.hip, the
    headers it includes, the build flags): counter figures taken on other
    sources are not reported."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_1603_08357_amd")
    csrc = os.path.join(pkg, "csrc")
    files = [os.path.join(csrc, "csr.hip")]
    files += sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith(".hpp"))
    files += [os.path.join(ROOT, "include", "ccl.h"), os.path.join(pkg, "build.py")]
    for path in files:
        with open(path, "rb") as fh:
            h.update(os.path.basename(path).encode() + fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """Measured HBM bytes per launch from the committed counter summary, or
    None when it is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    rec = d.get(workload, {}).get(kernel)
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


COPY_PROBE_BYTES = 1 << 30  # the copy probe reads and writes this much
KERNEL_NAMES = {"k_csr_tile": "ccl_csr_tile", "k_csr_tile_grid": "ccl_csr_tile", "k_csr_cross": "ccl_csr_cross",
                "k_ell_init": "ccl_ell_init", "k_ell_reduce": "ccl_ell_reduce",
                "k_sizes_own": "ccl_sizes_own", "k_sizes_foreign": "ccl_sizes_foreign",
                "k_flatten": "ccl_flatten", "k_flatten_window": "ccl_flatten_window",
                "k_flatten_grid": "ccl_flatten_grid",
                "k_init": "ccl_init", "k_merge_edges": "ccl_merge_edges"}


def ingest_counters(fetch_csv: str, write_csv: str, workload: str) -> dict:
    """Measured HBM bytes per launch from two rocprofv3 --pmc runs (FETCH_SIZE,
    then WRITE_SIZE, KiB per dispatch) of
        bench.py --steps 3 --warmup 1 --no-cpu-baseline --extras none --probe-copy
    each scaled by what the counter reads for the copy probe (known bytes),
    stored in profiles/traffic.json with the kernel-source hash."""
    import csv
    from collections import defaultdict

    def per_kernel(path, counter):
        vals = defaultdict(list)
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name", counter) != counter:
                    continue
                name = row["Kernel_Name"].split("(")[0].split("<")[0]
                name = name.replace("void ", "").replace("ccl::", "").strip()
                vals[name].append(float(row["Counter_Value"]) * 1024.0)
        return {k: sum(v) / len(v) for k, v in vals.items()}

    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    f_scale = COPY_PROBE_BYTES / fetch["k_probe_copy"]
    w_scale = COPY_PROBE_BYTES / write["k_probe_copy"]
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    rec = data.setdefault(workload, {})
    for k, pub in KERNEL_NAMES.items():
        if k in fetch and k in write:
            rec[pub] = {"fetch_bytes": round(fetch[k] * f_scale), "write_bytes": round(write[k] * w_scale),
                        "bytes_per_launch": round(fetch[k] * f_scale + write[k] * w_scale),
                        "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
                        "source_hash": kernel_source_hash()}
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    return rec


# ---------------------------------------------------------------- timing

_WORK_STREAM = []


def work_stream():
    """A stream of its own for the timed labelings (launches on the legacy
    default stream carry its implicit synchronization: 0.012-0.02 ms per
    three-kernel step on MI355X)."""
    import torch
    if not _WORK_STREAM:
        _WORK_STREAM.append(torch.cuda.Stream())
    return _WORK_STREAM[0]


def time_steps(fn, steps: int, warmup: int, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def step_distribution(fn, steps: int, stream, before=None):
    """Per-step HIP-event durations (ms): median, p99 and min.  `before`, if
    given, runs ahead of each step outside the events (a cache flush)."""
    import torch
    times = []
    for _ in range(steps):
        if before is not None:
            before()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    t = np.sort(np.asarray(times))
    return {"median": round(float(np.median(t)), 5), "p99": round(float(np.quantile(t, 0.99)), 5),
            "min": round(float(t[0]), 5), "steps": steps}


def make_flush(nbytes=1 << 30):
    """A 1 GiB device write that evicts the labels from L2 and the MALL,
    enqueued on the timed labelings' stream (so it ends before a step starts)."""
    import torch
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()

    def flush():
        with torch.cuda.stream(work_stream()):
            buf.fill_(1)
    return flush


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "cpu_count": os.cpu_count(), "usable_cpus": usable}


def traced_kernels(fn, steps: int):
    """Mean duration (ms) and launch count per kernel over `steps` steps."""
    import torch
    import paper_1603_08357_amd as ccl
    torch.cuda.synchronize()
    with ccl.trace() as rec:
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
    agg = {}
    for name, ms in rec:
        t, c = agg.get(name, (0.0, 0))
        agg[name] = (t + ms, c + 1)
    return {k: {"mean_ms": t / c, "launches": c, "total_ms": t} for k, (t, c) in agg.items()}


def roofline(kernels, bytes_fn, n, m, workload):
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    ab = bytes_fn(dom, n, m)
    achieved = ab / (kernels[dom]["mean_ms"] * 1e-3) / 1e9
    traffic = load_traffic(dom, workload)
    return {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "alg_bytes_per_launch": ab, "mean_launch_ms": round(kernels[dom]["mean_ms"], 5)}


# ---------------------------------------------------------------- workloads

def bench_csr(L, p, seed, steps, warmup, grid_width=0):
    import torch
    import gen
    import paper_1603_08357_amd as ccl
    t0 = time.perf_counter()
    g = gen.triangle_csr_realization(L, p, seed)
    log(f"generated triangle L={L} p={p}: {time.perf_counter() - t0:.1f}s")
    n, m = g.n_sites, len(g.col)
    rp = torch.from_numpy(g.row_ptr).cuda()
    col = torch.from_numpy(g.col).cuda()
    occ = torch.from_numpy(g.occ).cuda()
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = torch.empty(max(ccl.csr_workspace_bytes(n, m), 8), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()  # the inputs are resident before the first step
    stream = work_stream()
    fn = lambda: ccl.label_csr(rp, col, occ, out=out, workspace=ws, stream=stream, grid_width=grid_width)
    ms, wall = time_steps(fn, steps, warmup, stream)
    kern = traced_kernels(fn, steps)
    dist = step_distribution(fn, steps, stream)
    torch.cuda.synchronize()  # the labels are read on other streams afterwards
    return g, out, dict(n=n, m=m, ms=ms, wall=wall, kernels=kern, step_ms=dist)


def bench_edges(g, steps, warmup, cold=False):
    import torch
    import paper_1603_08357_amd as ccl
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    occ = torch.from_numpy(g.occ).cuda()
    out = torch.empty(g.n_sites, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()  # the inputs are resident before the first step
    stream = work_stream()
    fn = lambda: ccl.label(src, dst, g.n_sites, occ, out=out, stream=stream)
    ms, wall = time_steps(fn, steps, warmup, stream)
    kern = traced_kernels(fn, steps)  # ends with a device synchronization
    res = dict(n=g.n_sites, m=len(g.src), ms=ms, kernels=kern,
               n_clusters=int((out == torch.arange(g.n_sites, dtype=torch.int32, device="cuda")).sum().item()))
    if cold:  # warm: back to back; cold: a 1 GiB write ahead of every step
        res["warm_step_ms"] = step_distribution(fn, steps, stream)
        res["cold_step_ms"] = step_distribution(fn, steps, stream, before=make_flush())
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out, res


def bench_edges_monte_carlo(g, seed, steps, warmup):
    """Realizations per second on an edge list with the occupancy drawn on
    the device: a mask kernel (ccl_bernoulli) then ccl_label, against the draw
    inside the merge kernel (ccl_label_philox); both label the same draws."""
    import torch
    import gen
    import paper_1603_08357_amd as ccl
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    m = len(g.src)
    occ = torch.empty(m, dtype=torch.uint8, device="cuda")
    out = torch.empty(g.n_sites, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    k = [0]

    def masked():
        ccl.bernoulli(gen.mix_seed(seed, k[0]), gen.STREAM_OCC, m, g.p, out=occ, stream=stream)
        ccl.label(src, dst, g.n_sites, occ, out=out, stream=stream)
        k[0] += 1

    def drawn():
        ccl.label_philox(src, dst, g.n_sites, gen.mix_seed(seed, k[0]), gen.STREAM_OCC, g.p, out=out,
                         stream=stream)
        k[0] += 1

    res = {}
    for name, fn in (("mask_kernel", masked), ("drawn_in_merge", drawn)):
        ms, _ = time_steps(fn, steps, warmup, stream)
        kern = traced_kernels(fn, steps)
        res[name] = {"ms_per_realization": round(ms, 5), "realizations_per_s": round(1e3 / ms, 1),
                     "kernels": {k_: round(v["mean_ms"], 5) for k_, v in kern.items()}}
    ccl.bernoulli(gen.mix_seed(seed, 0), gen.STREAM_OCC, m, g.p, out=occ, stream=stream)
    ccl.label(src, dst, g.n_sites, occ, out=out, stream=stream)
    sep = out.clone()
    ccl.label_philox(src, dst, g.n_sites, gen.mix_seed(seed, 0), gen.STREAM_OCC, g.p, out=out, stream=stream)
    res["labels_equal_mask_path"] = bool(torch.equal(sep, out))
    return res


def bench_ell(nn, occ, steps, warmup):
    """ccl_label_ell on a (z_max, n) neighbour list already on the host."""
    import torch
    import paper_1603_08357_amd as ccl
    dnn = torch.from_numpy(nn).cuda()
    docc = torch.from_numpy(occ).cuda()
    out = torch.empty(nn.shape[1], dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    fn = lambda: ccl.label_ell(dnn, docc, out=out, stream=stream)
    ms, _ = time_steps(fn, steps, warmup, stream)
    kern = traced_kernels(fn, steps)
    res = {"ms_per_labeling": round(ms, 5), "Gsites_s": round(nn.shape[1] / (ms * 1e-3) / 1e9, 3),
           "kernels": {k: round(v["mean_ms"], 5) for k, v in kern.items()}}
    return out, res


def bench_ell_set(steps, warmup, shells=22):
    """The paper's own schedule on its neighbour-list form: the Cayley-tree
    experiment (z = 3, p_c = 1/2) in standard and random numbering at 0.5 and
    1.5 p_c, and the random 3-regular graph of 2^24 sites at p = 0.5."""
    import numpy as np
    import torch
    import gen
    import oracle
    res = {}
    for rp in (False, True):
        for p in (0.25, 0.75):
            t = gen.cayley_realization(shells, p, 7, rp)
            nn, oe = gen.ell_from_edges(t.n_sites, t.src, t.dst, t.occ, 3)
            out, r = bench_ell(nn, oe, steps, warmup)
            key = f"cayley_G{shells}_{'random' if rp else 'standard'}_p{p}"
            if rp and p == 0.75:
                r["labels_match_oracle"] = bool(np.array_equal(
                    out.cpu().numpy(), oracle.label_edges(t.n_sites, t.src, t.dst, t.occ)))
            res[key] = r
            del t, nn, oe, out
            torch.cuda.empty_cache()
    res["cayley_n_sites"] = gen.cayley_size(shells)
    a = res[f"cayley_G{shells}_random_p0.75"]["ms_per_labeling"]
    b = res[f"cayley_G{shells}_standard_p0.75"]["ms_per_labeling"]
    res["random_over_standard_at_1.5pc"] = round(a / b, 3)
    g = gen.bethe_random_regular(1 << 24, 3, 0.5, 3)
    nn, oe = gen.ell_from_edges(g.n_sites, g.src, g.dst, g.occ, 3)
    _, res["random3reg_2^24_p0.5"] = bench_ell(nn, oe, steps, warmup)
    return res


def bench_stats(lab_headline, steps, samples=32, L=512):
    """Cluster statistics on the GPU: the cost of sequential ids, sizes and
    the spanning test on the headline labeling, and the spanning probability
    R_span(p) of section 4 on cylinders (open top and bottom) of both
    lattices around their thresholds, from GPU labelings."""
    import numpy as np
    import torch
    import gen
    import paper_1603_08357_amd as ccl
    res = {}
    n = lab_headline.numel()
    side = int(round(n ** 0.5))
    top = torch.arange(side, dtype=torch.int32, device="cuda")
    bot = torch.arange(n - side, n, dtype=torch.int32, device="cuda")
    with ccl.trace() as rec:
        for _ in range(steps):
            ccl.cluster_ids(lab_headline)
            ccl.cluster_sizes(lab_headline)
            ccl.spans(lab_headline, top, bot)
        torch.cuda.synchronize()
    agg = {}
    for name, ms in rec:
        agg.setdefault(name, []).append(ms)
    res["headline_kernels_ms"] = {k: round(sum(v) / len(v), 5) for k, v in agg.items()}
    _, count = ccl.cluster_ids(lab_headline)
    res["headline_clusters"] = int(count.item())
    for kind, pc in (("triangle", 0.3473), ("honeycomb", 0.6527)):
        if kind == "triangle":
            src, dst = gen.triangle_edges(L)
            nn, wrap = L * L, gen.y_wrap_bonds_triangle(L)
            row = np.arange(nn) // L
        else:
            src, dst = gen.honeycomb_edges(L)
            nn, wrap = 2 * L * L, gen.y_wrap_bonds_honeycomb(L)
            row = (np.arange(nn) // 2) // L
        ds, dd = torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda()
        t = torch.from_numpy(np.nonzero(row == 0)[0].astype(np.int32)).cuda()
        b = torch.from_numpy(np.nonzero(row == L - 1)[0].astype(np.int32)).cuda()
        curve = {}
        for p in (round(pc - 0.02, 4), pc, round(pc + 0.02, 4)):
            hits = 0
            for k in range(samples):
                occ = gen.bernoulli(gen.mix_seed(1000 + k, 7), len(src), p)
                occ[wrap] = 0
                lab = ccl.label(ds, dd, nn, torch.from_numpy(occ).cuda())
                hits += int(ccl.spans(lab, t, b).item())
            curve[str(p)] = round(hits / samples, 4)
        res[f"R_span_{kind}_L{L}"] = {"n_sites": nn, "samples": samples, "R_span": curve}
    return res


def bench_monte_carlo_set(L, seed, steps, warmup):
    """bench_monte_carlo at the paper's three occupancies, 0.5, 1 and 1.5 p_c
    (section 4's timing runs); the p_c entry also checks the device draws."""
    return {f"p{p}": bench_monte_carlo(L, p, seed, steps, warmup) for p in (0.3473, 0.1736, 0.5209)}


def bench_monte_carlo(L, p, seed, steps, warmup):
    """Realizations per second of the headline workload with each
    realization's occupancy drawn on the device (ccl_bernoulli, the same
    Philox stream the host generator uses) before it is labelled: nothing
    crosses PCIe inside the loop.  `fused_draw`: the same realizations with
    the draw inside the tile kernel (ccl_label_csr_philox), no mask at all."""
    import numpy as np
    import torch
    import gen
    import paper_1603_08357_amd as ccl
    row_ptr, col = gen.triangle_csr(L)
    n, m = L * L, len(col)
    rp, dc = torch.from_numpy(row_ptr).cuda(), torch.from_numpy(col).cuda()
    occ = torch.empty(m, dtype=torch.uint8, device="cuda")
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = torch.empty(max(ccl.csr_workspace_bytes(n, m), 8), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    k = [0]

    def one():
        ccl.bernoulli(gen.mix_seed(seed, k[0]), gen.STREAM_OCC, m, p, out=occ, stream=stream)
        ccl.label_csr(rp, dc, occ, out=out, workspace=ws, stream=stream, grid_width=L)
        k[0] += 1

    def fused():
        ccl.label_csr_philox(rp, dc, gen.mix_seed(seed, k[0]), gen.STREAM_OCC, p, out=out,
                             workspace=ws, stream=stream, grid_width=L)
        k[0] += 1

    ms, _ = time_steps(one, steps, warmup, stream)
    kern = traced_kernels(one, steps)
    ms_f, _ = time_steps(fused, steps, warmup, stream)
    kern_f = traced_kernels(fused, steps)
    # the device draws what the host generator draws (a prefix, bit for bit)
    ccl.bernoulli(gen.mix_seed(seed, 0), gen.STREAM_OCC, m, p, out=occ, stream=stream)
    head = occ[: 1 << 22].cpu().numpy()
    same = bool(np.array_equal(head, gen.bernoulli(gen.mix_seed(seed, 0), 1 << 22, p)))
    # and the draw inside the tile kernel labels as the drawn mask does
    ccl.label_csr(rp, dc, occ, out=out, workspace=ws, stream=stream, grid_width=L)
    sep = out.clone()
    ccl.label_csr_philox(rp, dc, gen.mix_seed(seed, 0), gen.STREAM_OCC, p, out=out, workspace=ws,
                         stream=stream, grid_width=L)
    return {"ms_per_realization": round(ms, 5), "realizations_per_s": round(1e3 / ms, 1),
            "kernels": {k_: round(v["mean_ms"], 5) for k_, v in kern.items()},
            "device_mask_equals_host_generator": same,
            "fused_draw": {"ms_per_realization": round(ms_f, 5),
                           "realizations_per_s": round(1e3 / ms_f, 1),
                           "kernels": {k_: round(v["mean_ms"], 5) for k_, v in kern_f.items()},
                           "labels_equal_mask_path": bool(torch.equal(sep, out))}}


def crossing(ps, ra, rb, sa, sb):
    """The p where two R_span curves on the same p grid cross (linear
    interpolation of their difference at its sign change nearest the middle
    of the grid) and its standard error from the binomial errors of the two
    bracketing points."""
    import numpy as np
    d = np.asarray(rb) - np.asarray(ra)
    sig = np.sqrt(np.asarray(ra) * (1 - np.asarray(ra)) / sa + np.asarray(rb) * (1 - np.asarray(rb)) / sb)
    idx = [i for i in range(len(ps) - 1) if d[i] < 0 <= d[i + 1] or d[i] > 0 >= d[i + 1]]
    if not idx:
        return None, None
    mid = len(ps) // 2
    i = min(idx, key=lambda j: abs(j - mid))
    slope = (d[i + 1] - d[i]) / (ps[i + 1] - ps[i])
    if slope == 0:
        return None, None
    pc = ps[i] - d[i] / slope
    err = float(max(sig[i], sig[i + 1]) / abs(slope))
    return float(pc), err


def bench_rspan_crossing(samples, sizes=None):
    """Section 4, Figs. 5-6: R_span(p) on cylinders (open top and bottom,
    periodic sides) of four sizes per lattice, occupancy drawn on the device,
    labelled on the GPU (triangle: CSR with grid tiles; honeycomb: edge list),
    spanning tested on the device; p_c estimated where the curves of
    successive sizes cross, beside the paper's estimate and the exact
    value."""
    import math
    import numpy as np
    import torch
    import gen
    import paper_1603_08357_amd as ccl
    exact = {"triangle": 2 * math.sin(math.pi / 18), "honeycomb": 1 - 2 * math.sin(math.pi / 18)}
    paper = {"triangle": (0.3472, 0.0002), "honeycomb": (0.6527, 0.0002)}
    sizes = sizes or {"triangle": (512, 1024, 2048, 4096), "honeycomb": (256, 512, 1024, 2048)}
    offs = (-0.008, -0.006, -0.004, -0.003, -0.002, -0.001, -0.0005, 0.0, 0.0005, 0.001, 0.002, 0.003,
            0.004, 0.006, 0.008)
    res = {}
    for kind in ("triangle", "honeycomb"):
        pc0 = round(exact[kind], 4)
        ps = [round(pc0 + o, 5) for o in offs]
        curves = {}
        t0 = time.perf_counter()
        for L in sizes[kind]:
            if kind == "triangle":
                row_ptr, col = gen.triangle_csr(L)
                n, wrap = L * L, gen.y_wrap_bonds_triangle(L)
                row = np.arange(n) // L
                a, b = torch.from_numpy(row_ptr).cuda(), torch.from_numpy(col).cuda()
                m = len(col)
            else:
                src, dst = gen.honeycomb_edges(L)
                n, wrap = 2 * L * L, gen.y_wrap_bonds_honeycomb(L)
                row = (np.arange(n) // 2) // L
                a, b = torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda()
                m = len(src)
            dwrap = torch.from_numpy(np.nonzero(wrap)[0]).cuda()
            top = torch.from_numpy(np.nonzero(row == 0)[0].astype(np.int32)).cuda()
            bot = torch.from_numpy(np.nonzero(row == L - 1)[0].astype(np.int32)).cuda()
            occ = torch.empty(m, dtype=torch.uint8, device="cuda")
            lab = torch.empty(n, dtype=torch.int32, device="cuda")
            ws = torch.empty(max(ccl.csr_workspace_bytes(n, m), 8), dtype=torch.uint8, device="cuda")
            hits = torch.zeros(len(ps), dtype=torch.int32, device="cuda")
            for i, p in enumerate(ps):
                for r in range(samples):
                    ccl.bernoulli(gen.mix_seed(7000 + 97 * L + r, int(round(p * 1e5))), gen.STREAM_OCC, m, p,
                                  out=occ)
                    occ.index_fill_(0, dwrap, 0)
                    if kind == "triangle":
                        ccl.label_csr(a, b, occ, out=lab, workspace=ws, grid_width=L)
                    else:
                        ccl.label(a, b, n, occ, out=lab)
                    hits[i:i + 1] += ccl.spans(lab, top, bot)
            curves[L] = (hits.cpu().numpy() / samples).tolist()
            log(f"R_span {kind} L={L}: {time.perf_counter() - t0:.1f}s")
            del a, b, occ, lab, ws
            torch.cuda.empty_cache()
        Ls = list(sizes[kind])
        xs = []
        for L1, L2 in zip(Ls, Ls[1:]):
            pc, err = crossing(ps, curves[L1], curves[L2], samples, samples)
            xs.append({"sizes": [L1, L2], "p_cross": None if pc is None else round(pc, 5),
                       "stderr": None if err is None else round(err, 5)})
        good = [x for x in xs if x["p_cross"] is not None]
        est = float(np.mean([x["p_cross"] for x in good])) if good else None
        res[kind] = {"p": ps, "samples_per_point": samples,
                     "n_sites": {str(L): (L * L if kind == "triangle" else 2 * L * L) for L in Ls},
                     "R_span": {str(L): [round(v, 4) for v in curves[L]] for L in Ls},
                     "crossings": xs,
                     "p_c_estimate": None if est is None else round(est, 5),
                     "p_c_spread": round(float(np.std([x["p_cross"] for x in good])), 5) if len(good) > 1 else None,
                     "p_c_exact": round(exact[kind], 6),
                     "p_c_paper": {"value": paper[kind][0], "error": paper[kind][1]},
                     "seconds": round(time.perf_counter() - t0, 1)}
    return res


def probe_copy(nbytes=1 << 30):
    """One plain copy of known size: calibrates the traffic counters."""
    import torch
    import paper_1603_08357_amd as ccl
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    ccl.probe_copy(a, b)
    torch.cuda.synchronize()
    with ccl.trace() as rec:
        ccl.probe_copy(a, b)
        torch.cuda.synchronize()
    ms = rec[0][1]
    del a, b
    return {"bytes": 2 * nbytes, "ms": ms, "GBs": round(2 * nbytes / ms / 1e6, 1)}


def probe_random_access(table_len=1 << 24, n_ops=1 << 27):
    """Ceilings of scattered 4-byte accesses on a table the size of the random
    graphs' label array (2^24 int32 = 64 MiB): independent loads, device-scope
    atomicMin with the result discarded and used, and dependent-load chains
    (steps per second over all chains, with the chip full of chains)."""
    import torch
    import paper_1603_08357_amd as ccl
    table = torch.zeros(table_len, dtype=torch.int32, device="cuda")
    out = {"table_int32": table_len, "ops": n_ops}
    ccl.probe_random(table, 0, 4)  # hashed next-indices: the chase's table, gathered too
    for mode, name in ((3, "chase"), (0, "gather"), (1, "atomic_min"), (2, "atomic_min_ret")):
        ccl.probe_random(table, n_ops // 8, mode)  # warm-up
        torch.cuda.synchronize()
        with ccl.trace() as rec:
            ccl.probe_random(table, n_ops, mode)
            torch.cuda.synchronize()
        ms = rec[-1][1]
        out[name + "_Gops"] = round(n_ops / (ms * 1e-3) / 1e9, 2)
    del table
    return out


def random_access_roofline(g, rb, ceil):
    """The random graph's labeling against the random-access ceilings: at
    least two scattered label reads per occupied bond (merge), one atomicMin
    per join (N minus the number of clusters), and one scattered parent read
    per site (flatten); their ideal time at the probed rates beside the
    measured path."""
    import numpy as np
    occupied = int(np.count_nonzero(g.occ))
    n = g.n_sites
    joins = n - int(rb.get("n_clusters", 0)) if rb.get("n_clusters") else None
    reads = 2 * occupied + n
    t_reads = reads / (ceil["gather_Gops"] * 1e9)
    t_atom = (joins or 0) / (ceil["atomic_min_ret_Gops"] * 1e9)
    ideal_ms = (t_reads + t_atom) * 1e3
    return {"bound": "random-access", "scattered_reads": reads, "joins": joins,
            "ideal_ms": round(ideal_ms, 5), "measured_ms": round(rb["ms"], 5),
            "frac": round(ideal_ms / rb["ms"], 4)}


def upload_batch(specs, chunk=64):
    """Generate a batch instance by instance on the host (in chunks) and copy
    it into device arrays; host memory stays at one chunk."""
    import numpy as np
    import torch
    import gen
    site_off, bond_off = gen.batch_offsets(specs)
    m = int(bond_off[-1])
    src = torch.empty(m, dtype=torch.int32, device="cuda")
    dst = torch.empty(m, dtype=torch.int32, device="cuda")
    occ = torch.empty(m, dtype=torch.uint8, device="cuda")
    for a in range(0, len(specs), chunk):
        b = min(a + chunk, len(specs))
        lo, hi = int(bond_off[a]), int(bond_off[b])
        hs, hd, ho = np.empty(hi - lo, np.int32), np.empty(hi - lo, np.int32), np.empty(hi - lo, np.uint8)
        for k in range(a, b):
            x, y = int(bond_off[k]) - lo, int(bond_off[k + 1]) - lo
            gen.fill_instance(specs[k], hs[x:y], hd[x:y], ho[x:y])
        src[lo:hi].copy_(torch.from_numpy(hs))
        dst[lo:hi].copy_(torch.from_numpy(hd))
        occ[lo:hi].copy_(torch.from_numpy(ho))
    torch.cuda.synchronize()
    return site_off, bond_off, src, dst, occ


def check_all_instances(specs, site_off, bond_off, labels, chunk=64):
    """Every instance of the batch against the oracle: the GPU labels come
    back once; host tasks (all usable cores) each regenerate a chunk of
    instances, label it with the oracle and compare.  Returns the number of
    instances that differ (0: all bit-exact) and the seconds taken."""
    import concurrent.futures as cf
    import numpy as np
    import gen
    import oracle
    t0 = time.perf_counter()
    host = labels.cpu().numpy()
    so = np.asarray(site_off, np.int64)

    def task(a):
        b = min(a + chunk, len(specs))
        sub = specs[a:b]
        s_off, b_off, src, dst, occ = gen.batch_arrays(sub)
        want = oracle.label_batched(s_off, b_off, src, dst, occ, n_threads=1)
        got = host[int(so[a]):int(so[b])]
        bad = 0
        for k in range(b - a):
            if not np.array_equal(got[int(s_off[k]):int(s_off[k + 1])], want[int(s_off[k]):int(s_off[k + 1])]):
                bad += 1
        return bad

    threads = host_info()["usable_cpus"] or 1
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        bad = sum(ex.map(task, range(0, len(specs), chunk)))
    return bad, round(time.perf_counter() - t0, 1)


# the autotuner's search space for the benchmark's batch (a subset of
# autotune.DEFAULT_SPACE, so the search takes seconds; the result is cached)
BENCH_TUNE_SPACE = {"schedule": (3, 2), "block_threads": (256, 512), "blocks_per_cu": (2, 4),
                    "bonds_per_chunk": (65536, 262144), "sites_per_chunk": (32768,), "small_sites": (0,)}


def bench_batched(n_inst, base_seed, steps, warmup, check=True):
    """4096-instance mixed honeycomb / triangle batch: the plan's persistent
    kernel with the tuning the autotuner picks (and the library's defaults of
    each schedule beside it), captured in a graph and replayed, against one
    ccl_label call per instance on the same buffers."""
    import torch
    import gen
    import paper_1603_08357_amd as ccl
    from paper_1603_08357_amd import autotune
    t0 = time.perf_counter()
    specs = gen.batch_specs(n_inst, base_seed)
    site_off, bond_off, src, dst, occ = upload_batch(specs)
    n, m = int(site_off[-1]), int(bond_off[-1])
    log(f"batch of {n_inst}: {n} sites, {m} bonds, uploaded in {time.perf_counter() - t0:.1f}s")
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    res = {"instances": n_inst, "sites": n, "bonds": m,
           "resident_GB": round((9 * m + 4 * n) / 1e9, 2)}
    t0 = time.perf_counter()
    tuned = autotune.tune(site_off, bond_off, src, dst, occ, space=BENCH_TUNE_SPACE, reps=2)
    res["autotune"] = {"tuning": tuned, "seconds": round(time.perf_counter() - t0, 1),
                       "cache": autotune.cache_path()}
    log(f"autotuned batch tuning {tuned} in {res['autotune']['seconds']} s")
    for name, tuning in (("batched_tuned", tuned), ("batched_phased_default", dict(schedule=2)),
                         ("batched_fused_default", dict(schedule=1)), ("batched_tiled_default", dict(schedule=3))):
        plan = ccl.Plan(site_off, bond_off, tuning)
        with torch.cuda.stream(stream):
            plan.label(src, dst, occ, out=out, stream=stream)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            plan.label(src, dst, occ, out=out, stream=stream)
        torch.cuda.synchronize()
        ms, _ = time_steps(graph.replay, steps, warmup, torch.cuda.current_stream())
        rec = {"tuning": plan.tuning.as_dict(), "ms": round(ms, 4), "Gsites_s": round(n / (ms * 1e-3) / 1e9, 3),
               "path_hbm_frac": round(path_bytes_edges(n, m) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "plan_error": plan.check()}
        if check and name == "batched_tuned":
            bad, secs = check_all_instances(specs, site_off, bond_off, out)
            rec["all_instances_match_oracle"] = bad == 0
            rec["instances_differing"] = bad
            rec["oracle_check_s"] = secs
        kern = traced_kernels(lambda: plan.label(src, dst, occ, out=out), 2)
        rec["kernels"] = {k: round(v["mean_ms"], 4) for k, v in kern.items()}
        res[name] = rec
        plan.close()
        del graph
    base_steps = max(1, min(3, steps))
    fn = lambda: ccl.label_batched_per_instance(site_off, bond_off, src, dst, occ, out=out)
    ms, _ = time_steps(fn, base_steps, 1, torch.cuda.current_stream())
    res["per_instance"] = {"ms": round(ms, 4), "Gsites_s": round(n / (ms * 1e-3) / 1e9, 3),
                           "launches": 3 * n_inst}
    if check:
        bad, secs = check_all_instances(specs, site_off, bond_off, out)
        res["per_instance"]["all_instances_match_oracle"] = bad == 0
        res["per_instance"]["instances_differing"] = bad
    res["batched_speedup_vs_per_instance"] = round(ms / res["batched_tuned"]["ms"], 3)
    if check:
        res["cpu_oracle_threads"] = cpu_oracle_batched(specs)
    del src, dst, occ, out
    torch.cuda.empty_cache()
    return res


def serving_pool(count, base_seed, n_max=10_000_000):
    """Pre-generated request graphs (random z-regular, random position) in
    pinned host memory: generating a 10^7-site graph per request would
    dominate the run, so requests draw from this seeded pool."""
    import torch
    import gen
    reqs = gen.request_trace(count, 1.0, base_seed, n_max=n_max)
    pool = []
    for r in reqs:
        g = gen.request_graph(r)
        assert g.src.min() >= 0 and max(g.src.max(), g.dst.max()) < g.n_sites and g.dst.min() >= 0
        pins = tuple(torch.from_numpy(a).pin_memory() for a in (g.src, g.dst, g.occ))
        pool.append((r, g, pins))
    return pool


def make_jobs(pool, n_req, rate, seed):
    import gen
    from paper_1603_08357_amd.serving import Job
    u = gen.uniform(seed, gen.STREAM_TRACE, 2 * n_req).reshape(n_req, 2)
    jobs, t = [], 0.0
    for i in range(n_req):
        if rate is not None:
            t += -np.log(1.0 - u[i, 0]) / rate
        r, g, pins = pool[min(int(u[i, 1] * len(pool)), len(pool) - 1)]
        j = Job(i, t, g.n_sites, g.src, g.dst, g.occ)
        j.pinned = pins
        j.validated = True  # the pool's ids were checked when it was built
        j.graph = g
        jobs.append(j)
    return jobs


def bench_serving(pool_size, n_req, seed, budget_gb=64.0, slots=4096, n_streams=8, check=True):
    """Config 5: a saturation run (every request present at t = 0, so the
    64 GB budget binds) and Poisson arrivals at 0.5 / 0.8 / 0.95 of the
    saturated rate; small requests are admitted in batched ticks.  Every
    request's labels are compared with the oracle's labels of its graph."""
    import concurrent.futures as cf
    import torch
    import oracle
    from paper_1603_08357_amd.serving import GpuExecutor, Scheduler, latency_summary
    t0 = time.perf_counter()
    pool = serving_pool(pool_size, seed)
    log(f"serving pool of {pool_size} graphs in {time.perf_counter() - t0:.1f}s")
    ex = GpuExecutor(n_streams=n_streams, max_sites=max(g.n_sites for _, g, _ in pool))
    budget = int(budget_gb * 1e9)
    # warm-up: every pool graph once, alone and in a tick
    warm = make_jobs(pool, 2 * len(pool), None, seed + 1)
    Scheduler(ex, budget, slots).serve(warm)
    res = {"pool_graphs": pool_size, "slots": slots, "streams": n_streams, "budget_GB": budget_gb,
           "tick_limits": ex.tick_limits}
    runs = []
    # saturation: every request present at t = 0
    jobs = make_jobs(pool, n_req, None, seed + 2)
    sch = Scheduler(ex, budget, slots)
    t_a = time.perf_counter()
    sch.serve(jobs, t0=t_a)
    t_b = time.perf_counter()
    sat = latency_summary(jobs, t_a, t_b)
    sat.update(launches=sch.launches, ticks=sch.ticks, peak_admitted_GB=round(sch.peak_used / 1e9, 3),
               peak_jobs_in_flight=sch.peak_running)
    res["saturation"] = sat
    res["peak_admitted_GB"] = sat["peak_admitted_GB"]
    runs.append(jobs)
    rate_sat = sat["throughput_req_s"]
    n_load = max(1, n_req // 2)
    for frac in (0.5, 0.8, 0.95):
        jobs = make_jobs(pool, n_load, frac * rate_sat, seed + 3)
        sch = Scheduler(ex, budget, slots)
        t_a = time.perf_counter()
        sch.serve(jobs, t0=t_a)
        t_b = time.perf_counter()
        r = latency_summary(jobs, t_a, t_b)
        r.update(offered_req_s=round(frac * rate_sat, 2), launches=sch.launches, ticks=sch.ticks,
                 peak_admitted_GB=round(sch.peak_used / 1e9, 3))
        res[f"load_{frac}"] = r
        assert sch.peak_used <= budget
        runs.append(jobs)
    if check:
        # each request's labels equal the oracle's labels of its graph (the
        # pool's graphs labelled once each, on all host cores)
        graphs = {id(g): g for _, g, _ in pool}
        with cf.ThreadPoolExecutor(max_workers=host_info()["usable_cpus"] or 1) as tp:
            want = dict(zip(graphs, tp.map(lambda g: oracle.label_edges(g.n_sites, g.src, g.dst, g.occ),
                                           graphs.values())))
        bad = sum(not np.array_equal(want[id(j.graph)], j.labels) for jobs in runs for j in jobs)
        res["requests_checked"] = sum(len(jobs) for jobs in runs)
        res["all_requests_match_oracle"] = bad == 0
        res["requests_differing"] = bad
    del ex
    torch.cuda.empty_cache()
    return res


def cpu_oracle_batched(specs, count=256, seed=11):
    """The oracle's thread pool (one instance per task, all usable host cores)
    over a seeded sample of the batch's instances, generated on the host."""
    import gen
    import oracle
    u = gen.uniform(seed, gen.STREAM_SPEC, count)
    pick = sorted({min(int(x * len(specs)), len(specs) - 1) for x in u})
    sub = [specs[k] for k in pick]
    site_off, bond_off, src, dst, occ = gen.batch_arrays(sub)
    threads = host_info()["usable_cpus"] or 1
    t0 = time.perf_counter()
    oracle.label_batched(site_off, bond_off, src, dst, occ, n_threads=threads)
    dt = time.perf_counter() - t0
    n = int(site_off[-1])
    return {"value": round(n / dt / 1e9, 5), "unit": "Gsites/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sub)} seeded instances of the batch ({n} sites), {dt:.2f} s"}


def cpu_oracle_csr(g, reps=10):
    """The oracle on the headline realization, one host core, median of
    `reps` labelings (about a second each)."""
    import oracle
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        oracle.label_csr(g.n_sites, g.row_ptr, g.col, g.occ)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    return {"value": round(g.n_sites / dt / 1e9, 5), "unit": "Gsites/s", "cores": 1,
            "kind": "oracle",
            "sample": f"the full headline realization ({g.n_sites} sites), sequential union-find on one "
                      f"host core, median of {reps} labelings: {dt:.2f} s (min {min(times):.2f}, "
                      f"max {max(times):.2f}; {sum(times):.1f} s in all)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=8192)
    ap.add_argument("--p", type=float, default=0.3473)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", default="all",
                    help="all, none, or a comma list of: " + ",".join(EXTRA_GROUPS))
    ap.add_argument("--batch", type=int, default=4096, help="instances in the batched workload")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run the 1 GiB copy probe (counter calibration) when --extras none")
    ap.add_argument("--pool", type=int, default=24, help="graphs in the serving pool")
    ap.add_argument("--requests", type=int, default=10000,
                    help="requests of the serving saturation run (each load run takes half as many)")
    ap.add_argument("--rspan-samples", type=int, default=1000,
                    help="realizations per (size, p) point of the spanning-probability curves")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="store measured traffic from two rocprofv3 --pmc runs and exit")
    args = ap.parse_args()
    if args.ingest_counters:
        print(json.dumps(ingest_counters(*args.ingest_counters, f"triangle-csr L={args.L} p={args.p}"),
                         indent=1))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the labeling kernels run on a single MI355X "
              "and no multi-GPU path is built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import gen
    import paper_1603_08357_amd as ccl  # noqa: F401  (fails loudly without libccl.so)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    log(f"device: {torch.cuda.get_device_name(0)}")

    # the lattice's ids number its rows of L sites: grid tiles (ccl_label_csr_grid)
    g, out, r = bench_csr(args.L, args.p, args.seed, args.steps, args.warmup, grid_width=args.L)
    n, m = r["n"], r["m"]
    workload = f"triangle-csr L={args.L} p={args.p}"
    value = n / (r["ms"] * 1e-3) / 1e9
    path_gbs = path_bytes_csr(n, m) / (r["ms"] * 1e-3) / 1e9
    rl = roofline(r["kernels"], alg_bytes_csr, n, m, workload)

    # a sampled correctness check of the timed output (oracle on the host)
    extra = {"ms_per_step_traced": round(sum(k["total_ms"] for k in r["kernels"].values()) / args.steps, 5),
             "kernels": {k: round(v["mean_ms"], 5) for k, v in r["kernels"].items()},
             "path_alg_bytes": path_bytes_csr(n, m),
             "path_hbm_GBs": round(path_gbs, 1),
             "path_hbm_frac": round(path_gbs / HBM_PEAK_GBS, 4),
             "wall_s_timed": round(r["wall"], 4),
             "step_ms": r["step_ms"],
             "host": host_info()}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        want = None
        cpu = cpu_oracle_csr(g)
        want = oracle.label_csr(g.n_sites, g.row_ptr, g.col, g.occ)
        extra["labels_match_oracle"] = bool(np.array_equal(out.cpu().numpy(), want))
    del g

    if args.extras == "none" and args.probe_copy:
        extra["probe_copy"] = probe_copy()
    groups = EXTRA_GROUPS if args.extras == "all" else ([] if args.extras == "none" else args.extras.split(","))
    unknown = [g_ for g_ in groups if g_ not in EXTRA_GROUPS]
    if unknown:
        raise SystemExit(f"unknown --extras groups {unknown}; choose from {EXTRA_GROUPS}, all or none")

    def run(name, fn):
        if name in groups:
            try:
                fn()
            except Exception as e:  # an extra never takes the headline line down
                extra[name] = f"failed: {type(e).__name__}: {e}"

    def do_probes():
        extra["probe_copy"] = probe_copy()
        extra["probe_random_access"] = probe_random_access()
        # the headline path against the measured streaming ceiling as well as the nominal peak
        extra["path_frac_of_copy_ceiling"] = round(path_gbs / extra["probe_copy"]["GBs"], 4)

    def do_slab():  # the same labeling with slab tiles (65536 consecutive ids; ccl_label_csr)
        gs, outs, rs = bench_csr(args.L, args.p, args.seed, max(5, args.steps // 2), args.warmup)
        extra["slab_tiles"] = {"Gsites_s": round(rs["n"] / (rs["ms"] * 1e-3) / 1e9, 3),
                               "ms_per_step": round(rs["ms"], 5),
                               "kernels": {k: round(v["mean_ms"], 5) for k, v in rs["kernels"].items()},
                               "labels_equal_grid_tiles": bool(torch.equal(outs, out))}
        del gs, outs
        torch.cuda.empty_cache()

    def do_fig7():  # 0.5 p_c and 1.5 p_c of the same lattice
        for pp in (0.1736, 0.5209):
            gp, outp, rp_ = bench_csr(args.L, pp, args.seed, max(5, args.steps // 2), args.warmup,
                                      grid_width=args.L)
            extra[f"triangle_L{args.L}_p{pp}"] = {
                "Gsites_s": round(rp_["n"] / (rp_["ms"] * 1e-3) / 1e9, 3),
                "ms_per_step": round(rp_["ms"], 5), "step_ms": rp_["step_ms"],
                "kernels": {k: round(v["mean_ms"], 5) for k, v in rp_["kernels"].items()}}
            del gp, outp
            torch.cuda.empty_cache()

    def cpu_oracle_edges(g, reps=5):
        """The oracle on one core, median of `reps` labelings (ms)."""
        import oracle
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.label_edges(g.n_sites, g.src, g.dst, g.occ)
            times.append(time.perf_counter() - t0)
        return {"ms": round(1e3 * float(np.median(times)), 3), "cores": 1, "kind": "oracle",
                "sample": f"the same realization, median of {reps} labelings"}

    def do_honeycomb():
        h = gen.honeycomb_realization(256, 0.6527, 1)
        _, rh = bench_edges(h, max(args.steps, 50), args.warmup)
        extra["honeycomb_L256"] = {"Gsites_s": round(rh["n"] / (rh["ms"] * 1e-3) / 1e9, 3),
                                   "ms_per_step": round(rh["ms"], 5),
                                   "kernels": {k: round(v["mean_ms"], 5) for k, v in rh["kernels"].items()},
                                   "cpu_oracle": cpu_oracle_edges(h)}

    def do_random3reg():
        ceil = extra.get("probe_random_access")
        if not isinstance(ceil, dict):
            ceil = extra["probe_random_access"] = probe_random_access()
        for pp in (0.45, 0.5, 0.55):
            b = gen.bethe_random_regular(1 << 24, 3, pp, 3)
            _, rb = bench_edges(b, args.steps, args.warmup, cold=True)
            gbs = path_bytes_edges(rb["n"], rb["m"]) / (rb["ms"] * 1e-3) / 1e9
            row = {"Gsites_s": round(rb["n"] / (rb["ms"] * 1e-3) / 1e9, 3),
                   "ms_per_step": round(rb["ms"], 5), "path_hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                   "warm_step_ms": rb["warm_step_ms"], "cold_step_ms": rb["cold_step_ms"],
                   "kernels": {k: round(v["mean_ms"], 5) for k, v in rb["kernels"].items()},
                   "random_access_roofline": random_access_roofline(b, rb, ceil)}
            if pp == 0.5:
                row["cpu_oracle"] = cpu_oracle_edges(b)
            extra[f"random3reg_2^24_p{pp}"] = row
            if pp == 0.5:
                try:
                    extra["monte_carlo_random3reg_2^24_p0.5"] = bench_edges_monte_carlo(
                        b, 3, args.steps, args.warmup)
                except Exception as e:
                    extra["monte_carlo_random3reg_2^24_p0.5"] = f"failed: {type(e).__name__}: {e}"
            del b

    run("probes", do_probes)
    run("slab", do_slab)
    run("fig7", do_fig7)
    run("honeycomb", do_honeycomb)
    run("batched", lambda: extra.__setitem__("batched_4096", bench_batched(args.batch, 4, max(3, args.steps // 4), 1)))
    run("serving", lambda: extra.__setitem__("serving", bench_serving(args.pool, args.requests, 5)))
    run("monte_carlo", lambda: extra.__setitem__("monte_carlo",
                                                 bench_monte_carlo_set(args.L, args.seed, args.steps, args.warmup)))
    run("rspan", lambda: extra.__setitem__("R_span_crossing", bench_rspan_crossing(args.rspan_samples)))
    run("stats", lambda: extra.__setitem__("cluster_statistics", bench_stats(out, args.steps)))
    run("ell", lambda: extra.__setitem__("ell", bench_ell_set(args.steps, args.warmup)))
    run("random3reg", do_random3reg)

    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Gsites/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded Philox bond occupancy)",
        "config": {"workload": f"triangle lattice L={args.L} periodic, bond percolation p={args.p}, "
                               "int32 half-CSR + uint8 mask, int32 labels",
                   "n_sites": n, "n_bonds": m, "seed": args.seed, "grid_width": args.L},
        "roofline": rl,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
