"""Benchmark of the FGraft harvest on one MI355X.

A step is one whole build on the GloVe-shaped workload (n = 1,183,514 unit
float32 rows of d = 100, cosine distance; T=8 trees, B=8 blocks, ef_h=128,
R=64, alpha=1.2): scaffold, 8 x (harvest + merge), finalize.  The reported
value is harvest distance evaluations per second (evaluations summed over
the timed builds / harvest kernel time from HIP events on the build's
stream); build seconds, the recall@10 ladder of the built graph and the
roofline of the harvest kernel are reported beside it, with the
SIFT-shaped uint8 and GIST-shaped d = 960 builds as extra keys.  The data
is synthetic (seeded mixtures) and resident in HBM before the timed
region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2609_30493_amd import datagen as gen  # noqa: E402
from paper_2609_30493_amd import fgraft as F  # noqa: E402

HBM_PEAK_GBS = 8000.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_beam_harvest_u8_1M_pmc.md")


def measured_traffic(path=PMC_SUMMARY):
    """Bytes per harvest launch from a committed counter summary, or None
    when there is none or the beam kernel's source changed since the
    counters were taken."""
    import hashlib
    if path is None:
        return None
    try:
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith(("|", "#", "`")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        src = b"".join(open(os.path.join(ROOT, "paper_2609_30493_amd", "csrc", f), "rb").read()
                       for f in ("fg_beam.h", "fg_device.h"))
        if hashlib.sha256(src).hexdigest()[:16] != kv.get("kernel_source_sha256_16"):
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def ground_truth_u8(xd: torch.Tensor, qd: torch.Tensor, k: int):
    """Exact k-NN distances for uint8 rows: every quantity is an integer
    below 2^24, so float32 products and sums are exact."""
    xf = xd.float()
    xn = (xf * xf).sum(1)
    out = []
    for s in range(0, qd.shape[0], 256):
        qf = qd[s:s + 256].float()
        d = (qf * qf).sum(1)[:, None] + xn[None, :] - 2.0 * (qf @ xf.T)
        out.append(torch.topk(d, k, dim=1, largest=False).values)
    return torch.cat(out)


def recall_ladder(data, G, ws, qd, true_d, k=10, target=0.95):
    res = []
    nq = qd.shape[0]
    for L in (10, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512):
        oi = torch.empty(nq, k, dtype=torch.int32, device="cuda")
        od = torch.empty(nq, k, dtype=torch.int32, device="cuda")
        oe = torch.empty(nq, dtype=torch.int32, device="cuda")
        F.search(data, G, qd, k, L, oi, od, oe, ws)
        torch.cuda.synchronize()
        found = od.cpu().numpy().view(np.uint32).astype(np.float64)
        rec = float(np.mean(found <= true_d[:, -1:]))
        res.append(dict(L=L, recall=rec, evals_per_query=float(oe.cpu().numpy().mean())))
        if rec >= target:
            break
    return res


def cpu_baseline(w, n_sample: int, threads: int):
    """The oracle (plain C, untuned), whole build on a prefix-sized sample of
    the same recipe and parameters; harvest evaluations per second."""
    from oracle import fgo
    x = gen.workload_data(w, n_sample)
    P = fgo.params(w.T, w.ef_h, w.R, w.alpha, w.B, 0, threads)
    t0 = time.perf_counter()
    G = fgo.build_graph(fgo.Data(x, metric="cosine" if w.metric == "cosine" else "l2"), w.build_seed, P)
    wall = time.perf_counter() - t0
    c = G["counters"]
    return {"value": c["harvest_evals"] / c["t_harvest"], "unit": "dist-evals/s",
            "cores": threads, "kind": "oracle",
            "sample": f"whole oracle build (scaffold, {w.B} blocks, finalize) on the first n={n_sample} "
                      f"points of the same {w.recipe} recipe, T={w.T} B={w.B} ef_h={w.ef_h} R={w.R}; "
                      f"{c['harvest_evals'] / n_sample:.0f} harvest evaluations per point; "
                      f"{wall:.1f} s wall, build {c['t_scaffold'] + c['t_harvest'] + c['t_merge'] + c['t_finalize']:.2f} s"}


def dsweep(args):
    """Tab. 5 re-measured (Sec. 5.4): adaptive cost per evaluation (the harvest of a
    whole build, T=8 B=8 ef_h=128 R=64) against blocked cost per pair (every
    point's 64 nearest inside leaves of 2048 consecutive points on matrix
    cores, float32 and bfloat16 operands), n = 200,000 power-law rows
    truncated to each d."""
    n = args.n or 200_000
    out = []
    all_dims = (32, 64, 128, 256, 512, 960)
    dims = [int(v) for v in args.dims.split(",")] if args.dims else list(all_dims)
    for d in dims:
        i = all_dims.index(d)  # the draw's seed follows d's place in the full sweep
        x = gen.powerlaw_f32(n, d, 500, 40 + i, d_total=960)
        xd = torch.from_numpy(x).cuda()
        data = F.make_data(xd)
        params = F.make_params(8, 128, 64, 1.2, 8)
        ws = F.alloc_workspace(data, params)
        u32 = lambda *sh: torch.full(sh, -1, dtype=torch.int32, device="cuda")  # noqa: E731
        G = F.make_graph(u32(n, 64), u32(n), u32(n), u32(8), 8)
        F.build_graph(data, 42, params, G, ws, timings=True)
        c, t = F.build_graph(data, 42, params, G, ws, timings=True)
        del ws
        rec = {"d": d, "n": n, "harvest_evals": c["harvest_evals"], "harvest_ms": t["harvest_ms"],
               "adaptive_ns_per_eval": t["harvest_ms"] * 1e6 / c["harvest_evals"],
               "build_ms": sum(t[k] for k in ("scaffold_ms", "harvest_ms", "merge_ms", "finalize_ms"))}
        S, R = 2048, 64
        pairs = sum(min(S, n - l0) ** 2 for l0 in range(0, n, S))
        oi = torch.empty(n, R, dtype=torch.int32, device="cuda")
        od = torch.empty(n, R, dtype=torch.float32, device="cuda")
        for bf16 in (False, True):
            lws = F.leaf_knn(data, S, R, bf16, oi, od)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            reps = 3
            for _ in range(reps):
                F.leaf_knn(data, S, R, bf16, oi, od, lws)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            key = "bf16" if bf16 else "fp32"
            rec[f"blocked_{key}_ms"] = ms
            rec[f"blocked_{key}_ns_per_pair"] = ms * 1e6 / pairs
            rec[f"blocked_{key}_tflops"] = pairs * 2 * d / (ms / 1e3) / 1e12
        rec["W_fp32"] = rec["adaptive_ns_per_eval"] / rec["blocked_fp32_ns_per_pair"]
        log(f"[dsweep] {json.dumps(rec)}")
        out.append(rec)
        del xd, data, G
        torch.cuda.empty_cache()
    ds = np.log([r["d"] for r in out])
    fit = {k: float(np.polyfit(ds, np.log([r[k] for r in out]), 1)[0])
           for k in ("adaptive_ns_per_eval", "blocked_fp32_ns_per_pair", "blocked_bf16_ns_per_pair", "W_fp32")
           } if len(out) >= 2 else None
    print(json.dumps({"mode": "dsweep", "n": n, "rows": out, "loglog_exponents": fit}), flush=True)


def wsweep(args):
    """Throughput against working set (Sec. 5.2's prefix table): whole builds of
    prefixes of one GloVe-shaped matrix (d = 100, unit rows, cosine, T=8 B=8
    ef_h=128 R=64), from a few MB (inside the L2s and the Infinity Cache) to
    past the 256 MB Infinity Cache, each beside the blocked kernel on the same
    prefix (every point's 64 nearest inside leaves of 2048 consecutive rows on
    matrix cores, squared L2 on the unit rows: the same Gram work).  The
    prefixes are slices of one draw, so every smaller set is a true prefix of
    the larger ones.  With --sweep-workload u8 the same over the 128-byte
    uint8 rows of the benchmark line's workload (T=8 B=8 ef_h=64 R=32, its
    1024-slot visited table), 250,000 to 4,000,000 rows (32 to 512 MB), the
    blocked kernel on a float32 copy of the rows.  With --sweep-workload gist
    the GIST-shaped float32 rows (d = 960, 3840 B, T=8 B=8 ef_h=128 R=64),
    25,000 to 1,000,000 rows (96 MB to 3.8 GB)."""
    w = {"u8": gen.SIFT_1M, "gist": gen.GIST_1M}.get(args.sweep_workload, gen.GLOVE_1183514)
    default = {id(gen.SIFT_1M): [250_000, 500_000, 1_000_000, 2_000_000, 4_000_000],
               id(gen.GIST_1M): [25_000, 50_000, 100_000, 200_000, 500_000, 1_000_000]}.get(
        id(w), [20_000, 50_000, 100_000, 200_000, 500_000, w.n])
    sizes = [int(v) for v in args.sizes.split(",")] if args.sizes else default
    metric = "cosine" if w.metric == "cosine" else "l2"
    table = 1024 if w is gen.SIFT_1M else 0
    N = max(sizes)
    log(f"[wsweep] generating {N} x {w.d} rows ({w.recipe})")
    x = gen.workload_data(w, N)
    xd_all = torch.from_numpy(x).cuda()
    row_bytes = xd_all.stride(0) * xd_all.element_size()
    out = []
    for n in sorted(sizes):
        xd = xd_all[:n]
        data = F.make_data(xd, metric)
        params = F.make_params(w.T, w.ef_h, w.R, w.alpha, w.B, beam_table_slots=table)
        ws = F.alloc_workspace(data, params)
        u32 = lambda *sh: torch.full(sh, -1, dtype=torch.int32, device="cuda")  # noqa: E731
        G = F.make_graph(u32(n, w.R), u32(n), u32(n), u32(w.T), w.T)
        F.build_graph(data, w.build_seed, params, G, ws, timings=True)
        runs = [F.build_graph(data, w.build_seed, params, G, ws, timings=True) for _ in range(args.reps)]
        c = runs[0][0]
        hms = float(np.median([t["harvest_ms"] for _, t in runs]))
        bms = float(np.median([sum(t[k] for k in ("scaffold_ms", "harvest_ms", "merge_ms", "finalize_ms"))
                               for _, t in runs]))
        rate = c["harvest_evals"] / (hms / 1e3)
        rec = {"n": n, "MB": n * row_bytes / 1e6, "harvest_evals": c["harvest_evals"], "harvest_ms": hms,
               "build_ms": bms, "harvest_G_evals_per_s": rate / 1e9,
               "evals_per_point": c["harvest_evals"] / n,
               # one exact evaluation reads one row; at HBM peak that is 8e12 / row_bytes rows/s
               "frac_of_hbm_row_rate": rate * row_bytes / 8e12}
        del ws, G
        S, R = 2048, 64
        pairs = sum(min(S, n - l0) ** 2 for l0 in range(0, n, S))
        xf = xd if xd.dtype == torch.float32 else xd.float()
        dl2 = F.make_data(xf, "l2")
        oi = torch.empty(n, R, dtype=torch.int32, device="cuda")
        od = torch.empty(n, R, dtype=torch.float32, device="cuda")
        for bf16 in (False, True):
            lws = F.leaf_knn(dl2, S, R, bf16, oi, od)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                F.leaf_knn(dl2, S, R, bf16, oi, od, lws)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 3
            key = "bf16" if bf16 else "fp32"
            rec[f"blocked_{key}_G_pairs_per_s"] = pairs / (ms / 1e3) / 1e9
            rec[f"blocked_{key}_over_harvest"] = rec[f"blocked_{key}_G_pairs_per_s"] / rec["harvest_G_evals_per_s"]
            del lws
        log(f"[wsweep] {json.dumps(rec)}")
        out.append(rec)
        del oi, od, data, dl2, xf
        torch.cuda.empty_cache()
    base = out[0]["harvest_G_evals_per_s"]
    print(json.dumps({"mode": "wsweep", "workload": w.name, "row_bytes": row_bytes, "rows": out,
                      "harvest_rate_largest_over_smallest": out[-1]["harvest_G_evals_per_s"] / base}),
          flush=True)


def ground_truth_f32(xd: torch.Tensor, qd: torch.Tensor, k: int, metric: str):
    """Exact k-NN distances in float64 (brute force on the device)."""
    x64 = xd.double()
    xn = (x64 * x64).sum(1)
    out = []
    for s in range(0, qd.shape[0], 128):
        q = qd[s:s + 128].double()
        ip = q @ x64.T
        d = 1.0 - ip if metric == "cosine" else (q * q).sum(1)[:, None] + xn[None, :] - 2.0 * ip
        out.append(torch.topk(d, k, dim=1, largest=False).values)
    return torch.cat(out)


def recall_ladder_f32(data, G, ws, qd, true_d, k=10, target=0.95):
    """Tie-aware recall@k: a returned point counts when its distance is
    within the true k-th distance (float64 brute force) up to float32
    rounding of the declared order."""
    res = []
    nq = qd.shape[0]
    kth = true_d[:, -1:]
    tol = 1e-5 * np.abs(kth) + 1e-6
    for L in (10, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512):
        oi = torch.empty(nq, k, dtype=torch.int32, device="cuda")
        od = torch.empty(nq, k, dtype=torch.float32, device="cuda")
        oe = torch.empty(nq, dtype=torch.int32, device="cuda")
        F.search(data, G, qd, k, L, oi, od, oe, ws)
        torch.cuda.synchronize()
        found = od.cpu().numpy().astype(np.float64)
        rec = float(np.mean(found <= kth + tol))
        res.append(dict(L=L, recall=rec, evals_per_query=float(oe.cpu().numpy().mean())))
        if rec >= target:
            break
    return res


LADDER = (10, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512)


def d_at_recall(ladder, r):
    """Distances per query at recall r (Sec. 2's quality measure): linear in
    recall between the two adjacent beam widths whose recalls bracket r.
    None when the sweep does not bracket r (its first width already reaches
    r, or no width does)."""
    for i, pt in enumerate(ladder):
        if pt["recall"] >= r:
            if i == 0:
                return None
            lo = ladder[i - 1]
            if pt["recall"] == lo["recall"]:
                return float(pt["evals_per_query"])
            f = (r - lo["recall"]) / (pt["recall"] - lo["recall"])
            return float(lo["evals_per_query"] + f * (pt["evals_per_query"] - lo["evals_per_query"]))
    return None


def completeness(x: torch.Tensor, nbrs: np.ndarray, cnt: np.ndarray, metric: str, sample: np.ndarray, k=10):
    """Local completeness (Sec. 2): the fraction of a point's true k nearest
    other points (float64 brute force on the device) present in its row."""
    x64 = x.double()
    xn = (x64 * x64).sum(1)
    hit = 0
    for s in range(0, len(sample), 128):
        ids = torch.from_numpy(sample[s:s + 128].astype(np.int64)).cuda()
        q = x64[ids]
        ip = q @ x64.T
        d = 1.0 - ip if metric == "cosine" else xn[ids][:, None] + xn[None, :] - 2.0 * ip
        d[torch.arange(len(ids), device="cuda"), ids] = float("inf")
        tk = torch.topk(d, k, dim=1, largest=False).indices.cpu().numpy()
        for j, p in enumerate(sample[s:s + 128]):
            row = set(nbrs[p, :cnt[p]].tolist())
            hit += sum(int(t) in row for t in tk[j])
    return hit / (k * len(sample))


def coherent_blocks(parent: np.ndarray, cap: int = 512) -> np.ndarray:
    """Sizes of the coherent blocks of Sec. 5.5: the maximal subtrees of the
    tree-0 spine (parent[v], 0xFFFFFFFF at the root) holding at most `cap`
    points, i.e. subtrees of at most cap points whose parent's subtree is
    larger (or that are the whole tree)."""
    n = len(parent)
    par = parent.astype(np.int64)
    par[parent == 0xFFFFFFFF] = -1
    roots = np.flatnonzero(par < 0)
    # breadth-first order from the root(s): children grouped by parent
    kids = np.argsort(np.where(par < 0, n, par), kind="stable")
    cnt = np.bincount(par[par >= 0], minlength=n)
    start = np.concatenate([[0], np.cumsum(cnt)])
    order = list(roots)
    i = 0
    while i < len(order):
        v = order[i]
        order.extend(kids[start[v]:start[v + 1]].tolist())
        i += 1
    if len(order) != n:
        raise ValueError("the spine is not a forest over every point")
    size = np.ones(n, dtype=np.int64)
    for v in reversed(order):
        if par[v] >= 0:
            size[par[v]] += size[v]
    top = np.where(par >= 0, size[np.maximum(par, 0)], cap + 1)
    return size[(size <= cap) & (top > cap)]


def coherent_block_members(parent: np.ndarray, cap: int = 512):
    """The coherent blocks of Sec. 5.5 with their points: every maximal
    subtree of the tree-0 spine holding at most `cap` points, its points in
    depth-first preorder from the subtree's root (so that consecutive points
    are close in the tree)."""
    n = len(parent)
    par = parent.astype(np.int64)
    par[parent == 0xFFFFFFFF] = -1
    kids = [[] for _ in range(n)]
    for v in np.flatnonzero(par >= 0):
        kids[par[v]].append(int(v))
    order = [int(v) for v in np.flatnonzero(par < 0)]
    i = 0
    while i < len(order):
        order.extend(kids[order[i]])
        i += 1
    if len(order) != n:
        raise ValueError("the spine is not a forest over every point")
    size = np.ones(n, dtype=np.int64)
    for v in reversed(order):
        if par[v] >= 0:
            size[par[v]] += size[v]
    blocks = []
    for v in range(n):
        if size[v] <= cap and (par[v] < 0 or size[par[v]] > cap):
            mem, stack = [], [v]
            while stack:
                a = stack.pop()
                mem.append(a)
                stack.extend(reversed(kids[a]))
            blocks.append(np.array(mem, dtype=np.int64))
    return blocks


def lockstep_stats(V, W, repeat: int = 8):
    """Sec. 5.5's measures for one block of points, from each point's visited
    ids V[i] (one 1-D integer tensor per point, in block order) and the ids
    it visited in expansions 1..10 W[i]: the density sum |V_i| / (B |U V_i|);
    the share of adjacent points' expansion-1..10 evaluations that both make
    (sum over consecutive pairs of |W_i n W_j| over the sum of their mean
    |W|); and the share of all evaluations whose target at least `repeat`
    points of the block evaluate."""
    B = len(V)
    allv = torch.cat(V)
    uniq, counts = torch.unique(allv, return_counts=True)
    tot = int(allv.numel())
    inter = mean = 0.0
    for a, b in zip(W[:-1], W[1:]):
        if a.numel() and b.numel():
            inter += int(torch.isin(a, b).sum())
        mean += (a.numel() + b.numel()) / 2
    return {"B": B, "mean_V": tot / B, "union": int(uniq.numel()),
            "density": tot / (B * uniq.numel()) if tot else 0.0,
            "shared_exp_1_10": inter / mean if mean else 0.0,
            f"evals_to_targets_seen_by_{repeat}_or_more": float(counts[counts >= repeat].sum()) / tot if tot else 0.0}


def density(args):
    """Lockstep density (Sec. 5.5, Tab. 6) of the harvest on the GloVe-shaped
    workload (--density-workload u8: the SIFT-shaped uint8 one): a plain build
    gives the tree-0 spine; 64 coherent blocks (maximal spine subtrees of at
    most 512 points) are drawn at random, and 64 random blocks of the same
    sizes from the other points; a logged build (the same graph) records
    every one of their points' visited sequences V_i; per block the density
    sum |V_i| / (B |U V_i|), the share of expansion-1..10 evaluations that
    adjacent points share, and the share of evaluations whose target at least
    eight points of the block evaluate."""
    w = gen.SIFT_1M if args.density_workload == "u8" else gen.GLOVE_1183514
    n = args.n or w.n
    metric = "cosine" if w.metric == "cosine" else "l2"
    log(f"[density] generating {n} x {w.d} rows ({w.recipe})")
    xd = torch.from_numpy(gen.workload_data(w, n)).cuda()
    data = F.make_data(xd, metric)
    params = F.make_params(w.T, w.ef_h, w.R, w.alpha, w.B)
    ws = F.alloc_workspace(data, params)
    u32 = lambda *sh: torch.full(sh, -1, dtype=torch.int32, device="cuda")  # noqa: E731
    G = F.make_graph(u32(n, w.R), u32(n), u32(n), u32(w.T), w.T)
    c0, _ = F.build_graph(data, w.build_seed, params, G, ws, timings=True)
    h0 = F.graph_hash(G)
    parent = G._keep[2].cpu().numpy().view(np.uint32)
    coh = coherent_block_members(parent, 512)
    rng = np.random.default_rng(5005)
    pick = rng.choice(len(coh), size=min(64, len(coh)), replace=False)
    cblocks = [coh[i] for i in pick]
    used = np.zeros(n, bool)
    for b in cblocks:
        used[b] = True
    rest = rng.permutation(np.flatnonzero(~used))
    rblocks, o = [], 0
    for b in cblocks:
        rblocks.append(np.sort(rest[o:o + len(b)]))
        o += len(b)
    slot = np.full(n, -1, np.int32)
    pts = np.concatenate(cblocks + rblocks)
    slot[pts] = np.arange(len(pts), dtype=np.int32)
    cap = args.log_cap
    log(f"[density] logging {len(pts)} points ({len(cblocks)} coherent + {len(rblocks)} random blocks), cap {cap}")
    c1, t1, lids, lens, marks = F.build_graph_log(data, w.build_seed, params, G, ws, torch.from_numpy(slot).cuda(),
                                                  cap)
    assert F.graph_hash(G) == h0 and c1["harvest_evals"] == c0["harvest_evals"]
    lens_h = lens.cpu().numpy().astype(np.int64)
    marks_h = marks.cpu().numpy().astype(np.int64)
    truncated = int((lens_h > cap).sum())

    def block_stats(b):
        V, W = [], []
        for p in b:
            s_ = int(slot[p])
            m = min(int(lens_h[s_]), cap)
            V.append(lids[s_, :m].long())
            W.append(lids[s_, min(int(marks_h[s_, 0]), m):min(int(marks_h[s_, 10]), m)].long())
        return lockstep_stats(V, W)

    out = {"mode": "density", "workload": w.name, "n": n, "graph_hash": f"{h0:#018x}",
           "logged_points": int(len(pts)), "log_cap": cap, "truncated_logs": truncated,
           "coherent_blocks_available": len(coh), "kinds": {}}
    for kind, blocks in (("coherent", cblocks), ("random", rblocks)):
        st = [block_stats(b) for b in blocks]
        agg = {k: float(np.mean([r[k] for r in st])) for k in st[0] if k != "B"}
        agg["B_median"] = float(np.median([r["B"] for r in st]))
        agg["B_mean"] = float(np.mean([r["B"] for r in st]))
        agg["density_median"] = float(np.median([r["density"] for r in st]))
        out["kinds"][kind] = agg
        log(f"[density] {kind}: {json.dumps(agg)}")
    print(json.dumps(out), flush=True)


def quality(args):
    """The quality columns of Tab. 2 for arms of T (trees) and B (blocks) on
    the GloVe-shaped workload: build time and evaluations, local
    completeness, the recall@10 ladder with distances and queries per second
    at each beam width, and d@0.95 / d@0.97 against the first arm.  With
    --quality-workload gist the same on the GIST-shaped rows (d = 960, L2,
    1,000 held-out queries)."""
    w = gen.GIST_1M if args.quality_workload == "gist" else gen.GLOVE_1183514
    n = args.n or w.n
    metric = "cosine" if w.metric == "cosine" else "l2"
    arms = [tuple(int(v) for v in a.split(":")) for a in args.arms.split(",")]
    log(f"[quality] generating {n} x {w.d} rows and {w.nq} queries")
    xd = torch.from_numpy(gen.workload_data(w, n)).cuda()
    qd = torch.from_numpy(gen.workload_queries(w)).cuda()
    true_d = ground_truth_f32(xd, qd, 10, metric).cpu().numpy()
    kth = true_d[:, -1:]
    tol = 1e-5 * np.abs(kth) + 1e-6
    sample = np.random.default_rng(17).choice(n, min(n, 2000), replace=False)
    data = F.make_data(xd, metric)
    nq = qd.shape[0]
    out = []
    for T, B, ef in arms:
        params = F.make_params(T, ef, w.R, w.alpha, B)
        ws = F.alloc_workspace(data, params)
        u32 = lambda *sh: torch.full(sh, -1, dtype=torch.int32, device="cuda")  # noqa: E731
        G = F.make_graph(u32(n, w.R), u32(n), u32(n), u32(T), T)
        F.build_graph(data, w.build_seed, params, G, ws, timings=True)
        c, t = F.build_graph(data, w.build_seed, params, G, ws, timings=True)
        rec = {"arm": f"T{T}/ef_h {ef} B={B}", "T": T, "B": B, "ef_h": ef,
               "build_s": sum(t[k] for k in ("scaffold_ms", "harvest_ms", "merge_ms", "finalize_ms")) / 1e3,
               "G_dist": (c["scaffold_evals"] + c["harvest_evals"] + c["finalize_evals"]) / 1e9,
               "hash": hex(F.graph_hash(G))}
        nb, cn = G._keep[0].cpu().numpy().view(np.uint32), G._keep[1].cpu().numpy().view(np.uint32)
        rec["completeness"] = completeness(xd, nb, cn, metric, sample)
        cb = coherent_blocks(G._keep[2].cpu().numpy().view(np.uint32))
        rec["coherent_blocks"] = {"count": int(len(cb)), "median": float(np.median(cb)),
                                  "p10": float(np.percentile(cb, 10)), "p90": float(np.percentile(cb, 90)),
                                  "points_covered": float(cb.sum() / n)}
        ladder = []
        oi = torch.empty(nq, 10, dtype=torch.int32, device="cuda")
        od = torch.empty(nq, 10, dtype=torch.float32, device="cuda")
        oe = torch.empty(nq, dtype=torch.int32, device="cuda")
        for L in LADDER:
            F.search(data, G, qd, 10, L, oi, od, oe, ws)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            F.search(data, G, qd, 10, L, oi, od, oe, ws)
            e1.record()
            torch.cuda.synchronize()
            found = od.cpu().numpy().astype(np.float64)
            ladder.append({"L": L, "recall": float(np.mean(found <= kth + tol)),
                           "evals_per_query": float(oe.cpu().numpy().mean()),
                           "qps": nq / (e0.elapsed_time(e1) / 1e3)})
        rec["ladder"] = ladder
        for r in (0.95, 0.97):
            rec[f"d@{r}"] = d_at_recall(ladder, r)
        log(f"[quality] {json.dumps({k: v for k, v in rec.items() if k != 'ladder'})}")
        out.append(rec)
        del ws, G
        torch.cuda.empty_cache()
    for r in (0.95, 0.97):
        base = out[0][f"d@{r}"]
        for rec in out:
            v = rec[f"d@{r}"]
            rec[f"d@{r}_rel"] = None if v is None or base is None else v / base
    print(json.dumps({"mode": "quality", "workload": w.name, "n": n, "queries": nq, "arms": out}), flush=True)


def result_error_f64(data, G, ws, xd, qd, metric, k=10, L=256):
    """Relative error of the search's float32 distances (k per query, beam
    L) against the same (query, point) distances recomputed in float64:
    max, mean and 99.9th percentile over every returned result."""
    nq = qd.shape[0]
    oi = torch.empty(nq, k, dtype=torch.int32, device="cuda")
    od = torch.empty(nq, k, dtype=torch.float32, device="cuda")
    F.search(data, G, qd, k, L, oi, od, None, ws)
    torch.cuda.synchronize()
    rows = xd[oi.long()].double()
    q = qd.double()[:, None, :]
    d64 = 1.0 - (rows * q).sum(-1) if metric == "cosine" else ((rows - q) ** 2).sum(-1)
    rel = ((od.double() - d64).abs() / d64.abs().clamp_min(1e-300)).flatten()
    return {"results": int(rel.numel()), "max_rel": float(rel.max()), "mean_rel": float(rel.mean()),
            "p999_rel": float(torch.quantile(rel.float(), 0.999)), "L": L, "k": k}


def hodges_lehmann(logr: np.ndarray) -> float:
    w = [(logr[i] + logr[j]) / 2 for i in range(len(logr)) for j in range(i, len(logr))]
    return float(np.exp(np.median(w)))


def screen_compare(args):
    """Mixed precision against float32 (paired protocol): whole builds of
    the same workload plain, bf16-screened, fp8-screened and (d > 256)
    with the bf16-split prune tiles alone, in a seeded random order within
    each repetition; the graph hash must be identical
    on every run.  Ratio = plain time / screened time; Hodges-Lehmann
    estimate over repetitions and the exact Wilcoxon signed-rank p."""
    from scipy import stats
    rows = []
    names = {"glove": gen.GLOVE_1183514, "gist": gen.GIST_1M}
    for key in args.workloads.split(","):
        w = names[key]
        n = args.n or w.n
        log(f"[screen] {key}: generating {n} x {w.d} rows ({w.recipe})")
        x = gen.workload_data(w, n)
        xd = torch.from_numpy(x).cuda()
        metric = "cosine" if w.metric == "cosine" else "l2"
        data = F.make_data(xd, metric)
        forms = (F.SCREEN_NONE, F.SCREEN_BF16, F.SCREEN_FP8E4M3, F.SCREEN_INT8)
        if w.d > 256:
            forms += (F.SCREEN_BF16_PRUNE,)
        if args.forms:
            forms = (F.SCREEN_NONE,) + tuple(int(f) for f in args.forms.split(",") if int(f) in forms[1:])
        params = {f: F.make_params(w.T, w.ef_h, w.R, w.alpha, w.B, screen=f) for f in forms}
        ws = F.alloc_workspace(data, params[max(forms, key=lambda f: F.workspace_size(data, params[f]))])
        G = F.make_graph(*(torch.full(sh, -1, dtype=torch.int32, device="cuda")
                           for sh in ((n, w.R), (n,), (n,), (w.T,))), w.T)
        hashes = {}
        for f in forms:  # warm-up: one build per form
            c, t = F.build_graph(data, w.build_seed, params[f], G, ws, timings=True)
            hashes[f] = F.graph_hash(G)
            log(f"[screen] warm-up form {f}: harvest {t['harvest_ms']:.0f} ms, rejected "
                f"{c['screen_rejected']} of {c['harvest_evals']}")
        assert len(set(hashes.values())) == 1, hashes
        rng = np.random.default_rng(20260)
        res = {f: [] for f in forms}
        for rep in range(args.reps):
            for f in rng.permutation(len(forms)):
                f = forms[f]
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                c, t = F.build_graph(data, w.build_seed, params[f], G, ws, timings=True)
                wall = time.perf_counter() - t0
                assert F.graph_hash(G) == hashes[F.SCREEN_NONE]
                res[f].append(dict(harvest_ms=t["harvest_ms"], build_s=wall, screen_ms=t["screen_ms"],
                                   finalize_ms=t["finalize_ms"], scaffold_ms=t["scaffold_ms"],
                                   evals=c["harvest_evals"],
                                   rejected=c["screen_rejected"], rechecks=c["prune_rechecks"]))
                log(f"[screen] rep {rep} form {f}: harvest {t['harvest_ms']:.0f} ms build {wall:.2f} s")
        row = {"workload": w.name, "n": n, "d": w.d, "metric": metric, "graph_hash": f"{hashes[0]:#018x}",
               "harvest_evals": res[0][0]["evals"], "forms": {}}
        base_h = np.array([r["harvest_ms"] for r in res[0]])
        base_b = np.array([r["build_s"] for r in res[0]])
        row_bytes = 4 * w.d
        form_names = {0: "fp32", 1: "bf16", 2: "fp8e4m3", 3: "bf16split_prune", 4: "int8"}
        for f, name in ((f, form_names[f]) for f in forms):
            h = np.array([r["harvest_ms"] for r in res[f]])
            b = np.array([r["build_s"] for r in res[f]])
            ev = res[f][0]["evals"]
            rej = res[f][0]["rejected"]
            # a screened evaluation reads the narrow row's codes and its
            # 16-byte trailer (error norm, norm, fp8 factor)
            narrow = {0: 0, 1: (2 * w.d + 31) // 32 * 32 + 16, 2: (w.d + 15) // 16 * 16 + 16, 3: 0,
                      4: (w.d + 15) // 16 * 16 + 16}[f]
            e = {"harvest_ms_median": float(np.median(h)), "build_s_median": float(np.median(b)),
                 "harvest_evals_per_s": float(ev / (np.median(h) / 1e3)),
                 "screen_rejected_frac": rej / ev,
                 "bytes_per_eval": narrow + (1 - rej / ev) * row_bytes if f else row_bytes,
                 "screen_copy_ms": float(np.median([r["screen_ms"] for r in res[f]])),
                 "finalize_ms_median": float(np.median([r["finalize_ms"] for r in res[f]])),
                 "scaffold_ms_median": float(np.median([r["scaffold_ms"] for r in res[f]])),
                 "prune_rechecks": int(res[f][0]["rechecks"])}
            if f:
                lr_h, lr_b = np.log(base_h / h), np.log(base_b / b)
                e["harvest_speedup_hl"] = hodges_lehmann(lr_h)
                e["build_speedup_hl"] = hodges_lehmann(lr_b)
                if len(h) >= 2:
                    e["wilcoxon_p_harvest"] = float(stats.wilcoxon(lr_h, method="exact").pvalue)
                    e["wilcoxon_p_build"] = float(stats.wilcoxon(lr_b, method="exact").pvalue)
            row["forms"][name] = e
        # error against float64, stated per result: every form builds the
        # same graph (hash above), so the search's float32 distances (the
        # declared order) on it are compared with float64 recomputations of
        # the same pairs
        qd = torch.from_numpy(gen.workload_queries(w, min(w.nq, 1000))).cuda()
        F.build_graph(data, w.build_seed, params[0], G, ws)
        row["error_vs_float64"] = result_error_f64(data, G, ws, xd, qd, metric)
        log(f"[screen] error vs float64: {row['error_vs_float64']}")
        if not args.no_recall:
            true_d = ground_truth_f32(xd, qd, 10, metric).cpu().numpy()
            row["recall_ladder"] = recall_ladder_f32(data, G, ws, qd, true_d)
        log(f"[screen] {json.dumps(row)}")
        rows.append(row)
        del ws, G, xd, data
        torch.cuda.empty_cache()
    print(json.dumps({"mode": "screen", "reps": args.reps, "rows": rows}), flush=True)


def batched_compare(args):
    """Batched form (the 64-instance workload): 64 uneven instances built together -- eager, and
    with the blocks captured in one HIP graph -- against 64 sequential
    build_graph calls, paired repetitions in seeded random order; every
    instance's graph hash must equal its sequential build's."""
    from scipy import stats
    count = args.instances
    insts = gen.batched_instances(count=count, scale=args.scale)
    ntot = sum(i["x"].shape[0] for i in insts)
    log(f"[batched] {count} instances, {ntot} points in all")
    datas, params, graphs = [], [], []

    def u32(*shape):
        return torch.full(shape, -1, dtype=torch.int32, device="cuda")

    for i in insts:
        n = i["x"].shape[0]
        datas.append(F.make_data(torch.from_numpy(i["x"]).cuda()))
        params.append(F.make_params(i["T"], i["ef_h"], i["R"], i["alpha"], i["B"]))
        graphs.append(F.make_graph(u32(n, i["R"]), u32(n), u32(n), u32(i["T"]), i["T"]))
    seeds = [i["seed"] for i in insts]
    big = max(range(count), key=lambda k: insts[k]["x"].shape[0])
    ws_seq = F.alloc_workspace(datas[big], F.make_params(8, 128, 32, 1.2, 8))

    def sequential():
        ev = 0
        for k in range(count):
            c, _ = F.build_graph(datas[k], seeds[k], params[k], graphs[k], ws_seq)
            ev += c["harvest_evals"]
        return ev

    ws_b = None

    def batched(use_graph, tune=False):
        nonlocal ws_b
        c, ws_b = F.build_graph_batched(datas, params, seeds, graphs, ws=ws_b, use_hipgraph=use_graph,
                                        autotune=tune)
        return c["harvest_evals"]

    # the autotuned forms tune on their first call (block 0 of the batch over
    # the scaffold) and reuse the cached choice afterwards
    runs = {"sequential": sequential, "batched": lambda: batched(False), "batched_hipgraph": lambda: batched(True),
            "batched_autotune": lambda: batched(False, True),
            "batched_hipgraph_autotune": lambda: batched(True, True)}
    # warm-up and hash check
    sequential()
    want = [F.graph_hash(g) for g in graphs]
    for name in [k for k in runs if k != "sequential"]:
        runs[name]()
        got = [F.graph_hash(g) for g in graphs]
        assert got == want, name
    rng = np.random.default_rng(5150)
    times = {k: [] for k in runs}
    evals = {}
    for rep in range(args.reps):
        for j in rng.permutation(len(runs)):
            name = list(runs)[j]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            evals[name] = runs[name]()
            torch.cuda.synchronize()
            times[name].append(time.perf_counter() - t0)
            log(f"[batched] rep {rep} {name}: {times[name][-1]:.3f} s")
    got = [F.graph_hash(g) for g in graphs]
    assert got == want
    seq = np.array(times["sequential"])
    out = {"mode": "batched", "instances": count, "points": ntot, "reps": args.reps,
           "harvest_evals": evals["sequential"], "forms": {}}
    for name in runs:
        t = np.array(times[name])
        e = {"build_s_median": float(np.median(t)), "points_per_s": ntot / float(np.median(t))}
        if name != "sequential":
            lr = np.log(seq / t)
            e["speedup_hl"] = hodges_lehmann(lr)
            if len(t) >= 2:
                e["wilcoxon_p"] = float(stats.wilcoxon(lr, method="exact").pvalue)
        out["forms"][name] = e
    print(json.dumps(out), flush=True)


def recheck_rates(args):
    """Share of the occlusion prune's kill tests, alpha d(r, c) <= d(p, c),
    that a tile form's proven margin leaves undecided (each one an exact
    recheck), measured on the host in float64 over sampled points of a
    workload: each point's 128 nearest candidates pruned in distance order
    (R = 64, alpha = 1.2) and every test the prune makes.  Forms: the
    float32 tiles and the bf16 split on the rows as stored, and single bf16
    or fp8 operands on candidates centred on the point (c - p), whose
    product error is (2u + u^2) |a'| |c'| with u = 2^-8 / 2^-4."""
    names = {"glove": gen.GLOVE_1183514, "gist": gen.GIST_1M}
    out = {"mode": "recheck", "rows": []}
    for key in args.workloads.split(","):
        w = names[key]
        n = args.n or 200_000
        x = gen.workload_data(w, n).astype(np.float32)
        X = torch.from_numpy(x).double()
        rng = np.random.default_rng(5)
        P = rng.choice(n, 300, replace=False)
        d, M, R, alpha, u = x.shape[1], 128, 64, 1.2, 2.0 ** -24
        gg = (d + 4) * 2 * u
        tot = {"tests": 0, "f32": 0, "bf16_split": 0, "bf16_centred": 0, "fp8_centred": 0}
        xn2 = (X * X).sum(1)
        for p in P:
            q = X[p]
            dist = 1.0 - X @ q if w.metric == "cosine" else xn2 - 2 * X @ q + xn2[p]
            dist[p] = np.inf
            idx = torch.topk(dist, M, largest=False).indices.numpy()
            C, dpc = X[idx], dist[idx].numpy()
            nc = np.linalg.norm((C - q).numpy(), axis=1)
            nraw = np.linalg.norm(C.numpy(), axis=1)
            if w.metric == "cosine":
                Dcc = 1.0 - (C @ C.T).numpy()
            else:
                Gm = (C @ C.T).numpy()
                Dcc = np.diag(Gm)[:, None] + np.diag(Gm)[None, :] - 2 * Gm
            alive, kept = np.ones(M, bool), 0
            for i in range(M):
                if not alive[i]:
                    continue
                kept += 1
                if kept >= R:
                    break
                js = np.nonzero(alive[i + 1:])[0] + i + 1
                t = np.abs(alpha * Dcc[i, js] - dpc[js])
                tot["tests"] += len(js)
                if w.metric == "cosine":
                    m32 = 2 * (gg + 2 * u) * nraw[i] * nraw[js]
                    msp = 2 * (3.1 * 2.0 ** -16 + gg) * nraw[i] * nraw[js]
                else:
                    m32 = 4 * (gg + 2 * u) * (nraw[i] ** 2 + nraw[js] ** 2)
                    msp = 4 * (3.1 * 2.0 ** -16 + gg) * (nraw[i] ** 2 + nraw[js] ** 2)
                mbf = 4 * (2 * 2.0 ** -8 + 2.0 ** -16 + gg) * nc[i] * nc[js]
                mf8 = 4 * (2 * 2.0 ** -4 + 2.0 ** -8 + gg) * nc[i] * nc[js]
                for k, m in (("f32", m32), ("bf16_split", msp), ("bf16_centred", mbf), ("fp8_centred", mf8)):
                    tot[k] += int((t <= alpha * m).sum())
                alive[js[alpha * Dcc[i, js] <= dpc[js]]] = False
        row = {"workload": w.name, "sample_rows": n, "points": len(P), "tests": tot["tests"]}
        row.update({f"undecided_{k}": tot[k] / tot["tests"] for k in tot if k != "tests"})
        log(f"[recheck] {row}")
        out["rows"].append(row)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", default="build",
                    choices=("build", "dsweep", "screen", "batched", "wsweep", "quality", "density", "recheck"),
                    help="build: the benchmark line (default); dsweep: wall vs dimension; "
                         "screen: int8 / fp8 / bf16 screened builds against float32; "
                         "batched: 64 instances built together against sequential builds; "
                         "wsweep: throughput against working set (GloVe-shaped prefixes); "
                         "quality: completeness, recall ladder and d@r for T/B arms; "
                         "density: lockstep density of coherent and random blocks (visit log); "
                         "recheck: share of prune tests a tile form's margin leaves undecided (host only)")
    ap.add_argument("--density-workload", default="glove", choices=("glove", "u8"),
                    help="density mode: the GloVe-shaped float32 rows or the SIFT-shaped uint8 rows")
    ap.add_argument("--log-cap", type=int, default=131072,
                    help="density mode: visited ids kept per logged point")
    ap.add_argument("--instances", type=int, default=64, help="batched mode: instance count")
    ap.add_argument("--scale", type=float, default=1.0, help="batched mode: shrink every instance's n")
    ap.add_argument("--workloads", default="glove,gist", help="screen mode: glove, gist or both")
    ap.add_argument("--reps", type=int, default=3, help="screen mode: paired repetitions; wsweep: timed builds per prefix")
    ap.add_argument("--sizes", default="", help="wsweep mode: comma-separated prefix sizes")
    ap.add_argument("--dims", default="", help="dsweep mode: a subset of 32,64,128,256,512,960")
    ap.add_argument("--sweep-workload", default="glove", choices=("glove", "u8", "gist"),
                    help="wsweep mode: the GloVe-shaped float32 rows, the benchmark line's uint8 rows "
                         "or the GIST-shaped float32 rows")
    ap.add_argument("--quality-workload", default="glove", choices=("glove", "gist"),
                    help="quality mode: the GloVe-shaped or the GIST-shaped rows")
    ap.add_argument("--arms", default="8:8:128,8:1:128,8:32:128,16:8:128",
                    help="quality mode: comma-separated T:B:ef_h arms (the first is the reference)")
    ap.add_argument("--forms", default="", help="screen mode: fg_screen values to compare with float32 "
                                                 "(default: all that apply)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=None, help="override n (default: the workload's)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the screened builds and the batched comparison after the line")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="rows of the oracle's sample build (0: 50,000 for the GloVe-shaped "
                         "workload, 300,000 otherwise)")
    ap.add_argument("--workload", default="glove", choices=tuple(WORKLOADS),
                    help="the benchmark line's workload: glove the GloVe-shaped float32 cosine "
                         "build (default), sift the SIFT-shaped uint8 build, gist the GIST-shaped "
                         "d = 960 build")
    ap.add_argument("--extra", default="sift,gist",
                    help="other full-size workloads measured once each after the line (extra keys)")
    ap.add_argument("--table", type=int, default=0, choices=(0, 512, 1024, 2048, 4096),
                    help="on-chip visited-table slots per search (0 = library default)")
    ap.add_argument("--tune", action="store_true",
                    help="pick the visited-table size, searches per compute unit and lanes per row "
                         "with fg_autotune before the warm-up (off by default: the tuner times block 0 "
                         "of a 50,000-row prefix, and the library's defaults come from full-size sweeps)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed steps, copy 1 GiB device to device (a plain copy "
                         "kernel of known size, to scale profiler byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the harvest would shard by points over replicated rows and substrate).", file=sys.stderr)
        sys.exit(2)
    if args.mode == "dsweep":
        return dsweep(args)
    if args.mode == "screen":
        return screen_compare(args)
    if args.mode == "batched":
        return batched_compare(args)
    if args.mode == "wsweep":
        return wsweep(args)
    if args.mode == "quality":
        return quality(args)
    if args.mode == "density":
        return density(args)
    if args.mode == "recheck":
        return recheck_rates(args)

    return headline(args)


WORKLOADS = {"glove": gen.GLOVE_1183514, "sift": gen.SIFT_1M, "gist": gen.GIST_1M}
# the dominant kernel's counter summaries (two rocprofv3 --pmc passes of this
# script's default run), one per workload
PMC_SUMMARIES = {"glove": os.path.join(ROOT, "profiles", "k_beam_harvest_f32_cosine_1183514_pmc.md"),
                 "sift": PMC_SUMMARY}


def oracle_golden(key: str):
    """The committed record of the oracle's full-size build of a workload
    (tests/golden/fullsize.txt, written by an oracle-only script), or None."""
    path = os.path.join(ROOT, "tests", "golden", "fullsize.txt")
    recs, cur = {}, None
    try:
        for line in open(path):
            line = line.strip()
            if line.startswith("[") and line.endswith("]"):
                cur = recs.setdefault(line[1:-1], {})
            elif cur is not None and "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                cur[k.strip()] = v.strip()
    except OSError:
        return None
    return recs.get(key)


def run_builds(key, w, args, steps, warmup, xd=None, x=None):
    """Whole builds of a workload (data resident in HBM before timing):
    warm-up builds, then `steps` timed ones between device synchronisations.
    Returns the measurement record and what later steps need."""
    import hashlib
    n = args.n or w.n
    if xd is None:
        log(f"[bench] {key}: generating {n} x {w.d} rows ({w.recipe})")
        x = gen.workload_data(w, n)
        xd = torch.from_numpy(x).cuda()
    metric = "cosine" if w.metric == "cosine" else "l2"
    data = F.make_data(xd, metric)
    params = F.make_params(w.T, w.ef_h, w.R, w.alpha, w.B, beam_table_slots=args.table)
    ws = F.alloc_workspace(data, params)
    log(f"[bench] {key}: workspace {ws.numel() / 2**30:.2f} GiB")
    tuned = None
    if getattr(args, "tune", False):
        t0 = time.perf_counter()
        params = F.autotune(data, params, ws)
        tuned = {"beam_table_slots": params.beam_table_slots, "waves_per_cu": params.waves_per_cu,
                 "lanes_per_row": params.lanes_per_row, "tune_s": time.perf_counter() - t0}
        log(f"[bench] {key}: tuned {tuned}")

    def u32(*shape):
        return torch.full(shape, -1, dtype=torch.int32, device="cuda")

    G = F.make_graph(u32(n, w.R), u32(n), u32(n), u32(w.T), w.T)
    for i in range(warmup):
        c, t = F.build_graph(data, w.build_seed, params, G, ws, timings=True)
        log(f"[bench] {key} warmup {i}: harvest {t['harvest_ms']:.1f} ms, scaffold {t['scaffold_ms']:.1f} ms")
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for i in range(steps):
        c, t = F.build_graph(data, w.build_seed, params, G, ws, timings=True)
        recs.append((c, t))
        log(f"[bench] {key} step {i}: harvest {t['harvest_ms']:.1f} ms scaffold {t['scaffold_ms']:.1f} ms "
            f"merge {t['merge_ms']:.1f} ms finalize {t['finalize_ms']:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = sum(c["harvest_evals"] for c, _ in recs)
    hms = sum(t["harvest_ms"] for _, t in recs)
    launches = sum(len(t["block_harvest_ms"]) for _, t in recs)
    row_bytes = w.d * (4 if w.dtype == "f32" else 1)  # one row per evaluation
    c0, t0_ = recs[0]
    ghash = F.graph_hash(G)
    rec = {"workload": w.name, "n": n, "d": w.d, "metric": metric, "T": w.T, "B": w.B, "ef_h": w.ef_h,
           "R": w.R, "alpha": w.alpha, "seed": w.build_seed,
           "beam_table_slots": (tuned["beam_table_slots"] if tuned else args.table) or "library default",
           "tuned": tuned,
           "harvest_evals_per_s": ev / (hms / 1e3), "build_s": wall / steps,
           "phase_ms": {k: t0_[k] for k in ("scaffold_ms", "harvest_ms", "merge_ms", "finalize_ms")},
           "harvest_evals_per_build": c0["harvest_evals"], "counters": c0, "graph_hash": f"{ghash:#018x}",
           "harvest_launches": launches, "harvest_ms_per_launch": hms / launches,
           "algorithmic_bytes_per_eval": row_bytes,
           "achieved_GBs": ev * row_bytes / (hms / 1e3) / 1e9,
           "block_harvest_ms": [round(v, 3) for v in t0_["block_harvest_ms"]],
           "block_evals": t0_["block_evals"]}
    gold = oracle_golden(key) if n == w.n else None
    if gold is not None and x is not None:
        same_input = hashlib.sha256(np.ascontiguousarray(x).tobytes()).hexdigest() == gold["input_sha256"]
        rec["oracle_full_size"] = {
            "input_digest_matches": same_input,
            "graph_hash_equals_oracle": same_input and gold["graph_hash"] == f"{ghash:#018x}",
            "counters_equal_oracle": same_input and all(int(gold[k]) == int(c0[k]) for k in
                                                        ("scaffold_evals", "harvest_evals", "prune_evals",
                                                         "finalize_evals", "expansions")),
            "oracle_build_wall_s": float(gold["oracle_build_wall_s"]),
            "oracle_threads": int(gold["oracle_threads"])}
    return rec, dict(x=x, xd=xd, data=data, G=G, ws=ws, metric=metric, wall=wall)


def forms_vs_fp32(key, w, st):
    """The precision form beside the plain one on the benchmark line's data:
    one warm-up and one timed build per screened form (its own workspace,
    the narrow copy included); the graph hash must equal the plain build's."""
    data, G, base = st["data"], st["G"], F.graph_hash(st["G"])
    out = {}
    if w.dtype != "f32" or w.d <= 64:
        return out
    for f, name in ((F.SCREEN_FP8E4M3, "fp8e4m3"), (F.SCREEN_BF16, "bf16"), (F.SCREEN_INT8, "int8")):
        params = F.make_params(w.T, w.ef_h, w.R, w.alpha, w.B, screen=f)
        ws = F.alloc_workspace(data, params)
        F.build_graph(data, w.build_seed, params, G, ws, timings=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c, t = F.build_graph(data, w.build_seed, params, G, ws, timings=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        assert F.graph_hash(G) == base, name
        out[name] = {"harvest_ms": t["harvest_ms"], "build_s": wall,
                     "screen_rejected_frac": c["screen_rejected"] / c["harvest_evals"]}
        log(f"[bench] {key} screen {name}: harvest {t['harvest_ms']:.1f} ms build {wall:.2f} s")
        del ws
        torch.cuda.empty_cache()
    return out


def batched_vs_sequential():
    """The batched form on its workload (64 uneven float32 instances, 3.1 M
    points): 64 sequential builds against one autotuned batched build with
    the blocks in one HIP graph, each after a warm-up; every instance's
    hash must equal its sequential build's."""
    insts = gen.batched_instances(count=64, scale=1.0)

    def u32(*shape):
        return torch.full(shape, -1, dtype=torch.int32, device="cuda")

    datas, params, graphs = [], [], []
    for i in insts:
        n = i["x"].shape[0]
        datas.append(F.make_data(torch.from_numpy(i["x"]).cuda()))
        params.append(F.make_params(i["T"], i["ef_h"], i["R"], i["alpha"], i["B"]))
        graphs.append(F.make_graph(u32(n, i["R"]), u32(n), u32(n), u32(i["T"]), i["T"]))
    seeds = [i["seed"] for i in insts]
    big = max(range(len(insts)), key=lambda k: insts[k]["x"].shape[0])
    ws_seq = F.alloc_workspace(datas[big], F.make_params(8, 128, 32, 1.2, 8))
    res, ws_b = {}, None
    for rep in range(2):  # the first pass of each is the warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(len(insts)):
            F.build_graph(datas[k], seeds[k], params[k], graphs[k], ws_seq)
        torch.cuda.synchronize()
        res["sequential_s"] = time.perf_counter() - t0
        want = [F.graph_hash(g) for g in graphs]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, ws_b = F.build_graph_batched(datas, params, seeds, graphs, ws=ws_b, use_hipgraph=True, autotune=True)
        torch.cuda.synchronize()
        res["batched_s"] = time.perf_counter() - t0
        assert [F.graph_hash(g) for g in graphs] == want
    res["speedup"] = res["sequential_s"] / res["batched_s"]
    res["instances"] = len(insts)
    res["points"] = int(sum(i["x"].shape[0] for i in insts))
    log(f"[bench] batched: {res}")
    return res


def headline(args):
    """The benchmark line: whole builds of the GloVe-shaped workload
    (n = 1,183,514, d = 100, unit float32 rows, cosine; T=8 B=8 ef_h=128
    R=64 alpha=1.2), the largest configuration and the one the metric's
    recall condition is met on.  value = harvest evaluations / harvest
    kernel time (HIP events on the build's stream around each block's
    launch).  Then the recall@10 ladder of the built graph (10,000 held-out
    queries against a float64 brute force), the oracle on a bounded sample
    of the same recipe, and single timed builds of the other full-size
    workloads as extra keys."""
    key = args.workload
    w = WORKLOADS[key]
    rec, st = run_builds(key, w, args, args.steps, args.warmup)
    row_bytes = rec["algorithmic_bytes_per_eval"]
    achieved = rec["achieved_GBs"]
    out = {
        "metric": "harvest dist-evals/s + build s at recall@10>=0.95; mixed/batched vs FP32",
        "value": rec["harvest_evals_per_s"],
        "unit": "dist-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": st["wall"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.dtype == "f32" else "int32",
        "data": "synthetic",
        "config": {"workload": w.name, **{k: rec[k] for k in ("n", "d", "metric", "T", "B", "ef_h", "R", "alpha",
                                                               "seed", "beam_table_slots")},
                   "waves_per_cu": "max resident"},
        "build_s": rec["build_s"],
        "phase_ms": rec["phase_ms"],
        "harvest_evals_per_build": rec["harvest_evals_per_build"],
        "counters": rec["counters"],
        "graph_hash": rec["graph_hash"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(PMC_SUMMARIES.get(key)),
                     "kernel": "k_beam (harvest)", "launches": rec["harvest_launches"],
                     "ms_per_launch": rec["harvest_ms_per_launch"], "bytes_per_eval": row_bytes},
        "block_harvest_ms": rec["block_harvest_ms"],
        "block_evals": rec["block_evals"],
    }
    if "oracle_full_size" in rec:
        out["oracle_full_size"] = rec["oracle_full_size"]
    if not args.no_forms:
        out["forms_vs_fp32"] = forms_vs_fp32(key, w, st)
    if args.calib_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = a.numel()
        del a, b
    if not args.no_recall:
        qd = torch.from_numpy(gen.workload_queries(w)).cuda()
        if w.dtype == "f32":
            true_d = ground_truth_f32(st["xd"], qd, 10, st["metric"]).cpu().numpy()
            lad = recall_ladder_f32(st["data"], st["G"], st["ws"], qd, true_d)
        else:
            true_d = ground_truth_u8(st["xd"], qd, 10).cpu().numpy().astype(np.float64)
            lad = recall_ladder(st["data"], st["G"], st["ws"], qd, true_d)
        out["recall_ladder"] = lad
        out["recall@10"] = lad[-1]["recall"]
        out["recall_target_met"] = lad[-1]["recall"] >= 0.95
        out["recall_L"] = lad[-1]["L"]
    del st
    torch.cuda.empty_cache()
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        n_cpu = args.cpu_sample or (50_000 if w is gen.GLOVE_1183514 else 300_000)
        log(f"[bench] cpu baseline: oracle on {n_cpu} points, {threads} threads")
        out["cpu_baseline"] = cpu_baseline(w, n_cpu, threads)
    if not args.no_forms:
        out["batched_vs_sequential"] = batched_vs_sequential()
    extra = [k for k in args.extra.split(",") if k and k != key]
    if extra:
        out["extra_workloads"] = {}
        for k in extra:
            r, st = run_builds(k, WORKLOADS[k], args, 1, 1)
            r["roofline_frac_8TBs"] = r["achieved_GBs"] / HBM_PEAK_GBS
            out["extra_workloads"][k] = r
            del st
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
