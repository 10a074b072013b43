"""Write tests/golden/fullsize.txt: the oracle's whole builds of the full-size
workloads (the SIFT-shaped uint8 build, n = 10^6, d = 128; the GIST-shaped
float32 build, n = 10^6, d = 960; the GloVe-shaped cosine build,
n = 1,183,514, d = 100), each with the sha256 of its generated input, the
graph hash and every work counter.

This script calls only the seeded generators (paper_2609_30493_amd.datagen,
which hold none of the method's arithmetic) and the CPU oracle (oracle/).
Nothing here reads a result of the HIP path.  The GPU tests compare a build
in the benchmark's launch configuration with these records; they first
check the input digest, since the generators run on another host there.

Usage: python tests/golden/make_fullsize.py [sift,gist,glove] [--threads N]
(an existing record of another workload is kept).  Hours of CPU time.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fgo  # noqa: E402
from paper_2609_30493_amd import datagen as gen  # noqa: E402

OUT = os.path.join(HERE, "fullsize.txt")
WORKLOADS = {"sift": gen.SIFT_1M, "gist": gen.GIST_1M, "glove": gen.GLOVE_1183514}
COUNTERS = ("scaffold_evals", "harvest_evals", "prune_evals", "finalize_evals", "expansions")


def read_records(path: str = OUT) -> dict:
    """{workload key: {field: value}} from the text file ([key] sections of
    `field = value` lines)."""
    recs, cur = {}, None
    if not os.path.exists(path):
        return recs
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("[") and line.endswith("]"):
            cur = recs.setdefault(line[1:-1], {})
        elif cur is not None and "=" in line:
            k, v = line.split("=", 1)
            cur[k.strip()] = v.strip()
    return recs


def input_digest(x) -> str:
    return hashlib.sha256(x.tobytes(order="C")).hexdigest()


def record(key: str, threads: int) -> dict:
    w = WORKLOADS[key]
    t0 = time.perf_counter()
    x = gen.workload_data(w)
    tg = time.perf_counter() - t0
    metric = "cosine" if w.metric == "cosine" else "l2"
    P = fgo.params(w.T, w.ef_h, w.R, w.alpha, w.B, 0, threads)
    t1 = time.perf_counter()
    G = fgo.build_graph(fgo.Data(x, metric=metric), w.build_seed, P)
    wall = time.perf_counter() - t1
    c = G["counters"]
    rec = {"workload": w.name, "n": str(x.shape[0]), "d": str(x.shape[1]), "dtype": str(x.dtype),
           "metric": metric, "T": str(w.T), "B": str(w.B), "ef_h": str(w.ef_h), "R": str(w.R),
           "alpha": repr(w.alpha), "seed": str(w.build_seed), "input_sha256": input_digest(x),
           "graph_hash": f"{G['hash']:#018x}"}
    for k in COUNTERS:
        rec[k] = str(int(c[k]))
    rec["oracle_threads"] = str(threads)
    rec["oracle_build_wall_s"] = f"{wall:.1f}"
    rec["oracle_harvest_s"] = f"{c['t_harvest']:.1f}"
    rec["generate_s"] = f"{tg:.1f}"
    return rec


def write_records(recs: dict, path: str = OUT) -> None:
    with open(path, "w") as f:
        f.write("# Oracle whole builds at full size (written by tests/golden/make_fullsize.py;\n"
                "# seeded inputs from paper_2609_30493_amd.datagen, graphs from oracle/ only).\n")
        for key in ("sift", "gist", "glove"):
            if key not in recs:
                continue
            f.write(f"\n[{key}]\n")
            for k, v in recs[key].items():
                f.write(f"{k} = {v}\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="?", default="sift,gist,glove")
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    recs = read_records()
    for key in args.which.split(","):
        print(f"[golden] {key}: {WORKLOADS[key].name}, oracle on {args.threads} threads", flush=True)
        recs[key] = record(key, args.threads)
        print(f"[golden] {key}: {recs[key]}", flush=True)
        write_records(recs)


if __name__ == "__main__":
    main()
