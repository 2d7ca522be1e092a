"""Schedule sweep and selector training for the look-ahead LU library.

The learned schedule selector (a 4 -> 32 -> 10 perceptron, see include/lu.h)
picks the block size b, the look-ahead depth and the panel CU share for a
problem size and precision.  It learns from timings the factorization itself
produces on the machine it runs on:

  sweep   time lu_factor_ex for every schedule of the grid
          b in {64,128,256,512} x depth in {0,1,2} x panel CUs in {8,16,32}
          at the given sizes and precisions (medians of --reps runs, HIP
          events on the factorization's stream) and write a JSON table;
  train   label every (n, precision) of the training sizes with its fastest
          schedule and fit the network on the GPU with the library's own
          forward/backward/Adam kernels (lu_selector_train); write the weights
          file the library loads by default (selector_weights.bin next to the
          shared library);
  regret  for held-out sizes, compare the selected schedule's time with the
          best of the sweep (and with the fixed default).

Example:
  python -m paper_1804_07017_amd.tune sweep --sizes 1024,2048,4096 --precs 0,1,2 --out sweep.json
  python -m paper_1804_07017_amd.tune train --sweep sweep.json --out weights.bin
  python -m paper_1804_07017_amd.tune regret --sweep sweep.json --weights weights.bin --heldout 12000,20000
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

# The library sources that decide how long lu_factor_ex takes (kernels of the
# factorization, its scheduler and the panel boundaries).  A sweep records their
# hash; timings taken with other sources describe another library.
TIMED_SOURCES = ("panel.hip", "update.hip", "gemm.hip", "api.cpp", "plan.cpp", "plan.hpp", "kernels.hpp",
                 "common.hpp", "moves.hpp", "mfma.hpp", "state.hpp")
# environment settings that change the schedule or the kernels' launch shapes
SCHEDULE_ENV = ("LU_B", "LU_DEPTH", "LU_PANEL_CUS", "LU_TAPER", "LU_TAPER_MID", "LU_TAPER_NARROW", "LU_WIDE_ROWS",
                "LU_PANEL_OCC", "LU_PANEL_XCD", "LU_ISLAND")


def build_identity():
    """Hash (first 16 hex digits of SHA-256) of TIMED_SOURCES, in that order,
    and the taper setting the sweep runs with (the library default: on)."""
    import hashlib
    h = hashlib.sha256()
    for name in TIMED_SOURCES:
        with open(os.path.join(HERE, "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return {"lu_sources_sha256_16": h.hexdigest()[:16], "sources": list(TIMED_SOURCES), "taper": 1}


B_CHOICES = (64, 128, 256, 512)
DEPTH_CHOICES = (0, 1, 2)
CU_CHOICES = (8, 16, 32)
PRECS = {0: "fp64", 1: "fp32", 2: "mixed_fp16"}
DEFAULT = (256, 1, 16)


def schedules():
    return [(b, d, p) for b in B_CHOICES for d in DEPTH_CHOICES for p in CU_CHOICES]


def features(n: int, prec: int):
    """Network inputs: (log2 n - 14) / 3 and a one-hot of FP64 / FP32 / mixed."""
    x = [(math.log2(n) - 14.0) / 3.0, 0.0, 0.0, 0.0]
    x[1 + (2 if prec >= 2 else prec)] = 1.0
    return x


def labels(sched):
    b, d, p = sched
    return [B_CHOICES.index(b), DEPTH_CHOICES.index(d), CU_CHOICES.index(p)]


METHOD = ("median of lu_factor_ex runs timed with HIP events on the factorization's stream after one warm-up run "
          "per size and precision; uniform[-1,1) matrices from torch's device generator, seed 1; default taper; "
          "{train} runs per point at the training sizes, {held} at the held-out sizes")


def sweep(sizes, precs, reps, out, seed=1, role="train"):
    import torch
    import paper_1804_07017_amd as lu
    lu.load()
    torch.cuda.set_device(0)
    set_env = [k for k in SCHEDULE_ENV if os.environ.get(k)]
    if set_env:
        raise RuntimeError("schedule settings in the environment (%s): the sweep times the defaults" % set_env)
    ident = build_identity()
    table = {"device": torch.cuda.get_device_name(0), "reps": reps, "build": ident, "entries": []}
    if os.path.exists(out):
        with open(out) as f:
            table = json.load(f)
        if table.get("build") != ident:
            raise RuntimeError("%s was swept with other library sources or taper (%s), not %s" %
                               (out, table.get("build"), ident))
    key = "train_sizes" if role == "train" else "heldout_sizes"
    table.setdefault("train_sizes", [])
    table.setdefault("heldout_sizes", [])
    table.setdefault("runs", {})
    table["runs"][role] = reps
    for n in sizes:
        if n not in table[key]:
            table[key].append(n)
    table[key].sort()
    table["method"] = METHOD.format(train=table["runs"].get("train", "?"), held=table["runs"].get("heldout", "?"))
    done = {(e["n"], e["prec"], e["b"], e["depth"], e["panel_cus"]) for e in table["entries"]}
    stream = torch.cuda.Stream()
    for prec in precs:
        dt = torch.float64 if prec == 0 else torch.float32
        for n in sizes:
            g = torch.Generator(device="cuda")
            g.manual_seed(seed)
            A0 = lu.colmajor(n, dtype=dt)
            A0.uniform_(-1.0, 1.0, generator=g)
            A = lu.colmajor(n, dtype=dt)
            ipiv = torch.zeros(n, dtype=torch.int32, device="cuda")
            warm = False
            for sc in schedules():
                if (n, prec, *sc) in done:
                    continue
                times = []
                for r in range(reps + (0 if warm else 1)):
                    with torch.cuda.stream(stream):
                        A.copy_(A0)
                        e0 = torch.cuda.Event(enable_timing=True)
                        e1 = torch.cuda.Event(enable_timing=True)
                        e0.record(stream)
                        rc = lu.lu_factor_ex(A, ipiv, prec=prec, sched=sc, stream=stream)
                        e1.record(stream)
                    stream.synchronize()
                    if rc != 0:
                        raise RuntimeError("lu_factor_ex returned %d for n=%d prec=%d %s" % (rc, n, prec, sc))
                    if warm:
                        times.append(e0.elapsed_time(e1))
                    warm = True
                entry = {"n": n, "prec": prec, "b": sc[0], "depth": sc[1], "panel_cus": sc[2],
                         "ms": [round(t, 4) for t in times], "median": round(statistics.median(times), 4)}
                table["entries"].append(entry)
                print("sweep prec=%s n=%d b=%d depth=%d cus=%d: %.3f ms" % (PRECS[prec], n, *sc, entry["median"]),
                      flush=True)
                with open(out, "w") as f:
                    json.dump(table, f, indent=0)
            del A0, A, ipiv
            torch.cuda.empty_cache()
    return table


def best_table(entries):
    """(n, prec) -> {schedule: median ms}."""
    tab = {}
    for e in entries:
        tab.setdefault((e["n"], e["prec"]), {})[(e["b"], e["depth"], e["panel_cus"])] = e["median"]
    return tab


def train(sweep_files, sizes, out, epochs=3000, lr=0.02, seed=0):
    import numpy as np
    import paper_1804_07017_amd as lu
    lu.load()
    entries = []
    for s in sweep_files:
        with open(s) as f:
            entries += json.load(f)["entries"]
    tab = best_table(entries)
    X, Y = [], []
    for (n, prec), times in sorted(tab.items()):
        if sizes and n not in sizes:
            continue
        if len(times) < len(schedules()):
            continue
        bestsc = min(times, key=times.get)
        X.append(features(n, prec))
        Y.append(labels(bestsc))
    X = np.array(X, dtype=np.float32)
    Y = np.array(Y, dtype=np.int32)
    if len(X) == 0:
        raise SystemExit("no complete (n, precision) rows in the sweep")
    assert lu.lu_selector_load(None) == 0           # start from the seeded initialisation
    rc, losses = lu.lu_selector_train(X, Y, epochs, lr=lr, seed=seed)
    if rc != 0:
        raise SystemExit("lu_selector_train returned %d" % rc)
    rc = lu.lu_selector_save(out)
    if rc != 0:
        raise SystemExit("lu_selector_save returned %d" % rc)
    print("train: %d examples, loss %.4f -> %.4f, weights -> %s" % (len(X), losses[0], losses[-1], out), flush=True)
    return losses


def regret(sweep_files, weights, sizes):
    import paper_1804_07017_amd as lu
    lu.load()
    entries = []
    for s in sweep_files:
        with open(s) as f:
            entries += json.load(f)["entries"]
    tab = best_table(entries)
    if lu.lu_selector_load(weights) != 0:
        raise SystemExit("cannot load %s" % weights)
    rows = []
    for (n, prec), times in sorted(tab.items()):
        if sizes and n not in sizes:
            continue
        if len(times) < len(schedules()):
            continue
        best = min(times.values())
        rc, sc = lu.lu_selector_predict(n, prec)
        rows.append({"n": n, "prec": prec, "selected": sc, "regret": times[sc] / best - 1.0,
                     "default_regret": times[DEFAULT] / best - 1.0, "best": min(times, key=times.get)})
        print("regret prec=%s n=%d selected=%s %.2f%% (default %.2f%%, best %s)" % (
            PRECS[prec], n, sc, 100 * rows[-1]["regret"], 100 * rows[-1]["default_regret"], rows[-1]["best"]),
            flush=True)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("sweep")
    s.add_argument("--sizes", required=True)
    s.add_argument("--precs", default="0,1,2")
    s.add_argument("--reps", type=int, default=3)
    s.add_argument("--out", required=True)
    s.add_argument("--role", choices=("train", "heldout"), default="train",
                   help="list the sizes among the training or the held-out sizes of the table")
    t = sub.add_parser("train")
    t.add_argument("--sweep", required=True, help="comma-separated sweep JSON files")
    t.add_argument("--sizes", default="", help="training sizes (default: every complete size)")
    t.add_argument("--epochs", type=int, default=3000)
    t.add_argument("--lr", type=float, default=0.02)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--out", required=True)
    r = sub.add_parser("regret")
    r.add_argument("--sweep", required=True)
    r.add_argument("--weights", required=True)
    r.add_argument("--heldout", default="")
    a = ap.parse_args(argv)
    ints = lambda txt: [int(v) for v in txt.split(",") if v]
    if a.cmd == "sweep":
        t0 = time.time()
        sweep(ints(a.sizes), ints(a.precs), a.reps, a.out, role=a.role)
        print("sweep done in %.1f s" % (time.time() - t0), flush=True)
    elif a.cmd == "train":
        train(a.sweep.split(","), set(ints(a.sizes)), a.out, a.epochs, a.lr, a.seed)
    else:
        regret(a.sweep.split(","), a.weights, set(ints(a.heldout)))


if __name__ == "__main__":
    main()
