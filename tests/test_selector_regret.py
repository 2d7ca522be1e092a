"""The trained schedule selector against the exhaustive sweep it was trained
from (measured on MI355X, stored next to the library): on the held-out sizes
the selected schedule is within 5 % of the fastest schedule of the sweep, and
on average it beats the fixed default the library uses without the network.

The predictions here come from the FP64 oracle of the network applied to the
committed weights; the GPU test in test_gpu_selector.py checks that the
library's own inference kernel makes the same choices."""
import json
import os
import struct

import numpy as np
import pytest

from oracle import mlp
from paper_1804_07017_amd import tune

PKG = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1804_07017_amd")


def load_weights(path=os.path.join(PKG, "selector_weights.bin")):
    with open(path, "rb") as f:
        raw = f.read()
    assert raw[:8] == b"LUSEL001"
    n_min, n_max, npar = struct.unpack("<3i", raw[8:20])
    assert npar == mlp.N_PARAM
    theta = np.frombuffer(raw[20:20 + 4 * npar], dtype="<f4").astype(np.float64)
    return theta, n_min, n_max


def sweep():
    with open(os.path.join(PKG, "selector_sweep_mi355x.json")) as f:
        d = json.load(f)
    return d, tune.best_table(d["entries"])


def choose(theta, n, prec):
    pr = mlp.predict(theta, np.array([tune.features(n, prec)]))[0]
    return tune.B_CHOICES[pr[0]], tune.DEPTH_CHOICES[pr[1]], tune.CU_CHOICES[pr[2]]


def test_sweep_matches_the_library_sources():
    """The sweep was timed with the factorization sources and the taper
    setting of this tree; after a change to any of them the timings describe
    another library, and the sweep (and the training) must be redone."""
    d, _ = sweep()
    assert d.get("build") == tune.build_identity(), (
        "selector_sweep_mi355x.json was taken with %s; the tree has %s: re-run tune.py sweep/train"
        % (d.get("build"), tune.build_identity()))


def test_sweep_is_exhaustive_on_every_size():
    d, tab = sweep()
    for n in d["train_sizes"] + d["heldout_sizes"]:
        for prec in (0, 1, 2):
            assert set(tab[(n, prec)]) == set(tune.schedules()), (n, prec)
    assert not set(d["train_sizes"]) & set(d["heldout_sizes"])


def test_weights_cover_the_training_range():
    theta, n_min, n_max = load_weights()
    d, _ = sweep()
    assert np.isfinite(theta).all()
    assert n_min == min(d["train_sizes"]) and n_max == max(d["train_sizes"])


def test_held_out_regret_within_5_percent_and_gain_over_default():
    theta, _, _ = load_weights()
    d, tab = sweep()
    regrets, default_regrets = [], []
    for n in d["heldout_sizes"]:
        for prec in (0, 1, 2):
            times = tab[(n, prec)]
            best = min(times.values())
            regrets.append(times[choose(theta, n, prec)] / best - 1.0)
            default_regrets.append(times[tune.DEFAULT] / best - 1.0)
    print("selector regret: mean %.2f%% max %.2f%%; fixed default: mean %.2f%% max %.2f%%" % (
        100 * np.mean(regrets), 100 * max(regrets), 100 * np.mean(default_regrets), 100 * max(default_regrets)))
    assert max(regrets) <= 0.05
    # what the network gains over the fixed default on unseen sizes
    assert np.mean(regrets) < np.mean(default_regrets)
    assert sum(r < dr for r, dr in zip(regrets, default_regrets)) >= len(regrets) // 2


def test_training_labels_are_fitted():
    theta, _, _ = load_weights()
    d, tab = sweep()
    hits = 0
    total = 0
    for n in d["train_sizes"]:
        for prec in (0, 1, 2):
            times = tab[(n, prec)]
            total += 1
            hits += choose(theta, n, prec) == min(times, key=times.get)
    assert hits >= 0.9 * total
