"""CPU tests of the learned rank predictor's host side: the features exported
by the library for every slot, the BF16 rounding of the weight writer, and
the compiled-in weights against the training data they were fitted to."""
import os
import re

import numpy as np

import synth
from paper_1809_04384_amd import dh2
from paper_1809_04384_amd.rank_model import weights as W
from paper_1809_04384_amd.rank_model.collect import DATA


def test_features_describe_the_slots():
    w = synth.WORKLOADS["dir2k_t4"]
    V, T = synth.make_mesh(w)
    plan = dh2.Plan(V, T, w.kappa, w.order, w.eta, w.leaf, w.eta1)
    e = plan.export()
    for kind, flag in (("row", 1), ("col", 2)):
        f = plan.rank_features(w.tol, kind)
        assert f.shape == (len(e["slots"]), 12) and np.all(np.isfinite(f))
        t = e["slots"][:, 0]
        assert np.allclose(f[:, 0], np.log2(e["size"][t]), atol=1e-6)
        assert np.allclose(f[:, 3], np.log10(w.tol), atol=1e-6)
        assert np.all(f[:, 4] == w.order) and np.all(f[:, 11] == w.eta)
        # slots whose list holds blocks (the active set of this kind) have f6 > 0 or inherit blocks (f7 > 0)
        active = (e["slots"][:, 2] & flag) != 0
        assert np.all((f[active, 6] > 0) | (f[active, 7] > 0))
        assert np.all((f[:, 5] == 0) | (f[:, 5] == 1)) and np.all((f[:, 9] >= 0) & (f[:, 9] <= 1))


def test_bf16_rounding_is_nearest_even():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(2000).astype(np.float32),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8], dtype=np.float32)])
    r = W.bf16_round(x)
    # the nearest of the two BF16 neighbours (upper 16 bits truncated, and the next one up in magnitude)
    u = x.view(np.uint32)
    lo = (u & 0xFFFF0000).view(np.float32)
    hi = ((u & 0xFFFF0000) + 0x10000).view(np.float32)
    best = np.where(np.abs(x - lo) < np.abs(hi - x), lo, hi)
    tie = np.abs(x - lo) == np.abs(hi - x)
    even = np.where(((u >> 16) & 1) == 0, lo, hi)
    assert np.array_equal(np.where(tie, even, best), r)
    assert r[-3] == 1.0 and r[-2] == np.float32(1.0 + 4 * 2 ** -8) and r[-1] == -1.0


def test_compiled_weights_fit_the_training_ranks():
    """The weight file parses, and its forward pass (BF16 weights) predicts the
    collected ranks closely, under-predicting rarely (each under-prediction
    costs an exact fallback)."""
    txt = open(W.INC).read()

    def arr(name, bf):
        vals = [v.strip() for v in re.search(r"%s\[\d+\] = \{([^}]*)\}" % name, txt).group(1).split(",")]
        if bf:
            return (np.array([int(v, 16) for v in vals], dtype=np.uint32) << 16).view(np.float32).astype(np.float64)
        return np.array([float(v.rstrip("f")) for v in vals])
    d = np.load(DATA)
    X = d["X"].astype(np.float64)
    xs = (X - arr("kMlpMean", False)) / arr("kMlpStd", False)
    h = np.maximum(xs @ arr("kMlpW1", True).reshape(128, 12).T + arr("kMlpB1", False), 0)
    h = np.maximum(h @ arr("kMlpW2", True).reshape(128, 128).T + arr("kMlpB2", False), 0)
    h = np.maximum(h @ arr("kMlpW3", True).reshape(128, 128).T + arr("kMlpB3", False), 0)
    b4 = float(re.search(r"kMlpB4 = ([^;]*);", txt).group(1).rstrip("f"))
    pred = np.maximum(0, np.rint(2.0 ** (h @ arr("kMlpW4", True) + b4) - 1.0))
    y = d["y"]
    assert np.mean(np.abs(pred - y)) <= 1.0
    assert np.mean(pred < y) <= 0.02
