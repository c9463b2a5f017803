"""GPU checks of the learned-rank form (options.rank_mode = learned): the
predicted rank of each (cluster, direction) sizes a randomized range finder
(Gaussian sketch), and the exact FP64 truncation is the fallback and the
judge.  Against the FP64 oracle (exact truncation of Section 3.2) on
workloads at tol 1e-4 and 1e-6:
  - every truncation meets the same block-relative rule, so the product's
    error against the interpolated matrix G_int stays within the tolerance and
    within twice the exact truncation's error;
  - ranks are never below the exact ones (up to near-ties of the rule);
  - the predictor kernel (BF16 weights, FP32 accumulation) gives the ranks a
    numpy forward pass of the same rounded weights gives (up to one, at
    rounding boundaries of 2^y - 1);
  - a planted under-prediction (every predicted rank 1, no oversampling)
    makes the sketches miss the tolerance, the fallback truncates those
    slots exactly, and the product still matches the exact one within the
    tolerance."""
import numpy as np
import pytest

import synth
from tests.gpu_common import say, oracle_for, build_handle, rel

pytestmark = pytest.mark.gpu

CASES = ["dir2k_t4", "cube1200dir", "sphere2k"]


def _matvec(h, X):
    import torch
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0")
    Yd = torch.empty_like(Xd)
    h.matvec(Xd, Yd)
    torch.cuda.synchronize()
    return Yd.cpu().numpy()


def _near_tie(sig, r_lo, eps):
    tail = np.cumsum((np.asarray(sig) ** 2)[::-1])[::-1]
    return np.any(np.abs(tail - eps * eps) <= 1e-6 * eps * eps)


@pytest.mark.parametrize("name", CASES)
def test_learned_ranks_meet_the_tolerance(name):
    from paper_1809_04384_amd import dh2
    o = oracle_for(name)
    h, slots = build_handle(name, rank_mode=dh2.RANKS_LEARNED)
    try:
        s = h.stats()
        say("[gpu] %s learned ranks: %d sketch slots, %d fallbacks, prediction %.2f ms"
            % (name, s["sketch_slots"], s["sketch_fallbacks"], s["ms_rank_predict"]))
        X = synth.complex_gaussian(o.n, 3, seed=0)
        Y = _matvec(h, X)
        Gi = o.dense_interp()
        Yi = (Gi @ X.T).T
        err = rel(Y, Yi)
        err_exact = rel(o.matvec(X.T).T, Yi)
        say("[gpu] %s vs G_int: learned %.3e, exact (oracle) %.3e, tol %g" % (name, err, err_exact, o.tol))
        assert err <= o.tol
        assert err <= 2.0 * err_exact + 1e-13
        for kind, ranks_o, sig_o in (("row", o.rank, o.sig), ("col", o.rankW, o.sigW)):
            rk = h.inspect("rank_" + kind)[:, 0].real.astype(int)
            for q, (t, c, f) in enumerate(slots.tolist()):
                if (t, c) in ranks_o and rk[q] < ranks_o[(t, c)]:
                    assert _near_tie(sig_o[(t, c)], rk[q], o.tol), (kind, t, c, rk[q], ranks_o[(t, c)])
    finally:
        h.free()


def test_predictor_kernel_matches_numpy():
    """The inference kernel against a numpy forward pass of the compiled-in
    weights (read back from the weight file)."""
    import os
    import re
    from paper_1809_04384_amd import dh2
    from paper_1809_04384_amd.rank_model.weights import INC
    txt = open(INC).read()

    def arr(name, dtype):
        body = re.search(r"%s\[\d+\] = \{([^}]*)\}" % name, txt).group(1)
        vals = [v.strip() for v in body.split(",")]
        if dtype == "bf16":
            return (np.array([int(v, 16) for v in vals], dtype=np.uint32) << 16).view(np.float32).astype(np.float64)
        return np.array([float(v.rstrip("f")) for v in vals])
    p = {"mean": arr("kMlpMean", "f"), "std": arr("kMlpStd", "f"),
         "W1": arr("kMlpW1", "bf16").reshape(128, 12), "b1": arr("kMlpB1", "f"),
         "W2": arr("kMlpW2", "bf16").reshape(128, 128), "b2": arr("kMlpB2", "f"),
         "W3": arr("kMlpW3", "bf16").reshape(128, 128), "b3": arr("kMlpB3", "f"),
         "W4": arr("kMlpW4", "bf16"), "b4": float(re.search(r"kMlpB4 = ([^;]*);", txt).group(1).rstrip("f"))}
    name = "dir2k_t4"
    w = synth.WORKLOADS[name]
    V, T = synth.make_mesh(w)
    h, slots = build_handle(name, rank_mode=dh2.RANKS_LEARNED)
    try:
        plan = dh2.Plan(V, T, w.kappa, w.order, w.eta, w.leaf, w.eta1)
        for kind in ("row", "col"):
            f = plan.rank_features(w.tol, kind).astype(np.float64)
            xs = (f - p["mean"]) / p["std"]
            h1 = np.maximum(xs @ p["W1"].T + p["b1"], 0)
            h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0)
            h3 = np.maximum(h2 @ p["W3"].T + p["b3"], 0)
            ref = np.maximum(0, np.rint(2.0 ** (h3 @ p["W4"] + p["b4"]) - 1.0))
            got = h.inspect("rank_pred_" + kind)[:, 0].real
            say("[gpu] predictor %s: %d slots, largest difference %d" % (kind, len(got), int(np.max(np.abs(got - ref)))))
            assert np.max(np.abs(got - ref)) <= 1
    finally:
        h.free()


def test_planted_under_prediction_falls_back_to_exact():
    from paper_1809_04384_amd import dh2
    name = "dir2k_t4"
    o = oracle_for(name)
    h, _ = build_handle(name, rank_mode=dh2.RANKS_LEARNED, sketch_rank=1)
    try:
        s = h.stats()
        say("[gpu] planted rank 1: %d sketch slots, %d fallbacks" % (s["sketch_slots"], s["sketch_fallbacks"]))
        assert s["sketch_slots"] > 0
        assert s["sketch_fallbacks"] >= s["sketch_slots"] // 2
        X = synth.complex_gaussian(o.n, 2, seed=3)
        Y = _matvec(h, X)
        Yo = o.matvec(X.T).T
        err = rel(Y, Yo)
        say("[gpu] planted rank 1: vs exact truncation (oracle) %.3e" % err)
        assert err <= o.tol
    finally:
        h.free()
