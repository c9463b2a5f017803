"""Trains the learned rank predictor on the collected ranks and writes the
compiled-in weights (paper_1809_04384_amd/csrc/rank_mlp_weights.inc).

Model: 12 standardised features -> 128 -> 128 -> 128 -> 1 with ReLU, target
log2(1 + rank), mean squared error, full-batch Adam (numpy, float64), seeded.
Under-prediction costs an exact fallback, over-prediction a larger sketch, so
the loss weights errors below the target twice.  The weights are rounded to
BF16 at the end (the inference kernel multiplies BF16 weights with FP32
accumulation); the reported fit is that of the rounded model.

    python -m paper_1809_04384_amd.rank_model.train [data.npz]
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1809_04384_amd.rank_model.weights import write_inc, bf16_round, NF, NH  # noqa: E402
from paper_1809_04384_amd.rank_model.collect import DATA  # noqa: E402


def forward(p, Xs):
    h1 = np.maximum(Xs @ p["W1"].T + p["b1"], 0)
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0)
    h3 = np.maximum(h2 @ p["W3"].T + p["b3"], 0)
    return h3 @ p["W4"] + p["b4"], (h1, h2, h3)


def predict_ranks(p, X):
    """Ranks as the inference kernel computes them (BF16 weights)."""
    q = dict(p)
    for key in ("W1", "W2", "W3", "W4"):
        q[key] = bf16_round(p[key]).astype(np.float64)
    Xs = (X - p["mean"]) / p["std"]
    y, _ = forward(q, Xs)
    return np.maximum(0, np.rint(2.0 ** y - 1.0)).astype(int)


def train(data=DATA, steps=4000, lr=2e-3, seed=7):
    d = np.load(data)
    X = d["X"].astype(np.float64)
    t = np.log2(1.0 + d["y"].astype(np.float64))
    mean = X.mean(axis=0)
    std = X.std(axis=0)
    std[std < 1e-6] = 1.0
    Xs = (X - mean) / std
    rng = np.random.default_rng(seed)
    he = lambda fi, fo: rng.standard_normal((fo, fi)) * np.sqrt(2.0 / fi)
    p = {"W1": he(NF, NH), "b1": np.zeros(NH), "W2": he(NH, NH), "b2": np.zeros(NH),
         "W3": he(NH, NH), "b3": np.zeros(NH), "W4": rng.standard_normal(NH) * np.sqrt(1.0 / NH),
         "b4": float(t.mean())}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v2 = {k: np.zeros_like(v) for k, v in p.items()}
    n = len(t)
    for it in range(1, steps + 1):
        y, (h1, h2, h3) = forward(p, Xs)
        r = y - t
        w = np.where(r < 0, 2.0, 1.0)
        gy = 2.0 * w * r / n
        g = {"W4": h3.T @ gy, "b4": gy.sum()}
        d3 = np.outer(gy, p["W4"]) * (h3 > 0)
        g["W3"], g["b3"] = d3.T @ h2, d3.sum(0)
        d2 = (d3 @ p["W3"]) * (h2 > 0)
        g["W2"], g["b2"] = d2.T @ h1, d2.sum(0)
        d1 = (d2 @ p["W2"]) * (h1 > 0)
        g["W1"], g["b1"] = d1.T @ Xs, d1.sum(0)
        for k in p:
            m[k] = 0.9 * m[k] + 0.1 * g[k]
            v2[k] = 0.999 * v2[k] + 0.001 * g[k] * g[k]
            p[k] = p[k] - lr * (m[k] / (1 - 0.9 ** it)) / (np.sqrt(v2[k] / (1 - 0.999 ** it)) + 1e-8)
        if it % 1000 == 0:
            print("[train] step %d loss %.4f" % (it, float(np.mean(w * r * r))), flush=True)
    p["mean"], p["std"] = mean, std
    pr = predict_ranks(p, X)
    y = d["y"]
    print("[train] BF16 model: mean |rank error| %.2f, under-predicted %.1f %%, within 8 below or above %.1f %%"
          % (np.mean(np.abs(pr - y)), 100 * np.mean(pr < y), 100 * np.mean(np.abs(pr - y) <= 8)), flush=True)
    return p


if __name__ == "__main__":
    params = train(sys.argv[1] if len(sys.argv) > 1 else DATA)
    write_inc(params, note="trained on %s" % os.path.basename(DATA))
