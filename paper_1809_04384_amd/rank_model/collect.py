"""Training data of the learned rank predictor: the exact FP64 ranks of the
row and column bases of the unit-sphere workloads n = 2048 (kappa 4, m 4,
leaf 32, tol 1e-6), n = 32768 (kappa 16, m 5, leaf 64, tol 1e-6) and
n = 131072 (kappa 32, m 5, leaf 64, tol 1e-4), with the library's features of
the same slots.  Needs a GPU (one build per workload).

    python -m paper_1809_04384_amd.rank_model.collect [out.npz]
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DATA = os.path.join(HERE, "ranks_sphere_2k_32k_131k.npz")
WORKLOADS = ["sphere2k", "sphere32k", "sphere131k"]


def collect(out=DATA):
    import synth
    from paper_1809_04384_amd import dh2
    X, y, wid = [], [], []
    for i, name in enumerate(WORKLOADS):
        w = synth.WORKLOADS[name]
        V, T = synth.make_mesh(w)
        print("[collect] %s: build" % name, flush=True)
        h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, max_nrhs=1)
        plan = dh2.Plan(V, T, w.kappa, w.order, w.eta, w.leaf, w.eta1)
        for kind in ("row", "col"):
            r = h.inspect("rank_" + kind)[:, 0].real.astype(int)
            f = plan.rank_features(w.tol, kind)
            keep = r >= 0
            X.append(f[keep])
            y.append(r[keep])
            wid.append(np.full(int(keep.sum()), i))
        h.free()
        print("[collect] %s: %d slots" % (name, int(keep.sum())), flush=True)
    np.savez_compressed(out, X=np.vstack(X), y=np.concatenate(y), workload=np.concatenate(wid),
                        names=np.array(WORKLOADS))
    print("[collect] wrote %s" % out, flush=True)


if __name__ == "__main__":
    collect(sys.argv[1] if len(sys.argv) > 1 else DATA)
