"""GPU parity of the Gram form of the total weights (dh2_options.weights =
GRAM) against the FP64 oracle, which factors the stacked rows by Householder
QR as the construction of the total weights states.

Bounds.  The Gram matrix of a slot is a sum of FP64 products over up to a few
thousand stacked rows, and pivoted Cholesky stops at a pivot of nw 2^-52 of
the largest diagonal entry, so |R^H R - Z^H Z| <= c (K + nw^2) 2^-52 |Z|^2 per
level, compounded over the levels through the inherited rows; GRAM_EPS = 1e-10
covers that with a margin for nw <= 216 and the depths here.  Singular values,
ranks and Zhat^H Zhat are checked against it (tests/gpu_common.py), the
product against the oracle's to the accuracy the same bound allows: a basis
vector kept at singular value s moves by at most GRAM_EPS s_1^2 / gap, so the
product moves by at most the discarded tail plus that, which stays below the
tolerance eps of the workload (both products approximate the same matrix to
eps)."""
import numpy as np
import pytest

import synth
from tests.gpu_common import (say, oracle_for, build_handle, rel, check_ranks_and_sigma,
                               check_weight_invariants)

pytestmark = pytest.mark.gpu

GRAM_EPS = 1e-10
CASES = ["dir512", "cube768", "sphere2k", "cube1200dir", "dir2k", "dir2k_t4", "cube768_m6"]


@pytest.mark.parametrize("name", CASES)
def test_gram_weights_match_oracle(name):
    import torch
    from paper_1809_04384_amd import dh2
    o = oracle_for(name)
    h, slots = build_handle(name, weights=dh2.WEIGHTS_GRAM)
    try:
        st = h.stats()
        assert st["weights_gram"] == 1
        check_ranks_and_sigma(h, slots, o, name + " gram", gram_eps=GRAM_EPS)
        check_weight_invariants(h, slots, o, name + " gram", tol_total=GRAM_EPS)
        X = synth.complex_gaussian(o.n, 3, seed=7)
        Xd = torch.from_numpy(X).to("cuda:0")
        Yd = torch.empty_like(Xd)
        h.matvec(Xd, Yd)
        torch.cuda.synchronize()
        Y = Yd.cpu().numpy()
        Yo = o.matvec(X.T).T
        err = rel(Y, Yo)
        say("[gpu] %s gram matvec rel err vs oracle %.3e (tol %g)" % (name, err, o.tol))
        assert err <= o.tol
    finally:
        h.free()


def test_gram_falls_back_below_its_tolerance():
    """tol below 1e-7: the Gram form is not taken (the Householder factors
    run, and the result is the Householder handle's bit for bit)."""
    import torch
    from paper_1809_04384_amd import dh2
    w = synth.WORKLOADS["dir512"]
    V, T = synth.make_mesh(w)
    hs = [dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, 1e-9, eta1=w.eta1, weights=m)
          for m in (dh2.WEIGHTS_GRAM, dh2.WEIGHTS_HOUSEHOLDER)]
    try:
        assert [h.stats()["weights_gram"] for h in hs] == [0, 0]
        X = torch.from_numpy(synth.complex_gaussian(len(T), 2, seed=3)).to("cuda:0")
        Ys = []
        for h in hs:
            Y = torch.empty_like(X)
            h.matvec(X, Y)
            Ys.append(Y)
        torch.cuda.synchronize()
        assert torch.equal(Ys[0], Ys[1])
    finally:
        for h in hs:
            h.free()
