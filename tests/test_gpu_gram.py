"""GPU parity of the Gram form of the block and total weights
(dh2_options.weights = GRAM) against the FP64 oracle, which factors the
stacked rows by Householder QR as the construction of the total weights
states.

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
from oracle.dh2 import OracleDH2
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
        # regression level: these seeded cases have a clear gap at every
        # truncation, where the perturbation stays near GRAM_EPS (seen: <= 2e-11)
        assert err <= 1e-9
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


@pytest.mark.parametrize("name", ["dir512", "sphere2k", "cube1200dir"])
def test_gram_weights_spectral_control(name):
    """Spectral error control in the Gram form: the block weights (norms of
    R_tc S_b R_sc^*, formed from the same stacked rows the Gram matrices take)
    element by element, ranks and singular values within the Gram bounds, and
    the product against the oracle built with the same rule."""
    import torch
    from paper_1809_04384_amd import dh2
    o = oracle_for(name, norm="spectral")
    h, slots = build_handle(name, norm=dh2.NORM_SPECTRAL, weights=dh2.WEIGHTS_GRAM)
    try:
        assert h.stats()["weights_gram"] == 1
        om = h.inspect("omega")[:, 0].real
        assert om.shape == o.omega.shape
        if len(om):
            err = np.max(np.abs(om - o.omega) / o.omega)
            say("[gpu] %s gram spectral block weights: max rel err %.3e" % (name, err))
            assert err <= 1e-12
        check_ranks_and_sigma(h, slots, o, name + " gram spectral", gram_eps=GRAM_EPS, spectral=True)
        X = synth.complex_gaussian(o.n, 3, seed=0)
        Xd = torch.from_numpy(X).to("cuda:0")
        Yd = torch.empty_like(Xd)
        h.matvec(Xd, Yd)
        torch.cuda.synchronize()
        err = rel(Yd.cpu().numpy(), o.matvec(X.T).T)
        say("[gpu] %s gram spectral matvec rel err vs oracle %.3e (tol %g)" % (name, err, o.tol))
        assert err <= o.tol
    finally:
        h.free()


def test_gram_weights_small_workspace():
    """A workspace of a few blocks: many batches in the block pass and chunks
    in the top-down pass give the Gram matrices of the default workspace (the
    same products, summed in another grouping) to rounding."""
    import torch
    from paper_1809_04384_amd import dh2
    name = "dir2k"
    w = synth.WORKLOADS[name]
    V, T = synth.make_mesh(w)
    big = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, weights=dh2.WEIGHTS_GRAM)
    k = w.order ** 3
    ws_gb = 60 * 5 * k * k * 16 / 2.0 ** 30        # 60 blocks per batch
    small = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, weights=dh2.WEIGHTS_GRAM,
                       workspace_gb=ws_gb)
    try:
        sb, ss = big.stats(), small.stats()
        say("[gpu] %s gram batches: default %d / %d / %d, small workspace %d / %d / %d"
            % (name, sb["batches_block_weights"], sb["batches_total_weights_row"], sb["batches_total_weights_col"],
               ss["batches_block_weights"], ss["batches_total_weights_row"], ss["batches_total_weights_col"]))
        assert ss["batches_block_weights"] > 10 * sb["batches_block_weights"]
        assert ss["batches_total_weights_row"] > sb["batches_total_weights_row"]
        for kind in ("row", "col"):
            assert np.array_equal(big.inspect("rank_" + kind), small.inspect("rank_" + kind))
        X = torch.from_numpy(synth.complex_gaussian(len(T), 2, seed=5)).to("cuda:0")
        Y1, Y2 = torch.empty_like(X), torch.empty_like(X)
        big.matvec(X, Y1)
        small.matvec(X, Y2)
        torch.cuda.synchronize()
        d = float(torch.linalg.norm(Y1 - Y2) / torch.linalg.norm(Y1))
        say("[gpu] %s gram small workspace product rel diff %.3e" % (name, d))
        assert d <= 1e-9
    finally:
        big.free()
        small.free()


@pytest.mark.parametrize("name", ["sphere2k", "dir2k"])
def test_gram_weights_fp32_form(name):
    """FP32 form with Gram weights: the stacked rows come from the FP32
    matrix cores, their Gram matrices from the FP64 ones.  The product agrees
    with the FP64 oracle to the FP32 form's 1e-4, and ranks differ from the
    FP64 Gram build in a few slots at most (FP32-sized perturbations of the
    rows, as in the Householder FP32 form)."""
    import torch
    from paper_1809_04384_amd import dh2
    o = oracle_for(name)
    w = synth.WORKLOADS[name]
    V, T = synth.make_mesh(w)
    h32 = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, precision=dh2.FP32,
                     max_nrhs=4, weights=dh2.WEIGHTS_GRAM)
    h64 = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, weights=dh2.WEIGHTS_GRAM)
    try:
        assert h32.stats()["weights_gram"] == 1
        for kind in ("row", "col"):
            r32 = h32.inspect("rank_" + kind)[:, 0].real.astype(int)
            r64 = h64.inspect("rank_" + kind)[:, 0].real.astype(int)
            nd = int(np.count_nonzero(r32 != r64))
            say("[gpu] %s gram FP32 %s ranks differing from FP64: %d of %d" % (name, kind, nd, r32.size))
            assert nd <= max(3, r32.size // 50)
        X = synth.complex_gaussian(o.n, 4, seed=11)
        Xd = torch.from_numpy(X.astype(np.complex64)).to("cuda:0")
        Yd = torch.empty_like(Xd)
        h32.matvec(Xd, Yd)
        torch.cuda.synchronize()
        err = rel(Yd.cpu().numpy().astype(np.complex128), o.matvec(X.T).T)
        say("[gpu] %s gram FP32 matvec rel err vs oracle %.3e" % (name, err))
        assert err <= 1e-4
    finally:
        h32.free()
        h64.free()


def test_gram_weights_edge_cases():
    """Gram weights where the structure degenerates: a mesh smaller than one
    leaf (no admissible block, so both block passes and the top-down pass
    have nothing to do) and kappa = 0 (one direction per level, real
    couplings); both against the oracle, built as the benchmark builds
    (autotuned block rows)."""
    import torch
    from paper_1809_04384_amd import dh2
    V, T = synth.sphere_octahedral(2)                       # n = 32 <= leaf
    o = OracleDH2(V, T, 3.0, 3, 1.0, 64, 1e-6)
    assert len(o.st.adm) == 0
    h = dh2.Handle(V, T, 3.0, 3, 1.0, 64, 1e-6, weights=dh2.WEIGHTS_GRAM, autotune=1)
    try:
        assert h.stats()["n_adm"] == 0 and h.stats()["weights_gram"] == 1
        X = synth.complex_gaussian(len(T), 3, seed=2)
        Xd = torch.from_numpy(X).to("cuda:0")
        Yd = torch.empty_like(Xd)
        h.matvec(Xd, Yd)
        torch.cuda.synchronize()
        err = rel(Yd.cpu().numpy(), o.matvec(X.T).T)
        say("[gpu] gram single leaf rel err %.3e" % err)
        assert err <= 1e-12
    finally:
        h.free()
    w = synth.WORKLOADS["sphere2k"]
    V, T = synth.make_mesh(w)
    o = OracleDH2(V, T, 0.0, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1)
    h = dh2.Handle(V, T, 0.0, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, weights=dh2.WEIGHTS_GRAM, autotune=1)
    try:
        assert h.stats()["n_adm"] == len(o.st.adm)
        X = synth.complex_gaussian(len(T), 5, seed=1)
        Xd = torch.from_numpy(X).to("cuda:0")
        Yd = torch.empty_like(Xd)
        h.matvec(Xd, Yd)
        torch.cuda.synchronize()
        err = rel(Yd.cpu().numpy(), o.matvec(X.T).T)
        say("[gpu] gram kappa 0 rel err %.3e" % err)
        assert err <= 1e-9
    finally:
        h.free()


def test_couplings_formed_inside_products():
    """Where a phase needs a coupling S_b only through a product with it, FP64
    builds evaluate S_b inside that product (k_gemm_coupling) and never store
    it: both Gram passes with the Frobenius norm (R_tc S_b, R_sc S_b^H /
    omega_b) and the projection (C_tc S_b).  The spectral norm needs S_b
    itself in the first pass, the Householder form stores it for its block and
    total weights; the products of every form are checked against the oracle
    by the tests above.  The FP32 and split-BF16x3 forms do the same in their
    own product arithmetic.
    Counts per admissible block, k = 64 (one 128-row chunk per product)."""
    from paper_1809_04384_amd import dh2
    cases = [
        ("gram, frobenius, fp64", dict(weights=dh2.WEIGHTS_GRAM), 3.0, 3.0),
        ("gram, spectral, fp64", dict(weights=dh2.WEIGHTS_GRAM, norm=dh2.NORM_SPECTRAL), 3.0, 2.0),
        ("householder, fp64", dict(weights=dh2.WEIGHTS_HOUSEHOLDER), 4.0, 1.0),
        ("gram, fp32", dict(weights=dh2.WEIGHTS_GRAM, precision=dh2.FP32), 3.0, 3.0),
        ("gram, bf16x3", dict(weights=dh2.WEIGHTS_GRAM, precision=dh2.BF16X3), 3.0, 3.0),
    ]
    for label, kw, gen, inside in cases:
        h, _ = build_handle("sphere2k", **kw)
        try:
            st = h.stats()
            say("[gpu] sphere2k %s: S_b generated %.2f x per block, %.2f x inside products"
                % (label, st["coupling_regeneration"], st["coupling_in_products"]))
            assert st["n_adm"] > 0
            assert st["coupling_regeneration"] == gen, label
            assert st["coupling_in_products"] == inside, label
        finally:
            h.free()
