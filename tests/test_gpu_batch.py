"""Batch of products as one graph launch (dh2_batch_*): problems of several
sizes, surfaces and wave numbers recorded into one HIP graph and replayed.
Every replay must reproduce the products of dh2_matvec bit for bit (the same
kernels in the same order per problem), with eager work between replays, and
one problem is checked against the FP64 oracle."""
import numpy as np
import pytest

import synth
from oracle.dh2 import OracleDH2
from tests.gpu_common import say, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec_name", ["fp64", "fp32"])
def test_batch_graph_replays_match_single_products(prec_name):
    import torch
    from paper_1809_04384_amd import dh2
    prec = dh2.FP64 if prec_name == "fp64" else dh2.FP32
    cdt = torch.complex128 if prec == dh2.FP64 else torch.complex64
    # two parity workloads with admissible blocks (at these sizes the batching
    # recipe's wave numbers leave only near fields) and three of the recipe
    ws = [synth.WORKLOADS["dir512"], synth.WORKLOADS["cube768"]] + \
        synth.batch_workloads(count=3, seed=7, n_lo=300, n_hi=2500)
    nrhs = 6
    hs, X, Ye, Yb, meshes = [], [], [], [], []
    try:
        for i, w in enumerate(ws):
            V, T = synth.make_mesh(w)
            meshes.append((V, T))
            say("[gpu] batch: build %s %s n=%d kappa=%g (%s)" % (w.name, w.surface, len(T), w.kappa, prec_name))
            hs.append(dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, precision=prec,
                                 max_nrhs=nrhs))
            X.append(torch.from_numpy(synth.complex_gaussian(len(T), nrhs, seed=30 + i)).to("cuda:0").to(cdt))
            Ye.append(torch.empty_like(X[-1]))
            Yb.append(torch.empty_like(X[-1]))
        for h, x, y in zip(hs, X, Ye):
            h.matvec(x, y)
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        say("[gpu] batch: capture %d problems" % len(hs))
        b = dh2.Batch(hs, X, Yb, stream=s.cuda_stream)
        try:
            for rep in range(3):
                for y in Yb:
                    y.zero_()
                torch.cuda.synchronize()
                with torch.cuda.stream(s):
                    b.run()
                s.synchronize()
                for i in range(len(hs)):
                    assert torch.equal(Yb[i], Ye[i]), (rep, i)
                # eager work between replays
                hs[0].matvec(X[0], Ye[0])
                torch.cuda.synchronize()
            say("[gpu] batch: 3 replays equal the single products")
        finally:
            b.free()
        # a problem with a far field against the oracle
        i0 = 0
        w = ws[i0]
        V, T = meshes[i0]
        o = OracleDH2(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1)
        Xn = X[i0].cpu().numpy().astype(np.complex128)
        err = rel(Yb[i0].cpu().numpy().astype(np.complex128), o.matvec(Xn.T).T)
        say("[gpu] batch: %s vs oracle rel err %.3e" % (w.name, err))
        assert err <= (1e-10 if prec == dh2.FP64 else 1e-4)
    finally:
        for h in hs:
            h.free()


def test_batch_rejects_repeated_handle_and_mixed_precision():
    import torch
    from paper_1809_04384_amd import dh2
    V, T = synth.sphere_octahedral(8)
    h64 = dh2.Handle(V, T, 4.0, 3, 1.0, 32, 1e-6)
    h32 = dh2.Handle(V, T, 4.0, 3, 1.0, 32, 1e-6, precision=dh2.FP32)
    try:
        x = torch.zeros((2, len(T)), dtype=torch.complex128, device="cuda:0")
        y = torch.empty_like(x)
        with pytest.raises(dh2.Dh2Error) as e:
            dh2.Batch([h64, h64], [x, x], [y, y])
        assert e.value.status == 1
        x32 = torch.zeros((2, len(T)), dtype=torch.complex64, device="cuda:0")
        with pytest.raises(dh2.Dh2Error) as e:
            dh2.Batch([h64, h32], [x, x32], [y, torch.empty_like(x32)])
        assert e.value.status == 1
    finally:
        h64.free()
        h32.free()


def test_build_many_equals_single_builds():
    """Builds side by side on per-problem streams (dh2_build_many) give the
    handles of one-by-one builds: the products agree bit for bit."""
    import torch
    from paper_1809_04384_amd import dh2
    ws = [synth.WORKLOADS["dir512"], synth.WORKLOADS["cube768"], synth.WORKLOADS["sphere2k"]] + \
        synth.batch_workloads(count=3, seed=7, n_lo=300, n_hi=2500)
    probs = []
    for w in ws:
        V, T = synth.make_mesh(w)
        probs.append((V, T, w.kappa, w.order, w.eta, w.leaf, w.tol))
    say("[gpu] build_many: %d problems, 4 threads" % len(probs))
    many = dh2.build_many(probs, max_nrhs=4, threads=4)
    single = []
    try:
        for (V, T, kappa, order, eta, leaf, tol) in probs:
            single.append(dh2.Handle(V, T, kappa, order, eta, leaf, tol, max_nrhs=4))
        for i, (hm, hs) in enumerate(zip(many, single)):
            X = torch.from_numpy(synth.complex_gaussian(hm.n, 3, seed=50 + i)).to("cuda:0")
            Ym, Ys = torch.empty_like(X), torch.empty_like(X)
            hm.matvec(X, Ym)
            hs.matvec(X, Ys)
            torch.cuda.synchronize()
            assert torch.equal(Ym, Ys), i
            assert hm.stats()["n_adm"] == hs.stats()["n_adm"]
        say("[gpu] build_many: products equal those of single builds")
    finally:
        for h in many + single:
            h.free()


def test_build_many_reports_the_failing_problem():
    """A problem that fails its build (a triangle index out of range, caught on
    the host) fails the whole call: the status is the problem's, the message
    names it, and no handle is returned."""
    from paper_1809_04384_amd import dh2
    V, T = synth.sphere_octahedral(4)
    bad = T.copy()
    bad[5, 2] = len(V) + 3
    probs = [(V, T, 4.0, 3, 1.0, 16, 1e-6), (V, bad, 4.0, 3, 1.0, 16, 1e-6), (V, T, 2.0, 3, 1.0, 16, 1e-6)]
    with pytest.raises(dh2.Dh2Error) as e:
        dh2.build_many(probs, threads=3)
    assert e.value.status == 2
    assert "problem 1" in str(e.value)
