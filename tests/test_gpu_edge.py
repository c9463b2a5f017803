"""GPU edge cases of the C ABI against the FP64 oracle: a mesh smaller than
one leaf (no admissible block: the matvec is the dense near field), the
Laplace case kappa = 0 (one direction per level), tol = 0 (every nonzero
singular value kept), the largest right-hand-side count a handle reserves and
one beyond it, a handle on a non-default stream and a product on a per-call
stream, and bitwise repeatability (the matvec adds partial sums in a fixed
order, without atomics)."""
import numpy as np
import pytest

import synth
from oracle.dh2 import OracleDH2
from tests.gpu_common import say, rel

pytestmark = pytest.mark.gpu


def _oracle(V, T, kappa, order, eta, leaf, tol, eta1=10.0):
    return OracleDH2(V, T, kappa, order, eta, leaf, tol, eta1=eta1)


def _run(h, X, dtype=np.complex128):
    import torch
    Xd = torch.from_numpy(np.ascontiguousarray(X.astype(dtype))).to("cuda:0")
    Yd = torch.empty_like(Xd)
    h.matvec(Xd, Yd)
    torch.cuda.synchronize()
    return Yd.cpu().numpy().astype(np.complex128)


def test_single_leaf_mesh_is_dense_near_field():
    from paper_1809_04384_amd import dh2
    V, T = synth.sphere_octahedral(2)                       # n = 32 <= leaf
    o = _oracle(V, T, 3.0, 3, 1.0, 64, 1e-8)
    assert len(o.st.adm) == 0
    for prec, dtype, bound in ((dh2.FP64, np.complex128, 1e-12), (dh2.FP32, np.complex64, 1e-5),
                               (dh2.BF16X3, np.complex64, 1e-5)):
        say("[gpu] edge: single leaf n=%d precision=%d" % (len(T), prec))
        h = dh2.Handle(V, T, 3.0, 3, 1.0, 64, 1e-8, precision=prec)
        try:
            s = h.stats()
            assert s["n_adm"] == 0 and s["n_near"] == 1
            for nrhs in (1, 2, 7):
                X = synth.complex_gaussian(len(T), nrhs, seed=nrhs)
                err = rel(_run(h, X, dtype), o.matvec(X.T).T)
                assert err <= bound, (prec, nrhs, err)
        finally:
            h.free()


def test_laplace_kappa_zero():
    from paper_1809_04384_amd import dh2
    w = synth.WORKLOADS["sphere2k"]
    V, T = synth.make_mesh(w)
    o = _oracle(V, T, 0.0, w.order, w.eta, w.leaf, w.tol)
    say("[gpu] edge: kappa 0 n=%d" % len(T))
    h = dh2.Handle(V, T, 0.0, w.order, w.eta, w.leaf, w.tol)
    try:
        assert h.stats()["n_adm"] == len(o.st.adm)
        X = synth.complex_gaussian(len(T), 5, seed=1)
        err = rel(_run(h, X), o.matvec(X.T).T)
        say("[gpu] kappa 0 matvec rel err %.3e" % err)
        assert err <= 1e-10
    finally:
        h.free()


def test_tol_zero_keeps_full_rank():
    """tol = 0: no truncation beyond the numerical rank, so the compressed
    matrix equals the interpolated one up to rounding."""
    from paper_1809_04384_amd import dh2
    w = synth.WORKLOADS["dir512"]
    V, T = synth.make_mesh(w)
    o = _oracle(V, T, w.kappa, w.order, w.eta, w.leaf, 0.0, eta1=w.eta1)
    say("[gpu] edge: tol 0 n=%d" % len(T))
    h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, 0.0, eta1=w.eta1)
    try:
        X = synth.complex_gaussian(len(T), 3, seed=2)
        Y = _run(h, X)
        err = rel(Y, o.matvec(X.T).T)
        ref = o.matvec_interp(X.T).T
        say("[gpu] tol 0 matvec rel err vs oracle %.3e, vs interpolated %.3e" % (err, rel(Y, ref)))
        assert err <= 1e-10
        assert rel(Y, ref) <= 1e-10
    finally:
        h.free()


def test_largest_reserved_rhs_count_and_one_beyond():
    from paper_1809_04384_amd import dh2
    import torch
    w = synth.WORKLOADS["dir2k"]
    V, T = synth.make_mesh(w)
    o = _oracle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1)
    say("[gpu] edge: max_nrhs 37 n=%d" % len(T))
    h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, max_nrhs=37)
    try:
        X = synth.complex_gaussian(len(T), 37, seed=3)        # two full chunks of 16 and a ragged 5
        err = rel(_run(h, X), o.matvec(X.T).T)
        say("[gpu] nrhs 37 rel err %.3e" % err)
        assert err <= 1e-10
        X38 = torch.zeros((38, len(T)), dtype=torch.complex128, device="cuda:0")
        with pytest.raises(dh2.Dh2Error) as e:
            h.matvec(X38, torch.empty_like(X38))
        assert e.value.status == 1
        X0 = torch.zeros((1, len(T)), dtype=torch.complex128, device="cuda:0")
        with pytest.raises(dh2.Dh2Error):
            h.matvec_ptr(X0.data_ptr(), X0.data_ptr(), 0)     # nrhs 0 is out of range
    finally:
        h.free()


def test_side_stream_and_bitwise_repeatability():
    from paper_1809_04384_amd import dh2
    import torch
    w = synth.WORKLOADS["sphere2k"]
    V, T = synth.make_mesh(w)
    n = len(T)
    say("[gpu] edge: side stream n=%d" % n)
    h0 = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol)
    s = torch.cuda.Stream()
    h1 = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, stream=s.cuda_stream)
    try:
        X = torch.from_numpy(synth.complex_gaussian(n, 16, seed=4)).to("cuda:0")
        Ya, Yb, Yc = (torch.empty_like(X) for _ in range(3))
        h0.matvec(X, Ya)
        h0.matvec(X, Yb)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            h1.matvec(X, Yc)
        s.synchronize()
        torch.cuda.synchronize()
        assert torch.equal(Ya, Yb)
        assert torch.equal(Ya, Yc)
        # the per-call stream of dh2_matvec_stream
        Yd = torch.empty_like(X)
        with torch.cuda.stream(s):
            h0.matvec_on(X, Yd, s.cuda_stream)
        s.synchronize()
        assert torch.equal(Ya, Yd)
    finally:
        h0.free()
        h1.free()
