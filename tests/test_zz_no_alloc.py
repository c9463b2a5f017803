"""The allocation-free product (dh2_matvec_noalloc: staging in the library's
static device scratch) against dh2_matvec on the same handles and inputs: two
calls in a row, the second on a smaller problem and fewer right-hand sides
(the scratch keeps the first call's contents), each bit for bit equal to the
handle's own product; an FP32 handle; and the rejection of a handle whose
staging exceeds the scratch."""
import numpy as np
import pytest

import synth
from tests.gpu_common import say, oracle_for, rel

pytestmark = pytest.mark.gpu


def _pair(h, X, dtype):
    import torch
    Xd = torch.from_numpy(np.ascontiguousarray(X.astype(dtype))).to("cuda:0")
    Ya, Yb = torch.empty_like(Xd), torch.empty_like(Xd)
    Yb.fill_(float("nan"))
    h.matvec(Xd, Ya)
    torch.cuda.synchronize()
    say("[gpu] dh2_matvec_noalloc n=%d nrhs=%d" % (X.shape[1], X.shape[0]))
    h.matvec_noalloc(Xd, Yb)
    torch.cuda.synchronize()
    return Ya.cpu().numpy(), Yb.cpu().numpy()


def test_noalloc_equals_matvec_on_consecutive_calls():
    from paper_1809_04384_amd import dh2
    handles = []
    try:
        for name, nrhs, prec in (("dir2k", 5, dh2.FP64), ("dir512", 2, dh2.FP64), ("sphere2k", 3, dh2.FP32)):
            w = synth.WORKLOADS[name]
            V, T = synth.make_mesh(w)
            say("[gpu] dh2_build %s precision %d" % (name, prec))
            h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, precision=prec,
                           max_nrhs=8)
            handles.append(h)
            X = synth.complex_gaussian(len(T), nrhs, seed=40 + nrhs)
            Ya, Yb = _pair(h, X, np.complex128 if prec == dh2.FP64 else np.complex64)
            assert np.array_equal(Ya, Yb), name
            if prec == dh2.FP64:
                err = rel(Yb, oracle_for(name).matvec(X.T).T)
                say("[gpu] %s allocation-free product vs oracle %.3e" % (name, err))
                assert err <= 1e-10
        # the first handle again, after the others used the scratch
        w = synth.WORKLOADS["dir2k"]
        X = synth.complex_gaussian(w.n, 1, seed=77)
        Ya, Yb = _pair(handles[0], X, np.complex128)
        assert np.array_equal(Ya, Yb)
    finally:
        for h in handles:
            h.free()


def test_noalloc_rejects_staging_beyond_scratch():
    import torch
    from paper_1809_04384_amd import dh2
    w = synth.WORKLOADS["dir512"]
    V, T = synth.make_mesh(w)
    # staging for 4096 right-hand sides: 3 n 4096 complex128 = 100 MB > 64 MiB
    h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, max_nrhs=4096)
    try:
        Xd = torch.zeros((1, len(T)), dtype=torch.complex128, device="cuda:0")
        Yd = torch.empty_like(Xd)
        with pytest.raises(dh2.Dh2Error) as e:
            h.matvec_noalloc(Xd, Yd)
        assert e.value.status == 1 and "static scratch" in str(e.value)
    finally:
        h.free()
