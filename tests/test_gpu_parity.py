"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  FP64 form: matvec within 1e-10 relative; deterministic
intermediates (near field, leaf bases, transfers, block weights) element by
element; ranks equal up to flagged near-ties; singular values to 1e-12."""
import numpy as np
import pytest

import synth
from tests.gpu_common import (say, oracle_for, build_handle, rel, check_ranks_and_sigma,
                               check_weight_invariants, fp32_rank_shift)

pytestmark = pytest.mark.gpu

CASES = ["dir512", "cube768", "sphere2k", "cube1200dir", "dir2k"]
_handles = {}


def handle(name):
    if name not in _handles:
        _handles[name] = build_handle(name)
    return _handles[name]


@pytest.fixture(scope="module", autouse=True)
def _cleanup():
    yield
    for h, _ in _handles.values():
        h.free()
    _handles.clear()


def _matvec(h, X):
    import torch
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0")
    Yd = torch.empty_like(Xd)
    say("[gpu] dh2_matvec n=%d nrhs=%d" % (X.shape[1], X.shape[0]))
    h.matvec(Xd, Yd)
    torch.cuda.synchronize()
    return Yd.cpu().numpy()


@pytest.mark.parametrize("name", CASES)
def test_matvec_fp64_matches_oracle(name):
    o = oracle_for(name)
    h, _ = handle(name)
    X = synth.complex_gaussian(o.n, 3, seed=0)            # (nrhs, n)
    Y = _matvec(h, X)
    Yo = o.matvec(X.T).T
    err = rel(Y, Yo)
    say("[gpu] %s matvec rel err %.3e" % (name, err))
    assert err <= 1e-10


@pytest.mark.parametrize("name", ["sphere2k", "dir2k"])
def test_matvec_rhs_counts(name):
    """Right-hand-side counts below, at and above one 16-wide matrix-core tile
    (1 and 2: one ragged tile; 16: one full tile; 20: one full tile plus a
    ragged one); each column must match the oracle."""
    from paper_1809_04384_amd import dh2
    o = oracle_for(name)
    w = synth.WORKLOADS[name]
    V, T = synth.make_mesh(w)
    h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, max_nrhs=20)
    try:
        for nrhs in (1, 2, 5, 16, 20):
            X = synth.complex_gaussian(o.n, nrhs, seed=nrhs)
            Y = _matvec(h, X)
            Yo = o.matvec(X.T).T
            for r in range(nrhs):
                err = rel(Y[r], Yo[r])
                assert err <= 1e-10, (nrhs, r, err)
            say("[gpu] %s nrhs=%d max column rel err ok" % (name, nrhs))
    finally:
        h.free()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_pipeline_shapes_and_autotune(precision):
    """Every pipeline shape of the block-row products (forced through the
    autotune hook) gives the product of the default shape bit for bit, for one
    ragged and one two-tile right-hand-side count; an autotuned handle records the shapes
    it picked, each a valid one, and its product matches the oracle."""
    import torch
    from paper_1809_04384_amd import dh2
    name = "dir2k"
    o = oracle_for(name)
    w = synth.WORKLOADS[name]
    V, T = synth.make_mesh(w)
    prec = dh2.FP64 if precision == "fp64" else dh2.FP32
    ctype = torch.complex128 if precision == "fp64" else torch.complex64
    # against the oracle: the bounds of the FP64 and FP32 forms
    tol = 1e-10 if precision == "fp64" else 1e-4
    first = {}
    ref = {}
    for nrhs in (1, 20):
        X = synth.complex_gaussian(o.n, nrhs, seed=40 + nrhs)
        Yo = o.matvec(X.T).T
        ref[nrhs] = (X, Yo)
    for mode in [2 + v for v in range(4)] + [1]:
        h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, precision=prec,
                       max_nrhs=20, autotune=mode)
        try:
            st = h.stats()
            say("[gpu] %s %s autotune=%d shapes %s (%.1f ms)" % (name, precision, mode, st["mv_variant"],
                                                                 st["ms_autotune"]))
            if mode >= 2:
                assert st["mv_variant"] == [mode - 2] * 4
                assert st["ms_autotune"] == 0
            else:
                assert all(0 <= v < 4 for v in st["mv_variant"])
                assert st["ms_autotune"] > 0
            for nrhs, (X, Yo) in ref.items():
                Xd = torch.from_numpy(np.ascontiguousarray(X)).to("cuda:0").to(ctype)
                Yd = torch.empty_like(Xd)
                h.matvec(Xd, Yd)
                torch.cuda.synchronize()
                Y = Yd.cpu().numpy().astype(np.complex128)
                for r in range(nrhs):
                    err = rel(Y[r], Yo[r])
                    assert err <= tol, (mode, nrhs, r, err)
                if nrhs in first:
                    # the shapes change the pipelining, not the order of the
                    # accumulation: the same bits (builds are deterministic)
                    assert np.array_equal(Y, first[nrhs]), (mode, nrhs, rel(Y, first[nrhs]))
                else:
                    first[nrhs] = Y
        finally:
            h.free()


@pytest.mark.parametrize("name", CASES)
def test_near_field_elementwise(name):
    o = oracle_for(name)
    h, _ = handle(name)
    nb = len(o.st.near)
    for b in list(range(0, nb, max(1, nb // 40))) + [nb - 1]:
        N = h.inspect("near", b)
        ref = o.N[b]
        assert N.shape == ref.shape
        assert np.max(np.abs(N - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("name", CASES)
def test_bases_transfers_weights_elementwise(name):
    o = oracle_for(name)
    h, slots = handle(name)
    st = o.st
    for q, (t, c, flags) in enumerate(slots.tolist()):
        assert (t, c) in o.basis_active
        if st.is_leaf(t):
            V = h.inspect("leaf_basis", q)
            ref = o.Vleaf[(t, c)]
            assert np.max(np.abs(V - ref)) <= 1e-13 * max(np.max(np.abs(ref)), 1e-300)
        elif q % 7 == 0:
            for i, t1 in enumerate(st.children[t]):
                E = h.inspect("transfer", 2 * q + i)
                ref = o.E[(t1, c)]
                assert np.max(np.abs(E - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert {(int(t), int(c)) for t, c, f in slots.tolist() if f & 1} == o.row_active
    assert {(int(t), int(c)) for t, c, f in slots.tolist() if f & 2} == o.col_active
    om = h.inspect("omega")[:, 0].real
    if len(om):
        assert np.max(np.abs(om - o.omega) / o.omega) <= 1e-11


@pytest.mark.parametrize("name", CASES)
def test_ranks_and_singular_values(name):
    o = oracle_for(name)
    h, slots = handle(name)
    check_ranks_and_sigma(h, slots, o, name)


@pytest.mark.parametrize("name", CASES)
def test_couplings_and_weight_invariants(name):
    """S_b element by element; R^* R and Zhat^* Zhat (unique although R and Zhat
    are defined up to a unitary factor) against the oracle."""
    o = oracle_for(name)
    h, slots = handle(name)
    nb = len(o.st.adm)
    for b in list(range(0, nb, max(1, nb // 30))):
        S = h.inspect("coupling", b)
        ref = o.coupling(b)
        assert np.max(np.abs(S - ref)) <= 1e-13 * np.max(np.abs(ref))
    check_weight_invariants(h, slots, o, name)


FP32_CASES = ["dir512", "sphere2k", "cube1200dir", "dir2k", "dir2k_t4"]


@pytest.mark.parametrize("name", FP32_CASES)
def test_fp32_form_matches_fp64(name):
    """FP32 form: near field evaluated in FP32, the recompression's matrix
    products on the FP32 matrix cores (QR and SVD in FP64), couplings and
    bases rounded to complex64, matvec in FP32.  Every right-hand-side count (1, 2, 5, 20, 37) must agree with the
    FP64 oracle to 1e-4 relative, the near field entry by entry to 1e-5 of its
    largest entry."""
    import torch
    from paper_1809_04384_amd import dh2
    o = oracle_for(name)
    w = synth.WORKLOADS[name]
    V, T = synth.make_mesh(w)
    say("[gpu] dh2_build FP32 workload=%s n=%d" % (name, len(T)))
    h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, precision=dh2.FP32, max_nrhs=40)
    h64, h64_slots = handle(name)
    try:
        # the recompression products run in FP32: a rank may move only where
        # the FP64 singular values put the rank rule within an FP32-sized
        # perturbation of its threshold (fp32_rank_shift: the smallest uniform
        # change of the singular values that moves the rank, bounded by 1e-5
        # of the largest, about 170 units of FP32 rounding), and only in a few
        # slots
        plan_slots = h64_slots
        for kind, sig_o in (("row", o.sig), ("col", o.sigW)):
            r32 = h.inspect("rank_" + kind)[:, 0].real.astype(int)
            r64 = h64.inspect("rank_" + kind)[:, 0].real.astype(int)
            diff = np.nonzero(r32 != r64)[0]
            worst = 0.0
            for q in diff.tolist():
                t, c, _ = plan_slots[q].tolist()
                s_o = sig_o[(t, c)]
                shift = fp32_rank_shift(s_o, r32[q], r64[q], o.tol) / max(s_o[0], 1e-300)
                worst = max(worst, shift)
                assert shift <= 1e-5, (name, kind, q, r32[q], r64[q], shift)
            say("[gpu] %s FP32 %s ranks differing from FP64: %d of %d, largest needed shift %.2e"
                % (name, kind, len(diff), r32.size, worst))
            assert len(diff) <= max(3, r32.size // 50)
        nb = len(o.st.near)
        for b in list(range(0, nb, max(1, nb // 20))) + [nb - 1]:
            N = h.inspect("near", b)
            ref = o.N[b]
            assert np.max(np.abs(N - ref)) <= 1e-5 * np.max(np.abs(ref))
        # 20 and 37: FP32 passes of two 16-wide chunks (37 = one full pass and a
        # ragged one)
        for nrhs in (1, 2, 5, 20, 37):
            X = synth.complex_gaussian(o.n, nrhs, seed=10 + nrhs)
            Xd = torch.from_numpy(X.astype(np.complex64)).to("cuda:0")
            Yd = torch.empty_like(Xd)
            say("[gpu] FP32 dh2_matvec %s nrhs=%d" % (name, nrhs))
            h.matvec(Xd, Yd)
            torch.cuda.synchronize()
            Y = Yd.cpu().numpy().astype(np.complex128)
            Yo = o.matvec(X.T).T
            err = rel(Y, Yo)
            say("[gpu] %s FP32 nrhs=%d rel err vs oracle %.3e" % (name, nrhs, err))
            assert err <= 1e-4
    finally:
        h.free()


@pytest.mark.parametrize("name", FP32_CASES)
def test_bf16x3_form_matches_fp64(name):
    """Split-BF16x3 form: the FP32 form with the recompression's matrix
    products on the BF16 matrix cores (three bf16 part products per real
    product, FP32 accumulation; QR and SVD in FP64).  Every right-hand-side
    path must agree with the FP64 oracle to 1e-4 relative (the products carry
    about 2^-16 relative error, below the tolerance of the FP32 form)."""
    import torch
    from paper_1809_04384_amd import dh2
    o = oracle_for(name)
    w = synth.WORKLOADS[name]
    V, T = synth.make_mesh(w)
    say("[gpu] dh2_build BF16x3 workload=%s n=%d" % (name, len(T)))
    h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, precision=dh2.BF16X3)
    try:
        for nrhs in (1, 2, 5):
            X = synth.complex_gaussian(o.n, nrhs, seed=20 + nrhs)
            Xd = torch.from_numpy(X.astype(np.complex64)).to("cuda:0")
            Yd = torch.empty_like(Xd)
            say("[gpu] BF16x3 dh2_matvec %s nrhs=%d" % (name, nrhs))
            h.matvec(Xd, Yd)
            torch.cuda.synchronize()
            Y = Yd.cpu().numpy().astype(np.complex128)
            err = rel(Y, o.matvec(X.T).T)
            say("[gpu] %s BF16x3 nrhs=%d rel err vs oracle %.3e" % (name, nrhs, err))
            assert err <= 1e-4
    finally:
        h.free()


SPECTRAL_CASES = ["dir512", "sphere2k", "cube1200dir", "dir2k"]


@pytest.mark.parametrize("name", SPECTRAL_CASES)
def test_spectral_control_matches_oracle(name):
    """Spectral error control (options.norm = spectral): block weights
    |R_tc S_b R_sc^*|_2 element by element, ranks and singular values, and the
    matvec against the oracle built with the same rule."""
    from paper_1809_04384_amd import dh2
    o = oracle_for(name, norm="spectral")
    h, slots = build_handle(name, norm=dh2.NORM_SPECTRAL)
    try:
        om = h.inspect("omega")[:, 0].real
        assert om.shape == o.omega.shape
        if len(om):
            err = np.max(np.abs(om - o.omega) / o.omega)
            say("[gpu] %s spectral block weights: max rel err %.3e" % (name, err))
            assert err <= 1e-12
        for kind, ranks_o, sig_o in (("row", o.rank, o.sig), ("col", o.rankW, o.sigW)):
            ranks = h.inspect("rank_" + kind)[:, 0].real.astype(int)
            for q, (t, c, flags) in enumerate(slots.tolist()):
                key = (t, c)
                if key not in ranks_o:
                    continue
                s_o = sig_o[key]
                s_g = h.inspect("sigma_" + kind, q)[:, 0].real
                m = min(len(s_o), len(s_g))
                if m:
                    assert np.max(np.abs(s_o[:m] - s_g[:m])) <= 1e-12 * s_o[0] + 1e-300
                if ranks[q] != ranks_o[key]:
                    # only a singular value at the threshold may change a rank
                    assert np.any(np.abs(s_o - o.tol) <= 1e-8 * o.tol), (kind, key, ranks[q], ranks_o[key])
        X = synth.complex_gaussian(o.n, 3, seed=0)
        Y = _matvec(h, X)
        err = rel(Y, o.matvec(X.T).T)
        say("[gpu] %s spectral control matvec rel err %.3e" % (name, err))
        assert err <= 1e-10
    finally:
        h.free()
