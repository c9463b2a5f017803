"""Algebraic and accuracy pins of the oracle's DH^2 construction
(Sections 2, 3.1, 3.2) on tiny inputs."""
import math

import numpy as np
import pytest

import synth
from oracle.dh2 import OracleDH2, spectral_norm_power
from oracle.general import general_row_svd

H = lambda a: a.conj().T
CASES = ["dir512", "sphere2k", "cube768", "cube1200dir"]
_cache = {}


def build(name, **over):
    key = (name, tuple(sorted(over.items())))
    if key not in _cache:
        w = synth.WORKLOADS[name]
        V, T = synth.make_mesh(w)
        p = dict(kappa=w.kappa, order=w.order, eta=w.eta, leaf=w.leaf, tol=w.tol, eta1=w.eta1)
        p.update(over)
        _cache[key] = OracleDH2(V, T, p["kappa"], p["order"], p["eta"], p["leaf"], p["tol"],
                                eta1=p["eta1"], norm=p.get("norm", "fro"))
    return _cache[key]


@pytest.fixture(scope="module", params=CASES)
def o(request):
    return build(request.param)


def test_fast_matvec_equals_plain_definition(o):
    X = synth.complex_gaussian(o.n, 3, seed=5).T
    Y = o.matvec(X)
    ref = o.matvec_expanded(X)
    assert np.linalg.norm(Y - ref) <= 1e-13 * np.linalg.norm(ref)
    G = o.dense_compressed()
    assert np.linalg.norm(G @ X - Y) <= 1e-13 * np.linalg.norm(Y)


def test_basis_weights_reproduce_gram(o):
    """R_tc^* R_tc = V_tc^* V_tc (eq. (basis_weights_def), P isometric)."""
    for (t, c) in list(o.basis_active)[:400]:
        Vx = o.expanded_basis(t, c, o.Vleaf, o.E)
        Gm = H(Vx) @ Vx
        R = o.R[(t, c)]
        assert np.linalg.norm(H(R) @ R - Gm) <= 1e-13 * np.linalg.norm(Gm)


def test_block_weights_are_block_norms(o):
    for b in range(0, len(o.st.adm), max(1, len(o.st.adm) // 50)):
        t, s, c = o.st.adm[b]
        blk = o.expanded_basis(t, c, o.Vleaf, o.E) @ o.coupling(b) @ H(o.expanded_basis(s, c, o.Vleaf, o.E))
        assert abs(np.linalg.norm(blk) - o.omega[b]) <= 1e-12 * o.omega[b]


def test_fast_recompression_matches_general_algorithm(o):
    """Singular values and ranks of the fast algorithm (Section 3.2) equal those
    of the dense algorithm of Section 3.1 applied to the expanded G_int."""
    _fast_vs_general(o)


def _fast_vs_general(o):
    if not o.st.adm:
        pytest.skip("no admissible blocks")
    Gi = o.dense_interp()
    for adjoint, sig_fast, rank_fast in ((False, o.sig, o.rank), (True, o.sigW, o.rankW)):
        sig, rank, _ = general_row_svd(o, Gi, adjoint=adjoint)
        assert set(sig) == set(sig_fast)
        for key in sig:
            a, b = sig[key], sig_fast[key]
            m = min(len(a), len(b))
            scale = max(a[0] if len(a) else 0.0, 1e-300)
            assert np.all(np.abs(a[:m] - b[:m]) <= 1e-12 * scale + 1e-15)
            assert np.all(a[m:] <= 1e-12 * scale) and np.all(b[m:] <= 1e-12 * scale)
            assert rank[key] == rank_fast[key]


def test_total_weights_reproduce_weighted_gram(o):
    """V_tc Zhat^* Zhat V_tc^* = G_tc G_tc^* (eq. (recomp_weight_full))."""
    if not o.st.adm:
        pytest.skip("no admissible blocks")
    from oracle.general import ancestors
    Gi = o.dense_interp()
    st = o.st
    for (t, c) in list(o.row_active)[:200]:
        cols = [Gi[np.ix_(st.idx(t), st.idx(st.adm[b][1]))] / o.omega[b]
                for (ta, ca) in ancestors(o, t, c) for b in o.brow.get((ta, ca), [])]
        Gtc = np.hstack(cols)
        Vx = o.expanded_basis(t, c, o.Vleaf, o.E)
        lhs = Vx @ H(o.Zrow[(t, c)]) @ o.Zrow[(t, c)] @ H(Vx)
        ref = Gtc @ H(Gtc)
        assert np.linalg.norm(lhs - ref) <= 1e-12 * np.linalg.norm(ref)


def test_new_bases_orthonormal_nested_and_basis_change(o):
    for Q, F, C, act in ((o.Q, o.F, o.C, o.row_active), (o.QW, o.FW, o.CW, o.col_active)):
        for (t, c) in list(act)[:300]:
            Qx = o.expanded_basis(t, c, Q, F)
            k = Qx.shape[1]
            assert np.linalg.norm(H(Qx) @ Qx - np.eye(k)) <= 1e-13 * max(k, 1)
            Vx = o.expanded_basis(t, c, o.Vleaf, o.E)
            assert np.linalg.norm(C[(t, c)] - H(Qx) @ Vx) <= 1e-12 * max(1.0, np.linalg.norm(Vx))


def test_recompression_error_within_tolerance(o):
    """|G_int - Gtilde|_2 <= tol |G_int|_2 (the paper's error notion of Section 5)."""
    Gi = o.dense_interp()
    Gt = o.dense_compressed()
    rel = np.linalg.norm(Gi - Gt, 2) / np.linalg.norm(Gi, 2)
    assert rel <= o.tol


SPECTRAL_CASES = ["dir512", "cube768"]


@pytest.mark.parametrize("name", SPECTRAL_CASES)
def test_spectral_block_weights_are_block_norms(name):
    """Spectral error control (Section 5): omega_b is the spectral norm of the
    interpolated block V_tc S_b V_sc^*, here from the expanded bases and a dense
    SVD (the oracle takes it from the basis weights, R_tc S_b R_sc^*)."""
    o = build(name, norm="spectral")
    for b in range(0, len(o.st.adm), max(1, len(o.st.adm) // 50)):
        t, s, c = o.st.adm[b]
        blk = o.expanded_basis(t, c, o.Vleaf, o.E) @ o.coupling(b) @ H(o.expanded_basis(s, c, o.Vleaf, o.E))
        ref = np.linalg.svd(blk, compute_uv=False)[0]
        assert abs(ref - o.omega[b]) <= 1e-12 * ref
        # the spectral norm lies between |.|_F / sqrt(rank) and |.|_F
        fro = np.linalg.norm(blk)
        assert o.omega[b] <= fro * (1 + 1e-14) and o.omega[b] >= fro / math.sqrt(min(blk.shape)) * (1 - 1e-14)


def test_rank_rules_by_enumeration():
    """Both rank rules against their definitions by enumerating k: the smallest
    k whose discarded singular values sigma_{k+1}, sigma_{k+2}, ... have a sum of
    squares within eps^2 (Frobenius) or are all within eps (spectral)."""
    rng = np.random.default_rng(7)
    for trial in range(300):
        m = int(rng.integers(0, 14))
        sig = np.sort(10.0 ** rng.uniform(-9, 0, size=m))[::-1]
        eps = 10.0 ** rng.uniform(-8, 0)
        fro = min(k for k in range(m + 1) if np.sum(sig[k:] ** 2) <= eps * eps)
        spec = min(k for k in range(m + 1) if np.all(sig[k:] <= eps))
        r = OracleDH2.__new__(OracleDH2)
        r.tol = eps
        r.norm = "fro"
        assert r.rank_rule(sig) == fro
        r.norm = "spectral"
        assert r.rank_rule(sig) == spec
        assert spec <= fro


@pytest.mark.parametrize("name", SPECTRAL_CASES)
def test_spectral_fast_recompression_matches_general_algorithm(name):
    """The fast algorithm of Section 3.2 against the dense one of Section 3.1,
    both under the spectral rank rule and spectral block weights."""
    _fast_vs_general(build(name, norm="spectral"))


@pytest.mark.parametrize("name", SPECTRAL_CASES)
def test_spectral_block_errors_within_tolerance(name):
    """Spectral control: per admissible block |G_int,b - Gtilde_b|_2 <= 2 eps
    omega_b (eps omega_b for the row and for the column truncation, whose
    weighted matrices hold G_int,b / omega_b), and the whole matrix within
    eps |G_int|_2."""
    o = build(name, norm="spectral")
    Gi = o.dense_interp()
    Gt = o.dense_compressed()
    st = o.st
    for b, (t, s, c) in enumerate(st.adm):
        blk = np.ix_(st.idx(t), st.idx(s))
        assert np.linalg.norm(Gi[blk] - Gt[blk], 2) <= 2 * o.tol * o.omega[b]
    assert np.linalg.norm(Gi - Gt, 2) <= o.tol * np.linalg.norm(Gi, 2)


def test_power_iteration_matches_dense_norm():
    o = build("dir512")
    Gi = o.dense_interp()
    Gt = o.dense_compressed()
    ref = np.linalg.norm(Gi - Gt, 2)
    est = spectral_norm_power(lambda x: o.matvec_interp(x) - o.matvec(x),
                              lambda x: o.matvec_interp(x, adjoint=True) - H(Gt) @ x,
                              o.n, iters=300, rtol=1e-10)
    assert abs(est - ref) <= 1e-3 * ref


def test_dense_galerkin_is_symmetric_and_matches_near_field(o):
    G = o.dense_galerkin()
    assert np.linalg.norm(G - G.T) <= 1e-14 * np.linalg.norm(G)
    # G_int is symmetric only up to the interpolation error (blocks (t,s) and
    # (s,t) use different directions); recompression adds at most 2 tol
    Gi = o.dense_interp()
    Gt = o.dense_compressed()
    asym = np.linalg.norm(Gi - Gi.T, 2)
    assert np.linalg.norm(Gt - Gt.T, 2) <= asym + 2 * o.tol * np.linalg.norm(Gi, 2) + 1e-14


def test_interpolation_error_decreases_with_order():
    """|G - G_int| falls with m, at zero and positive wave number (Section 2)."""
    for kappa in (0.0, 4.0):
        errs = []
        for m in (2, 3, 4, 5):
            w = synth.WORKLOADS["sphere2k"]
            o = build("sphere2k", kappa=kappa, order=m)
            G = o.dense_galerkin()
            Gi = o.dense_interp()
            errs.append(np.linalg.norm(G - Gi) / np.linalg.norm(G))
        assert all(errs[i + 1] < 0.5 * errs[i] for i in range(len(errs) - 1)), errs


def test_kappa_zero_is_real_h2():
    o = build("sphere2k", kappa=0.0)
    assert all(m == 0 for m in o.st.dir_m)
    X = synth.complex_gaussian(o.n, 2, seed=9).real.T.astype(np.complex128)
    Y = o.matvec(X)
    assert np.linalg.norm(Y.imag) <= 1e-14 * np.linalg.norm(Y.real)


def test_scaling_and_translation_invariance():
    w = synth.WORKLOADS["dir512"]
    V, T = synth.make_mesh(w)
    base = build("dir512")
    X = synth.complex_gaussian(base.n, 1, seed=2).T
    Y0 = base.matvec(X)
    # mesh x2, kappa / 2: every entry scales by 2^3 (Galerkin area^2 / distance)
    o2 = OracleDH2(2.0 * V, T, w.kappa / 2, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1)
    assert np.linalg.norm(o2.matvec(X) - 8.0 * Y0) <= 1e-12 * np.linalg.norm(Y0)
    # translation: the Galerkin matrix is invariant; the cluster tree may split
    # differently after rounding, so the compressed operators agree only up to
    # their approximation error
    o3 = OracleDH2(V + np.array([0.5, -0.25, 0.125]), T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1)
    G = base.dense_galerkin()
    G3 = o3.dense_galerkin()
    GX = G @ X
    err0 = np.linalg.norm(Y0 - GX)
    err3 = np.linalg.norm(o3.matvec(X) - G3 @ X)
    # same quadrature entries (near rule on a sample of pairs)
    from oracle import cquad
    rows = np.arange(0, base.n, 7)
    assert np.max(np.abs(cquad.near_block(o3.tri, rows, rows, w.kappa)
                         - cquad.near_block(base.tri, rows, rows, w.kappa))) <= 1e-12 * np.max(np.abs(G))
    assert err3 <= 3 * err0 and err0 <= 3 * err3


def test_planted_transfer_mistake_is_caught(monkeypatch):
    """A transfer matrix built with c instead of c - c' must break the basis-weight
    pin: the pins are sensitive to the nested-basis arithmetic."""
    from oracle import dh2 as mod
    orig = mod.OracleDH2.transfer

    def wrong(self, t1, c):
        E = orig(self, t1, c)
        t = self.st.parent[t1]
        c1 = self.sd(t, c)
        xi1 = self.points[t1]
        fix = np.exp(-1j * self.kappa * (xi1 @ (self.dir(t, c) - self.dir(t1, c1))))
        return E * fix[:, None] * np.exp(1j * self.kappa * (xi1 @ self.dir(t, c)))[:, None]

    monkeypatch.setattr(mod.OracleDH2, "transfer", wrong)
    w = synth.WORKLOADS["dir512"]
    V, T = synth.make_mesh(w)
    bad = OracleDH2(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1)
    good = build("dir512")
    X = synth.complex_gaussian(good.n, 1, seed=4).T
    G = good.dense_galerkin()
    err_good = np.linalg.norm(good.matvec(X) - G @ X) / np.linalg.norm(G @ X)
    err_bad = np.linalg.norm(bad.matvec(X) - G @ X) / np.linalg.norm(G @ X)
    assert err_bad > 100 * err_good
