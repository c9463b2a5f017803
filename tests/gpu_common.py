"""Shared helpers of the GPU tests: oracle builds (cached per process) and
slot mapping between the library and the oracle."""
import sys

import numpy as np

import synth
from oracle.dh2 import OracleDH2

_oracles = {}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_for(name, norm="fro"):
    key = (name, norm)
    if key not in _oracles:
        w = synth.WORKLOADS[name]
        V, T = synth.make_mesh(w)
        _oracles[key] = OracleDH2(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, norm=norm)
    return _oracles[key]


def build_handle(name, **kw):
    from paper_1809_04384_amd import dh2
    w = synth.WORKLOADS[name]
    V, T = synth.make_mesh(w)
    say("[gpu] dh2_build workload=%s n=%d kappa=%g m=%d leaf=%d eta=%g eta1=%g tol=%g"
        % (name, len(T), w.kappa, w.order, w.leaf, w.eta, w.eta1, w.tol))
    h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, **kw)
    slots = dh2.Plan(V, T, w.kappa, w.order, w.eta, w.leaf, w.eta1).export()["slots"]
    return h, slots


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


H = lambda a: a.conj().T


def check_ranks_and_sigma(h, slots, o, label, gram_eps=None, spectral=False):
    """Ranks and singular values of both truncation passes against the oracle:
    singular values to 1e-12 of the largest, ranks equal except at a near-tie
    of the rank rule (a tail sum within 1e-8 of eps^2).

    gram_eps: the Gram form of the total weights, whose factor R has
    |R^H R - Z^H Z| <= gram_eps |Z|^2.  The squares of the singular values
    then move by at most gram_eps s_1^2 (Weyl), so each singular value by at
    most min(sqrt(gram_eps) s_1, gram_eps s_1^2 / s_i), and the rank rule's
    tail sums by at most m gram_eps s_1^2: a rank may differ only where a tail
    is that close to eps^2.

    spectral: the spectral rule (rank = number of singular values above
    eps), where a rank may differ only where a singular value is within its
    bound of eps."""
    worst = 0.0
    for kind, ranks_o, sig_o in (("row", o.rank, o.sig), ("col", o.rankW, o.sigW)):
        ranks = h.inspect("rank_" + kind)[:, 0].real.astype(int)
        mism = 0
        for q, (t, c, flags) in enumerate(slots.tolist()):
            key = (t, c)
            if key not in ranks_o:
                assert ranks[q] == -1
                continue
            s_o = sig_o[key]
            s_g = h.inspect("sigma_" + kind, q)[:, 0].real
            m = min(len(s_o), len(s_g))
            if m:
                d = np.abs(s_o[:m] - s_g[:m])
                if gram_eps is None:
                    bound = 1e-12 * s_o[0] + 1e-300
                else:
                    s1 = s_o[0]
                    bound = np.minimum(np.sqrt(gram_eps) * s1,
                                       gram_eps * s1 * s1 / np.maximum(s_o[:m], 1e-300)) + 1e-13 * s1 + 1e-300
                    worst = max(worst, float(np.max(d / bound)))
                assert np.all(d <= bound), (label, kind, key, float(np.max(d)))
            if ranks[q] != ranks_o[key] and spectral:
                s1 = s_o[0]
                b = 1e-8 * o.tol if gram_eps is None else (
                    np.minimum(np.sqrt(gram_eps) * s1, gram_eps * s1 * s1 / np.maximum(s_o, 1e-300)) + 1e-8 * o.tol)
                near = np.any(np.abs(s_o - o.tol) <= b)
                assert near, (label, kind, key, ranks[q], ranks_o[key])
                mism += 1
            elif ranks[q] != ranks_o[key]:
                tail = np.cumsum((s_o ** 2)[::-1])[::-1]
                eps2 = o.tol ** 2
                if gram_eps is None:
                    near = np.any(np.abs(tail - eps2) <= 1e-8 * eps2)
                else:
                    j = min(ranks[q], ranks_o[key])
                    tj = tail[j] if j < len(tail) else 0.0
                    near = abs(tj - eps2) <= len(s_o) * gram_eps * s_o[0] ** 2 + 1e-8 * eps2
                assert near, (label, kind, key, ranks[q], ranks_o[key])
                mism += 1
        say("[gpu] %s %s ranks: %d near-tie mismatches" % (label, kind, mism))
    if gram_eps is not None:
        say("[gpu] %s singular values: largest deviation / bound %.3e" % (label, worst))


def check_weight_invariants(h, slots, o, label, tol_total=1e-11):
    """R^* R and Zhat^* Zhat of every slot (unique although R and Zhat are
    defined up to a unitary factor) against the oracle; Zhat^* Zhat to
    tol_total relative (Frobenius)."""
    worst = 0.0
    for q, (t, c, flags) in enumerate(slots.tolist()):
        R = h.inspect("basis_weight", q)
        Ro = o.R[(t, c)]
        G, Go = H(R) @ R, H(Ro) @ Ro
        assert R.shape[0] <= o.k
        assert np.linalg.norm(G - Go) <= 1e-12 * np.linalg.norm(Go), (label, "R", q, t, c)
        for kind, Zo in (("row", o.Zrow), ("col", o.Zcol)):
            if (t, c) not in Zo:
                continue
            Z = h.inspect("total_weight_" + kind, q)
            Go = H(Zo[(t, c)]) @ Zo[(t, c)]
            if o.st.is_leaf(t) and o.st.size[t] < o.k:
                # projected total weight of a leaf: Gram V Zhat^H Zhat V^H
                Vo = o.Vleaf[(t, c)]
                Go = Vo @ Go @ H(Vo)
            G = H(Z) @ Z
            assert Z.shape[0] <= o.k, (label, kind, q)
            assert G.shape == Go.shape, (label, kind, q, G.shape, Go.shape)
            e = np.linalg.norm(G - Go) / max(np.linalg.norm(Go), 1e-300)
            worst = max(worst, e)
            assert e <= tol_total, (label, kind, q, t, c, e)
    say("[gpu] %s total weights: largest relative Gram deviation %.3e" % (label, worst))


def fp32_rank_shift(sig, r_a, r_b, eps, m=None):
    """Smallest perturbation Delta (absolute, in the units of sig) of every
    singular value that moves the Frobenius rank rule from r_a to r_b or back.
    With T_j = sum_{i >= j} sigma_i^2 (0-based) and j = min(r_a, r_b), Weyl's
    bound |sigma_i' - sigma_i| <= Delta changes T_j by at most
    2 Delta sqrt(m) sqrt(T_j) + m Delta^2, so a rank change needs
    |T_j - eps^2| <= that; the root of the quadratic is returned."""
    sig = np.asarray(sig, dtype=np.float64)
    m = len(sig) if m is None else m
    j = min(r_a, r_b)
    T = float(np.sum(sig[j:] ** 2))
    s = np.sqrt(max(T, eps * eps))
    return (-s + np.sqrt(s * s + abs(T - eps * eps))) / np.sqrt(max(m, 1))
