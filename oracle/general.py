"""Compression of a general (dense) matrix, Section 3.1 -- pin only.

Used on tiny inputs to check the fast recompression of Section 3.2: for every
(t,c) it forms G_tc = G restricted to t-hat x R_tc (the column clusters of
row(t~,c~) for all (t~,c~) in anc(t,c), eq. (ancestors)), each block scaled by
1/omega_b, and computes the singular values of G_tc (leaves) or of
Ghat_tc = [Q_{t1c1}^* G_tc|t1; Q_{t2c2}^* G_tc|t2] (eq. (Ghat)), with Q from
this same algorithm.  The paper states that the fast algorithm yields the same
left singular vectors and non-zero singular values (eq. (recomp_weight_full)).
"""
import numpy as np


def ancestors(o, t, c, _memo=None):
    """anc(t,c) of eq. (ancestors): (t,c) and, recursively, anc(t+,c+) for all
    directions c+ of the parent with sd(c+) = c."""
    st = o.st
    if not hasattr(o, "_sd_inverse"):
        inv = []
        for l in range(st.depth):
            d = {}
            for cp, cc in enumerate(st.sd[l]):
                d.setdefault(int(cc), []).append(cp)
            inv.append(d)
        o._sd_inverse = inv
        o._anc_memo = {}
    key = (t, c)
    if key in o._anc_memo:
        return o._anc_memo[key]
    out = [(t, c)]
    tp = st.parent[t]
    if tp >= 0:
        for cp in o._sd_inverse[st.level[tp]].get(c, []):
            out.extend(ancestors(o, tp, cp))
    o._anc_memo[key] = out
    return out


def general_row_svd(o, G, adjoint=False):
    """Singular values and ranks per active (t,c) from the dense algorithm.

    G is the dense matrix in the caller's index order (the expanded G_int).
    adjoint=True runs the same algorithm on G^* (column bases)."""
    st = o.st
    lists = o.bcol if adjoint else o.brow
    active = o.col_active if adjoint else o.row_active
    A = G.conj().T if adjoint else G
    Q, sig, rank = {}, {}, {}
    for (t, c) in o._by_level(active, descending=True):
        cols = []
        for (ta, ca) in ancestors(o, t, c):
            for b in lists.get((ta, ca), []):
                tb, sb, _ = st.adm[b]
                other = tb if adjoint else sb
                if o.omega[b] == 0.0:
                    continue
                blk = A[np.ix_(st.idx(t), st.idx(other))] / o.omega[b]
                cols.append(blk)
        Gtc = np.hstack(cols) if cols else np.zeros((st.size[t], 0), dtype=np.complex128)
        if st.is_leaf(t):
            M = Gtc
        else:
            c1 = o.sd(t, c)
            parts = []
            off = 0
            for t1 in st.children[t]:
                n1 = st.size[t1]
                parts.append(Q[(t1, c1)].conj().T @ Gtc[off:off + n1])
                off += n1
            M = np.vstack(parts)
        if M.shape[0] == 0 or M.shape[1] == 0:
            U = np.zeros((M.shape[0], 0), dtype=np.complex128)
            s = np.zeros(0)
        else:
            U, s, _ = np.linalg.svd(M, full_matrices=False)
        kk = o.rank_rule(s)
        sig[(t, c)] = s
        rank[(t, c)] = kk
        if st.is_leaf(t):
            Q[(t, c)] = U[:, :kk]
        else:
            c1 = o.sd(t, c)
            parts = []
            off = 0
            for t1 in st.children[t]:
                parts.append(Q[(t1, c1)] @ U[off:off + Q[(t1, c1)].shape[1], :kk])
                off += Q[(t1, c1)].shape[1]
            Q[(t, c)] = np.vstack(parts)
    return sig, rank, Q
