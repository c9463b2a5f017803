"""Benchmark: DH^2 build + compressed matvec on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sphere131k]

One step = the whole hot path over one problem: dh2_build (structure, near
field, interpolation, recompression) followed by the matvec on the workload's
right-hand sides.  The printed JSON line reports:
  value        matvec throughput in GB/s (algorithmic bytes: every stored matrix
               entry read once plus the vectors) with X, Y resident in HBM
  build_s      wall time of dh2_build (median over the timed steps)
  roofline     the near-field matvec kernel (the dominant HBM stream) against
               the MI355X HBM peak, timed with HIP events on its stream
  cpu_baseline the FP64 oracle on a bounded sample of the same workload
               (near-field rows of a few leaf clusters), on the host cores
"""
import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "DH² build s + matvec GB/s, n=131k κ=32 at rel.err 1e-4, FP32 vs FP64"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere131k")
    ap.add_argument("--matvec-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-leaves", type=int, default=3)
    ap.add_argument("--cpu-build-workloads", default="sphere2k,dir2k",
                    help="workloads whose whole oracle build is timed beside the GPU build ('' = none)")
    ap.add_argument("--err-sample-leaves", type=int, default=4,
                    help="leaf row clusters of the error check against the interpolated matrix (0 = skip)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32 form")
    ap.add_argument("--no-spectral", action="store_true", help="skip the spectral-control build")
    ap.add_argument("--no-paper-config", action="store_true",
                    help="skip the build at the paper's own n = 131072 setting (kappa 64, m 4, leaf 32, "
                         "spectral control)")
    ap.add_argument("--no-bf16x3", action="store_true", help="skip the split-BF16x3 form")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-rank form")
    ap.add_argument("--no-paper-quadrature", action="store_true",
                    help="skip the build with the paper's quadrature (Sauter-Erichsen-Schwab / Duffy-Gauss)")
    ap.add_argument("--learned-cube", default="cube28k_m6",
                    help="cube workload of the learned-rank family (cube7k_m6, cube28k_m6, cube110k_m6)")
    ap.add_argument("--weights", default="gram", choices=["gram", "householder"],
                    help="factorisation of the total weights in the timed build (gram: Gram matrix on the "
                         "FP64 matrix cores and pivoted Cholesky; householder: skinny QR)")
    ap.add_argument("--no-householder-build", action="store_true",
                    help="skip the comparison build with Householder total weights")
    ap.add_argument("--autotune", type=int, default=0, choices=[0, 1],
                    help="timed FP64 steps: time the block-row pipeline shapes at build and keep the "
                         "fastest (1) or use the default shape (0; at n = 131072 the tuner keeps it, "
                         "after 0.23 s of timing).  The batching form always autotunes.")
    ap.add_argument("--batch", type=int, default=64, metavar="COUNT",
                    help="problems of the batching form (the recipe's 64; 0 = skip)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain streaming kernel (read MIB MiB, write MIB MiB) and exit; "
                         "its HBM counters calibrate the traffic of the profiled kernels")
    return ap.parse_args()


PMC_FILE = os.path.join(ROOT, "profiles", "k_mv_rows_mfma_near_sphere131k_pmc.txt")
MATVEC_SRCS = [os.path.join(ROOT, "paper_1809_04384_amd", "csrc", f) for f in ("matvec.hip", "api.cpp")]


def source_sha256():
    """Hash of the matvec kernels (matvec.hip) and of the parts of api.cpp that
    build their row lists and issue their launches (the text between the
    "matvec schedule (begin)" and "(end)" markers)."""
    import hashlib
    h = hashlib.sha256()
    h.update(open(MATVEC_SRCS[0], "rb").read())
    keep = False
    for line in open(MATVEC_SRCS[1], "rb"):
        if b"matvec schedule (begin)" in line:
            keep = True
        if keep:
            h.update(line)
        if b"matvec schedule (end)" in line:
            keep = False
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of the near-field kernel from the stored rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE per dispatch, scaled by the
    streaming-kernel calibration), or None when the summary is missing, was
    taken on another pipeline shape than `kernel`, or the kernel source
    changed since the counters were taken."""
    if not os.path.exists(PMC_FILE):
        return None
    kv = {}
    for line in open(PMC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    sha = source_sha256()
    if kv.get("source_sha256") != sha or kv.get("kernel") != kernel:
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_peaks(torch):
    """Achievable rates on this GPU for context: HBM read bandwidth of a plain
    streaming reduction (torch sum over 16 GiB) and the FP64 matrix-core rate of
    a large library GEMM (torch.matmul, 8192^3)."""
    x = torch.ones(2 * 1024 ** 3, dtype=torch.float64, device="cuda:0")
    a = torch.randn(8192, 8192, dtype=torch.float64, device="cuda:0")
    out = {}
    for name, f, work in (("hbm_read_gbs", lambda: x.sum(), 16 * 2 ** 30 / 1e9),
                          ("fp64_gemm_tflops", lambda: a @ a, 2 * 8192 ** 3 / 1e12)):
        f()
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            f()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        out[name] = round(work / (statistics.median(ts) * 1e-3), 1)
    del x, a
    torch.cuda.empty_cache()
    return out


def copy_probe(mib):
    import torch
    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": a.numel() * 4, "copy_probe_bytes_written": b.numel() * 4}))


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(w, V, T, X, nleaves, pre=None):
    """Oracle near-field matvec on the rows of a few leaf clusters (seeded
    choice), timed on the host.  pre = (structure, triangle data, seconds) of
    an oracle already built for this workload.  Returns the baseline object."""
    from oracle.structure import build_structure
    from oracle.quadrature import triangle_data
    from oracle import cquad
    if pre is None:
        t0 = time.time()
        st = build_structure(V, T, w.kappa, w.eta, w.leaf, w.eta1)
        tri = triangle_data(V, T)
        t_struct = time.time() - t0
    else:
        st, tri, t_struct = pre
    leaves = [t for t in range(len(st.first)) if st.is_leaf(t)]
    rng = np.random.default_rng(2)
    pick = sorted(rng.choice(len(leaves), size=min(nleaves, len(leaves)), replace=False).tolist())
    chosen = [leaves[i] for i in pick]
    # near blocks covering the chosen rows: blocks (t', s) with t' an ancestor-or-self of t
    anc = {}
    for t in chosen:
        a = t
        while a >= 0:
            anc.setdefault(a, []).append(t)
            a = int(st.parent[a])
    t0 = time.time()
    blocks = []
    for (tb, sb) in st.near:
        for t in anc.get(tb, []):
            blocks.append((t, sb, cquad.near_block(tri, st.idx(t), st.idx(sb), w.kappa)))
    t_assemble = time.time() - t0
    Xc = X.T                                           # n x nrhs
    Y = {t: np.zeros((int(st.size[t]), Xc.shape[1]), dtype=np.complex128) for t in chosen}
    nbytes = sum(N.size for _, _, N in blocks) * 16 + 2 * 16 * Xc.shape[1] * sum(Y[t].shape[0] for t in chosen)
    reps = 0
    t0 = time.time()
    while True:
        for t, sb, N in blocks:
            Y[t] += N @ Xc[st.idx(sb)]
        reps += 1
        if time.time() - t0 > 3.0:
            break
    t_mv = (time.time() - t0) / reps
    threads = os.environ.get("OMP_NUM_THREADS")
    cores = int(threads) if threads else os.cpu_count()
    return {
        "value": nbytes / t_mv / 1e9, "unit": "GB/s", "cores": cores, "kind": "oracle",
        "sample": ("near-field matvec of %d leaf row clusters (%d rows, %d blocks, %.2f GB of entries) "
                   "of the same mesh and parameters, %d right-hand sides; oracle structure %.1f s, "
                   "assembly of the sampled near-field rows %.1f s (C, OpenMP)"
                   % (len(chosen), sum(Y[t].shape[0] for t in chosen), len(blocks),
                      sum(N.size for _, _, N in blocks) * 16 / 1e9, Xc.shape[1], t_struct, t_assemble)),
    }


def oracle_matvec_bytes(o, nrhs):
    """Algorithmic bytes of one compressed matvec of the oracle's result, by the
    library's formula: every stored entry (near field, recompressed couplings,
    leaf bases and transfers of both bases) read once, 16 bytes each, plus per
    right-hand side X and Y and the coefficient vectors read and written."""
    st = o.st
    near = sum(int(st.size[t]) * int(st.size[s]) for (t, s) in st.near)
    coup = sum(S.size for S in o.St)
    basis = sum(Q.size for Q in o.Q.values()) + sum(F.size for F in o.F.values())
    basis += sum(Q.size for Q in o.QW.values()) + sum(F.size for F in o.FW.values())
    coef = sum(o.rank.values()) + sum(o.rankW.values())
    return 16.0 * (near + coup + basis) + nrhs * 16.0 * (2.0 * o.n + 2.0 * coef)


def cpu_build_baseline(names, dh2, torch):
    """The FP64 oracle's whole build and one matvec on small workloads, per
    phase, on the host cores, beside the FP64 GPU build of the same problem."""
    from oracle.dh2 import OracleDH2
    out = {}
    for name in names:
        w = synth.WORKLOADS[name]
        V, T = synth.make_mesh(w)
        t0 = time.perf_counter()
        o = OracleDH2(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1)
        tb = time.perf_counter() - t0
        X = synth.complex_gaussian(len(T), 1, seed=0)
        t0 = time.perf_counter()
        o.matvec(X.T)
        tm = time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, max_nrhs=1, weights=WEIGHTS)
        torch.cuda.synchronize()
        tg = time.perf_counter() - t0
        h.free()
        out[name] = {
            "workload": "%s: %s n=%d, kappa=%g, m=%d, leaf %d, eta=%g, eta1=%g, tol=%g, FP64"
                        % (name, w.surface, len(T), w.kappa, w.order, w.leaf, w.eta, w.eta1, w.tol),
            "build_s": round(tb, 2),
            "build_phases_s": dict({"structure": round(o.structure_s, 2)},
                                   **{k: round(v, 2) for k, v in o.phase_s.items()}),
            "matvec_s": round(tm, 3),
            "matvec_gbs": round(oracle_matvec_bytes(o, 1) / tm / 1e9, 3),
            "gpu_build_s": round(tg, 3),
        }
        log("cpu baseline build %s: oracle %.1f s, GPU %.3f s" % (name, tb, tg))
    return out


def interp_error(w, V, T, X, results, nleaves):
    """Relative error of the compressed matvec against the interpolated matrix
    G_int (the error the recompression tolerance bounds, Section 5) on the rows
    of a seeded sample of leaf clusters, for every form, beside the error
    against the reference Galerkin matrix G on the same rows (interpolation
    plus recompression).  G_int X and G X on those rows come from the oracle."""
    from oracle.dh2 import OracleDH2
    t0 = time.perf_counter()
    o = OracleDH2(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, lazy=True)
    st = o.st
    leaves = [t for t in range(len(st.first)) if st.is_leaf(t)]
    rng = np.random.default_rng(2)
    pick = [leaves[i] for i in sorted(rng.choice(len(leaves), size=nleaves, replace=False).tolist())]
    rows, Yi = o.interp_rows(pick, X.T)
    t_int = time.perf_counter() - t0
    t0 = time.perf_counter()
    G = o.galerkin_rows(rows)
    Yg = G @ X.T
    t_gal = time.perf_counter() - t0
    out = {"sample": "%d leaf row clusters (default_rng(2)), %d rows x %d right-hand sides; oracle G_int rows "
                     "%.1f s, Galerkin rows %.1f s" % (nleaves, len(rows), X.shape[0], t_int, t_gal)}
    for label, Y in results.items():
        Yr = Y[:, rows].T
        out[label] = {"vs_interp": float(np.linalg.norm(Yr - Yi) / np.linalg.norm(Yi)),
                      "vs_galerkin": float(np.linalg.norm(Yr - Yg) / np.linalg.norm(Yg))}
    out["interp_vs_galerkin"] = float(np.linalg.norm(Yi - Yg) / np.linalg.norm(Yg))
    log("errors on sampled rows: %s" % json.dumps(out))
    return out, (st, o.tri, o.structure_s)


def householder_build(w, V, T, Xd, Y64, dh2, torch, results):
    """The same FP64 build with the total weights factored by Householder QR
    (the construction as stated) beside the Gram form of the timed steps: its
    build time and phases, and the relative difference of its product."""
    nrhs = Xd.shape[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, max_nrhs=max(nrhs, 1),
                   weights=dh2.WEIGHTS_HOUSEHOLDER)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    st = h.stats()
    Yd = torch.empty_like(Xd)
    h.matvec(Xd, Yd)
    torch.cuda.synchronize()
    results["fp64_householder"] = Yd.cpu().numpy()
    diff = float(torch.linalg.norm(Yd - Y64) / torch.linalg.norm(Y64))
    h.free()
    log("householder build %.2f s (total weights %.0f ms), product vs Gram form %.3e"
        % (tb, st["ms_total_weights"], diff))
    return {"build_s": round(tb, 3), "total_weights_ms": round(st["ms_total_weights"], 1),
            "qr_flops": st["qr_flops"], "rel_diff_vs_timed": diff,
            "rank_mean_row": round(st["rank_mean_row"], 3), "rank_mean_col": round(st["rank_mean_col"], 3)}


def paper_quadrature_form(args, w, V, T, X, Xd, Y64, dh2, torch):
    """The timed build with the paper's quadrature (Section 5: Sauter-Erichsen-
    Schwab order 5 for touching pairs, Duffy-Gauss order 3 otherwise; the timed
    steps use the 16-point near rule with the closed-form self term): build
    time and phases, touching pairs, matvec time, the relative difference of its
    product from the timed one (the two quadratures), and its errors against
    the interpolated and the Galerkin matrix of the same quadrature on the
    sampled rows (oracle with quadrature="paper")."""
    from oracle.dh2 import OracleDH2
    nrhs = Xd.shape[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, max_nrhs=max(nrhs, 1),
                   weights=WEIGHTS, quadrature=dh2.QUAD_PAPER)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    st = h.stats()
    Yd = torch.empty_like(Xd)
    h.matvec(Xd, Yd)
    torch.cuda.synchronize()
    reps = 5
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        h.matvec(Xd, Yd)
    e1.record()
    torch.cuda.synchronize()
    mv_ms = e0.elapsed_time(e1) / reps
    Y = Yd.cpu().numpy()
    diff = float(torch.linalg.norm(Yd - Y64) / torch.linalg.norm(Y64))
    h.free()
    out = {"build_s": round(tb, 3),
           "build_phases_ms": {k[3:]: round(st[k], 1) for k in ("ms_near", "ms_interp", "ms_block_weights",
                                                                "ms_total_weights", "ms_truncation",
                                                                "ms_projection", "ms_total")},
           "touching_pairs": st["touching_pairs"], "matvec_ms": round(mv_ms, 3),
           "rank_mean_row": round(st["rank_mean_row"], 3),
           "rel_diff_vs_timed_quadrature": diff}
    log("paper quadrature: build %.2f s (near field %.0f ms, %d touching pairs), matvec %.3f ms, "
        "product vs timed quadrature %.3e" % (tb, st["ms_near"], st["touching_pairs"], mv_ms, diff))
    if args.err_sample_leaves > 0:
        t0 = time.perf_counter()
        o = OracleDH2(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, lazy=True, quadrature="paper")
        ost = o.st
        leaves = [t for t in range(len(ost.first)) if ost.is_leaf(t)]
        rng = np.random.default_rng(2)
        pick = [leaves[i] for i in sorted(rng.choice(len(leaves), size=args.err_sample_leaves,
                                                     replace=False).tolist())]
        rows, Yi = o.interp_rows(pick, X.T)
        Yg = o.galerkin_rows(rows) @ X.T
        Yr = Y[:, rows].T
        out["rel_err"] = {"sample": "the same %d leaf row clusters as rel_err (%d rows), oracle with the "
                                    "paper's quadrature, %.1f s" % (len(pick), len(rows), time.perf_counter() - t0),
                          "vs_interp": float(np.linalg.norm(Yr - Yi) / np.linalg.norm(Yi)),
                          "vs_galerkin": float(np.linalg.norm(Yr - Yg) / np.linalg.norm(Yg)),
                          "interp_vs_galerkin": float(np.linalg.norm(Yi - Yg) / np.linalg.norm(Yg))}
        log("paper quadrature errors on sampled rows: %s" % json.dumps(out["rel_err"]))
    return out


def fp32_form(args, w, V, T, X, Y64, dh2, torch, results, precision=None):
    """The FP32 form (or, with precision = BF16X3, its split-BF16x3 variant)
    on the same workload: one build, event-timed matvecs on complex64
    right-hand sides (the FP64 draw rounded), and the relative Frobenius
    difference of the full n x nrhs result from the FP64 form."""
    if precision is None:
        precision = dh2.FP32
    label = "fp32" if precision == dh2.FP32 else "bf16x3"
    nrhs = X.shape[0]
    Xd = torch.from_numpy(X.astype(np.complex64)).to("cuda:0")
    Yd = torch.empty_like(Xd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, precision=precision,
                   max_nrhs=max(nrhs, 1), weights=WEIGHTS)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    st = h.stats()
    h.matvec(Xd, Yd)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(args.matvec_reps):
        ev0.record()
        h.matvec(Xd, Yd)
        ev1.record()
        ev1.synchronize()
        times.append(ev0.elapsed_time(ev1))
    mv_ms = statistics.median(times)
    mv_bytes = st["matvec_bytes"] + nrhs * st["matvec_bytes_per_rhs"]
    phases = {}
    near_ms = []
    near_bytes = 0.0
    for _ in range(args.matvec_reps):
        ph, near_bytes = h.matvec_profile(Xd, Yd)
        near_ms.append(ph["near"])
        for k, v in ph.items():
            phases.setdefault(k, []).append(v)
    near_avg = sum(near_ms) / len(near_ms)
    near_alg = near_bytes + 2.0 * 8.0 * len(T) * nrhs
    h.matvec(Xd, Yd)
    torch.cuda.synchronize()
    err = (torch.linalg.vector_norm(Yd.to(torch.complex128) - Y64) / torch.linalg.vector_norm(Y64)).item()
    results[label] = Yd.cpu().numpy().astype(np.complex128)
    h.free()
    log("%s form: build %.2f s, matvec %.3f ms (%.1f GB/s), near %.3f ms (%.1f GB/s), rel. diff vs FP64 %.2e"
        % (label, tb, mv_ms, mv_bytes / (mv_ms * 1e-3) / 1e9, near_avg, near_alg / (near_avg * 1e-3) / 1e9, err))
    return {
        "dtype": ("f32 matvec and near field; recompression products f32 on matrix cores with f32 "
                  "accumulation, FP64 QR and SVD" if precision == dh2.FP32 else
                  "f32 matvec and near field; recompression products split-BF16x3 with f32 accumulation, "
                  "FP64 QR and SVD"),
        "build_s": round(tb, 3),
        "build_gemm": {"flops": st["gemm_flops"], "launches": st["gemm_launches"]},
        "weights_gram": bool(st["weights_gram"]),
        "ranks": {"row_mean": round(st["rank_mean_row"], 2), "row_max": st["rank_max_row"]},
        "matvec_ms": round(mv_ms, 3), "value": round(mv_bytes / (mv_ms * 1e-3) / 1e9, 2), "unit": "GB/s",
        "rel_diff_vs_fp64": err,
        "matvec_phases_ms": {k: round(sum(v) / len(v), 4) for k, v in phases.items()},
        "near": {"achieved": round(near_alg / (near_avg * 1e-3) / 1e9, 1), "unit": "GB/s",
                 "frac": round(near_alg / (near_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "bytes_per_launch": near_alg, "avg_launch_ms": round(near_avg, 4)},
        "build_phases_ms": {k[3:]: round(v, 1) for k, v in st.items() if k.startswith("ms_")},
    }


# The paper's row for this workload in its table of the spectral-norm sphere
# experiment (Section 5): mean rank, recompressed basis and matrix storage in
# KB per degree of freedom, relative spectral error.
SPECTRAL_PAPER = {"rank": 15, "basis_kb_per_dof": 1.7, "matrix_kb_per_dof": 312.3, "rel_error": 1.74e-5}


# the largest row of the paper's unit-sphere table at its own wave number, and
# the paper's CPU times for that size (context: other hardware, its quadrature)
TABLE3_131K = {"n": 131072, "kappa": 64, "rank": 21, "basis_kb_per_dof": 3.9, "matrix_kb_per_dof": 586.7,
               "rel_error": 2.64e-5,
               "cpu_times_s": {"setup_interpolation": 203, "recompression": 1475,
                               "hardware": "2x Xeon Platinum 8160, 48 cores, OpenMP"}}


def spectral_form(args, dh2, torch, name="sphere32k_spec", paper_row=None, builds=2):
    """The spectral-norm error control on its own workload (default sphere
    n = 32768, kappa 32, m 4, leaf 32, eps 1e-4): the last of `builds` builds,
    ranks and storage against the paper's row, event-timed single-vector
    matvecs."""
    w = synth.WORKLOADS[name]
    V, T = synth.make_mesh(w)
    n = len(T)
    X = synth.complex_gaussian(n, 1, seed=0)
    Xd = torch.from_numpy(X).to("cuda:0")
    Yd = torch.empty_like(Xd)
    tb = []
    for _ in range(builds):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, max_nrhs=1,
                       norm=dh2.NORM_SPECTRAL, weights=WEIGHTS)
        torch.cuda.synchronize()
        tb.append(time.perf_counter() - t0)
        if len(tb) < builds:
            h.free()
    st = h.stats()
    h.matvec(Xd, Yd)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(args.matvec_reps):
        ev0.record()
        h.matvec(Xd, Yd)
        ev1.record()
        ev1.synchronize()
        times.append(ev0.elapsed_time(ev1))
    h.free()
    mv_ms = statistics.median(times)
    mv_bytes = st["matvec_bytes"] + st["matvec_bytes_per_rhs"]
    matrix = (st["near_entries"] + st["coupling_entries"]) * 16 / 1024 / n
    basis = st["basis_entries"] * 16 / 1024 / n
    log("spectral control %s: build %.2f s, mean rank %.1f / %.1f, matrix %.1f KB/DOF, basis %.2f KB/DOF, "
        "matvec %.3f ms" % (w.name, tb[-1], st["rank_mean_row"], st["rank_mean_col"], matrix, basis, mv_ms))
    return {
        "workload": "%s: unit sphere n=%d, kappa=%g, m=%d, leaf %d, eta=%g, eta1=%g, tol=%g, spectral control, "
                    "FP64, 1 right-hand side" % (w.name, n, w.kappa, w.order, w.leaf, w.eta, w.eta1, w.tol),
        "build_s": round(tb[-1], 3),
        "build_phases_ms": {k[3:]: round(v, 1) for k, v in st.items() if k.startswith("ms_")},
        "rank_mean_row": round(st["rank_mean_row"], 2), "rank_mean_col": round(st["rank_mean_col"], 2),
        "rank_max_row": st["rank_max_row"],
        "matrix_kb_per_dof": round(matrix, 1), "basis_kb_per_dof": round(basis, 2),
        "matvec_ms": round(mv_ms, 3), "matvec_gbs": round(mv_bytes / (mv_ms * 1e-3) / 1e9, 1),
        "paper_row": SPECTRAL_PAPER if paper_row is None else paper_row,
    }


def learned_form(args, w, V, T, X, Y64, dh2, torch, results, st_exact, build_exact):
    """The learned-rank form on the benchmark workload (FP64): one build with
    the predictor sizing randomized truncations, its truncation time and build
    time against the exact FP64 form's, sketch and fallback counts, ranks, and
    the difference of its n x nrhs product from the exact form's; then the
    same comparison on a side-2 cube of the learned-rank family (k = 216)."""
    nrhs = X.shape[0]
    Xd = torch.from_numpy(X).to("cuda:0")
    Yd = torch.empty_like(Xd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, max_nrhs=max(nrhs, 1),
                   rank_mode=dh2.RANKS_LEARNED, weights=WEIGHTS)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    st = h.stats()
    h.matvec(Xd, Yd)
    torch.cuda.synchronize()
    err = (torch.linalg.vector_norm(Yd - Y64) / torch.linalg.vector_norm(Y64)).item()
    results["learned"] = Yd.cpu().numpy()
    h.free()
    out = {"workload": w.name, "build_s": round(tb, 3), "build_s_exact": round(build_exact, 3),
           "truncation_ms": round(st["ms_truncation"], 1), "truncation_ms_exact": round(st_exact["ms_truncation"], 1),
           "predict_ms": round(st["ms_rank_predict"], 2), "sketch_slots": st["sketch_slots"],
           "fallbacks": st["sketch_fallbacks"], "rank_mean_row": round(st["rank_mean_row"], 3),
           "rank_mean_row_exact": round(st_exact["rank_mean_row"], 3), "rel_diff_vs_exact": err}
    log("learned form: build %.2f s (exact %.2f s), truncation %.0f ms (exact %.0f ms), %d sketches, %d fallbacks, "
        "rel. diff vs exact %.2e" % (tb, build_exact, st["ms_truncation"], st_exact["ms_truncation"],
                                    st["sketch_slots"], st["sketch_fallbacks"], err))
    wc = synth.WORKLOADS[args.learned_cube]
    Vc, Tc = synth.make_mesh(wc)
    Xc = torch.from_numpy(synth.complex_gaussian(len(Tc), 4, seed=0)).to("cuda:0")
    cube = {"workload": "%s: side-2 cube n=%d, kappa=%g, m=%d (k=%d), leaf %d, tol %g"
                        % (wc.name, len(Tc), wc.kappa, wc.order, wc.order ** 3, wc.leaf, wc.tol)}
    ys = {}
    for label, mode in (("exact", dh2.RANKS_EXACT), ("learned", dh2.RANKS_LEARNED)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hc = dh2.Handle(Vc, Tc, wc.kappa, wc.order, wc.eta, wc.leaf, wc.tol, eta1=wc.eta1, max_nrhs=4,
                        rank_mode=mode, weights=WEIGHTS)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        sc = hc.stats()
        Yc = torch.empty_like(Xc)
        hc.matvec(Xc, Yc)
        torch.cuda.synchronize()
        ys[label] = Yc
        hc.free()
        cube[label] = {"build_s": round(tc, 3), "truncation_ms": round(sc["ms_truncation"], 1),
                       "total_weights_ms": round(sc["ms_total_weights"], 1), "sketch_slots": sc["sketch_slots"],
                       "fallbacks": sc["sketch_fallbacks"], "rank_mean_row": round(sc["rank_mean_row"], 3)}
    cube["rel_diff_learned_vs_exact"] = (torch.linalg.vector_norm(ys["learned"] - ys["exact"])
                                         / torch.linalg.vector_norm(ys["exact"])).item()
    log("learned form, %s: %s" % (wc.name, json.dumps(cube)))
    out["cube_family"] = cube
    return out


def batch_form(args, dh2, torch, count):
    """The batching form: count problems of the seeded recipe (sphere, cube and
    ellipsoid surfaces, n ~ U[2k, 32k], kappa ~ U[4, 24], m 4, leaf 32, tol
    1e-5), FP32 form, 64 complex64 right-hand sides each, block-row pipeline
    shapes autotuned per problem.  Builds one by one;
    all products then run as one graph launch (dh2_batch_run), timed against
    the same products issued one handle after another, and checked bit for
    bit against them."""
    ws = synth.batch_workloads(count=count)
    nrhs = 64
    hs, X, Ye, Yb = [], [], [], []
    bytes_total = 0.0
    tb = 0.0
    shapes, tune_ms = {}, 0.0
    for i, w in enumerate(ws):
        V, T = synth.make_mesh(w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, precision=dh2.FP32,
                       max_nrhs=nrhs, weights=WEIGHTS, autotune=1)
        torch.cuda.synchronize()
        tb += time.perf_counter() - t0
        st = h.stats()
        shapes[tuple(st["mv_variant"])] = shapes.get(tuple(st["mv_variant"]), 0) + 1
        tune_ms += st["ms_autotune"]
        bytes_total += st["matvec_bytes"] + nrhs * st["matvec_bytes_per_rhs"]
        hs.append(h)
        X.append(torch.from_numpy(synth.complex_gaussian(len(T), nrhs, seed=100 + i).astype(np.complex64))
                 .to("cuda:0"))
        Ye.append(torch.empty_like(X[-1]))
        Yb.append(torch.empty_like(X[-1]))
    log("batch form: %d problems, n total %d, builds one after another %.1f s" % (count, sum(w.n for w in ws), tb))
    # the same builds side by side (dh2_build_many): 8 host threads, a stream per problem
    probs = []
    for w in ws:
        V, T = synth.make_mesh(w)
        probs.append((V, T, w.kappa, w.order, w.eta, w.leaf, w.tol))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hm = dh2.build_many(probs, precision=dh2.FP32, max_nrhs=nrhs, threads=8, weights=WEIGHTS, autotune=1)
    torch.cuda.synchronize()
    tbm = time.perf_counter() - t0
    same_build = True
    for h1, h2, x in zip(hs, hm, X):
        y1, y2 = torch.empty_like(x), torch.empty_like(x)
        h1.matvec(x, y1)
        h2.matvec(x, y2)
        torch.cuda.synchronize()
        same_build = same_build and torch.equal(y1, y2)
    for h in hm:
        h.free()
    log("batch form: builds side by side %.1f s (x%.2f), products equal %s" % (tbm, tb / tbm, same_build))
    s = torch.cuda.Stream()
    b = dh2.Batch(hs, X, Yb, stream=s.cuda_stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    seq, bat = [], []
    with torch.cuda.stream(s):
        for rep in range(args.matvec_reps + 1):
            ev0.record(s)
            for h, x, y in zip(hs, X, Ye):
                h.matvec_on(x, y, s.cuda_stream)
            ev1.record(s)
            ev1.synchronize()
            if rep:
                seq.append(ev0.elapsed_time(ev1))
            ev0.record(s)
            b.run()
            ev1.record(s)
            ev1.synchronize()
            if rep:
                bat.append(ev0.elapsed_time(ev1))
    same = all(torch.equal(a, c) for a, c in zip(Yb, Ye))
    b.free()
    for h in hs:
        h.free()
    t_seq, t_bat = statistics.median(seq), statistics.median(bat)
    log("batch form: one graph launch %.3f ms, one product after another %.3f ms (x%.2f), %.1f GB/s, "
        "equal bits %s" % (t_bat, t_seq, t_seq / t_bat, bytes_total / (t_bat * 1e-3) / 1e9, same))
    return {
        "workload": "%d problems: sphere / side-2 cube / ellipsoid 1:2:3, n ~ U[2048, 32768] (total %d), "
                    "kappa ~ U[4, 24], m=4, leaf 32, tol 1e-5, FP32 form, %d complex64 right-hand sides each"
                    % (count, sum(w.n for w in ws), nrhs),
        "build_s_total": round(tb, 2), "build_s_side_by_side": round(tbm, 2),
        "side_by_side_builds_equal": same_build,
        "autotune": {"shapes_near_coupling_le16_gt16": {"%d,%d,%d,%d" % k: v for k, v in sorted(shapes.items())},
                     "tune_ms_total": round(tune_ms, 1)},
        "graph_ms": round(t_bat, 3), "one_after_another_ms": round(t_seq, 3),
        "speedup": round(t_seq / t_bat, 3), "value": round(bytes_total / (t_bat * 1e-3) / 1e9, 1), "unit": "GB/s",
        "bytes_per_batch": bytes_total, "bitwise_equal_to_single_products": same,
    }


# factorisation of the total weights in every build of this run (dh2_options.weights)
WEIGHTS = 0

# pipeline shapes of the block-row kernel (KU slices, S stages, WPE waves per SIMD)
SHAPES = [(1, 4, 2), (1, 3, 2), (1, 6, 1), (2, 3, 1)]


def shape_name(v, role):
    ku, stg, wpe = SHAPES[v]
    return "k_mv_rows_mfma<double,%d,%d,%d,1,%d>" % (ku, stg, role, wpe)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported (the path runs on one "
              "MI355X; see the design notes for how it would shard)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    import torch
    from paper_1809_04384_amd import dh2

    w = synth.WORKLOADS[args.workload]
    V, T = synth.make_mesh(w)
    n = len(T)
    nrhs = w.nrhs
    X = synth.complex_gaussian(n, nrhs, seed=0)                 # (nrhs, n) complex128
    torch.cuda.set_device(0)
    Xd = torch.from_numpy(X).to("cuda:0")
    Yd = torch.empty_like(Xd)
    log("workload %s n=%d kappa=%g m=%d leaf=%d tol=%g nrhs=%d" % (w.name, n, w.kappa, w.order, w.leaf, w.tol, nrhs))

    global WEIGHTS
    WEIGHTS = weights = dh2.WEIGHTS_GRAM if args.weights == "gram" else dh2.WEIGHTS_HOUSEHOLDER

    def step():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = dh2.Handle(V, T, w.kappa, w.order, w.eta, w.leaf, w.tol, eta1=w.eta1, max_nrhs=max(nrhs, 1),
                       autotune=args.autotune, weights=weights)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        t1 = time.perf_counter()
        h.matvec(Xd, Yd)
        torch.cuda.synchronize()
        tm = time.perf_counter() - t1
        return h, tb, tm

    for i in range(args.warmup):
        h, tb, tm = step()
        log("warmup %d: build %.2f s" % (i, tb))
        h.free()
    builds, steps_ms, h = [], [], None
    t_all = time.perf_counter()
    for i in range(args.steps):
        if h is not None:
            h.free()
        h, tb, tm = step()
        builds.append(tb)
        steps_ms.append((tb + tm) * 1e3)
        log("step %d: build %.2f s, matvec %.2f ms" % (i, tb, tm * 1e3))
    t_all = time.perf_counter() - t_all
    st = h.stats()
    log("stats " + json.dumps({k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}))

    # matvec throughput: median of event-timed calls on the current stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(args.matvec_reps):
        ev0.record()
        h.matvec(Xd, Yd)
        ev1.record()
        ev1.synchronize()
        times.append(ev0.elapsed_time(ev1))
    mv_ms = statistics.median(times)
    mv_bytes = st["matvec_bytes"] + nrhs * st["matvec_bytes_per_rhs"]
    mv_gbs = mv_bytes / (mv_ms * 1e-3) / 1e9
    # near field (the dominant kernel) and coupling, timed with events around their launches
    phases = {}
    near_ms = []
    near_bytes = 0.0
    for _ in range(args.matvec_reps):
        ph, near_bytes = h.matvec_profile(Xd, Yd)
        near_ms.append(ph["near"])
        for k, v in ph.items():
            phases.setdefault(k, []).append(v)
    near_avg = sum(near_ms) / len(near_ms)
    e = 16.0
    near_alg = near_bytes + 2.0 * e * n * nrhs
    near_gbs = near_alg / (near_avg * 1e-3) / 1e9
    log("matvec %.3f ms (%.1f GB/s); near field %.3f ms, %.2f GB -> %.1f GB/s"
        % (mv_ms, mv_gbs, near_avg, near_alg / 1e9, near_gbs))
    # coupling kernel: every recompressed coupling read once, x_sc read and y_tc written once
    coup_avg = sum(phases["coupling"]) / len(phases["coupling"])
    coup_alg = e * st["coupling_entries"] + e * nrhs * (st["rank_mean_row"] * st["n_row_slots"]
                                                        + st["rank_mean_col"] * st["n_col_slots"])
    coup_gbs = coup_alg / (coup_avg * 1e-3) / 1e9
    # build: complex products and Householder steps of the recompression against the FP64 peak
    build_tflops = (st["gemm_flops"] + st["qr_flops"]) / statistics.median(builds) / 1e12
    h.matvec(Xd, Yd)
    Y64 = Yd.clone()
    h.free()

    results = {"fp64": Y64.cpu().numpy()}
    hh = None
    if not args.no_householder_build and args.weights == "gram":
        hh = householder_build(w, V, T, Xd, Y64, dh2, torch, results)
    paperq = None
    if not args.no_paper_quadrature:
        paperq = paper_quadrature_form(args, w, V, T, X, Xd, Y64, dh2, torch)
    fp32 = None
    if not args.no_fp32:
        fp32 = fp32_form(args, w, V, T, X, Y64, dh2, torch, results)

    bf = None
    if not args.no_bf16x3:
        bf = fp32_form(args, w, V, T, X, Y64, dh2, torch, results, precision=dh2.BF16X3)

    learned = None
    if not args.no_learned:
        learned = learned_form(args, w, V, T, X, Y64, dh2, torch, results, st, statistics.median(builds))

    batch = None
    if args.batch > 0:
        batch = batch_form(args, dh2, torch, args.batch)

    spec = None
    if not args.no_spectral:
        spec = spectral_form(args, dh2, torch)
    paper_cfg = None
    if not args.no_paper_config:
        paper_cfg = spectral_form(args, dh2, torch, "sphere131k_k64", TABLE3_131K, builds=1)

    peaks = measured_peaks(torch)
    log("measured peaks: %s" % peaks)

    errs, pre = None, None
    if args.err_sample_leaves > 0:
        log("errors against the interpolated matrix on sampled rows (oracle) ...")
        errs, pre = interp_error(w, V, T, X, results, args.err_sample_leaves)

    base = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        base = cpu_baseline(w, V, T, X, args.cpu_sample_leaves, pre)
        log("cpu baseline %.3f GB/s" % base["value"])
        if args.cpu_build_workloads:
            base["build"] = cpu_build_baseline(args.cpu_build_workloads.split(","), dh2, torch)

    out = {
        "metric": METRIC,
        "value": round(mv_gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_all * 1e3 / max(args.steps, 1), 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s: unit sphere n=%d, kappa=%g, m=%d (k=%d), leaf %d, eta=%g, eta1=%g, "
                               "tol=%g, %d complex128 right-hand sides, FP64 form, %s total weights"
                               % (w.name, n, w.kappa, w.order, w.order ** 3, w.leaf, w.eta, w.eta1,
                                  w.tol, nrhs, args.weights),
                   "n": n, "kappa": w.kappa, "order": w.order, "leafsize": w.leaf, "tol": w.tol,
                   "nrhs": nrhs, "precision": "fp64", "weights": args.weights},
        "build_s": round(statistics.median(builds), 3),
        "matvec_ms": round(mv_ms, 3),
        "build_phases_ms": {k[3:]: round(v, 1) for k, v in st.items() if k.startswith("ms_")},
        "build_gemm": {"flops": st["gemm_flops"], "launches": st["gemm_launches"]},
        "weights": {"timed": args.weights, "gram_taken": bool(st["weights_gram"]),
                    "householder_build": hh},
        "mv_shapes": {"autotune": args.autotune, "near": shape_name(st["mv_variant"][0], 0),
                      "coupling": shape_name(st["mv_variant"][1], 1), "tune_ms": round(st["ms_autotune"], 1)},
        "matvec_phases_ms": {k: round(sum(v) / len(v), 4) for k, v in phases.items()},
        "ranks": {"row_max": st["rank_max_row"], "row_mean": round(st["rank_mean_row"], 2),
                  "col_max": st["rank_max_col"], "col_mean": round(st["rank_mean_col"], 2)},
        "storage_kb_per_dof": {
            "near": round(st["near_entries"] * 16 / 1024 / n, 1),
            "coupling": round(st["coupling_entries"] * 16 / 1024 / n, 1),
            "basis": round(st["basis_entries"] * 16 / 1024 / n, 1)},
        "roofline": {"bound": "hbm", "achieved": round(near_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(near_gbs / HBM_PEAK_GBS, 4),
                     "traffic": (measured_traffic(shape_name(st["mv_variant"][0], 0))
                                 if args.workload == "sphere131k" and nrhs == 16 else None),
                     "kernel": "%s (near-field block rows on matrix cores)" % shape_name(st["mv_variant"][0], 0),
                     "bytes_per_launch": near_alg, "avg_launch_ms": round(near_avg, 4),
                     "measured_peaks": peaks,
                     "frac_of_measured_read": round(near_gbs / peaks["hbm_read_gbs"], 4) if peaks else None,
                     "whole_matvec": {"achieved": round(mv_gbs, 1), "unit": "GB/s",
                                      "frac": round(mv_gbs / HBM_PEAK_GBS, 4), "bytes": mv_bytes,
                                      "ms": round(mv_ms, 4)},
                     "coupling_kernel": {"kernel": shape_name(st["mv_variant"][1], 1), "achieved": round(coup_gbs, 1),
                                         "unit": "GB/s", "frac": round(coup_gbs / HBM_PEAK_GBS, 4),
                                         "bytes_per_launch": coup_alg, "avg_launch_ms": round(coup_avg, 4)},
                     "build": {"bound": "fp64", "achieved": round(build_tflops, 2), "unit": "TFLOP/s",
                               "peak": FP64_PEAK_TFLOPS, "frac": round(build_tflops / FP64_PEAK_TFLOPS, 4),
                               "flops": st["gemm_flops"] + st["qr_flops"],
                               "note": "complex products (8 MNK, only the products outside the zeros "
                                       "of a trapezoidal basis weight) and Householder QR steps (8 M n^2) "
                                       "of the recompression over the whole build time"}},
        "rel_err": errs,
        "cpu_baseline": base,
        "fp32_form": fp32,
        "bf16x3_form": bf,
        "spectral_form": spec,
        "paper_quadrature_form": paperq,
        "paper_table3_131k": paper_cfg,
        "batch_form": batch,
        "learned_form": learned,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
