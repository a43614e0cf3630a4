#!/usr/bin/env python3
"""Throughput of the G-REST eigenpair update on one MI355X.

Default workload (``--config c3``, the headline): stochastic block model with
n0 = 1,000,000 nodes, 32 blocks with Dirichlet(2) sizes, mean degree 20 (80 %
intra-block), adjacency operator, K = 32 tracked pairs, G-REST_RSVD with L = P = 32
(subspace width 3K = 96); every step appends 10,000 nodes and about 50,000 edges.
Other configurations: ``c1`` (SBM n0 = 2000, K = 8, G-REST3, FP64), ``c2`` (Chung-Lu
n0 = 1e5, normalised Laplacian, K = 32, FP32) and ``c5`` (Chung-Lu n0 = 4e6,
combinatorial Laplacian, 64 non-trivial pairs).  Data are synthetic (seeded
generator); the initial pairs come from the library's device eigensolver.  The change
lists and Gaussian test matrices are uploaded to HBM before the timed region, which
contains exactly ``--steps`` updates bracketed by device synchronisations.

Printed JSON line: the headline updates/s, the comparison path and (c3) the truncated
low-rank form beside it; for each an accuracy gate against the FP64 oracle (the oracle
replays the first updates from the state's own initial pairs: eigenvalue error, subspace
sine, residual ||M u - lambda u|| / ||M||) and the properties of the timed state after
its updates (graph, Rayleigh quotients, orthonormality); per-stage times; the roofline of
the dominant kernel measured with HIP events around it; (c3) the serving latencies of
the many-graph mix; and the oracle's own speed on this host (``cpu_baseline``).  The
oracle runs only in the accuracy replays, which double as the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TOL_EIG = {"fp64": 1e-10, "fp32": 1e-5, "mixed": 1e-3}
TOL_SINE = {"fp64": 1e-8, "fp32": 1e-3, "mixed": 1e-3}
TOL_ORTH = {"fp64": 1e-12, "fp32": 1e-5, "mixed": 1e-5}

# workloads of the measured configurations (the SBM and Chung-Lu generators of workloads.py)
CONFIGS = {
    "c3": dict(preset="sbm_n1e6", op="adj", k=32, variant="rsvd", L=32, P=32, max_new=0, precision="mixed",
               compare="fp32", lowrank=True, serving=256, oracle_steps=2,
               workload="SBM n0=1e6, 32 Dirichlet(2) blocks, mean degree 20, +10k nodes/+50k edges per step; "
                        "adjacency, k=32, G-REST_RSVD L=P=32 (width 96)"),
    "c1": dict(preset="sbm_n2000", op="adj", k=8, variant="g3", L=0, P=0, max_new=100, precision="fp64",
               compare="", lowrank=False, serving=0, oracle_steps=10,
               workload="SBM n0=2000, 4 equal blocks, p_in=0.05, p_out=0.005, +100 nodes/+300/-100 edges per "
                        "step; adjacency, k=8, G-REST3, FP64"),
    "c2": dict(preset="chunglu_n1e5", op="nlap", k=32, variant="g2", L=0, P=0, max_new=0, precision="fp32",
               compare="mixed", lowrank=False, serving=0, oracle_steps=4,
               workload="Chung-Lu n0=1e5, pdf exponent 2.5, mean degree 16, max 2000; +0.5%/-0.2% edges per "
                        "step; normalised Laplacian (2I - L_n), k=32 smallest, G-REST2 (S=0), FP32"),
    "c5": dict(preset="chunglu_n4e6", op="lap", k=65, variant="rsvd", L=64, P=64, max_new=0, precision="mixed",
               compare="", lowrank=False, serving=0, oracle_steps=1,
               workload="Chung-Lu n0=4e6, pdf exponent 2.2, mean degree 16; +1% nodes per step; combinatorial "
                        "Laplacian (alpha I - L), k=65 smallest (64 non-trivial), G-REST_RSVD L=P=64 (width 194), "
                        "mixed"),
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=sorted(CONFIGS))
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default=None, choices=["mixed", "fp32", "fp64"],
                    help="headline precision (default: the configuration's)")
    ap.add_argument("--compare", default=None, help="second path timed beside the headline ('' to skip)")
    ap.add_argument("--no-lowrank", action="store_true",
                    help="skip timing the low-rank projected matrix (eq. ..._main3) beside the headline")
    ap.add_argument("--scale", type=float, default=1.0, help="shrink node counts (quick runs only)")
    ap.add_argument("--init-iters", type=int, default=300,
                    help="product budget of the device's initial eigensolver (it stops earlier on its residual)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run each update's graph stage on the state's stream (no second stream)")
    ap.add_argument("--no-host-inputs", action="store_true",
                    help="skip the headline path timed with its inputs in host memory (PCIe copies included)")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle replays (no accuracy against the oracle, no CPU baseline)")
    ap.add_argument("--oracle-steps", type=int, default=None,
                    help="updates replayed by the oracle per timed path (default: the configuration's)")
    ap.add_argument("--serving-graphs", type=int, default=None,
                    help="graphs in the many-graph serving leg (0 skips it; default 256 for c3)")
    ap.add_argument("--serving-rates", default="50,100,200,500,1000,2000", help="Poisson arrival rates, requests/s")
    ap.add_argument("--serving-requests", default="200,300,500,1000,2000,3000", help="requests per rate")
    ap.add_argument("--serving-lanes", type=int, default=8)
    ap.add_argument("--serving-batch", type=int, default=1,
                    help="requests of distinct graphs a lane runs as one batched update (1: one at a time)")
    ap.add_argument("--serving-burst", type=int, default=512,
                    help="requests of the saturation burst (served path vs plain FP32 per-graph path)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a reference kernel of "
                         "known traffic for hardware byte counters)")
    ap.add_argument("--quiet", action="store_true")
    args = ap.parse_args()
    cfg = CONFIGS[args.config]
    if args.precision is None:
        args.precision = cfg["precision"]
    if args.compare is None:
        args.compare = cfg["compare"]
    if args.oracle_steps is None:
        args.oracle_steps = cfg["oracle_steps"]
    if args.serving_graphs is None:
        args.serving_graphs = cfg["serving"]
    if not cfg["lowrank"]:
        args.no_lowrank = True
    return args, cfg


def log(args, *msg):
    if not args.quiet:
        print("[bench]", *msg, file=sys.stderr, flush=True)


def spmm_bytes(n2: int, nnz: int, width: int, elem: int) -> float:
    """Algorithmic bytes of one product with the updated operator: column ids (4 B per
    stored entry), row offsets (8 B per row), the basis read once and the product
    written once (n' x width elements each)."""
    return 4.0 * nnz + 8.0 * (n2 + 1) + 2.0 * elem * n2 * width


def width_mix(wm: float, D: int, K: int) -> dict:
    """Widths of the timed sparse products and their shares, from their mean width wm: with
    the kept product of the tracked block (adjacency) an update multiplies the D - K new
    columns and a refresh all D, so a mean strictly between the two is that mix (a mean of
    66 at D = 96, K = 32 is 15 updates at 64 and one at 96, not 16 at 66); otherwise every
    product has the mean width."""
    if D - K + 1e-6 < wm < D - 1e-6:
        f_full = (wm - (D - K)) / K
        return {D - K: 1.0 - f_full, D: f_full}
    return {int(round(wm)): 1.0}


def gather_ceiling(res, K):
    """Average time of grest_calib_gather (random gathers of whole rows, the column ids from
    a hash) at the timed updates' mean row and entry counts, the entries spread evenly over
    the rows, and their mix of product widths: the ceiling of the sparse product's own
    access pattern."""
    import torch
    from paper_2603_19439_amd import grest as G
    sizes, wm = res["sizes"], res["spmm_width"]
    if not sizes or wm <= 0:
        return None
    n2 = int(round(sum(s[0] for s in sizes) / len(sizes)))
    nnz = int(round(sum(s[1] for s in sizes) / len(sizes)))
    D = int(sizes[0][2])
    mix = width_mix(wm, D, K)
    ld = (D + 3) // 4 * 4
    Z = torch.randn(n2, ld, device="cuda")
    Y = torch.empty(n2, ld, device="cuda")
    rp = torch.arange(n2 + 1, dtype=torch.int64, device="cuda") * nnz // n2  # entries spread evenly
    t = 0.0
    per_width = {}
    for w, f in mix.items():
        wp = (w + 3) // 4 * 4
        for _ in range(40):  # warm-up: the chip's clocks ramp up after the host-side checks
            G.calib_gather(rp, Z, wp, Y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            G.calib_gather(rp, Z, wp, Y)
        e1.record()
        e1.synchronize()
        per_width[wp] = e0.elapsed_time(e1) / 20
        t += f * per_width[wp]
    print(f"[bench] gather ceiling (ms per launch by width): {per_width}", file=sys.stderr, flush=True)
    del Z, Y, rp
    torch.cuda.empty_cache()
    return t


def cpu_info():
    """Host CPU model and logical core count (from /proc/cpuinfo)."""
    model, count = "unknown", os.cpu_count()
    try:
        names = [ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")]
        if names:
            model, count = names[0], len(names)
    except OSError:
        pass
    return model, count


def blas_threads():
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        return max((i.get("num_threads") or 1) for i in info) if info else os.cpu_count()
    except Exception:
        return os.cpu_count()


# ------------------------------------------------------------------------------------
# accuracy against the oracle
# ------------------------------------------------------------------------------------
def reported_matrix(A, op):
    """The matrix whose values are reported: A, L = D - A or L_n = I - D^-1/2 A D^-1/2
    (isolated nodes: (L_n)_ii = 1)."""
    import numpy as np
    import scipy.sparse as sp
    if op == "adj":
        return A
    deg = np.asarray(A.sum(axis=1)).ravel()
    if op == "lap":
        return (sp.diags(deg) - A).tocsr()
    s = np.zeros_like(deg)
    s[deg > 0] = 1.0 / np.sqrt(deg[deg > 0])
    S = sp.diags(s)
    return (sp.identity(A.shape[0], format="csr") - S @ A @ S).tocsr()


def matrix_norm(Mm):
    import numpy as np
    from scipy.sparse.linalg import eigsh
    v = eigsh(Mm, k=1, which="LM", tol=1e-6, return_eigenvectors=False)
    return float(np.abs(v).max())


def compare_step(vals, X, r, op, k, Mm, norm_m):
    """Errors of one GPU result (vals, X) against the oracle's step r: eigenvalue relative
    error and subspace sine over the prefix k* <= K that the oracle separates from the rest
    by a gap >= 1e-3 of |theta_1| (adjacency) or of the largest tracked nu (Laplacians,
    whose shift would otherwise set the scale; nu without the trivial pair), the residual
    max_j ||M u_j - lambda_j u_j|| / ||M|| of both results on the reported matrix M, and
    the orthonormality of the GPU block."""
    import numpy as np
    from oracle import grest_oracle as O
    from paper_2603_19439_amd import metrics as Mx
    th_all = np.linalg.eigvalsh(r.H)
    order = O.select(th_all, th_all.size, O.which_for(op))
    if op == "adj":
        kk = Mx.gap_prefix(np.abs(th_all[order]), k, 1e-3)
    else:  # gaps between the nu = shift - theta of L or L_n, relative to the tracked nu's scale
        nu = r.shift - th_all[order]
        kk = Mx.gap_prefix(nu, k, 1e-3, scale=max(float(np.abs(nu[:k]).max()), 1e-300))
    ref = r.theta if op == "adj" else r.nu_rq
    if op == "adj":
        e = Mx.eig_rel_error(vals[:kk], ref[:kk])
    else:
        e = Mx.eig_rel_error(vals[1:kk], ref[1:kk]) if kk > 1 else 0.0
    sine = Mx.subspace_sine(X[:, :kk], r.X[:, :kk]) if kk > 0 else 0.0
    return {"k_star": int(kk), "e_lambda": float(e), "sine": float(sine),
            "resid_gpu": Mx.residual(Mm, X, vals, norm_m), "resid_oracle": Mx.residual(Mm, r.X, ref, norm_m),
            "orthonormality": Mx.orthonormality(X)}


class OracleReplays:
    """Replays of the first updates of each timed path through the FP64 oracle, from the
    path's own initial pairs; the norms of the reported matrices are shared by the paths."""

    def __init__(self, wl, cfg, steps):
        self.wl, self.cfg, self.steps = wl, cfg, steps
        self.mats = {}
        self.seconds = []

    def matrix(self, t, A):
        if t not in self.mats:
            Mm = reported_matrix(A, self.cfg["op"])
            self.mats[t] = (Mm, matrix_norm(Mm))
        return self.mats[t]

    def replay(self, start, outs, proj, prec, args, exact_for_distance=None):
        import numpy as np
        from oracle import grest_oracle as O
        from paper_2603_19439_amd import workloads as W
        cfg, wl = self.cfg, self.wl
        op, k = cfg["op"], cfg["k"]
        vals0, X0 = start
        A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
        shift0 = 0.0
        if op != "adj":
            _, shift0 = O.operator_matrix(A, op)
        th = vals0 if op == "adj" else shift0 - vals0
        X = X0
        res, steps_out = [], []
        t0 = time.perf_counter()
        for t, d in enumerate(wl.deltas[:len(outs)]):
            om = W.omega(wl.cfg_id, 0, t + 1, d.n_new, cfg["L"] + cfg["P"]) \
                if cfg["variant"] == "rsvd" and d.n_new > 0 else None
            r = O.grest_step(A, X, th, d.n_new, d.i, d.j, d.sign, k, variant=cfg["variant"], op=op,
                             proj=proj, L=cfg["L"] or None, Omega=om)
            A, X, th = r.A, r.X, r.theta
            res.append(r)
        dt = time.perf_counter() - t0
        if proj == "exact":
            self.seconds.append((dt, len(outs)))
        gate = True
        for t, (r, (vals, Xg)) in enumerate(zip(res, outs)):
            Mm, nm = self.matrix(t + 1, r.A)
            c = compare_step(vals, Xg, r, op, k, Mm, nm)
            c["step"] = t + 1
            if exact_for_distance is not None:  # the low-rank form against the exact form's oracle
                ex = exact_for_distance[t]
                dist = compare_step(vals, Xg, ex, op, k, Mm, nm)
                c["vs_exact_form"] = {"e_lambda": dist["e_lambda"], "sine": dist["sine"], "k_star": dist["k_star"]}
            ok = c["e_lambda"] <= TOL_EIG[prec] and c["sine"] <= TOL_SINE[prec] and \
                c["orthonormality"] <= TOL_ORTH[prec]
            c["passed"] = bool(ok)
            gate &= ok
            steps_out.append(c)
            log(args, f"oracle replay ({prec}, {proj}) step {t + 1}: e_lambda {c['e_lambda']:.2e} sine "
                      f"{c['sine']:.2e} (k*={c['k_star']}) resid gpu {c['resid_gpu']:.2e} oracle "
                      f"{c['resid_oracle']:.2e}")
        return {"steps": steps_out, "gate_passed": bool(gate), "oracle_seconds": round(dt, 2)}, res


def main():
    args, cfg = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the update of one graph is not "
                                   "sharded across GPUs (see the design notes for how it would shard)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2603_19439_amd import grest as G
    from paper_2603_19439_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.calib_copy_mib > 0:
        nel = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(args, f"reference copy: {args.calib_copy_mib} MiB read and {args.calib_copy_mib} MiB written")
        del src, dst
    K, L, P, op, variant = cfg["k"], cfg["L"], cfg["P"], cfg["op"], cfg["variant"]
    n_steps = max(16, args.steps, args.warmup, args.oracle_steps)
    t0 = time.time()
    wl = W.preset(cfg["preset"], scale=args.scale, steps=n_steps)
    log(args, f"{args.config}: workload generated in {time.time() - t0:.1f}s: n0={wl.n0} nnz={wl.col0.size}")
    # device-resident inputs
    dev_steps = []
    for t, d in enumerate(wl.deltas):
        om = W.omega(wl.cfg_id, 0, t + 1, d.n_new, L + P) if variant == "rsvd" and d.n_new > 0 else None
        dev_steps.append((d.n_new,
                          torch.from_numpy(d.i.astype(np.int32)).to(dev),
                          torch.from_numpy(d.j.astype(np.int32)).to(dev),
                          torch.from_numpy(d.sign.astype(np.int8)).to(dev),
                          None if om is None else torch.from_numpy(om).to(dev),
                          d.n_changes))
    n_final = wl.n_at(n_steps)
    nnz_cap = int(wl.col0.size + 2 * sum(s[5] for s in dev_steps) + 1024)
    torch.cuda.synchronize()

    def make_state(prec, proj="exact"):
        st = G.State(wl.rowptr0, wl.col0, k=K, variant=variant, op=op, precision=prec, L=L, P=P,
                     max_new=cfg["max_new"], stream=torch.cuda.current_stream().cuda_stream,
                     node_capacity=n_final + 1, nnz_capacity=nnz_cap, proj=proj)
        init_stats.append(st.init_pairs(iterations=args.init_iters, seed=7))
        start = st.get()
        if proj == "lowrank":  # the low-rank form needs Delta and the pairs only
            st.release_graph()
        st.set_overlap(not args.no_overlap)
        return st, start

    final_graph = {}
    init_stats = []  # (products, residual) of every initial eigensolve

    def final_checks(st, prec, lowrank):
        """Properties of a timed state after its updates that hold for any Rayleigh-Ritz
        output (the oracle replays cover the first updates): its graph equals the one the
        seeded generator reaches, every returned value is the Rayleigh quotient of its
        returned vector on that graph (Alg. 1), and the block is orthonormal.  The low-rank
        state has released its graph, and its values are Ritz values of the truncated
        operator (eq. RR_eigen_graph_upd_main3): their distance to the graph's quotients
        measures the truncation and is reported only."""
        import scipy.sparse as sp
        if not final_graph:
            n_t = wl.n_at(args.steps)
            rp, col = W.csr_from_keys(n_t, wl.keys_at(args.steps))
            A = sp.csr_matrix((np.ones(col.size), col.astype(np.int64), rp.astype(np.int64)), shape=(n_t, n_t))
            final_graph.update(rp=rp, col=col, A=A, M=reported_matrix(A, op))
        fg = final_graph
        vals, X = st.get()
        res = {}
        if not lowrank:
            rp_g, col_g = st.graph()
            res["graph_exact"] = bool(np.array_equal(rp_g, fg["rp"]) and np.array_equal(col_g, fg["col"]))
        k = X.shape[1]
        res["orthonormality"] = float(np.abs(X.T @ X - np.eye(k)).max())
        rq = ((fg["M"] @ X) * X).sum(axis=0)
        if op == "adj":
            rel = np.abs(vals - rq) / np.maximum(np.abs(rq), 1e-8 * np.abs(rq).max())
        else:  # nu: relative to the tracked spectrum's scale, the trivial pair included
            rel = np.abs(vals - rq) / max(np.abs(rq).max(), 1e-300)
        res["value_vs_rayleigh_quotient"] = float(rel.max())
        orth_ok = res["orthonormality"] <= TOL_ORTH[prec]
        if lowrank:
            res["gate_passed"] = bool(orth_ok)
        else:
            res["gate_passed"] = bool(res["graph_exact"] and orth_ok and
                                      res["value_vs_rayleigh_quotient"] <= TOL_EIG[prec])
        return res

    def run_path(prec, proj="exact"):
        # 1. accuracy run: the first updates from the state's initial pairs, each result
        #    read back for the oracle replay (untimed)
        acc_start, acc_outs = None, []
        if not args.no_cpu_baseline and args.oracle_steps > 0:
            st, acc_start = make_state(prec, proj)
            for s in dev_steps[:args.oracle_steps]:
                st.update(s[0], s[1], s[2], s[3], s[4])
                st.sync()
                acc_outs.append(st.get())
            st.close()
        # 2. warm-up on its own state (same trajectory); its updates carry every stage's
        #    timing events, the timed ones only the two around the sparse product (each
        #    event between two kernels costs a few microseconds)
        st, _ = make_state(prec, proj)
        st.profile(True)
        for s in dev_steps[:args.warmup]:
            st.update(s[0], s[1], s[2], s[3], s[4])
        st.sync()
        stages, _, stage_n, _ = st.stage_times()
        st.close()
        # 3. timed updates on a fresh state
        st, _ = make_state(prec, proj)
        init = init_stats[-1]
        st.profile(2)
        sizes = []
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for s in dev_steps[:args.steps]:
            st.update(s[0], s[1], s[2], s[3], s[4])
            n2, nnz, _, width = st.shape()
            sizes.append((n2, nnz, width))
        st.sync()
        torch.cuda.synchronize()
        te = time.perf_counter()
        _, spmm_ms, nupd, spmm_cols = st.stage_times()
        vals = st.values()
        dev_bytes = st.memory()
        checks = final_checks(st, prec, proj == "lowrank")
        st.close()
        elem = 8 if prec == "fp64" else 4
        # the product multiplies every column of Z, or only the new ones when the kept A X
        # is reused; the bytes follow the width actually multiplied
        width = spmm_cols / max(1, nupd)
        byts = sum(spmm_bytes(n2, nnz, width, elem) for n2, nnz, _ in sizes) if width > 0 else 0.0
        return {"seconds": te - ts, "stages_ms": stages, "stage_updates": stage_n, "spmm_ms": spmm_ms, "updates": nupd,
                "spmm_bytes": byts, "spmm_width": width, "sizes": sizes, "lambda1": float(vals[0]),
                "state_gib": dev_bytes / 2**30, "final": checks, "acc_start": acc_start, "acc_outs": acc_outs,
                "init": init}

    log(args, f"timing {args.precision} path: warmup {args.warmup}, steps {args.steps}")
    main_res = run_path(args.precision)
    cmp_res = None
    if args.compare and args.compare != args.precision:
        log(args, f"timing {args.compare} path")
        cmp_res = run_path(args.compare)
    lr_res = None
    if not args.no_lowrank:
        log(args, f"timing the {args.precision} path with the low-rank projected matrix")
        lr_res = run_path(args.precision, "lowrank")

    # the same headline updates with the change lists and test matrices handed over from
    # host memory (pageable NumPy arrays): the copies over PCIe are then inside the timed
    # region; reported beside the headline, never as it
    host_res = None
    if not args.no_host_inputs:
        log(args, "timing the headline path with host-resident inputs")
        host_steps = []
        for t, d in enumerate(wl.deltas[:args.steps]):
            om = W.omega(wl.cfg_id, 0, t + 1, d.n_new, L + P) if variant == "rsvd" and d.n_new > 0 else None
            host_steps.append((d.n_new, d.i.astype(np.int32), d.j.astype(np.int32), d.sign.astype(np.int8), om))
        st, _ = make_state(args.precision)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for s in host_steps:
            st.update(*s)
        st.sync()
        torch.cuda.synchronize()
        host_res = args.steps / (time.perf_counter() - ts)
        st.close()

    # oracle replays of the first updates of every timed path (accuracy gate + CPU baseline)
    replays = OracleReplays(wl, cfg, args.oracle_steps)
    cpu = None
    exact_oracle = None
    for name, res, proj, prec in (("headline", main_res, "exact", args.precision),
                                  ("compare", cmp_res, "exact", args.compare),
                                  ("lowrank", lr_res, "lowrank", args.precision)):
        if res is None:
            continue
        if res["acc_start"] is None:
            res["oracle"] = None
            continue
        log(args, f"oracle replay of the {name} path ({len(res['acc_outs'])} updates)")
        res["oracle"], ora = replays.replay(res["acc_start"], res["acc_outs"], proj, prec, args,
                                            exact_for_distance=exact_oracle if proj == "lowrank" else None)
        if name == "headline":
            exact_oracle = ora
    if replays.seconds:
        cpu = cpu_baseline(wl, cfg, args, replays, main_res["acc_start"])

    secs = main_res["seconds"]
    value = args.steps / secs
    stages = main_res["stages_ms"]
    dominant = max(stages, key=stages.get)
    spmm_avg_ms = main_res["spmm_ms"] / max(1, main_res["updates"])
    achieved = main_res["spmm_bytes"] / (main_res["spmm_ms"] * 1e-3) / 1e9 if main_res["spmm_ms"] > 0 else 0.0
    ceil_ms = gather_ceiling(main_res, K) if args.precision != "fp64" and spmm_avg_ms > 0 else None
    n0_main = wl.n0
    del wl, dev_steps, replays, exact_oracle
    serve = serving_leg(args) if args.serving_graphs > 0 else None

    def accuracy(res, prec):
        acc = dict(res["final"])
        acc["final_note"] = "properties of the timed state after all its updates"
        if res.get("oracle") is not None:
            acc["oracle_replay"] = res["oracle"]
            acc["gate_passed"] = bool(acc["gate_passed"] and res["oracle"]["gate_passed"])
        acc["tolerances"] = {"e_lambda": TOL_EIG[prec], "sine": TOL_SINE[prec], "orthonormality": TOL_ORTH[prec]}
        return acc

    out = {
        "metric": "eigen-updates/sec at n=1M,k=32 (mixed vs FP32) + p50/p99 latency @ accuracy",
        "value": round(value, 3),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * secs / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f32+bf16", "fp32": "f32", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": cfg["workload"], "name": args.config, "n0": n0_main, "k": K, "L": L, "P": P,
                   "variant": variant, "op": op, "precision": args.precision, "scale": args.scale,
                   "graph_stage_overlap": not args.no_overlap},
        "accuracy": accuracy(main_res, args.precision),
        "stages_ms_per_update": {k: round(v / max(1, main_res["stage_updates"]), 4) for k, v in stages.items()},
        "stages_note": "HIP events around every stage, from the untimed warm-up updates",
        "initial_pairs": {"method": "device Chebyshev-filtered block iteration with a residual stop",
                          "products": main_res["init"][0], "residual": main_res["init"][1],
                          "residual_note": "max_j ||M x_j - lambda_j x_j|| / max_j |lambda_j| of the timed state's "
                                           "initial pairs"},
        "dominant_stage": dominant,
        "roofline": {"kernel": "spmm (product with the updated operator)", "bound": "hbm",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.config, main_res["spmm_width"]) if args.scale == 1.0 else None,
                     "traffic_unit": "GB per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
                     "algorithmic_gb_per_launch": round(main_res["spmm_bytes"] / max(1, len(main_res["sizes"])) / 1e9, 4),
                     "avg_launch_ms": round(spmm_avg_ms, 4),
                     "width": round(main_res["spmm_width"], 2),
                     "gather_ceiling": None if ceil_ms is None else {
                         "avg_launch_ms": round(ceil_ms, 4),
                         "frac": round(ceil_ms / spmm_avg_ms, 3),
                         "note": "grest_calib_gather: the same count of whole-row gathers at the same widths, "
                                 "from uniformly random rows (column ids from a hash instead of memory); "
                                 "frac = its time / the product's"}},
    }
    if host_res is not None:
        out["host_inputs"] = {"value": round(host_res, 3), "unit": "updates/s",
                              "note": "the headline updates with change lists and test matrices in host memory, "
                                      "their copies to the device inside the timed region"}
    if cmp_res is not None:
        cv = args.steps / cmp_res["seconds"]
        out["compare"] = {"precision": args.compare, "value": round(cv, 3),
                          "ms_per_step": round(1e3 * cmp_res["seconds"] / args.steps, 3),
                          "speedup_of_headline": round(value / cv, 3),
                          "accuracy": accuracy(cmp_res, args.compare),
                          "stages_ms_per_update": {k: round(v / max(1, cmp_res["stage_updates"]), 4)
                                                   for k, v in cmp_res["stages_ms"].items()}}
    if lr_res is not None:
        lv = args.steps / lr_res["seconds"]
        out["lowrank"] = {"note": "same workload and precision, H = Z^T (Xbar Theta Xbar^T + Delta) Z (eq. "
                                  "RR_eigen_graph_upd_main3) instead of the product with the stored graph; "
                                  "the state releases its graph after the initial pairs and keeps Delta alone. "
                                  "Its gate is parity with the oracle's low-rank trajectory; its distance to the "
                                  "exact form (vs_exact_form) is the truncation and is not gated, so its "
                                  "throughput is not an equal-accuracy comparison with the headline",
                          "value": round(lv, 3), "ms_per_step": round(1e3 * lr_res["seconds"] / args.steps, 3),
                          "throughput_ratio_to_headline_unequal_accuracy": round(lv / value, 3),
                          "state_gib": round(lr_res["state_gib"], 3),
                          "accuracy": accuracy(lr_res, args.precision),
                          "headline_state_gib": round(main_res["state_gib"], 3),
                          "stages_ms_per_update": {k: round(v / max(1, lr_res["stage_updates"]), 4)
                                                   for k, v in lr_res["stages_ms"].items()}}
    if serve is not None:
        out["serving"] = serve
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def _serving_graph_job(job):
    from paper_2603_19439_amd import workloads as W
    g, per_graph = job
    return W.serving_graph(g, per_graph)


def serving_leg(args):
    """Update latency of many graphs served together: Poisson arrivals with uniform target
    graphs, each request one update of its graph (G-REST_RSVD, L = P = K), run by the
    library's server.  Latency = completion time - scheduled arrival time.  Accuracy on
    two probe graphs (the smallest): after all the requests they received, their graph
    equals the generator's, entry for entry, and the oracle replays every one of their
    updates from the same initial pairs (eigenvalue error, subspace sine, residual)."""
    import concurrent.futures as cf
    import multiprocessing as mp

    import numpy as np
    import scipy.sparse as sp
    import torch
    from paper_2603_19439_amd import grest as G
    from paper_2603_19439_amd import workloads as W

    rates = [float(x) for x in args.serving_rates.split(",")]
    counts = [int(x) for x in args.serving_requests.split(",")]
    ng = args.serving_graphs
    per_graph = int(np.ceil((sum(counts) + args.serving_burst) / ng * 1.5)) + 8
    t0 = time.time()
    workers = max(1, min(16, (os.cpu_count() or 1)))
    # spawned workers import only NumPy and the generators, never the GPU runtime
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        graphs = list(ex.map(_serving_graph_job, [(g, per_graph) for g in range(ng)], chunksize=4))
    log(args, f"serving: {ng} graphs generated in {time.time() - t0:.1f}s on {workers} processes "
              f"(n0 {min(g.workload.n0 for g in graphs)}..{max(g.workload.n0 for g in graphs)})")
    probes = sorted(range(ng), key=lambda g: graphs[g].workload.n0)[:2]
    states, starts = [], {}
    for g, sg in enumerate(graphs):
        wl = sg.workload
        n_fin = wl.n0 + sum(d.n_new for d in wl.deltas) + 1
        nnz = int(wl.col0.size + 2 * sum(d.n_changes for d in wl.deltas) + 1024)
        st = G.State(wl.rowptr0, wl.col0, k=sg.k, variant="rsvd", op="adj", precision=args.precision, L=sg.k,
                     P=sg.k, node_capacity=n_fin, nnz_capacity=nnz)
        st.init_pairs(iterations=20, seed=g)
        if g in probes:
            starts[g] = st.get()
        states.append(st)
    torch.cuda.synchronize()
    mem = [st.memory() for st in states]
    sv = G.Server(lanes=args.serving_lanes, max_queue=1 << 16, batch=args.serving_batch)
    ids = [sv.attach(st) for st in states]
    nxt = [0] * ng
    results = []
    for seg, (rate, count) in enumerate(zip(rates, counts)):
        t_arr, tgt = W.arrivals(rate, count, ng, seed=seg)
        reqs = []
        for q in range(count):
            g = int(tgt[q])
            for _ in range(ng):  # a graph whose requests are used up passes to the next one
                if nxt[g] < per_graph:
                    break
                g = (g + 1) % ng
            d = graphs[g].workload.deltas[nxt[g]]
            om = W.omega(4, g, nxt[g] + 1, d.n_new, 2 * graphs[g].k) if d.n_new > 0 else None
            reqs.append((g, d.n_new, d.i.astype(np.int32), d.j.astype(np.int32), d.sign, om))
            nxt[g] += 1
        start = G.now_ns() + 20_000_000
        arr_ns = start + (t_arr * 1e9).astype(np.int64)
        retries = 0
        for q, (g, s_new, i, j, sg_, om) in enumerate(reqs):
            wait = (arr_ns[q] - G.now_ns()) / 1e9
            if wait > 2e-4:
                time.sleep(wait - 2e-4)
            while G.now_ns() < arr_ns[q]:
                pass
            while True:
                rc = sv.submit(ids[g], s_new, i, j, sg_, om, tag=q)
                if rc != G.EAGAIN:
                    break
                retries += 1
                time.sleep(1e-4)
            if rc != G.OK:
                raise RuntimeError(f"serving: request {q} (graph {g}) refused with status {rc}")
        sv.drain()
        tags, status, ts, td = sv.poll(count + 16)
        if tags.size != count or np.any(status != G.OK):
            bad = [(int(t), reqs[int(t)][0], int(st_)) for t, st_ in zip(tags, status) if st_ != G.OK]
            raise RuntimeError(f"serving: {tags.size}/{count} completions; failed (tag, graph, status): {bad[:20]}")
        lat_ms = (td - arr_ns[tags.astype(np.int64)]) / 1e6
        makespan = (td.max() - start) / 1e9
        results.append({"rate_req_s": rate, "requests": count, "p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
                        "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
                        "mean_ms": round(float(lat_ms.mean()), 3),
                        "throughput_req_s": round(count / makespan, 1), "queue_full_retries": retries})
        log(args, f"serving at {rate:g} req/s: p50 {results[-1]['p50_ms']} ms, p99 {results[-1]['p99_ms']} ms, "
                  f"throughput {results[-1]['throughput_req_s']} req/s")
    # saturation: a burst of requests (all due at once) on the served path, against the same
    # requests run one after another on plain FP32 per-graph states
    burst = []
    for q in range(args.serving_burst):
        g = q % ng
        if nxt[g] >= per_graph:
            continue
        d = graphs[g].workload.deltas[nxt[g]]
        om = W.omega(4, g, nxt[g] + 1, d.n_new, 2 * graphs[g].k) if d.n_new > 0 else None
        burst.append((g, d.n_new, d.i.astype(np.int32), d.j.astype(np.int32), d.sign, om))
        nxt[g] += 1
    sat = None
    if burst:
        t0_ns = G.now_ns()
        for q, (g, s_new, i, j, sg_, om) in enumerate(burst):
            rc = sv.submit(ids[g], s_new, i, j, sg_, om, tag=q)
            if rc != G.OK:
                raise RuntimeError(f"serving burst: request {q} refused with status {rc}")
        sv.drain()
        tags, status, ts, td = sv.poll(len(burst) + 16)
        if tags.size != len(burst) or np.any(status != G.OK):
            raise RuntimeError("serving burst: missing or failed completions")
        served = len(burst) / ((td.max() - t0_ns) / 1e9)
        sv.close()
        # plain path: FP32 states of the same graphs (from their initial graphs, with the
        # same number of requests each, taken from the start of their streams), each
        # request an update and a wait
        plain_states = {}
        plain_reqs = []
        for (g, *_rest) in burst:
            if g not in plain_states:
                wl = graphs[g].workload
                n_fin = wl.n0 + sum(d.n_new for d in wl.deltas) + 1
                nnz = int(wl.col0.size + 2 * sum(d.n_changes for d in wl.deltas) + 1024)
                ps = G.State(wl.rowptr0, wl.col0, k=graphs[g].k, variant="rsvd", op="adj", precision="fp32",
                             L=graphs[g].k, P=graphs[g].k, node_capacity=n_fin, nnz_capacity=nnz)
                ps.init_pairs(iterations=20, seed=g)
                plain_states[g] = [ps, 0]
            t = plain_states[g][1]
            d = graphs[g].workload.deltas[t]
            om = W.omega(4, g, t + 1, d.n_new, 2 * graphs[g].k) if d.n_new > 0 else None
            plain_reqs.append((g, d, om))
            plain_states[g][1] += 1
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for g, d, om in plain_reqs:
            plain_states[g][0].update_delta(d, om)
            plain_states[g][0].sync()
        plain = len(plain_reqs) / (time.perf_counter() - tp)
        for ps, _ in plain_states.values():
            ps.close()
        sat = {"requests": len(burst), "served_req_s": round(served, 1), "plain_fp32_per_graph_req_s": round(plain, 1),
               "speedup": round(served / plain, 2)}
        log(args, f"serving burst of {len(burst)}: {served:.0f} req/s served ({args.precision}, "
                  f"{args.serving_lanes} lanes, batches of up to {args.serving_batch}) vs {plain:.0f} req/s plain "
                  f"FP32 per graph")
    else:
        sv.close()
    # accuracy of the probe graphs: graph, and the oracle's replay of all their updates
    from oracle import grest_oracle as O
    tol = TOL_EIG[args.precision]
    acc = []
    for g in probes:
        wl, k = graphs[g].workload, graphs[g].k
        vals0, X0 = starts[g]
        A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
        X, th, r = X0, vals0, None
        for t, d in enumerate(wl.deltas[:nxt[g]]):
            om = W.omega(4, g, t + 1, d.n_new, 2 * k) if d.n_new > 0 else None
            r = O.grest_step(A, X, th, d.n_new, d.i, d.j, d.sign, k, variant=O.RSVD, L=k, Omega=om)
            A, X, th = r.A, r.X, r.theta
        if r is None:
            continue
        rp_g, col_g = states[g].graph()
        vals, Xg = states[g].get()
        c = compare_step(vals, Xg, r, "adj", k, A, matrix_norm(A))
        c.update({"graph": g, "n0": wl.n0, "k": k, "updates": nxt[g],
                  "graph_exact": bool(np.array_equal(rp_g, A.indptr) and np.array_equal(col_g, A.indices))})
        acc.append(c)
        log(args, f"serving probe {g}: {nxt[g]} updates, e_lambda {c['e_lambda']:.2e}, sine {c['sine']:.2e}")
    for st in states:
        st.close()
    passed = all(a["graph_exact"] and a["orthonormality"] <= TOL_ORTH[args.precision]
                 and a["e_lambda"] <= tol and a["sine"] <= TOL_SINE[args.precision] for a in acc)
    return {"workload": f"{ng} graphs (SBM or Chung-Lu, n0 {min(g.workload.n0 for g in graphs)}.."
                        f"{max(g.workload.n0 for g in graphs)}, mean degree 8-32, K in {{8,16,32}}, "
                        f"G-REST_RSVD L=P=K), requests of 0.1-1 % new nodes + 0.1-1 % insertions",
            "lanes": args.serving_lanes, "batch": args.serving_batch, "precision": args.precision,
            "device_gib_of_states": round(sum(mem) / 2**30, 2), "rates": results, "saturation": sat,
            "accuracy_probes": acc, "accuracy_gate_passed": passed}


def cpu_baseline(wl, cfg, args, replays, start):
    """The FP64 oracle's speed on this host: the accuracy replay of the headline path (the
    first updates of the same workload from the same initial pairs, with the host's BLAS
    threads), and one update of it again limited to one thread."""
    from oracle import grest_oracle as O
    from paper_2603_19439_amd import workloads as W
    model, logical = cpu_info()
    dt, steps = replays.seconds[0]
    out = {"value": round(steps / dt, 5), "unit": "updates/s", "cores": int(blas_threads()), "kind": "oracle",
           "cpu_model": model, "logical_cpus": logical,
           "sample": f"the first {steps} updates of the same workload from the headline state's initial pairs, "
                     f"n0={wl.n0}, FP64 NumPy/SciPy, {dt:.1f} s (the accuracy replay)"}
    try:
        import threadpoolctl
        vals0, X0 = start
        op = cfg["op"]
        A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
        th = vals0
        if op != "adj":
            _, shift0 = O.operator_matrix(A, op)
            th = shift0 - vals0
        d = wl.deltas[0]
        om = W.omega(wl.cfg_id, 0, 1, d.n_new, cfg["L"] + cfg["P"]) \
            if cfg["variant"] == "rsvd" and d.n_new > 0 else None
        with threadpoolctl.threadpool_limits(limits=1):
            t = time.perf_counter()
            O.grest_step(A, X0, th, d.n_new, d.i, d.j, d.sign, cfg["k"], variant=cfg["variant"], op=op,
                         L=cfg["L"] or None, Omega=om)
            dt1 = time.perf_counter() - t
        out["single_core"] = {"value": round(1.0 / dt1, 5), "unit": "updates/s", "cores": 1,
                              "sample": f"the first update again with one BLAS thread, {dt1:.1f} s"}
        log(args, f"oracle: {steps / dt:.4f} updates/s on {out['cores']} threads, {1.0 / dt1:.4f} on one")
    except Exception as e:  # threadpoolctl missing: the all-core figure stands alone
        out["single_core"] = {"error": str(e)}
    return out


def kernel_source_sha1(csrc):
    """Short hash of the product kernel's source: spmm.hip and the row-slice helpers it
    includes (rowvec.h)."""
    import hashlib
    h = hashlib.sha1()
    for name in ("spmm.hip", "rowvec.h"):
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:12]


def measured_traffic(config, width):
    """HBM bytes per launch of the product kernel at this workload, from the committed
    byte-counter summary: measured at two widths and linear in the width in between (a
    fixed part for the graph, a per-column part for the gathered rows), so the mean width
    of the timed updates picks its point on that line.  None when there is no summary for
    the configuration, the kernel source changed since the counters were taken or the
    width lies outside the measured range."""
    names = {"c3": "spmm_traffic_sbm_n1e6_k32.txt"}
    if config not in names:
        return None
    path = os.path.join(ROOT, "profiles", names[config])
    csrc = os.path.join(ROOT, "paper_2603_19439_amd", "csrc")
    try:
        rec = {}
        for line in open(path):
            if "=" in line and not line.startswith(" "):
                k, v = line.split("=", 1)
                rec[k.strip()] = v.split()[0]
        cur = kernel_source_sha1(csrc)
        if rec.get("kernel_source_sha1") != cur:
            return None
        pts = sorted((float(w), float(t)) for w, t in (p.split(":") for p in rec["traffic_points"].split(",")))
        (w0, t0), (w1, t1) = pts[0], pts[-1]
        if not (w0 - 0.5 <= width <= w1 + 0.5):
            return None
        if w1 == w0:
            return t0
        return round(t0 + (t1 - t0) * (width - w0) / (w1 - w0), 4)
    except (OSError, KeyError, ValueError, IndexError):
        return None


if __name__ == "__main__":
    main()
