#!/usr/bin/env python3
"""Throughput of the G-REST eigenpair update on one MI355X.

Workload: stochastic block model with n0 = 1,000,000 nodes, 32 blocks with
Dirichlet(2) sizes, mean degree 20 (80 % intra-block), adjacency operator,
K = 32 tracked pairs, G-REST_RSVD with L = P = 32 (subspace width 3K = 96);
every step appends 10,000 nodes and about 50,000 edges.  Data are synthetic
(seeded generator); the initial pairs come from the library's device subspace
iteration.  The change lists and Gaussian test matrices are uploaded to HBM
before the timed region, which contains exactly ``--steps`` updates bracketed by
device synchronisations.

Printed JSON line: the headline updates/s of the mixed-precision path, the plain
FP32 path and the truncated low-rank form beside it, each with its accuracy gate
(graph, Rayleigh quotients, orthonormality after the timed updates), per-stage times,
the roofline of the dominant kernel measured with HIP events around it, the serving
latencies of many graphs, and the FP64 CPU oracle timed on the first updates of the
same workload (``cpu_baseline``, the only part that runs the oracle).
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
K, L, P = 32, 32, 32


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp32", "fp64"])
    ap.add_argument("--compare", default="fp32", help="second path timed beside the headline ('' to skip)")
    ap.add_argument("--no-lowrank", action="store_true",
                    help="skip timing the low-rank projected matrix (eq. ..._main3) beside the headline")
    ap.add_argument("--scale", type=float, default=1.0, help="shrink node counts (quick runs only)")
    ap.add_argument("--init-iters", type=int, default=40)
    ap.add_argument("--no-overlap", action="store_true",
                    help="run each update's graph stage on the state's stream (no second stream)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-graphs", type=int, default=32,
                    help="graphs in the many-graph serving leg (0 skips it; the full mix has 256)")
    ap.add_argument("--serving-rates", default="100,400", help="Poisson arrival rates, requests/s")
    ap.add_argument("--serving-requests", default="300,800", help="requests per rate")
    ap.add_argument("--serving-lanes", type=int, default=8)
    ap.add_argument("--serving-burst", type=int, default=256,
                    help="requests of the saturation burst (served path vs plain FP32 per-graph path)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a reference kernel of "
                         "known traffic for hardware byte counters)")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


def log(args, *msg):
    if not args.quiet:
        print("[bench]", *msg, file=sys.stderr, flush=True)


def spmm_bytes(n2: int, nnz: int, width: int, elem: int) -> float:
    """Algorithmic bytes of one product with the updated operator: column ids (4 B per
    stored entry), row offsets (8 B per row), the basis read once and the product
    written once (n' x width elements each)."""
    return 4.0 * nnz + 8.0 * (n2 + 1) + 2.0 * elem * n2 * width


def main():
    args = parse()
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
    n_steps = max(16, args.steps, args.warmup)
    t0 = time.time()
    wl = W.preset("sbm_n1e6", scale=args.scale, steps=n_steps)
    log(args, f"workload generated in {time.time() - t0:.1f}s: n0={wl.n0} nnz={wl.col0.size}")
    # device-resident inputs
    dev_steps = []
    for t, d in enumerate(wl.deltas):
        om = W.omega(wl.cfg_id, 0, t + 1, d.n_new, L + P) if d.n_new > 0 else None
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
        st = G.State(wl.rowptr0, wl.col0, k=K, variant="rsvd", op="adj", precision=prec, L=L, P=P,
                     stream=torch.cuda.current_stream().cuda_stream, node_capacity=n_final + 1,
                     nnz_capacity=nnz_cap, proj=proj)
        st.init_pairs(iterations=args.init_iters, seed=7)
        if proj == "lowrank":  # the low-rank form needs Delta and the pairs only
            st.release_graph()
        st.set_overlap(not args.no_overlap)
        return st

    final_graph = {}

    def accuracy(st, prec, lowrank):
        """Accuracy gate of a timed state after its updates, with properties that hold for
        any Rayleigh-Ritz output (the exact pairs of this graph are out of the oracle's
        reach): its graph equals the one the seeded generator reaches, every returned value
        is the Rayleigh quotient of its returned vector on that graph (Alg. 1) to the
        precision's eigenvalue tolerance, and the block is orthonormal.  The low-rank state
        has released its graph, and its values are Ritz values of the truncated operator
        (eq. RR_eigen_graph_upd_main3), not of the graph: for it the distance to the graph's
        quotients measures the truncation and is reported, and the gate is orthonormality."""
        import scipy.sparse as sp
        if not final_graph:
            n_t = wl.n_at(args.steps)
            rp, col = W.csr_from_keys(n_t, wl.keys_at(args.steps))
            final_graph.update(rp=rp, col=col, A=sp.csr_matrix(
                (np.ones(col.size), col.astype(np.int64), rp.astype(np.int64)), shape=(n_t, n_t)))
        fg = final_graph
        vals, X = st.get()
        res = {}
        if not lowrank:
            rp_g, col_g = st.graph()
            res["graph_exact"] = bool(np.array_equal(rp_g, fg["rp"]) and np.array_equal(col_g, fg["col"]))
        k = X.shape[1]
        res["orthonormality"] = float(np.abs(X.T @ X - np.eye(k)).max())
        rq = ((fg["A"] @ X) * X).sum(axis=0)
        res["value_vs_rayleigh_quotient"] = float(
            (np.abs(vals - rq) / np.maximum(np.abs(rq), 1e-8 * np.abs(rq).max())).max())
        tol = {"fp64": 1e-10, "fp32": 1e-5, "mixed": 1e-3}[prec]
        orth_ok = res["orthonormality"] <= (1e-12 if prec == "fp64" else 1e-5)
        if lowrank:
            res["note"] = "values are Ritz values of the truncated operator; their distance to the graph's " \
                          "Rayleigh quotients is the truncation, not part of the gate"
            res["gate_passed"] = bool(orth_ok)
        else:
            res["gate_passed"] = bool(res["graph_exact"] and orth_ok and res["value_vs_rayleigh_quotient"] <= tol)
        return res

    def run_path(prec, proj="exact"):
        # warmup on its own state (same trajectory), then a fresh state for the timed steps
        # the warm-up updates carry every stage's timing events; the timed ones only the two
        # around the sparse product (each event between two kernels costs a few microseconds)
        st = make_state(prec, proj)
        st.profile(True)
        for s in dev_steps[:args.warmup]:
            st.update(s[0], s[1], s[2], s[3], s[4])
        st.sync()
        stages, _, stage_n, _ = st.stage_times()
        st.close()
        st = make_state(prec, proj)
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
        acc = accuracy(st, prec, proj == "lowrank")
        st.close()
        elem = 8 if prec == "fp64" else 4
        # the product multiplies every column of Z, or only the new ones when the kept A X
        # is reused; the bytes follow the width actually multiplied
        width = spmm_cols / max(1, nupd)
        byts = sum(spmm_bytes(n2, nnz, width, elem) for n2, nnz, _ in sizes) if width > 0 else 0.0
        return {"seconds": te - ts, "stages_ms": stages, "stage_updates": stage_n, "spmm_ms": spmm_ms, "updates": nupd,
                "spmm_bytes": byts, "spmm_width": width, "sizes": sizes, "lambda1": float(vals[0]),
                "state_gib": dev_bytes / 2**30, "accuracy": acc}

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

    secs = main_res["seconds"]
    value = args.steps / secs
    stages = main_res["stages_ms"]
    dominant = max(stages, key=stages.get)
    spmm_avg_ms = main_res["spmm_ms"] / max(1, main_res["updates"])
    achieved = main_res["spmm_bytes"] / (main_res["spmm_ms"] * 1e-3) / 1e9 if main_res["spmm_ms"] > 0 else 0.0

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, args)
    n0_main = wl.n0
    del wl, dev_steps
    serve = serving_leg(args) if args.serving_graphs > 0 else None

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
        "config": {"workload": "SBM n0=1e6, 32 Dirichlet(2) blocks, mean degree 20, +10k nodes/+50k edges "
                               "per step; adjacency, k=32, G-REST_RSVD L=P=32 (width 96)",
                   "n0": n0_main, "k": K, "L": L, "P": P, "variant": "rsvd", "precision": args.precision,
                   "scale": args.scale, "graph_stage_overlap": not args.no_overlap},
        "accuracy": main_res["accuracy"],
        "stages_ms_per_update": {k: round(v / max(1, main_res["stage_updates"]), 4) for k, v in stages.items()},
        "stages_note": "HIP events around every stage, from the untimed warm-up updates",
        "dominant_stage": dominant,
        "roofline": {"kernel": "spmm (product with the updated operator)", "bound": "hbm",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(main_res["spmm_width"]),
                     "traffic_unit": "GB per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
                     "algorithmic_gb_per_launch": round(main_res["spmm_bytes"] / max(1, len(main_res["sizes"])) / 1e9, 4),
                     "avg_launch_ms": round(spmm_avg_ms, 4),
                     "width": round(main_res["spmm_width"], 2)},
    }
    if cmp_res is not None:
        cv = args.steps / cmp_res["seconds"]
        out["compare"] = {"precision": args.compare, "value": round(cv, 3),
                          "ms_per_step": round(1e3 * cmp_res["seconds"] / args.steps, 3),
                          "speedup_of_headline": round(value / cv, 3),
                          "accuracy": cmp_res["accuracy"],
                          "stages_ms_per_update": {k: round(v / max(1, cmp_res["stage_updates"]), 4)
                                                   for k, v in cmp_res["stages_ms"].items()}}
    if lr_res is not None:
        lv = args.steps / lr_res["seconds"]
        out["lowrank"] = {"note": "same workload and precision, H = Z^T (Xbar Theta Xbar^T + Delta) Z (eq. "
                                  "RR_eigen_graph_upd_main3) instead of the product with the stored graph; "
                                  "the state releases its graph after the initial pairs and keeps Delta alone",
                          "value": round(lv, 3), "ms_per_step": round(1e3 * lr_res["seconds"] / args.steps, 3),
                          "speedup_of_headline": round(lv / value, 3),
                          "state_gib": round(lr_res["state_gib"], 3),
                          "accuracy": lr_res["accuracy"],
                          "headline_state_gib": round(main_res["state_gib"], 3),
                          "stages_ms_per_update": {k: round(v / max(1, lr_res["stage_updates"]), 4)
                                                   for k, v in lr_res["stages_ms"].items()}}
    if serve is not None:
        out["serving"] = serve
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def serving_leg(args):
    """Update latency of many graphs served together: Poisson arrivals with uniform target
    graphs, each request one update of its graph (G-REST_RSVD, L = P = K), run by the
    library's server.  Latency = completion time - scheduled arrival time.  Accuracy gate
    on two probe graphs (the smallest), after all the requests they received: their graph
    equals the generator's, entry for entry; every returned value is the Rayleigh quotient
    of its returned vector on that graph (Ritz values are Rayleigh quotients of Ritz
    vectors, Alg. 1) to the precision's eigenvalue tolerance; the block is orthonormal."""
    import numpy as np
    import scipy.sparse as sp
    import torch
    from paper_2603_19439_amd import grest as G
    from paper_2603_19439_amd import workloads as W

    rates = [float(x) for x in args.serving_rates.split(",")]
    counts = [int(x) for x in args.serving_requests.split(",")]
    ng = args.serving_graphs
    per_graph = int(np.ceil((sum(counts) + args.serving_burst) / ng * 1.6)) + 8
    t0 = time.time()
    graphs = [W.serving_graph(g, per_graph) for g in range(ng)]
    log(args, f"serving: {ng} graphs generated in {time.time() - t0:.1f}s "
              f"(n0 {min(g.workload.n0 for g in graphs)}..{max(g.workload.n0 for g in graphs)})")
    probes = sorted(range(ng), key=lambda g: graphs[g].workload.n0)[:2]
    states = []
    for g, sg in enumerate(graphs):
        wl = sg.workload
        n_fin = wl.n0 + sum(d.n_new for d in wl.deltas) + 1
        nnz = int(wl.col0.size + 2 * sum(d.n_changes for d in wl.deltas) + 1024)
        st = G.State(wl.rowptr0, wl.col0, k=sg.k, variant="rsvd", op="adj", precision=args.precision, L=sg.k,
                     P=sg.k, node_capacity=n_fin, nnz_capacity=nnz)
        st.init_pairs(iterations=20, seed=g)
        states.append(st)
    torch.cuda.synchronize()
    sv = G.Server(lanes=args.serving_lanes, max_queue=1 << 16)
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
        log(args, f"serving at {rate:g} req/s: p50 {results[-1]['p50_ms']} ms, p99 {results[-1]['p99_ms']} ms")
    # saturation: a burst of requests (all due at once) on the served path, against the same
    # number of requests run one after another on plain FP32 per-graph states
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
        # plain path: FP32 states of the same graphs, each request an update and a wait
        plain_states = []
        for g in range(ng):
            wl = graphs[g].workload
            n_fin = wl.n0 + sum(d.n_new for d in wl.deltas) + 1
            nnz = int(wl.col0.size + 2 * sum(d.n_changes for d in wl.deltas) + 1024)
            ps = G.State(wl.rowptr0, wl.col0, k=graphs[g].k, variant="rsvd", op="adj", precision="fp32",
                         L=graphs[g].k, P=graphs[g].k, node_capacity=n_fin, nnz_capacity=nnz)
            ps.init_pairs(iterations=20, seed=g)
            plain_states.append(ps)
        pn = [0] * ng
        plain_reqs = []
        for (g, *_rest) in burst:
            d = graphs[g].workload.deltas[pn[g]]
            om = W.omega(4, g, pn[g] + 1, d.n_new, 2 * graphs[g].k) if d.n_new > 0 else None
            plain_reqs.append((g, d, om))
            pn[g] += 1
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for g, d, om in plain_reqs:
            plain_states[g].update_delta(d, om)
            plain_states[g].sync()
        plain = len(plain_reqs) / (time.perf_counter() - tp)
        for ps in plain_states:
            ps.close()
        sat = {"requests": len(burst), "served_req_s": round(served, 1), "plain_fp32_per_graph_req_s": round(plain, 1),
               "speedup": round(served / plain, 2)}
        log(args, f"serving burst of {len(burst)}: {served:.0f} req/s served ({args.precision}, "
                  f"{args.serving_lanes} lanes) vs {plain:.0f} req/s plain FP32 per graph")
    sv.close()
    # accuracy of the probe graphs after all the requests they received
    tol = {"fp64": 1e-10, "fp32": 1e-5, "mixed": 1e-3}[args.precision]
    acc = []
    for g in probes:
        wl, k = graphs[g].workload, graphs[g].k
        n_t = wl.n_at(nxt[g])
        rp, col = W.csr_from_keys(n_t, wl.keys_at(nxt[g]))
        rp_g, col_g = states[g].graph()
        A = sp.csr_matrix((np.ones(col.size), col.astype(np.int64), rp.astype(np.int64)), shape=(n_t, n_t))
        vals, Xg = states[g].get()
        orth = float(np.abs(Xg.T @ Xg - np.eye(k)).max())
        rq = ((A @ Xg) * Xg).sum(axis=0)
        rq_rel = float((np.abs(vals - rq) / np.maximum(np.abs(rq), 1e-8 * np.abs(rq).max())).max())
        acc.append({"graph": g, "n0": wl.n0, "k": k, "updates": nxt[g],
                    "graph_exact": bool(np.array_equal(rp_g, rp) and np.array_equal(col_g, col)),
                    "orthonormality": orth, "value_vs_rayleigh_quotient": rq_rel})
    for st in states:
        st.close()
    passed = all(a["graph_exact"] and a["orthonormality"] <= (1e-12 if args.precision == "fp64" else 1e-5)
                 and a["value_vs_rayleigh_quotient"] <= tol for a in acc)
    return {"workload": f"{ng} graphs (SBM or Chung-Lu, n0 {min(g.workload.n0 for g in graphs)}.."
                        f"{max(g.workload.n0 for g in graphs)}, mean degree 8-32, K in {{8,16,32}}, "
                        f"G-REST_RSVD L=P=K), requests of 0.1-1 % new nodes + 0.1-1 % insertions",
            "lanes": args.serving_lanes, "precision": args.precision, "rates": results, "saturation": sat,
            "accuracy_probes": acc, "accuracy_gate_passed": passed}


def cpu_baseline(wl, args):
    """The FP64 oracle on one update of the same workload (random orthonormal start, same
    change list and test matrix), timed on this host's cores."""
    import numpy as np
    from oracle import grest_oracle as O
    from paper_2603_19439_amd import workloads as W
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max((i.get("num_threads") or 1) for i in info) if info else os.cpu_count()
    except Exception:
        cores = os.cpu_count()
    A = O.adjacency_from_csr(wl.rowptr0, wl.col0)
    X = W.random_orthonormal(wl.n0, K, 0)
    theta = np.zeros(K)
    steps = 2
    log(args, f"timing the CPU oracle on {steps} updates")
    t = time.perf_counter()
    for s in range(steps):
        d = wl.deltas[s]
        om = W.omega(wl.cfg_id, 0, s + 1, d.n_new, L + P)
        r = O.grest_step(A, X, theta, d.n_new, d.i, d.j, d.sign, K, variant=O.RSVD, L=L, Omega=om)
        A, X, theta = r.A, r.X, r.theta
    dt = time.perf_counter() - t
    return {"value": round(steps / dt, 5), "unit": "updates/s", "cores": int(cores), "kind": "oracle",
            "sample": f"the first {steps} updates of the same workload from a random orthonormal start, "
                      f"n0={wl.n0}, FP64 NumPy/SciPy, {dt:.1f} s"}


def measured_traffic(width):
    """HBM bytes per launch of the product kernel at this workload, from the committed
    byte-counter summary: measured at the 64-column (kept A X) and 96-column (full) widths,
    and linear in the width in between (a fixed part for the graph, a per-column part for
    the gathered rows), so the mean width of the timed updates picks its point on that
    line.  None when the kernel source changed since the counters were taken or the width
    lies outside the measured range."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "spmm_traffic_sbm_n1e6_k32.txt")
    src = os.path.join(ROOT, "paper_2603_19439_amd", "csrc", "spmm.hip")
    try:
        rec = {}
        for line in open(path):
            if "=" in line and not line.startswith(" "):
                k, v = line.split("=", 1)
                rec[k.strip()] = v.split()[0]
        cur = hashlib.sha1(open(src, "rb").read()).hexdigest()[:12]
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
