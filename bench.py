#!/usr/bin/env python
"""Benchmark: exact k-NN pair evaluations per second, DK vs DTW+LB_Box.

One step = one exact k-NN batch under DK (greedy-bound seed, sparse-DK
semantics; unbanded) followed by one exact k-NN batch under DTW with LB_Box
(Sakoe-Chiba band 10 %), both over the same queries and database, inputs
resident in HBM.  value = (queries x series) / step time, i.e. pairs whose
exact k-NN membership was decided under both distances per second.

The default workload is the large one (4096 queries x 1 000 000 series,
L = 512, d = 6, 12.3 GB resident), scanned in the library's default
configuration; the learned candidate order (encoder trained first, untimed)
is timed beside it at identical rows.  Smaller workloads run with
--workload.

Prints one JSON line.  Also reports each distance's own rate, the DK/DTW
and learned/plain speed-ups, the roofline of the dominant kernel (device
time from HIP events recorded on the launch stream during the timed steps),
the CPU oracle's pruned scan timed on a bounded sample, and a check of the
GPU rows against the oracle at full size (a sample of queries against every
series, and every returned (id, distance) recomputed).
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

METRIC = "exact k-NN pair evals/sec (DK vs DTW+LB_Box); learned-order vs plain speedup"

# name -> workload (synthetic stand-ins for the paper's data sets)
WORKLOADS = {
    "classwarp-q100-n20000-L256-d3": dict(cfg_id=2, gen="classwarp", classes=10, Q=100, N=20000,
                                          L=256, d=3, k=10, dk_band=None, dtw_band=0.1),
    "randomwalk-q1-n1000-L64-d3": dict(cfg_id=1, gen="randomwalk", Q=1, N=1000, L=64, d=3, k=1,
                                       dk_band=None, dtw_band=None),
    # the large configuration: 200 classes, two independent 3-D tracks per series
    "classwarp-q4096-n1000000-L512-d6": dict(cfg_id=5, gen="classwarp", classes=200, Q=4096,
                                             N=1000000, L=512, d=6, k=10, dk_band=None,
                                             dtw_band=0.1, large=True),
    # uneven lengths: members of length U{64..1024} from 50 prototypes of length 1024
    "classwarp-q1024-n100000-L64to1024-d3": dict(cfg_id=3, gen="classwarp", classes=50, Q=1024,
                                                 N=100000, L=1024, lengths=(64, 1024), d=3,
                                                 k=10, dk_band=None, dtw_band=0.1),
}
DEFAULT = "classwarp-q4096-n1000000-L512-d6"
SECONDARY = "classwarp-q100-n20000-L256-d3"

# MI355X fp32 vector rate: 157.3 TFLOP/s with an FMA as two flops, i.e.
# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz x 2 lane-ops per cycle (the
# scan's non-packed VALU code issues above one op per lane-cycle: 46 T
# lane-instructions/s measured in the LB_Box kernel)
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9 * 2
HBM_PEAK_BPS = 8.0e12


def load_traffic(kernel, workload):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's reading), or
    None if there is none for this kernel and workload or the kernel sources
    changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get(f"{kernel}|{workload}")
    if not rec:
        return None
    h = hashlib.sha256()
    for name in rec["sources"]:
        with open(os.path.join(ROOT, name), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["bytes_per_launch"]


def make_data(w):
    from paper_1811_11076_amd import synth
    if w["gen"] == "randomwalk":
        db, dbo = synth.flat_equal(synth.random_walks(w["N"], w["L"], w["d"], w["cfg_id"], "db"))
        qs, qo = synth.flat_equal(synth.random_walks(w["Q"], w["L"], w["d"], w["cfg_id"], "query"))
    else:
        g = synth.ClassWarp(w["cfg_id"], w["classes"], w["L"], w["d"])
        length = w.get("lengths", w["L"])
        db, dbo, _ = g.members(w["N"], "db", length=length)
        qs, qo, _ = g.members(w["Q"], "query", length=length, class_mode="uniform")
    return db, dbo, qs, qo


def kernel_rooflines(prof, dist, d, fast_kernel, uneven=False, cascade=None):
    """Per-kernel device time and algorithmic work of one distance's
    profile, per launch: HIP events around each stage on its launch stream,
    summed over the profiled calls and divided by the launches (one per
    query chunk).  Work units: DP = in-band in-matrix cells of live pairs,
    2d+2 ops each; LB_Box = terms, 4d+1 ops each; corner bound = 2 point
    costs per pair (4d+1 ops); greedy seed = moves (~6d+4 ops).  cascade:
    the corner bound runs inside the seed stage (DK by default; DTW on
    equal lengths in the plain order by default), and DTW's LB_Box kernel is
    the survivors' one (k_bound_lb_surv)."""
    if cascade is None:
        cascade = dist == "dk" or not uneven
    n = max(1, prof["chunks"])
    cell_ops = 2 * d + 2
    fast_cells = prof["dp_valid_cells"] - prof["dp_valid_cells_general"]
    out = {
        fast_kernel: dict(ms=prof["ms_dp_fast"] / n, units=fast_cells / n, unit_ops=cell_ops),
        "k_dp_wave": dict(ms=prof["ms_dp_general"] / n,
                          units=prof["dp_valid_cells_general"] / n, unit_ops=cell_ops),
    }
    seed_name = ("seed stage (k_corner, k_compact_sorted, k_seed_ring)" if cascade
                 else ("k_seed_ring" if (uneven or dist == "dk") else "k_seed_diag"))
    out[seed_name] = dict(ms=prof["ms_seed"] / n, units=prof["seed_steps"] / n, unit_ops=6 * d + 4)
    if dist == "dtw":
        name = "k_bound_lbu" if uneven else ("k_bound_lb_surv" if cascade else "k_bound_lb")
        out[name] = dict(ms=prof["ms_bound_kernel"] / n, units=prof["bound_steps"] / n,
                         unit_ops=4 * d + 1)
    elif not cascade:
        out["k_corner"] = dict(ms=prof["ms_bound_kernel"] / n, units=prof["pairs"] / n,
                               unit_ops=4 * d + 1)
    for v in out.values():
        v["ops"] = v["units"] * v["unit_ops"]
        v["tops"] = v["ops"] / (v["ms"] * 1e-3) / 1e12 if v["ms"] > 0 else 0.0
    return out


def tuned_graph(w, args, idx_dk, idx_dtw, dev_q, qs, qo, eager_res):
    """Autotunes both distances on a query sample (untimed), then times the
    step as one captured HIP graph per distance with the tuned options;
    also times a sample of queries batched against one call per query."""
    import numpy as np
    import torch
    k, nq = w["k"], w["Q"]
    tuned = {}
    t0 = time.perf_counter()
    for name, idx, band in (("dk", idx_dk, w["dk_band"]), ("dtw", idx_dtw, w["dtw_band"])):
        best, ms = idx.tune(dev_q, qo, k, name, band, sample_queries=min(nq, 256), reps=3)
        tuned[name] = {"options": best, "sample_ms": ms}
    t_tune = time.perf_counter() - t0
    outs = {name: (torch.empty((nq, k), dtype=torch.int64, device="cuda"),
                   torch.empty((nq, k), dtype=torch.float32, device="cuda")) for name in ("dk", "dtw")}

    # the two distances' graphs run on two streams (default priority) at
    # once: each call's latency-bound stages overlap the other's
    # throughput-bound ones
    streams = (torch.cuda.Stream(), torch.cuda.Stream())
    torch.cuda.synchronize()

    def make_step(use_tuned):
        def step():
            with torch.cuda.stream(streams[0]):
                a = idx_dk.knn(dev_q, qo, k, "dk", w["dk_band"], use_graph=True, tune=use_tuned,
                               out=outs["dk"])
            with torch.cuda.stream(streams[1]):
                b = idx_dtw.knn(dev_q, qo, k, "dtw", w["dtw_band"], use_graph=True,
                                tune=use_tuned, out=outs["dtw"])
            return a, b
        return step

    # the options were tuned per distance alone; the step runs both at once,
    # so a short untimed trial of the concurrent step decides between the
    # tuned and the default options before the timed steps
    trial_ms = {}
    for use_tuned in (True, False):
        st = make_step(use_tuned)
        for _ in range(3):
            st()
        torch.cuda.synchronize()
        tt = time.perf_counter()
        for _ in range(10):
            st()
        torch.cuda.synchronize()
        trial_ms["tuned" if use_tuned else "default"] = (time.perf_counter() - tt) * 100.0
    chosen = min(trial_ms, key=trial_ms.get)
    step = make_step(chosen == "tuned")
    for _ in range(max(1, args.warmup)):
        res = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    same = all(torch.equal(x, y) for x, y in zip(res[0][:2] + res[1][:2],
                                                 eager_res[0][:2] + eager_res[1][:2]))
    print(f"[bench] tuned graph: {args.steps} steps in {el:.3f}s (tuning {t_tune:.1f}s)",
          file=sys.stderr, flush=True)
    # batched vs one call per query on a sample of queries
    S = min(nq, args.per_query_sample)
    sub_q = dev_q[:int(qo[S])]
    sub_o = qo[:S + 1]
    per = [(dev_q[int(qo[i]):int(qo[i + 1])], np.array([0, qo[i + 1] - qo[i]])) for i in range(S)]

    def batched():
        idx_dk.knn(sub_q, sub_o, k, "dk", w["dk_band"])
        idx_dtw.knn(sub_q, sub_o, k, "dtw", w["dtw_band"])

    def one_by_one():
        for qv, qoff in per:
            idx_dk.knn(qv, qoff, k, "dk", w["dk_band"])
            idx_dtw.knn(qv, qoff, k, "dtw", w["dtw_band"])

    times = {}
    for name, fn in (("batched", batched), ("per_query", one_by_one)):
        fn()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t2) / 3 * 1e3
    return {"ms_per_step": el * 1e3 / args.steps, "rows_equal_eager": bool(same),
            "tuned": tuned, "tuning_seconds": t_tune, "step_options": chosen,
            "trial_ms_per_step": trial_ms,
            "sample_queries": S, "batched_ms": times["batched"],
            "per_query_ms": times["per_query"],
            "batched_vs_per_query_speedup": times["per_query"] / times["batched"]}


def learned_order(w, args, db, dbo, dev_db, dev_q, qo, idx_dk, idx_dtw, plain_res):
    """Trains the encoder on DK distances of the train stream (untimed), then
    times the same step with each query's candidates in learned order and
    checks the rows equal the plain scan's."""
    import numpy as np
    import torch
    from paper_1811_11076_amd import Model, synth
    from paper_1811_11076_amd.learned import dk_training_set
    t0 = time.perf_counter()
    gen = synth.ClassWarp(w["cfg_id"], w["classes"], w["L"], w["d"])
    # 200k pairs: 500 anchors x (200 same-class + 200 random) of a 2000-series pool
    tv, to, ta, tb, ty = dk_training_set(gen, 2000, 500, 200, w.get("lengths", w["L"]), seed=1)
    model = Model(w["d"], seed=1)
    losses = model.train(torch.from_numpy(tv).cuda(), to, ta, tb, ty, epochs=10, batch=1024,
                         lr=1e-3, seed=1)
    t_train = time.perf_counter() - t0
    print(f"[bench] encoder trained on {ta.size} pairs in {t_train:.1f}s, loss "
          f"{losses[0]:.3f} -> {losses[-1]:.3f}", file=sys.stderr, flush=True)
    k = w["k"]

    # the encoder orders DK's candidates (the distance it is trained on);
    # DTW keeps the plain order (learned order measured 0.98-1.04x there)
    def step(profile):
        a = idx_dk.knn(dev_q, qo, k, "dk", w["dk_band"], profile=profile, order="learned",
                       model=model)
        b = idx_dtw.knn(dev_q, qo, k, "dtw", w["dtw_band"], profile=profile)
        return a, b

    for _ in range(args.warmup):
        res = step(False)
    torch.cuda.synchronize()
    idx_dk.profile(reset=True)
    idx_dtw.profile(reset=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        res = step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    pdk = idx_dk.profile(reset=True)
    pdtw = idx_dtw.profile(reset=True)
    same = all(torch.equal(x, y) for x, y in zip(res[0][:2] + res[1][:2],
                                                 plain_res[0][:2] + plain_res[1][:2]))
    pairs = w["Q"] * w["N"]
    calls = max(1, pdk["calls"])
    controls = None
    if pairs <= 10_000_000:
        controls = order_controls(w, idx_dk, dev_q, qo, model, plain_res[0], pdk)
    model.close()
    return {"ms_per_step": elapsed * 1e3 / args.steps,
            "pairs_per_s": pairs / (elapsed / args.steps),
            "rows_equal_plain": bool(same),
            "train": {"pairs": int(ta.size), "epochs": 10, "batch": 1024, "seconds": t_train,
                      "loss_first_epoch": float(losses[0]), "loss_last_epoch": float(losses[-1])},
            "dk": {"device_ms": pdk["ms_total"] / calls, "order_ms": pdk["ms_order"] / calls,
                   "dp_completed": pdk["dp_completed"] / calls,
                   "dp_valid_cells": pdk["dp_valid_cells"] / calls},
            "dtw": {"device_ms": pdtw["ms_total"] / max(1, pdtw["calls"]), "order": "plain"},
            "dk_fraction_full_dps": pdk["dp_completed"] / calls / pairs,
            "dk_controls": controls}


def order_controls(w, idx_dk, dev_q, qo, model, plain_dk, learned_prof, reps=3):
    """DK work under the order and seeding controls: the plain order with
    Alg. 1 over every candidate (the paper's own first pass), the learned
    order with that full seed, the learned order with the library's top-M
    seed (its first 512 candidates), the plain order with the top-M seed
    (the 512 candidates of smallest corner bound, the library default), the
    plain order with the first 512 candidates as the seed set, and an
    untrained (random-init) encoder with the top-M seed.  Each row
    gives the fraction of (query, series) pairs whose DP ran to
    completion, DPs started, DP cells and device time per call; every
    control's rows must equal the plain scan's."""
    import torch
    from paper_1811_11076_amd import Model
    pairs = w["Q"] * w["N"]
    k = w["k"]
    untrained = Model(w["d"], seed=2)
    full = {"seed_count": w["N"]}
    runs = [("plain_full_seed", full),
            ("learned_full_seed", dict(order="learned", model=model, **full)),
            ("plain_top_m_seed", {}),
            ("plain_head_seed", {"bound_seed": 2}),
            ("untrained_top_m_seed", dict(order="learned", model=untrained))]
    if learned_prof is None:
        runs.append(("learned_top_m_seed", dict(order="learned", model=model)))
    out = {}
    for name, kw in runs:
        ids, dist, _ = idx_dk.knn(dev_q, qo, k, "dk", w["dk_band"], **kw)
        torch.cuda.synchronize()
        same = torch.equal(ids, plain_dk[0]) and torch.equal(dist, plain_dk[1])
        idx_dk.profile(reset=True)
        for _ in range(reps):
            idx_dk.knn(dev_q, qo, k, "dk", w["dk_band"], profile=True, **kw)
        p = idx_dk.profile(reset=True)
        out[name] = _control_row(p, pairs, same)
        print(f"[bench] order control {name}: {out[name]['fraction_full_dps']:.5f} full DPs, "
              f"{out[name]['device_ms']:.3f} ms", file=sys.stderr, flush=True)
    untrained.close()
    if learned_prof is not None:
        out["learned_top_m_seed"] = _control_row(learned_prof, pairs, True)
    return out


def _control_row(p, pairs, same):
    c = max(1, p["calls"])
    return {"fraction_full_dps": p["dp_completed"] / c / pairs,
            "dp_started": p["dp_started"] / c, "dp_completed": p["dp_completed"] / c,
            "dp_valid_cells": p["dp_valid_cells"] / c, "seed_pairs": p["seed_pairs"] / c,
            "device_ms": p["ms_total"] / c, "seed_ms": p["ms_seed"] / c,
            "order_ms": p["ms_order"] / c, "rows_equal_plain": bool(same)}


def cpu_baseline(db, dbo, qs, qo, w, nq_sample, n_series=0):
    import numpy as np
    import oracle as O
    sel = min(nq_sample, w["Q"])
    qsub = qs[:qo[sel]]
    qosub = qo[:sel + 1]
    N = w["N"]
    if 0 < n_series < N:
        N = n_series
        db = db[:dbo[N]]
        dbo = dbo[:N + 1]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    print(f"[bench] cpu baseline: {sel} queries x {N} series on {threads} cores", file=sys.stderr,
          flush=True)
    t0 = time.perf_counter()
    dk = O.knn_scan(db, dbo, qsub, qosub, w["k"], "dk", w["dk_band"])
    t1 = time.perf_counter()
    print(f"[bench] cpu baseline: DK pruned scan {t1 - t0:.1f}s", file=sys.stderr, flush=True)
    dtw = O.knn_scan(db, dbo, qsub, qosub, w["k"], "dtw", w["dtw_band"])
    t2 = time.perf_counter()
    pairs = sel * N
    out = dict(value=pairs / (t2 - t0), unit="pairs/s", cores=threads, kind="oracle",
               sample=f"first {sel} of {w['Q']} queries x first {N} of {w['N']} series, DK then DTW, "
                      f"oracle.knn_scan (the paper's pruned scan: Alg. 1 seed + Alg. 3; "
                      f"LB_Box + early-abandoning DTW), OpenMP over queries",
               dk_pairs_per_s=pairs / (t1 - t0), dtw_pairs_per_s=pairs / (t2 - t1),
               seconds=t2 - t0)
    print(f"[bench] cpu baseline: pruned scan on {threads} cores done", file=sys.stderr, flush=True)
    # the same scan on one core (the paper's own setting), and the plain
    # definition (full DP of every pair) on all cores, each on a small sample
    # (one query x the first 5000 series; up to 16 queries x the first 2000)
    n1, s1 = 1, min(N, 5000)
    nb, sb = min(threads, sel, 16), min(N, 2000)
    prev = O.set_threads(1)
    t0 = time.perf_counter()
    O.knn_scan(db[:dbo[s1]], dbo[:s1 + 1], qs[:qo[n1]], qo[:n1 + 1], w["k"], "dk", w["dk_band"])
    O.knn_scan(db[:dbo[s1]], dbo[:s1 + 1], qs[:qo[n1]], qo[:n1 + 1], w["k"], "dtw", w["dtw_band"])
    t1 = time.perf_counter()
    O.set_threads(prev)
    print("[bench] cpu baseline: pruned scan on one core done", file=sys.stderr, flush=True)
    O.knn_brute(db[:dbo[sb]], dbo[:sb + 1], qs[:qo[nb]], qo[:nb + 1], w["k"], "dk", w["dk_band"])
    O.knn_brute(db[:dbo[sb]], dbo[:sb + 1], qs[:qo[nb]], qo[:nb + 1], w["k"], "dtw", w["dtw_band"])
    t2 = time.perf_counter()
    print("[bench] cpu baseline: brute force done", file=sys.stderr, flush=True)
    out["pruned_scan_1_core"] = {"pairs_per_s": n1 * s1 / (t1 - t0), "queries": n1, "series": s1,
                                 "seconds": t1 - t0}
    out["brute_force_all_cores"] = {"pairs_per_s": nb * sb / (t2 - t1), "queries": nb,
                                    "series": sb, "cores": threads, "seconds": t2 - t1,
                                    "what": "oracle.knn_brute: full DP of every pair, then "
                                            "a (key, id) sort"}
    return out, (sel, dk, dtw)


# subsequence search (Alg. 2 + Alg. 3 with SUB): one long 3-D random walk,
# queries cut from it, warped and noised (the long-recording experiment)
SUBSEQ = dict(cfg_id=6, n=1 << 22, d=3, Q=64, m=256, k=1)


def subsequence(args):
    """Times tsk_subseq_query on the long-series workload (device time of
    the call from its own HIP events; the call is synchronous and allocates
    its working memory, which the wall-clock figure includes) and times the
    oracle's pruned scan on a query sample, checking the GPU rows for it."""
    import numpy as np
    import torch
    from paper_1811_11076_amd import subseq_query, synth
    w = SUBSEQ
    ser = synth.long_walk(w["n"], w["d"], w["cfg_id"])
    soff = np.array([0, w["n"]], np.int64)
    qs, qo, _ = synth.planted_queries(ser, soff, w["Q"], w["m"], w["cfg_id"])
    dser, dq = torch.from_numpy(ser).cuda(), torch.from_numpy(qs).cuda()
    for _ in range(2):
        subseq_query(dser, soff, dq, qo, w["k"])
    dev_ms, wall, st = [], [], None
    for _ in range(5):
        t0 = time.perf_counter()
        ids, dist, end, start, st = subseq_query(dser, soff, dq, qo, w["k"], stats=True)
        wall.append(time.perf_counter() - t0)
        dev_ms.append(st["ms_total"])
    ms = float(np.median(dev_ms))
    positions = w["Q"] * w["n"]
    out = {
        "workload": f"walk-n{w['n']}-d{w['d']}-q{w['Q']}-m{w['m']}-k{w['k']}",
        "unit": "query-positions/s",
        "positions_per_s": positions / (ms * 1e-3),
        "ms_per_call": ms,
        "wall_ms_per_call": float(np.median(wall)) * 1e3,
        "stages_ms": {"seed": st["ms_seed"], "dp": st["ms_dp"], "final_and_start": st["ms_final"]},
        "work_items": st["dp_started"] + st["bound_pruned"],
        "items_skipped_by_row0_bound": st["bound_pruned"],
        "dp_lane_cells": st["dp_cells"],
        "seed_moves_and_scans": st["bound_steps"],
        "dense_cells": positions * w["m"],
    }
    if not args.no_cpu_baseline:
        import oracle as O
        sel = 8
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        rids, rkeys, rend, rstart, _ = O.subseq_scan(ser, soff, qs[:qo[sel]], qo[:sel + 1], w["k"])
        sec = time.perf_counter() - t0
        out["cpu_oracle"] = {"positions_per_s": sel * w["n"] / sec, "queries": sel, "cores": threads,
                             "seconds": sec, "kind": "oracle",
                             "sample": f"first {sel} of {w['Q']} queries, oracle.subseq_scan (Alg. 2 "
                                       "threshold + Alg. 3 with SUB), OpenMP over queries"}
        ok = (np.array_equal(ids[:sel].cpu().numpy(), rids)
              and np.array_equal(dist[:sel].cpu().numpy(), np.sqrt(rkeys.astype(np.float32)))
              and np.array_equal(end[:sel].cpu().numpy(), rend)
              and np.array_equal(start[:sel].cpu().numpy(), rstart))
        out["verified"] = {"queries": sel, "rows_equal_oracle": bool(ok)}
    return out


# tightness and pruning power of LB_Box over dimension x length (Thm. 3.3;
# Sec. 5, tightness and pruning-power heat maps), on three generators:
# class-warp, independent random walks, and i.i.d. Gaussian points (the
# theorem's own assumption)
SWEEP = dict(cfg_id=7, classes=10, Q=16, N=2000, k=10, band=0.1,
             gens=("classwarp", "randomwalk", "iid"),
             dims=(1, 2, 3, 4, 5, 6, 7, 8, 12, 16, 20, 24, 27), lengths=(32, 64, 128, 256, 512))


def tightness_sweep():
    """Per (generator, d, L): mean LB_Box / DTW over all (query, series)
    pairs, the pruning power (share of pairs whose LB_Box exceeds the
    query's k-th nearest DTW, i.e. prunable whatever the scan order) and the
    share the scan itself pruned (tsk_knn_query counters).  LB_Box and DTW
    come from tsk_pair_bounds / tsk_pair_distances (the scan's own kernels)."""
    import numpy as np
    import torch
    from paper_1811_11076_amd import Index, synth
    w = SWEEP
    rows = []
    for gen in w["gens"]:
        for d in w["dims"]:
            for L in w["lengths"]:
                cfg = w["cfg_id"] * 100 + d
                if gen == "classwarp":
                    g = synth.ClassWarp(cfg, w["classes"], L, d)
                    db, dbo, _ = g.members(w["N"], "db", length=L)
                    qs, qo, _ = g.members(w["Q"], "query", length=L, class_mode="uniform")
                else:
                    f = synth.random_walks if gen == "randomwalk" else synth.gaussian_iid
                    db, dbo = synth.flat_equal(f(w["N"], L, d, cfg, "db"))
                    qs, qo = synth.flat_equal(f(w["Q"], L, d, cfg, "query"))
                idx = Index(torch.from_numpy(db).cuda(), dbo)
                dq = torch.from_numpy(qs).cuda()
                lb, _, _ = idx.pair_bounds(dq, qo, "dtw", w["band"])
                dtw = idx.pair_distances(dq, qo, "dtw", w["band"])
                _, _, st = idx.knn(dq, qo, w["k"], "dtw", w["band"], stats=True)
                lb = lb.double().cpu().numpy()
                dtw = dtw.double().cpu().numpy()
                tau = np.sort(dtw, axis=1)[:, w["k"] - 1:w["k"]]
                pos = dtw > 0
                rows.append({"gen": gen, "d": d, "L": L,
                             "tightness": float((lb[pos] / dtw[pos]).mean()),
                             "pruning_power": float((lb > tau).mean()),
                             "scan_pruned": st["bound_pruned"] / max(1, st["pairs"])})
                idx.close()
                print(f"[sweep] {gen} d={d} L={L} tightness {rows[-1]['tightness']:.4f} "
                      f"pruning {rows[-1]['pruning_power']:.4f}", file=sys.stderr, flush=True)
    return {"queries": w["Q"], "series": w["N"], "k": w["k"], "band": w["band"], "rows": rows}


# DK against DTW + LB_Box as the dimension grows (Sec. 5.2, Table 1 spans
# d = 1 .. 27), class-warp series of one length, library defaults
DIM_SWEEP = dict(cfg_id=8, classes=50, Q=256, N=100000, L=128, k=10,
                 dims=(1, 2, 3, 6, 8, 13, 22, 27), reps=3)


def dim_sweep():
    """Per d: device time of one k-NN call (all queries) for DK (no band),
    DTW with a 10 % band and unbanded DTW, the DTW / DK time ratio, and the
    share of pairs that reached a DP (tsk_knn_query counters)."""
    import torch
    from paper_1811_11076_amd import Index, synth
    w = DIM_SWEEP
    rows = []
    for d in w["dims"]:
        t0 = time.perf_counter()
        g = synth.ClassWarp(w["cfg_id"] * 100 + d, w["classes"], w["L"], d)
        db, dbo, _ = g.members(w["N"], "db", length=w["L"])
        qs, qo, _ = g.members(w["Q"], "query", length=w["L"], class_mode="uniform")
        idx = Index(torch.from_numpy(db).cuda(), dbo)
        dq = torch.from_numpy(qs).cuda()
        row = {"d": d}
        for name, dist, band in (("dk", "dk", None), ("dtw_band10", "dtw", 0.1),
                                 ("dtw_full", "dtw", None)):
            _, _, st = idx.knn(dq, qo, w["k"], dist, band, stats=True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(w["reps"]):
                idx.knn(dq, qo, w["k"], dist, band)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t1) * 1e3 / w["reps"]
            row[name] = {"ms": ms, "pairs_per_s": w["Q"] * w["N"] / (ms * 1e-3),
                         "dp_share": st["dp_started"] / max(1, st["pairs"])}
        row["dtw_band10_over_dk"] = row["dtw_band10"]["ms"] / row["dk"]["ms"]
        row["dtw_full_over_dk"] = row["dtw_full"]["ms"] / row["dk"]["ms"]
        idx.close()
        del dq
        rows.append(row)
        print(f"[dims] d={d} dk {row['dk']['ms']:.1f} ms, dtw 10% {row['dtw_band10']['ms']:.1f} ms, "
              f"dtw full {row['dtw_full']['ms']:.1f} ms ({time.perf_counter() - t0:.1f}s)",
              file=sys.stderr, flush=True)
    return {"queries": w["Q"], "series": w["N"], "length": w["L"], "k": w["k"], "rows": rows}


def full_size_check(db, dbo, qs, qo, w, res_dk, res_dtw, nq_dk=16, nq_dtw=8):
    """Checks the GPU rows against the oracle at full size: the first nq_dk
    (DK) and nq_dtw (DTW) queries against every series (the oracle's pruned
    scan with its envelope kept per length, equal to the plain definition),
    ids and distance bits; and every (id, distance) returned for every query
    recomputed by the oracle's full DP."""
    import numpy as np
    import oracle as O
    out = {}
    t0 = time.perf_counter()
    for name, (ids, dist), nsel, band in (("dk", res_dk, nq_dk, w["dk_band"]),
                                         ("dtw", res_dtw, nq_dtw, w["dtw_band"])):
        nsel = min(nsel, w["Q"])
        t1 = time.perf_counter()
        rids, rkeys, _ = O.knn_verify(db, dbo, qs[:qo[nsel]], qo[:nsel + 1], w["k"], name, band)
        t2 = time.perf_counter()
        g_ids = ids.cpu().numpy()
        g_dist = dist.cpu().numpy()
        exp = np.sqrt(rkeys.astype(np.float32)) if name == "dk" else rkeys.astype(np.float32)
        rows_ok = (np.array_equal(g_ids[:nsel], rids)
                   and np.array_equal(g_dist[:nsel].view(np.uint32), exp.view(np.uint32)))
        # every returned pair of every query: the oracle's full DP of that pair
        q_idx, r_idx = np.nonzero(g_ids >= 0)
        keys = O.pair_list_keys(db, dbo, qs, qo, q_idx, g_ids[q_idx, r_idx], name, band)
        got = g_dist[q_idx, r_idx]
        want = np.sqrt(keys) if name == "dk" else keys
        pairs_ok = bool(np.array_equal(got.view(np.uint32), want.astype(np.float32).view(np.uint32)))
        # each row ascending by (distance, id), padding only at the end
        order_ok = True
        for q in range(g_ids.shape[0]):
            row = [(g_dist[q, r], g_ids[q, r]) for r in range(g_ids.shape[1]) if g_ids[q, r] >= 0]
            if row != sorted(row) or len(row) != len(set(x[1] for x in row)):
                order_ok = False
                break
        t3 = time.perf_counter()
        out[name] = {"queries_vs_all_series": nsel, "series": int(dbo.shape[0] - 1),
                     "rows_equal_oracle": bool(rows_ok),
                     "returned_pairs_rechecked": int(q_idx.size),
                     "returned_pairs_equal_oracle": pairs_ok, "rows_sorted": order_ok,
                     "oracle_seconds": t2 - t1, "recheck_seconds": t3 - t2}
        print(f"[bench] full-size check {name}: {nsel} queries x all series "
              f"{'equal' if rows_ok else 'DIFFER'}; {q_idx.size} returned pairs "
              f"{'equal' if pairs_ok else 'DIFFER'} ({t3 - t1:.1f}s)", file=sys.stderr, flush=True)
    out["verified_queries"] = bool(all(out[n]["rows_equal_oracle"] and
                                       out[n]["returned_pairs_equal_oracle"] and
                                       out[n]["rows_sorted"] for n in ("dk", "dtw")))
    out["seconds"] = time.perf_counter() - t0
    return out


def roofline_of(prof_dk, prof_dtw, w, uneven, workload):
    kern = {"dk": kernel_rooflines(prof_dk, "dk", w["d"], "k_dp_tube", uneven),
            "dtw": kernel_rooflines(prof_dtw, "dtw", w["d"], "k_dp_band", uneven)}
    if uneven:
        kern["dtw"].pop("k_dp_band")  # uneven lengths: every DTW DP is a general one
    dist_dom, kname = max(((dd, kk) for dd in kern for kk in kern[dd] if "stage" not in kk),
                          key=lambda x: kern[x[0]][x[1]]["ms"])
    dom = kern[dist_dom][kname]
    roof = {"bound": "alu", "kernel": f"{kname} ({dist_dom})",
            "achieved": dom["tops"], "peak": VALU_PEAK_OPS / 1e12, "unit": "TOP/s",
            "frac": dom["tops"] * 1e12 / VALU_PEAK_OPS,
            "traffic": load_traffic(kname, workload),
            "ms_per_launch": dom["ms"], "algorithmic_ops_per_launch": dom["ops"],
            "per_unit_ops": dom["unit_ops"], "units_per_launch": dom["units"]}
    return roof, kern


def dist_summary(prof, kern, pairs):
    c = max(1, prof["calls"])
    ms = prof["ms_total"] / c
    return {"pairs_per_s": pairs / (ms * 1e-3), "device_ms": ms,
            "stages_ms": {"order": prof["ms_order"] / c, "seed": prof["ms_seed"] / c,
                          "bound": prof["ms_bound"] / c, "dp": prof["ms_dp"] / c,
                          "final": prof["ms_final"] / c},
            "launches_per_call": prof["chunks"] / c,
            "kernels_per_launch": {k: {"ms": round(v["ms"], 4), "TOP/s": round(v["tops"], 3)}
                                   for k, v in kern.items()},
            "dp_started": prof["dp_started"] / c, "dp_completed": prof["dp_completed"] / c,
            "dp_valid_cells": prof["dp_valid_cells"] / c,
            "fallback_pairs": prof["fallback_pairs"] / c}


def train_encoder(w, seed=1):
    import torch
    from paper_1811_11076_amd import Model, synth
    from paper_1811_11076_amd.learned import dk_training_set
    t0 = time.perf_counter()
    gen = synth.ClassWarp(w["cfg_id"], w["classes"], w["L"], w["d"])
    # 200k pairs: 500 anchors x (200 same-class + 200 random) of a 2000-series pool
    tv, to, ta, tb, ty = dk_training_set(gen, 2000, 500, 200, w.get("lengths", w["L"]), seed=1)
    model = Model(w["d"], seed=seed)
    losses = model.train(torch.from_numpy(tv).cuda(), to, ta, tb, ty, epochs=10, batch=1024,
                         lr=1e-3, seed=1)
    t_train = time.perf_counter() - t0
    print(f"[bench] encoder trained on {ta.size} pairs in {t_train:.1f}s, loss "
          f"{losses[0]:.3f} -> {losses[-1]:.3f}", file=sys.stderr, flush=True)
    return model, {"pairs": int(ta.size), "epochs": 10, "batch": 1024, "seconds": t_train,
                   "loss_first_epoch": float(losses[0]), "loss_last_epoch": float(losses[-1])}


def graph_step_large(w, args, idx_dk, idx_dtw, dev_q, qo, eager_res, model):
    """The large workload's step as one captured HIP graph per distance (all
    the call's query chunks in it), the two graphs replayed on two streams
    of default priority at once; rows checked against the eager step.  The
    DK call in the learned candidate order is also timed as a replayed
    graph."""
    import torch
    k, nq = w["k"], w["Q"]
    outs = {name: (torch.empty((nq, k), dtype=torch.int64, device="cuda"),
                   torch.empty((nq, k), dtype=torch.float32, device="cuda"))
            for name in ("dk", "dtw", "dk_learned")}
    streams = (torch.cuda.Stream(), torch.cuda.Stream())
    torch.cuda.synchronize()

    def step():
        with torch.cuda.stream(streams[0]):
            idx_dk.knn(dev_q, qo, k, "dk", w["dk_band"], use_graph=True, out=outs["dk"])
        with torch.cuda.stream(streams[1]):
            idx_dtw.knn(dev_q, qo, k, "dtw", w["dtw_band"], use_graph=True, out=outs["dtw"])

    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    same = all(torch.equal(x, y) for x, y in zip(outs["dk"] + outs["dtw"],
                                                 eager_res[0][:2] + eager_res[1][:2]))
    print(f"[bench] graph step: {args.steps} steps in {el:.3f}s", file=sys.stderr, flush=True)
    # DK in the learned order, one replayed graph per call
    reps = max(1, args.plain_reps)
    for _ in range(2):
        idx_dk.knn(dev_q, qo, k, "dk", w["dk_band"], order="learned", model=model,
                   use_graph=True, out=outs["dk_learned"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(reps):
        idx_dk.knn(dev_q, qo, k, "dk", w["dk_band"], order="learned", model=model,
                   use_graph=True, out=outs["dk_learned"])
    torch.cuda.synchronize()
    el2 = time.perf_counter() - t2
    same_l = all(torch.equal(x, y) for x, y in zip(outs["dk_learned"], eager_res[0][:2]))
    return {"ms_per_step": el * 1e3 / args.steps, "rows_equal_eager": bool(same),
            "mode": "one captured HIP graph per distance (every query chunk of the call), "
                    "replayed on two concurrent streams of default priority",
            "dk_learned_graph_ms": el2 * 1e3 / reps, "dk_learned_graph_rows_equal": bool(same_l)}


def run_large(name, w, args):
    """The large workload: the step is DK plus DTW over all queries in the
    library's default configuration (plain candidate order; the threshold
    seeded from the candidates of smallest corner bound; DTW prunes by the
    corner bound before LB_Box), eager calls with per-stage HIP events; the
    learned candidate order, DTW with LB_Box on every pair, the order / seed
    controls (on a query subset), the full-size oracle check and the CPU
    baseline follow."""
    import numpy as np
    import torch
    from paper_1811_11076_amd import Index, Model
    t_gen = time.perf_counter()
    db, dbo, qs, qo = make_data(w)
    print(f"[bench] workload {name}: data in {time.perf_counter() - t_gen:.1f}s",
          file=sys.stderr, flush=True)
    dev_db = torch.from_numpy(db).cuda()
    dev_q = torch.from_numpy(qs).cuda()
    idx_dk = Index(dev_db, dbo)
    idx_dtw = Index(dev_db, dbo)
    del dev_db
    torch.cuda.synchronize()
    k, pairs = w["k"], w["Q"] * w["N"]
    model, train_info = train_encoder(w)
    dtw_kw = {}

    def step(profile):
        a = idx_dk.knn(dev_q, qo, k, "dk", w["dk_band"], profile=profile)
        b = idx_dtw.knn(dev_q, qo, k, "dtw", w["dtw_band"], profile=profile, **dtw_kw)
        return a, b

    for _ in range(max(1, args.warmup)):
        res = step(False)
    torch.cuda.synchronize()
    idx_dk.profile(reset=True)
    idx_dtw.profile(reset=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] {args.steps} steps in {elapsed:.3f}s", file=sys.stderr, flush=True)
    prof_dk = idx_dk.profile(reset=True)
    prof_dtw = idx_dtw.profile(reset=True)
    ms_step = elapsed * 1e3 / args.steps
    eager = {"ms_per_step": ms_step, "pairs_per_s": w["Q"] * w["N"] / (ms_step * 1e-3)}
    roof, kern = roofline_of(prof_dk, prof_dtw, w, False, name)
    graph = None
    mode = ("eager calls with per-stage HIP events: DK, then DTW, each over all queries in "
            "the library's default configuration")
    if not args.eager:
        graph = graph_step_large(w, args, idx_dk, idx_dtw, dev_q, qo, res, model)
        # the step is the faster of the two modes, timed over the same steps
        # with identical rows
        if graph["rows_equal_eager"] and graph["ms_per_step"] < ms_step:
            ms_step = graph["ms_per_step"]
            mode = graph["mode"] + "; the library's default configuration"

    # the learned candidate order (trained encoder): same rows
    plain_reps = max(1, args.plain_reps)
    for _ in range(plain_reps):
        ldk_res = idx_dk.knn(dev_q, qo, k, "dk", w["dk_band"], profile=True, order="learned",
                             model=model)
    torch.cuda.synchronize()
    prof_learned = idx_dk.profile(reset=True)
    learned_same = torch.equal(ldk_res[0], res[0][0]) and torch.equal(ldk_res[1], res[0][1])
    kern_learned = kernel_rooflines(prof_learned, "dk", w["d"], "k_dp_tube", cascade=False)
    print(f"[bench] learned-order DK: "
          f"{prof_learned['ms_total'] / max(1, prof_learned['calls']):.1f} ms per call",
          file=sys.stderr, flush=True)
    dk = dist_summary(prof_dk, kern["dk"], pairs)
    dtw = dist_summary(prof_dtw, kern["dtw"], pairs)
    dk_learned = dist_summary(prof_learned, kern_learned, pairs)

    # DTW without the corner-bound cascade (LB_Box of every pair, threshold
    # from the diagonal paths of the first candidates): same rows, timed
    # beside the default cascade
    dtw_lb_all = None
    if not args.no_controls:
        for _ in range(plain_reps):
            cres = idx_dtw.knn(dev_q, qo, k, "dtw", w["dtw_band"], profile=True, dtw_cascade=2,
                               bound_seed=2)
        torch.cuda.synchronize()
        prof_all = idx_dtw.profile(reset=True)
        kern_all = kernel_rooflines(prof_all, "dtw", w["d"], "k_dp_band", cascade=False)
        dtw_lb_all = dist_summary(prof_all, kern_all, pairs)
        dtw_lb_all["rows_equal_default"] = bool(torch.equal(cres[0], res[1][0]) and
                                                torch.equal(cres[1], res[1][1]))
        print(f"[bench] DTW with LB_Box on every pair: {dtw_lb_all['device_ms']:.1f} ms per "
              f"call", file=sys.stderr, flush=True)

    controls = None
    if not args.no_controls:
        sub = min(w["Q"], args.control_queries)
        sq = dev_q[:int(qo[sub])]
        so = qo[:sub + 1]
        sw = dict(w, Q=sub)
        plain_rows = (res[0][0][:sub].contiguous(), res[0][1][:sub].contiguous())
        controls = order_controls(sw, idx_dk, sq, so, model, plain_rows, None, reps=1)
        controls["queries"] = sub
    out = {
        "metric": METRIC, "value": pairs / (ms_step * 1e-3), "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "queries": w["Q"], "series": w["N"], "length": w["L"],
                   "dim": w["d"], "k": k, "dk_band": w["dk_band"], "dtw_band": w["dtw_band"],
                   "order": "plain (threshold seeded from the smallest corner bounds)"},
        "roofline": roof,
        "dk": dk, "dtw": dtw,
        "dk_vs_dtw_speedup": dtw["device_ms"] / dk["device_ms"],
        "dtw_lb_box_every_pair": dtw_lb_all,
        "dtw_cascade_speedup": (dtw_lb_all["device_ms"] / dtw["device_ms"]) if dtw_lb_all else None,
        "step": mode,
        "eager_profiled": eager,
        "graph": graph,
        "learned_order": {
            "train": train_info,
            "dk_learned_order": dk_learned,
            "rows_equal_plain": bool(learned_same),
            "dk_speedup_vs_plain": dk["device_ms"] / dk_learned["device_ms"],
            "step_speedup_vs_plain": (dk["device_ms"] + dtw["device_ms"]) /
                                     (dk_learned["device_ms"] + dtw["device_ms"]),
            "dk_fraction_full_dps": dk_learned["dp_completed"] / pairs,
            "dk_fraction_full_dps_plain": dk["dp_completed"] / pairs,
            "dk_controls": controls,
        },
    }
    model.close()
    if not args.no_verify:
        out["full_size_check"] = full_size_check(db, dbo, qs, qo, w, res[0][:2], res[1][:2])
        out["verified_queries"] = out["full_size_check"]["verified_queries"]
    if not args.no_cpu_baseline:
        cb, _ = cpu_baseline(db, dbo, qs, qo, w, args.cpu_queries, args.cpu_series)
        out["cpu_baseline"] = cb
    idx_dk.close()
    idx_dtw.close()
    return out


def run_standard(name, w, args, secondary=False):
    """Workloads that fit a query call in one chunk: eager profiled steps,
    then the tuned graph step (the faster of the two is the step), the
    learned order and its controls, the CPU baseline with a row check."""
    import numpy as np
    import torch
    from paper_1811_11076_amd import Index

    t_gen = time.perf_counter()
    db, dbo, qs, qo = make_data(w)
    print(f"[bench] workload {name}: data in {time.perf_counter() - t_gen:.1f}s",
          file=sys.stderr, flush=True)
    dev_db = torch.from_numpy(db).cuda()
    dev_q = torch.from_numpy(qs).cuda()
    idx_dk = Index(dev_db, dbo)
    idx_dtw = Index(dev_db, dbo)
    k = w["k"]

    def step(profile):
        a = idx_dk.knn(dev_q, qo, k, "dk", w["dk_band"], profile=profile)
        b = idx_dtw.knn(dev_q, qo, k, "dtw", w["dtw_band"], profile=profile)
        return a, b

    for _ in range(args.warmup):
        res = step(False)
    torch.cuda.synchronize()
    idx_dk.profile(reset=True)
    idx_dtw.profile(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] {args.steps} steps in {elapsed:.3f}s", file=sys.stderr, flush=True)
    prof_dk = idx_dk.profile(reset=True)
    prof_dtw = idx_dtw.profile(reset=True)
    eager = {"ms_per_step": elapsed * 1e3 / args.steps}

    batching = None
    mode = "eager calls with per-stage HIP events"
    if not args.eager:
        batching = tuned_graph(w, args, idx_dk, idx_dtw, dev_q, qs, qo, res)
        # the step is the library's faster configuration of the two, both
        # timed over the same number of steps with identical rows
        if batching["rows_equal_eager"] and batching["ms_per_step"] < eager["ms_per_step"]:
            elapsed = batching["ms_per_step"] * args.steps * 1e-3
            mode = ("tuned options; one captured HIP graph per distance, replayed, the two "
                    "on concurrent streams")

    learned = None
    if not args.no_learned and w["gen"] == "classwarp" and not secondary:
        learned = learned_order(w, args, db, dbo, dev_db, dev_q, qo, idx_dk, idx_dtw, res)

    pairs = w["Q"] * w["N"]
    ms_step = elapsed * 1e3 / args.steps
    value = pairs / (ms_step * 1e-3)
    eager["pairs_per_s"] = pairs / (eager["ms_per_step"] * 1e-3)
    uneven = "lengths" in w
    roof, kern = roofline_of(prof_dk, prof_dtw, w, uneven, name)
    dk = dist_summary(prof_dk, kern["dk"], pairs)
    dtw = dist_summary(prof_dtw, kern["dtw"], pairs)
    out = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": name, "queries": w["Q"], "series": w["N"],
                   "length": w["L"], "dim": w["d"], "k": k, "dk_band": w["dk_band"],
                   "dtw_band": w["dtw_band"], "order": "plain"},
        "roofline": roof,
        "dk": dk, "dtw": dtw,
        "dk_vs_dtw_speedup": dtw["device_ms"] / dk["device_ms"],
        "step": mode,
        "eager_profiled": eager,
    }
    if batching is not None:
        out["batching"] = batching
    if learned is not None:
        # both legs eager and sequential: the learned order's effect alone
        learned["step_speedup_vs_plain"] = eager["ms_per_step"] / learned["ms_per_step"]
        learned["dk_speedup_vs_plain"] = dk["device_ms"] / learned["dk"]["device_ms"]
        learned["dk_fraction_full_dps_plain"] = prof_dk["dp_completed"] / max(1, prof_dk["calls"]) / pairs
        out["learned_order"] = learned
    if secondary:
        # rows of a query sample against the oracle's plain definition
        import oracle as O
        sel = min(w["Q"], 16)
        ok = {}
        for dist, r, band in (("dk", res[0], w["dk_band"]), ("dtw", res[1], w["dtw_band"])):
            rids, _, _ = O.knn_verify(db, dbo, qs[:qo[sel]], qo[:sel + 1], k, dist, band)
            ok[dist] = bool(np.array_equal(r[0][:sel].cpu().numpy(), rids))
        out["verified_queries"] = {"count": sel, "dk_ids_equal": ok["dk"], "dtw_ids_equal": ok["dtw"]}
    elif not args.no_cpu_baseline:
        import oracle as O
        cb, (sel, dk_ref, dtw_ref) = cpu_baseline(db, dbo, qs, qo, w, args.cpu_queries,
                                                  args.cpu_series)
        out["cpu_baseline"] = cb
        (ids_dk, dist_dk, _), (ids_dtw, dist_dtw, _) = res
        if not (0 < args.cpu_series < w["N"]):
            ok_dk = np.array_equal(ids_dk[:sel].cpu().numpy(), dk_ref[0])
            ok_dtw = np.array_equal(ids_dtw[:sel].cpu().numpy(), dtw_ref[0])
            out["verified_queries"] = {"count": sel, "dk_ids_equal": bool(ok_dk),
                                       "dtw_ids_equal": bool(ok_dtw)}
        else:
            # the CPU sample covers part of the database: the first queries
            # against every series through the oracle's verify scan
            nv = min(8, w["Q"])
            ok = {}
            for dist, ids, band in (("dk", ids_dk, w["dk_band"]), ("dtw", ids_dtw, w["dtw_band"])):
                t0 = time.perf_counter()
                rids, _, _ = O.knn_verify(db, dbo, qs[:qo[nv]], qo[:nv + 1], k, dist, band)
                ok[dist] = bool(np.array_equal(ids[:nv].cpu().numpy(), rids))
                print(f"[bench] {dist}: {nv} queries x all series against the oracle "
                      f"({time.perf_counter() - t0:.1f}s)", file=sys.stderr, flush=True)
            out["verified_queries"] = {"count": nv, "dk_ids_equal": ok["dk"],
                                       "dtw_ids_equal": ok["dtw"]}
    idx_dk.close()
    idx_dtw.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-queries", type=int, default=0,
                    help="queries of the CPU baseline sample (0 = 16)")
    ap.add_argument("--cpu-series", type=int, default=0,
                    help="limit the CPU baseline sample to the first S series (0 = 20000 on "
                         "the large workload, 10000 on uneven lengths, else all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true",
                    help="skip the full-size oracle check of the large workload")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-controls", action="store_true",
                    help="skip the order / seed controls of the large workload")
    ap.add_argument("--control-queries", type=int, default=512,
                    help="queries of the large workload's order / seed controls")
    ap.add_argument("--plain-reps", type=int, default=2,
                    help="plain-order DK calls timed on the large workload")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 100 x 20 000 workload that the large one reports beside it")
    ap.add_argument("--no-subseq", action="store_true",
                    help="skip the subsequence-search measurement")
    ap.add_argument("--tightness-sweep", action="store_true",
                    help="run only the LB_Box tightness / pruning-power sweep (one JSON line)")
    ap.add_argument("--dim-sweep", action="store_true",
                    help="run only the DK / DTW time over the dimension d (one JSON line)")
    ap.add_argument("--subseq-only", action="store_true",
                    help="run only the subsequence-search measurement (one JSON line)")
    ap.add_argument("--eager", action="store_true",
                    help="time the profiled eager step instead of the tuned graph step")
    ap.add_argument("--per-query-sample", type=int, default=32)
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (the reference "
                         "dispatch that scales the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the scan runs on exactly one GPU; --gpus must be 1 "
                                   "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)
    if args.tightness_sweep:
        print(json.dumps({"tightness_sweep": tightness_sweep()}), flush=True)
        return
    if args.subseq_only:
        print(json.dumps({"subsequence": subsequence(args)}), flush=True)
        return
    if args.dim_sweep:
        print(json.dumps({"dim_sweep": dim_sweep()}), flush=True)
        return

    import torch

    if args.copy_calib_mib > 0:
        n = args.copy_calib_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    w = WORKLOADS[args.workload]
    large = bool(w.get("large"))
    # the CPU sample: 16 queries (one per host core) against a bounded
    # slice of the database, so the oracle runs 10-30 s
    if args.cpu_queries <= 0:
        args.cpu_queries = 16
    if args.cpu_series <= 0:
        args.cpu_series = 20000 if large else (10000 if "lengths" in w else 0)
    if large:
        out = run_large(args.workload, w, args)
    else:
        out = run_standard(args.workload, w, args)
    if large and not args.no_secondary:
        t0 = time.perf_counter()
        sec = run_standard(SECONDARY, WORKLOADS[SECONDARY], args, secondary=True)
        keep = ("value", "unit", "ms_per_step", "config", "roofline", "dk", "dtw",
                "dk_vs_dtw_speedup", "step", "verified_queries")
        out["secondary"] = {key: sec[key] for key in keep if key in sec}
        print(f"[bench] secondary workload {SECONDARY} in {time.perf_counter() - t0:.1f}s",
              file=sys.stderr, flush=True)
    if not args.no_subseq:
        out["subsequence"] = subsequence(args)
        print(f"[bench] subsequence search: {out['subsequence']['ms_per_call']:.3f} ms per call",
              file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
