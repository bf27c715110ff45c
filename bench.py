"""Benchmark: reachable pairs per second of the Kronecker-product fixpoint on
one MI355X.

Workload (one "step" = one whole query, every step of the hot path):
  regular path query (a|b)* c d* compiled to its minimal 2-state automaton,
  on a seeded power-law directed graph, n = 100,000, out-degrees
  round(Pareto(2.1)) with mean 4, uniform targets, labels Zipf(1.2) over
  {a, b, c, d}.  The graph is resident in HBM before timing starts, as the
  paper excludes graph loading from its timings.

Prints one JSON line with the throughput, the roofline of the dominant
kernel (one frontier level of the incremental closure, HBM-bound), and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

INT8_PEAK_TOPS = 5000.0    # dense int8 matrix-core peak, TOP/s
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the level kernel from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE passes (scaled by a 1 GiB copy kernel: fetch x2.0, write x1.0),
# keyed by the library version they were taken on; see profiles/.  A kernel
# change bumps the version and the figure is reported as null until the
# counters are taken again.
PMC_TRAFFIC = {("cfpq-gfx950 0.1", "levels"): 3.4596e9,
               ("cfpq-gfx950 0.2", "auto"): 57.28e6, ("cfpq-gfx950 0.2", "condensed"): 57.28e6,
               ("cfpq-gfx950 0.3", "auto"): 100.9e6, ("cfpq-gfx950 0.3", "condensed"): 100.9e6,
               ("cfpq-gfx950 0.4", "auto"): 101.0e6, ("cfpq-gfx950 0.4", "condensed"): 101.0e6,
               ("cfpq-gfx950 0.5", "auto"): 107.1e6, ("cfpq-gfx950 0.5", "condensed"): 107.1e6,
               ("cfpq-gfx950 0.6", "auto"): 107.2e6, ("cfpq-gfx950 0.6", "condensed"): 107.2e6,
               ("cfpq-gfx950 0.7", "auto"): 109.0e6, ("cfpq-gfx950 0.7", "condensed"): 109.0e6}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--tile-words", type=int, default=0)
    ap.add_argument("--strategy", choices=["auto", "levels", "condensed"], default="auto",
                    help="closure strategy of the plain single-query path (auto = condensed for a regular query)")
    ap.add_argument("--nt-mode", choices=["auto", "rows", "mfma"], default="auto",
                    help="box-labelled transitions in closure levels (grammar workloads): automatic, "
                         "whole-row OR, or the int8 matrix-core product")
    ap.add_argument("--recompute", action="store_true",
                    help="grammar workloads: recompute the closure from scratch every iteration")
    ap.add_argument("--cpu-sources", type=int, default=20000, help="oracle sample size (sources)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-queries", type=int, default=400)
    ap.add_argument("--serve-nmax", type=int, default=20000)
    ap.add_argument("--serve-slots", type=int, default=8, help="execution slots (streams) of the batched server")
    ap.add_argument("--serve-rates", default="0.5,1,2,4",
                    help="open-loop arrival rates as multiples of the plain closed-loop throughput")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--workload", choices=["rpq", "brackets", "samegen", "alias", "paths"], default="rpq",
                    help="rpq (default, the headline) or one of the other measured workloads")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 3 times (reference kernel for the "
                         "FETCH_SIZE/WRITE_SIZE scale factor) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding is "
              f"described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        a = torch.ones(args.calibrate_copy * (1 << 20) // 8, dtype=torch.int64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 8, "copies": 3}), flush=True)
        return

    import synth
    from paper_2103_14688_amd import cfpq, rsm

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload != "rpq":
        print(json.dumps(other_workload(args)), flush=True)
        return
    g = synth.powerlaw(args.n, seed=synth.BASE_SEED + 2)
    R = rsm.from_regex(synth.RPQ_C2, g.labels)
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(R)
    strat = {"auto": cfpq.STRATEGY_AUTO, "levels": cfpq.STRATEGY_LEVELS,
             "condensed": cfpq.STRATEGY_CONDENSED}[args.strategy]
    kw = dict(strategy=strat, tile_words=args.tile_words)
    dominant = cfpq.KERNEL_LEVEL if args.strategy == "levels" else cfpq.KERNEL_COND_LEVEL
    print(f"# graph n={g.n} m={len(g.src)} states={R.n_states}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        cfpq.query(graph, q, **kw).close()
    torch.cuda.synchronize()

    # a steady query loop: each step's result is read (its statistics and
    # per-kernel profile, host-side) and released when the next one exists,
    # so its memory returns to the allocator's cache as a server's would
    rows, last = [], None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = cfpq.query(graph, q, profile=True, **kw)
        rows.append((r.stats(), r.profile(dominant), r.profile(cfpq.KERNEL_SEED), r.profile(cfpq.KERNEL_WRITEBACK),
                     r.profile(cfpq.KERNEL_COND_SCC)))
        if last is not None:
            last.close()
        last = r
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    pairs = last.count(0)
    it, deltas, fix_ms = rows[-1][0]
    fix = [x[0][2] for x in rows]
    # dominant kernel: closure level launches, summed over the timed steps
    lv_n = lv_ms = lv_bytes = 0
    for x in rows:
        n_l, ms_l, by_l = x[1]
        lv_n += n_l
        lv_ms += ms_l
        lv_bytes += by_l
    seed = [x[2] for x in rows]
    wb = [x[3] for x in rows]
    scc = [x[4] for x in rows]
    last.close()
    avg_launch_ms = lv_ms / max(lv_n, 1)
    bytes_per_launch = lv_bytes / max(lv_n, 1)
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9 if avg_launch_ms > 0 else 0.0

    cpu = None
    if not args.no_cpu:
        import oracle
        threads = min(os.cpu_count() or 1, 16)
        rng = np.random.default_rng(synth.BASE_SEED + 7)
        srcs = np.sort(rng.choice(g.n, size=min(args.cpu_sources, g.n), replace=False)).astype(np.uint32)
        tc = time.perf_counter()
        rows = oracle.rpq_rows(g.n, g.src, g.lbl, g.dst, g.labels, synth.RPQ_C2, srcs, threads=threads)
        dt = time.perf_counter() - tc
        cpu_pairs = int(np.unpackbits(rows.view(np.uint8)).sum())
        cpu = {"value": cpu_pairs / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
               "sample": f"{len(srcs)} of {g.n} sources (product-automaton BFS per source), "
                         f"{cpu_pairs} pairs in {dt:.2f} s"}

    serving = None if args.no_serve else measure_serving(args)

    out = {
        "metric": "reachable pairs/s (fixpoint, plain single query)",
        "value": pairs * args.steps / wall,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": f"RPQ (a|b)* c d* on power-law graph n={g.n} (Pareto(2.1) out-degree mean 4, "
                        f"Zipf(1.2) labels), plain one-query-at-a-time path",
            "n": g.n, "edges": int(len(g.src)), "rsm_states": int(R.n_states), "pairs": int(pairs),
            "iterations": it, "fixpoint_ms_median": float(np.median(fix)), "fixpoint_ms_mean": float(np.mean(fix)),
            "tile_words": args.tile_words,
            "level_launches_per_step": lv_n / args.steps,
            "strategy": args.strategy,
            "component_search_ms_per_step": sum(s[1] for s in scc) / args.steps,
            "seed_ms_per_step": sum(s[1] for s in seed) / args.steps,
            "writeback_ms_per_step": sum(w[1] for w in wb) / args.steps,
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": PMC_TRAFFIC.get((cfpq.cfpq_version(), args.strategy)),
            "kernel": "k_gather<false> (closure frontier level)" if args.strategy == "levels"
                      else "k_cond_level (one topological level of the component graph)",
            "avg_launch_ms": avg_launch_ms, "algorithmic_bytes_per_launch": bytes_per_launch,
        },
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = [fn() for _ in range(steps)]
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) / steps


def other_workload(args):
    """The other measured workloads (one JSON line each):
    brackets -- S -> a S b | a b on directed Erdos-Renyi n = 256, p = 2/n per
                label: the latency-bound plain query (levels and fused
                strategies) and 1024 such queries (seeds) in one fused launch;
    samegen  -- same-generation grammar G1 on a hierarchy (tree with Poisson(4)
                branching, 20% type edges, inverse labels), n = args.n;
    alias    -- memory-alias grammar on a clustered program-like graph, n = args.n."""
    import numpy as np

    import synth
    from paper_2103_14688_amd import cfpq, rsm

    out = {"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "data": "synthetic", "dtype": "u64",
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None}
    if args.workload == "brackets":
        g = synth.erdos_renyi(256, seed=synth.BASE_SEED + 1)
        graph = cfpq.Graph.from_synth(g)
        q = cfpq.Query(rsm.from_grammar(synth.BRACKETS, g.labels))
        res = {}
        for name, st in (("levels", cfpq.STRATEGY_LEVELS), ("fused", cfpq.STRATEGY_FUSED)):
            rs, dt = timed(lambda: cfpq.query(graph, q, strategy=st), args.steps, args.warmup)
            it, deltas, ms = rs[-1].stats()
            res[name] = {"ms_per_query_wall": dt * 1e3, "fixpoint_ms": ms, "iterations": it,
                         "us_per_iteration": ms * 1e3 / it, "pairs": rs[-1].count(0)}
        # batch: 1024 graphs (seeds), one persistent fused launch
        gs = [synth.erdos_renyi(256, seed=synth.BASE_SEED + 1000 + i) for i in range(1024)]
        hs = [cfpq.Graph.from_synth(x) for x in gs]
        qs = [q] * len(hs)
        rs, dt = timed(lambda: cfpq.query_batch(hs, qs), max(1, args.steps // 2), 1)
        pairs = sum(r.count(0) for r in rs[-1])
        res["batched_1024"] = {"ms_per_batch_wall": dt * 1e3, "queries_per_s": 1024 / dt,
                               "pairs_per_s": pairs / dt, "pairs": pairs}
        out.update({"metric": "reachable pairs/s, balanced brackets (plain vs fused vs batched)",
                    "value": res["batched_1024"]["pairs_per_s"], "unit": "pairs/s",
                    "ms_per_step": res["fused"]["ms_per_query_wall"],
                    "config": {"workload": "S -> a S b | a b on directed Erdos-Renyi n=256, p=2/n per label",
                               **res}})
        return out
    if args.workload == "paths":
        return paths_workload(args, out)
    if args.workload == "samegen":
        g, depth = synth.hierarchy(args.n, seed=synth.BASE_SEED + 3)
        text = synth.SAME_GEN_G1
    else:
        g = synth.clustered(args.n, seed=synth.BASE_SEED + 4)
        text = synth.MEM_ALIAS
    R = rsm.from_grammar(text, g.labels)
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(R)
    nt_mode = {"auto": cfpq.NT_AUTO, "rows": cfpq.NT_ROWS, "mfma": cfpq.NT_MFMA}[args.nt_mode]
    rs, dt = timed(lambda: cfpq.query(graph, q, strategy=cfpq.STRATEGY_LEVELS, tile_words=args.tile_words,
                                      profile=True, nt_mode=nt_mode, recompute=args.recompute),
                   args.steps, args.warmup)
    r = rs[-1]
    it, deltas, ms = r.stats()
    pairs = r.count(0)
    lv = r.profile(cfpq.KERNEL_LEVEL)
    sd = r.profile(cfpq.KERNEL_SEED)
    wb = r.profile(cfpq.KERNEL_WRITEBACK)
    mf = r.profile(cfpq.KERNEL_NT_MFMA)
    sp = r.profile(cfpq.KERNEL_NT_SPARSE)
    achieved = lv[2] / (lv[1] * 1e-3) / 1e9 if lv[1] else 0.0
    out.update({
        "metric": f"reachable pairs/s ({args.workload})", "value": pairs / dt, "unit": "pairs/s",
        "ms_per_step": dt * 1e3,
        "config": {"workload": (f"same-generation G1 on hierarchy n={g.n}" if args.workload == "samegen"
                                else f"memory alias MA on clustered graph n={g.n}"),
                   "n": g.n, "edges": int(len(g.src)), "rsm_states": int(R.n_states), "pairs": pairs,
                   "all_box_pairs": {b: r.count(b) for b in R.box_names}, "iterations": it,
                   "fixpoint_ms": ms, "deltas_head": deltas[:12],
                   "level": {"launches": lv[0], "ms": lv[1], "GB": lv[2] / 1e9},
                   "seed": {"launches": sd[0], "ms": sd[1]}, "writeback": {"launches": wb[0], "ms": wb[1]},
                   "nt_mode": args.nt_mode, "nt_sparse": {"launches": sp[0], "ms": sp[1]},
                   "closure": "recomputed each iteration" if args.recompute else "incremental",
                   "nt_mfma": {"launches": mf[0], "ms": mf[1], "int8_TOPS": mf[2] / (mf[1] * 1e9) if mf[1] else 0.0,
                               "frac_of_int8_peak": mf[2] / (mf[1] * 1e9) / INT8_PEAK_TOPS if mf[1] else 0.0}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_gather<false> (closure frontier level)"},
    })
    return out


def paths_workload(args, out):
    """All paths of at most 20 edges (the bound of the paper's experiment,
    Sec. 4.2) for same-generation G1 on a hierarchy graph, over sampled pairs
    of the relation: time and number of paths per pair."""
    import numpy as np

    import synth
    from paper_2103_14688_amd import cfpq, rsm

    n = min(args.n, 4000)
    g, _ = synth.hierarchy(n, seed=synth.BASE_SEED + 3)
    R = rsm.from_grammar(synth.SAME_GEN_G1, g.labels)
    res = cfpq.query(cfpq.Graph.from_synth(g), cfpq.Query(R), keep_rank=True)
    pairs = res.pairs(0)
    rng = np.random.default_rng(synth.BASE_SEED + 11)
    pick = pairs[rng.choice(len(pairs), size=min(200, len(pairs)), replace=False)]
    times, counts, edges = [], [], 0
    for u, v in pick.tolist():
        t0 = time.perf_counter()
        k = 0
        for p in res.paths(int(u), int(v), 20):
            k += 1
            edges += len(p)
        times.append(time.perf_counter() - t0)
        counts.append(k)
    total = sum(times)
    out.update({
        "metric": "paths extracted per second (all paths of at most 20 edges per pair)",
        "value": sum(counts) / total if total else 0.0, "unit": "paths/s", "ms_per_step": 1e3 * total / len(pick),
        "config": {"workload": f"same-generation G1 on hierarchy n={n}, all paths of <= 20 edges for "
                               f"{len(pick)} sampled pairs of the relation", "n": n, "pairs_in_relation": len(pairs),
                   "ms_per_pair_mean": 1e3 * total / len(pick), "ms_per_pair_max": 1e3 * max(times),
                   "paths_per_pair_mean": float(np.mean(counts)), "paths_per_pair_max": int(max(counts)),
                   "edges_returned": edges},
    })
    return out


def measure_serving(args):
    """Batched vs plain on the serving mix: 64 resident power-law graphs
    (n log-uniform in [1000, serve_nmax], mean out-degree 3, 8 Zipf labels),
    random regex / normal-form grammar queries.  Closed loop (all requests at
    t = 0) gives throughput; open loops with Poisson arrivals at 0.5, 1, 2 and
    4 times the plain throughput give p50/p99 latency.  Every batched answer
    is compared with the plain one (count, hash, iterations)."""
    import numpy as np

    import synth
    from paper_2103_14688_amd import cfpq, rsm, serve

    labels, recipes, qs = synth.serving_mix(n_graphs=64, n_queries=args.serve_queries,
                                            n_range=(1000, args.serve_nmax))
    graphs = [synth.serving_graph(n, seed, labels) for n, seed in recipes]
    handles = [cfpq.Graph.from_synth(g) for g in graphs]
    print(f"# serving: {len(graphs)} graphs resident", file=sys.stderr, flush=True)
    comp = []
    for gi, kind, text in qs:
        R = rsm.from_regex(text, labels) if kind == "regex" else rsm.from_grammar(text, labels)
        comp.append((gi, R, cfpq.Query(R)))
        if len(comp) % 1000 == 0:
            print(f"# serving: {len(comp)} queries compiled", file=sys.stderr, flush=True)

    def requests():
        return [serve.Request(i, handles[gi], q, graphs[gi].n, R.n_states, R.n_boxes)
                for i, (gi, R, q) in enumerate(comp)]

    backend = serve.GpuBackend()

    def run(mode, arrivals=None):
        srv = serve.Server(backend, mode=mode, slots=args.serve_slots)
        rs = requests()
        t0 = time.perf_counter()
        if arrivals is None:
            for r in rs:
                srv.submit(r)
            # report every 1000 finished requests (long mixes run for minutes)
            shown = 0
            while True:
                try:
                    srv.drain(timeout=1.0)
                    break
                except TimeoutError:
                    done = len(srv.finished) // 1000
                    if done > shown:
                        shown = done
                        print(f"# serving {mode}: {done * 1000} finished", file=sys.stderr, flush=True)
        else:
            serve.replay(srv, rs, arrivals,
                         report=lambda k: print(f"# serving {mode} open loop: {k} submitted", file=sys.stderr,
                                                flush=True))
        wall = time.perf_counter() - t0
        srv.close()
        bad = [r.error for r in rs if r.error]
        assert not bad, bad[:3]
        return rs, wall, srv

    print(f"# serving: {len(comp)} queries on 64 graphs, n <= {args.serve_nmax}", file=sys.stderr, flush=True)
    run("batched")                                   # warm-up (allocator, code objects)
    print("# serving: warm-up done", file=sys.stderr, flush=True)
    plain, wall_p, _ = run("plain")
    print(f"# serving: plain closed loop {wall_p:.1f} s", file=sys.stderr, flush=True)
    batched, wall_b, srv_b = run("batched")
    print(f"# serving: batched closed loop {wall_b:.1f} s", file=sys.stderr, flush=True)
    same = all(a.result == b.result for a, b in zip(plain, batched))
    pairs = sum(r.result[0] for r in plain)
    mu = len(plain) / wall_p
    same_open = True
    sweep = []
    for factor in [float(x) for x in args.serve_rates.split(",") if x]:
        lam = factor * mu
        arr = np.cumsum(np.random.default_rng(synth.BASE_SEED + 9).exponential(1.0 / lam, size=len(comp)))
        plain_o, _, _ = run("plain", arr)
        batched_o, _, _ = run("batched", arr)
        pp = serve.percentiles([r.latency for r in plain_o])
        pb = serve.percentiles([r.latency for r in batched_o])
        same_open &= all(a.result == b.result for a, b in zip(plain_o, batched_o))
        sweep.append({"arrival_rate_per_s": lam, "x_plain_capacity": factor,
                      "plain_p50_ms": pp[50] * 1e3, "plain_p99_ms": pp[99] * 1e3,
                      "batched_p50_ms": pb[50] * 1e3, "batched_p99_ms": pb[99] * 1e3})
        print(f"# serving open loop {factor}x: plain p50/p99 {pp[50] * 1e3:.1f}/{pp[99] * 1e3:.1f} ms, "
              f"batched {pb[50] * 1e3:.1f}/{pb[99] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return {
        "workload": f"{len(comp)} queries (half regex, half CFG) on 64 resident power-law graphs, "
                    f"n log-uniform in [1000, {args.serve_nmax}]",
        "slots": args.serve_slots,
        "closed_loop": {
            "plain_queries_per_s": mu, "batched_queries_per_s": len(batched) / wall_b,
            "plain_pairs_per_s": pairs / wall_p, "batched_pairs_per_s": pairs / wall_b,
            "speedup": wall_p / wall_b, "batched_launch_groups": srv_b.batches,
            "max_concurrent_slots": srv_b.max_concurrent,
        },
        "open_loop": sweep,
        "answers_identical_alone_vs_mix": same and same_open,
        "total_pairs": pairs,
    }


if __name__ == "__main__":
    main()
