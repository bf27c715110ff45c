"""Benchmark: the Kronecker-product fixpoint on one MI355X.

Headline (the JSON line's "value"): reachable pairs per second of the plain
single query on the RPQ workload -- (a|b)* c d* compiled to its minimal
automaton, on a seeded power-law directed graph, n = 100,000, out-degrees
round(Pareto(2.1)) with mean 4, uniform targets, labels Zipf(1.2) over
{a, b, c, d}.  One step = one whole query (every step of the hot path:
staging of the query tables, the Kronecker seed, the closure, the write-back
and the fixpoint test); the graph is resident in HBM before timing starts,
as the paper excludes graph loading from its timings.

The line also carries, under config.workloads, one block per measured
workload, each with its own roofline for its dominant kernel and its own
CPU-oracle baseline:
  brackets_n256        S -> a S b | a b on Erdos-Renyi n = 256 (plain, fused,
                       1024 queries in one fused launch)
  rpq_four_state       the headline query with a 4-state automaton
  samegen_n50000/200000  same-generation G1 on the hierarchy graph
  alias_n20000         memory alias on the clustered graph
  serving              the batched-serving mix, plain vs batched
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of a kernel from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE passes (each scaled by the same counter's reading on a 1 GiB copy
# kernel: fetch x2.0, write x1.0), keyed by (digest of the kernel sources,
# workload, kernel).  Any change to a kernel source changes the digest, and
# the figure is reported as null until the counters are taken again.
# Taken with `rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE` passes over
# the bench commands in profiles/ (k_cond_level: the headline run's 7 queries
# of 18 productive level launches each; the grammar blocks: every launch of
# the block's runs, without the autotuner's).
PMC_TRAFFIC = {
    ("42c7087aab9f7720", "rpq_powerlaw_n100000", "k_cond_level"): 101210941,
    ("42c7087aab9f7720", "samegen_n200000", "k_nt_sparse"): 498617806,
    ("42c7087aab9f7720", "alias_n20000", "k_nt_dense"): 76436347,
    ("42c7087aab9f7720", "samegen_n50000", "k_writeback"): 232384853,
}


def source_digest():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2103_14688_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def host_info():
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    info["ram_gb"] = round(int(line.split()[1]) / 1e6, 1)
                    break
    except OSError:
        pass
    return info


def cpu_threads():
    """Threads for the oracle's all-thread timing: the CPU share the process
    may run on (sched affinity), unless CFPQ_BENCH_THREADS says otherwise."""
    env = os.environ.get("CFPQ_BENCH_THREADS")
    return int(env) if env else len(os.sched_getaffinity(0))


def roofline(kernel, launches, ms, nbytes, workload):
    """HBM roofline of one kernel from its launches in the timed steps: the
    bytes its algorithm reads and writes per launch over its average launch
    duration (HIP events around each launch on the query stream)."""
    avg_ms = ms / launches if launches else 0.0
    per_launch = nbytes / launches if launches else 0.0
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "kernel": kernel, "launches": launches, "avg_launch_ms": avg_ms,
            "algorithmic_bytes_per_launch": per_launch,
            "traffic": PMC_TRAFFIC.get((source_digest(), workload, kernel))}


def timed_queries(fn, steps, warmup, collect=None):
    """Runs fn() steps times after warmup runs; each result's collect(r) is
    kept and the result released when the next one exists (a steady query
    loop).  Returns (collected, seconds per step, last result, still open)."""
    import torch
    for _ in range(warmup):
        fn().close()
    torch.cuda.synchronize()
    out = []
    t0 = time.perf_counter()
    last = None
    for _ in range(steps):
        r = fn()
        out.append(collect(r) if collect else None)
        if last is not None:
            last.close()
        last = r
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) / steps, last


# ---------------------------------------------------------------------------
# headline: RPQ on the power-law graph, plain single query
# ---------------------------------------------------------------------------

def headline(args):
    import numpy as np
    import synth
    from paper_2103_14688_amd import cfpq, rsm

    g = synth.powerlaw(args.n, seed=synth.BASE_SEED + 2)
    R = rsm.from_regex(synth.RPQ_C2, g.labels)
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(R)
    strat = {"auto": cfpq.STRATEGY_AUTO, "levels": cfpq.STRATEGY_LEVELS,
             "condensed": cfpq.STRATEGY_CONDENSED}[args.strategy]
    kw = dict(strategy=strat, tile_words=args.tile_words)
    dominant = cfpq.KERNEL_LEVEL if args.strategy == "levels" else cfpq.KERNEL_COND_LEVEL
    print(f"# headline: graph n={g.n} m={len(g.src)} states={R.n_states}", file=sys.stderr, flush=True)

    # the first query on a fresh graph handle (launch chains sized from fixed
    # hints, several host reads), then the steady loop
    torch_sync()
    t = time.perf_counter()
    r0 = cfpq.query(graph, q, **kw)
    torch_sync()
    cold_ms = (time.perf_counter() - t) * 1e3
    r0.close()
    for _ in range(args.warmup):
        cfpq.query(graph, q, **kw).close()
    torch_sync()
    rows, last = [], None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = cfpq.query(graph, q, profile=True, **kw)
        rows.append((r.stats(), r.profile(dominant), r.profile(cfpq.KERNEL_WRITEBACK), r.profile(cfpq.KERNEL_COND_SCC)))
        if last is not None:
            last.close()
        last = r
    torch_sync()
    wall = time.perf_counter() - t0
    pairs = last.count(0)
    it = rows[-1][0][0]
    fix = [x[0][2] for x in rows]
    lv_n = sum(x[1][0] for x in rows)
    lv_ms = sum(x[1][1] for x in rows)
    lv_by = sum(x[1][2] for x in rows)
    last.close()
    kernel = "k_gather<false>" if args.strategy == "levels" else "k_cond_level"
    roof = roofline(kernel, lv_n, lv_ms, lv_by, "rpq_powerlaw_n100000")

    cpu = None
    if not args.no_cpu:
        import oracle
        th = cpu_threads()
        rng = np.random.default_rng(synth.BASE_SEED + 7)
        srcs = np.sort(rng.choice(g.n, size=min(args.cpu_sources, g.n), replace=False)).astype(np.uint32)
        tc = time.perf_counter()
        rows_o = oracle.rpq_rows(g.n, g.src, g.lbl, g.dst, g.labels, synth.RPQ_C2, srcs, threads=th)
        dt = time.perf_counter() - tc
        cpu_pairs = int(np.unpackbits(rows_o.view(np.uint8)).sum())
        one = srcs[: max(1, len(srcs) // (8 * th))]
        tc = time.perf_counter()
        rows_1 = oracle.rpq_rows(g.n, g.src, g.lbl, g.dst, g.labels, synth.RPQ_C2, one, threads=1)
        dt1 = time.perf_counter() - tc
        pairs_1 = int(np.unpackbits(rows_1.view(np.uint8)).sum())
        cpu = {"value": cpu_pairs / dt, "unit": "pairs/s", "cores": th, "kind": "oracle",
               "sample": f"{len(srcs)} of {g.n} sources (product-automaton BFS per source), "
                         f"{cpu_pairs} pairs in {dt:.2f} s on {th} threads",
               "value_1thread": pairs_1 / dt1,
               "sample_1thread": f"{len(one)} sources, {pairs_1} pairs in {dt1:.2f} s",
               "host": host_info()}
    return {
        "value": pairs * args.steps / wall, "ms_per_step": wall / args.steps * 1e3,
        "config": {"workload": f"RPQ (a|b)* c d* on power-law graph n={g.n} (Pareto(2.1) out-degree mean 4, "
                               f"Zipf(1.2) labels), plain one-query-at-a-time path",
                   "n": g.n, "edges": int(len(g.src)), "rsm_states": int(R.n_states), "pairs": int(pairs),
                   "iterations": it, "fixpoint_ms_median": float(np.median(fix)),
                   "fixpoint_ms_mean": float(np.mean(fix)), "first_query_ms": cold_ms,
                   "tile_words": args.tile_words, "strategy": args.strategy,
                   "level_launches_per_step": lv_n / args.steps,
                   "search_and_setup_ms_per_step": sum(x[3][1] for x in rows) / args.steps,
                   "writeback_ms_per_step": sum(x[2][1] for x in rows) / args.steps},
        "roofline": roof, "cpu_baseline": cpu,
    }


def torch_sync():
    import torch
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# the other workloads
# ---------------------------------------------------------------------------

def block_rpq_four_state(args):
    """The headline query with a 4-state (non-minimal) automaton: the same
    relation, twice the product nodes."""
    import numpy as np
    import synth
    from paper_2103_14688_amd import cfpq, rsm

    g = synth.powerlaw(args.n, seed=synth.BASE_SEED + 2)
    graph = cfpq.Graph.from_synth(g)
    R = rsm.from_automaton(*synth.RPQ_C2_FOUR_STATE, g.labels)
    q = cfpq.Query(R)
    prof, dt, r = timed_queries(lambda: cfpq.query(graph, q, profile=True), max(3, args.steps // 2), 2,
                                lambda x: x.profile(cfpq.KERNEL_COND_LEVEL))
    n_l = sum(x[0] for x in prof)
    ms_l = sum(x[1] for x in prof)
    by_l = sum(x[2] for x in prof)
    out = {"workload": f"RPQ (a|b)* c d* as a 4-state automaton on the same power-law graph n={g.n}",
           "rsm_states": int(R.n_states), "pairs": r.count(0), "ms_per_query": dt * 1e3,
           "pairs_per_s": r.count(0) / dt, "fixpoint_ms": r.stats()[2], "level_launches_per_query": n_l / len(prof),
           "roofline": roofline("k_cond_level", n_l, ms_l, by_l, "rpq_four_state")}
    r.close()
    return out


def block_brackets(args):
    import numpy as np
    import oracle
    import synth
    from paper_2103_14688_amd import cfpq, rsm

    g = synth.erdos_renyi(256, seed=synth.BASE_SEED + 1)
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(rsm.from_grammar(synth.BRACKETS, g.labels))
    res = {"workload": "S -> a S b | a b on directed Erdos-Renyi n=256, p=2/n per label (each ordered pair, "
                       "self-pairs included)"}
    for name, st in (("levels", cfpq.STRATEGY_LEVELS), ("fused", cfpq.STRATEGY_FUSED)):
        _, dt, r = timed_queries(lambda: cfpq.query(graph, q, strategy=st), 20, 3)
        it, deltas, ms = r.stats()
        res[name] = {"ms_per_query_wall": dt * 1e3, "fixpoint_ms": ms, "iterations": it,
                     "us_per_iteration": ms * 1e3 / it, "kernel_over_wall": ms / (dt * 1e3),
                     "pairs": r.count(0)}
        r.close()
    gs = [synth.erdos_renyi(256, seed=synth.BASE_SEED + 1000 + i) for i in range(1024)]
    hs = [cfpq.Graph.from_synth(x) for x in gs]
    qs = [q] * len(hs)
    import torch
    for _ in range(2):
        for r in cfpq.query_batch(hs, qs):
            r.close()
    torch.cuda.synchronize()
    t = time.perf_counter()
    rs = cfpq.query_batch(hs, qs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    pairs = sum(r.count(0) for r in rs)
    res["batched_1024"] = {"ms_per_batch_wall": dt * 1e3, "queries_per_s": 1024 / dt, "pairs_per_s": pairs / dt,
                           "pairs": pairs}
    res["roofline"] = {"bound": "latency",
                       "note": "one workgroup runs the whole fixpoint with its working set (112 KiB) in LDS, "
                               "so neither HBM nor the matrix cores bound it: us per iteration is the figure"}
    if not args.no_autotune:
        res["autotuned"] = autotune_report(graph, q)
    if not args.no_cpu:
        tc = time.perf_counter()
        k = 0
        while time.perf_counter() - tc < 2.0:
            oracle.cfl_reach(g.n, g.src, g.lbl, g.dst, g.labels, synth.BRACKETS)
            k += 1
        dt = (time.perf_counter() - tc) / k
        res["cpu_baseline"] = {"value": res["levels"]["pairs"] / dt, "unit": "pairs/s", "cores": 1, "kind": "oracle",
                               "sample": f"the whole query (worklist over the normal form), {k} runs, "
                                         f"{dt * 1e3:.2f} ms each on 1 thread"}
    return res


def autotune_report(graph, q):
    """What the autotuner picks for this query's class, measured afresh
    (a cache file of its own, removed afterwards): every candidate's time
    and the choice."""
    import tempfile
    from paper_2103_14688_amd import cfpq, tune
    names = {cfpq.STRATEGY_FUSED: "fused", cfpq.STRATEGY_LEVELS: "levels", cfpq.STRATEGY_CONDENSED: "condensed",
             cfpq.STRATEGY_PEREDGE: "peredge"}

    def label(o):
        parts = [names.get(o.get("strategy"), str(o.get("strategy")))]
        if "nt_mode" in o:
            parts.append({cfpq.NT_AUTO: "sparse", cfpq.NT_ROWS: "rows", cfpq.NT_MFMA: "mfma"}[o["nt_mode"]])
        if o.get("tile_words"):
            parts.append(f"tile{o['tile_words']}")
        if o.get("recompute"):
            parts.append("recomputed")
        return "/".join(parts)

    with tempfile.TemporaryDirectory() as d:
        t = tune.Tuner(os.path.join(d, "tune.json"), runs=2)
        opts, entry = t.tune(graph, q)
    return {"class": tune.key_of(entry["features"]), "choice": label(opts),
            "measured_ms": {label(m["options"]): m["ms"] for m in entry["measured"]}}


def block_grammar(args, which, n, steps, warmup, cpu_n):
    """Same-generation G1 on the hierarchy graph or memory alias on the
    clustered graph: levels strategy, every kernel profiled; the dominant
    kernel (most time) gets the roofline."""
    import numpy as np
    import oracle
    import synth
    from paper_2103_14688_amd import cfpq, rsm

    if which == "samegen":
        g = synth.hierarchy(n, seed=synth.BASE_SEED + 3)[0]
        text = synth.SAME_GEN_G1
        desc = f"same-generation G1 on hierarchy graph n={n} (Poisson(4) tree, 20% type edges, inverses)"
    else:
        g = synth.clustered(n, seed=synth.BASE_SEED + 4)
        text = synth.MEM_ALIAS
        desc = f"memory alias MA on clustered program-like graph n={n} (clusters of 64..512 vertices)"
    R = rsm.from_grammar(text, g.labels)
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(R)
    nt_mode = {"auto": cfpq.NT_AUTO, "rows": cfpq.NT_ROWS, "mfma": cfpq.NT_MFMA}[args.nt_mode]
    print(f"# {which} n={n}: {len(g.src)} edges, {R.n_states} states", file=sys.stderr, flush=True)
    kinds = {"k_gather<true> (seed)": cfpq.KERNEL_SEED, "k_gather<false> (level)": cfpq.KERNEL_LEVEL,
             "k_nt_sparse": cfpq.KERNEL_NT_SPARSE, "k_nt_dense": cfpq.KERNEL_NT_DENSE,
             "k_ell_build": cfpq.KERNEL_ELL, "k_writeback": cfpq.KERNEL_WRITEBACK,
             "k_nt_mfma": cfpq.KERNEL_NT_MFMA}
    per, dt, r = timed_queries(lambda: cfpq.query(graph, q, strategy=cfpq.STRATEGY_LEVELS, profile=True,
                                                  nt_mode=nt_mode, recompute=args.recompute,
                                                  tile_words=args.tile_words), steps, warmup,
                               lambda x: {name: x.profile(kind) for name, kind in kinds.items()})
    prof = {name: [sum(p[name][i] for p in per) for i in range(3)] for name in kinds}
    rs = per
    it, deltas, ms = r.stats()
    pairs = r.count(0)
    counted = {k: v for k, v in prof.items() if k not in ("k_gather<true> (seed)", "k_ell_build", "k_nt_mfma")}
    dom = max(counted, key=lambda k: counted[k][1])
    out = {"workload": desc, "n": n, "edges": int(len(g.src)), "rsm_states": int(R.n_states), "pairs": pairs,
           "all_box_pairs": {b: r.count(b) for b in R.box_names}, "iterations": it, "ms_per_query": dt * 1e3,
           "pairs_per_s": pairs / dt, "fixpoint_ms": ms,
           "kernels_ms_per_query": {k: v[1] / len(rs) for k, v in prof.items()},
           "kernel_launches_per_query": {k: v[0] / len(rs) for k, v in prof.items()},
           "closure": "recomputed each iteration" if args.recompute else "incremental", "nt_mode": args.nt_mode,
           "roofline": roofline(dom.split(" ")[0], prof[dom][0], prof[dom][1], prof[dom][2], f"{which}_n{n}")}
    r.close()
    if not args.no_autotune and n <= 50000:
        out["autotuned"] = autotune_report(graph, q)
    if cpu_n and not args.no_cpu:
        if which == "samegen":
            gc = synth.hierarchy(cpu_n, seed=synth.BASE_SEED + 3)[0]
        else:
            gc = synth.clustered(cpu_n, seed=synth.BASE_SEED + 4)
        th = cpu_threads()
        res = {}
        for t in (th, 1):
            tc = time.perf_counter()
            rel, _ = oracle.cfl_reach_rounds(gc.n, gc.src, gc.lbl, gc.dst, gc.labels, text, ["S"], threads=t,
                                             bitmaps=False)
            res[t] = (rel["S"][0], time.perf_counter() - tc)
        out["cpu_baseline"] = {"value": res[th][0] / res[th][1], "unit": "pairs/s", "cores": th, "kind": "oracle",
                               "sample": f"the whole query on the same generator at n={cpu_n} (semi-naive rounds "
                                         f"over bitsets): {res[th][0]} pairs in {res[th][1]:.2f} s on {th} threads",
                               "value_1thread": res[1][0] / res[1][1],
                               "sample_1thread": f"same, {res[1][1]:.2f} s on 1 thread", "host": host_info()}
    return out


def block_serving(args):
    """Batched vs plain on the serving mix: 64 resident power-law graphs
    (n log-uniform in [1e3, 2e5], mean out-degree 3, 8 Zipf labels), random
    regular and context-free queries, Poisson arrivals.  The mix's first
    serve_queries requests are served (see the cut below); every batched
    answer is compared with the plain one (count, hash, iterations)."""
    import numpy as np
    import synth
    from paper_2103_14688_amd import cfpq, rsm, serve

    labels, recipes, qs = synth.serving_mix(n_graphs=64, n_queries=10000, n_range=(1000, args.serve_nmax))
    use = [i for i, (gi, _, _) in enumerate(qs) if recipes[gi][0] <= args.serve_cut_n][: args.serve_queries]
    gids = sorted({qs[i][0] for i in use})
    graphs = {gi: synth.serving_graph(*recipes[gi], labels) for gi in gids}
    handles = {gi: cfpq.Graph.from_synth(graphs[gi]) for gi in gids}
    print(f"# serving: {len(use)} queries on {len(gids)} resident graphs", file=sys.stderr, flush=True)
    comp = []
    for i in use:
        gi, kind, text = qs[i]
        R = rsm.from_regex(text, labels) if kind == "regex" else rsm.from_grammar(text, labels)
        comp.append((gi, R, cfpq.Query(R)))

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
            srv.drain()
        else:
            serve.replay(srv, rs, arrivals)
        wall = time.perf_counter() - t0
        srv.close()
        bad = [r.error for r in rs if r.error]
        assert not bad, bad[:3]
        return rs, wall, srv

    run("batched")   # warm-up
    plain, wall_p, _ = run("plain")
    batched, wall_b, srv_b = run("batched")
    print(f"# serving: closed loop plain {wall_p:.1f} s, batched {wall_b:.1f} s", file=sys.stderr, flush=True)
    same = all(a.result == b.result for a, b in zip(plain, batched))
    pairs = sum(r.result[0] for r in plain)
    mu = len(plain) / wall_p
    sweep = []
    for factor in [float(x) for x in args.serve_rates.split(",") if x]:
        lam = factor * mu
        arr = np.cumsum(np.random.default_rng(synth.BASE_SEED + 9).exponential(1.0 / lam, size=len(comp)))
        plain_o, _, _ = run("plain", arr)
        batched_o, _, _ = run("batched", arr)
        pp = serve.percentiles([r.latency for r in plain_o])
        pb = serve.percentiles([r.latency for r in batched_o])
        same &= all(a.result == b.result for a, b in zip(plain_o, batched_o))
        sweep.append({"arrival_rate_per_s": lam, "x_plain_capacity": factor,
                      "plain_p50_ms": pp[50] * 1e3, "plain_p99_ms": pp[99] * 1e3,
                      "batched_p50_ms": pb[50] * 1e3, "batched_p99_ms": pb[99] * 1e3})
        print(f"# serving open loop {factor}x: plain p50/p99 {pp[50] * 1e3:.1f}/{pp[99] * 1e3:.1f} ms, "
              f"batched {pb[50] * 1e3:.1f}/{pb[99] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    return {
        "workload": f"serving mix: 64 power-law graphs with n log-uniform in [1000, {args.serve_nmax}], 10,000 "
                    f"queries (half random regexes, half random grammars with 2-6 nonterminals)",
        "cut": f"the first {len(use)} queries of the mix whose graph has at most {args.serve_cut_n} vertices "
               f"({len(gids)} graphs resident)",
        "slots": args.serve_slots,
        "closed_loop": {"plain_queries_per_s": mu, "batched_queries_per_s": len(batched) / wall_b,
                        "plain_pairs_per_s": pairs / wall_p, "batched_pairs_per_s": pairs / wall_b,
                        "speedup": wall_p / wall_b, "batched_launch_groups": srv_b.batches,
                        "max_concurrent_slots": srv_b.max_concurrent},
        "open_loop": sweep, "answers_identical_alone_vs_mix": same, "total_pairs": pairs,
    }


def paths_workload(args):
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
    return {"workload": f"same-generation G1 on hierarchy n={n}, all paths of <= 20 edges for {len(pick)} "
                        f"sampled pairs of the relation", "n": n, "pairs_in_relation": len(pairs),
            "paths_per_s": sum(counts) / total if total else 0.0, "ms_per_pair_mean": 1e3 * total / len(pick),
            "ms_per_pair_max": 1e3 * max(times), "paths_per_pair_mean": float(np.mean(counts)),
            "paths_per_pair_max": int(max(counts)), "edges_returned": edges}


def peredge_workload(args):
    """The closure arms on small instances of the workloads: the literal
    per-edge insertion (Sec. 3.1.1), the frontier-incremental levels and the
    closure recomputed from scratch each iteration; ms per query and the
    pairs each found (equal)."""
    import synth
    from paper_2103_14688_amd import cfpq, rsm

    cases = [("brackets n=256", synth.erdos_renyi(256, seed=synth.BASE_SEED + 1), "cfg", synth.BRACKETS),
             ("samegen G1 n=500", synth.hierarchy(500, seed=synth.BASE_SEED + 3)[0], "cfg", synth.SAME_GEN_G1),
             ("samegen G1 n=1000", synth.hierarchy(1000, seed=synth.BASE_SEED + 3)[0], "cfg", synth.SAME_GEN_G1),
             ("alias n=500 (clusters 16..64)", synth.clustered(500, cluster=(16, 64), seed=synth.BASE_SEED + 4),
              "cfg", synth.MEM_ALIAS),
             ("alias n=1000 (clusters 16..64)", synth.clustered(1000, cluster=(16, 64), seed=synth.BASE_SEED + 4),
              "cfg", synth.MEM_ALIAS),
             ("rpq n=5000", synth.powerlaw(5000), "regex", synth.RPQ_C2)]
    out = {"workload": "closure arms: per-edge insertion vs frontier levels vs recomputed", "cases": []}
    for name, g, kind, text in cases:
        R = rsm.from_regex(text, g.labels) if kind == "regex" else rsm.from_grammar(text, g.labels)
        graph, q = cfpq.Graph.from_synth(g), cfpq.Query(R)
        row = {"case": name, "n": g.n, "states": R.n_states}
        arms = [("peredge", {"strategy": cfpq.STRATEGY_PEREDGE}), ("levels", {"strategy": cfpq.STRATEGY_LEVELS})]
        if kind != "regex":
            arms.append(("recomputed", {"strategy": cfpq.STRATEGY_LEVELS, "recompute": True}))
        for label, opts in arms:
            _, dt, r = timed_queries(lambda: cfpq.query(graph, q, **opts), 2, 1)
            row[label] = {"ms": dt * 1e3, "pairs": r.count(0), "iterations": r.stats()[0]}
            r.close()
        print(f"# {json.dumps(row)}", file=sys.stderr, flush=True)
        out["cases"].append(row)
    return out


BLOCKS = ["brackets", "rpq_four_state", "samegen50k", "samegen200k", "alias", "serving"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--tile-words", type=int, default=0)
    ap.add_argument("--strategy", choices=["auto", "levels", "condensed"], default="auto",
                    help="closure strategy of the headline query (auto = condensed for a regular query)")
    ap.add_argument("--nt-mode", choices=["auto", "rows", "mfma"], default="auto",
                    help="grammar workloads: box-labelled transitions in closure levels")
    ap.add_argument("--recompute", action="store_true",
                    help="grammar workloads: recompute the closure from scratch every iteration")
    ap.add_argument("--cpu-sources", type=int, default=20000, help="headline oracle sample (sources)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="blocks skip the autotuner report (profiling runs: only the block's own queries)")
    ap.add_argument("--blocks", default=",".join(BLOCKS),
                    help="workload blocks to add to the line (comma list of " + ",".join(BLOCKS) + ", or none)")
    ap.add_argument("--only", choices=BLOCKS + ["paths", "peredge"], default=None,
                    help="run just this block and print it as the JSON line (no headline)")
    ap.add_argument("--grammar-n", type=int, default=0, help="--only samegen*/alias: graph size override")
    ap.add_argument("--serve-queries", type=int, default=2000)
    ap.add_argument("--serve-nmax", type=int, default=200000)
    ap.add_argument("--serve-cut-n", type=int, default=20000)
    ap.add_argument("--serve-slots", type=int, default=8, help="execution slots (streams) of the batched server")
    ap.add_argument("--serve-rates", default="0.5,1,2,4",
                    help="open-loop arrival rates as multiples of the plain closed-loop throughput")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 3 times (reference kernel for the "
                         "FETCH_SIZE/WRITE_SIZE scale factor) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library has no multi-GPU path "
              f"(one process drives one GPU)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        a = torch.ones(args.calibrate_copy * (1 << 20) // 8, dtype=torch.int64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 8, "copies": 3}), flush=True)
        return

    from paper_2103_14688_amd import cfpq
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cfpq.load()

    def run_block(name):
        print(f"# block {name}", file=sys.stderr, flush=True)
        t = time.perf_counter()
        if name == "brackets":
            out = block_brackets(args)
        elif name == "rpq_four_state":
            out = block_rpq_four_state(args)
        elif name == "samegen50k":
            out = block_grammar(args, "samegen", args.grammar_n or 50000, 5, 1, 20000)
        elif name == "samegen200k":
            out = block_grammar(args, "samegen", args.grammar_n or 200000, 3, 1, 20000)
        elif name == "alias":
            out = block_grammar(args, "alias", args.grammar_n or 20000, 5, 1, 8000)
        elif name == "serving":
            out = block_serving(args)
        elif name == "peredge":
            out = peredge_workload(args)
        else:
            out = paths_workload(args)
        out["block_wall_s"] = time.perf_counter() - t
        return out

    base = {"n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
            "data": "synthetic (seeded generators shaped like the paper's workloads)",
            "kernel_source_digest": source_digest(), "library": cfpq.cfpq_version()}
    if args.only:
        blk = run_block(args.only)
        print(json.dumps({"metric": f"workload block {args.only}", **base, "steps": args.steps,
                          "warmup": args.warmup, "block": blk}), flush=True)
        return

    head = headline(args)
    blocks = {}
    for name in [b for b in args.blocks.split(",") if b and b != "none"]:
        blocks[name] = run_block(name)
    out = {"metric": "reachable pairs/s (fixpoint, plain single query)", "value": head["value"], "unit": "pairs/s",
           **base, "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
           "config": {**head["config"], "workloads": blocks},
           "roofline": head["roofline"], "cpu_baseline": head["cpu_baseline"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
