"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  All arithmetic is Boolean, so every comparison is
bit-exact: pair bitmaps, counts, order-independent hashes, iteration counts
where the paper fixes them."""
import json
import os

import numpy as np
import pytest

import synth
from paper_2103_14688_amd import cfpq, rsm as rsm_mod
from tests import helpers as H

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
STRATS = [cfpq.STRATEGY_LEVELS, cfpq.STRATEGY_FUSED]
RPQ_STRATS = [cfpq.STRATEGY_LEVELS, cfpq.STRATEGY_CONDENSED]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfpq.load()
    yield
    torch.cuda.synchronize()


def run(g, R, **kw):
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(R)
    res = cfpq.query(graph, q, **kw)
    return graph, q, res


def check_box(res, bm_oracle, n, box=0):
    bm = res.bitmap(box)
    assert H.padding_clear(bm, n)
    if not np.array_equal(bm, bm_oracle):
        diff = H.bits_to_pairs(bm, n) ^ H.bits_to_pairs(bm_oracle, n)
        raise AssertionError(f"bitmaps differ in {len(diff)} pairs, e.g. {sorted(diff)[:5]}")
    assert res.count(box) == H.popcount(bm_oracle)
    assert res.hash(box) == H.bitmap_hash(bm_oracle, n)


# ---------------------------------------------------------------------------
# the paper's worked example (Sec. 3.3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("strategy", STRATS)
@pytest.mark.parametrize("figure_rsm", [True, False])
def test_paper_example(strategy, figure_rsm):
    fx = json.load(open(os.path.join(GOLDEN, "paper_example.json")))
    g = synth.make_graph(fx["n"], [tuple(e) for e in fx["edges"]], fx["labels"])
    R = rsm_mod.paper_example_rsm(g.labels) if figure_rsm else rsm_mod.from_grammar(fx["grammar"], g.labels)
    _, _, res = run(g, R, strategy=strategy, keep_rank=True)
    assert {tuple(p) for p in res.pairs(0).tolist()} == {tuple(p) for p in fx["S"]}
    it, deltas, _ = res.stats()
    assert it == fx["iterations"]
    assert deltas == fx["new_nonterminal_edges_per_iteration"]
    # witnesses: valid paths spelling words of the language
    edges = {tuple(e) for e in fx["edges"]}
    for u, v in fx["S"]:
        path = res.extract_path(u, v)
        assert path[0][0] == u and path[-1][2] == v
        word = [g.labels[int(l)] for _, l, _ in path]
        k = len(word) // 2
        assert word == ["a"] * k + ["b"] * k and k >= 1
        assert all((int(a), g.labels[int(l)], int(b)) in edges for a, l, b in path)


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("k", [1, 3, 9])
@pytest.mark.parametrize("strategy", STRATS)
def test_chain_anbn(k, strategy):
    g = synth.chain("a" * k + "b" * k)
    _, _, res = run(g, rsm_mod.from_grammar(synth.BRACKETS, g.labels), strategy=strategy)
    assert {tuple(p) for p in res.pairs(0).tolist()} == {(k - j, k + j) for j in range(1, k + 1)}
    it, deltas, _ = res.stats()
    assert it == k + 1 and deltas == [1] * k + [0]


def test_same_generation_closed_form():
    g, depth = synth.hierarchy(3000, with_type=False, seed=5)
    _, _, res = run(g, rsm_mod.from_grammar(synth.SAME_GEN_SC, g.labels))
    levels = np.bincount(depth)
    assert res.count(0) == int((levels[1:] ** 2).sum())
    bm = res.bitmap(0)
    bits = np.unpackbits(bm.view(np.uint8), axis=1, bitorder="little")[:, :g.n].astype(bool)
    assert np.array_equal(bits, (depth[:, None] == depth[None, :]) & (depth[:, None] >= 1))


# ---------------------------------------------------------------------------
# balanced brackets on Erdos-Renyi n = 256 (the plain single-query workload)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [synth.BASE_SEED + 1] + [synth.BASE_SEED + 1 + 100 + i for i in range(10)])
@pytest.mark.parametrize("strategy", STRATS)
def test_brackets_er256(seed, strategy):
    g = synth.erdos_renyi(256, seed=seed)
    want = H.oracle_grammar(g, synth.BRACKETS)["S"][1]
    _, _, res = run(g, rsm_mod.from_grammar(synth.BRACKETS, g.labels), strategy=strategy)
    check_box(res, want, g.n)


def test_brackets_er256_strategies_same_iterations():
    g = synth.erdos_renyi(256, seed=synth.BASE_SEED + 1)
    R = rsm_mod.from_grammar(synth.BRACKETS, g.labels)
    a = run(g, R, strategy=cfpq.STRATEGY_LEVELS)[2].stats()
    b = run(g, R, strategy=cfpq.STRATEGY_FUSED)[2].stats()
    assert a[0] == b[0] and a[1] == b[1]


# ---------------------------------------------------------------------------
# regular path queries on power-law graphs, with source tiling
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,tile", [(2000, 0), (2000, 1), (2000, 7), (4100, 16), (129, 0), (65, 1)])
@pytest.mark.parametrize("minimize", [True, False])
@pytest.mark.parametrize("strategy", RPQ_STRATS)
def test_rpq_powerlaw(n, tile, minimize, strategy):
    g = synth.powerlaw(n, seed=synth.BASE_SEED + 2 + n)
    want = H.oracle_regex(g, synth.RPQ_C2)
    R = rsm_mod.from_regex(synth.RPQ_C2, g.labels, minimize=minimize)
    _, _, res = run(g, R, strategy=strategy, tile_words=tile, keep_blocks=True)
    check_box(res, want, g.n)
    it, deltas, _ = res.stats()
    # a regular query has one productive iteration (Sec. 3.1.2)
    assert it == 2 and deltas[1] == 0 and deltas[0] == H.popcount(want)
    # the start -> final block equals the answer when the box has one final state
    finals = np.nonzero(R.is_final)[0]
    if len(finals) == 1:
        assert np.array_equal(res.block(int(R.box_start[0]), int(finals[0])), want)


# ---------------------------------------------------------------------------
# the paper's CFPQ workload shapes at oracle-friendly sizes
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("tile", [0, 3])
def test_same_generation_g1(seed, tile):
    g, _ = synth.hierarchy(2500, seed=synth.BASE_SEED + 3 + seed)
    want = H.oracle_grammar(g, synth.SAME_GEN_G1)["S"][1]
    _, _, res = run(g, rsm_mod.from_grammar(synth.SAME_GEN_G1, g.labels), tile_words=tile)
    check_box(res, want, g.n)


def test_same_generation_g2():
    g, _ = synth.hierarchy(2000, seed=synth.BASE_SEED + 33)
    want = H.oracle_grammar(g, synth.SAME_GEN_G2)["S"][1]
    _, _, res = run(g, rsm_mod.from_grammar(synth.SAME_GEN_G2, g.labels))
    check_box(res, want, g.n)


@pytest.mark.parametrize("n", [1500, 4000])
def test_memory_alias(n):
    g = synth.clustered(n, cluster=(16, 64), seed=synth.BASE_SEED + 4 + n)
    want = H.oracle_grammar(g, synth.MEM_ALIAS, ["S", "V"])
    R = rsm_mod.from_grammar(synth.MEM_ALIAS, g.labels)
    _, _, res = run(g, R)
    check_box(res, want["S"][1], g.n, R.box("S"))
    check_box(res, want["V"][1], g.n, R.box("V"))


# ---------------------------------------------------------------------------
# random queries on small random graphs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(24))
def test_random_queries(seed):
    rng = np.random.default_rng(5000 + seed)
    labels = [f"l{i}" for i in range(6)]
    n = int(rng.integers(1, 300))
    g = synth.powerlaw(max(n, 2), labels=tuple(labels), mean_deg=float(rng.uniform(1, 4)), seed=seed) if n > 1 \
        else synth.make_graph(1, [(0, "l0", 0)], labels)
    use = [str(x) for x in rng.choice(labels, size=4, replace=False)]
    if seed % 2:
        text = synth.random_regex(rng, use)
        want = H.oracle_regex(g, text)
        R = rsm_mod.from_regex(text, g.labels)
    else:
        text = synth.random_cfg(rng, use)
        want = H.oracle_grammar(g, text)["N0"][1]
        R = rsm_mod.from_grammar(text, g.labels)
    for strategy in STRATS:
        _, _, res = run(g, R, strategy=strategy)
        check_box(res, want, g.n)


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------
def test_single_vertex_self_loop_nullable():
    g = synth.make_graph(1, [(0, "a", 0)], ["a", "b"])
    for text, want in [("S -> a S | eps", {(0, 0)}), ("S -> b", set()), ("S -> a a a", {(0, 0)})]:
        for strategy in STRATS:
            _, _, res = run(g, rsm_mod.from_grammar(text, g.labels), strategy=strategy)
            assert {tuple(p) for p in res.pairs(0).tolist()} == want, text


def test_empty_graph():
    g = synth.make_graph(70, [], ["a"])
    for text, cnt in [("S -> a S | eps", 70), ("S -> a", 0)]:
        for strategy in STRATS:
            _, _, res = run(g, rsm_mod.from_grammar(text, g.labels), strategy=strategy)
            assert res.count(0) == cnt
            assert H.padding_clear(res.bitmap(0), 70)


def test_query_terminal_missing_from_graph():
    g = synth.powerlaw(300, labels=("a", "b"), seed=3)
    text = "S -> a zz | b"
    want = H.oracle_grammar(g, text)["S"][1]
    _, _, res = run(g, rsm_mod.from_grammar(text, g.labels))
    check_box(res, want, g.n)


def test_max_iters_limit():
    g = synth.chain("aaaabbbb")
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(rsm_mod.from_grammar(synth.BRACKETS, g.labels))
    for strategy in STRATS:
        with pytest.raises(cfpq.CfpqError) as e:
            cfpq.query(graph, q, strategy=strategy, max_iters=2)
        assert e.value.status == cfpq.ERR_LIMIT


# ---------------------------------------------------------------------------
# batch: every result is the same alone and in the mix
# ---------------------------------------------------------------------------
def test_batch_alone_vs_mix():
    rng = np.random.default_rng(77)
    labels = [f"l{i}" for i in range(8)]
    graphs, queries, wants = [], [], []
    for i in range(12):
        n = int(rng.choice([100, 500, 900, 1500]))
        g = synth.powerlaw(n, labels=tuple(labels), mean_deg=3.0, seed=100 + i)
        use = [str(x) for x in rng.choice(labels, size=5, replace=False)]
        text = synth.random_regex(rng, use) if i % 2 else synth.random_cfg(rng, use)
        R = rsm_mod.from_regex(text, labels) if i % 2 else rsm_mod.from_grammar(text, labels)
        graphs.append(cfpq.Graph.from_synth(g))
        queries.append(cfpq.Query(R))
        wants.append((H.oracle_regex(g, text) if i % 2 else H.oracle_grammar(g, text)["N0"][1], n))
    mix = cfpq.query_batch(graphs, queries)
    for (want, n), res, gr, q in zip(wants, mix, graphs, queries):
        alone = cfpq.query(gr, q)
        assert np.array_equal(res.bitmap(0), want)
        assert np.array_equal(alone.bitmap(0), want)
        assert res.stats()[:2] == alone.stats()[:2]


def test_fused_batch_lds_and_global_queries():
    # one fused launch whose small queries run in LDS and whose larger ones
    # (past the per-workgroup LDS) run on their global buffers; the answer
    # matrices share one block, released here out of order
    rng = np.random.default_rng(91)
    labels = ["a", "b", "c", "d"]
    graphs, queries, wants = [], [], []
    for i, n in enumerate([64, 256, 700, 1500, 256, 97]):
        g = synth.powerlaw(n, labels=tuple(labels), mean_deg=3.0, seed=300 + i)
        text = synth.random_cfg(rng, labels) if i % 2 == 0 else "S -> a S b | a b"
        graphs.append(cfpq.Graph.from_synth(g))
        queries.append(cfpq.Query(rsm_mod.from_grammar(text, labels)))
        wants.append(H.oracle_grammar(g, text)["N0" if i % 2 == 0 else "S"][1])
    mix = cfpq.query_batch(graphs, queries, strategy=cfpq.STRATEGY_FUSED)
    for j in (3, 0, 5, 1, 4, 2):
        assert np.array_equal(mix[j].bitmap(0), wants[j]), j
        alone = cfpq.query(graphs[j], queries[j], strategy=cfpq.STRATEGY_FUSED)
        assert mix[j].stats()[:2] == alone.stats()[:2]
        alone.close()
        mix[j].close()


# ---------------------------------------------------------------------------
# full bench size: sampled source rows against the oracle's per-source BFS
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("strategy", RPQ_STRATS)
def test_rpq_bench_size_sampled_rows(strategy):
    import oracle
    g = synth.powerlaw(100000, seed=synth.BASE_SEED + 2)
    R = rsm_mod.from_regex(synth.RPQ_C2, g.labels)
    graph, q, res = run(g, R, strategy=strategy)
    bm = res.bitmap(0)
    assert H.padding_clear(bm, g.n)
    rng = np.random.default_rng(11)
    srcs = np.sort(rng.choice(g.n, size=48, replace=False)).astype(np.uint32)
    srcs = np.concatenate([srcs, np.array([0, g.n - 1], dtype=np.uint32)])
    want = oracle.rpq_rows(g.n, g.src, g.lbl, g.dst, g.labels, synth.RPQ_C2, srcs, threads=8)
    assert np.array_equal(bm[srcs], want)
    # whole-answer invariants: count = popcount = first iteration's delta
    it, deltas, _ = res.stats()
    total = int(np.unpackbits(bm.view(np.uint8)).sum())
    assert res.count(0) == total == deltas[0] and it == 2
    # the same query again on the same graph handle (for the condensed
    # strategy: the one-read path the bench times) gives the same answer
    again = cfpq.query(graph, q, strategy=strategy)
    assert again.count(0) == total and again.hash(0) == res.hash(0)
    assert np.array_equal(again.bitmap(0)[srcs], want)


@pytest.mark.parametrize("n", [30000, 36865, 74000, 120000])
def test_rpq_sampled_rows_uneven_chunks(n):
    # component rows of 469, 577, 1157 and 1875 words: one, two, three and
    # four chunks (at most 576 words each, widths rounded to 16 words, a
    # shorter last chunk), none a multiple of the wavefront's 64 words
    import oracle
    g = synth.powerlaw(n, seed=synth.BASE_SEED + 5)
    R = rsm_mod.from_regex(synth.RPQ_C2, g.labels)
    _, _, res = run(g, R, strategy=cfpq.STRATEGY_CONDENSED)
    bm = res.bitmap(0)
    assert H.padding_clear(bm, g.n)
    rng = np.random.default_rng(n)
    srcs = np.sort(rng.choice(g.n, size=24, replace=False)).astype(np.uint32)
    srcs = np.concatenate([srcs, np.array([0, g.n - 1], dtype=np.uint32)])
    want = oracle.rpq_rows(g.n, g.src, g.lbl, g.dst, g.labels, synth.RPQ_C2, srcs, threads=8)
    assert np.array_equal(bm[srcs], want)
    _, _, lv = run(g, R, strategy=cfpq.STRATEGY_LEVELS)
    assert np.array_equal(lv.bitmap(0), bm)
    assert res.count(0) == int(np.unpackbits(bm.view(np.uint8)).sum())


# ---------------------------------------------------------------------------
# condensed closure (components of the product graph) on regular queries
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(16))
def test_condensed_random_regex(seed):
    rng = np.random.default_rng(7000 + seed)
    labels = [f"l{i}" for i in range(5)]
    n = int(rng.integers(2, 3000))
    g = synth.powerlaw(n, labels=tuple(labels), mean_deg=float(rng.uniform(0.5, 5)), seed=seed)
    text = synth.random_regex(rng, [str(x) for x in rng.choice(labels, size=4, replace=False)])
    want = H.oracle_regex(g, text)
    R = rsm_mod.from_regex(text, g.labels, minimize=bool(seed % 2))
    _, _, res = run(g, R, strategy=cfpq.STRATEGY_CONDENSED, keep_blocks=True)
    check_box(res, want, g.n)
    it, deltas, _ = res.stats()
    assert it == 2 and deltas[1] == 0


@pytest.mark.parametrize("text", ["a*", "(a | b)+", "a b a", "eps", "(a b)* | b", "zz", "a zz"])
def test_condensed_cycles_and_chains(text):
    # a long chain (deep condensation), a ring (one big component), self-loops
    chain = [(i, "a" if i % 3 else "b", i + 1) for i in range(4999)]
    ring = [(5000 + i, "a", 5000 + (i + 1) % 9500) for i in range(9500)]   # one component, 9500 hops round
    loops = [(i, "b", i) for i in range(0, 14500, 97)]
    g = synth.make_graph(14500, chain + ring + loops, ["a", "b"])
    want = H.oracle_regex(g, text)
    R = rsm_mod.from_regex(text, g.labels)
    for strategy in RPQ_STRATS:
        for kw in ({}, {"keep_blocks": True}):
            _, _, res = run(g, R, strategy=strategy, **kw)
            check_box(res, want, g.n)


@pytest.mark.parametrize("seed", range(6))
def test_condensed_repeated_queries_on_one_graph(seed):
    # the first query on a graph handle sizes the launch chains; later ones go
    # out in one piece with those sizes and finish synchronously from the
    # first step the sizes did not cover (searches, colouring, levels)
    rng = np.random.default_rng(9100 + seed)
    labels = [f"l{i}" for i in range(5)]
    n = int(rng.integers(300, 4000))
    g = synth.powerlaw(n, labels=tuple(labels), mean_deg=float(rng.uniform(0.7, 4)), seed=seed + 40)
    graph = cfpq.Graph.from_synth(g)
    texts = [synth.random_regex(rng, [str(x) for x in rng.choice(labels, size=4, replace=False)]) for _ in range(4)]
    want = {t: H.oracle_regex(g, t) for t in texts}
    for text in texts + texts[::-1] + texts:
        res = cfpq.query(graph, cfpq.Query(rsm_mod.from_regex(text, g.labels)), strategy=cfpq.STRATEGY_CONDENSED)
        check_box(res, want[text], g.n)
        assert res.stats()[0] == 2


def test_condensed_repeated_queries_deep_and_shallow():
    # one handle: a shallow query, then a 5000-level chain and a 9500-node
    # ring (chain sizes far too short), then shallow again
    chain = [(i, "a" if i % 3 else "b", i + 1) for i in range(4999)]
    ring = [(5000 + i, "a", 5000 + (i + 1) % 9500) for i in range(9500)]
    loops = [(i, "b", i) for i in range(0, 14500, 97)]
    g = synth.make_graph(14500, chain + ring + loops, ["a", "b"])
    graph = cfpq.Graph.from_synth(g)
    texts = ["b", "a*", "(a | b)+", "b", "a b a", "(a b)* | b", "b"]
    want = {t: H.oracle_regex(g, t) for t in set(texts)}
    for text in texts:
        res = cfpq.query(graph, cfpq.Query(rsm_mod.from_regex(text, g.labels)), strategy=cfpq.STRATEGY_CONDENSED)
        check_box(res, want[text], g.n)


@pytest.mark.parametrize("graph_kind", ["dag", "ring", "empty"])
def test_condensed_repeated_degenerate_queries(graph_kind):
    # one handle: nullable, missing-label and plain queries after each other
    # on a graph that trimming empties (a DAG), one big cycle, or no edges
    if graph_kind == "dag":
        edges = [(i, "a" if i % 2 else "b", j) for i in range(200) for j in (i + 1, i + 7) if j < 200]
    elif graph_kind == "ring":
        edges = [(i, "a" if i % 3 else "b", (i + 1) % 300) for i in range(300)]
    else:
        edges = []
    n = {"dag": 200, "ring": 300, "empty": 50}[graph_kind]
    g = synth.make_graph(n, edges, ["a", "b"])
    graph = cfpq.Graph.from_synth(g)
    texts = ["a*", "eps", "(a | b)+", "zz", "a b* | b", "a*", "(a b)*", "eps", "(a | b)+"]
    want = {t: H.oracle_regex(g, t) for t in set(texts)}
    for text in texts:
        res = cfpq.query(graph, cfpq.Query(rsm_mod.from_regex(text, g.labels)), strategy=cfpq.STRATEGY_CONDENSED)
        check_box(res, want[text], g.n)


def test_condensed_rejects_grammars():
    g = synth.chain("aabb")
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(rsm_mod.from_grammar(synth.BRACKETS, g.labels))
    with pytest.raises(cfpq.CfpqError) as e:
        cfpq.query(graph, q, strategy=cfpq.STRATEGY_CONDENSED)
    assert e.value.status == cfpq.ERR_INVALID


def test_condensed_and_levels_agree_with_witnesses():
    g = synth.powerlaw(1500, seed=21)
    R = rsm_mod.from_regex(synth.RPQ_C2, g.labels)
    _, _, a = run(g, R, strategy=cfpq.STRATEGY_CONDENSED, keep_rank=True)
    _, _, b = run(g, R, strategy=cfpq.STRATEGY_LEVELS)
    assert np.array_equal(a.bitmap(0), b.bitmap(0))
    assert a.stats()[:2] == b.stats()[:2]
    pairs = a.pairs(0)
    import re
    pat = re.compile("(a|b)*cd*")
    edges = set(zip(g.src.tolist(), g.lbl.tolist(), g.dst.tolist()))
    for u, v in pairs[:: max(1, len(pairs) // 20)].tolist():
        path = a.extract_path(u, v)
        assert path[0][0] == u and path[-1][2] == v
        assert all((int(x), int(l), int(y)) in edges for x, l, y in path)
        assert pat.fullmatch("".join(g.labels[int(l)] for _, l, _ in path))


# ---------------------------------------------------------------------------
# nonterminal product: sparse rows (ELL + LDS accumulator) in the seed,
# whole-row OR, and the int8 matrix-core product in the closure levels
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["samegen", "alias", "brackets", "random0", "random1", "random2"])
def test_nonterminal_product_modes_agree(case):
    rng = np.random.default_rng(sum(map(ord, case)))
    if case == "samegen":
        g, _ = synth.hierarchy(3000, seed=31)
        text = synth.SAME_GEN_G1
    elif case == "alias":
        g = synth.clustered(2500, cluster=(16, 64), seed=32)
        text = synth.MEM_ALIAS
    elif case == "brackets":
        g = synth.erdos_renyi(700, seed=33)
        text = synth.BRACKETS
    else:
        labels = [f"l{i}" for i in range(6)]
        g = synth.powerlaw(1200, labels=tuple(labels), mean_deg=2.5, seed=34 + int(case[-1]))
        text = synth.random_cfg(rng, [str(x) for x in rng.choice(labels, size=4, replace=False)])
    R = rsm_mod.from_grammar(text, g.labels)
    start = R.box_names[0]
    want = H.oracle_grammar(g, text)[start][1]
    outs = []
    for mode in (cfpq.NT_AUTO, cfpq.NT_ROWS, cfpq.NT_MFMA):
        for tile in (0, 5, 20):
            graph = cfpq.Graph.from_synth(g)
            q = cfpq.Query(R)
            res = cfpq.query(graph, q, strategy=cfpq.STRATEGY_LEVELS, tile_words=tile, nt_mode=mode)
            check_box(res, want, g.n)
            outs.append(res.stats()[:2])
    assert all(o == outs[0] for o in outs)


# int8 matrix-core product in every closure level: target rows in 128-row
# wavefront tasks, so sizes below, at and past a task boundary with a ragged
# tail, tiles of 1, 3 and all source words, and relations dense enough that
# most 64 x 64 blocks are live
@pytest.mark.parametrize("n,tile", [(1, 0), (63, 0), (128, 0), (129, 1), (300, 3), (777, 0), (1100, 5)])
def test_mfma_product_brackets_er(n, tile):
    g = synth.erdos_renyi(n, p=min(1.0, 3.0 / max(n, 1)), seed=40 + n)
    want = H.oracle_grammar(g, synth.BRACKETS)["S"][1]
    R = rsm_mod.from_grammar(synth.BRACKETS, g.labels)
    _, _, res = run(g, R, strategy=cfpq.STRATEGY_LEVELS, tile_words=tile, nt_mode=cfpq.NT_MFMA)
    check_box(res, want, g.n)
    _, _, ref = run(g, R, strategy=cfpq.STRATEGY_LEVELS, tile_words=tile, nt_mode=cfpq.NT_ROWS)
    assert res.stats()[:2] == ref.stats()[:2]


@pytest.mark.parametrize("k", [64, 150])
def test_mfma_product_nested_chain(k):
    # a^k b^k on a path: one nesting depth per iteration, k + 1 iterations
    g = synth.chain("a" * k + "b" * k)
    want = H.oracle_grammar(g, synth.BRACKETS)["S"][1]
    R = rsm_mod.from_grammar(synth.BRACKETS, g.labels)
    _, _, res = run(g, R, strategy=cfpq.STRATEGY_LEVELS, nt_mode=cfpq.NT_MFMA)
    check_box(res, want, g.n)
    assert res.stats()[0] == k + 1


def test_mfma_product_profile_counts_operations():
    g = synth.clustered(1200, cluster=(16, 64), seed=42)
    R = rsm_mod.from_grammar(synth.MEM_ALIAS, g.labels)
    want = H.oracle_grammar(g, synth.MEM_ALIAS)[R.box_names[0]][1]
    _, _, res = run(g, R, strategy=cfpq.STRATEGY_LEVELS, nt_mode=cfpq.NT_MFMA, profile=True)
    check_box(res, want, g.n)
    launches, ms, ops = res.profile(cfpq.KERNEL_NT_MFMA)
    assert launches > 0 and ms > 0 and ops > 0 and ops % 65536 == 0
    _, _, rows = run(g, R, strategy=cfpq.STRATEGY_LEVELS, nt_mode=cfpq.NT_ROWS, profile=True)
    assert rows.profile(cfpq.KERNEL_NT_MFMA)[0] == 0


def test_sparse_product_runs_in_closure_levels():
    g = synth.clustered(3000, cluster=(16, 64), seed=43)
    R = rsm_mod.from_grammar(synth.MEM_ALIAS, g.labels)
    want = H.oracle_grammar(g, synth.MEM_ALIAS)[R.box_names[0]][1]
    _, _, res = run(g, R, strategy=cfpq.STRATEGY_LEVELS, nt_mode=cfpq.NT_AUTO, profile=True)
    check_box(res, want, g.n)
    assert res.profile(cfpq.KERNEL_NT_SPARSE)[0] > 0
    _, _, rows = run(g, R, strategy=cfpq.STRATEGY_LEVELS, nt_mode=cfpq.NT_ROWS, profile=True)
    assert rows.profile(cfpq.KERNEL_NT_SPARSE)[0] == 0
    assert rows.stats()[:2] == res.stats()[:2]


def test_large_same_generation_selector_summary():
    # rows of at least 1024 words: the seed reads its selectors (the new
    # nonterminal edges) through a summary of their non-zero words; checked
    # against the closed form (pairs of vertices at equal depth >= 1, count
    # and order-independent hash) untiled and tiled, and against whole-row OR
    g, depth = synth.hierarchy(70000, with_type=False, seed=81)
    R = rsm_mod.from_grammar(synth.SAME_GEN_SC, g.labels)
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(R)
    res = cfpq.query(graph, q, strategy=cfpq.STRATEGY_LEVELS)
    levels = np.bincount(depth)
    assert res.count(0) == int((levels[1:] ** 2).sum())
    want = np.uint64(0)
    with np.errstate(over="ignore"):
        for d in range(1, len(levels)):
            vs = np.nonzero(depth == d)[0].astype(np.uint64)
            for c in range(0, len(vs), 512):
                keys = (vs[c:c + 512, None] << np.uint64(32)) | vs[None, :]
                want += H.splitmix64_np(keys.ravel()).sum(dtype=np.uint64)
    assert res.hash(0) == int(want)
    tiled = cfpq.query(graph, q, strategy=cfpq.STRATEGY_LEVELS, tile_words=300)
    assert (tiled.count(0), tiled.hash(0)) == (res.count(0), res.hash(0))
    rows = cfpq.query(graph, q, strategy=cfpq.STRATEGY_LEVELS, nt_mode=cfpq.NT_ROWS)
    assert rows.stats()[:2] == res.stats()[:2] and rows.hash(0) == res.hash(0)


def test_source_tiles_count_cached_allocator_memory():
    # the source tiles are as wide as the memory a query can get allows:
    # blocks that torch's caching allocator keeps unused count (it hands
    # them out again), although the device reports them as taken.  With
    # nearly all device memory parked in the cache the query still runs in
    # one tile: the seed launches once per iteration, as with an empty cache
    import gc
    import torch
    g = synth.hierarchy(50000, seed=synth.BASE_SEED + 3)[0]
    R = rsm_mod.from_grammar(synth.SAME_GEN_G1, g.labels)
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(R)
    gc.collect()
    torch.cuda.empty_cache()
    ref = cfpq.query(graph, q, strategy=cfpq.STRATEGY_LEVELS, profile=True)
    seeds = ref.profile(cfpq.KERNEL_SEED)[0]
    assert 0 < seeds <= ref.stats()[0]   # one tile: at most one seed per iteration
    free, _ = torch.cuda.mem_get_info()
    hold = free - (4 << 30)
    if hold <= 0:
        pytest.skip("less than 4 GiB of device memory free")
    parked = torch.empty(hold, dtype=torch.uint8, device="cuda")
    del parked   # back in the cache: the device no longer counts it as free
    try:
        res = cfpq.query(graph, q, strategy=cfpq.STRATEGY_LEVELS, profile=True)
        assert res.profile(cfpq.KERNEL_SEED)[0] == seeds
        assert res.stats()[:2] == ref.stats()[:2]
        assert (res.count(0), res.hash(0)) == (ref.count(0), ref.hash(0))
        del res
    finally:
        gc.collect()
        torch.cuda.empty_cache()


# closure recomputed from scratch each iteration (the variant the paper
# evaluated) against the incremental closure: same relation, iterations and
# per-iteration counts; one case also against the oracle
@pytest.mark.parametrize("case", ["samegen", "alias", "brackets", "nullable", "tiled"])
def test_recompute_matches_incremental(case):
    text = synth.BRACKETS
    kw = {}
    if case == "samegen":
        g, _ = synth.hierarchy(2500, seed=91)
        text = synth.SAME_GEN_G1
    elif case == "alias":
        g = synth.clustered(1500, cluster=(16, 64), seed=92)
        text = synth.MEM_ALIAS
    elif case == "nullable":
        g = synth.erdos_renyi(300, seed=93)
        text = "S -> a S b S | eps"
    else:
        g = synth.erdos_renyi(900, seed=94)
        kw = {"tile_words": 5} if case == "tiled" else {}
    R = rsm_mod.from_grammar(text, g.labels)
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(R)
    inc = cfpq.query(graph, q, strategy=cfpq.STRATEGY_LEVELS, **kw)
    scr = cfpq.query(graph, q, strategy=cfpq.STRATEGY_LEVELS, recompute=True, **kw)
    assert scr.stats()[:2] == inc.stats()[:2]
    for b in range(R.n_boxes):
        assert (scr.count(b), scr.hash(b)) == (inc.count(b), inc.hash(b))
    if case in ("alias", "nullable"):
        want = H.oracle_grammar(g, text)[R.box_names[0]][1]
        check_box(scr, want, g.n)
