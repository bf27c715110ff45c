"""Vertex masks (the multiple-source variant named as future work in Sec. 6)
and graphs handed over as device arrays, against the oracle's relation
restricted to the masks, element by element."""
import numpy as np
import pytest

import synth
from paper_2103_14688_amd import cfpq, rsm as rsm_mod
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def restrict(bm, n, src, dst):
    """Oracle bitmap (row u = targets v) restricted to src x dst."""
    out = bm.copy()
    if src is not None:
        out[~src] = 0
    if dst is not None:
        out &= cfpq.vertex_mask(dst, n)[None, :]
    return out


def masks(n, seed, ps=0.3, pd=0.5):
    rng = np.random.default_rng(seed)
    return rng.random(n) < ps, rng.random(n) < pd


def check(res, want, n, box=0):
    bm = res.bitmap(box)
    assert H.padding_clear(bm, n)
    assert np.array_equal(bm, want), len(H.bits_to_pairs(bm, n) ^ H.bits_to_pairs(want, n))
    assert res.count(box) == H.popcount(want)
    assert res.hash(box) == H.bitmap_hash(want, n)


STRATS = [cfpq.STRATEGY_LEVELS, cfpq.STRATEGY_CONDENSED, cfpq.STRATEGY_FUSED, cfpq.STRATEGY_AUTO]


@pytest.mark.parametrize("strategy", STRATS)
@pytest.mark.parametrize("which", ["src", "dst", "both"])
def test_rpq_masks(strategy, which):
    g = synth.powerlaw(1900, seed=51)
    full = H.oracle_regex(g, synth.RPQ_C2)
    src, dst = masks(g.n, 52)
    src = src if which in ("src", "both") else None
    dst = dst if which in ("dst", "both") else None
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(rsm_mod.from_regex(synth.RPQ_C2, g.labels))
    res = cfpq.query(graph, q, strategy=strategy, src_mask=src, dst_mask=dst)
    check(res, restrict(full, g.n, src, dst), g.n)


@pytest.mark.parametrize("strategy", [cfpq.STRATEGY_LEVELS, cfpq.STRATEGY_FUSED])
def test_grammar_masks_restrict_start_box_only(strategy):
    g = synth.clustered(900, cluster=(16, 64), seed=53)
    ora = H.oracle_grammar(g, synth.MEM_ALIAS)
    R = rsm_mod.from_grammar(synth.MEM_ALIAS, g.labels)
    src, dst = masks(g.n, 54)
    graph = cfpq.Graph.from_synth(g)
    res = cfpq.query(graph, cfpq.Query(R), strategy=strategy, src_mask=src, dst_mask=dst)
    start, other = R.box_names[0], R.box_names[1]
    check(res, restrict(ora[start][1], g.n, src, dst), g.n, box=0)
    check(res, ora[other][1], g.n, box=1)


def test_mask_edge_cases():
    g = synth.powerlaw(700, seed=55)
    full = H.oracle_regex(g, synth.RPQ_C2)
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(rsm_mod.from_regex(synth.RPQ_C2, g.labels))
    none = np.zeros(g.n, dtype=bool)
    for st in (cfpq.STRATEGY_LEVELS, cfpq.STRATEGY_CONDENSED):
        assert cfpq.query(graph, q, strategy=st, src_mask=none).count(0) == 0
        assert cfpq.query(graph, q, strategy=st, dst_mask=none).count(0) == 0
        # all-ones words, bits past n included: the same as no mask
        ones = np.full((g.n + 63) // 64, np.uint64(0xFFFFFFFFFFFFFFFF))
        check(cfpq.query(graph, q, strategy=st, src_mask=ones, dst_mask=ones), full, g.n)
    # one source: the single row of the oracle
    one = np.zeros(g.n, dtype=bool)
    u = min(H.bits_to_pairs(full, g.n))[0]
    one[u] = True
    check(cfpq.query(graph, q, src_mask=one), restrict(full, g.n, one, None), g.n)


def test_witness_respects_masks():
    g = synth.erdos_renyi(200, seed=56)
    text = synth.BRACKETS
    want = H.oracle_grammar(g, text)["S"][1]
    pairs = sorted(H.bits_to_pairs(want, g.n))
    src = np.zeros(g.n, dtype=bool)
    src[pairs[0][0]] = True
    graph = cfpq.Graph.from_synth(g)
    R = rsm_mod.from_grammar(text, g.labels)
    res = cfpq.query(graph, cfpq.Query(R), strategy=cfpq.STRATEGY_LEVELS, keep_rank=True, src_mask=src)
    u, v = pairs[0]
    path = res.extract_path(u, v)
    assert path[0][0] == u and path[-1][2] == v
    outside = [p for p in pairs if p[0] != u]
    if outside:
        with pytest.raises(cfpq.CfpqError) as e:
            res.extract_path(*outside[0])
        assert e.value.status == cfpq.ERR_NOT_FOUND


def test_batch_rejects_masks():
    g = synth.powerlaw(300, seed=57)
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(rsm_mod.from_regex(synth.RPQ_C2, g.labels))
    sm = cfpq.vertex_mask(np.ones(g.n, dtype=bool), g.n)
    o = cfpq.make_opts(src_mask=sm, alloc=graph._alloc, stream=cfpq.current_stream())
    with pytest.raises(cfpq.CfpqError) as e:
        cfpq.cfpq_query_batch([graph.h], [q.h], o)
    assert e.value.status == cfpq.ERR_INVALID


def test_graph_from_device_arrays():
    import torch
    g = synth.powerlaw(1500, seed=58)
    want = H.oracle_regex(g, synth.RPQ_C2)
    dev = [torch.from_numpy(np.asarray(x, dtype=np.int32)).cuda() for x in (g.src, g.lbl, g.dst)]
    graph = cfpq.Graph(g.n, *dev, g.labels, flags=cfpq.DEVICE_PTRS)
    assert graph.info() == (g.n, len(g.labels), len(set(zip(g.src.tolist(), g.lbl.tolist(), g.dst.tolist()))))
    res = cfpq.query(graph, cfpq.Query(rsm_mod.from_regex(synth.RPQ_C2, g.labels)))
    check(res, want, g.n)


def test_condensed_repeated_queries_with_masks_and_ranks():
    # one graph handle, so later queries take the one-read path sized by the
    # previous one: unmasked, masked, with ranks, again unmasked; every answer
    # against the oracle restricted to the masks
    g = synth.powerlaw(3000, seed=83)
    R = rsm_mod.from_regex(synth.RPQ_C2, g.labels)
    want = H.oracle_regex(g, synth.RPQ_C2)
    graph = cfpq.Graph.from_synth(g)
    q = cfpq.Query(R)
    src, dst = masks(g.n, 84)
    runs = [dict(), dict(src_mask=src), dict(src_mask=src, dst_mask=dst, keep_rank=True), dict(),
            dict(keep_rank=True), dict(dst_mask=dst), dict()]
    for kw in runs:
        res = cfpq.query(graph, q, strategy=cfpq.STRATEGY_CONDENSED, **kw)
        check(res, restrict(want, g.n, kw.get("src_mask"), kw.get("dst_mask")), g.n)
        if kw.get("keep_rank"):
            pairs = res.pairs(0)
            for u, v in pairs[:: max(1, len(pairs) // 5)].tolist():
                path = res.extract_path(u, v)   # every word of the query has a c edge
                assert path[0][0] == u and path[-1][2] == v
