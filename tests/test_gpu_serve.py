"""GPU serving: every request's answer is the same alone (plain mode, one
cfpq_query per request) and in the continuous-batching mix (fused batches +
overlapping streams), tolerance 0 on (pair count, pair hash, iterations); a
sample is also checked against the oracle."""
import numpy as np
import pytest

import synth
from paper_2103_14688_amd import cfpq, rsm as rsm_mod, serve
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mix():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    labels, recipes, qs = synth.serving_mix(n_graphs=8, n_queries=48, n_range=(150, 6000), seed=synth.BASE_SEED + 55)
    graphs = [synth.serving_graph(n, seed, labels) for n, seed in recipes]
    handles = [cfpq.Graph.from_synth(g) for g in graphs]
    reqs = []
    for i, (gi, kind, text) in enumerate(qs):
        R = rsm_mod.from_regex(text, labels) if kind == "regex" else rsm_mod.from_grammar(text, labels)
        reqs.append((gi, kind, text, R, cfpq.Query(R)))
    return labels, graphs, handles, reqs


def build(mix_):
    labels, graphs, handles, reqs = mix_
    return [serve.Request(i, handles[gi], q, graphs[gi].n, R.n_states, R.n_boxes)
            for i, (gi, kind, text, R, q) in enumerate(reqs)]


def test_alone_vs_mix_identical(mix):
    backend = serve.GpuBackend()
    plain = serve.Server(backend, mode="plain")
    a = build(mix)
    for r in a:
        plain.submit(r)
    plain.drain(timeout=300)
    plain.close()
    batched = serve.Server(backend, mode="batched", slots=4)
    b = build(mix)
    arrivals = np.cumsum(np.random.default_rng(3).exponential(0.002, size=len(b)))
    serve.replay(batched, b, arrivals)
    batched.close()
    assert all(not r.error for r in a + b), [r.error for r in a + b if r.error][:3]
    for x, y in zip(a, b):
        assert x.result == y.result, (x.rid, x.result, y.result)
    assert any(r.batched for r in b)


def test_mix_sample_against_oracle(mix):
    labels, graphs, handles, reqs = mix
    backend = serve.GpuBackend()
    s = serve.Server(backend, mode="batched", slots=3)
    rs = build(mix)
    for r in rs:
        s.submit(r)
    s.drain(timeout=300)
    s.close()
    for r in rs[:12]:
        gi, kind, text, R, _ = reqs[r.rid]
        g = graphs[gi]
        want = H.oracle_regex(g, text) if kind == "regex" else H.oracle_grammar(g, text)["N0"][1]
        assert r.result[0] == H.popcount(want)
        assert r.result[1] == H.bitmap_hash(want, g.n)
