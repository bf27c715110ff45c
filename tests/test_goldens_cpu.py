"""The stored goldens cover what they claim (no GPU needed): the serving
subset holds every query on a graph of at most 16,000 vertices and a 2%
sample of the others; the per-block RPQ values add up to the whole."""
import json
import os

import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fullsize.json")


@pytest.fixture(scope="module")
def gold():
    with open(GOLDEN) as f:
        return json.load(f)


def test_rpq_blocks_add_up(gold):
    g = gold["rpq_powerlaw_n100000"]
    assert sum(b["count"] for b in g["blocks"]) == g["count"]
    assert sum(int(b["hash"], 16) for b in g["blocks"]) % (1 << 64) == int(g["hash"], 16)
    assert len(g["blocks"]) * g["block_sources"] == 100000


@pytest.mark.parametrize("n", [200000, 500000])
def test_typefree_closed_form_count(gold, n):
    e = gold[f"samegen_typefree_n{n}"]
    assert e["boxes"]["S"]["count"] == sum(x * x for x in e["levels"])
    assert sum(e["levels"]) < n


def test_serving_subset_covers_the_definition(gold):
    if "serving" not in gold:
        pytest.skip("serving goldens not generated")
    s = gold["serving"]
    _, recipes, qs = synth.serving_mix()
    small = {i for i, (gi, _, _) in enumerate(qs) if recipes[gi][0] <= s["small_n"]}
    full = {int(i) for i in s["full"]}
    assert small <= full
    sampled = (full - small) | {int(i) for i in s["rows"]} | set(s["unpinned"])
    big = len(qs) - len(small)
    assert len(sampled) == int(round(s["sample_fraction"] * big))
