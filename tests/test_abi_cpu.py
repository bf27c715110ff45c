"""CPU-side checks of the product: the C-ABI library loads and exports every
declared entry point, host-side validation, and the query compiler's
automata against Python's re module (an independent recogniser)."""
import itertools
import os
import re

import numpy as np
import pytest

import synth
from paper_2103_14688_amd import cfpq, rsm as rsm_mod
from tests import brute

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "cfpq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cfpq_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = cfpq.load()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(cfpq.EXPORTS)
    assert cfpq.cfpq_version().startswith("cfpq-gfx950")


def _header_struct_fields(name):
    """Field names, in order, of `typedef struct { ... } name;` in the header."""
    text = open(os.path.join(ROOT, "include", "cfpq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", text).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ptr = re.search(r"\(\s*\*\s*(\w+)\s*\)", decl)   # function pointer
        fields.append(ptr.group(1) if ptr else re.findall(r"\w+", decl)[-1])
    return fields


@pytest.mark.parametrize("cname, pytype", [("cfpq_allocator", "Allocator"), ("cfpq_query_opts", "QueryOpts")])
def test_binding_structs_mirror_the_header(cname, pytype):
    # the ctypes structures the binding passes across the boundary list the
    # header's fields in the header's order (a missing or moved field would
    # be read as another one by the library)
    got = [f[0] for f in getattr(cfpq, pytype)._fields_]
    assert got == _header_struct_fields(cname)


def test_rsm_validation_errors():
    ok = dict(n_states=2, n_terminals=1, n_boxes=1, box_start=[0], state_box=[0, 0], is_final=[0, 1],
              t_src=[0], t_sym=[0], t_dst=[1])
    h = cfpq.cfpq_rsm_create(**ok)
    cfpq.cfpq_rsm_destroy(h)
    bad = [
        dict(ok, state_box=[0, 1]),                       # state in a missing box
        dict(ok, t_sym=[2]),                              # symbol out of range
        dict(ok, t_dst=[5]),                              # state out of range
        dict(ok, n_boxes=2, box_start=[0, 0], state_box=[0, 1]),  # start owned by another box
        dict(ok, n_boxes=2, box_start=[0, 1], state_box=[0, 1]),  # transition crosses boxes
        dict(ok, n_states=0),
    ]
    for b in bad:
        with pytest.raises(cfpq.CfpqError) as e:
            cfpq.cfpq_rsm_create(**b)
        assert e.value.status == cfpq.ERR_INVALID


def test_graph_validation_errors_before_device():
    for args in [(0, 1, [], [], []), (3, 1, [0], [0], [3]), (3, 1, [0], [1], [2]), (3, 0, [], [], [])]:
        with pytest.raises(cfpq.CfpqError) as e:
            cfpq.cfpq_graph_create(*args)
        assert e.value.status == cfpq.ERR_INVALID


def accepts(R, box, word, labels):
    """Run a compiled (deterministic) box on a word of label names."""
    q = int(R.box_start[box])
    ids = {x: i for i, x in enumerate(labels)}
    for x in word:
        nxt = [int(d) for s, y, d in zip(R.t_src, R.t_sym, R.t_dst) if s == q and y == ids[x]]
        assert len(nxt) <= 1
        if not nxt:
            return False
        q = nxt[0]
    return bool(R.is_final[q])


REGEXES = ["a", "a b*", "(a | b)* c d*", "a? b*", "(a b)+ | (c d)+", "a b (c | d | e)", "(a | b)+ (c | d)+",
           "(a (b c)*)+ | (d e)+", "(a b (c d)*)+ (e | a)*", "eps", "a*", "(a | eps) b", "((a | b) c?)* d+"]


@pytest.mark.parametrize("regex", REGEXES)
@pytest.mark.parametrize("minimize", [True, False])
def test_regex_dfa_matches_python_re(regex, minimize):
    labels = ["a", "b", "c", "d", "e"]
    R = rsm_mod.from_regex(regex, labels, minimize=minimize)
    alphabet = {x: x for x in labels}
    pat = re.compile(brute.regex_to_python(regex, alphabet))
    for k in range(0, 6):
        for word in itertools.product(labels, repeat=k):
            assert accepts(R, 0, word, labels) == bool(pat.fullmatch("".join(word))), (regex, word)


def test_minimal_dfa_sizes():
    labels = ["a", "b", "c", "d"]
    assert rsm_mod.from_regex("(a | b)* c d*", labels).n_states == 2
    assert rsm_mod.from_regex("(a | b)* c d*", labels, minimize=False).n_states >= 3
    assert rsm_mod.from_grammar(synth.BRACKETS, ["a", "b"]).n_states == 4
    ma = rsm_mod.from_grammar(synth.MEM_ALIAS, ["a", "d", "a_r", "d_r"])
    assert ma.n_states == 8 and len(ma.t_src) == 11


def test_paper_figure_rsm_matches_compiled_language():
    labels = ["a", "b"]
    fig = rsm_mod.paper_example_rsm(labels)
    comp = rsm_mod.from_grammar(synth.BRACKETS, labels)
    for R in (fig, comp):
        assert R.n_states == 4 and R.n_boxes == 1
        assert sorted(zip(R.t_src.tolist(), R.t_sym.tolist(), R.t_dst.tolist())) == \
            sorted(zip(fig.t_src.tolist(), fig.t_sym.tolist(), fig.t_dst.tolist()))


def test_grammar_boxes_and_symbols():
    labels = ["sc", "type", "sc_r", "type_r"]
    R = rsm_mod.from_grammar(synth.SAME_GEN_G1, labels)
    assert R.box_names == ["S"]
    assert R.n_states == 6 and len(R.t_src) == 8
    nt = R.n_terminals
    assert sum(1 for s in R.t_sym if s >= nt) == 2       # two calls of S
    rs = rsm_mod.from_grammar("A -> B c\nB -> b | eps", ["b", "c"])
    assert rs.box_names == ["A", "B"]
    assert rs.is_final[rs.box_start[1]] == 1             # B is nullable


def test_unknown_terminal_is_dropped():
    R = rsm_mod.from_regex("a zz | b", ["a", "b"])
    assert set(R.t_sym.tolist()) <= {0, 1}


def test_synth_generators_are_seeded_and_shaped():
    g1 = synth.powerlaw(5000, seed=1)
    g2 = synth.powerlaw(5000, seed=1)
    assert np.array_equal(g1.src, g2.src) and np.array_equal(g1.dst, g2.dst)
    assert 3.0 < len(g1.src) / g1.n < 5.0
    assert not np.any(g1.src == g1.dst)
    key = g1.src.astype(np.int64) * g1.n + g1.dst
    assert len(np.unique(key)) == len(key)
    g, depth = synth.hierarchy(5000, seed=2)
    assert depth.max() >= 5
    c = synth.clustered(4000, seed=3)
    assert set(c.labels) == {"a", "d", "a_r", "d_r"}
    labels, graphs, qs = synth.serving_mix(n_graphs=4, n_queries=50)
    assert len(graphs) == 4 and len(qs) == 50
    for gi, kind, text in qs:
        (rsm_mod.from_regex if kind == "regex" else rsm_mod.from_grammar)(text, labels)


def test_vertex_mask_packing():
    n = 130
    m = np.zeros(n, dtype=bool)
    m[[0, 63, 64, 129]] = True
    w = cfpq.vertex_mask(m, n)
    assert w.dtype == np.uint64 and w.shape == (3,)
    assert [int(x) for x in w] == [1 | (1 << 63), 1, 2]
    assert cfpq.vertex_mask(None, n) is None
    assert np.array_equal(cfpq.vertex_mask(w, n), w)
    with pytest.raises(ValueError):
        cfpq.vertex_mask(np.zeros(n - 1, dtype=bool), n)
    with pytest.raises(ValueError):
        cfpq.vertex_mask(np.zeros(2, dtype=np.uint64), n)


def test_unknown_graph_flag_rejected():
    with pytest.raises(cfpq.CfpqError) as e:
        cfpq.cfpq_graph_create(3, 1, [0], [0], [1], flags=4)
    assert e.value.status == cfpq.ERR_INVALID
