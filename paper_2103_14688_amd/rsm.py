"""Query compiler: regular expressions and grammars to recursive state machines.

A regular expression becomes a one-box RSM whose box is a deterministic,
epsilon-free automaton (Sec. 2.2 and Sec. 3.1.2: an RPQ is a single
component state machine with no calls).  A grammar becomes one box per
nonterminal, each box a deterministic automaton over terminals and box labels
built from the union of that nonterminal's right-hand sides (Sec. 2.3, CFG to
RSM with one box per nonterminal; extended right-hand sides allowed).

Construction: Glushkov position automaton (epsilon-free by construction),
subset construction, then Moore partition refinement.  The automaton is only
a representation of the query language; the answer does not depend on which
equivalent automaton is used.

Text syntax: symbols are runs of letters, digits and underscores, ``eps`` is
the empty word; postfix ``*``, ``+``, ``?``; infix ``|``; juxtaposition is
concatenation; parentheses group.  A grammar has one ``A -> expr`` rule per
line (repeated left-hand sides are alternatives); the first left-hand side is
the start nonterminal; symbols that never appear on a left-hand side are
edge labels.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# expression trees
# ---------------------------------------------------------------------------


@dataclass
class Node:
    op: str                       # 'sym', 'eps', 'cat', 'alt', 'star', 'plus', 'opt'
    kids: list = field(default_factory=list)
    name: str = ""
    pos: int = -1                 # position index for 'sym'


def _lex(text):
    toks, i = [], 0
    while i < len(text):
        c = text[i]
        if c.isspace():
            i += 1
        elif c.isalnum() or c == "_":
            j = i
            while j < len(text) and (text[j].isalnum() or text[j] == "_"):
                j += 1
            toks.append(text[i:j])
            i = j
        elif c in "()|*+?":
            toks.append(c)
            i += 1
        else:
            raise ValueError(f"unexpected character {c!r} in {text!r}")
    return toks


def parse(text):
    """Expression text -> Node tree (precedence: postfix > concatenation > |)."""
    toks = _lex(text)
    k = [0]

    def peek():
        return toks[k[0]] if k[0] < len(toks) else None

    def union():
        parts = [concat()]
        while peek() == "|":
            k[0] += 1
            parts.append(concat())
        return parts[0] if len(parts) == 1 else Node("alt", parts)

    def concat():
        parts = []
        while peek() is not None and peek() not in ("|", ")"):
            parts.append(postfix())
        if not parts:
            return Node("eps")
        return parts[0] if len(parts) == 1 else Node("cat", parts)

    def postfix():
        node = primary()
        while peek() in ("*", "+", "?"):
            op = {"*": "star", "+": "plus", "?": "opt"}[toks[k[0]]]
            k[0] += 1
            node = Node(op, [node])
        return node

    def primary():
        t = peek()
        if t is None:
            raise ValueError(f"expression ends early: {text!r}")
        k[0] += 1
        if t == "(":
            node = union()
            if peek() != ")":
                raise ValueError(f"missing ')' in {text!r}")
            k[0] += 1
            return node
        if t in ("|", ")", "*", "+", "?"):
            raise ValueError(f"unexpected {t!r} in {text!r}")
        return Node("eps") if t == "eps" else Node("sym", name=t)

    node = union()
    if peek() is not None:
        raise ValueError(f"unexpected {peek()!r} in {text!r}")
    return node


# ---------------------------------------------------------------------------
# Glushkov automaton -> DFA -> minimal DFA
# ---------------------------------------------------------------------------

def _glushkov(root):
    """Returns (symbols by position, nullable, first, last, follow)."""
    syms = []

    def number(n):
        if n.op == "sym":
            n.pos = len(syms)
            syms.append(n.name)
        for c in n.kids:
            number(c)

    number(root)
    follow = [set() for _ in syms]

    def walk(n):
        # returns (nullable, first, last) and fills follow
        if n.op == "eps":
            return True, set(), set()
        if n.op == "sym":
            return False, {n.pos}, {n.pos}
        if n.op == "alt":
            res = [walk(c) for c in n.kids]
            return any(r[0] for r in res), set().union(*[r[1] for r in res]), set().union(*[r[2] for r in res])
        if n.op == "cat":
            res = [walk(c) for c in n.kids]
            nul, first, last = True, set(), set()
            for r in res:
                for p in last:
                    follow[p] |= r[1]
                if nul:
                    first |= r[1]
                last = (last | r[2]) if r[0] else set(r[2])
                nul = nul and r[0]
            return nul, first, last
        nul, first, last = walk(n.kids[0])
        if n.op in ("star", "plus"):
            for p in last:
                follow[p] |= first
        return (True if n.op in ("star", "opt") else nul), first, last

    nul, first, last = walk(root)
    return syms, nul, first, last, follow


def _dfa(root):
    """Subset construction over Glushkov positions.
    Returns (n_states, transitions {(state, symbol): state}, finals); state 0 is initial."""
    syms, nul, first, last, follow = _glushkov(root)
    init = frozenset([-1])
    index = {init: 0}
    order = [init]
    trans = {}
    finals = set()
    i = 0
    while i < len(order):
        S = order[i]
        if (-1 in S and nul) or (S & last):
            finals.add(i)
        succ = set(first) if -1 in S else set()
        for p in S:
            if p >= 0:
                succ |= follow[p]
        by_sym = {}
        for p in succ:
            by_sym.setdefault(syms[p], set()).add(p)
        for a in sorted(by_sym):
            T = frozenset(by_sym[a])
            if T not in index:
                index[T] = len(order)
                order.append(T)
            trans[(i, a)] = index[T]
        i += 1
    return len(order), trans, finals


def _minimize(n, trans, finals):
    """Moore partition refinement of a partial DFA (missing moves go to an
    implicit dead state, which is dropped again).  State 0 stays initial."""
    alphabet = sorted({a for (_, a) in trans})
    dead = n
    block = [1 if q in finals else 0 for q in range(n)] + [0]
    # states that cannot reach a final state behave like the dead state
    while True:
        sig = {}
        new = []
        for q in range(n + 1):
            key = (block[q],) + tuple(block[trans.get((q, a), dead)] if q < n else block[dead] for a in alphabet)
            new.append(sig.setdefault(key, len(sig)))
        if len(sig) == len(set(block)):
            block = new
            break
        block = new
    dead_block = block[dead]
    # renumber: initial first, drop the dead block
    remap = {}
    order = []
    for q in range(n):
        b = block[q]
        if b == dead_block or b in remap:
            continue
        remap[b] = None
        order.append(b)
    if block[0] == dead_block:
        return 1, {}, set()  # empty language: a single non-final state
    order.remove(block[0])
    order.insert(0, block[0])
    num = {b: i for i, b in enumerate(order)}
    t2 = {}
    for (q, a), r in trans.items():
        if block[q] == dead_block or block[r] == dead_block:
            continue
        t2[(num[block[q]], a)] = num[block[r]]
    f2 = {num[block[q]] for q in finals if block[q] != dead_block}
    return len(order), t2, f2


def compile_expr(text, minimize=True):
    """Expression text -> (n_states, {(state, symbol): state}, finals), state 0 initial."""
    n, trans, finals = _dfa(parse(text))
    if minimize:
        n, trans, finals = _minimize(n, trans, finals)
    return n, trans, finals


# ---------------------------------------------------------------------------
# RSM
# ---------------------------------------------------------------------------

@dataclass
class RSM:
    """Arrays of a recursive state machine in the layout of cfpq_rsm_create."""
    n_states: int
    n_terminals: int
    box_names: list
    box_start: np.ndarray
    state_box: np.ndarray
    is_final: np.ndarray
    t_src: np.ndarray
    t_sym: np.ndarray
    t_dst: np.ndarray
    start_box: int = 0

    @property
    def n_boxes(self):
        return len(self.box_names)

    def box(self, name):
        return self.box_names.index(name)


def _split_rules(text):
    order, bodies = [], {}
    for raw in text.splitlines():
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        if "->" not in line:
            raise ValueError(f"rule without '->': {raw!r}")
        lhs, rhs = (s.strip() for s in line.split("->", 1))
        if not lhs or not all(c.isalnum() or c == "_" for c in lhs):
            raise ValueError(f"bad left-hand side {lhs!r}")
        if lhs not in bodies:
            order.append(lhs)
            bodies[lhs] = []
        bodies[lhs].append(rhs if rhs else "eps")
    if not order:
        raise ValueError("empty grammar")
    return order, bodies


def _assemble(boxes, labels, minimize):
    """boxes: ordered list of (name, expression text)."""
    names = [b for b, _ in boxes]
    label_id = {x: i for i, x in enumerate(labels)}
    nt = len(labels)
    starts, state_box, final, src, sym, dst = [], [], [], [], [], []
    base = 0
    for bi, (name, expr) in enumerate(boxes):
        n, trans, finals = compile_expr(expr, minimize)
        starts.append(base)
        state_box += [bi] * n
        final += [1 if q in finals else 0 for q in range(n)]
        for (q, a), r in sorted(trans.items()):
            if a in names:
                s = nt + names.index(a)
            elif a in label_id:
                s = label_id[a]
            else:
                continue  # a terminal the graph does not have never matches
            src.append(base + q)
            sym.append(s)
            dst.append(base + r)
        base += n
    u32 = lambda a: np.asarray(a, dtype=np.uint32)
    return RSM(base, nt, names, u32(starts), u32(state_box), np.asarray(final, dtype=np.uint8),
               u32(src), u32(sym), u32(dst), 0)


def from_regex(text, labels, minimize=True, box_name="S"):
    """One-box RSM for a regular path query over the graph's label list."""
    return _assemble([(box_name, text)], list(labels), minimize)


def from_grammar(text, labels, minimize=True):
    """One box per nonterminal; box 0 is the start nonterminal."""
    order, bodies = _split_rules(text)
    boxes = [(a, " | ".join(f"({b})" for b in bodies[a])) for a in order]
    return _assemble(boxes, list(labels), minimize)


def paper_example_rsm(labels=("a", "b")):
    """The RSM of the Sec. 2.3 figure for S -> a S b | a b, state for state:
    q0 -a-> q1, q1 -S-> q2, q2 -b-> q3, q1 -b-> q3, final q3."""
    a, b = labels.index("a"), labels.index("b")
    nt = len(labels)
    u32 = lambda x: np.asarray(x, dtype=np.uint32)
    return RSM(4, nt, ["S"], u32([0]), u32([0, 0, 0, 0]), np.asarray([0, 0, 0, 1], dtype=np.uint8),
               u32([0, 1, 2, 1]), u32([a, nt + 0, b, b]), u32([1, 2, 3, 3]), 0)


def from_automaton(n_states, transitions, finals, labels, start=0, box_name="S"):
    """One-box RSM from an explicit automaton (a regular query given state by
    state): transitions are (state, label name, state) triples, finals a set
    of states; any epsilon-free automaton serves (Sec. 2.2), deterministic or
    not.  Labels absent from the graph's list never match and are dropped."""
    label_id = {x: i for i, x in enumerate(labels)}
    if not 0 <= start < n_states:
        raise ValueError("start state out of range")
    order = [start] + [q for q in range(n_states) if q != start]   # the box starts at state 0
    ren = {q: i for i, q in enumerate(order)}
    kept = [(ren[a], label_id[x], ren[b]) for a, x, b in transitions if x in label_id]
    u32 = lambda a: np.asarray(a, dtype=np.uint32)
    final = np.zeros(n_states, dtype=np.uint8)
    for q in finals:
        final[ren[q]] = 1
    return RSM(n_states, len(labels), [box_name], u32([0]), u32([0] * n_states), final,
               u32([t[0] for t in kept]), u32([t[1] for t in kept]), u32([t[2] for t in kept]), 0)
