"""The oracle's own query-language front end (test infrastructure only).

Parses regular expressions and context-free grammars written in the
extended form the paper uses for its queries (alternation, concatenation,
Kleene star from the regular-expression definition in Sec. 2.2; optional and
plus as in the memory-alias query of Sec. 4.2), builds Thompson
epsilon-NFAs, and rewrites a grammar into the normal form the worklist in
``cfl_oracle.c`` understands:

    A -> eps      A -> t      A -> B      A -> B C

This module is written independently of the product's query compiler: it
never determinises or minimises, and it keeps epsilon moves (they become
unit rules).

Text syntax shared by both sides (a file format, not code):
  * symbols are runs of letters, digits and underscores; ``eps`` is the
    empty word;
  * postfix ``*``, ``+``, ``?``; infix ``|``; juxtaposition concatenates;
    parentheses group;
  * a grammar is one rule per line, ``A -> expr``; several lines for one
    left-hand side are alternatives; the first left-hand side is the start
    nonterminal; every symbol that is some line's left-hand side is a
    nonterminal, every other symbol is an edge label.
"""
from __future__ import annotations

import re

_TOKEN = re.compile(r"\s*(?:([A-Za-z0-9_]+)|(.))")


def _tokens(text):
    out = []
    for m in _TOKEN.finditer(text):
        if m.group(1) is not None:
            out.append(("sym", m.group(1)))
        elif m.group(2) is not None and not m.group(2).isspace():
            out.append(("op", m.group(2)))
    return out


class _Parser:
    """Recursive descent over: alt := seq ('|' seq)*; seq := post*;
    post := atom ('*'|'+'|'?')*; atom := SYM | 'eps' | '(' alt ')'."""

    def __init__(self, text):
        self.toks = _tokens(text)
        self.i = 0

    def peek(self):
        return self.toks[self.i] if self.i < len(self.toks) else None

    def take(self):
        t = self.peek()
        self.i += 1
        return t

    def parse(self):
        node = self.alt()
        if self.peek() is not None:
            raise ValueError(f"unexpected token {self.peek()!r}")
        return node

    def alt(self):
        parts = [self.seq()]
        while self.peek() == ("op", "|"):
            self.take()
            parts.append(self.seq())
        return parts[0] if len(parts) == 1 else ("alt", parts)

    def seq(self):
        parts = []
        while True:
            t = self.peek()
            if t is None or t == ("op", "|") or t == ("op", ")"):
                break
            parts.append(self.post())
        if not parts:
            return ("eps",)
        return parts[0] if len(parts) == 1 else ("cat", parts)

    def post(self):
        node = self.atom()
        while self.peek() in (("op", "*"), ("op", "+"), ("op", "?")):
            node = ({"*": "star", "+": "plus", "?": "opt"}[self.take()[1]], node)
        return node

    def atom(self):
        t = self.take()
        if t is None:
            raise ValueError("unexpected end of expression")
        if t == ("op", "("):
            node = self.alt()
            if self.take() != ("op", ")"):
                raise ValueError("missing ')'")
            return node
        if t[0] == "sym":
            return ("eps",) if t[1] == "eps" else ("sym", t[1])
        raise ValueError(f"unexpected token {t!r}")


def parse_expr(text):
    return _Parser(text).parse()


class ENFA:
    """Thompson epsilon-NFA: states 0..n-1, moves (q, symbol-or-None, q')."""

    def __init__(self):
        self.n = 0
        self.moves = []

    def new(self):
        self.n += 1
        return self.n - 1

    def build(self, node):
        """Returns (entry, exit) of a fragment for the AST node."""
        kind = node[0]
        if kind == "eps":
            a, b = self.new(), self.new()
            self.moves.append((a, None, b))
            return a, b
        if kind == "sym":
            a, b = self.new(), self.new()
            self.moves.append((a, node[1], b))
            return a, b
        if kind == "cat":
            first = self.build(node[1][0])
            entry, ex = first
            for part in node[1][1:]:
                e2, x2 = self.build(part)
                self.moves.append((ex, None, e2))
                ex = x2
            return entry, ex
        if kind == "alt":
            a, b = self.new(), self.new()
            for part in node[1]:
                e, x = self.build(part)
                self.moves.append((a, None, e))
                self.moves.append((x, None, b))
            return a, b
        if kind in ("star", "plus", "opt"):
            a, b = self.new(), self.new()
            e, x = self.build(node[1])
            self.moves.append((a, None, e))
            self.moves.append((x, None, b))
            if kind in ("star", "opt"):
                self.moves.append((a, None, b))       # zero times
            if kind in ("star", "plus"):
                self.moves.append((x, None, e))       # again
            return a, b
        raise ValueError(kind)


def regex_enfa(text):
    """Returns (n_states, moves, start, accept) of the Thompson NFA."""
    nfa = ENFA()
    s, f = nfa.build(parse_expr(text))
    return nfa.n, nfa.moves, s, f


def parse_grammar(text):
    """Returns (ordered list of nonterminals, {A: AST of the union of its rules})."""
    order, rhs = [], {}
    for raw in text.splitlines():
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        if "->" not in line:
            raise ValueError(f"rule without '->': {raw!r}")
        lhs, body = line.split("->", 1)
        lhs = lhs.strip()
        if not re.fullmatch(r"[A-Za-z0-9_]+", lhs):
            raise ValueError(f"bad left-hand side {lhs!r}")
        if lhs not in rhs:
            order.append(lhs)
            rhs[lhs] = []
        rhs[lhs].append(parse_expr(body))
    if not order:
        raise ValueError("empty grammar")
    return order, {a: (alts[0] if len(alts) == 1 else ("alt", alts)) for a, alts in rhs.items()}


R_EPS, R_TERM, R_UNIT, R_BIN = 0, 1, 2, 3


def grammar_normal_form(text, label_ids):
    """Rewrite a grammar into normal-form rules for the worklist.

    label_ids maps edge-label names to the integer labels of the graph.  A
    terminal that is not a graph label can never be matched; it still gets
    its wrapper nonterminal, with no terminal rule.

    Returns (n_nonterminals, rules, names) where rules is a list of
    (kind, lhs, x, y) and the grammar's own nonterminals are numbered
    0..k-1 in order of first appearance (names lists them).
    """
    order, asts = parse_grammar(text)
    index = {a: i for i, a in enumerate(order)}
    count = [len(order)]
    rules = []
    term_nt = {}

    def fresh():
        count[0] += 1
        return count[0] - 1

    def wrap(t):
        if t not in term_nt:
            term_nt[t] = fresh()
            if t in label_ids:
                rules.append((R_TERM, term_nt[t], label_ids[t], 0))
        return term_nt[t]

    for a in order:
        nfa = ENFA()
        s, f = nfa.build(asts[a])
        local = [fresh() for _ in range(nfa.n)]
        rules.append((R_UNIT, index[a], local[s], 0))
        rules.append((R_EPS, local[f], 0, 0))
        for q, sym, q2 in nfa.moves:
            if sym is None:
                rules.append((R_UNIT, local[q], local[q2], 0))
            elif sym in index:
                rules.append((R_BIN, local[q], index[sym], local[q2]))
            else:
                rules.append((R_BIN, local[q], wrap(sym), local[q2]))
    return count[0], rules, list(order)
