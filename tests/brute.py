"""Brute-force references for tiny inputs (test helpers).

Written from the definitions only (Sec. 2.1: path, word of a path,
reachability semantics; Sec. 2.3: derivation and language of a grammar),
with no code from the oracle or the product.
"""
from __future__ import annotations

import re


def path_words(n, edges, max_len):
    """{(u, v): set of words} over every path of length <= max_len.
    edges: iterable of (u, label, v).  The empty path gives (u, u) -> ()."""
    out = {}
    succ = {}
    for u, x, v in set(edges):
        succ.setdefault(u, []).append((x, v))

    def walk(start, node, word):
        out.setdefault((start, node), set()).add(word)
        if len(word) == max_len:
            return
        for x, v in succ.get(node, ()):
            walk(start, v, word + (x,))

    for u in range(n):
        walk(u, u, ())
    return out


def bnf_accepts(prods, start, word):
    """Does the grammar derive the word?  prods: list of (A, [symbols]); a
    symbol is a nonterminal iff it is some production's left-hand side.
    Least fixpoint of span sets: (i, j) in D[A] iff A derives word[i:j]."""
    nts = {a for a, _ in prods}
    n = len(word)
    spans = {a: set() for a in nts}
    changed = True
    while changed:
        changed = False
        for a, rhs in prods:
            for i in range(n + 1):
                ends = {i}
                for sym in rhs:
                    nxt = set()
                    for j in ends:
                        if sym in nts:
                            nxt |= {e for (s, e) in spans[sym] if s == j}
                        elif j < n and word[j] == sym:
                            nxt.add(j + 1)
                    ends = nxt
                    if not ends:
                        break
                for e in ends:
                    if (i, e) not in spans[a]:
                        spans[a].add((i, e))
                        changed = True
    return (0, n) in spans[start]


def bnf_text(prods):
    order = []
    alts = {}
    for a, rhs in prods:
        if a not in alts:
            order.append(a)
            alts[a] = []
        alts[a].append(" ".join(rhs) if rhs else "eps")
    return "\n".join(f"{a} -> {' | '.join(alts[a])}" for a in order)


def brute_cfl(n, edges, prods, start, max_len):
    """Pairs (u, v) with a path of length <= max_len spelling a word of L(start)."""
    words = path_words(n, edges, max_len)
    cache = {}
    res = set()
    for (u, v), ws in words.items():
        for w in ws:
            if w not in cache:
                cache[w] = bnf_accepts(prods, start, w)
            if cache[w]:
                res.add((u, v))
                break
    return res


def relational_fixpoint(n, edges, prods):
    """Naive evaluation: R_A is the least relation containing the composition
    R_X1 ; ... ; R_Xk for every production A -> X1..Xk (terminal t: its
    edges; empty right-hand side: identity)."""
    nts = {a for a, _ in prods}
    rel = {a: set() for a in nts}
    term = {}
    for u, x, v in edges:
        term.setdefault(x, set()).add((u, v))
    ident = {(u, u) for u in range(n)}
    changed = True
    while changed:
        changed = False
        for a, rhs in prods:
            cur = ident
            for sym in rhs:
                r = rel[sym] if sym in nts else term.get(sym, set())
                by_src = {}
                for (p, q) in r:
                    by_src.setdefault(p, []).append(q)
                cur = {(u, q) for (u, p) in cur for q in by_src.get(p, ())}
                if not cur:
                    break
            new = cur - rel[a]
            if new:
                rel[a] |= new
                changed = True
    return rel


def regex_to_python(text, alphabet):
    """Translate the shared regex text syntax into Python's re syntax, each
    label becoming one character of alphabet ({label: char})."""
    out = []
    for m in re.finditer(r"\s*(?:([A-Za-z0-9_]+)|(.))", text):
        if m.group(1) is not None:
            out.append("()" if m.group(1) == "eps" else re.escape(alphabet[m.group(1)]))
        elif m.group(2) and not m.group(2).isspace():
            out.append(m.group(2))
    return "".join(out)


def brute_rpq(n, edges, regex, labels, max_len):
    alphabet = {x: chr(ord("a") + i) for i, x in enumerate(labels)}
    pat = re.compile(regex_to_python(regex, alphabet))
    words = path_words(n, edges, max_len)
    res = set()
    for (u, v), ws in words.items():
        if any(pat.fullmatch("".join(alphabet[x] for x in w)) for w in ws):
            res.add((u, v))
    return res
