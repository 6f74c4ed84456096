"""LTL -> LTL4 monitor compiler (host tooling for the C ABI).

The ABI consumes an LTL4 monitor as a transition table over event classes
(Def. 6: a deterministic Moore machine whose output after a word u is
[u |=4 psi]).  The paper synthesises monitors before run time with the method
of its reference [bls10-jlc] and does not describe it, so this module is our
own construction:

1. Finite-trace part (FLTL, Def. 4) by formula progression.  A state is the
   residual obligation after the word read so far, kept as a reduced ordered
   BDD over "obligation" variables O(chi): chi must hold from the next
   position on.  Progressing through a letter substitutes every O(chi) by the
   progression of chi.  Because X is a strong next and an until must be
   fulfilled inside the word, every obligation left open at the end of the
   word is false; the FLTL value of the word is the residual with all O := 0.
2. Infinite-extension part (the T / F cases of Def. 5): the residual, read
   as an LTL formula over infinite words, is checked for satisfiability and
   validity with the on-the-fly tableau of Gerth, Peled, Vardi and Wolper
   (generalised Buchi automaton plus a search for an accepting
   strongly-connected component).
3. Labels: T if the negated residual is unsatisfiable, F if the residual is
   unsatisfiable, otherwise Tp / Fp by the FLTL value.  The empty word is
   labelled by the same rule with the FLTL value of the formula computed with
   every proposition, X and U false (the empty word is never a verdict; this
   only fixes the initial state).
4. Moore minimisation over the letters 2^AP, expansion to event classes (each
   class carries a set of propositions), and a second minimisation over the
   classes.

Letters range over all subsets of the formula's propositions, as the
extensions v in Def. 5 do.
"""
from __future__ import annotations

import itertools
import re
from dataclasses import dataclass

import numpy as np

# Verdict codes of the ABI (lattice order of B6).
V_BOT, V_BOT_P, V_TOP_P, V_TOP = 0, 2, 3, 5

MAX_STATES = 16
MAX_CLASSES = 16


# ----------------------------------------------------------------------------
# Formulas: hash-consed nodes.
# ----------------------------------------------------------------------------
class Node:
    __slots__ = ("op", "a", "b", "name", "uid", "_hash")
    _table: dict = {}
    _count = 0

    def __new__(cls, op, a=None, b=None, name=None):
        key = (op, a.uid if a is not None else None, b.uid if b is not None else None, name)
        got = cls._table.get(key)
        if got is not None:
            return got
        self = object.__new__(cls)
        self.op, self.a, self.b, self.name = op, a, b, name
        self.uid = Node._count
        Node._count += 1
        self._hash = hash(key)
        cls._table[key] = self
        return self

    def __hash__(self):
        return self._hash

    def __repr__(self):
        if self.op == "ap":
            return self.name
        if self.op in ("tt", "ff"):
            return self.op
        if self.b is None:
            return f"{self.op}({self.a!r})"
        return f"({self.a!r} {self.op} {self.b!r})"


TT, FF = Node("tt"), Node("ff")


def ap(name):
    return Node("ap", name=name)


_LEX = re.compile(r"->|[()!&|]|[A-Za-z_][A-Za-z0-9_]*")


def parse_ltl(text):
    """Parse LTL text: ! & | -> X F G U, true/false, lower-case propositions.

    Binding from tightest: unary operators, U (right-associative), &, |, ->
    (right-associative).  F and G are expanded by their definitions
    F p = true U p and G p = !F!p (end of Section 2.2.1).
    """
    toks = _LEX.findall(text)
    if "".join(toks) != re.sub(r"\s+", "", text):
        raise ValueError(f"bad character in formula {text!r}")
    it = iter(toks + [None])
    cur = [next(it)]

    def eat(t=None):
        tok = cur[0]
        if t is not None and tok != t:
            raise ValueError(f"expected {t!r}, got {tok!r} in {text!r}")
        cur[0] = next(it)
        return tok

    def p_imp():
        lhs = p_or()
        if cur[0] == "->":
            eat()
            return Node("or", Node("not", lhs), p_imp())
        return lhs

    def p_or():
        f = p_and()
        while cur[0] == "|":
            eat()
            f = Node("or", f, p_and())
        return f

    def p_and():
        f = p_until()
        while cur[0] == "&":
            eat()
            f = Node("and", f, p_until())
        return f

    def p_until():
        f = p_un()
        if cur[0] == "U":
            eat()
            return Node("U", f, p_until())
        return f

    def p_un():
        tok = cur[0]
        if tok == "!":
            eat()
            return Node("not", p_un())
        if tok == "X":
            eat()
            return Node("X", p_un())
        if tok == "F":
            eat()
            return Node("U", TT, p_un())
        if tok == "G":
            eat()
            return Node("not", Node("U", TT, Node("not", p_un())))
        if tok == "(":
            eat()
            f = p_imp()
            eat(")")
            return f
        if tok == "true":
            eat()
            return TT
        if tok == "false":
            eat()
            return FF
        if tok is not None and re.fullmatch(r"[a-z_][a-z0-9_]*", tok):
            eat()
            return ap(tok)
        raise ValueError(f"unexpected {tok!r} in {text!r}")

    f = p_imp()
    if cur[0] is not None:
        raise ValueError(f"trailing {cur[0]!r} in {text!r}")
    return f


def propositions(f):
    seen, out, stack = set(), set(), [f]
    while stack:
        g = stack.pop()
        if g.uid in seen:
            continue
        seen.add(g.uid)
        if g.op == "ap":
            out.add(g.name)
        for c in (g.a, g.b):
            if c is not None:
                stack.append(c)
    return sorted(out)


# ----------------------------------------------------------------------------
# Reduced ordered BDDs over obligation variables.
# ----------------------------------------------------------------------------
class BDD:
    def __init__(self):
        self.nodes = [None, None]           # 0 = false, 1 = true
        self.unique = {}
        self.var_formula = []               # variable index -> Node chi of O(chi)
        self.var_of = {}
        self._and, self._not = {}, {}

    def var(self, chi):
        v = self.var_of.get(chi.uid)
        if v is None:
            v = len(self.var_formula)
            self.var_formula.append(chi)
            self.var_of[chi.uid] = v
        return self.mk(v, 0, 1)

    def mk(self, v, lo, hi):
        if lo == hi:
            return lo
        key = (v, lo, hi)
        n = self.unique.get(key)
        if n is None:
            n = len(self.nodes)
            self.nodes.append(key)
            self.unique[key] = n
        return n

    def top(self, u):
        return self.nodes[u][0] if u > 1 else 1 << 30

    def neg(self, u):
        if u <= 1:
            return 1 - u
        r = self._not.get(u)
        if r is None:
            v, lo, hi = self.nodes[u]
            r = self.mk(v, self.neg(lo), self.neg(hi))
            self._not[u] = r
        return r

    def conj(self, u, w):
        if u == 0 or w == 0:
            return 0
        if u == 1:
            return w
        if w == 1 or u == w:
            return u
        if u > w:
            u, w = w, u
        r = self._and.get((u, w))
        if r is None:
            vu, vw = self.top(u), self.top(w)
            v = min(vu, vw)
            ulo, uhi = (self.nodes[u][1], self.nodes[u][2]) if vu == v else (u, u)
            wlo, whi = (self.nodes[w][1], self.nodes[w][2]) if vw == v else (w, w)
            r = self.mk(v, self.conj(ulo, wlo), self.conj(uhi, whi))
            self._and[(u, w)] = r
        return r

    def disj(self, u, w):
        return self.neg(self.conj(self.neg(u), self.neg(w)))

    def ite(self, c, t, e):
        return self.disj(self.conj(c, t), self.conj(self.neg(c), e))

    def at_end(self, u):
        """Value with every obligation variable false."""
        while u > 1:
            u = self.nodes[u][1]
        return u == 1

    def to_formula(self, u, memo=None):
        memo = {} if memo is None else memo
        if u == 0:
            return FF
        if u == 1:
            return TT
        if u in memo:
            return memo[u]
        v, lo, hi = self.nodes[u]
        chi = self.var_formula[v]
        f = Node("or", Node("and", chi, self.to_formula(hi, memo)),
                 Node("and", Node("not", chi), self.to_formula(lo, memo)))
        memo[u] = f
        return f


# ----------------------------------------------------------------------------
# Satisfiability over infinite words: GPVW tableau on negation normal form.
# ----------------------------------------------------------------------------
def nnf(f, neg=False):
    op = f.op
    if op == "tt":
        return FF if neg else TT
    if op == "ff":
        return TT if neg else FF
    if op == "ap":
        return Node("nap", name=f.name) if neg else f
    if op == "not":
        return nnf(f.a, not neg)
    if op == "and":
        return Node("or" if neg else "and", nnf(f.a, neg), nnf(f.b, neg))
    if op == "or":
        return Node("and" if neg else "or", nnf(f.a, neg), nnf(f.b, neg))
    if op == "X":
        return Node("X", nnf(f.a, neg))           # X is self-dual on infinite words
    if op == "U":                                  # !(a U b) = !a R !b
        return Node("R", nnf(f.a, True), nnf(f.b, True)) if neg else Node("U", nnf(f.a), nnf(f.b))
    if op == "R":
        return Node("U", nnf(f.a, True), nnf(f.b, True)) if neg else Node("R", nnf(f.a), nnf(f.b))
    raise ValueError(op)


def _complement_literal(f):
    if f.op == "ap":
        return Node("nap", name=f.name)
    if f.op == "nap":
        return ap(f.name)
    return None


def satisfiable(f, _cache={}):
    """Is there an infinite word over 2^AP satisfying f?  (GPVW + emptiness.)"""
    g = nnf(f)
    hit = _cache.get(g.uid)
    if hit is not None:
        return hit
    if g is TT:
        return True
    if g is FF:
        return False
    INIT = -1
    nodes = {}                        # (old, nxt) -> index
    incoming, olds = [], []
    stack = [(frozenset([INIT]), frozenset([g]), frozenset(), frozenset())]
    while stack:
        inc, new, old, nxt = stack.pop()
        if not new:
            key = (old, nxt)
            idx = nodes.get(key)
            if idx is not None:
                incoming[idx] |= inc
                continue
            idx = len(olds)
            nodes[key] = idx
            incoming.append(set(inc))
            olds.append(old)
            stack.append((frozenset([idx]), nxt, frozenset(), frozenset()))
            continue
        eta = next(iter(new))
        new = new - {eta}
        if eta in old:
            stack.append((inc, new, old, nxt))
            continue
        op = eta.op
        if op in ("tt", "ff", "ap", "nap"):
            if op == "ff" or _complement_literal(eta) in old:
                continue
            stack.append((inc, new, old | {eta}, nxt))
        elif op == "and":
            stack.append((inc, new | ({eta.a, eta.b} - old), old | {eta}, nxt))
        elif op == "or":
            stack.append((inc, new | ({eta.a} - old), old | {eta}, nxt))
            stack.append((inc, new | ({eta.b} - old), old | {eta}, nxt))
        elif op == "U":
            stack.append((inc, new | ({eta.a} - old), old | {eta}, nxt | {eta}))
            stack.append((inc, new | ({eta.b} - old), old | {eta}, nxt))
        elif op == "R":
            stack.append((inc, new | ({eta.b} - old), old | {eta}, nxt | {eta}))
            stack.append((inc, new | ({eta.a, eta.b} - old), old | {eta}, nxt))
        elif op == "X":
            stack.append((inc, new, old | {eta}, nxt | {eta.a}))
        else:
            raise ValueError(op)
    n = len(olds)
    succ = [[] for _ in range(n)]
    init = []
    for j in range(n):
        for i in incoming[j]:
            if i == INIT:
                init.append(j)
            else:
                succ[i].append(j)
    untils = set()
    for o in olds:
        for h in o:
            if h.op == "U":
                untils.add(h)
    # reachable part
    seen, todo = set(init), list(init)
    while todo:
        v = todo.pop()
        for w in succ[v]:
            if w not in seen:
                seen.add(w)
                todo.append(w)
    res = False
    for comp in _sccs(n, succ):
        if not (comp[0] in seen):
            continue
        cs = set(comp)
        if len(comp) == 1 and comp[0] not in succ[comp[0]]:
            continue
        ok = all(any(u.b in olds[v] or u not in olds[v] for v in comp) for u in untils)
        if ok:
            res = True
            break
    _cache[g.uid] = res
    return res


def _sccs(n, succ):
    """Strongly connected components (iterative Tarjan)."""
    index, low, on, stack, out = {}, {}, set(), [], []
    counter = 0
    for s in range(n):
        if s in index:
            continue
        call = [(s, iter(succ[s]))]
        index[s] = low[s] = counter
        counter += 1
        stack.append(s)
        on.add(s)
        while call:
            v, it = call[-1]
            advanced = False
            for w in it:
                if w not in index:
                    index[w] = low[w] = counter
                    counter += 1
                    stack.append(w)
                    on.add(w)
                    call.append((w, iter(succ[w])))
                    advanced = True
                    break
                if w in on:
                    low[v] = min(low[v], index[w])
            if advanced:
                continue
            call.pop()
            if call:
                low[call[-1][0]] = min(low[call[-1][0]], low[v])
            if low[v] == index[v]:
                comp = []
                while True:
                    w = stack.pop()
                    on.discard(w)
                    comp.append(w)
                    if w == v:
                        break
                out.append(comp)
    return out


def bdd_satisfiable(bdd, u, _cache={}):
    """Is some infinite word a model of the residual u?

    u holds on a word iff some path of the BDD to 1 is consistent with it, so
    u is satisfiable iff the conjunction of the obligation literals along some
    path is satisfiable."""
    found = [False]
    lits = []

    def walk(x):
        if found[0] or x == 0:
            return
        if x == 1:
            key = frozenset(lits)
            hit = _cache.get(key)
            if hit is None:
                f = TT
                for chi_uid, val in sorted(key):
                    chi = bdd.var_formula[bdd.var_of[chi_uid]]
                    f = Node("and", f, chi if val else Node("not", chi))
                hit = satisfiable(f)
                _cache[key] = hit
            found[0] = hit
            return
        v, lo, hi = bdd.nodes[x]
        uid = bdd.var_formula[v].uid
        lits.append((uid, True))
        walk(hi)
        lits[-1] = (uid, False)
        walk(lo)
        lits.pop()

    walk(u)
    return found[0]


# ----------------------------------------------------------------------------
# Progression
# ----------------------------------------------------------------------------
def _fltl_empty(f):
    op = f.op
    if op == "tt":
        return True
    if op in ("ff", "ap", "X", "U"):
        return False
    if op == "not":
        return not _fltl_empty(f.a)
    if op == "and":
        return _fltl_empty(f.a) and _fltl_empty(f.b)
    if op == "or":
        return _fltl_empty(f.a) or _fltl_empty(f.b)
    raise ValueError(op)


class _Progressor:
    def __init__(self, bdd):
        self.bdd = bdd
        self.memo = {}

    def prog(self, f, letter):
        """BDD of the obligation left after reading `letter` at the current position."""
        key = (f.uid, letter)
        r = self.memo.get(key)
        if r is not None:
            return r
        bdd, op = self.bdd, f.op
        if op == "tt":
            r = 1
        elif op == "ff":
            r = 0
        elif op == "ap":
            r = 1 if f.name in letter else 0
        elif op == "not":
            r = bdd.neg(self.prog(f.a, letter))
        elif op == "and":
            r = bdd.conj(self.prog(f.a, letter), self.prog(f.b, letter))
        elif op == "or":
            r = bdd.disj(self.prog(f.a, letter), self.prog(f.b, letter))
        elif op == "X":
            r = bdd.var(f.a)
        elif op == "U":
            r = bdd.disj(self.prog(f.b, letter), bdd.conj(self.prog(f.a, letter), bdd.var(f)))
        else:
            raise ValueError(op)
        self.memo[key] = r
        return r

    def step(self, u, letter, memo):
        """Residual u after one more letter: substitute every O(chi) by prog(chi)."""
        if u <= 1:
            return u
        r = memo.get(u)
        if r is None:
            v, lo, hi = self.bdd.nodes[u]
            c = self.prog(self.bdd.var_formula[v], letter)
            r = self.bdd.ite(c, self.step(hi, letter, memo), self.step(lo, letter, memo))
            memo[u] = r
        return r


@dataclass
class Monitor:
    """An LTL4 monitor (Def. 6) as the C ABI consumes it."""
    formula: str
    delta: np.ndarray        # [n_states, n_classes] uint8
    label: np.ndarray        # [n_states] uint8, verdict codes 0/2/3/5
    q0: int
    letters: list = None     # for letter-level monitors: the letter of every column

    @property
    def n_states(self):
        return int(self.delta.shape[0])

    @property
    def n_classes(self):
        return int(self.delta.shape[1])

    def run(self, classes):
        q = self.q0
        for c in classes:
            q = int(self.delta[q, c])
        return int(self.label[q])


def _minimise(delta, label, q0):
    """Moore minimisation by partition refinement; drops unreachable states.
    The result numbers states in breadth-first order from q0."""
    n, k = len(delta), len(delta[0]) if delta else 0
    reach, order = {q0}, [q0]
    for q in order:
        for c in range(k):
            if delta[q][c] not in reach:
                reach.add(delta[q][c])
                order.append(delta[q][c])
    block = {q: label[q] for q in order}
    while True:
        sig = {q: (block[q],) + tuple(block[delta[q][c]] for c in range(k)) for q in order}
        ids = {}
        nb = {q: ids.setdefault(sig[q], len(ids)) for q in order}
        if len(ids) == len(set(block.values())):
            block = nb
            break
        block = nb
    # renumber blocks breadth-first from q0
    num, bfs = {block[q0]: 0}, [q0]
    for q in bfs:
        for c in range(k):
            b = block[delta[q][c]]
            if b not in num:
                num[b] = len(num)
                bfs.append(delta[q][c])
    rep = {}
    for q in order:
        rep.setdefault(num[block[q]], q)
    m = len(num)
    nd = [[num[block[delta[rep[i]][c]]] for c in range(k)] for i in range(m)]
    nl = [label[rep[i]] for i in range(m)]
    return nd, nl, 0


def compile_letters(formula, max_states=4096):
    """Minimal LTL4 monitor over the letters 2^AP of the formula.

    Returns (delta, label, q0, letters) with letters[j] a frozenset."""
    f = parse_ltl(formula) if isinstance(formula, str) else formula
    aps = propositions(f)
    letters = [frozenset(c) for r in range(len(aps) + 1) for c in itertools.combinations(aps, r)]
    letters.sort(key=lambda s: sum(1 << aps.index(p) for p in s))
    bdd = BDD()
    pr = _Progressor(bdd)
    step_memo = {lt: {} for lt in letters}

    def label_of(u, end_value):
        if not bdd_satisfiable(bdd, bdd.neg(u)):
            return V_TOP
        if not bdd_satisfiable(bdd, u):
            return V_BOT
        return V_TOP_P if end_value else V_BOT_P

    # state 0 is the empty word; the others are residual BDDs
    if not satisfiable(Node("not", f)):
        lab0 = V_TOP
    elif not satisfiable(f):
        lab0 = V_BOT
    else:
        lab0 = V_TOP_P if _fltl_empty(f) else V_BOT_P
    index = {}
    residual = [None]
    labels = [lab0]
    delta = [None]
    todo = [0]
    while todo:
        q = todo.pop()
        row = []
        for lt in letters:
            if q == 0:
                u = pr.prog(f, lt)
            else:
                u = pr.step(residual[q], lt, step_memo[lt])
            j = index.get(u)
            if j is None:
                j = len(residual)
                if j > max_states:
                    raise ValueError(f"monitor of {formula!r} exceeds {max_states} states")
                index[u] = j
                residual.append(u)
                labels.append(label_of(u, bdd.at_end(u)))
                delta.append(None)
                todo.append(j)
            row.append(j)
        delta[q] = row
    nd, nl, q0 = _minimise(delta, labels, 0)
    return nd, nl, q0, letters


def compile_monitor(formula, class_props):
    """Compile `formula` into a class-indexed LTL4 monitor.

    class_props[c] is the set of propositions that hold in events of class c.
    The table is minimised over the classes and must fit the ABI's limits
    (at most 16 states and 16 classes).
    """
    if len(class_props) > MAX_CLASSES:
        raise ValueError("at most 16 event classes")
    nd, nl, q0, letters = compile_letters(formula)
    col = [letters.index(frozenset(p for p in cp if any(p in lt for lt in letters)))
           for cp in class_props]
    cd = [[row[c] for c in col] for row in nd]
    cd, cl, cq0 = _minimise(cd, nl, q0)
    if len(cd) > MAX_STATES:
        raise ValueError(f"{formula!r} needs {len(cd)} states; the ABI takes at most {MAX_STATES}")
    return Monitor(formula, np.array(cd, dtype=np.uint8).reshape(len(cd), len(class_props)),
                   np.array(cl, dtype=np.uint8), cq0)
