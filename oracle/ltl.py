"""Oracle, part 1: 4-valued LTL on finite words, written from the paper's definitions.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this module; only the tests, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP path or with the product's
monitor compiler.

What it computes
----------------
* The LTL syntax of Section 2.1 (Def. 3 restricted to 0-arity predicates):
  true, p, not, and, X, U.  Derived forms are expanded exactly as the paper
  states them: F p = true U p and G p = not F not p (end of Section 2.2.1);
  "or" and "->" are the usual Boolean abbreviations.
* FLTL (Def. 4): a finite-word semantics with a strong next (X at the last
  position is false) and an until whose witness must lie inside the word.
  `fltl` is that definition written out recursively over suffixes, with the
  existential/universal of the until spelled out literally.
* LTL4 (Def. 5): T / F when every / no infinite extension satisfies the
  formula, otherwise Tp / Fp by the FLTL value.  "Does some infinite extension
  satisfy it" is decided with the textbook Lichtenstein-Pnueli atom tableau
  (not taken from the paper): maximal locally-consistent assignments to the
  closure, successor consistency on X-formulas, and a self-fulfilling
  strongly connected component for the until eventualities.
* An LTL4 monitor (Def. 6) built from the same semantic state: the pair of
  atom sets reachable at the last position from atoms where the formula holds
  / fails.  This is a deterministic machine whose label is exactly Def. 5, so
  [u |=4 phi] = lambda(delta(q0, u)).  It is not minimised; the oracle only
  steps it.

Readings of the paper used here (every one is listed in the design notes):
* the word u_k / u^l in the until clause of Def. 4 both mean the suffix that
  starts at that position;
* the empty word: Def. 4/5 leave it undefined.  The initial state is labelled
  T/F if the formula is valid/unsatisfiable, otherwise by evaluating the
  formula with every proposition, X and U false and Boolean connectives
  classical (Tp if that is true, Fp if false).  No cluster is ever empty, so
  this label is never a verdict; it only fixes how many states a monitor has.

Verdict codes follow the lattice order of B6 (Section 2.3):
  F=0, Fc=1, Fp=2, Tp=3, Tc=4, T=5.
"""
from __future__ import annotations

import itertools
import re
from functools import lru_cache

BOT, BOT_C, BOT_P, TOP_P, TOP_C, TOP = 0, 1, 2, 3, 4, 5
VERDICT_NAMES = {BOT: "F", BOT_C: "Fc", BOT_P: "Fp", TOP_P: "Tp", TOP_C: "Tc", TOP: "T"}

# ----------------------------------------------------------------------------
# Syntax.  Formulas are nested tuples over the core grammar of Def. 3:
#   ("true",) ("ap", name) ("not", f) ("and", f, g) ("X", f) ("U", f, g)
# ----------------------------------------------------------------------------
TRUE = ("true",)


def Not(f):
    return ("not", f)


def And(f, g):
    return ("and", f, g)


def Or(f, g):
    return Not(And(Not(f), Not(g)))


def Implies(f, g):
    return Or(Not(f), g)


def Next(f):
    return ("X", f)


def Until(f, g):
    return ("U", f, g)


def Eventually(f):
    # F p = true U p  (Section 2.2.1)
    return Until(TRUE, f)


def Always(f):
    # G p = not F not p  (Section 2.2.1)
    return Not(Eventually(Not(f)))


_TOKEN = re.compile(r"\s*(->|[()!&|]|[A-Za-z_][A-Za-z0-9_]*)")


def _tokenize(text):
    pos, out = 0, []
    text = text.strip()
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if not m:
            raise ValueError(f"cannot parse formula at {text[pos:]!r}")
        out.append(m.group(1))
        pos = m.end()
        while pos < len(text) and text[pos].isspace():
            pos += 1
    return out


def parse(text):
    """Parse an LTL formula into the core grammar.

    Precedence (loosest first): ->, |, &, U (right-assoc), unary !, X, F, G.
    Atoms are lower-case identifiers; `true` / `false` are constants.
    """
    toks = _tokenize(text)
    pos = [0]

    def peek():
        return toks[pos[0]] if pos[0] < len(toks) else None

    def take(expected=None):
        t = peek()
        if t is None or (expected is not None and t != expected):
            raise ValueError(f"expected {expected!r} in {text!r}")
        pos[0] += 1
        return t

    def imp():
        lhs = disj()
        if peek() == "->":
            take()
            return Implies(lhs, imp())
        return lhs

    def disj():
        f = conj()
        while peek() == "|":
            take()
            f = Or(f, conj())
        return f

    def conj():
        f = until()
        while peek() == "&":
            take()
            f = And(f, until())
        return f

    def until():
        f = unary()
        if peek() == "U":
            take()
            return Until(f, until())
        return f

    def unary():
        t = peek()
        if t == "!":
            take()
            return Not(unary())
        if t == "X":
            take()
            return Next(unary())
        if t == "F":
            take()
            return Eventually(unary())
        if t == "G":
            take()
            return Always(unary())
        if t == "(":
            take()
            f = imp()
            take(")")
            return f
        if t == "true":
            take()
            return TRUE
        if t == "false":
            take()
            return Not(TRUE)
        if t is not None and re.fullmatch(r"[a-z_][a-z0-9_]*", t):
            take()
            return ("ap", t)
        raise ValueError(f"unexpected token {t!r} in {text!r}")

    f = imp()
    if peek() is not None:
        raise ValueError(f"trailing input in {text!r}")
    return f


def props(f):
    """Atomic propositions occurring in f, sorted."""
    out = set()

    def walk(g):
        if g[0] == "ap":
            out.add(g[1])
        for c in g[1:]:
            if isinstance(c, tuple):
                walk(c)

    walk(f)
    return sorted(out)


# ----------------------------------------------------------------------------
# Def. 4: FLTL on a finite non-empty word.  A word is a sequence of letters;
# a letter is a frozenset of the propositions that hold in that event.
# ----------------------------------------------------------------------------
def fltl(f, word):
    """[word |=F f], Def. 4, by direct recursion over suffixes."""
    n = len(word)
    if n == 0:
        raise ValueError("FLTL is defined on non-empty words only")
    memo = {}

    def val(g, i):  # value of g on the suffix starting at position i
        key = (g, i)
        if key in memo:
            return memo[key]
        op = g[0]
        if op == "true":
            r = True
        elif op == "ap":
            r = g[1] in word[i]
        elif op == "not":
            r = not val(g[1], i)
        elif op == "and":
            r = val(g[1], i) and val(g[2], i)
        elif op == "X":
            # strong next: false when the suffix has no second position
            r = val(g[1], i + 1) if i + 1 < n else False
        elif op == "U":
            # exists k in [i, n-1] with g2 at k and g1 at every l in [i, k)
            r = any(val(g[2], k) and all(val(g[1], l) for l in range(i, k))
                    for k in range(i, n))
        else:
            raise ValueError(op)
        memo[key] = r
        return r

    return val(f, 0)


def fltl_empty(f):
    """Reading for the empty word: propositions, X and U false; not/and classical."""
    op = f[0]
    if op == "true":
        return True
    if op in ("ap", "X", "U"):
        return False
    if op == "not":
        return not fltl_empty(f[1])
    if op == "and":
        return fltl_empty(f[1]) and fltl_empty(f[2])
    raise ValueError(op)


# ----------------------------------------------------------------------------
# Infinite-word LTL on ultimately periodic words x y^omega (used only to
# confirm witnesses; the standard semantics, evaluated on the finite lasso).
# ----------------------------------------------------------------------------
def ltl_lasso(f, prefix, loop):
    """Does the infinite word prefix . loop^omega satisfy f (standard LTL)?"""
    if not loop:
        raise ValueError("loop must be non-empty")
    word = list(prefix) + list(loop)
    n, start = len(word), len(prefix)

    def succ(i):
        return i + 1 if i + 1 < n else start

    memo = {}

    def vec(g):
        if g in memo:
            return memo[g]
        op = g[0]
        if op == "true":
            r = [True] * n
        elif op == "ap":
            r = [g[1] in word[i] for i in range(n)]
        elif op == "not":
            r = [not b for b in vec(g[1])]
        elif op == "and":
            a, b = vec(g[1]), vec(g[2])
            r = [x and y for x, y in zip(a, b)]
        elif op == "X":
            a = vec(g[1])
            r = [a[succ(i)] for i in range(n)]
        elif op == "U":
            # least fixpoint of  r = g2 | (g1 & X r)  on the lasso graph
            a, b = vec(g[1]), vec(g[2])
            r = list(b)
            changed = True
            while changed:
                changed = False
                for i in range(n):
                    if not r[i] and a[i] and r[succ(i)]:
                        r[i] = True
                        changed = True
        else:
            raise ValueError(op)
        memo[g] = r
        return r

    return vec(f)[0]


# ----------------------------------------------------------------------------
# Lichtenstein-Pnueli atom tableau for satisfiability over infinite words.
# ----------------------------------------------------------------------------
MAX_FREE_BITS = 14


class Tableau:
    """Atoms of the closure of `f`.

    Free bits of an atom: every proposition of f and every X-formula of the
    closure, where the closure contains X(g U h) for every until g U h.  All
    other closure members are fixed by local consistency:
      not g = not(g), g and h = g & h, g U h = h | (g & X(g U h)).
    Atom A may be followed by atom B iff for every X g in the closure,
    A[X g] == B[g].
    """

    def __init__(self, f):
        self.f = f
        subs = []

        def walk(g):
            for c in g[1:]:
                if isinstance(c, tuple):
                    walk(c)
            if g not in subs:
                subs.append(g)

        walk(f)
        for g in list(subs):
            if g[0] == "U" and ("X", g) not in subs:
                subs.append(("X", g))
        self.subs = subs
        self.aps = props(f)
        self.xforms = [g for g in subs if g[0] == "X"]
        self.untils = [g for g in subs if g[0] == "U"]
        nfree = len(self.aps) + len(self.xforms)
        if nfree > MAX_FREE_BITS:
            raise ValueError(f"formula too large for the oracle tableau ({nfree} free bits)")
        self.atoms = []          # list of dict: formula -> bool
        for bits in itertools.product((False, True), repeat=nfree):
            free = dict(zip([("ap", p) for p in self.aps] + self.xforms, bits))
            self.atoms.append(self._complete(free))
        self.n = len(self.atoms)
        # successor relation, grouped by the X-obligation vector
        want = [tuple(a[x] for x in self.xforms) for a in self.atoms]
        have = {}
        for j, b in enumerate(self.atoms):
            have.setdefault(tuple(b[x[1]] for x in self.xforms), []).append(j)
        self.succ = [have.get(w, []) for w in want]
        self.letter = [frozenset(p for p in self.aps if a[("ap", p)]) for a in self.atoms]
        self.good = self._good_atoms()

    def _complete(self, free):
        val = {}
        for g in self.subs:          # subs are in post-order: children first
            op = g[0]
            if op == "true":
                val[g] = True
            elif op in ("ap", "X"):
                val[g] = free[g]
            elif op == "not":
                val[g] = not val[g[1]]
            elif op == "and":
                val[g] = val[g[1]] and val[g[2]]
            elif op == "U":
                val[g] = val[g[2]] or (val[g[1]] and free[("X", g)])
        return val

    def _good_atoms(self):
        """Atoms from which an infinite, eventuality-fulfilling path starts."""
        n, succ = self.n, self.succ
        # Tarjan's SCC (iterative)
        index, low, onstack, stack, comp = [None] * n, [0] * n, [False] * n, [], [None] * n
        counter, ncomp = [0], [0]
        for root in range(n):
            if index[root] is not None:
                continue
            work = [(root, 0)]
            while work:
                v, pi = work.pop()
                if pi == 0:
                    index[v] = low[v] = counter[0]
                    counter[0] += 1
                    stack.append(v)
                    onstack[v] = True
                recurse = False
                for k in range(pi, len(succ[v])):
                    w = succ[v][k]
                    if index[w] is None:
                        work.append((v, k + 1))
                        work.append((w, 0))
                        recurse = True
                        break
                    if onstack[w]:
                        low[v] = min(low[v], index[w])
                if recurse:
                    continue
                if low[v] == index[v]:
                    while True:
                        w = stack.pop()
                        onstack[w] = False
                        comp[w] = ncomp[0]
                        if w == v:
                            break
                    ncomp[0] += 1
                if work:
                    u = work[-1][0]
                    low[u] = min(low[u], low[v])
        members = {}
        for v in range(n):
            members.setdefault(comp[v], []).append(v)
        fulfilling = set()
        for c, vs in members.items():
            vset = set(vs)
            nontrivial = len(vs) > 1 or any(w in vset for w in succ[vs[0]])
            if not nontrivial:
                continue
            ok = True
            for u in self.untils:
                if any(self.atoms[v][u] for v in vs) and not any(self.atoms[v][u[2]] for v in vs):
                    ok = False
                    break
            if ok:
                fulfilling.add(c)
        # backward reachability to fulfilling components
        pred = [[] for _ in range(n)]
        for v in range(n):
            for w in succ[v]:
                pred[w].append(v)
        good = [False] * n
        todo = [v for v in range(n) if comp[v] in fulfilling]
        for v in todo:
            good[v] = True
        while todo:
            w = todo.pop()
            for v in pred[w]:
                if not good[v]:
                    good[v] = True
                    todo.append(v)
        return good

    # -- per-word queries ---------------------------------------------------
    def reachable(self, word, polarity):
        """Atoms at the last position of atom sequences over `word` whose
        first atom gives f the truth value `polarity`."""
        f = self.f
        cur = {j for j, a in enumerate(self.atoms)
               if a[f] == polarity and self.letter[j] == _restrict(word[0], self.aps)}
        for letter in word[1:]:
            lt = _restrict(letter, self.aps)
            cur = {w for v in cur for w in self.succ[v] if self.letter[w] == lt}
        return cur

    def satisfiable(self):
        return any(self.good[j] for j, a in enumerate(self.atoms) if a[self.f])

    def valid(self):
        return not any(self.good[j] for j, a in enumerate(self.atoms) if not a[self.f])


def _restrict(letter, aps):
    return frozenset(p for p in letter if p in aps)


@lru_cache(maxsize=256)
def tableau(f):
    return Tableau(f)


def ltl4(f, word):
    """[word |=4 f], Def. 5, for a non-empty finite word."""
    if len(word) == 0:
        raise ValueError("LTL4 verdicts are taken on non-empty words")
    t = tableau(f)
    can_sat = any(t.good[j] for j in t.reachable(word, True))
    can_viol = any(t.good[j] for j in t.reachable(word, False))
    if not can_viol:
        return TOP
    if not can_sat:
        return BOT
    return TOP_P if fltl(f, word) else BOT_P


def ltl4_empty(f):
    """Label of the empty word under the reading stated in the module header."""
    t = tableau(f)
    if t.valid():
        return TOP
    if not t.satisfiable():
        return BOT
    return TOP_P if fltl_empty(f) else BOT_P


# ----------------------------------------------------------------------------
# Def. 6: a monitor whose states are the semantic state of the tableau.
# ----------------------------------------------------------------------------
class OracleMonitor:
    """Deterministic machine over the letters 2^AP of the formula.

    State 0 is the empty word.  Every other state is the pair
    (atoms reachable with f true at position 0, atoms reachable with f false),
    taken at the last position read.  `letters` lists the alphabet in the
    order used by `delta[q][letter_index]`.
    """

    def __init__(self, f, max_states=4096):
        t = tableau(f)
        self.f, self.aps = f, t.aps
        self.letters = [frozenset(c) for r in range(len(t.aps) + 1)
                        for c in itertools.combinations(t.aps, r)]
        self.letters.sort(key=lambda s: sum(1 << t.aps.index(p) for p in s))
        states = {None: 0}
        order = [None]
        delta, label = [], []
        q = 0
        while q < len(order):
            s = order[q]
            if s is None:
                label.append(ltl4_empty(f))
            else:
                pos, neg = s
                if not any(t.good[j] for j in neg):
                    label.append(TOP)
                elif not any(t.good[j] for j in pos):
                    label.append(BOT)
                else:
                    end_ok = any(not any(t.atoms[j][x] for x in t.xforms) for j in pos)
                    label.append(TOP_P if end_ok else BOT_P)
            row = []
            for lt in self.letters:
                if s is None:
                    pos = frozenset(j for j, a in enumerate(t.atoms) if a[f] and t.letter[j] == lt)
                    neg = frozenset(j for j, a in enumerate(t.atoms) if not a[f] and t.letter[j] == lt)
                else:
                    pos = frozenset(w for v in s[0] for w in t.succ[v] if t.letter[w] == lt)
                    neg = frozenset(w for v in s[1] for w in t.succ[v] if t.letter[w] == lt)
                nxt = (pos, neg)
                if nxt not in states:
                    if len(order) >= max_states:
                        raise ValueError("oracle monitor exceeds its state bound")
                    states[nxt] = len(order)
                    order.append(nxt)
                row.append(states[nxt])
            delta.append(row)
            q += 1
        self.delta, self.label, self.q0 = delta, label, 0
        self.n_states = len(order)

    def letter_index(self, letter):
        return self.letters.index(_restrict(letter, self.aps))

    def run(self, word):
        q = self.q0
        for lt in word:
            q = self.delta[q][self.letter_index(lt)]
        return self.label[q]

    def class_table(self, class_letters):
        """delta over event classes: class c carries the propositions class_letters[c]."""
        idx = [self.letter_index(frozenset(cl)) for cl in class_letters]
        return [[row[i] for i in idx] for row in self.delta]
