"""Reference implementation of the paper's XOR straight-line-program passes.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Plain Python written
from the paper's definitions; used to pin the product compiler's passes.

Terms.  Constants (input arrays) and variables are both small non-negative
ints.  A program is a list of statements ``(var, [operands])`` plus a return
list of terms.  Value semantics are the set semantics of Sec. 4.1: the value
of a term is a set of constants and XOR is symmetric difference; sets are
encoded as Python ints used as bitsets over constant indices.

Readings where the paper leaves details open:
 * term order (Sec. 4.3): temporaries in creation order come before every
   constant; constants are ordered by index (strip index 8*block + strip);
 * pair frequency counts the original definitions containing both terms;
 * Rebuild (Sec. 4.4) considers every temporary, takes the one minimising the
   remainder (ties to the earliest temporary) and its result replaces the
   definition only when strictly shorter;
 * fusion (Sec. 5.2) never unfolds a returned variable; repeated operands
   cancel after unfolding; the earliest unfoldable statement is unfolded first;
 * the abstract LRU cache (Sec. 6.2) counts every load and every eviction;
 * the greedy heuristic (Sec. 6.6) breaks ties among movable cached pebbles by
   the term order of the variables they hold, and its ratio counts the
   distinct children of a node.
"""
from __future__ import annotations

from collections import Counter

ZERO = -1  # the all-zero array (value of an empty XOR)


# ------------------------------------------------------------ semantics
def const_bits(c: int) -> int:
    return 1 << c


def evaluate(stmts, outputs, n_const: int, is_const=None):
    """Set semantics (Sec. 4.1): returns the value (bitset) of every returned
    term.  ``is_const(t)`` tells constants from variables; by default terms
    below ``n_const`` are constants."""
    if is_const is None:
        is_const = lambda t: 0 <= t < n_const
    env = {}

    def val(t):
        if t == ZERO:
            return 0
        if is_const(t):
            return const_bits(t)
        return env[t]

    for v, ops in stmts:
        x = 0
        for o in ops:
            x ^= val(o)
        env[v] = x
    return [val(t) for t in outputs]


def count_xor(stmts) -> int:
    """#xor: a k-ary XOR statement costs k-1 binary XORs (Sec. 4.1, 5.1)."""
    return sum(len(ops) - 1 for _, ops in stmts)


def count_mem(stmts) -> int:
    """#M: k loads plus one store per k-ary statement (Sec. 5.1)."""
    return sum(len(ops) + 1 for _, ops in stmts)


def nvar(stmts) -> int:
    return len({v for v, _ in stmts})


# ------------------------------------------------------------ matrix -> SLP
def rows_from_bitmatrix(bits):
    """One returned original per bit row: the set of input strips (column
    indices) whose entry is 1 (the matrix-to-program map of Sec. 2)."""
    rows = []
    for r in range(len(bits)):
        s = 0
        for c, b in enumerate(bits[r]):
            if b:
                s |= 1 << c
        rows.append(s)
    return rows


def bits_to_list(s: int):
    out = []
    i = 0
    while s:
        if s & 1:
            out.append(i)
        s >>= 1
        i += 1
    return out


# ------------------------------------------------------------ RePair / XorRePair
class Compressed:
    """Result of (Xor)RePair: binary temporaries t_k = x xor y in creation
    order, and one returned term per original."""

    def __init__(self, n_const, temps, outputs):
        self.n_const = n_const
        self.temps = temps  # list of (x, y) term keys
        self.outputs = outputs  # list of term keys (or ZERO)

    # term key space: temporaries are 0..T-1, constant c is BIG + c
    BIG = 1 << 20

    def to_program(self):
        """Statements with variables numbered 0..T-1 and constants shifted to
        ``BIG + c``; returned terms likewise."""
        stmts = [(k, [x, y]) for k, (x, y) in enumerate(self.temps)]
        return stmts, list(self.outputs)

    def is_const(self, t):
        return t >= Compressed.BIG

    def xor_count(self):
        return len(self.temps)


def repair(rows, n_const: int, xor_rebuild: bool):
    """RePair (Sec. 4.3) and, with ``xor_rebuild``, XorRePair (Sec. 4.4).

    ``rows`` is one bitset of constants per original variable (flat
    definitions, as produced from a bitmatrix).  Returns ``Compressed``."""
    BIG = Compressed.BIG
    temps = []  # (x, y)
    tval = []  # bitset value of each temporary
    # current definitions of the originals still "below the line"
    defs = {}
    vals = {}
    alias = {}
    for i, s in enumerate(rows):
        vals[i] = s
        d = {BIG + c for c in bits_to_list(s)}
        defs[i] = d

    def settle():
        for i in list(defs):
            d = defs[i]
            if len(d) <= 1:
                alias[i] = next(iter(d)) if d else ZERO
                del defs[i]

    def term_val(t):
        return tval[t] if t < BIG else (1 << (t - BIG))

    def rebuild(i):
        rem = vals[i]
        chosen = []
        while True:
            best = None
            best_sz = rem.bit_count()
            for k, tv in enumerate(tval):
                sz = (rem ^ tv).bit_count()
                if sz < best_sz:
                    best, best_sz = k, sz
            if best is None:
                break
            rem ^= tval[best]
            chosen.append(best)
        return {BIG + c for c in bits_to_list(rem)} | set(chosen)

    settle()
    while defs:
        cnt = Counter()
        for d in defs.values():
            ds = sorted(d)
            for a in range(len(ds)):
                for b in range(a + 1, len(ds)):
                    cnt[(ds[a], ds[b])] += 1
        best_f = max(cnt.values())
        pair = min(p for p, f in cnt.items() if f == best_f)
        x, y = pair
        k = len(temps)
        temps.append(pair)
        tval.append(term_val(x) ^ term_val(y))
        for d in defs.values():
            if x in d and y in d:
                d.discard(x)
                d.discard(y)
                d.add(k)
        if xor_rebuild:
            for i in list(defs):
                nd = rebuild(i)
                if len(nd) < len(defs[i]):
                    defs[i] = nd
        settle()
    outputs = [alias[i] for i in range(len(rows))]
    return Compressed(n_const, temps, outputs)


# ------------------------------------------------------------ fusion
def fuse(stmts, outputs, is_const):
    """XOR fusion (Sec. 5.2): unfold every non-returned variable used exactly
    once into its user, until none is left.  The unfolded operands take the
    variable's place in the user's operand list; a term that then occurs an
    even number of times cancels (x xor x = 0), one that occurs an odd number
    of times keeps its first occurrence.  Statements keep their order; the
    earliest unfoldable statement is unfolded first, and statements left
    unused by a cancellation are dropped."""
    stmts = [(v, list(ops)) for v, ops in stmts]
    outset = set(outputs)
    while True:
        uses = Counter()
        for _, ops in stmts:
            for o in ops:
                if not is_const(o) and o != ZERO:
                    uses[o] += 1
        dead = {i for i, (v, _) in enumerate(stmts) if uses[v] == 0 and v not in outset}
        if dead:
            stmts = [s for i, s in enumerate(stmts) if i not in dead]
            continue
        target = None
        for i, (v, ops) in enumerate(stmts):
            if v not in outset and uses[v] == 1:
                target = i
                break
        if target is None:
            return stmts
        v, vops = stmts[target]
        for j, (w, wops) in enumerate(stmts):
            if v in wops:
                pos = wops.index(v)
                spliced = wops[:pos] + list(vops) + wops[pos + 1:]
                stmts[j] = (w, cancel(spliced))
                break
        del stmts[target]


def cancel(ops):
    """x xor x = 0: drop terms occurring an even number of times, keep the
    first occurrence of terms occurring an odd number of times."""
    cnt = Counter(ops)
    out = []
    for o in ops:
        if cnt[o] % 2 == 1 and o not in out:
            out.append(o)
    return out


# ------------------------------------------------------------ DFS schedule
def dfs_order(stmts, outputs, is_const):
    """Post-order of the computation graph (Sec. 6.4, 6.6): the goals (the
    returned variables) are the roots, visited in the order they are
    returned, then any other statement no statement uses, by variable;
    children are visited in term order (variables before constants).
    Returns the statements in the new order."""
    by_var = {v: ops for v, ops in stmts}
    used = set()
    for _, ops in stmts:
        for o in ops:
            if o in by_var:
                used.add(o)
    roots = []
    for o in outputs:
        if o in by_var and o not in roots:
            roots.append(o)
    roots += sorted(v for v, _ in stmts if v not in used and v not in roots)
    # goals not reachable as roots are still computed (they are used)
    seen = set()
    order = []

    def key(t):
        return (1, t) if is_const(t) else (0, t)

    def visit(v):
        stack = [(v, False)]
        while stack:
            node, done = stack.pop()
            if done:
                order.append(node)
                continue
            if node in seen:
                continue
            seen.add(node)
            stack.append((node, True))
            kids = sorted((o for o in by_var[node] if o in by_var), key=key)
            for kid in reversed(kids):
                if kid not in seen:
                    stack.append((kid, False))

    for r in roots:
        visit(r)
    return [(v, by_var[v]) for v in order]


def assign_pebbles(stmts, outputs, is_const):
    """Pebble assignment of the DFS heuristic (Sec. 6.6): each statement
    reuses a movable pebble (one on a node that is no longer needed and is
    not a goal) or takes a fresh one.  Among movable pebbles the most
    recently placed one is taken.  Returns (pebbled statements, returned
    pebbles, number of pebbles)."""
    last_use = {}
    for i, (v, ops) in enumerate(stmts):
        for o in ops:
            if not is_const(o) and o != ZERO:
                last_use[o] = i
    goals = set(o for o in outputs if not is_const(o) and o != ZERO)
    where = {}
    placed_at = {}
    free = []
    npeb = 0
    out = []
    for i, (v, ops) in enumerate(stmts):
        pops = [o if (is_const(o) or o == ZERO) else ("p", where[o]) for o in ops]
        # children whose last use is this statement and which are not goals
        for o in ops:
            if not is_const(o) and o != ZERO and last_use.get(o) == i and o not in goals:
                free.append(where[o])
        if free:
            p = max(free, key=lambda q: (placed_at[q], q))
            free.remove(p)
        else:
            p = npeb
            npeb += 1
        where[v] = p
        placed_at[p] = i
        out.append((("p", p), pops))
        if v not in goals and v not in last_use:
            free.append(p)
    ret = [o if (is_const(o) or o == ZERO) else ("p", where[o]) for o in outputs]
    return out, ret, npeb


def greedy_schedule(stmts, outputs, is_const, capacity: int):
    """Bottom-up greedy heuristic of Sec. 6.6 for an LRU cache of `capacity`
    entries.  Repeatedly: among the statements whose variable children are
    computed, take the one with the largest share of children already in the
    cache (ties to the earliest variable); touch the cached children, then
    the others, each group in term order; put the result on a movable
    pebble that is in the cache if there is one, else on any movable pebble,
    else on a fresh one (movable: it holds a variable that is neither
    returned nor used again; ties to the earliest held variable).
    Returns (pebbled statements, returned pebbles, number of pebbles) in the
    form of ``assign_pebbles``; cache entries are constants and ("p", k)."""
    def key(t):
        return (1, t) if is_const(t) else (0, t)

    kids = {}
    for v, ops in stmts:
        seen = []
        for o in ops:
            if o != ZERO and o not in seen:
                seen.append(o)
        kids[v] = seen
    uses = Counter(o for v in kids for o in kids[v] if not is_const(o))
    goals = set(o for o in outputs if not is_const(o) and o != ZERO)
    where = {}   # variable -> pebble
    holds = {}   # pebble -> variable it holds
    cache = []   # LRU entry first

    def entry(t):
        return t if is_const(t) else ("p", where[t])

    def touch(x):
        if x in cache:
            cache.remove(x)
        elif len(cache) >= capacity:
            cache.pop(0)
        cache.append(x)

    todo = sorted((v for v, _ in stmts), key=key)
    out = []
    npeb = 0
    while todo:
        best = None
        for v in todo:
            if any(not is_const(o) and o not in where for o in kids[v]):
                continue
            h = sum(1 for o in kids[v] if entry(o) in cache)
            c = len(kids[v])
            # h/c > bh/bc, with an empty statement scoring 0
            if best is None or h * best[2] > best[1] * max(c, 1):
                best = (v, h, max(c, 1))
        v = best[0]
        todo.remove(v)
        hit = sorted((o for o in kids[v] if entry(o) in cache), key=key)
        miss = sorted((o for o in kids[v] if entry(o) not in cache), key=key)
        args = [entry(o) for o in hit + miss]
        for x in args:
            touch(x)
        for o in kids[v]:
            if not is_const(o):
                uses[o] -= 1
        movable = [q for q, u in holds.items() if u not in goals and uses[u] == 0]
        cached = [q for q in movable if ("p", q) in cache]
        pool = cached or movable
        if pool:
            q = min(pool, key=lambda q: key(holds[q]))
        else:
            q = npeb
            npeb += 1
        touch(("p", q))
        where[v] = q
        holds[q] = v
        out.append((("p", q), args))
    ret = [o if (is_const(o) or o == ZERO) else ("p", where[o]) for o in outputs]
    return out, ret, npeb


# ------------------------------------------------------------ abstract LRU cache
def lru_run(stmts, capacity: int):
    """Run a program on the abstract LRU cache of Sec. 6.2.  Every statement
    touches/loads its arguments in order, then allocates/touches its result.
    Returns (loads, evictions, reloads).  Terms are any hashables; a term is
    a "load" the first time it appears as an argument and is not yet cached;
    a result is allocated for free."""
    cache = []  # LRU first
    seen = set()
    loads = evictions = reloads = 0

    def make_room():
        nonlocal evictions
        if len(cache) >= capacity:
            cache.pop(0)
            evictions += 1

    for v, ops in stmts:
        for o in ops:
            if o in cache:
                cache.remove(o)
                cache.append(o)
            else:
                make_room()
                cache.append(o)
                loads += 1
                if o in seen:
                    reloads += 1
            seen.add(o)
        if v in cache:
            cache.remove(v)
            cache.append(v)
        else:
            make_room()
            cache.append(v)
            seen.add(v)
    return loads, evictions, reloads


def iocost(stmts, capacity: int) -> int:
    """IOcost (Sec. 6.2): transfers memory->cache plus cache->memory."""
    loads, ev, _ = lru_run(stmts, capacity)
    return loads + ev


def ccap(stmts) -> int:
    """CCap (Sec. 6.2): the least capacity that runs without reloading.

    LRU has the inclusion property (what a cache of c entries holds at any
    moment, one of c + 1 entries holds too), so a program that runs without
    reloading at capacity c does so at every larger capacity and the least
    such capacity can be found by bisection.  It is at least the largest
    statement's arity + 1."""
    lo = max(len(ops) + 1 for _, ops in stmts)
    hi = lo
    while lru_run(stmts, hi)[2] != 0:
        hi *= 2
    while lo < hi:
        mid = (lo + hi) // 2
        if lru_run(stmts, mid)[2] != 0:
            lo = mid + 1
        else:
            hi = mid
    return lo
