"""Interleavings of the hook's per-entry protocol, checked on the CPU.

The hook kernels run Algorithm 1 (Algorithm 3 with the zero root's keys when a
zero root is used, Sec. IV) with many threads on one parent array. This file
models the steps one thread takes, in the order the kernels take them:

- a thread holds a few entries; it tests all their bitmap bits, marks the
  unmarked endpoint of every entry with exactly one marked endpoint (that mark
  is the entry's link to the zero root), then reads the parents of the
  entries with neither endpoint marked, then hooks those one after the other;
- the walks use path splitting;
- a link is a CAS on the root's own entry, retried from the new parent when
  it fails;
- an entry found to end in the zero root's tree marks both endpoints in the
  bitmap.

Every access to the shared arrays is one step, and several such threads run
under every interleaving (small cases), under every interleaving with few
preemptions, or under many random schedules.

Every schedule must:
- give the oracle's labels;
- link each vertex at most once, only while it is a root, and never one the
  Initial Push already placed;
- leave a forest whose parents have smaller keys;
- set bitmap bits only for vertices in the zero root's component;
- with a zero root, give the oracle's labels after the compress and resolve
  model below (marks passed on to roots), in more than one vertex order.

Planted mistakes in the model (a link that is a plain store, a failed CAS
taken as done, an entry with one marked endpoint dropped without its mark)
must each be caught by one of these checks. In this model the zero root never
takes part in a link: its tree is z and the pushed vertices, all marked before
the hook starts, so an entry reaching it is settled by its bits. (On the
device a stale bit can still send such an entry to a walk that ends in z,
which is why the kernels keep Formula 1's keys.)

A second model, at the end of the file, covers the regrouped zero-root hook:
- the filter's marks stand in for links to z;
- the survivor hook follows;
- compress passes marks to roots and finds the smallest member of z's
  component, in any vertex order;
- resolve gives the final labels.

The model is sequentially consistent: each step sees every earlier write. The
device's weaker ordering across its L2 caches is covered by the kernels'
coherent stores and loads and tested on the device."""
import random

import numpy as np
import pytest

import oracle


class Shared:
    """The parent array and the zero root's membership bitmap, plus counters of
    what the protocol did (for the checks, not part of the method)."""

    def __init__(self, n, z):
        self.n = n
        self.z = z                    # None: plain path (Algorithm 1 keys)
        self.P = list(range(n))
        self.bit = [False] * n
        if z is not None:
            self.bit[z] = True        # the bitmap starts with z alone
        self.links = [0] * n          # successful link CASes per vertex
        self.linked_nonroot = False
        self.pushed = set()

    def copy(self):
        c = Shared(self.n, self.z)
        c.P, c.bit = list(self.P), list(self.bit)
        c.links, c.linked_nonroot, c.pushed = list(self.links), self.linked_nonroot, set(self.pushed)
        return c


def key(x, z):
    """Algorithm 3's Root-Function keys: the zero root first, then by ID."""
    if z is None:
        return x
    return 0 if x == z else x + 1


def find_root(sh, x, px, split):
    """Root of x, given px read from P[x] earlier; splitting points each visited
    vertex at its grandparent. Yields before every shared access."""
    if px == x:
        return x
    yield
    gp = sh.P[px]
    while gp != px:
        yield
        ggp = sh.P[gp]
        if split:
            yield
            sh.P[x] = gp
        x, px, gp = px, gp, ggp
    return px


def link(sh, u, pu, v, pv, split, bug, keyz):
    """Join the trees of u and v: the root with the greater key is linked under
    the other by a CAS that expects it to still be a root."""
    while True:
        ru = yield from find_root(sh, u, pu, split)
        rv = yield from find_root(sh, v, pv, split)
        if ru == rv:
            return ru
        lo, hi = (ru, rv) if key(ru, keyz) < key(rv, keyz) else (rv, ru)
        yield
        old = sh.P[hi]                          # the CAS: one indivisible step
        if bug == "store":
            if old != hi:
                sh.linked_nonroot = True
            sh.P[hi] = lo
            old = hi
        elif old == hi:
            sh.P[hi] = lo
        if old == hi:
            sh.links[hi] += 1
            return lo
        if bug == "no_retry":
            return lo
        u, pu, v, pv = hi, old, lo, lo


def thread(sh, entries, split, bug=None, stale=False):
    """One thread's entries: bitmap tests and marks, then parent reads, then the
    hooks. stale: the bit tests read a copy of the bitmap taken when the thread
    starts (the device may read bits through a stale cache line: set bits can
    read as clear, never the reverse)."""
    z = sh.z
    keyz = z
    k = len(entries)
    live = [u != v for u, v in entries]
    if z is not None:
        inu, inv = [False] * k, [False] * k
        yield
        bits = list(sh.bit) if stale else sh.bit
        for i, (u, v) in enumerate(entries):
            if live[i]:
                yield
                inu[i] = bits[u]
                yield
                inv[i] = bits[v]
        for i, (u, v) in enumerate(entries):
            if live[i] and inu[i] != inv[i] and bug != "no_mark":
                yield
                sh.bit[v if inu[i] else u] = True
            live[i] = live[i] and not inu[i] and not inv[i]
    pu, pv = [0] * k, [0] * k
    for i, (u, v) in enumerate(entries):
        if not live[i]:
            continue
        yield
        pu[i] = sh.P[u]
        yield
        pv[i] = sh.P[v]
    for i, (u, v) in enumerate(entries):
        if not live[i]:
            continue
        if pu[i] == pv[i]:
            r = pu[i]
        elif pu[i] == v:
            r = v
        elif pv[i] == u:
            r = u
        else:
            r = yield from link(sh, u, pu[i], v, pv[i], split, bug, keyz)
        if z is not None and r == z:
            yield
            sh.bit[u] = True
            yield
            sh.bit[v] = True


def initial_push(sh, edges):
    """Sec. IV's Initial Push before the hook: every neighbour of z is placed
    directly under z and marked."""
    z = sh.z
    for u, v in edges:
        if u == v:
            continue
        x = v if u == z else u if v == z else None
        if x is not None:
            sh.P[x] = z
            sh.bit[x] = True
            sh.pushed.add(x)


class Run:
    """A fresh shared state and its threads, advanced one step at a time."""

    def __init__(self, n, z, per_thread, split, bug=None, stale=False):
        self.sh = Shared(n, z)
        edges = [e for t in per_thread for e in t]
        if z is not None:
            initial_push(self.sh, edges)
        self.gens = {}
        for t, entries in enumerate(per_thread):
            g = thread(self.sh, entries, split, bug, stale)
            try:
                next(g)                     # up to the first shared access
                self.gens[t] = g
            except StopIteration:
                pass

    def enabled(self):
        return sorted(self.gens)

    def step(self, t):
        try:
            next(self.gens[t])
        except StopIteration:
            del self.gens[t]


def root(P, x):
    while P[x] != x:
        x = P[x]
    return x


def problems(sh, n, edges):
    """What is wrong with the final state, as a list of strings (empty: fine)."""
    out = []
    z = sh.z
    P = sh.P
    for x in range(n):
        if P[x] != x and not key(P[x], z) < key(x, z):
            out.append(f"parent of {x} is {P[x]}: key not smaller")
    if out:
        return out                      # not a forest: the walks below may not end
    if sh.linked_nonroot or any(c > 1 for c in sh.links):
        out.append(f"a vertex was linked twice or while not a root: {sh.links}")
    if any(sh.links[x] for x in sh.pushed):
        out.append("a pushed vertex was linked again")
    want = oracle.cc_labels(n, np.asarray(edges, np.uint32).reshape(-1, 2))
    ncomp = oracle.count_components(want)
    if z is None:
        if sum(sh.links) != n - ncomp:
            out.append(f"{sum(sh.links)} links != n - #components")
        roots = [root(P, x) for x in range(n)]
        low = {}
        for x in range(n):
            low.setdefault(roots[x], x)     # x increasing: the first member is the least
        got = np.array([low[r] for r in roots], np.uint32)
        if not np.array_equal(got, want):
            out.append(f"labels {got.tolist()} != oracle {want.tolist()}")
        return out
    # with a zero root some connections are recorded only as marks
    if sum(sh.links) + len(sh.pushed) > n - ncomp:
        out.append(f"{sum(sh.links)} links + {len(sh.pushed)} pushed > n - #components")
    for x in range(n):
        if sh.bit[x] and want[x] != want[z]:
            out.append(f"{x} is marked but not in the zero root's component")
    for order in (list(range(n)), list(range(n - 1, -1, -1))):
        got = compress_resolve(sh.copy(), order)
        if not np.array_equal(got, want):
            out.append(f"labels {got.tolist()} != oracle {want.tolist()} (order {order})")
    return out


def replay(case, prefix):
    r = Run(*case)
    for t in prefix:
        r.step(t)
    return r


def all_schedules(case, max_preempt=None):
    """Every schedule of the case's threads (depth-first, each prefix replayed
    from a fresh state), optionally only those with at most max_preempt
    switches away from a thread that could have continued. Yields the final
    state of each."""
    stack = [((), None, 0)]
    while stack:
        prefix, last, pre = stack.pop()
        r = replay(case, prefix)
        en = r.enabled()
        if not en:
            yield prefix, r.sh
            continue
        for t in en:
            cost = 1 if (last is not None and t != last and last in en) else 0
            if max_preempt is not None and pre + cost > max_preempt:
                continue
            stack.append((prefix + (t,), t, pre + cost))


def random_schedule(case, rng, stick=0.7):
    r = Run(*case)
    t = None
    while True:
        en = r.enabled()
        if not en:
            return r.sh
        if t not in en or rng.random() > stick:
            t = rng.choice(en)
        r.step(t)


def first_failure(case, schedules):
    n, per_thread = case[0], case[2]
    edges = [e for t in per_thread for e in t]
    for prefix, sh in schedules:
        bad = problems(sh, n, edges)
        if bad:
            return prefix, bad
    return None


# ---- exhaustive: two threads, tiny graphs ------------------------------------------

TINY = [
    # (n, z, per-thread entries): z None is the plain path
    (3, None, [[(2, 0)], [(2, 1)]]),            # two threads link the same root
    (4, None, [[(3, 1)], [(2, 0)], [(3, 2)]]),
    (4, None, [[(1, 2), (3, 0)], [(2, 3)]]),
    (5, None, [[(4, 3), (1, 0)], [(3, 1), (2, 4)]]),
    (4, 2, [[(0, 1)], [(3, 1)]]),               # zero root with no neighbours pushed
    (5, 2, [[(2, 0), (1, 3)], [(3, 4), (1, 0)]]),
    (5, 4, [[(0, 1), (4, 3)], [(1, 3), (2, 0)]]),
    (6, 0, [[(5, 4), (0, 3)], [(4, 3)], [(1, 2), (2, 5)]]),
]


@pytest.mark.parametrize("split", [True, False])
@pytest.mark.parametrize("i", range(len(TINY)))
def test_every_interleaving(i, split):
    n, z, per_thread = TINY[i]
    case = (n, z, per_thread, split)
    bound = None if sum(len(t) for t in per_thread) <= 3 else 3
    count = 0

    def counted():
        nonlocal count
        for s in all_schedules(case, bound):
            count += 1
            yield s

    assert first_failure(case, counted()) is None
    assert count > 1


# ---- random: three or four threads, random multigraphs ------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_random_schedules_stale_bits(seed):
    """As below, with every thread testing bits against a copy of the bitmap
    taken when it starts: a mark made meanwhile is missed, so the entry takes
    the walk (or marks again), and the labels are still the oracle's."""
    rng = random.Random(3000 + seed)
    n = rng.randint(3, 9)
    m = rng.randint(2, 12)
    edges = [(rng.randrange(n), rng.randrange(n)) for _ in range(m)]
    nt = rng.randint(2, 4)
    per_thread = [edges[t::nt] for t in range(nt)]
    z = rng.randrange(n)
    for split in (True, False):
        runs = []
        for _ in range(150):
            r = Run(n, z, per_thread, split, None, True)
            t = None
            while True:
                en = r.enabled()
                if not en:
                    break
                if t not in en or rng.random() > 0.7:
                    t = rng.choice(en)
                r.step(t)
            runs.append((None, r.sh))
        assert first_failure((n, z, per_thread, split), runs) is None, (n, z, per_thread, split)


@pytest.mark.parametrize("seed", range(12))
def test_random_schedules(seed):
    rng = random.Random(1000 + seed)
    n = rng.randint(3, 9)
    m = rng.randint(2, 12)
    edges = [(rng.randrange(n), rng.randrange(n)) for _ in range(m)]
    nt = rng.randint(3, 4)
    per_thread = [edges[t::nt] for t in range(nt)]
    for z in (None, rng.randrange(n)):
        for split in (True, False):
            case = (n, z, per_thread, split)
            runs = ((None, random_schedule(case, rng)) for _ in range(150))
            assert first_failure(case, runs) is None, (n, z, per_thread, split)


# ---- the checks catch planted mistakes ---------------------------------------------

@pytest.mark.parametrize("bug,case", [
    ("store", (3, None, [[(2, 0)], [(2, 1)]], True)),
    ("no_retry", (3, None, [[(2, 0)], [(2, 1)]], True)),
    ("store", (5, 2, [[(4, 1)], [(4, 3)]], True)),
    ("no_mark", (3, 2, [[(2, 0)], [(0, 1)]], True)),
    ("no_mark", (5, 0, [[(0, 1), (3, 4)], [(1, 2), (2, 3)]], True)),
])
def test_planted_mistakes_are_caught(bug, case):
    n, z, per_thread, split = case

    def buggy():
        stack = [()]
        while stack:
            prefix = stack.pop()
            r = Run(n, z, per_thread, split, bug)
            for t in prefix:
                r.step(t)
            en = r.enabled()
            if not en:
                yield prefix, r.sh
            stack.extend(prefix + (t,) for t in en)

    found = first_failure(case, buggy())
    assert found is not None, f"{bug}: no schedule shows it"
    prefix, bad = found
    assert bad


# ---- the regrouped zero-root hook: marks as links, then compress and resolve -------
#
# The regrouped hook runs the direct hook (with the bitmap) over a short warm-up,
# then a filter over the rest: an entry whose endpoints are both marked is
# dropped; with one marked, the other is marked (its link to z) and the entry is
# dropped; with neither, it is kept. A filter workgroup tests against its own
# copy of the bitmap, loaded when it starts and updated with its own marks, so it
# may miss marks set elsewhere meanwhile. The kept entries are then hooked with
# Algorithm 3's keys and no bitmap. Compress passes each marked vertex's mark to
# its root and collects the candidates for the smallest member of z's
# component; resolve labels every member of z's component with that minimum.

def warmup_thread(sh, entries, split):
    yield from thread(sh, entries, split)


def filter_thread(sh, entries, survivors, bug=None):
    yield
    seen = list(sh.bit)
    for u, v in entries:
        if u == v:
            continue
        mu, mv = seen[u], seen[v]
        if mu and mv:
            continue
        if mu != mv:
            if bug == "drop_unmarked":
                continue
            w = v if mu else u
            seen[w] = True
            yield
            sh.bit[w] = True
            continue
        survivors.append((u, v))


def survivor_thread(sh, entries, split):
    for u, v in entries:
        yield
        pu = sh.P[u]
        yield
        pv = sh.P[v]
        if pu == pv or pu == v or pv == u:
            continue
        yield from link(sh, u, pu, v, pv, split, None, sh.z)


def run_threads(gens, rng, stick=0.7):
    live = {}
    for i, g in enumerate(gens):
        try:
            next(g)
            live[i] = g
        except StopIteration:
            pass
    t = None
    while live:
        if t not in live or rng.random() > stick:
            t = rng.choice(sorted(live))
        try:
            next(live[t])
        except StopIteration:
            del live[t]


def compress_resolve(sh, order, bug=None):
    """Labels after compress (vertices visited in `order`: a root's own bit may
    be read before or after another vertex marks it) and resolve."""
    P, z = sh.P, sh.z
    bit = sh.bit
    cand = []
    for v in order:
        p = P[v]
        marked = bit[v]
        if p == v:
            if v == z or (marked and bug != "no_own_bit"):
                cand.append(v)
            continue
        r = root(P, v)
        if r == z:
            cand.append(v)
        elif marked:
            if bug != "no_propagation":
                bit[r] = True
            cand.append(r)
    minz = min(cand)
    out = []
    for v in range(sh.n):
        r = root(P, v)
        inz = r == z or bit[v] or bit[r]
        out.append(minz if inz else r)
    return np.array(out, np.uint32)


def regrouped_run(n, z, edges, rng, split=True, nwarm=1, nfilt=2, nsurv=2, bug=None):
    sh = Shared(n, z)
    initial_push(sh, edges)
    w = max(1, len(edges) // 5)
    warm, rest = edges[:w], edges[w:]
    run_threads([warmup_thread(sh, warm[i::nwarm], split) for i in range(nwarm)], rng)
    kept = [[] for _ in range(nfilt)]
    run_threads([filter_thread(sh, rest[i::nfilt], kept[i], bug) for i in range(nfilt)], rng)
    surv = [e for k in kept for e in k]
    run_threads([survivor_thread(sh, surv[i::nsurv], split) for i in range(nsurv)], rng)
    for x in range(n):
        if sh.P[x] != x:
            assert key(sh.P[x], z) < key(x, z), "parent with a greater key"
    order = list(range(n))
    rng.shuffle(order)
    return sh, compress_resolve(sh, order, bug)


@pytest.mark.parametrize("seed", range(16))
def test_regrouped_marks_compress_resolve(seed):
    """Random multigraphs and zero roots, random schedules of every phase and
    random compress orders: the labels are the oracle's, and every marked vertex
    lies in the zero root's component."""
    rng = random.Random(2000 + seed)
    for _ in range(40):
        n = rng.randint(2, 10)
        m = rng.randint(1, 16)
        edges = [(rng.randrange(n), rng.randrange(n)) for _ in range(m)]
        z = rng.randrange(n)
        want = oracle.cc_labels(n, np.asarray(edges, np.uint32).reshape(-1, 2))
        for split in (True, False):
            sh, got = regrouped_run(n, z, edges, rng, split)
            assert np.array_equal(got, want), (n, z, edges, got.tolist(), want.tolist())
            marked = [x for x in range(n) if sh.bit[x]]
            assert all(want[x] == want[z] for x in marked), (n, z, edges)


# Each case is built so that one planted mistake changes its labels:
# - a root marked by the filter whose tree has no other marked member is the
#   component's minimum (only its own bit makes it a candidate);
# - a vertex marked by the filter whose root is unmarked (only the mark passed
#   on to the root joins that tree to z's component).
REGROUPED_BUGS = [
    ("no_own_bit", 4, 3, [(3, 1), (0, 2), (1, 0), (1, 0), (1, 0), (1, 0)]),
    ("no_propagation", 5, 4, [(4, 3), (2, 1), (4, 0), (3, 2), (3, 2), (3, 2), (3, 2)]),
    ("drop_unmarked", 5, 4, [(4, 3), (2, 1), (4, 0), (3, 2), (3, 2), (3, 2), (3, 2)]),
]


@pytest.mark.parametrize("bug,n,z,edges", REGROUPED_BUGS)
def test_regrouped_planted_mistakes_are_caught(bug, n, z, edges):
    want = oracle.cc_labels(n, np.asarray(edges, np.uint32).reshape(-1, 2))
    rng = random.Random(7)
    sh, good = regrouped_run(n, z, edges, rng, nwarm=1, nfilt=1, nsurv=1)
    assert np.array_equal(good, want)
    caught = False
    for s in range(20):
        sh, got = regrouped_run(n, z, edges, random.Random(s), nwarm=1, nfilt=1, nsurv=1, bug=bug)
        caught |= not np.array_equal(got, want)
    assert caught, f"{bug}: not caught"
