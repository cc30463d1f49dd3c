"""Oracle: the two-level layout selection.  TEST INFRASTRUCTURE ONLY.

Level 1 (the ODS pass, section 2, first paragraph): an affinity graph over
the fields a section accesses, then greedy clustering of the fields into
structures whose size is bounded by an architecture-dependent capacity.

Level 2 (the PDL pass, section 2, second and third paragraphs): a rooted
DAG over the sections in program order, where keeping one layout across
consecutive sections is the "combine" choice (the layout of a combined run
is the ODS of the merged section) and changing layout costs a "remap";
the whole-program layout is a shortest path.

Plain Python on small inputs (at most 32 fields, a few sections, a few dozen
candidate layouts); brute-force enumerations are included for the tests.
"""
from __future__ import annotations

import itertools

from .layout import Layout, aos, soa, from_partition


# --------------------------------------------------------------- affinity
def affinity(sections, n_fields: int):
    """Affinity weights w[a][b] (symmetric, zero diagonal) summed over `sections`.

    Each section is (read_ids, write_ids, degree).  Per loop iteration, two
    fields touched at the same record co-occur once: a direct section
    (degree 0) adds 1 to every pair of R u W; a gather section adds `degree`
    to every pair of R (read together at each of the d neighbours), 1 to
    every pair of W, and nothing between R and W (different records).
    """
    w = [[0] * n_fields for _ in range(n_fields)]

    def bump(ids, amount):
        ids = sorted(set(ids))
        for x in range(len(ids)):
            for y in range(x + 1, len(ids)):
                w[ids[x]][ids[y]] += amount
                w[ids[y]][ids[x]] += amount

    for rd, wr, d in sections:
        if d == 0:
            bump(list(rd) + list(wr), 1)
        else:
            bump(rd, d)
            bump(wr, 1)
    return w


def accessed(sections):
    out = set()
    for rd, wr, _ in sections:
        out |= set(rd) | set(wr)
    return out


# --------------------------------------------------------------- greedy ODS
def ods_greedy(sections, elem_bytes, cap_bytes: int):
    """Greedy clustering of the affinity graph; returns the multi-field clusters.

    Clusters start as single fields.  Edges of positive weight are visited by
    decreasing weight, ties by (smaller id, larger id); an edge joins its two
    clusters when they differ and their combined bytes stay within cap_bytes.
    Fields no section touches stay on their own.
    """
    n = len(elem_bytes)
    w = affinity(sections, n)
    edges = sorted(((w[a][b], a, b) for a in range(n) for b in range(a + 1, n) if w[a][b] > 0),
                   key=lambda e: (-e[0], e[1], e[2]))
    cluster = list(range(n))
    members = {f: [f] for f in range(n)}
    size = {f: elem_bytes[f] for f in range(n)}
    for _, a, b in edges:
        ca, cb = cluster[a], cluster[b]
        if ca == cb or size[ca] + size[cb] > cap_bytes:
            continue
        keep, drop = min(ca, cb), max(ca, cb)
        for f in members[drop]:
            cluster[f] = keep
        members[keep] += members.pop(drop)
        size[keep] += size.pop(drop)
    return sorted(sorted(m) for m in members.values() if len(m) > 1)


def intra_weight(parts, w):
    return sum(w[a][b] for p in parts for a in p for b in p if a < b)


def set_partitions(items):
    """All set partitions of `items` (Bell-number many; tiny inputs only)."""
    items = list(items)
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for p in set_partitions(rest):
        yield [[first]] + p
        for i in range(len(p)):
            yield p[:i] + [[first] + p[i]] + p[i + 1:]


def best_partition_bruteforce(sections, elem_bytes, cap_bytes: int, fields=None):
    """Maximum intra-cluster affinity over all partitions within the cap."""
    n = len(elem_bytes)
    w = affinity(sections, n)
    fields = sorted(accessed(sections)) if fields is None else list(fields)
    best = -1
    for p in set_partitions(fields):
        if any(sum(elem_bytes[f] for f in part) > cap_bytes for part in p):
            continue
        best = max(best, intra_weight(p, w))
    return best


# --------------------------------------------------------------- catalogue
AOSOA_TILE = 64


def catalogue(sections, n: int, elem_bytes, cap_bytes: int, full: bool = True):
    """Candidate layouts, deduplicated, in a fixed order:
    AoS, SoA, AoS tiled by 64 records, then for every run of consecutive
    sections i..j (by i, then j) the ODS layout of the merged run, first
    interleaved (T = 1) then tiled (T = 64).  With full=False only AoS, SoA."""
    out = [aos(n, elem_bytes), soa(n, elem_bytes)]
    if full:
        out.append(Layout(n, elem_bytes, [0] * len(elem_bytes), [AOSOA_TILE]))
        k = len(sections)
        for i in range(k):
            for j in range(i, k):
                parts = ods_greedy(sections[i:j + 1], elem_bytes, cap_bytes)
                out.append(from_partition(n, elem_bytes, parts, 1))
                out.append(from_partition(n, elem_bytes, parts, AOSOA_TILE))
    seen, uniq = set(), []
    for L in out:
        if L.key() not in seen:
            seen.add(L.key())
            uniq.append(L)
    return uniq


def moving_fields(La: Layout, Lb: Layout):
    """Fields whose placement differs between La and Lb (section 2: the remap
    edge is weighted by the fields the two layouts have in common).  A
    field keeps its placement when its group in La and its group in Lb hold
    the same fields with the same tile: that group's bytes are then the
    same in both layouts and need not move.  Every other field moves."""
    out = []
    for f in range(len(La.elem_bytes)):
        if La.groups[La.group_of[f]] != Lb.groups[Lb.group_of[f]]:
            out.append(f)
    return out


def remap_bytes(La: Layout, Lb: Layout) -> int:
    """Algorithmic bytes of the remap La -> Lb: every moving field of every
    record is read once and written once, 2 * N * (sum of their element
    bytes); nothing when the layouts are equal."""
    return 2 * La.n * sum(La.elem_bytes[f] for f in moving_fields(La, Lb))


# --------------------------------------------------------------- shortest path
def pdl_dp(T, R, R0=None):
    """Shortest path through the layered DAG.

    T[s][c]: cost of section s under candidate c; R[a][b]: cost of remapping
    a -> b (R[a][a] = 0); R0[c]: cost of starting in c (0 if None).  Nodes
    are (s, c); source -> (0, c) weighs R0[c] + T[0][c]; (s-1, a) -> (s, b)
    weighs R[a][b] + T[s][b]; (k-1, c) -> sink weighs 0.  Ties go to the
    smallest candidate index.  Returns (cost, [c_0, ..., c_{k-1}])."""
    k, C = len(T), len(T[0])
    R0 = R0 if R0 is not None else [0] * C
    dist = [R0[c] + T[0][c] for c in range(C)]
    back = []
    for s in range(1, k):
        nd, bk = [], []
        for b in range(C):
            best, arg = None, -1
            for a in range(C):
                v = dist[a] + R[a][b]
                if best is None or v < best:
                    best, arg = v, a
            nd.append(best + T[s][b])
            bk.append(arg)
        dist = nd
        back.append(bk)
    end = min(range(C), key=lambda c: (dist[c], c))
    path = [end]
    for bk in reversed(back):
        path.append(bk[path[-1]])
    return dist[end], path[::-1]


def path_cost(T, R, path, R0=None):
    c = (R0[path[0]] if R0 is not None else 0) + T[0][path[0]]
    for s in range(1, len(path)):
        c += R[path[s - 1]][path[s]] + T[s][path[s]]
    return c


def pdl_bruteforce(T, R, R0=None):
    """Minimum over all C^k assignments (tiny k and C only)."""
    k, C = len(T), len(T[0])
    best, arg = None, None
    for combo in itertools.product(range(C), repeat=k):
        v = path_cost(T, R, combo, R0)
        if best is None or v < best:
            best, arg = v, list(combo)
    return best, arg


# --------------------------------------------------------------- branches
TOK_IF, TOK_ELSE, TOK_END = -1, -2, -3


def flow_paths(tokens, probs):
    """Every execution path of a structured program, with its probability.

    A path is a list of steps: ("s", section) runs a section, ("j", branch)
    is the join after branch `branch`.  A branch's first part runs with
    probability probs[branch], its second part (after ELSE, possibly empty)
    otherwise."""
    def parse(pos, counter):
        # a sequence up to ELSE / END / the end: list of items
        items = []
        while pos < len(tokens) and tokens[pos] not in (TOK_ELSE, TOK_END):
            t = tokens[pos]
            if t >= 0:
                items.append(("s", t))
                pos += 1
            else:
                b = counter[0]
                counter[0] += 1
                first, pos = parse(pos + 1, counter)
                second = []
                if tokens[pos] == TOK_ELSE:
                    second, pos = parse(pos + 1, counter)
                pos += 1                                   # END
                items.append(("b", b, first, second))
        return items, pos

    root, _ = parse(0, [0])

    def expand(items):
        # list of (probability, steps)
        out = [(1.0, [])]
        for it in items:
            if it[0] == "s":
                out = [(p, st + [it]) for p, st in out]
            else:
                _, b, first, second = it
                pa = probs[b]
                # each part with its own inner branches' probabilities
                alts = [(pa * q, s1 + [("j", b)]) for q, s1 in expand(first)] + \
                       [((1 - pa) * q, s2 + [("j", b)]) for q, s2 in expand(second)]
                out = [(p * q, st + s) for p, st in out for q, s in alts if q > 0.0]
        return out

    return expand(root)


def flow_expected_cost(tokens, probs, T, R, R0, start, nodes, joins):
    """Expected cost of an assignment: start node, a node per section and a
    node per join.  Along a path the data moves from node to node (R, zero
    when it stays) and every section costs T at its node."""
    total = 0.0
    for p, steps in flow_paths(tokens, probs):
        cur = start
        cost = R0[start] if R0 is not None else 0.0
        for st in steps:
            nxt = nodes[st[1]] if st[0] == "s" else joins[st[1]]
            if nxt != cur:
                cost += R[cur][nxt]
            cur = nxt
            if st[0] == "s":
                cost += T[st[1]][nxt]
        total += p * cost
    return total


def flow_bruteforce(tokens, probs, T, R, R0=None):
    """Least expected cost over every assignment (tiny cases only)."""
    k, C = len(T), len(T[0])
    nb = len(probs)
    best = None
    for start in range(C):
        for nodes in itertools.product(range(C), repeat=k):
            for joins in itertools.product(range(C), repeat=nb):
                c = flow_expected_cost(tokens, probs, T, R, R0, start, list(nodes), list(joins))
                if best is None or c < best[0]:
                    best = (c, start, list(nodes), list(joins))
    return best
