"""Pins for the oracle's affinity graph, greedy clustering and shortest path."""
import os
import random

import networkx as nx
import pytest

from oracle import planner as P
from oracle.layout import aos, soa
from paper_1407_4859_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _sec(s):
    return (s.read, s.write, s.degree)


def test_affinity_config1_by_hand():
    secs = [_sec(s) for s in synth.config1_sections()]
    w = P.affinity(secs[:1], 8)
    # S1 touches f0, f1, f2, f3 at the same record: a 4-clique of weight 1
    for a in range(8):
        for b in range(8):
            want = 1 if (a != b and a < 4 and b < 4) else 0
            assert w[a][b] == want
    w = P.affinity(secs, 8)
    # S1 + S3 share f0..f3; S2 + S3 share f3..f5; S3 alone pairs everything else
    assert w[0][1] == 2 and w[0][3] == 2 and w[3][4] == 2 and w[3][5] == 2
    assert w[4][5] == 2 and w[0][7] == 1 and w[5][6] == 1 and w[0][6] == 1 and w[1][4] == 1
    assert min(w[a][b] for a in range(8) for b in range(8) if a != b) == 1


def test_affinity_gather_by_hand():
    w = P.affinity([([0, 1, 2], [3, 4], 16)], 6)
    assert w[0][1] == w[1][2] == w[0][2] == 16
    assert w[3][4] == 1
    assert w[0][3] == w[2][4] == 0 and w[5][0] == 0


def _read_table3():
    kv = {}
    with open(os.path.join(GOLDEN, "table3_kmeans_gpu_ods.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    groups = [list(range(int(a), int(b) + 1)) for a, b in
              (g.split("-") for g in kv["groups"].split())]
    return int(kv["fields"]), int(kv["elem_bytes"]), int(kv["cap_bytes"]), groups


def test_table3_four_structures_of_eight():
    F, e, cap, groups = _read_table3()
    got = P.ods_greedy([(list(range(F)), [], 0)], [e] * F, cap)
    assert got == groups


def _uniform_clique_opt(n, cap_fields):
    # best split of an n-clique into groups of at most c: as many full groups as possible
    q, r = divmod(n, cap_fields)
    return q * cap_fields * (cap_fields - 1) // 2 + r * (r - 1) // 2


@pytest.mark.parametrize("n,cap", [(5, 8), (6, 8), (7, 12), (8, 16), (9, 12)])
def test_greedy_optimal_on_uniform_cliques(n, cap):
    eb = [4] * n
    secs = [(list(range(n)), [], 0)]
    parts = P.ods_greedy(secs, eb, cap)
    w = P.affinity(secs, n)
    opt = P.best_partition_bruteforce(secs, eb, cap)
    assert P.intra_weight(parts, w) == opt == _uniform_clique_opt(n, cap // 4)


def test_greedy_feasible_and_bounded_by_bruteforce():
    rng = random.Random(5)
    gaps = 0
    for trial in range(150):
        n = rng.randint(2, 8)
        eb = [rng.choice([4, 8]) for _ in range(n)]
        secs = []
        for _ in range(rng.randint(1, 3)):
            fs = rng.sample(range(n), rng.randint(2, n))
            cut = rng.randint(1, len(fs))
            d = rng.choice([0, 0, 4, 16])
            secs.append((fs[:cut], fs[cut:] if d == 0 else fs[cut:][:2], d))
        cap = rng.choice([8, 12, 16, 24, 32])
        parts = P.ods_greedy(secs, eb, cap)
        acc = P.accessed(secs)
        for p in parts:
            assert sum(eb[f] for f in p) <= cap
            assert set(p) <= acc
        flat = [f for p in parts for f in p]
        assert len(flat) == len(set(flat))
        w = P.affinity(secs, n)
        opt = P.best_partition_bruteforce(secs, eb, cap)
        got = P.intra_weight(parts, w)
        assert got <= opt
        gaps += got < opt
    assert gaps < 150  # greedy is approximate, but usually optimal on small cases


def test_catalogue_order_and_dedup():
    n, eb = 100, [4] * 8
    secs = [_sec(s) for s in synth.config1_sections()]
    assert [L.key() for L in P.catalogue(secs, n, eb, 64, full=False)] == \
        [aos(n, eb).key(), soa(n, eb).key()]
    cat = P.catalogue(secs, n, eb, 64, full=True)
    keys = [L.key() for L in cat]
    assert len(keys) == len(set(keys))
    assert keys[0] == aos(n, eb).key() and keys[1] == soa(n, eb).key()
    # S1 alone clusters its four fields into one 16-byte structure
    assert any(L.groups[0] == ((0, 1, 2, 3), 1) for L in cat)


def _rand_tables(rng, k, C, lo=0, hi=50):
    T = [[rng.randint(lo, hi) for _ in range(C)] for _ in range(k)]
    R = [[0 if a == b else rng.randint(lo, hi) for b in range(C)] for a in range(C)]
    R0 = [rng.randint(lo, hi) for _ in range(C)]
    return T, R, R0


def test_dp_equals_bruteforce():
    rng = random.Random(9)
    for _ in range(200):
        k, C = rng.randint(1, 5), rng.randint(1, 5)
        T, R, R0 = _rand_tables(rng, k, C)
        for r0 in (None, R0):
            cost, path = P.pdl_dp(T, R, r0)
            bcost, _ = P.pdl_bruteforce(T, R, r0)
            assert cost == bcost
            assert P.path_cost(T, R, path, r0) == cost


def test_dp_unique_argmin_and_networkx():
    rng = random.Random(10)
    for _ in range(100):
        k, C = rng.randint(1, 6), rng.randint(2, 6)
        T, R, R0 = _rand_tables(rng, k, C, 0, 10 ** 6)
        cost, path = P.pdl_dp(T, R, R0)
        G = nx.DiGraph()
        for c in range(C):
            G.add_edge("src", (0, c), weight=R0[c] + T[0][c])
            G.add_edge((k - 1, c), "sink", weight=0)
        for s in range(1, k):
            for a in range(C):
                for b in range(C):
                    G.add_edge((s - 1, a), (s, b), weight=R[a][b] + T[s][b])
        assert nx.shortest_path_length(G, "src", "sink", weight="weight") == cost
        # with wide random costs the optimum is almost surely unique: paths agree
        if C ** k <= 5000:
            bcost, bpath = P.pdl_bruteforce(T, R, R0)
            assert bpath == path and bcost == cost


def test_dp_config1_brute_force_shape():
    # 3 sections, catalogue {AoS, SoA}: 8 combinations
    T = [[5, 3], [4, 6], [2, 9]]
    R = [[0, 1], [1, 0]]
    cost, path = P.pdl_dp(T, R)
    assert (cost, path) == (3 + 1 + 4 + 0 + 2, [1, 0, 0])
