"""Pins of the oracle's Section 4 extensions against facts that do not come
from the oracle: brute-force enumeration on graphs of at most 16 nodes, an
identity with the plain clustering of the graph without the input
partition's cut edges, closed forms (member permutations, overlays, cliques,
the coarse-level bounds) and hand-worked examples (sub-rounds, two V-cycles).
"""
import json
import os
import random
from fractions import Fraction
from math import ceil, floor, gcd

import numpy as np
import pytest

import graphgen
import oracle
from tinygraphs import clique, family, from_edges

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def nbrs(g):
    ew = g.edge_weights()
    return [[(int(g.col[e]), int(ew[e])) for e in range(g.row_ptr[v], g.row_ptr[v + 1])] for v in range(g.n)]


def respecting_labels(rng, vblk, n):
    """Random labels whose clusters each lie inside one block: every node
    takes the label of a node of its own block."""
    by_block = {}
    for v in range(n):
        by_block.setdefault(int(vblk[v]), []).append(v)
    return np.array([rng.choice(by_block[int(vblk[v])]) for v in range(n)], np.int32)


def brute_rate_respect(g, lab, W, cap, rnd, vblk, active):
    """Every label t in [0, n) for every active node; t is a candidate iff it
    is the own label or a neighbour's label whose members all lie in v's
    block (membership read from the labels themselves)."""
    c = g.node_weights()
    N = nbrs(g)
    members = {}
    for u in range(g.n):
        members.setdefault(int(lab[u]), []).append(u)
    out, visits = [], 0
    for v in range(g.n):
        own = int(lab[v])
        if active is not None and not active[v]:
            out.append(own)
            continue
        visits += sum(1 for u, _ in N[v] if vblk[u] == vblk[v])
        best_key, best_t = None, own
        for t in range(g.n):
            conn = sum(w for u, w in N[v] if lab[u] == t)
            if t != own:
                if not any(lab[u] == t for u, _ in N[v]):
                    continue
                if any(vblk[u] != vblk[v] for u in members.get(t, [])):
                    continue
                if rnd % 2 == 1 and t > own:
                    continue
                if rnd % 2 == 0 and t < own:
                    continue
                if W[t] + c[v] > cap:
                    continue
            key = (conn, -t)
            if best_key is None or key > best_key:
                best_key, best_t = key, t
        out.append(best_t)
    return np.array(out, np.int32), visits


def test_respect_rating_brute_force():
    rng = random.Random(11)
    cases = 0
    for name, g in family(seed=5, count=70):
        n = g.n
        c = g.node_weights()
        for trial in range(3):
            k = rng.randint(1, max(1, min(n, 4)))
            vblk = np.array([rng.randrange(k) for _ in range(n)], np.int32)
            lab = respecting_labels(rng, vblk, n)
            W = np.zeros(n, np.int64)
            np.add.at(W, lab, c)
            lblk = np.zeros(n, np.int32)
            lblk[lab] = vblk  # the block of every used label
            cap = int(W.max()) + rng.randint(0, 3) if n else 1
            active = None if trial == 0 else np.array([rng.random() < 0.6 for _ in range(n)], np.uint8)
            for rnd in (1, 2):
                got, vis = oracle.rate_ext(g, lab, W, cap, rnd, 1, vblk, lblk, active)
                want, wvis = brute_rate_respect(g, lab, W, cap, rnd, vblk, active)
                assert np.array_equal(got, want), (name, trial, rnd)
                assert vis == wvis, (name, trial, rnd)
                cases += 1
    assert cases > 300


def test_respect_equals_plain_on_graph_without_cut_edges():
    """Clustering that respects a partition P (Appendix B.1) chooses among
    clusters inside v's block only; every neighbour u of such a cluster lies
    in v's block, so it equals the plain clustering of G minus P's cut edges,
    visit for visit."""
    rng = random.Random(3)
    graphs = [g for _, g in family(seed=9, count=40)] + [graphgen.rmat(9, 8, seed=s) for s in (1, 2)] + \
        [graphgen.rgg(400, 8.0, seed=4)]
    for gi, g in enumerate(graphs):
        n = g.n
        k = rng.randint(1, 5)
        vblk = np.array([rng.randrange(k) for _ in range(n)], np.int32)
        src = np.repeat(np.arange(n), np.diff(g.row_ptr))
        keep = vblk[src] == vblk[g.col]
        rp = np.zeros(n + 1, np.int64)
        rp[1:] = np.cumsum(np.bincount(src[keep], minlength=n))
        ew = None if g.ew is None else g.ew[keep]
        gp = graphgen.Graph(rp, g.col[keep].copy(), ew=ew, nw=g.nw)
        U = rng.randint(2, 12)
        for stop_rule in (0, 1):
            a = oracle.cluster_ext(g, U, 6, stop_rule, 1, vblk=vblk)
            b = oracle.cluster(gp, U, 6, stop_rule, 1)
            assert np.array_equal(a.labels, b.labels), gi
            assert a.rounds == b.rounds and a.moved == b.moved and a.visits == b.visits, gi


def test_respect_identity_with_member_labels():
    """The same identity from any initial labelling: a cluster starts as one
    node and only takes nodes of that node's block."""
    rng = random.Random(13)
    for gi in range(6):
        g = graphgen.rmat(9, 8, seed=gi + 1) if gi % 2 else graphgen.rgg(500, 8.0, seed=gi)
        n = g.n
        vblk = np.array([rng.randrange(3) for _ in range(n)], np.int32)
        src = np.repeat(np.arange(n), np.diff(g.row_ptr))
        keep = vblk[src] == vblk[g.col]
        rp = np.zeros(n + 1, np.int64)
        rp[1:] = np.cumsum(np.bincount(src[keep], minlength=n))
        gp = graphgen.Graph(rp, g.col[keep].copy(), ew=None, nw=g.nw)
        lab0 = oracle.member_labels(n, gi + 1)
        a = oracle.cluster_ext(g, 8, 6, 1, 1, vblk=vblk, lab0=lab0)
        b = oracle.cluster_ext(gp, 8, 6, 1, 1, lab0=lab0)
        assert np.array_equal(a.labels, b.labels) and a.moved == b.moved and a.visits == b.visits, gi


def test_respect_singletons_and_one_block():
    rng = random.Random(4)
    for name, g in family(seed=2, count=30):
        n = g.n
        # every node its own block: no move is possible
        r = oracle.cluster_ext(g, 10 ** 6, 4, 0, 1, vblk=np.arange(n, dtype=np.int32))
        assert np.array_equal(r.labels, np.arange(n)), name
        assert r.visits == 0 and sum(r.moved) == 0, name
        # one block: the plain clustering
        U = rng.randint(1, 8)
        a = oracle.cluster_ext(g, U, 5, 1, 1, vblk=np.zeros(n, np.int32))
        b = oracle.cluster(g, U, 5, 1, 1)
        assert np.array_equal(a.labels, b.labels) and a.moved == b.moved and a.visits == b.visits, name


def test_respecting_clusters_never_cross_blocks():
    rng = random.Random(8)
    for seed in range(6):
        g = graphgen.rmat(10, 8, seed=seed + 1) if seed % 2 == 0 else graphgen.rgg(900, 7.0, seed=seed)
        k = rng.choice((2, 4, 8))
        vblk = np.array([rng.randrange(k) for _ in range(g.n)], np.int32)
        r = oracle.cluster_ext(g, rng.randint(3, 40), 10, 1, 1, vblk=vblk, subrounds=rng.choice((0, 3)))
        for t in np.unique(r.labels):
            assert len(np.unique(vblk[r.labels == t])) == 1
        # contracting keeps every cut edge: the cut of the blocks is unchanged
        c = oracle.contract(g, r.labels)
        coarse_blk = np.zeros(c.n, np.int32)
        coarse_blk[c.coarse_of] = vblk
        assert oracle.cut(c, coarse_blk, k)[0] == oracle.cut(g, vblk, k)[0]


# ---------------------------------------------------------------- sub-rounds


def test_subround_hand_worked():
    d = json.load(open(os.path.join(GOLDEN, "subround_example.json")))
    g = from_edges(d["graph"]["n"], d["graph"]["edges"])
    p = oracle.cluster_ext(g, d["U"], d["rounds"], 0, 1)
    assert p.labels.tolist() == d["plain"]["labels"]
    assert p.moved == d["plain"]["moved"] and p.visits == d["plain"]["visits"]
    s = oracle.cluster_ext(g, d["U"], d["rounds"], 0, 1, subrounds=d["subrounds"]["S"])
    assert s.labels.tolist() == d["subrounds"]["labels"]
    assert s.moved == d["subrounds"]["moved"] and s.visits == d["subrounds"]["visits"]


def test_subrounds_brute_force_sequence():
    """A round of S sub-rounds is S plain rating + admission steps, each over
    the nodes of one degree class (0 below degree 4, else floor(log4 d),
    capped at S - 1), from the state the previous step left."""
    rng = random.Random(17)

    def cls(d, S):
        c = 0
        while d >= 4 and c < S - 1:
            d //= 4
            c += 1
        return c

    for name, g in family(seed=12, count=50):
        S = rng.choice((2, 3, 4))
        U = rng.randint(1, 9)
        deg = np.diff(g.row_ptr)
        lab = np.arange(g.n, dtype=np.int32)
        W = g.node_weights().astype(np.int64).copy()
        moved = []
        for rnd in (1, 2, 3):
            mv = 0
            for s in range(S):
                act = np.array([cls(int(x), S) == s for x in deg], np.uint8)
                desire, _ = oracle.rate_ext(g, lab, W, U, rnd, 1, None, None, act)
                assert np.all(desire[act == 0] == lab[act == 0])
                lab, W, _, m = oracle.admit_apply(g, desire, lab, W, U)
                mv += m
            moved.append(mv)
        r = oracle.cluster_ext(g, U, 3, 0, 1, subrounds=S)
        assert np.array_equal(r.labels, lab), name
        assert r.moved == moved, name
        assert r.visits == 3 * g.m, name


# ---------------------------------------------------------------- ensembles


def test_member_labels_closed_form():
    # worked by hand: n = 10, e = 1: a = 2654435761 mod 10 = 1, b = 2246822519 mod 10 = 9
    assert oracle.member_labels(10, 1).tolist() == [9, 0, 1, 2, 3, 4, 5, 6, 7, 8]
    # n = 12, e = 2: 5308871522 mod 12 = 2 -> 3, 4 share factors with 12 -> a = 5;
    # b = 4493645038 mod 12 = 10
    assert oracle.member_labels(12, 2).tolist() == [10, 3, 8, 1, 6, 11, 4, 9, 2, 7, 0, 5]
    assert oracle.member_labels(7, 0).tolist() == list(range(7))
    for n in (1, 2, 3, 16, 97, 1000):
        for e in range(5):
            p = oracle.member_labels(n, e)
            assert sorted(p.tolist()) == list(range(n))


def test_overlay_brute_force():
    rng = random.Random(21)
    for trial in range(200):
        n = rng.randint(0, 16)
        O = np.array([rng.randrange(max(1, n)) for _ in range(n)], np.int32)
        C = np.array([rng.randrange(max(1, n)) for _ in range(n)], np.int32)
        R, cnt = oracle.overlay(O, C)
        for u in range(n):
            for v in range(n):
                assert (R[u] == R[v]) == (O[u] == O[v] and C[u] == C[v])
        # numbered by first occurrence in node order
        seen = []
        for v in range(n):
            if R[v] not in seen:
                seen.append(int(R[v]))
        assert seen == list(range(len(seen))) and cnt == len(seen)


def test_member_on_disjoint_cliques():
    """Round 1 moves every node of a clique to the clique's smallest label
    (all its neighbours' labels tie at conn 1 and are smaller than its own
    or it is the smallest), for any initial labelling, when the clique fits
    in U; the overlay of such members is the cliques."""
    sizes = [3, 5, 4, 2, 6]
    edges, off, groups = [], 0, []
    for s in sizes:
        edges += clique(range(off, off + s))
        groups.append(list(range(off, off + s)))
        off += s
    g = from_edges(off, edges)
    for e in range(4):
        lab0 = oracle.member_labels(g.n, e)
        r = oracle.cluster_ext(g, 6, 3, 0, 1, lab0=lab0)
        for grp in groups:
            assert set(r.labels[grp].tolist()) == {int(lab0[grp].min())}
    ens = oracle.ensemble(g, 6, 4, 3, 0, 1)
    for grp in groups:
        assert len(set(ens.labels[grp].tolist())) == 1
    assert len(np.unique(ens.labels)) == len(groups)


def test_ensemble_invariants():
    rng = random.Random(5)
    for seed in range(4):
        g = graphgen.rmat(10, 8, seed=seed + 3) if seed % 2 else graphgen.rgg(800, 8.0, seed=seed)
        U = rng.randint(4, 30)
        E = rng.randint(2, 4)
        ens = oracle.ensemble(g, U, E, 10, 1, 1)
        c = g.node_weights()
        w = np.bincount(ens.labels, weights=c, minlength=g.n)
        assert w.max() <= U
        counts, visits, rounds = [], 0, 0
        moved = [0] * 10
        for e in range(E):
            r = oracle.cluster_ext(g, U, 10, 1, 1, lab0=oracle.member_labels(g.n, e))
            counts.append(len(np.unique(r.labels)))
            visits += r.visits
            rounds = max(rounds, r.rounds)
            for i, x in enumerate(r.moved):
                moved[i] += x
            # every overlay cluster lies inside one cluster of every member
            for t in np.unique(ens.labels):
                assert len(np.unique(r.labels[ens.labels == t])) == 1
        assert len(np.unique(ens.labels)) >= max(counts)
        assert ens.visits == visits and ens.rounds == rounds and ens.moved == moved[:rounds]
        one = oracle.ensemble(g, U, 1, 10, 1, 1)
        plain = oracle.cluster(g, U, 10, 1, 1)
        assert np.array_equal(one.labels, plain.labels)


# ---------------------------------------------------------------- coarse-level imbalance, V-cycles


def test_level_lmax_hand_values():
    # C = 1000, k = 4, eps = 3/100, delta = 1/10, q = 3 levels: ceil(C/k) = 250;
    # level 1: 1.03 + 0.1/2 = 1.08 -> 270; level 2: 1.03 + 0.1/1 = 1.13 -> 282.5 -> 282;
    # level 0: the plain L_max 257
    assert oracle.level_lmax(1000, 4, (3, 100), (1, 10), 3, 0, 257) == 257
    assert oracle.level_lmax(1000, 4, (3, 100), (1, 10), 3, 1, 257) == 270
    assert oracle.level_lmax(1000, 4, (3, 100), (1, 10), 3, 2, 257) == 282
    # C = 7, k = 2: ceil = 4; delta = 1/3, q = 2, level 1: (1 + 3/100 + 1/3) * 4 = 5.4533 -> 5
    assert oracle.level_lmax(7, 2, (3, 100), (1, 3), 2, 1, 4) == 5
    # delta 0: the plain bound on every level
    assert oracle.level_lmax(1000, 4, (3, 100), (0, 1), 5, 3, 257) == 257


def test_vcycle_hand_worked():
    d = json.load(open(os.path.join(GOLDEN, "vcycle_example.json")))
    g = from_edges(d["graph"]["n"], d["graph"]["edges"])
    part, st, cy = oracle.partition_ext(g, d["k"], tuple(d["eps"]), d["f"], threshold=d["threshold"], vcycles=2)
    assert st["lmax"] == d["bounds"]["lmax"] and st["U"] == d["bounds"]["U"]
    assert cy["cycles"] == 2 and cy["best"] == d["best"] and cy["visits"] == d["cycle_visits"]
    assert cy["cut"] == [d["cycle1"]["cut"], d["cycle2"]["cut"]]
    assert part.tolist() == d["cycle2"]["part"]
    # st describes the last cycle
    c2 = d["cycle2"]
    assert st["levels"] == c2["levels"] and st["rounds_c"][0] == c2["rounds_c"]
    assert st["moved_c"][0] == c2["moved_c"] and st["visits_c"][0] == c2["visits_c"]
    assert st["visits_r"] == c2["visits_r"] and st["ip_cut"] == c2["ip_cut"]
    # one cycle: the first cycle's hand-worked values
    part1, st1, cy1 = oracle.partition_ext(g, d["k"], tuple(d["eps"]), d["f"], threshold=d["threshold"])
    c1 = d["cycle1"]
    assert part1.tolist() == c1["part"] and st1["cut"] == c1["cut"] and st1["ip_cut"] == c1["ip_cut"]
    assert st1["rounds_c"][0] == c1["rounds_c"] and st1["moved_c"][0] == c1["moved_c"]
    assert st1["visits_c"][0] == c1["visits_c"] and st1["visits_r"] == c1["visits_r"]


def test_vcycle_coarsest_partition_keeps_cut_and_balance():
    """Cycle c >= 2 contracts no cut edge of its start partition, so its
    coarsest partition has the same cut (the start partition's, without the
    isolated nodes, which cut nothing)."""
    for seed, k in ((1, 4), (2, 8), (3, 2)):
        g = graphgen.rmat(11, 8, seed=seed)
        part, st, cy = oracle.partition_ext(g, k, vcycles=2)
        assert st["ip_cut"] == cy["cut"][0]
        part3, st3, cy3 = oracle.partition_ext(g, k, vcycles=3)
        assert cy3["cut"][:2] == cy["cut"]
        best = min(range(2), key=lambda i: (cy["max_block"][i] > st["lmax"], cy["cut"][i]))
        assert st3["ip_cut"] == cy["cut"][best]
        assert oracle.cut(g, part3, k)[0] == st3["cut"] == min(cy3["cut"]) or \
            max(cy3["max_block"]) > st3["lmax"]


def test_ext_defaults_equal_plain_partition():
    for g, k in ((graphgen.rmat(11, 8, seed=7), 8), (graphgen.rgg(3000, 8.0, seed=2), 4)):
        p1, s1 = oracle.partition(g, k)
        p2, s2, cy = oracle.partition_ext(g, k)
        assert np.array_equal(p1, p2) and s1 == s2 and cy["cycles"] == 1


def test_extra_imbalance_first_cycle_coarse_levels_only():
    """The refinement bounds used: level_lmax on the coarse levels of the
    first cycle, the plain L_max on level 0 and in every later cycle."""
    g = graphgen.rmat(11, 8, seed=5)
    part, st, cy = oracle.partition_ext(g, 4, vcycles=3, delta=(1, 5))
    C = g.n
    for c in range(cy["cycles"]):
        q = cy["levels"][c]
        for i in range(q):
            want = oracle.level_lmax(C, 4, (3, 100), (1, 5), q, i, st["lmax"]) if c == 0 else st["lmax"]
            assert cy["lmax"][c][i] == want, (c, i)
    assert cy["levels"][0] > 1 and cy["lmax"][0][1] > st["lmax"]


def test_extra_imbalance_only_changes_coarse_caps():
    """With delta > 0 the first cycle's coarse levels are refined against the
    larger bound; level 0 keeps L_max, so when refinement leaves no block
    overloaded the result is balanced; with a single level there is no
    coarse level and nothing changes."""
    g = graphgen.rmat(11, 8, seed=5)
    p0, s0, _ = oracle.partition_ext(g, 4)
    p1, s1, _ = oracle.partition_ext(g, 4, delta=(1, 5))
    assert s1["levels"] == s0["levels"] and s1["n_level"] == s0["n_level"]
    assert s1["ip_cut"] == s0["ip_cut"]
    small = graphgen.rmat(7, 8, seed=5)
    a, sa, _ = oracle.partition_ext(small, 2, threshold=10 ** 6)
    b, sb, _ = oracle.partition_ext(small, 2, threshold=10 ** 6, delta=(1, 2))
    assert np.array_equal(a, b) and sa == sb


def test_quality_at_scale_and_vcycles():
    """At larger sizes the synchronous reading cuts more than the paper's
    sequential SCLaP (the gap grows with n on mesh-like graphs); three
    V-cycles (Section 4) close it.  Bounds from the measured ratios (R-MAT
    2^16: 1.08, RGG 2^16: 1.17, RGG 2^17 with k = 16: 1.26; with three
    V-cycles 1.09, 0.94, 0.97)."""
    cases = [(graphgen.rmat(16, 16, seed=1), 8, 1.15, 1.12), (graphgen.rgg(1 << 16, 8.0, seed=1), 8, 1.25, 1.02),
             (graphgen.rgg(1 << 17, 10.0, seed=2), 16, 1.35, 1.02)]
    for g, k, sync_max, v3_max in cases:
        _, s_seq = oracle.seq_partition(g, k)
        _, s_sync = oracle.partition(g, k)
        _, s_v3, _ = oracle.partition_ext(g, k, vcycles=3)
        assert s_sync["cut"] <= sync_max * s_seq["cut"], g.name
        assert s_v3["cut"] <= v3_max * s_seq["cut"], g.name
        assert s_v3["cut"] <= s_sync["cut"], g.name
