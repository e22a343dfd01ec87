"""Composition and embedding of star forests (Section 3.3): the library's
host graph algebra against the definitions written out in the oracle, and
both against what the operations mean -- Bcast on A.B equals Bcast on A then
on B, Reduce on A.B equals Reduce on B then on A, an embedded SF moves exactly
the selected part (checked with the oracle's Bcast / Reduce on integers)."""
import numpy as np
import pytest

import oracle
from paper_2102_13018_amd import sf as S


def rand_sf(rng, nroots, nleaves, leafspace, dup=True):
    ir = rng.integers(0, nroots, nleaves) if dup else rng.permutation(nroots)[:nleaves]
    il = rng.permutation(leafspace)[:nleaves]
    rk = np.sort(rng.integers(0, 3, nleaves))
    return nroots, ir.astype(np.int64), il.astype(np.int64), rk.astype(np.int64)


def lib_sf(g):
    return S.StarForest(g[0], g[1], g[2], g[3])


def graph_of(sf):
    il, ir, rk = sf.graph()
    return sf.nroots, ir, il, rk


def same_graph(a, b):
    return a[0] == b[0] and all(np.array_equal(x, y) for x, y in zip(a[1:], b[1:]))


@pytest.mark.parametrize("seed", range(6))
def test_compose_matches_definition_and_meaning(seed):
    rng = np.random.default_rng(300 + seed)
    A = rand_sf(rng, 40, 60, 90)
    B = rand_sf(rng, 90, 150, 200)
    AB = lib_sf(A).compose(lib_sf(B))
    g = graph_of(AB)
    assert same_graph(g, oracle.compose(A, B))
    # Bcast on AB == Bcast on A, then on B (on AB's leaves; the rest untouched)
    x = rng.integers(-1000, 1000, A[0]).astype(np.int64)
    mid = oracle.bcast(A[0], A[1], A[2], x, np.full(90, -7, np.int64))
    two = oracle.bcast(B[0], B[1], B[2], mid, np.full(200, -9, np.int64))
    one = oracle.bcast(g[0], g[1], g[2], x, np.full(200, -9, np.int64))
    assert np.array_equal(one[g[2]], two[g[2]])
    rest = np.setdiff1d(np.arange(200), g[2])
    assert np.all(one[rest] == -9)
    # Reduce SUM on AB == Reduce on B (onto zeros), then on A
    y = rng.integers(-1000, 1000, 200).astype(np.int64)
    mid = oracle.reduce(B[0], B[1], B[2], y, np.zeros(90, np.int64), "sum")
    two = oracle.reduce(A[0], A[1], A[2], mid, np.zeros(A[0], np.int64), "sum")
    one = oracle.reduce(g[0], g[1], g[2], y, np.zeros(A[0], np.int64), "sum")
    assert np.array_equal(one, two)


@pytest.mark.parametrize("seed", range(4))
def test_compose_inverse(seed):
    rng = np.random.default_rng(310 + seed)
    A = rand_sf(rng, 30, 70, 100)
    B = rand_sf(rng, 120, 80, 100, dup=False)   # every root of B has at most one leaf
    AB = lib_sf(A).compose_inverse(lib_sf(B))
    g = graph_of(AB)
    assert same_graph(g, oracle.compose_inverse(A, B))
    # Bcast on AB == Bcast on A, then B's leaves reduced (REPLACE) onto B's roots
    x = rng.integers(-1000, 1000, A[0]).astype(np.int64)
    lv = oracle.bcast(A[0], A[1], A[2], x, np.full(100, -7, np.int64))
    two = oracle.reduce(B[0], B[1], B[2], lv, np.full(B[0], -9, np.int64), "replace")
    one = oracle.bcast(g[0], g[1], g[2], x, np.full(B[0], -9, np.int64))
    assert np.array_equal(one[g[2]], two[g[2]])
    with pytest.raises(S.SfError):             # B with a root of two leaves
        lib_sf(A).compose_inverse(lib_sf((5, np.array([0, 0]), np.array([1, 2]), np.zeros(2, np.int64))))


@pytest.mark.parametrize("seed", range(4))
def test_embedded_sfs(seed):
    rng = np.random.default_rng(320 + seed)
    G = rand_sf(rng, 50, 120, 150)
    sf = lib_sf(G)
    roots = rng.choice(50, 17, replace=False)
    e = graph_of(sf.embedded_root_sf(roots))
    assert same_graph(e, oracle.embedded_root(G, roots))
    # Reduce on the embedded SF touches exactly the selected roots
    y = rng.integers(-100, 100, 150).astype(np.int64)
    r0 = rng.integers(-100, 100, 50).astype(np.int64)
    full = oracle.reduce(G[0], G[1], G[2], y, r0, "sum")
    part = oracle.reduce(e[0], e[1], e[2], y, r0, "sum")
    sel = np.zeros(50, bool)
    sel[roots] = True
    assert np.array_equal(part[sel], full[sel]) and np.array_equal(part[~sel], r0[~sel])
    slots = rng.choice(150, 60, replace=False)
    e = graph_of(sf.embedded_leaf_sf(slots))
    assert same_graph(e, oracle.embedded_leaf(G, slots))
    # Bcast on the leaf-embedded SF writes exactly the selected connected slots
    x = rng.integers(-100, 100, 50).astype(np.int64)
    full = oracle.bcast(G[0], G[1], G[2], x, np.full(150, -5, np.int64))
    part = oracle.bcast(e[0], e[1], e[2], x, np.full(150, -5, np.int64))
    keep = np.isin(np.arange(150), np.intersect1d(slots, G[2]))
    assert np.array_equal(part[keep], full[keep]) and np.all(part[~keep] == -5)
    with pytest.raises(S.SfError):
        sf.embedded_root_sf([50])
