"""Pins for the oracle's symbolic analysis (hand-worked cases, brute force, invariants)."""
import numpy as np
import pytest

from oracle import sym


def graph_csr(n, edges):
    rows = [[] for _ in range(n)]
    for a, b in edges:
        rows[a].append(b)
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([c for r in rows for c in r], dtype=np.int32)
    return rp, ci


def rows_of(S):
    return [S.front_rows(f).tolist() for f in range(S.nfronts)]


def test_worked_example_path7():
    # path 0-1-...-6, R empty, leaf_max 2 (hand-worked)
    rp, ci = graph_csr(7, [(i, i + 1) for i in range(6)])
    S = sym.analyze(7, rp, ci, [], leaf_max=2)
    assert S.perm.tolist() == [0, 2, 1, 4, 6, 5, 3]
    assert S.front_parent.tolist() == [2, 2, 6, 5, 5, 6, -1]
    assert rows_of(S) == [[0, 1], [2, 1, 3], [1, 3], [4, 5, 3], [6, 5], [5, 3], [3]]
    assert np.diff(S.front_ptr).tolist() == [1] * 7


def test_grid3x3():
    # 0-1-2 / 3-4-5 / 6-7-8, 4-neighbour, leaf_max 2 (hand-worked)
    e = []
    for r in range(3):
        for c in range(3):
            v = 3 * r + c
            if c < 2:
                e.append((v, v + 1))
            if r < 2:
                e.append((v, v + 3))
    rp, ci = graph_csr(9, e)
    S = sym.analyze(9, rp, ci, [], leaf_max=2)
    assert S.perm.tolist() == [1, 3, 0, 5, 7, 8, 2, 4, 6]
    assert S.front_parent.tolist() == [2, 2, 6, 5, 5, 6, -1]
    assert S.front_ptr.tolist() == [0, 1, 2, 3, 4, 5, 6, 9]
    assert rows_of(S) == [[1, 0, 2, 4], [3, 0, 4, 6], [0, 2, 4, 6], [5, 8, 2, 4],
                          [7, 8, 4, 6], [8, 2, 4, 6], [2, 4, 6]]


def test_star():
    rp, ci = graph_csr(7, [(0, i) for i in range(1, 7)])
    S = sym.analyze(7, rp, ci, [], leaf_max=2)
    assert S.perm.tolist() == [1, 2, 3, 4, 5, 6, 0]
    assert S.front_parent.tolist() == [6] * 6 + [-1]
    assert rows_of(S) == [[i, 0] for i in range(1, 7)] + [[0]]


def test_two_disjoint_paths_forest():
    rp, ci = graph_csr(6, [(0, 1), (1, 2), (3, 4), (4, 5)])
    S = sym.analyze(6, rp, ci, [], leaf_max=3)
    assert S.front_parent.tolist() == [-1, -1]
    assert rows_of(S) == [[0, 1, 2], [3, 4, 5]]


def test_root_set():
    rp, ci = graph_csr(5, [(i, i + 1) for i in range(4)])
    S = sym.analyze(5, rp, ci, [2], leaf_max=1)
    assert S.perm.tolist() == [0, 1, 3, 4, 2]
    assert S.front_parent.tolist() == [2, 2, -1]
    assert rows_of(S) == [[0, 1, 2], [3, 4, 2], [2]]
    # root pivots keep the given order
    rp, ci = graph_csr(6, [(i, i + 1) for i in range(5)])
    S = sym.analyze(6, rp, ci, [5, 3], leaf_max=3)
    assert S.perm.tolist() == [0, 1, 2, 4, 5, 3]
    assert S.front_parent.tolist() == [2, 2, -1]


def brute_fill(n, ptr, adj, perm):
    """Dense boolean elimination of the permuted A + A^T; returns L pattern (i > k)."""
    newidx = np.empty(n, dtype=np.int64)
    newidx[perm] = np.arange(n)
    M = np.zeros((n, n), dtype=bool)
    for v in range(n):
        for u in adj[ptr[v]:ptr[v + 1]]:
            M[newidx[v], newidx[u]] = True
    for k in range(n):
        rows = np.flatnonzero(M[k + 1:, k]) + k + 1
        if rows.size:
            M[np.ix_(rows, rows)] = True
    return np.tril(M, -1)


def check_invariants(S, n, rp, ci, root):
    assert sorted(S.perm.tolist()) == list(range(n))
    nf = S.nfronts
    assert S.front_ptr[-1] == n
    for f in range(nf):
        p = S.front_parent[f]
        assert p == -1 or p > f
        rows = S.front_rows(f)
        piv = S.perm[S.front_ptr[f]:S.front_ptr[f + 1]]
        assert rows[:piv.size].tolist() == piv.tolist()
        if p >= 0:
            assert set(rows[piv.size:].tolist()) <= set(S.front_rows(p).tolist())
        else:
            assert rows.size == piv.size
    ptr, adj = sym.symmetric_pattern(n, rp, ci)
    L = brute_fill(n, ptr, adj, S.perm)
    newidx = np.empty(n, dtype=np.int64)
    newidx[S.perm] = np.arange(n)
    front_of = np.repeat(np.arange(nf), np.diff(S.front_ptr))
    for k in range(n):
        f = front_of[k]
        struct = set(S.perm[np.flatnonzero(L[:, k])].tolist())
        assert struct <= set(S.front_rows(f).tolist())
        below = np.flatnonzero(L[:, k])
        assert S.var_etree[k] == (below[0] if below.size else -1)
    if len(root):
        assert S.perm[-len(root):].tolist() == list(root)


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 41))
    m = int(rng.integers(0, 3 * n + 1))
    e = [(int(a), int(b)) for a, b in rng.integers(0, n, size=(m, 2))]   # unsymmetric, self loops allowed
    rp, ci = graph_csr(n, e)
    nr = int(rng.integers(0, min(3, n) + 1))
    root = rng.permutation(n)[:nr].tolist()
    leaf = int(rng.choice([1, 2, 4, 8]))
    S = sym.analyze(n, rp, ci, root, leaf_max=leaf)
    check_invariants(S, n, rp, ci, root)


def test_grid_fill_and_etree():
    # 2D 5-point grid 7x6 (structured) with a root vertex; checks fill containment
    nx, ny = 7, 6
    e = []
    for i in range(nx):
        for j in range(ny):
            v = i * ny + j
            if i + 1 < nx:
                e.append((v, v + ny))
            if j + 1 < ny:
                e.append((v + 1, v))
    rp, ci = graph_csr(nx * ny, e)
    S = sym.analyze(nx * ny, rp, ci, [17], leaf_max=4)
    check_invariants(S, nx * ny, rp, ci, [17])


def test_bad_input():
    rp, ci = graph_csr(3, [(0, 1)])
    with pytest.raises(ValueError):
        sym.analyze(3, rp, ci, [3])
    with pytest.raises(ValueError):
        sym.analyze(3, rp, ci, [1, 1])
    with pytest.raises(ValueError):
        sym.analyze(3, rp, np.array([0], dtype=np.int32) + 5)


def test_empty():
    S = sym.analyze(0, np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), [])
    assert S.nfronts == 0 and S.perm.size == 0


def test_config0_invariants(config0):
    s = config0
    S = sym.analyze(s.n, s.rowptr, s.colind, s.root, leaf_max=64)
    assert S.perm[-2:].tolist() == s.root.tolist()
    assert S.front_parent[-1] == -1 and np.sum(S.front_parent == -1) == 1
    npiv = np.diff(S.front_ptr)
    # leaves are components of at most leaf_max vertices (this mesh has no
    # component of eccentricity below 2 that would be a larger leaf), and the root
    # front holds exactly the two position unknowns
    has_kid = np.zeros(S.nfronts, dtype=bool)
    has_kid[S.front_parent[S.front_parent >= 0]] = True
    assert npiv[~has_kid].max() <= 64
    assert npiv[-1] == 2
    # every separator is a proper separator: smaller than the subtree it splits
    sub = npiv.astype(np.int64).copy()
    for f in range(S.nfronts - 1):
        sub[S.front_parent[f]] += sub[f]
    assert np.all(npiv[has_kid] < sub[has_kid])
    for f in range(S.nfronts - 1):
        p = S.front_parent[f]
        rows = S.front_rows(f)
        assert set(rows[npiv[f]:].tolist()) <= set(S.front_rows(p).tolist())
