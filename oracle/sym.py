"""Oracle symbolic analysis: the specified nested-dissection front tree.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper computes its fill-reducing ordering once, in the direct solver's
analysis phase, and reuses it for every later factorization because the
sparsity pattern never changes (Sec. 6, "Scaling").  Its orderings (ParMetis in
2D, Scotch in 3D) cannot be reproduced bit for bit, so the analysis is replaced
by a fully specified one whose every order-sensitive choice is an explicit
tie-break:

1. G = pattern(A) union pattern(A^T), no self loops; the root set R (the two
   rigid-position dofs) is removed.
2. Connected components of what remains, in order of their minimum vertex.
3. ND(K): |K| <= leaf_max -> leaf front (pivots: K ascending).  Otherwise a
   George-Liu pseudo-peripheral root: r = min(K); BFS levels L_0..L_e; in L_e
   take the vertex x of minimum degree within K (lowest index on ties); if
   ecc(x) > e then r = x and repeat, else keep r.  If e < 2, K is a leaf.
   Split level j = smallest index with 2|L_0..L_j| >= |K|, clamped to
   [1, e-1]; separator S = vertices of L_j with a neighbour in L_{j+1}.
   ND is applied to the components of K \\ S in min-index order, then S is
   emitted as a separator front (pivots ascending) whose children are those
   components' top fronts.
4. R is emitted as the root front (pivots in the given order) whose children
   are the top fronts of step 2; with R empty there may be several roots.
5. Fronts are numbered in completion order (a postorder); perm concatenates the
   front pivot lists.
6. rows(f) = pivots(f), then, ascending in the new numbering, the union of the
   children's non-pivot rows and the neighbours (in G with R kept) of f's pivots
   numbered after f's last pivot.
7. var_etree = Liu's elimination tree of the permuted A + A^T.

Pins: the hand-worked path-graph example, hand cases, brute-force boolean
elimination on small graphs (every fill entry lies inside a front), and
structural invariants -- see tests/test_oracle_sym.py.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

SPEC_VERSION = 1


@dataclass
class Symbolic:
    n: int
    leaf_max: int
    perm: np.ndarray          # int32[n]: new position -> original var
    front_ptr: np.ndarray     # int32[nf+1]: pivot ranges in the new numbering
    front_parent: np.ndarray  # int32[nf]: -1 for a root
    rows_ptr: np.ndarray      # int64[nf+1]
    rows: np.ndarray          # int32[...]: front rows as original vars (pivots first)
    var_etree: np.ndarray     # int32[n]: parent in the new numbering, -1 for roots

    @property
    def nfronts(self) -> int:
        return int(self.front_parent.size)

    def front_rows(self, f: int) -> np.ndarray:
        return self.rows[self.rows_ptr[f]:self.rows_ptr[f + 1]]

    def npiv(self, f: int) -> int:
        return int(self.front_ptr[f + 1] - self.front_ptr[f])


def symmetric_pattern(n, rowptr, colind):
    """Adjacency (CSR, sorted, no self loops) of pattern(A) union pattern(A^T)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    if rowptr.size != n + 1 or rowptr[0] != 0 or np.any(np.diff(rowptr) < 0):
        raise ValueError("bad rowptr")
    if colind.size != rowptr[-1] or (colind.size and (colind.min() < 0 or colind.max() >= n)):
        raise ValueError("bad colind")
    r = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    keep = r != colind
    r, c = r[keep], colind[keep]
    rr = np.concatenate([r, c])
    cc = np.concatenate([c, r])
    g = sp.coo_matrix((np.ones(rr.size, dtype=np.int8), (rr, cc)), shape=(n, n)).tocsr()
    g.sum_duplicates()
    g.sort_indices()
    return g.indptr.astype(np.int64), g.indices.astype(np.int64)


class _Graph:
    def __init__(self, n, ptr, adj):
        self.n, self.ptr, self.adj = n, ptr, adj
        self.mask = np.zeros(n, dtype=bool)      # current vertex subset
        self.lev = np.full(n, -1, dtype=np.int64)

    def neighbours(self, vs):
        """Concatenated adjacency lists of the vertices vs."""
        s = self.ptr[vs]
        ln = self.ptr[vs + 1] - s
        tot = int(ln.sum())
        if tot == 0:
            return np.empty(0, dtype=np.int64)
        off = np.repeat(s - np.cumsum(ln) + ln, ln)
        return self.adj[off + np.arange(tot)]

    def bfs_levels(self, r):
        """Level sets of a BFS from r inside the current mask."""
        levels = [np.array([r], dtype=np.int64)]
        self.lev[r] = 0
        front = levels[0]
        d = 0
        touched = [front]
        while True:
            nb = self.neighbours(front)
            nb = nb[self.mask[nb] & (self.lev[nb] < 0)]
            if nb.size == 0:
                break
            nb = np.unique(nb)
            d += 1
            self.lev[nb] = d
            levels.append(nb)
            touched.append(nb)
            front = nb
        return levels

    def clear_levels(self, levels):
        for lv in levels:
            self.lev[lv] = -1

    def components(self, K):
        """Components of the vertex set K (sorted), ordered by minimum vertex."""
        self.mask[K] = True
        seen_local = []
        comps = []
        for v in K:                      # ascending: each new component starts at its min
            if self.lev[v] >= 0:
                continue
            levels = self.bfs_levels(int(v))
            comp = np.sort(np.concatenate(levels))
            comps.append(comp)
            seen_local.append(levels)
        for levels in seen_local:
            self.clear_levels(levels)
        self.mask[K] = False
        return comps


def analyze(n, rowptr, colind, root=(), leaf_max=64) -> Symbolic:
    """Symbolic analysis of the spec; returns the bit-exact outputs."""
    if leaf_max < 1:
        raise ValueError("leaf_max must be >= 1")
    root = np.asarray(root, dtype=np.int64).ravel()
    if root.size and (root.min() < 0 or root.max() >= n or np.unique(root).size != root.size):
        raise ValueError("bad root list")
    ptr, adj = symmetric_pattern(n, rowptr, colind)
    g = _Graph(n, ptr, adj)

    fronts_piv = []      # pivots (original ids) per front, in completion order
    fronts_children = []

    def emit(piv, children):
        fronts_piv.append(np.asarray(piv, dtype=np.int64))
        fronts_children.append(list(children))
        return len(fronts_piv) - 1

    def nd(K):
        # explicit stack to avoid deep recursion: frames are (K, state)
        stack = [[K, None, None, 0, []]]   # K, S, comps, next comp, child tops
        ret = None
        while stack:
            fr = stack[-1]
            if fr[1] is None:
                Kc = fr[0]
                if Kc.size <= leaf_max:
                    ret = emit(Kc, [])
                    stack.pop()
                    if stack:
                        stack[-1][4].append(ret)
                    continue
                S = separator(Kc)
                if S is None:
                    ret = emit(Kc, [])
                    stack.pop()
                    if stack:
                        stack[-1][4].append(ret)
                    continue
                rest = np.setdiff1d(Kc, S, assume_unique=True)
                fr[1] = S
                fr[2] = g.components(rest)
                fr[3] = 0
            if fr[3] < len(fr[2]):
                C = fr[2][fr[3]]
                fr[3] += 1
                stack.append([C, None, None, 0, []])
                continue
            ret = emit(fr[1], fr[4])
            stack.pop()
            if stack:
                stack[-1][4].append(ret)
        return ret

    def separator(K):
        g.mask[K] = True
        r = int(K[0])
        levels = g.bfs_levels(r)
        e = len(levels) - 1
        while True:
            Le = levels[-1]
            nb_counts = _deg_within(g, Le)
            x = int(Le[np.lexsort((Le, nb_counts))[0]])
            g.clear_levels(levels)
            lx = g.bfs_levels(x)
            if len(lx) - 1 > e:
                levels, e, r = lx, len(lx) - 1, x
                continue
            g.clear_levels(lx)
            levels = g.bfs_levels(r)     # keep r's level structure
            break
        if e < 2:
            g.clear_levels(levels)
            g.mask[K] = False
            return None
        sizes = np.cumsum([lv.size for lv in levels])
        j = int(np.flatnonzero(2 * sizes >= K.size)[0])
        j = min(max(j, 1), e - 1)
        Lj = levels[j]
        # S = vertices of L_j with a neighbour in L_{j+1}
        s = g.ptr[Lj]
        ln = g.ptr[Lj + 1] - s
        nb = g.neighbours(Lj)
        owner = np.repeat(np.arange(Lj.size), ln)
        hit = g.mask[nb] & (g.lev[nb] == j + 1)
        S = np.unique(Lj[owner[hit]])
        g.clear_levels(levels)
        g.mask[K] = False
        return S

    active = np.ones(n, dtype=bool)
    active[root] = False
    tops = [nd(K) for K in g.components(np.flatnonzero(active))]
    if root.size:
        emit(root, tops)

    nf = len(fronts_piv)
    parent = np.full(nf, -1, dtype=np.int32)
    for f, ch in enumerate(fronts_children):
        for c in ch:
            parent[c] = f
    perm = np.concatenate(fronts_piv).astype(np.int32) if nf else np.empty(0, np.int32)
    front_ptr = np.zeros(nf + 1, dtype=np.int32)
    front_ptr[1:] = np.cumsum([p.size for p in fronts_piv])
    newidx = np.empty(n, dtype=np.int64)
    newidx[perm] = np.arange(n)

    # front rows (step 6)
    cb = [None] * nf                 # non-pivot rows of each front, as new indices
    rows_list = []
    for f in range(nf):
        lo, hi = int(front_ptr[f]), int(front_ptr[f + 1])
        piv = perm[lo:hi].astype(np.int64)
        parts = [newidx[g.neighbours(piv)]]
        for c in fronts_children[f]:
            parts.append(cb[c])
            cb[c] = None
        cand = np.unique(np.concatenate(parts)) if parts else np.empty(0, np.int64)
        cand = cand[cand >= hi]
        cb[f] = cand
        rows_list.append(np.concatenate([piv, perm[cand].astype(np.int64)]))
    rows_ptr = np.zeros(nf + 1, dtype=np.int64)
    rows_ptr[1:] = np.cumsum([r.size for r in rows_list])
    rows = np.concatenate(rows_list).astype(np.int32) if nf else np.empty(0, np.int32)

    etree = liu_etree(n, ptr, adj, perm, newidx)
    return Symbolic(n=n, leaf_max=leaf_max, perm=perm, front_ptr=front_ptr, front_parent=parent,
                    rows_ptr=rows_ptr, rows=rows, var_etree=etree)


def _deg_within(g, vs):
    s = g.ptr[vs]
    ln = g.ptr[vs + 1] - s
    nb = g.neighbours(vs)
    owner = np.repeat(np.arange(vs.size), ln)
    return np.bincount(owner[g.mask[nb]], minlength=vs.size)


def liu_etree(n, ptr, adj, perm, newidx):
    """Liu's elimination tree of the symmetrically permuted A + A^T (step 7):
    parent[j] = min{ i > j : L_ij != 0 }, computed with path compression."""
    parent = [-1] * n
    anc = [-1] * n
    ptr_l = ptr.tolist()
    adj_l = adj.tolist()
    perm_l = perm.tolist()
    new_l = newidx.tolist()
    for j in range(n):
        v = perm_l[j]
        for t in range(ptr_l[v], ptr_l[v + 1]):
            r = new_l[adj_l[t]]
            if r >= j:
                continue
            while True:
                a = anc[r]
                if a == j:
                    break
                anc[r] = j
                if a == -1:
                    parent[r] = j
                    break
                r = a
    return np.asarray(parent, dtype=np.int32)
