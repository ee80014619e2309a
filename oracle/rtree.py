"""Deterministic bisection R-tree over support points (oracle; test infrastructure only).

Paper, Section 3 (Definition of an R-tree of order (m,M)): every leaf holds between m and M entries, all
leaves sit at the same depth, and every node stores the minimum bounding rectangle (MBR) of its entries.
Section 4 (point-based agglomeration): the leaves of the R-tree are the support points themselves, so each
box owns its points uniquely.  The paper builds the tree with the Boost R*-tree (insertion heuristics that
depend on insertion order); it does not specify the construction, so this reading uses a deterministic
bulk load that satisfies the Definition:

  * depth t = smallest t >= 0 with 2^t * leaf >= n  (i.e. t = max(0, ceil(log2(n / leaf))));
  * split(S): extents e_a = max_S x_a - min_S x_a; a* = smallest axis attaining max e_a; order S
    lexicographically by (x_{a*}, x_{a*+1 mod d}, ..., original index); the left child is the first
    ceil(|S|/2) points, the right child the rest;
  * leaves are the depth-t nodes, left to right; each holds floor(n/2^t) or ceil(n/2^t) points, which is
    the occupancy window (M/2, M] of an order-(M/2, M) tree with M = leaf (Section 6 uses M = 2m);
  * every box is the MBR of all its points, constrained ones included.

Level choice (Section 6: the hierarchy is built bottom-up and does not use every R-tree level): level 0
is the fine space, level 1 sits at depth t (t - d when the leaf level is skipped), level l+1 at depth
max(depth_l - d, 0) so that each coarse box holds 2^d boxes of the level below.  The hierarchy stops at
the first level with (#boxes * B) <= max_coarse_dofs, at max_levels, or at the root.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np


@dataclasses.dataclass
class RTree:
    depth: int                  # t
    order: np.ndarray           # permutation: leaf-ordered position -> original point index
    offsets: List[np.ndarray]   # offsets[k]: (2^k + 1,) segment boundaries of the depth-k nodes in `order`

    def owner(self, k: int) -> np.ndarray:
        """Node index at depth k that owns each original point."""
        n = self.order.shape[0]
        own = np.empty(n, dtype=np.int64)
        off = self.offsets[k]
        seg = np.repeat(np.arange(len(off) - 1), np.diff(off))
        own[self.order] = seg
        return own

    def boxes(self, coords: np.ndarray, k: int):
        """(lo, hi) MBRs of the depth-k nodes, shape (2^k, d) each."""
        off = self.offsets[k]
        xs = coords[self.order]
        nb = len(off) - 1
        lo = np.empty((nb, coords.shape[1]))
        hi = np.empty((nb, coords.shape[1]))
        for b in range(nb):
            seg = xs[off[b]:off[b + 1]]
            lo[b] = seg.min(axis=0)
            hi[b] = seg.max(axis=0)
        return lo, hi


def tree_depth(n: int, leaf: int) -> int:
    """Smallest t >= 0 with 2^t * leaf >= n."""
    t = 0
    while (leaf << t) < n:
        t += 1
    return t


def _split(coords: np.ndarray, idx: np.ndarray):
    """One bisection of the point set `idx` (original indices, any order)."""
    x = coords[idx]
    d = coords.shape[1]
    ext = x.max(axis=0) - x.min(axis=0)
    astar = int(np.flatnonzero(ext == ext.max())[0])
    # np.lexsort sorts by the LAST key first
    keys = [idx]
    for m in reversed(range(d)):
        keys.append(x[:, (astar + m) % d])
    srt = idx[np.lexsort(keys)]
    nl = (len(idx) + 1) // 2
    return srt[:nl], srt[nl:]


def bisection_rtree(coords: np.ndarray, leaf: int) -> RTree:
    coords = np.asarray(coords, dtype=np.float64)
    n = coords.shape[0]
    if n < 1 or leaf < 1:
        raise ValueError("need n >= 1 and leaf >= 1")
    if not np.all(np.isfinite(coords)):
        raise ValueError("non-finite coordinates")
    t = tree_depth(n, leaf)
    segs = [np.arange(n, dtype=np.int64)]
    offsets = [np.array([0, n], dtype=np.int64)]
    for _ in range(t):
        nxt = []
        for s in segs:
            left, right = _split(coords, s)
            nxt.append(left)
            nxt.append(right)
        segs = nxt
        offsets.append(np.concatenate([[0], np.cumsum([len(s) for s in segs])]).astype(np.int64))
    order = np.concatenate(segs)
    # the parent segments are unions of consecutive children, so every depth's offsets index `order`
    return RTree(depth=t, order=order, offsets=offsets)


def select_levels(tree: RTree, d: int, B: int, *, max_levels: int = 0, max_coarse_dofs: int = 2000,
                  skip_leaf_level: bool = False) -> List[int]:
    """Depths of the agglomerated levels 1..L (level 0, the fine space, is not listed)."""
    if max_levels == 1:
        raise ValueError("a hierarchy needs at least two levels")
    depth = max(tree.depth - d, 0) if skip_leaf_level else tree.depth
    depths = [depth]
    while True:
        nlev = len(depths) + 1
        nboxes = 1 << depths[-1]
        if nboxes * B <= max_coarse_dofs:
            break
        if max_levels and nlev >= max_levels:
            break
        if depths[-1] == 0:
            break
        depths.append(max(depths[-1] - d, 0))
    return depths


@dataclasses.dataclass
class CellTree:
    """Cell-based agglomeration (Section 4): an R-tree whose leaves are the mesh cells.

    The bisection bulk load above runs on one point per cell, the centre of the cell's bounding box (a reading:
    the paper inserts the cell MBRs into Boost's R*-tree).  An agglomerate at depth k is a node of this tree; its
    box is the bounding box of all support points of its cells.  Support points shared by several agglomerates
    are assigned uniquely: the agglomerates are visited in array order and each takes the points of its cells
    not yet taken, i.e. a point belongs to the smallest node index among the nodes holding one of its cells.
    """
    depth: int
    cells: np.ndarray            # (ncells, nloc) support-point indices
    n: int                       # number of support points
    cell_tree: RTree             # the bisection tree over cell centres

    def cell_node(self, k: int) -> np.ndarray:
        """Node index at depth k of every cell."""
        return self.cell_tree.owner(k)

    def owner(self, k: int) -> np.ndarray:
        """Node at depth k that owns each support point (first-come over the nodes in array order)."""
        node = self.cell_node(k)
        own = np.full(self.n, np.iinfo(np.int64).max, dtype=np.int64)
        for j in range(self.cells.shape[1]):
            np.minimum.at(own, self.cells[:, j], node)
        if np.any(own == np.iinfo(np.int64).max):
            raise ValueError("support point in no cell")
        return own

    def boxes(self, coords: np.ndarray, k: int):
        """(lo, hi): bounding boxes of the depth-k nodes over all support points of their cells."""
        node = self.cell_node(k)
        nb = 1 << k
        d = coords.shape[1]
        lo = np.full((nb, d), np.inf)
        hi = np.full((nb, d), -np.inf)
        for j in range(self.cells.shape[1]):
            x = coords[self.cells[:, j]]
            for a in range(d):
                np.minimum.at(lo[:, a], node, x[:, a])
                np.maximum.at(hi[:, a], node, x[:, a])
        return lo, hi


def cell_rtree(coords: np.ndarray, cells: np.ndarray, leaf: int) -> CellTree:
    """Cell-based R-tree with at most `leaf` cells per leaf."""
    coords = np.asarray(coords, dtype=np.float64)
    cells = np.asarray(cells, dtype=np.int64)
    x = coords[cells]                                   # (ncells, nloc, d)
    centres = 0.5 * (x.min(axis=1) + x.max(axis=1))
    t = bisection_rtree(centres, leaf)
    return CellTree(depth=t.depth, cells=cells, n=coords.shape[0], cell_tree=t)
