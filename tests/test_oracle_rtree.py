"""Pins of the oracle's bisection R-tree and level selection (Section 3 Definition; Section 4
point-based agglomeration; Section 6 level choice)."""
import os

import numpy as np
import pytest

import oracle as O
from oracle.rtree import tree_depth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rtree_4x4.txt")


def _golden_leaves():
    leaves, boxes = [], []
    for line in open(GOLDEN):
        if line.startswith("leaf"):
            body = line.split(":", 1)[1].split()
            leaves.append([int(v) for v in body[:4]])
            boxes.append([float(v) / 3.0 for v in body[4:8]])
    return leaves, np.array(boxes)


def test_worked_example_4x4():
    ix, iy = np.meshgrid(np.arange(4), np.arange(4), indexing="xy")
    pts = np.stack([ix.ravel() / 3.0, iy.ravel() / 3.0], axis=1)       # index i = ix + 4 iy
    tree = O.bisection_rtree(pts, 4)
    leaves, boxes = _golden_leaves()
    assert tree.depth == 2
    off = tree.offsets[2]
    for k, ref in enumerate(leaves):
        assert sorted(tree.order[off[k]:off[k + 1]].tolist()) == sorted(ref)
    lo, hi = tree.boxes(pts, 2)
    np.testing.assert_array_equal(np.concatenate([lo, hi], axis=1), boxes)


def _key(x, i, a):
    d = len(x)
    return tuple(x[(a + m) % d] for m in range(d)) + (i,)


def _check_split(coords, parent, left, right):
    """Invariants of one split: sizes, axis choice, lexicographic separation (checked by brute force)."""
    assert len(left) == (len(parent) + 1) // 2 and len(left) + len(right) == len(parent)
    assert set(left) | set(right) == set(parent) and not (set(left) & set(right))
    x = coords[parent]
    ext = x.max(axis=0) - x.min(axis=0)
    a = int(np.argmax(ext))                    # argmax returns the smallest index among ties
    if len(right):
        kl = max(_key(coords[i], i, a) for i in left)
        kr = min(_key(coords[i], i, a) for i in right)
        assert kl < kr


@pytest.mark.parametrize("seed,n,d,leaf", [(0, 37, 2, 4), (1, 100, 3, 7), (2, 64, 2, 8), (3, 200, 3, 16)])
def test_split_invariants_with_ties(seed, n, d, leaf):
    g = np.random.default_rng(seed)
    # coordinates on a coarse lattice so that ties in every axis are frequent; a few duplicates
    coords = g.integers(0, 5, size=(n, d)).astype(np.float64) / 4.0
    coords[-3:] = coords[:3]
    tree = O.bisection_rtree(coords, leaf)
    assert tree.depth == tree_depth(n, leaf)
    assert (leaf << tree.depth) >= n and (tree.depth == 0 or (leaf << (tree.depth - 1)) < n)
    assert sorted(tree.order.tolist()) == list(range(n))
    for k in range(tree.depth):
        off, off2 = tree.offsets[k], tree.offsets[k + 1]
        for s in range(len(off) - 1):
            parent = tree.order[off[s]:off[s + 1]]
            left = tree.order[off2[2 * s]:off2[2 * s + 1]]
            right = tree.order[off2[2 * s + 1]:off2[2 * s + 2]]
            _check_split(coords, parent, left, right)
    sizes = np.diff(tree.offsets[tree.depth])
    t = tree.depth
    assert set(sizes.tolist()) <= {n >> t, -(-n >> t)}
    assert sizes.max() <= leaf
    # MBR nesting: every child box inside its parent box
    for k in range(1, tree.depth + 1):
        lo_c, hi_c = tree.boxes(coords, k)
        lo_p, hi_p = tree.boxes(coords, k - 1)
        par = np.arange(len(lo_c)) >> 1
        assert np.all(lo_c >= lo_p[par]) and np.all(hi_c <= hi_p[par])


def test_owner_is_a_partition():
    g = np.random.default_rng(5)
    coords = g.random((300, 3))
    tree = O.bisection_rtree(coords, 20)
    own = tree.owner(tree.depth)
    cnt = np.bincount(own, minlength=1 << tree.depth)
    np.testing.assert_array_equal(cnt, np.diff(tree.offsets[tree.depth]))


class _FakeTree:
    def __init__(self, depth):
        self.depth = depth


@pytest.mark.parametrize("n,leaf,d,B,max_levels,expect_boxes", [
    (1089, 64, 2, 4, 2, [32]),                         # 16x16 Q2 square, p'=1: 128 coarse DoFs
    (591361, 128, 2, 9, 4, [8192, 2048, 512]),         # 256^2 Q3 square, p'=2, 4 levels (4,608 dense)
    (2146689, 256, 3, 27, 0, [16384, 2048, 256, 32]),  # 64^3 Q2 cube, p'=2, down to <= 2000 (864)
])
def test_level_selection(n, leaf, d, B, max_levels, expect_boxes):
    t = tree_depth(n, leaf)
    depths = O.select_levels(_FakeTree(t), d, B, max_levels=max_levels, max_coarse_dofs=2000)
    assert [1 << k for k in depths] == expect_boxes
    if max_levels == 0:
        assert (1 << depths[-1]) * B <= 2000


def test_skip_leaf_level():
    depths = O.select_levels(_FakeTree(10), 2, 4, max_levels=0, max_coarse_dofs=2000, skip_leaf_level=True)
    assert depths[0] == 8


def test_rejects_non_finite():
    with pytest.raises(ValueError):
        O.bisection_rtree(np.array([[0.0, np.nan], [1.0, 1.0]]), 1)
