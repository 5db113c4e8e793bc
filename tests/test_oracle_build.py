"""Pins of the oracle's naive kD builder (Section 4.1) against facts that do not come from
the builder itself: partition invariants checked by brute force, and trees derived by hand
for small cases (tests/golden/kd_hand_cases.json)."""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import finest_boxes, kdbuild

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _check_partition(h, tree):
    boxes = finest_boxes(h)
    lev0 = boxes[boxes[:, 0] == 0]
    B_lo, B_hi = lev0[:, 1:4].min(0), lev0[:, 4:7].max(0)
    L = tree.leaf_array()
    lo, hi = L[:, 0:3], L[:, 3:6]
    assert np.all(hi > lo)
    # leaves tile B: volumes add up and leaves are pairwise interior-disjoint
    assert int(np.prod(hi - lo, axis=1).sum()) == int(np.prod(B_hi - B_lo))
    for i in range(len(L)):
        ov = np.all(np.minimum(hi[i], hi) > np.maximum(lo[i], lo), axis=1)
        ov[i] = False
        assert not ov.any(), "overlapping leaves"
    for i in range(len(L)):
        p, lev = int(L[i, 6]), int(L[i, 7])
        # the finest patch meeting the leaf interior must be unique and equal the leaf's patch
        meet = np.all(np.minimum(hi[i], boxes[:, 4:7]) > np.maximum(lo[i], boxes[:, 1:4]), axis=1)
        if p < 0:
            assert not meet.any(), "data under a transparent leaf"
            continue
        assert meet[p] and int(boxes[p, 0]) == lev
        assert np.all(boxes[p, 1:4] <= lo[i]) and np.all(boxes[p, 4:7] >= hi[i]), "leaf sticks out of its patch"
        finer = meet & (boxes[:, 0] > lev)
        assert not finer.any(), "a finer patch meets the leaf interior"
        # brute force over a few cell centres of the leaf: the max-level patch containing it
        rng = np.random.default_rng(i)
        for _ in range(3):
            c2 = 2 * (lo[i] + rng.integers(0, hi[i] - lo[i])) + 1
            inside = np.all((2 * boxes[:, 1:4] <= c2) & (c2 < 2 * boxes[:, 4:7]), axis=1)
            best = np.flatnonzero(inside)[np.argmax(boxes[inside, 0])]
            assert best == p


def test_partition_small_nested():
    h = workloads.tiny_samr(0)
    tree = kdbuild.build(finest_boxes(h), h.nlevels)
    _check_partition(h, tree)


@pytest.mark.parametrize("seed", range(100))
def test_partition_random_tiny(seed):
    h = workloads.random_tiny(seed, multi_root=(seed % 3 == 0))
    tree = kdbuild.build(finest_boxes(h), h.nlevels)
    _check_partition(h, tree)
    # split planes lie strictly inside their node; every internal node has two children
    for n in tree.nodes:
        if not n.is_leaf:
            assert n.lo[n.axis] < n.split < n.hi[n.axis]
            assert n.low.hi[n.axis] == n.split and n.high.lo[n.axis] == n.split


def _tree_signature(node):
    if node.is_leaf:
        return ["leaf", int(node.patch), int(node.level)]
    return ["split", "xyz"[node.axis], int(node.split), int(node.level),
            _tree_signature(node.low), _tree_signature(node.high)]


def test_hand_derived_trees():
    """Trees derived by hand from the split rule for small configurations."""
    with open(os.path.join(GOLDEN, "kd_hand_cases.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        boxes = np.array(case["boxes_finest"], dtype=np.int64)
        tree = kdbuild.build(boxes, case["nlevels"])
        assert _tree_signature(tree.root) == case["tree"], case["name"]
        kinds = tree.kinds()
        assert [("a", "b", "c")[k] for k in kinds] == case["kinds"], case["name"]


def test_shuffle_invariance():
    h = workloads.tiny_samr(1)
    t1 = kdbuild.build(finest_boxes(h), h.nlevels)
    perm = np.random.default_rng(5).permutation(len(h.patches))
    hs = workloads.Hierarchy(h.origin, h.h0, h.refine, h.nlevels, [h.patches[i] for i in perm])
    t2 = kdbuild.build(finest_boxes(hs), hs.nlevels)
    a1, a2 = t1.node_array(), t2.node_array()
    assert np.array_equal(a1[:, :3], a2[:, :3])
    leaf_p1 = a1[:, 3]
    leaf_p2 = np.where(a2[:, 3] >= 0, perm[np.maximum(a2[:, 3], 0)], -1)
    assert np.array_equal(leaf_p1, leaf_p2)
