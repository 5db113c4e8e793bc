"""Naive kD-tree builder of the FP64 oracle (test infrastructure only).

Follows the construction of Section 4.1 ("kD-tree construction") step by step, with
brute-force counting instead of any sweep data structure:

* The root region is the bounding box B of the root-level subgrids.
* A region is split by the axis-aligned plane that cuts the fewest subgrid boxes of the
  level being inserted, keeping at least one slab of cells on each side; among equal
  counts the plane whose two sides hold the most balanced number of cells wins.
  Recursion stops once the region holds cells of a single subgrid.
* Levels are inserted one after another: every current leaf that overlaps subgrids of
  the next level is refined with the same rule applied to (subgrid box ∩ leaf).

Readings of points the paper leaves open (each also listed in the design notes):

* candidate planes are the faces of the clipped boxes strictly inside the region;
* "cuts a box" means the plane lies strictly inside the box on that axis;
* "cells on each side" counts the region's cells, so the balance measure is
  min(c-lo, hi-c) / max(c-lo, hi-c) on the split axis (the cross-section cancels);
* remaining ties: lowest axis (x < y < z), then lowest plane position;
* children inherit the patch and level of the region they were cut from; regions of B
  covered by no root subgrid are leaves with patch -1 (transparent);
* node kinds: (b) leaf; (a) internal node lying inside a single subgrid all of whose cells
  are refined further; (c) any other internal node.

All coordinates are integers in units of finest-level cells, so the result is exact.
The oracle shares no code with the HIP library; this module imports only numpy.
"""
from __future__ import annotations

import sys
from typing import List, Optional

import numpy as np

KIND_A, KIND_B, KIND_C = 0, 1, 2


class Node:
    __slots__ = ("lo", "hi", "patch", "level", "axis", "split", "low", "high", "cover")

    def __init__(self, lo, hi, patch, level):
        self.lo = np.array(lo, dtype=np.int64)
        self.hi = np.array(hi, dtype=np.int64)
        self.patch = int(patch)     # leaf: patch id (-1 = no data); internal: patch held before split
        self.level = int(level)     # leaf: its patch level; internal: level of the split
        self.axis = -1
        self.split = 0
        self.low: Optional[Node] = None
        self.high: Optional[Node] = None
        self.cover = -1

    @property
    def is_leaf(self):
        return self.low is None


def _clip(boxes: np.ndarray, lo, hi) -> np.ndarray:
    """boxes: int64[k, 7] (id, lo3, hi3). Returns boxes clipped to [lo, hi) with positive volume."""
    if len(boxes) == 0:
        return boxes
    b = boxes.copy()
    b[:, 1:4] = np.maximum(b[:, 1:4], lo)
    b[:, 4:7] = np.minimum(b[:, 4:7], hi)
    keep = np.all(b[:, 4:7] > b[:, 1:4], axis=1)
    return b[keep]


def _choose_split(lo, hi, S):
    """Return (axis, c) minimising (cost, -balance, axis, c) by brute force."""
    best = None
    for a in range(3):
        faces = np.unique(np.concatenate([S[:, 1 + a], S[:, 4 + a]]))
        faces = faces[(faces > lo[a]) & (faces < hi[a])]
        for c in faces:
            c = int(c)
            cost = int(np.sum((S[:, 1 + a] < c) & (S[:, 4 + a] > c)))
            left, right = c - int(lo[a]), int(hi[a]) - c
            mn, mx = min(left, right), max(left, right)
            if best is None:
                best = (cost, mn, mx, a, c)
                continue
            bc, bmn, bmx, ba, bcc = best
            if cost != bc:
                better = cost < bc
            elif mn * bmx != bmn * mx:
                better = mn * bmx > bmn * mx          # larger min/max ratio is more balanced
            else:
                better = (a, c) < (ba, bcc)
            if better:
                best = (cost, mn, mx, a, c)
    if best is None:
        raise ValueError("no admissible split plane (overlapping same-level subgrids?)")
    return best[3], best[4]


def _split(node: Node, level: int, S: np.ndarray):
    if len(S) == 0:
        return
    if len(S) == 1 and np.array_equal(S[0, 1:4], node.lo) and np.array_equal(S[0, 4:7], node.hi):
        node.patch = int(S[0, 0])
        node.level = level
        return
    a, c = _choose_split(node.lo, node.hi, S)
    node.cover = node.patch
    node.axis, node.split = a, c
    lhi = node.hi.copy(); lhi[a] = c
    hlo = node.lo.copy(); hlo[a] = c
    node.low = Node(node.lo, lhi, node.patch, node.level)
    node.high = Node(hlo, node.hi, node.patch, node.level)
    node.level = level
    node.patch = -1
    _split(node.low, level, _clip(S, node.low.lo, node.low.hi))
    _split(node.high, level, _clip(S, node.high.lo, node.high.hi))


def _leaves(node: Node, out: List[Node]):
    stack = [node]
    while stack:
        n = stack.pop()
        if n.is_leaf:
            out.append(n)
        else:
            stack.append(n.high)
            stack.append(n.low)
    return out


class Tree:
    """Result of the naive build. Nodes and leaves are listed in depth-first pre-order,
    low child first; a leaf's id is its rank among the leaves in that order."""

    def __init__(self, root: Node, boxes: np.ndarray, nlevels: int):
        self.root = root
        self.nodes: List[Node] = []
        stack = [root]
        while stack:
            n = stack.pop()
            self.nodes.append(n)
            if not n.is_leaf:
                stack.append(n.high)
                stack.append(n.low)
        self.leaves = [n for n in self.nodes if n.is_leaf]
        self.boxes = boxes
        self.nlevels = nlevels

    def kinds(self) -> np.ndarray:
        """Node kind per node (pre-order): (b) leaf, (a) fully refined inside one subgrid, (c) other."""
        box_level = {int(b[0]): int(b[7]) for b in self.boxes}
        min_leaf_level = {}
        for n in reversed(self.nodes):            # children precede parents in reversed pre-order
            if n.is_leaf:
                min_leaf_level[id(n)] = n.level
            else:
                min_leaf_level[id(n)] = min(min_leaf_level[id(n.low)], min_leaf_level[id(n.high)])
        kinds = np.zeros(len(self.nodes), dtype=np.int32)
        for i, n in enumerate(self.nodes):
            if n.is_leaf:
                kinds[i] = KIND_B
            elif n.cover >= 0 and min_leaf_level[id(n)] > box_level[n.cover]:
                kinds[i] = KIND_A
            else:
                kinds[i] = KIND_C
        return kinds

    def node_array(self) -> np.ndarray:
        """int64[nnodes, 5]: axis (-1 leaf), split, level, patch (leaves, else -1), cover."""
        out = np.zeros((len(self.nodes), 5), dtype=np.int64)
        for i, n in enumerate(self.nodes):
            out[i] = (n.axis, n.split if not n.is_leaf else 0, n.level,
                      n.patch if n.is_leaf else -1, n.cover if not n.is_leaf else -1)
        return out

    def leaf_array(self) -> np.ndarray:
        """int64[nleaves, 8]: lo[3], hi[3], patch, level (finest-cell units)."""
        out = np.zeros((len(self.leaves), 8), dtype=np.int64)
        for i, n in enumerate(self.leaves):
            out[i, 0:3] = n.lo
            out[i, 3:6] = n.hi
            out[i, 6] = n.patch
            out[i, 7] = n.level
        return out


def build(boxes_finest: np.ndarray, nlevels: int) -> Tree:
    """boxes_finest: int64[np, 7] = level, lo[3], hi[3] in finest-level cells (patch order = ids)."""
    sys.setrecursionlimit(max(10000, sys.getrecursionlimit()))
    nb = len(boxes_finest)
    boxes = np.zeros((nb, 8), dtype=np.int64)
    boxes[:, 0] = np.arange(nb)
    boxes[:, 1:7] = boxes_finest[:, 1:7]
    boxes[:, 7] = boxes_finest[:, 0]
    lev0 = boxes[boxes[:, 7] == 0]
    if len(lev0) == 0:
        raise ValueError("no root-level subgrid")
    lo = lev0[:, 1:4].min(axis=0)
    hi = lev0[:, 4:7].max(axis=0)
    root = Node(lo, hi, -1, 0)
    _split(root, 0, _clip(lev0[:, :7], lo, hi))
    for lev in range(1, nlevels):
        bl = boxes[boxes[:, 7] == lev][:, :7]
        if len(bl) == 0:
            continue
        for leaf in _leaves(root, []):
            S = _clip(bl, leaf.lo, leaf.hi)
            if len(S):
                _split(leaf, lev, S)
    return Tree(root, boxes, nlevels)
