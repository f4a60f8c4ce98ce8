"""Brute-force checkers for tiny clouds (numpy / plain Python).

These are written independently of the oracle's C code and follow different
formulations, so that a mistake in the oracle shows up as a disagreement:

* ``quantize`` / ``morton``  -- vectorised numpy bit manipulation (the oracle
  uses a scalar per-bit loop);
* ``paper_merge_tree``       -- the paper's own bottom-up procedure (counting
  grid at the deepest level, 2x2x2 merging with an "unmergeable" flag,
  Sec. 4.1.2-4.1.3), while the oracle uses the equivalent top-down rule;
* ``recursive_voxels``       -- a dict-based recursion over the tree
  (Sec. 4.2.3), while the oracle uses dense 128^3 grids level by level;
* ``closed_form_*``          -- results that do not need the recursion at all
  (occupied cells, means of points, arg-min/arg-max picks);
* ``recursive_weighted``     -- the neighbourhood-weighted average (Sec. 4.2.4)
  gathered per occupied cell from every sample of the node (the oracle
  scatters every sample onto its 2x2x2 cells), plus a real-arithmetic
  variant with float64 weights.
"""
from __future__ import annotations

from collections import Counter, defaultdict

import math

import numpy as np

KEY_LEVELS = 21
M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 output function (Steele, Lea, Flood 2014) of one counter."""
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def pick_hash(pid: int, seed: int) -> int:
    return splitmix64(((seed & 0xFFFFFFFF) << 32) | (pid & 0xFFFFFFFF)) >> 32


def cube(pts):
    xyz = np.stack([pts["x"], pts["y"], pts["z"]], axis=1).astype(np.float32)
    lo = xyz.min(axis=0)
    hi = xyz.max(axis=0)
    side = float(np.max(hi.astype(np.float64) - lo.astype(np.float64)))
    if side == 0.0:
        side = 1.0
    return lo, hi, side, 2097152.0 / side


def quantize(pts):
    """(n, 3) uint32 grid coordinates at 2^21 cells per axis."""
    lo, _, _, scale = cube(pts)
    xyz = np.stack([pts["x"], pts["y"], pts["z"]], axis=1).astype(np.float64)
    v = (xyz - lo.astype(np.float64)) * scale
    return np.minimum(np.floor(v), 2097151.0).astype(np.uint32)


def quantize_in_cube(pts, lo, side):
    """(n, 3) uint32 grid coordinates in a given cube (minimum corner lo, edge
    side): the same IEEE double definition evaluated by numpy, vectorised."""
    xyz = np.stack([pts["x"], pts["y"], pts["z"]], axis=1).astype(np.float64)
    v = (xyz - np.asarray(lo, np.float32).astype(np.float64)) * (2097152.0 / float(side))
    return np.clip(np.floor(v), 0.0, 2097151.0).astype(np.uint32)


def morton(q):
    """Interleave (n, 3) coordinates of 21 bits: bit i of x/y/z -> bit 3i/3i+1/3i+2."""
    q = q.astype(np.uint64)
    key = np.zeros(q.shape[0], np.uint64)
    for axis in range(3):
        v = q[:, axis]
        for i in range(KEY_LEVELS):
            key |= ((v >> np.uint64(i)) & np.uint64(1)) << np.uint64(3 * i + axis)
    return key


def demorton(key):
    key = np.asarray(key, np.uint64)
    q = np.zeros((key.shape[0], 3), np.uint64)
    for axis in range(3):
        for i in range(KEY_LEVELS):
            q[:, axis] |= ((key >> np.uint64(3 * i + axis)) & np.uint64(1)) << np.uint64(i)
    return q.astype(np.uint32)


def prefix(keys, level):
    return (np.asarray(keys, np.uint64) >> np.uint64(3 * (KEY_LEVELS - level))).astype(np.uint64)


def paper_merge_tree(keys, leaf_cap, max_level):
    """The paper's counting -> merging -> target-pointer procedure, literally.

    Counting grid at level ``max_level``; going up, a 2x2x2 group merges into
    its parent when its total is at most T and none of its cells is flagged
    unmergeable; otherwise the parent is flagged unmergeable.  Non-zero cells
    are leaves, unmergeable cells are inner nodes.  Returns a set of
    (level, key, is_leaf, npoints)."""
    keys = [int(k) for k in keys]
    if not keys:
        return set()
    grid = {max_level: Counter(k >> (3 * (KEY_LEVELS - max_level)) for k in keys)}
    unm = {max_level: set()}
    for L in range(max_level, 0, -1):
        groups = defaultdict(list)
        for c in grid[L]:
            groups[c >> 3].append(c)
        for c in unm[L]:
            groups[c >> 3].append(c)
        up, up_unm = {}, set()
        for parent, members in groups.items():
            members = set(members)
            total = sum(grid[L].get(c, 0) for c in members)
            if total <= leaf_cap and not (members & unm[L]):
                up[parent] = total
                for c in members:
                    grid[L][c] = 0
            else:
                up_unm.add(parent)
        grid[L - 1] = Counter(up)
        unm[L - 1] = up_unm
    counts = {}
    for L in range(0, max_level + 1):
        pc = Counter(k >> (3 * (KEY_LEVELS - L)) for k in keys)
        counts[L] = pc
    nodes = set()
    for L in range(0, max_level + 1):
        for c, v in grid[L].items():
            if v > 0:
                nodes.add((L, c, True, v))
        for c in unm[L]:
            nodes.add((L, c, False, counts[L][c]))
    return nodes


def tree_nodes(tree):
    return {(int(l), int(k), bool(f), int(n)) for l, k, f, n in
            zip(tree["level"], tree["key"], tree["is_leaf"], tree["npoints"])}


def _point_cell(q, node_level):
    """Cell (x, y, z) of the node's 128^3 grid for points with coords q."""
    sh = KEY_LEVELS - (node_level + 7)
    return ((q >> np.uint32(sh)) & np.uint32(127)).astype(np.int64)


def subtree_members(keys, level, key):
    return np.nonzero(prefix(keys, level) == np.uint64(key))[0]


def closed_form_cells(q, keys, level, key):
    """Voxel positions of inner node (level, key): distinct occupied cells."""
    idx = subtree_members(keys, level, key)
    cells = _point_cell(q[idx], level)
    return {tuple(c) for c in cells.tolist()}


def closed_form_leaf_means(pts, q, keys, level, key):
    """floor(mean) of R, G, B of the points per cell of inner node (level, key).
    Equals the AVERAGE voxel whenever every child of the node is a leaf."""
    idx = subtree_members(keys, level, key)
    cells = _point_cell(q[idx], level)
    lin = (cells[:, 2] * 128 + cells[:, 1]) * 128 + cells[:, 0]
    n = np.bincount(lin, minlength=128 ** 3)
    out = {}
    sums = [np.bincount(lin, weights=pts[ch][idx].astype(np.float64), minlength=128 ** 3) for ch in "rgb"]
    for c in np.nonzero(n)[0]:
        out[(int(c % 128), int((c // 128) % 128), int(c // 16384))] = tuple(
            int(s[c]) // int(n[c]) for s in sums)
    return out


def closed_form_pick(pts, q, keys, level, key, sampling, seed):
    """Pick of every cell of inner node (level, key): the sample with min id
    (FIRST) or max (hash << 32 | id) (RANDOM) over ALL points under the node
    in that cell, because min and max are associative."""
    idx = subtree_members(keys, level, key)
    cells = _point_cell(q[idx], level)
    best = {}
    for i, c in zip(idx.tolist(), map(tuple, cells.tolist())):
        k = i if sampling == 1 else ((pick_hash(i, seed) << 32) | i)
        if c not in best or (k < best[c][0] if sampling == 1 else k > best[c][0]):
            best[c] = (k, i)
    return {c: v[1] for c, v in best.items()}


def recursive_voxels(pts, q, keys, nodes, leaf_cap, max_level, sampling=0, seed=0):
    """Voxel dict per inner node by plain recursion over the node set."""
    by = {(l, k): (leaf, n) for (l, k, leaf, n) in nodes}
    memo = {}

    def children(l, k):
        return [(l + 1, (k << 3) | o) for o in range(8) if (l + 1, (k << 3) | o) in by]

    def vox(l, k):
        if (l, k) in memo:
            return memo[(l, k)]
        samples = defaultdict(list)
        for (cl, ck) in children(l, k):
            o = ck & 7
            off = ((o & 1) * 64, ((o >> 1) & 1) * 64, ((o >> 2) & 1) * 64)
            if by[(cl, ck)][0]:
                for i in subtree_members(keys, cl, ck).tolist():
                    c = tuple(_point_cell(q[i:i + 1], l)[0].tolist())
                    samples[c].append((int(pts["r"][i]), int(pts["g"][i]), int(pts["b"][i]), int(pts["a"][i]), i))
            else:
                for (x, y, z), s in vox(cl, ck).items():
                    samples[(off[0] + x // 2, off[1] + y // 2, off[2] + z // 2)].append(s)
        out = {}
        for c, ss in samples.items():
            if sampling == 0:
                n = len(ss)
                out[c] = (sum(s[0] for s in ss) // n, sum(s[1] for s in ss) // n, sum(s[2] for s in ss) // n, 255, 0)
            elif sampling == 1:
                out[c] = min(ss, key=lambda s: s[4])
            else:
                out[c] = max(ss, key=lambda s: (pick_hash(s[4], seed) << 32) | s[4])
        memo[(l, k)] = out
        return out

    return {(l, k): vox(l, k) for (l, k, leaf, n) in nodes if not leaf}


def tree_voxels(tree, node):
    """Voxel dict {(x, y, z): (r, g, b, a, id)} of node index `node`."""
    off, cnt = int(tree["offset"][node]), int(tree["count"][node])
    v = tree["voxels"][off:off + cnt]
    ids = tree["voxel_ids"][off:off + cnt] if tree.get("voxel_ids") is not None else np.zeros(cnt, np.uint32)
    return {(int(a[0]), int(a[1]), int(a[2])): (int(a[4]), int(a[5]), int(a[6]), int(a[7]), int(i))
            for a, i in zip(v, ids)}


def _node_xyz(level, key):
    return tuple(int(v) for v in demorton(np.array([key], np.uint64) << np.uint64(3 * (KEY_LEVELS - level)))[0] >>
                 np.uint32(KEY_LEVELS - level))


def recursive_weighted(pts, q, keys, nodes, real=False, child_voxels=None):
    """Weighted-average voxels {(x, y, z): (r, g, b, 255)} per inner node.

    Sample positions are in units of half a cell of the 2^21 grid: a point at
    2q + 1, a child voxel at the centre of its cell.  For every occupied cell
    (one that contains a sample) the colour gathers w * colour over ALL samples
    of the node, w = 1 - distance (cells of the node's grid), clamped at 0;
    fixed point w = 65536 - floor(65536 d) via math.isqrt, or plain float64
    (real=True).  child_voxels, if given, maps (level, key) to the voxel dict
    used as the samples of an inner child (instead of the recursion)."""
    by = {(l, k): leaf for (l, k, leaf, n) in nodes}
    memo = {}

    def samples_of(l, k):
        out = []
        for o in range(8):
            ck = (k << 3) | o
            if (l + 1, ck) not in by:
                continue
            if by[(l + 1, ck)]:
                for i in subtree_members(keys, l + 1, ck).tolist():
                    pos = tuple(2 * int(q[i][a]) + 1 for a in range(3))
                    out.append((pos, (int(pts["r"][i]), int(pts["g"][i]), int(pts["b"][i]))))
            else:
                cxyz = _node_xyz(l + 1, ck)
                src = child_voxels[(l + 1, ck)] if child_voxels is not None else vox(l + 1, ck)
                for (x, y, z), col in src.items():
                    pos = tuple((2 * ((cxyz[a] << 7) + (x, y, z)[a]) + 1) << (13 - l) for a in range(3))
                    out.append((pos, col[:3]))
        return out

    def vox(l, k):
        if (l, k) in memo:
            return memo[(l, k)]
        cs = 15 - l
        nxyz = _node_xyz(l, k)
        ss = samples_of(l, k)
        occupied = {tuple((s[0][a] >> cs) - (nxyz[a] << 7) for a in range(3)) for s in ss}
        out = {}
        for c in occupied:
            centre = [(2 * ((nxyz[a] << 7) + c[a]) + 1) << (cs - 1) for a in range(3)]
            acc = [0, 0, 0, 0] if not real else [0.0, 0.0, 0.0, 0.0]
            for pos, col in ss:
                d2 = sum((pos[a] - centre[a]) ** 2 for a in range(3))
                if real:
                    w = max(0.0, 1.0 - math.sqrt(d2) / (1 << cs))
                else:
                    r = math.isqrt(d2 << (2 * l + 2))
                    w = 65536 - r if r < 65536 else 0
                for a in range(3):
                    acc[a] += w * col[a]
                acc[3] += w
            if real:
                out[c] = tuple(int(math.floor(acc[a] / acc[3])) for a in range(3)) + (255,)
            else:
                out[c] = tuple(acc[a] // acc[3] for a in range(3)) + (255,)
        memo[(l, k)] = out
        return out

    return {(l, k): vox(l, k) for (l, k, leaf, n) in nodes if not leaf}
