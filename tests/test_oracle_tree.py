"""Pins for the oracle's octree and lists (Sec. 3.2 neighbourhood, Sec. 3.3.2
interaction list, Sec. 4.2 count of 316 distinct offsets).  CPU only."""
import itertools

import numpy as np
import pytest


def _decode(key, bits):
    n = [0, 0, 0]
    for b in range(bits):
        for a in range(3):
            n[a] |= ((key >> (3 * b + a)) & 1) << b
    return n


def test_tree_geometry(oracle_lib):
    """Every point lies in the closed box of its leaf; sorting is by (key, index)."""
    r = np.random.default_rng(5)
    x = r.random((3, 3000))
    x[:, :5] = 1.0  # upper face clamps into the last cell
    x[:, 5:8] = 0.0
    depth = 4
    keys, perm, ls = oracle_lib.tree(x, [0, 0, 0], 1.0, depth)
    h = 1.0 / (1 << depth)
    for i in range(x.shape[1]):
        n = _decode(int(keys[i]), depth)
        for a in range(3):
            assert n[a] * h <= x[a, i] <= (n[a] + 1) * h
    assert sorted(perm.tolist()) == list(range(x.shape[1]))
    sk = keys[perm]
    assert np.all(np.diff(sk.astype(np.int64)) >= 0)
    same = np.diff(sk.astype(np.int64)) == 0
    assert np.all(np.diff(perm)[same] > 0)  # stable within a leaf
    counts = np.bincount(keys, minlength=1 << (3 * depth))
    np.testing.assert_array_equal(np.diff(ls), counts)
    assert ls[0] == 0 and ls[-1] == x.shape[1]


def test_tree_domain_errors(oracle_lib):
    x = np.full((3, 4), 0.5)
    x[1, 2] = 1.0 + 1e-12
    with pytest.raises(oracle_lib.OracleError) as e:
        oracle_lib.tree(x, [0, 0, 0], 1.0, 3)
    assert e.value.code == oracle_lib.EDOMAIN
    x[1, 2] = np.nan
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.tree(x, [0, 0, 0], 1.0, 3)


def _brute_lists(active, level):
    """O(B^2) lists from the geometric definitions: two boxes of half-width l
    are well separated iff min |x - y| >= 2l over the boxes, i.e. their index
    distance exceeds 1 along some axis; the interaction list keeps the
    well-separated children of the parent's neighbours."""
    out = {}
    for ki in active:
        ni = _decode(int(ki), level)
        near, il = [], []
        for kj in active:
            nj = _decode(int(kj), level)
            # box gap along each axis in units of the box side
            gap = max(max(abs(ni[a] - nj[a]) - 1, 0) for a in range(3))
            if gap == 0:
                near.append(int(kj))
            else:
                pi, pj = [c >> 1 for c in ni], [c >> 1 for c in nj]
                pgap = max(max(abs(pi[a] - pj[a]) - 1, 0) for a in range(3))
                if pgap == 0:
                    il.append((int(kj), tuple(nj[a] - ni[a] for a in range(3))))
        out[int(ki)] = (sorted(near), sorted(il))
    return out


@pytest.mark.parametrize("depth,level,npts", [(3, 2, 60), (3, 3, 150), (4, 3, 400)])
def test_lists_brute_force(oracle_lib, depth, level, npts):
    r = np.random.default_rng(depth * 10 + level)
    x = r.random((3, npts)) ** 2  # uneven occupancy, many empty boxes
    _, _, ls = oracle_lib.tree(x, [0, 0, 0], 1.0, depth)
    L = oracle_lib.lists(ls, depth, level)
    offs = oracle_lib.offset_table()
    ref = _brute_lists(L["active"], level)
    assert len(ref) == len(L["active"])
    for t, k in enumerate(L["active"]):
        near = L["near_src"][L["near_ptr"][t]:L["near_ptr"][t + 1]].tolist()
        src = L["il_src"][L["il_ptr"][t]:L["il_ptr"][t + 1]].tolist()
        oid = L["il_off"][L["il_ptr"][t]:L["il_ptr"][t + 1]].tolist()
        rn, ri = ref[int(k)]
        assert near == rn
        assert src == [a for a, _ in ri]
        assert [tuple(offs[o]) for o in oid] == [b for _, b in ri]


def test_offset_table(oracle_lib):
    """7^3 - 3^3 = 316 distinct interaction offsets (Sec. 4.2), ascending code."""
    t = oracle_lib.offset_table()
    assert t.shape == (316, 3)
    assert len({tuple(r) for r in t}) == 316
    assert np.all(np.abs(t).max(1) >= 2) and np.all(np.abs(t) <= 3)
    code = (t[:, 0] + 3) + 7 * (t[:, 1] + 3) + 49 * (t[:, 2] + 3)
    assert np.all(np.diff(code) > 0)


@pytest.mark.parametrize("level", [2, 3, 4])
def test_dense_level_counts(oracle_lib, level):
    """All boxes occupied: near pairs = (3 2^k - 2)^3, interaction pairs =
    (6 2^k - 8)^3 - (3 2^k - 2)^3; an interior box has 27 and 189 entries, and
    every one of the 316 offsets occurs."""
    side = 1 << level
    g = (np.arange(side) + 0.5) / side
    x = np.array(list(itertools.product(g, g, g))).T.copy()
    _, _, ls = oracle_lib.tree(x, [0, 0, 0], 1.0, level)
    L = oracle_lib.lists(ls, level, level)
    m = 1 << level
    assert len(L["near_src"]) == (3 * m - 2) ** 3
    assert len(L["il_src"]) == (6 * m - 8) ** 3 - (3 * m - 2) ** 3
    assert np.diff(L["near_ptr"]).max() == 27
    if level >= 3:  # level 2 has no box whose parent is surrounded
        assert np.diff(L["il_ptr"]).max() == 189
        assert len(set(L["il_off"].tolist())) == 316
