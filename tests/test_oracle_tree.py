"""Pins of the oracle's keys, ordering, canonical oct-tree and node moments
(Sect. 2.2: hierarchical cubes, each node split into eight half-size
children, leaves holding up to leaf_size particles).

The tree is checked against an independent enumeration of the key prefixes
at every level, against exact rational containment of each particle in its
cell, and the moments against closed forms."""
from fractions import Fraction

import numpy as np
import pytest

from paper_0912_1786_amd import inputs


def _decode(key):
    ix = iy = iz = 0
    for b in range(21):
        ix |= ((key >> (3 * b + 2)) & 1) << b
        iy |= ((key >> (3 * b + 1)) & 1) << b
        iz |= ((key >> (3 * b)) & 1) << b
    return ix, iy, iz


@pytest.mark.parametrize("seed", [1, 2])
def test_keys_are_cells_of_the_root_cube(orc, seed):
    ic = inputs.evrard(3000, seed=seed)
    t = orc.tree(ic, leaf_size=8)
    x0, e = t["x0"], t["e"]
    pos = np.stack([ic["x"], ic["y"], ic["z"]], 1)
    # x0 is the component-wise minimum; the side is the smallest power of two
    # not below the largest extent
    assert np.array_equal(x0, pos.min(0))
    ext = (pos.max(0) - pos.min(0)).max()
    assert 2.0 ** (e - 1) < ext <= 2.0 ** e
    side = Fraction(2) ** (e - 21)
    for p in range(0, ic["n"], 7):
        i = int(t["perm"][p])
        cell = _decode(int(t["keys"][p]))
        for d in range(3):
            lo = Fraction(float(x0[d])) + cell[d] * side
            v = Fraction(float(pos[i, d]))
            # cell containment up to the one rounding of (x - x0)
            assert lo - side * Fraction(1, 2 ** 20) <= v < lo + side * (1 + Fraction(1, 2 ** 20)) or cell[d] == 2 ** 21 - 1


def test_stable_key_order(orc):
    ic = inputs.cubic_lattice(6)  # many coincident-cell ties at coarse keys
    ic["x"] = np.round(ic["x"])  # force exact key ties
    t = orc.tree(ic, leaf_size=4)
    k, p = t["keys"], t["perm"]
    assert np.all(k[1:] >= k[:-1])
    tie = k[1:] == k[:-1]
    assert np.all(p[1:][tie] > p[:-1][tie])
    assert np.array_equal(np.sort(p), np.arange(ic["n"]))


def _enumerate_nodes(keys, leaf):
    """Canonical node set by brute force: every (level, prefix) with a
    non-empty count all of whose ancestors are split."""
    keys = [int(k) for k in keys]
    nodes = {(0, 0): (0, len(keys))}
    frontier = [(0, 0)]
    while frontier:
        nxt = []
        for (L, pre) in frontier:
            f, c = nodes[(L, pre)]
            if c <= leaf or L >= 21:
                continue
            sh = 3 * (21 - L - 1)
            groups = {}
            for q in range(f, f + c):
                groups.setdefault(keys[q] >> sh, []).append(q)
            for cp, qs in groups.items():
                nodes[(L + 1, cp)] = (qs[0], len(qs))
                nxt.append((L + 1, cp))
        frontier = nxt
    return nodes


@pytest.mark.parametrize("leaf", [1, 4, 16])
def test_topology_matches_prefix_enumeration(orc, leaf):
    ic = inputs.two_species_field(n_dm=1500, n_gas=1500, n_halo=6, seed=3)
    t = orc.tree(ic, leaf_size=leaf)
    ref = _enumerate_nodes(t["keys"], leaf)
    got = {(int(L), int(p)): (int(f), int(c)) for L, p, f, c in
           zip(t["level"], t["prefix"], t["first"], t["count"])}
    assert got == ref
    # level order: sorted by (level, prefix) == by (level, first)
    order = list(zip(t["level"], t["prefix"]))
    assert order == sorted(order)
    # children contiguous and partition the parent's range
    for k in range(len(t["level"])):
        if t["nchild"][k] == 0:
            assert t["count"][k] <= leaf or t["level"][k] == 21
            continue
        c0, nc = t["child"][k], t["nchild"][k]
        f = t["first"][k]
        for a in range(nc):
            assert t["parent"][c0 + a] == k
            assert t["first"][c0 + a] == f
            f += t["count"][c0 + a]
        assert f == t["first"][k] + t["count"][k]


def test_groups_partition_particles(orc):
    ic = inputs.evrard(5000, seed=4)
    G = 32
    t = orc.tree(ic, leaf_size=8, group_size=G)
    g = t["groups"]
    firsts = t["first"][g]
    assert np.all(np.diff(firsts) > 0)
    assert firsts[0] == 0
    assert np.array_equal(firsts[1:], firsts[:-1] + t["count"][g][:-1])
    assert firsts[-1] + t["count"][g][-1] == ic["n"]
    for k in g:
        assert t["count"][k] <= G or t["nchild"][k] == 0
        par = t["parent"][k]
        assert par < 0 or t["count"][par] > G


def test_moments_closed_forms(orc):
    # two masses on the x axis at +-d: Q_xx = 4 m d^2, Q_yy = Q_zz = -2 m d^2
    d, m = 0.25, 0.5
    t = orc.tree((np.array([-d, d]), np.zeros(2), np.zeros(2)), leaf_size=4, m=np.array([m, m]))
    assert t["mass"][0] == pytest.approx(1.0)
    assert np.allclose(t["com"][0], 0.0)
    assert np.allclose(t["quad"][0], [4 * m * d * d, -2 * m * d * d, -2 * m * d * d, 0, 0, 0])
    # eight equal masses at the corners of a cube: all quadrupole components vanish
    c = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], float)
    t = orc.tree((c[:, 0], c[:, 1], c[:, 2]), leaf_size=8, m=np.ones(8))
    assert np.allclose(t["quad"][0], 0.0, atol=1e-14)
    # traceless everywhere, delta = |com - centre|
    ic = inputs.evrard(2000, seed=5)
    t = orc.tree(ic, leaf_size=8)
    q = t["quad"]
    assert np.allclose(q[:, 0] + q[:, 1] + q[:, 2], 0.0, atol=1e-13)
    assert np.allclose(t["delta"], np.linalg.norm(t["com"] - t["centre"], axis=1), atol=1e-15)
    # node mass is the sum of its children
    for k in range(len(t["mass"])):
        if t["nchild"][k]:
            c0 = t["child"][k]
            assert t["mass"][k] == pytest.approx(t["mass"][c0:c0 + t["nchild"][k]].sum(), rel=1e-14)


@pytest.mark.parametrize("leaf,group,case", [(16, 64, "evrard"), (8, 32, "evrard"), (1, 8, "field"), (4, 16, "field")])
def test_walk_batches_are_the_greedy_sibling_packing(orc, leaf, group, case):
    """The walk batches (a reading of the grouped walk: runs of consecutive
    sibling groups packed greedily to at most 64 sinks) checked by their
    defining properties, not by re-running the packing:
    the batches cut the group list into consecutive runs; the groups of a
    run are consecutive children of one parent; a run of several groups
    holds at most 64 particles; and every cut is forced -- the next group
    is not the following sibling of the run's last group, or adding it
    would exceed 64.  These properties fix the greedy packing uniquely."""
    if case == "evrard":
        ic = inputs.evrard(5000, seed=21)
    else:
        ic = inputs.two_species_field(n_dm=2500, n_gas=2500, n_halo=6, seed=22)
    t = orc.tree(ic, leaf_size=leaf, group_size=group, batch_size=64, batch_mode=0)
    groups, batches = t["groups"], t["batches"]
    count, parent = t["count"], t["parent"]
    # groups: maximal nodes of <= group particles (or leaves), tiling the particles in order
    first = t["first"][groups]
    assert first[0] == 0 and np.array_equal(first[1:], first[:-1] + count[groups][:-1])
    assert first[-1] + count[groups][-1] == ic["n"]
    for k in groups:
        assert count[k] <= group or t["nchild"][k] == 0
        assert parent[k] < 0 or count[parent[k]] > group
    # batches partition the group list into consecutive runs
    assert batches[0, 0] == 0 and batches[-1, 1] == len(groups)
    assert np.array_equal(batches[1:, 0], batches[:-1, 1])
    assert np.all(batches[:, 1] > batches[:, 0])

    def sibling_next(a, b):
        return b == a + 1 and parent[a] == parent[b] and parent[a] >= 0

    for b0, b1 in batches:
        ks = groups[b0:b1]
        fill = int(count[ks].sum())
        if b1 - b0 > 1:
            assert fill <= 64
        for a, b in zip(ks[:-1], ks[1:]):
            assert sibling_next(a, b)
        if b1 < len(groups):
            nxt = groups[b1]
            assert not sibling_next(ks[-1], nxt) or fill + count[nxt] > 64
