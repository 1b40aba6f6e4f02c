"""Pins for the CPU oracle against things other than itself: hand-worked
labelings, breadth-first brute force (exhaustive on K5 / K6), scipy's
connected components, invariants, and closed forms on trees and lattices."""
import itertools
import random

import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.csgraph
from hypothesis import given, settings, strategies as st

import gen
import oracle
from conftest import read_golden


def check_invariants(labels, n, src, dst, occ):
    """Properties every correct min-index labeling has, at any size."""
    labels = np.asarray(labels)
    assert labels.shape == (n,)
    idx = np.arange(n)
    assert (labels <= idx).all()  # label[i] <= i
    assert (labels >= 0).all()
    assert (labels[labels] == labels).all()  # label is a root
    roots = labels == idx
    # label[i] == i  iff  i is the smallest site of its cluster
    first = np.full(n, n, np.int64)
    np.minimum.at(first, labels, idx)
    assert (first[labels] == labels).all()
    assert (roots == (first[labels] == idx)).all()
    if len(src):
        on = np.asarray(occ, bool) if occ is not None else np.ones(len(src), bool)
        assert (labels[src[on]] == labels[dst[on]]).all()  # occupied bonds join
    sizes = np.bincount(labels, minlength=n)
    assert sizes.sum() == n and (sizes[roots] >= 1).all() and (sizes[~roots] == 0).all()


def scipy_labels(n, src, dst, occ=None):
    """Textbook library routine, canonicalised to the minimum index."""
    on = np.ones(len(src), bool) if occ is None else np.asarray(occ, bool)
    a = scipy.sparse.coo_matrix((np.ones(on.sum()), (src[on], dst[on])), shape=(n, n))
    _, comp = scipy.sparse.csgraph.connected_components(a, directed=False)
    first = np.full(comp.max() + 1 if n else 0, n, np.int64)
    np.minimum.at(first, comp, np.arange(n))
    return first[comp].astype(np.int32)


def load_cases():
    cases, cur = [], None
    for r in read_golden("small_graphs.txt"):
        if r[0] == "case":
            cur = {"name": r[1], "n": int(r[2]), "bonds": []}
            cases.append(cur)
        elif r[0] == "b":
            cur["bonds"].append(tuple(int(x) for x in r[1:4]))
        elif r[0] == "expect":
            cur["expect"] = [int(x) for x in r[1:]]
    return cases


@pytest.mark.parametrize("case", load_cases(), ids=lambda c: c["name"])
def test_hand_worked_cases(case):
    n, b = case["n"], case["bonds"]
    src = np.array([x[0] for x in b], np.int32)
    dst = np.array([x[1] for x in b], np.int32)
    occ = np.array([x[2] for x in b], np.uint8)
    got = oracle.label_edges(n, src, dst, occ)
    assert got.tolist() == case["expect"]
    assert oracle.label_bfs(n, [(u, v) for u, v, o in b if o]) == case["expect"]
    check_invariants(got, n, src, dst, occ)


def test_empty_and_degenerate():
    e = np.zeros(0, np.int32)
    assert oracle.label_edges(0, e, e).tolist() == []
    assert oracle.label_edges(1, e, e).tolist() == [0]
    assert oracle.label_edges(5, e, e).tolist() == list(range(5))
    # every bond unoccupied: identity
    src, dst = gen.triangle_edges(8)
    np.testing.assert_array_equal(oracle.label_edges(64, src, dst, np.zeros(len(src), np.uint8)),
                                  np.arange(64))
    # all occupied on a connected lattice: one cluster labelled 0
    assert not oracle.label_edges(64, src, dst).any()
    # an id outside [0, n) is rejected
    with pytest.raises(ValueError):
        oracle.label_edges(3, np.array([0], np.int32), np.array([3], np.int32))
    with pytest.raises(ValueError):
        oracle.label_edges(3, np.array([-1], np.int32), np.array([0], np.int32))


def _all_subsets_check(k):
    pairs = list(itertools.combinations(range(k), 2))
    rng = random.Random(1234 + k)
    src_all = np.array([p[0] for p in pairs], np.int32)
    dst_all = np.array([p[1] for p in pairs], np.int32)
    for mask in range(1 << len(pairs)):
        occ = np.array([(mask >> j) & 1 for j in range(len(pairs))], np.uint8)
        perm = list(range(k))
        rng.shuffle(perm)
        perm = np.array(perm, np.int32)
        s, d = perm[src_all], perm[dst_all]
        if mask & 1:
            s, d = d, s  # orientation must not matter
        got = oracle.label_edges(k, s, d, occ)
        want = oracle.label_bfs(k, [(int(a), int(b)) for a, b, o in zip(s, d, occ) if o])
        assert got.tolist() == want, (k, mask)


def test_exhaustive_k5():
    _all_subsets_check(5)


@pytest.mark.slow
def test_exhaustive_k6():
    _all_subsets_check(6)


@st.composite
def multigraphs(draw):
    n = draw(st.integers(min_value=1, max_value=40))
    m = draw(st.integers(min_value=0, max_value=120))
    src = draw(st.lists(st.integers(0, n - 1), min_size=m, max_size=m))
    dst = draw(st.lists(st.integers(0, n - 1), min_size=m, max_size=m))
    occ = draw(st.lists(st.integers(0, 3), min_size=m, max_size=m))  # any nonzero = occupied
    return n, np.array(src, np.int32), np.array(dst, np.int32), np.array(occ, np.uint8)


@settings(max_examples=300, deadline=None, derandomize=True)
@given(multigraphs())
def test_random_multigraphs_vs_bfs_and_scipy(g):
    n, src, dst, occ = g
    got = oracle.label_edges(n, src, dst, occ)
    want = oracle.label_bfs(n, [(int(a), int(b)) for a, b, o in zip(src, dst, occ) if o])
    assert got.tolist() == want
    np.testing.assert_array_equal(got, scipy_labels(n, src, dst, occ))
    check_invariants(got, n, src, dst, occ)


@pytest.mark.parametrize("seed", [1, 2])
def test_lattices_vs_scipy(seed):
    for g in (gen.honeycomb_realization(64, 0.6527, seed), gen.triangle_realization(64, 0.3473, seed),
              gen.bethe_random_regular(20000, 3, 0.5, seed)):
        got = oracle.label_edges(g.n_sites, g.src, g.dst, g.occ)
        np.testing.assert_array_equal(got, scipy_labels(g.n_sites, g.src, g.dst, g.occ))
        check_invariants(got, g.n_sites, g.src, g.dst, g.occ)


def test_csr_and_ell_forms_match_bfs():
    L, p = 6, 0.4
    g = gen.triangle_csr_realization(L, p, 9)
    n = g.n_sites
    rows = np.repeat(np.arange(n, dtype=np.int32), np.diff(g.row_ptr))
    want = oracle.label_bfs(n, [(int(a), int(b)) for a, b, o in zip(rows, g.col, g.occ) if o])
    assert oracle.label_csr(n, g.row_ptr, g.col, g.occ).tolist() == want
    # the paper's padded, column-major neighbour list: each bond appears in
    # both endpoints' lists and carries the same occupancy in both
    z = 6
    nn = np.full((z, n), -1, np.int32)
    occ_ell = np.zeros((z, n), np.uint8)
    fill = np.zeros(n, np.int64)
    for a, b, o in zip(rows, g.col, g.occ):
        for u, v in ((a, b), (b, a)):
            nn[fill[u], u] = v
            occ_ell[fill[u], u] = o
            fill[u] += 1
    assert (fill == 6).all()
    assert oracle.label_ell(n, z, nn.ravel(), occ_ell.ravel()).tolist() == want
    # padding entries are skipped
    nn[5, :] = -1
    got = oracle.label_ell(n, z, nn.ravel(), occ_ell.ravel())
    check_invariants(got, n, np.zeros(0, np.int32), np.zeros(0, np.int32), None)


def test_ell_from_edges_round_trip():
    g = gen.triangle_realization(7, 0.5, 4)
    nn, oe = gen.ell_from_edges(g.n_sites, g.src, g.dst, g.occ, 6)
    assert nn.shape == (6, g.n_sites) and (nn >= 0).all()  # every triangle site has six neighbours
    back = {(min(int(nn[k, i]), i), max(int(nn[k, i]), i), int(oe[k, i]))
            for k in range(6) for i in range(g.n_sites)}
    want = {(min(int(a), int(b)), max(int(a), int(b)), int(o)) for a, b, o in zip(g.src, g.dst, g.occ)}
    assert back == want
    with pytest.raises(ValueError):
        gen.ell_from_edges(g.n_sites, g.src, g.dst, g.occ, 5)


@pytest.mark.parametrize("shells", [6, 9])
@pytest.mark.parametrize("p", [0.25, 0.5, 0.75])
def test_standard_cayley_leaves_no_residual_list(shells, p):
    """Section 3.3 of the paper: with the Bethe lattice numbered from the
    centre outward every residual list is empty after initialization, so
    steps (i) and (ii) alone give the final labels; with random numbering
    they do not."""
    for random_position in (False, True):
        g = gen.cayley_realization(shells, p, 5, random_position)
        n = g.n_sites
        nn, oe = gen.ell_from_edges(n, g.src, g.dst, g.occ, 3)
        left = oracle.ell_residual_left(n, 3, nn, oe)
        after_ii = oracle.analysis(oracle.ell_init(n, 3, nn, oe))
        final = oracle.label_ell(n, 3, nn.ravel(), oe.ravel())
        np.testing.assert_array_equal(final, oracle.label_edges(n, g.src, g.dst, g.occ))
        if not random_position:
            assert left.sum() == 0
            np.testing.assert_array_equal(after_ii, final)
        else:
            assert left.sum() > 0
            if p == 0.75:  # enough joins that step (iii) has work to do
                assert not np.array_equal(after_ii, final)


def test_ell_steps_i_ii_pinned():
    """Step (i) points every site at a lower neighbour (or itself), so step
    (ii) must give the minimum of each tree of that forest: the edge oracle
    on the forest's edges.  Every label after (ii) is a root."""
    rng = np.random.default_rng(17)
    n, z = 400, 7
    nn = rng.integers(-60, n, (z, n)).astype(np.int32)  # negatives are padding
    occ = (rng.random((z, n)) < 0.6).astype(np.uint8)
    init = oracle.ell_init(n, z, nn, occ)
    i = np.arange(n)
    assert (init <= i).all()
    lower = (nn >= 0) & (nn < i) & (occ != 0)
    assert ((init == i) == ~lower.any(axis=0)).all()
    after = oracle.analysis(init)
    assert (after[after] == after).all()
    moved = init != i
    np.testing.assert_array_equal(after, oracle.label_edges(n, i[moved].astype(np.int32), init[moved]))
    # and the full schedule equals brute force on the bonds seen from their
    # higher end (each listed bond here appears in one list only)
    bonds = [(int(i_), int(nn[k, i_])) for k in range(z) for i_ in range(n) if lower[k, i_]]
    want = oracle.label_bfs(n, bonds)
    src = np.array([a for a, _ in bonds], np.int32)
    dst = np.array([b for _, b in bonds], np.int32)
    assert oracle.label_edges(n, src, dst).tolist() == want


def test_cluster_statistics_pinned():
    """Sequential ids: consecutive from 0, ordered like the cluster minima,
    equal exactly within a cluster; sizes at the minima sum to N and match
    the ids' histogram; brute force on a small lattice."""
    g = gen.triangle_realization(12, 0.3473, 21)
    lab = oracle.label_edges(g.n_sites, g.src, g.dst, g.occ)
    ids, count = oracle.cluster_ids(lab)
    mins = np.flatnonzero(lab == np.arange(g.n_sites))
    assert count == mins.size
    np.testing.assert_array_equal(ids[mins], np.arange(count))  # k-th smallest minimum -> k
    assert ((ids[:, None] == ids[None, :]) == (lab[:, None] == lab[None, :])).all()
    sizes = oracle.sizes_by_minimum(lab)
    assert sizes.sum() == g.n_sites and (sizes[mins] > 0).all() and (np.delete(sizes, mins) == 0).all()
    np.testing.assert_array_equal(sizes[mins], np.bincount(ids))
    np.testing.assert_array_equal(sizes[mins], oracle.cluster_sizes(lab))
    clusters = oracle.label_bfs(g.n_sites, [(int(a), int(b)) for a, b, o in zip(g.src, g.dst, g.occ) if o])
    for r in mins:
        assert sizes[r] == clusters.count(int(r))


def test_csr_with_empty_rows_and_ragged_degrees():
    # honeycomb half-CSR has every B row empty
    L = 5
    row_ptr, col = gen.honeycomb_csr(L)
    occ = gen.bernoulli(3, len(col), 0.7)
    src, dst = gen.honeycomb_edges(L)
    np.testing.assert_array_equal(oracle.label_csr(2 * L * L, row_ptr, col, occ),
                                  oracle.label_bfs(2 * L * L,
                                                   [(int(a), int(b)) for a, b, o in
                                                    zip(src, dst, occ) if o]))
    # ragged degrees 0..5
    rng = np.random.default_rng(5)
    n = 50
    deg = rng.integers(0, 6, n)
    rp = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    c = rng.integers(0, n, rp[-1]).astype(np.int32)
    o = rng.integers(0, 2, rp[-1]).astype(np.uint8)
    rows = np.repeat(np.arange(n), deg)
    assert oracle.label_csr(n, rp, c, o).tolist() == oracle.label_bfs(
        n, [(int(a), int(b)) for a, b, x in zip(rows, c, o) if x])


@pytest.mark.parametrize("shells,p", [(10, 0.25), (10, 0.5), (12, 0.75), (12, 1.0)])
@pytest.mark.parametrize("random_position", [False, True])
def test_cayley_forest_cluster_count(shells, p, random_position):
    """A tree has no cycles (section 4), so every occupied bond removes exactly
    one cluster: #clusters = N - #occupied."""
    g = gen.cayley_realization(shells, p, seed=shells * 7 + int(p * 100), random_position=random_position)
    lab = oracle.label_edges(g.n_sites, g.src, g.dst, g.occ)
    assert len(np.unique(lab)) == g.n_sites - int(g.occ.sum())
    check_invariants(lab, g.n_sites, g.src, g.dst, g.occ)


def test_standard_position_labels_are_ancestors():
    """With sites numbered outward from the centre, every cluster's smallest
    site is its site nearest the centre; so a site's label is reached by
    walking occupied bonds towards the centre."""
    shells, p = 11, 0.75
    g = gen.cayley_realization(shells, p, 5, random_position=False)
    lab = oracle.label_edges(g.n_sites, g.src, g.dst, g.occ)
    parent = np.full(g.n_sites, -1, np.int64)
    parent[g.src] = g.dst  # src = child, dst = parent in standard position
    up = np.zeros(g.n_sites, bool)
    up[g.src] = g.occ.astype(bool)
    want = np.arange(g.n_sites)
    for v in range(1, g.n_sites):  # parents come first in standard numbering
        if up[v]:
            want[v] = want[parent[v]]
    np.testing.assert_array_equal(lab, want)


def test_batched_matches_single_instances():
    specs = [gen.InstanceSpec("honeycomb", 8, 0.65, 1), gen.InstanceSpec("triangle", 7, 0.35, 2),
             gen.InstanceSpec("triangle", 1, 0.35, 3), gen.InstanceSpec("honeycomb", 16, 0.9, 4)]
    site_off, bond_off, src, dst, occ = gen.batch_arrays(specs)
    got = oracle.label_batched(site_off, bond_off, src, dst, occ, n_threads=3)
    for k in range(len(specs)):
        a, b = bond_off[k], bond_off[k + 1]
        n = site_off[k + 1] - site_off[k]
        np.testing.assert_array_equal(got[site_off[k]:site_off[k + 1]],
                                      scipy_labels(n, src[a:b], dst[a:b], occ[a:b]))


def test_descending_path_and_star():
    n = 100_000
    src = np.arange(n - 1, 0, -1, dtype=np.int32)
    dst = src - 1
    assert not oracle.label_edges(n, src, dst).any()
    hub = n - 1
    leaves = np.arange(n - 1, dtype=np.int32)
    occ = (leaves % 3 != 0).astype(np.uint8)
    lab = oracle.label_edges(n, np.full(n - 1, hub, np.int32), leaves, occ)
    joined = leaves[occ.astype(bool)]
    assert (lab[joined] == joined.min()).all() and lab[hub] == joined.min()
    lone = leaves[~occ.astype(bool)]
    np.testing.assert_array_equal(lab[lone], lone)


def load_ell_cases():
    """Cases of tests/golden/ell_step_i.txt as (name, n, z, nn[z, n], occ[z, n], expected arrays)."""
    cases, cur = [], None
    for row in read_golden("ell_step_i.txt"):
        if row[0] == "case":
            n, z = int(row[2]), int(row[3])
            cur = dict(name=row[1], n=n, z=z, nn=np.full((z, n), -1, np.int32),
                       occ=np.zeros((z, n), np.uint8))
            cases.append(cur)
        elif row[0] == "s":
            i = int(row[1])
            for k, entry in enumerate(row[2:]):
                v, o = entry.split(":")
                cur["nn"][k, i] = int(v)
                cur["occ"][k, i] = int(o)
        else:
            cur[row[0]] = [int(x) for x in row[1:]]
    return cases


@pytest.mark.parametrize("case", load_ell_cases(), ids=lambda c: c["name"])
def test_ell_steps_hand_worked(case):
    """Step (i) takes the LOWEST occupied lower neighbour (section 3), not the
    first or last listed, not the highest, and not an unoccupied one; step
    (ii) and the whole schedule end where the hand-worked fixture says."""
    n, z, nn, occ = case["n"], case["z"], case["nn"], case["occ"]
    init = oracle.ell_init(n, z, nn, occ)
    assert init.tolist() == case["step_i"]
    assert oracle.ell_residual_left(n, z, nn, occ).tolist() == case["left"]
    assert oracle.analysis(init).tolist() == case["after_ii"]
    assert oracle.label_ell(n, z, nn.ravel(), occ.ravel()).tolist() == case["final"]
