"""Pins for the seeded input generators (host only)."""
import math

import numpy as np
import pytest

import gen
from conftest import read_golden


def test_philox_known_answers():
    rows = read_golden("philox4x32_10_kat.txt")
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = gen.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_u32_stream_layout_matches_block_function():
    seed, stream = 0x1234_5678_9ABC_DEF0, 7
    words = gen.u32(seed, stream, 40)
    for blk in range(10):
        ref = gen.philox4x32_10([blk, 0, stream, 0], [seed & 0xFFFFFFFF, seed >> 32])
        assert list(words[4 * blk:4 * blk + 4]) == list(ref)
    # an offset window is the same slice of the stream
    assert list(gen.u32(seed, stream, 13, first=7)) == list(words[7:20])


def test_threshold_and_mask():
    assert gen.threshold(0.0) == 0
    assert gen.threshold(-1.0) == 0
    assert gen.threshold(1.0) == 2**32
    assert gen.threshold(0.5) == 2**31
    assert gen.threshold(0.25) == 2**30
    seed, n = 99, 10_000
    w = gen.u32(seed, gen.STREAM_OCC, n)
    for p in (0.0, 0.3, 0.5, 0.97, 1.0):
        occ = gen.bernoulli(seed, n, p)
        assert occ.dtype == np.uint8
        np.testing.assert_array_equal(occ, (w.astype(np.uint64) < gen.threshold(p)).astype(np.uint8))
    assert gen.bernoulli(seed, n, 1.0).all() and not gen.bernoulli(seed, n, 0.0).any()


@pytest.mark.parametrize("p", [0.1736, 0.3473, 0.6527])
def test_occupied_fraction_binomial_band(p):
    n = 1 << 20
    k = int(gen.bernoulli(12345, n, p).sum())
    sigma = math.sqrt(n * p * (1 - p))
    assert abs(k - n * p) < 5 * sigma


def _degrees(n, src, dst):
    return np.bincount(src, minlength=n) + np.bincount(dst, minlength=n)


@pytest.mark.parametrize("L", [3, 4, 17])
def test_honeycomb_structure(L):
    src, dst = gen.honeycomb_edges(L)
    n = 2 * L * L
    assert len(src) == 3 * L * L
    assert (_degrees(n, src, dst) == 3).all()
    assert (src % 2 == 0).all() and (dst % 2 == 1).all()  # bipartite A-B
    keys = set(zip(np.minimum(src, dst).tolist(), np.maximum(src, dst).tolist()))
    assert len(keys) == len(src)  # simple graph
    # the hexagon A(x,y) B(x,y) A(x+1,y) B(x+1,y-1) A(x+1,y-1) B(x,y-1) closes
    A = lambda x, y: 2 * ((y % L) * L + (x % L))
    B = lambda x, y: A(x, y) + 1
    for (x, y) in [(0, 0), (L - 1, 0), (1, L - 1)]:
        ring = [A(x, y), B(x, y), A(x + 1, y), B(x + 1, y - 1), A(x + 1, y - 1), B(x, y - 1)]
        for a, b in zip(ring, ring[1:] + ring[:1]):
            assert (min(a, b), max(a, b)) in keys
    # CSR form holds the same bonds
    row_ptr, col = gen.honeycomb_csr(L)
    rows = np.repeat(np.arange(n, dtype=np.int32), np.diff(row_ptr))
    np.testing.assert_array_equal(rows, src)
    np.testing.assert_array_equal(col, dst)


@pytest.mark.parametrize("L", [3, 5, 16])
def test_triangle_structure(L):
    src, dst = gen.triangle_edges(L)
    n = L * L
    assert (_degrees(n, src, dst) == 6).all()
    keys = set(zip(np.minimum(src, dst).tolist(), np.maximum(src, dst).tolist()))
    assert len(keys) == 3 * n
    site = lambda x, y: (y % L) * L + (x % L)
    for (x, y) in [(0, 0), (L - 1, L - 1), (2, 1)]:
        nbrs = {site(x + 1, y), site(x - 1, y), site(x, y + 1), site(x, y - 1), site(x + 1, y + 1),
                site(x - 1, y - 1)}
        got = set(dst[src == site(x, y)].tolist()) | set(src[dst == site(x, y)].tolist())
        assert got == nbrs
    row_ptr, col = gen.triangle_csr(L)
    np.testing.assert_array_equal(row_ptr, 3 * np.arange(n + 1))
    np.testing.assert_array_equal(col, dst)


def test_wrap_masks():
    L = 6
    hs, hd = gen.honeycomb_edges(L)
    w = gen.y_wrap_bonds_honeycomb(L)
    assert w.sum() == L
    rows_s, rows_d = (hs // 2) // L, (hd // 2) // L
    assert (np.abs(rows_s - rows_d)[w] == L - 1).all() and (np.abs(rows_s - rows_d)[~w] <= 1).all()
    ts, td = gen.triangle_edges(L)
    w = gen.y_wrap_bonds_triangle(L)
    assert w.sum() == 2 * L
    assert (np.abs(ts // L - td // L)[w] == L - 1).all() and (np.abs(ts // L - td // L)[~w] <= 1).all()


@pytest.mark.parametrize("shells", [0, 1, 2, 5, 17])
def test_cayley_tree(shells):
    n = gen.cayley_size(shells)
    assert n == (1 if shells == 0 else 3 * 2**shells - 2)
    src, dst = gen.cayley_tree(shells)
    assert len(src) == n - 1
    if n > 1:
        deg = _degrees(n, src, dst)
        assert deg[0] == 3 or n == 1
        # internal sites have degree 3, leaves (the last shell) degree 1
        leaves = 3 * 2 ** (shells - 1)
        assert (deg[n - leaves:] == 1).all() and (deg[:n - leaves] == 3).all()
        # standard position: every site's parent has a smaller number
        assert (dst < src).all()


def test_paper_bethe_sizes():
    # the paper's Bethe-lattice sizes are exactly the Cayley trees with G = 17..22
    assert [gen.cayley_size(g) for g in range(17, 23)] == [393214, 786430, 1572862, 3145726,
                                                           6291454, 12582910]


@pytest.mark.parametrize("n,z", [(1000, 3), (5000, 4), (2000, 6), (1 << 16, 3)])
def test_random_regular_simple(n, z):
    src, dst = gen.random_regular(n, z, seed=42 + n + z)
    assert len(src) == n * z // 2
    assert (_degrees(n, src, dst) == z).all()
    assert (src != dst).all()
    keys = np.minimum(src, dst).astype(np.int64) * n + np.maximum(src, dst)
    assert len(np.unique(keys)) == len(keys)


def test_random_regular_rejects_bad_args():
    with pytest.raises(ValueError):
        gen.random_regular(5, 3, 1)  # n z odd


def test_randomize_positions_is_relabelling():
    n, z = 4000, 3
    src, dst = gen.random_regular(n, z, 5)
    s0, d0 = src.copy(), dst.copy()
    gen.randomize_positions(src, dst, n, 5)
    perm = gen.permutation(5, n)
    assert sorted(perm.tolist()) == list(range(n))
    k0 = set(zip(np.minimum(perm[s0], perm[d0]).tolist(), np.maximum(perm[s0], perm[d0]).tolist()))
    k1 = set(zip(np.minimum(src, dst).tolist(), np.maximum(src, dst).tolist()))
    assert k0 == k1
    assert not np.array_equal(src, perm[s0])  # order or orientation changed


def test_determinism_per_seed():
    a = gen.bethe_random_regular(3000, 3, 0.5, 11)
    b = gen.bethe_random_regular(3000, 3, 0.5, 11)
    c = gen.bethe_random_regular(3000, 3, 0.5, 12)
    for x, y in ((a.src, b.src), (a.dst, b.dst), (a.occ, b.occ)):
        np.testing.assert_array_equal(x, y)
    assert not np.array_equal(a.src, c.src)


def test_batch_specs_and_offsets():
    specs = gen.batch_specs(64, base_seed=7)
    assert {s.kind for s in specs} == {"honeycomb", "triangle"}
    for s in specs:
        pc = gen.PC_HONEYCOMB if s.kind == "honeycomb" else gen.PC_TRIANGLE
        assert pc - 0.05 <= s.p <= pc + 0.05 and s.L in gen.BATCH_LS
    assert len({s.seed for s in specs}) == 64
    site_off, bond_off = gen.batch_offsets(specs)
    assert site_off[0] == 0 and bond_off[0] == 0
    assert (np.diff(site_off) == [s.n_sites for s in specs]).all()
    small = [gen.InstanceSpec("honeycomb", 4, 0.6, 1), gen.InstanceSpec("triangle", 3, 0.3, 2)]
    so, bo, src, dst, occ = gen.batch_arrays(small)
    np.testing.assert_array_equal(src[:48], gen.honeycomb_edges(4)[0])
    np.testing.assert_array_equal(dst[48:], gen.triangle_edges(3)[1])
    np.testing.assert_array_equal(occ[48:], gen.bernoulli(2, 27, 0.3))


def test_request_trace():
    reqs = gen.request_trace(2000, rate=100.0, base_seed=3)
    t = np.array([r.arrival for r in reqs])
    assert (np.diff(t) > 0).all()
    # mean inter-arrival 1/rate within 5 sigma (exponential: sigma = mean / sqrt(n))
    assert abs(t[-1] / len(t) - 0.01) < 5 * 0.01 / math.sqrt(len(t))
    for r in reqs:
        assert r.z in (3, 4, 6) and 1000 <= r.n_sites <= 10_000_001 and (r.n_sites * r.z) % 2 == 0
        assert abs(r.p - 1.0 / (r.z - 1)) <= 0.02
    logn = np.log10([r.n_sites for r in reqs])
    assert abs(logn.mean() - 5.0) < 0.1  # log-uniform over [3, 7]
