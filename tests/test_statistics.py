"""Statistical pins of generators + oracle together against closed forms the
paper quotes (section 4): the bond thresholds of the honeycomb and triangle
lattices through the crossing of spanning-probability curves, and the Bethe
lattice threshold 1/(z-1) through tree-like branching results on random
z-regular graphs.  All inputs are seeded, so every run sees the same numbers."""
import math

import numpy as np
import pytest

import gen
import oracle
from conftest import read_golden


def _thresholds():
    return {r[0]: float(r[1]) for r in read_golden("thresholds.txt")}


def test_golden_thresholds_are_the_closed_forms():
    t = {r[0]: r for r in read_golden("thresholds.txt")}
    assert float(t["honeycomb"][1]) == pytest.approx(1 - 2 * math.sin(math.pi / 18), abs=1e-15)
    assert float(t["triangle"][1]) == pytest.approx(2 * math.sin(math.pi / 18), abs=1e-15)
    # the paper's estimates agree with the exact values within their error bars
    for k in ("honeycomb", "triangle"):
        assert abs(float(t[k][1]) - float(t[k][2])) <= float(t[k][3])
    assert gen.PC_HONEYCOMB == pytest.approx(float(t["honeycomb"][1]), abs=1e-15)
    assert gen.PC_TRIANGLE == pytest.approx(float(t["triangle"][1]), abs=1e-15)


def _cylinder(kind, L):
    """Lattice with the y-wrap bonds removed (open top and bottom, periodic
    sides); returns (n, src, dst, keep-mask, top-row sites, bottom-row sites)."""
    if kind == "honeycomb":
        src, dst = gen.honeycomb_edges(L)
        n, wrap = 2 * L * L, gen.y_wrap_bonds_honeycomb(L)
        row = (np.arange(n) // 2) // L
    else:
        src, dst = gen.triangle_edges(L)
        n, wrap = L * L, gen.y_wrap_bonds_triangle(L)
        row = np.arange(n) // L
    keep = ~wrap
    return n, src[keep], dst[keep], keep, np.nonzero(row == 0)[0], np.nonzero(row == L - 1)[0]


def spanning_thresholds(kind, L, samples, seed0):
    """Per realization, the smallest p at which it spans top to bottom.
    Each realization draws one word u_b per bond; the bond is occupied at p
    iff u_b < p 2^32, so spanning is monotone in p and a bisection over the
    sorted words finds the exact switching point, each probe being one oracle
    labeling followed by the spanning check."""
    n, s, d, keep, top, bot = _cylinder(kind, L)
    out = np.empty(samples)
    for k in range(samples):
        u = gen.u32(gen.mix_seed(seed0, k), gen.STREAM_OCC, len(keep))[keep]
        us = np.sort(u)
        lo, hi = 0, len(us)  # not spanning with lo bonds, spanning with hi
        while hi - lo > 1:
            mid = (lo + hi) // 2
            lab = oracle.label_edges(n, s, d, (u <= us[mid - 1]).astype(np.uint8))
            if oracle.spans(lab, top, bot):
                hi = mid
            else:
                lo = mid
        out[k] = (int(us[hi - 1]) + 1) / 2.0**32
    return out


def crossing_points(small, big, centre, half_width=0.03, grid=601):
    """Upward zero crossings of R_big(p) - R_small(p), R being the empirical
    spanning probability (fraction of realizations whose threshold is <= p)."""
    ps = np.linspace(centre - half_width, centre + half_width, grid)
    diff = (big[None, :] <= ps[:, None]).mean(1) - (small[None, :] <= ps[:, None]).mean(1)
    idx = np.nonzero((diff[:-1] < 0) & (diff[1:] >= 0))[0]
    return [ps[i] + (ps[i + 1] - ps[i]) * (-diff[i]) / (diff[i + 1] - diff[i]) for i in idx]


@pytest.mark.parametrize("kind", ["honeycomb", "triangle"])
def test_spanning_curves_cross_at_exact_threshold(kind):
    """The spanning probabilities of two sizes cross at p_c (section 4):
    honeycomb 1 - 2 sin(pi/18), triangle 2 sin(pi/18).  L = 64 and 256 with
    500 realizations each put the crossing within +-0.004 (the paper reached
    +-0.0002 with N up to 2^24)."""
    pc = _thresholds()[kind]
    small = spanning_thresholds(kind, 64, 500, seed0=640 + len(kind))
    big = spanning_thresholds(kind, 256, 500, seed0=2560 + len(kind))
    # curves are ordered away from p_c: the larger system is sharper
    assert (big <= pc - 0.02).mean() < (small <= pc - 0.02).mean()
    assert (big <= pc + 0.02).mean() > (small <= pc + 0.02).mean()
    roots = crossing_points(small, big, pc)
    assert roots, "spanning curves do not cross near p_c"
    assert abs(float(np.median(roots)) - pc) < 0.004, roots


def _bethe_labels(n, z, p, seed):
    g = gen.bethe_random_regular(n, z, p, seed)
    return oracle.label_edges(g.n_sites, g.src, g.dst, g.occ)


def test_bethe_mean_cluster_size_below_threshold():
    """Below p_c = 1/(z-1) a random z-regular graph is locally a Bethe lattice,
    and the mean size of the cluster holding a random site is
    S = 1 + z p T with T = 1 + (z-1) p T, i.e. S = (1 + p) / (1 - (z-1) p):
    14.5 at z = 3, p = 0.45."""
    z, p = 3, 0.45
    want = (1 + p) / (1 - (z - 1) * p)
    assert want == pytest.approx(14.5)
    got = np.mean([oracle.mean_cluster_size(_bethe_labels(1 << 20, z, p, 100 + s)) for s in range(8)])
    assert got == pytest.approx(want, rel=0.015)


def test_bethe_giant_fraction_above_threshold():
    """Above p_c a giant cluster appears.  With u = the probability that one
    bond end (the bond itself included) does not lead into the giant cluster,
    u = 1 - p + p u^(z-1) and the giant fraction is 1 - u^z.  z = 3, p = 0.55:
    u = 9/11 and P = 1 - (9/11)^3 = 602/1331 = 0.45229..."""
    z, p = 3, 0.55
    u = 9.0 / 11.0
    assert u == pytest.approx(1 - p + p * u ** (z - 1), abs=1e-15)
    want = 1 - u**z
    assert want == pytest.approx(602 / 1331, abs=1e-15)
    got = np.mean([oracle.largest_fraction(_bethe_labels(1 << 20, z, p, 200 + s)) for s in range(4)])
    assert abs(got - want) < 0.005


def test_bethe_no_giant_below_threshold():
    lab = _bethe_labels(1 << 20, 3, 0.45, 300)
    assert oracle.largest_fraction(lab) < 0.01


@pytest.mark.parametrize("z,p", [(4, 0.30), (6, 0.17)])
def test_bethe_mean_cluster_size_other_z(z, p):
    want = (1 + p) / (1 - (z - 1) * p)
    got = np.mean([oracle.mean_cluster_size(_bethe_labels(1 << 19, z, p, 400 + s)) for s in range(6)])
    assert got == pytest.approx(want, rel=0.03)


# ------------------------------------------------------------ cluster-size histogram

def test_size_histogram_hand_worked():
    # clusters {0,1}, {2,3,4}, {5}: one each of sizes 2, 3 and 1
    lab = np.array([0, 0, 2, 2, 2, 5], np.int32)
    assert oracle.size_histogram(lab, 8).tolist() == [0, 1, 1, 1, 0, 0, 0, 0]
    # the last bin takes every cluster at least that large
    assert oracle.size_histogram(lab, 3).tolist() == [0, 1, 2]


def test_size_histogram_sums_and_extremes():
    g = gen.triangle_realization(64, 0.35, 7)
    lab = oracle.label_edges(g.n_sites, g.src, g.dst, g.occ)
    h = oracle.size_histogram(lab, g.n_sites + 1)
    assert int((np.arange(len(h)) * h).sum()) == g.n_sites      # every site in one cluster
    assert int(h.sum()) == len(np.unique(lab))                 # every cluster counted once
    n = 1000
    ident = np.arange(n, dtype=np.int32)                       # no bond occupied
    assert oracle.size_histogram(ident, 5).tolist() == [0, n, 0, 0, 0]
    whole = np.zeros(n, np.int32)                              # one cluster of every site
    h = oracle.size_histogram(whole, n + 1)
    assert h[n] == 1 and h.sum() == 1
    assert oracle.size_histogram(whole, 10).tolist() == [0] * 9 + [1]


def test_size_histogram_one_dimensional_closed_form():
    """Bond percolation on an open chain of N sites: a cluster of s sites is
    a run of s - 1 occupied bonds between two empty ones, so the expected
    number of s-site clusters is about N (1 - p)^2 p^(s - 1) (textbook 1-D
    percolation); a chain of 2,000,000 sites at p = 0.5 matches it to 1%."""
    n, p = 2_000_000, 0.5
    src = np.arange(n - 1, dtype=np.int32)
    dst = src + 1
    occ = gen.bernoulli(31, n - 1, p)
    lab = oracle.label_edges(n, src, dst, occ)
    h = oracle.size_histogram(lab, 12)
    for s in range(1, 8):
        want = n * (1 - p) ** 2 * p ** (s - 1)
        assert abs(h[s] - want) / want < 0.01 + 4 / math.sqrt(want), (s, h[s], want)
