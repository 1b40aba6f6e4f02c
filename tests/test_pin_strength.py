"""The pins must catch plausible mistakes.  Each mutant below is the oracle's
union-find with one planted error (run on the CPU only); the pins used against
the real oracle -- hand-worked cases, breadth-first brute force and the
labeling invariants -- must reject every mutant."""
import numpy as np
import pytest

import oracle
from test_oracle import check_invariants, load_cases


def _uf_label(n, src, dst, occ, *, link_larger=False, ignore_occ=False, no_final=False,
              skip_reversed=False, drop_last=False, same_endpoint=False):
    parent = list(range(n))

    def root(x):
        while parent[x] != x:
            x = parent[x]
        return x

    m = len(src) - (1 if drop_last and len(src) else 0)
    for b in range(m):
        if not ignore_occ and not occ[b]:
            continue
        u, v = int(src[b]), int(dst[b])
        if same_endpoint:
            v = u
        if skip_reversed and u > v:
            continue
        ru, rv = root(u), root(v)
        if ru == rv:
            continue
        lo, hi = min(ru, rv), max(ru, rv)
        if link_larger:
            parent[lo] = hi
        else:
            parent[hi] = lo
    if no_final:
        return np.array(parent, np.int32)
    return np.array([root(i) for i in range(n)], np.int32)


MUTANTS = {
    "links the smaller root under the larger": dict(link_larger=True),
    "ignores the occupancy mask": dict(ignore_occ=True),
    "skips the final flatten": dict(no_final=True),
    "drops bonds listed high-to-low": dict(skip_reversed=True),
    "drops the last bond": dict(drop_last=True),
    "uses one endpoint twice": dict(same_endpoint=True),
}


def _pins_reject(fn) -> bool:
    for case in load_cases():
        n, b = case["n"], case["bonds"]
        src = np.array([x[0] for x in b], np.int32)
        dst = np.array([x[1] for x in b], np.int32)
        occ = np.array([x[2] for x in b], np.uint8)
        got = fn(n, src, dst, occ)
        if got.tolist() != case["expect"]:
            return True
        if got.tolist() != oracle.label_bfs(n, [(u, v) for u, v, o in b if o]):
            return True
        try:
            check_invariants(got, n, src, dst, occ)
        except AssertionError:
            return True
    return False


def test_unmutated_copy_passes_the_pins():
    assert not _pins_reject(lambda n, s, d, o: _uf_label(n, s, d, o))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name):
    kw = MUTANTS[name]
    assert _pins_reject(lambda n, s, d, o: _uf_label(n, s, d, o, **kw)), name


# ---- step (i) of the paper's schedule: the residual list's lowest entry

def _ell_init_mutant(n, z, nn, occ, *, pick="lowest", ignore_occ=False):
    """oracle.ell_init's definition with one planted error: the entry taken
    from the residual list ("highest", "first" or "last" listed instead of
    the lowest), or the mask ignored."""
    nn = np.asarray(nn).reshape(z, n)
    on = np.ones(nn.shape, bool) if ignore_occ else np.asarray(occ).reshape(z, n) != 0
    out = np.arange(n, dtype=np.int32)
    for i in range(n):
        lower = [int(nn[k, i]) for k in range(z)
                 if on[k, i] and 0 <= nn[k, i] < i]
        if not lower:
            continue
        out[i] = {"lowest": min, "highest": max, "first": lambda l: l[0], "last": lambda l: l[-1]}[pick](lower)
    return out


ELL_MUTANTS = {
    "takes the highest lower neighbour": dict(pick="highest"),
    "takes the first listed lower neighbour": dict(pick="first"),
    "takes the last listed lower neighbour": dict(pick="last"),
    "ignores the occupancy mask": dict(ignore_occ=True),
}


def _ell_pins_reject(fn) -> bool:
    from test_oracle import load_ell_cases

    for case in load_ell_cases():
        got = fn(case["n"], case["z"], case["nn"], case["occ"])
        if got.tolist() != case["step_i"]:
            return True
        if oracle.analysis(got).tolist() != case["after_ii"]:
            return True
    return False


def test_unmutated_ell_init_passes_the_pins():
    assert not _ell_pins_reject(lambda n, z, nn, o: _ell_init_mutant(n, z, nn, o))
    assert not _ell_pins_reject(oracle.ell_init)


@pytest.mark.parametrize("name", sorted(ELL_MUTANTS))
def test_pins_reject_ell_init_mutant(name):
    kw = ELL_MUTANTS[name]
    assert _ell_pins_reject(lambda n, z, nn, o: _ell_init_mutant(n, z, nn, o, **kw)), name


# ---- the cluster-size histogram

def _hist_mutant(labels, n_bins, *, count_sites=False, size_off_by_one=False, no_overflow_bin=False):
    """oracle.size_histogram's definition with one planted error: sites
    counted instead of clusters, sizes shifted by one, or clusters larger
    than the last bin dropped instead of counted there."""
    vals, counts = np.unique(np.asarray(labels, np.int64), return_counts=True)
    hist = np.zeros(n_bins, np.int64)
    for s in counts:
        s = int(s) + (1 if size_off_by_one else 0)
        if s >= n_bins and no_overflow_bin:
            continue
        hist[min(s, n_bins - 1)] += s if count_sites else 1
    return hist


HIST_MUTANTS = {
    "counts sites instead of clusters": dict(count_sites=True),
    "shifts every size by one": dict(size_off_by_one=True),
    "drops clusters past the last bin": dict(no_overflow_bin=True),
}


def _hist_pins_reject(fn) -> bool:
    import test_statistics as ts
    for test in (ts.test_size_histogram_hand_worked, ts.test_size_histogram_sums_and_extremes):
        saved = oracle.size_histogram
        oracle.size_histogram = fn
        try:
            test()
        except AssertionError:
            return True
        finally:
            oracle.size_histogram = saved
    return False


def test_unmutated_histogram_passes_the_pins():
    assert not _hist_pins_reject(lambda lab, nb: _hist_mutant(lab, nb))


@pytest.mark.parametrize("name", sorted(HIST_MUTANTS))
def test_pins_reject_histogram_mutant(name):
    kw = HIST_MUTANTS[name]
    assert _hist_pins_reject(lambda lab, nb: _hist_mutant(lab, nb, **kw)), name
