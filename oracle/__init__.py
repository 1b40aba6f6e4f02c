"""CPU oracle for connected-component labeling -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never imports, links or
calls it, and the two share no code (the seeded input generators in ``gen``
serve both and hold none of the labeling arithmetic).

What it computes: for the undirected multigraph of occupied bonds,
``label[i] = min{ j : j is connected to i }`` -- the label of each cluster is
its minimum site number (paper, section 3), bonds being occupied with
probability p (section 4).

* ``label_edges`` / ``label_csr`` / ``label_ell`` / ``label_batched``:
  sequential union-find in plain C (``oracle.c``), larger root pointed at the
  smaller, final find per site.
* ``label_bfs``: breadth-first search in pure Python, the brute force the C
  oracle is pinned against on tiny graphs.
* ``ell_init`` / ``ell_residual_left`` / ``analysis``: the paper's steps (i)
  and (ii) on its neighbour list, in numpy, for the paper's statement that
  standard numbering of the Bethe lattice leaves no residual list (so steps
  (i) and (ii) alone give the final labels).
* ``cluster_sizes`` / ``sizes_by_minimum`` / ``size_histogram`` /
  ``cluster_ids`` / ``spans`` / ``mean_cluster_size`` / ``largest_fraction``:
  percolation observables
  (section 4) and the sequential renumbering (section 3) computed from a
  labeling with numpy.
"""
from __future__ import annotations

import collections
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-pthread", "-shared", "-fPIC", "-Wall", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.oracle_label_edges.argtypes = [i64, i64, P, P, P, P]
        lib.oracle_label_csr.argtypes = [i64, P, P, P, P]
        lib.oracle_label_ell.argtypes = [i64, i32, P, P, P]
        lib.oracle_label_batched.argtypes = [i32, P, P, P, P, P, P, i32]
        for f in (lib.oracle_label_edges, lib.oracle_label_csr, lib.oracle_label_ell,
                  lib.oracle_label_batched):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _u8(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def label_edges(n_sites: int, src, dst, occ=None) -> np.ndarray:
    """Min-site-index cluster labels of the occupied bonds (src[b], dst[b])."""
    src, dst, occ = _i32(src), _i32(dst), _u8(occ)
    assert src.shape == dst.shape and (occ is None or occ.shape == src.shape)
    out = np.empty(n_sites, np.int32)
    if _L().oracle_label_edges(n_sites, len(src), _p(src), _p(dst), _p(occ), _p(out)) != 0:
        raise ValueError("oracle_label_edges: bad size or site id")
    return out


def label_csr(n_sites: int, row_ptr, col, occ=None) -> np.ndarray:
    row_ptr, col, occ = _i32(row_ptr), _i32(col), _u8(occ)
    assert len(row_ptr) == n_sites + 1
    out = np.empty(n_sites, np.int32)
    if _L().oracle_label_csr(n_sites, _p(row_ptr), _p(col), _p(occ), _p(out)) != 0:
        raise ValueError("oracle_label_csr: bad size or site id")
    return out


def label_ell(n_sites: int, z_max: int, nn, occ=None) -> np.ndarray:
    """Paper's padded, column-major neighbour list (slot k of site i at i + k*N)."""
    nn, occ = _i32(nn), _u8(occ)
    assert nn.size == n_sites * z_max
    out = np.empty(n_sites, np.int32)
    if _L().oracle_label_ell(n_sites, z_max, _p(nn), _p(occ), _p(out)) != 0:
        raise ValueError("oracle_label_ell: bad size or site id")
    return out


def ell_init(n_sites: int, z_max: int, nn, occ=None) -> np.ndarray:
    """Step (i) of the paper's schedule on its neighbour list (section 3):
    each site's residual list holds its occupied neighbours numbered below
    it; the site's label becomes the lowest of them (which leaves the list),
    or the site itself when the list is empty."""
    i = np.arange(n_sites, dtype=np.int64)
    if z_max == 0 or n_sites == 0:
        return i.astype(np.int32)
    nn = np.asarray(nn, np.int64).reshape(z_max, n_sites)
    on = np.ones(nn.shape, bool) if occ is None else np.asarray(occ).reshape(z_max, n_sites) != 0
    lower = on & (nn >= 0) & (nn < i)
    return np.where(lower, nn, i).min(axis=0).astype(np.int32)


def ell_residual_left(n_sites: int, z_max: int, nn, occ=None) -> np.ndarray:
    """Entries left on each site's residual list after step (i): its occupied
    lower neighbours less the one step (i) took."""
    if z_max == 0 or n_sites == 0:
        return np.zeros(n_sites, np.int64)
    i = np.arange(n_sites, dtype=np.int64)
    nn = np.asarray(nn, np.int64).reshape(z_max, n_sites)
    on = np.ones(nn.shape, bool) if occ is None else np.asarray(occ).reshape(z_max, n_sites) != 0
    return np.maximum((on & (nn >= 0) & (nn < i)).sum(axis=0) - 1, 0)


def analysis(label) -> np.ndarray:
    """The paper's analysis step: label[i] = label[label[i]] for every site,
    repeated until no label changes (section 3)."""
    lab = np.array(label, np.int64)
    while True:
        nxt = lab[lab]
        if np.array_equal(nxt, lab):
            return lab.astype(np.int32)
        lab = nxt


def label_batched(site_off, bond_off, src, dst, occ=None, n_threads: int = 0) -> np.ndarray:
    """Instance-local labels of independent instances, one per task."""
    site_off = np.ascontiguousarray(site_off, dtype=np.int64)
    bond_off = np.ascontiguousarray(bond_off, dtype=np.int64)
    src, dst, occ = _i32(src), _i32(dst), _u8(occ)
    out = np.empty(int(site_off[-1]), np.int32)
    nt = n_threads if n_threads > 0 else (os.cpu_count() or 1)
    r = _L().oracle_label_batched(len(site_off) - 1, _p(site_off), _p(bond_off), _p(src),
                                  _p(dst), _p(occ), _p(out), nt)
    if r != 0:
        raise ValueError("oracle_label_batched: bad size or site id")
    return out


def label_bfs(n_sites: int, edges) -> list:
    """Brute force for tiny graphs: breadth-first search from every unvisited
    site in increasing order; the site that starts a search is the smallest of
    its cluster, and it labels everything the search reaches."""
    adj = [[] for _ in range(n_sites)]
    for u, v in edges:
        adj[u].append(v)
        adj[v].append(u)
    label = [-1] * n_sites
    for s in range(n_sites):
        if label[s] >= 0:
            continue
        label[s] = s
        q = collections.deque([s])
        while q:
            u = q.popleft()
            for v in adj[u]:
                if label[v] < 0:
                    label[v] = s
                    q.append(v)
    return label


# ------------------------------------------------------------ observables

def cluster_sizes(labels: np.ndarray) -> np.ndarray:
    """Size of every cluster (one entry per root)."""
    counts = np.bincount(labels.astype(np.int64), minlength=len(labels))
    return counts[counts > 0]


def sizes_by_minimum(labels: np.ndarray) -> np.ndarray:
    """sizes[r] = number of sites labelled r: each cluster's size at its
    minimum site, zero elsewhere."""
    return np.bincount(np.asarray(labels, np.int64), minlength=len(labels)).astype(np.int32)


def size_histogram(labels: np.ndarray, n_bins: int) -> np.ndarray:
    """n_s, the number of clusters of exactly s sites (the cluster-size
    distribution of percolation theory, section 4's application): hist[s]
    for 1 <= s < n_bins - 1, the last bin counting every cluster of
    n_bins - 1 sites or more, hist[0] = 0.  Written from its definition:
    count the sites of each cluster, then count the clusters of each size."""
    sites_per_label = np.bincount(np.asarray(labels, np.int64))
    sizes = sites_per_label[sites_per_label > 0]  # one entry per cluster
    return np.bincount(np.minimum(sizes, n_bins - 1), minlength=n_bins).astype(np.int64)


def cluster_ids(labels: np.ndarray):
    """Sequential cluster ids (section 3, last paragraph): clusters numbered
    0, 1, ... in the order of their minimum site.  Returns (ids, count)."""
    uniq, inv = np.unique(np.asarray(labels, np.int64), return_inverse=True)
    return inv.astype(np.int32), int(uniq.size)


def mean_cluster_size(labels: np.ndarray) -> float:
    """Sum over clusters of |C|^2 / N: the mean size of the cluster holding a
    uniformly chosen site."""
    s = cluster_sizes(labels).astype(np.float64)
    return float((s * s).sum() / len(labels))


def largest_fraction(labels: np.ndarray) -> float:
    return float(cluster_sizes(labels).max() / len(labels))


def spans(labels: np.ndarray, first_row: np.ndarray, last_row: np.ndarray) -> bool:
    """True when one cluster holds a site of `first_row` and one of `last_row`
    (the spanning criterion of section 4, read as top-to-bottom)."""
    return bool(np.intersect1d(labels[first_row], labels[last_row]).size)
