"""Seeded synthetic inputs for bond percolation (paper, section 4).

Thin numpy wrapper over ``libcclgen.so`` (``gen.c``): Philox4x32-10 random
words, Bernoulli occupancy masks, honeycomb / triangle lattices (edge list and
half-CSR), the z = 3 Cayley tree, random z-regular graphs, and the workload
recipes built from them (single realizations, the 4096-instance batch, the
request trace for serving).

Holds none of the labeling arithmetic: the oracle and the GPU library both
consume these arrays unchanged.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libcclgen.so")

# stream ids of the counter-based generator
STREAM_OCC = 0
STREAM_GRAPH = 1  # configuration-model shuffle and repairs
STREAM_PERM = 2  # site relabelling ("random position")
STREAM_EDGE_ORDER = 3
STREAM_ORIENT = 4
STREAM_SPEC = 5  # batch instance specs
STREAM_TRACE = 6  # serving request trace

# exact bond-percolation thresholds (paper section 4)
PC_HONEYCOMB = 1.0 - 2.0 * math.sin(math.pi / 18.0)
PC_TRIANGLE = 2.0 * math.sin(math.pi / 18.0)


def pc_bethe(z: int) -> float:
    """Bond threshold of the Bethe lattice with coordination z: 1/(z-1)."""
    return 1.0 / (z - 1)


def build(force: bool = False) -> str:
    """Compile libcclgen.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-Wall", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, u32, u64, dbl = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_double)
        sig = {
            "gen_philox4x32_10": (None, [P, P, P]),
            "gen_u32": (None, [u64, u32, u64, i64, P]),
            "gen_threshold": (u64, [dbl]),
            "gen_bernoulli_mask": (None, [u64, u32, u64, i64, dbl, P]),
            "gen_permutation": (None, [u64, u32, i64, P]),
            "gen_honeycomb_edges": (None, [i32, P, P]),
            "gen_honeycomb_csr": (None, [i32, P, P]),
            "gen_triangle_edges": (None, [i32, P, P]),
            "gen_triangle_csr": (None, [i32, P, P]),
            "gen_cayley_size": (i64, [i32]),
            "gen_cayley_tree": (None, [i32, P, P]),
            "gen_random_regular": (i64, [i64, i32, u64, P, P]),
            "gen_apply_permutation": (None, [i64, P, P, P]),
            "gen_shuffle_edges": (None, [u64, u32, i64, P, P]),
            "gen_random_orientation": (None, [u64, u32, i64, P, P]),
            "gen_mix_seed": (u64, [u64, u64]),
            "gen_ell_from_edges": (ctypes.c_int, [i64, i64, P, P, P, i32, i32, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


# ---------------------------------------------------------------- random words

def philox4x32_10(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block: counter (4 x u32), key (2 x u32) -> 4 x u32."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, np.uint32)
    _L().gen_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def u32(seed: int, stream: int, n: int, first: int = 0) -> np.ndarray:
    out = np.empty(n, np.uint32)
    _L().gen_u32(seed & (2**64 - 1), stream, first, n, _p(out))
    return out


def uniform(seed: int, stream: int, n: int, first: int = 0) -> np.ndarray:
    """n doubles in [0, 1) from 53 bits of two consecutive words."""
    w = u32(seed, stream, 2 * n, 2 * first).astype(np.uint64)
    hi, lo = w[0::2] >> np.uint64(5), w[1::2] >> np.uint64(6)
    return (hi.astype(np.float64) * 67108864.0 + lo.astype(np.float64)) / 9007199254740992.0


def threshold(p: float) -> int:
    return int(_L().gen_threshold(float(p)))


def bernoulli(seed: int, n: int, p: float, stream: int = STREAM_OCC, first: int = 0) -> np.ndarray:
    """uint8 occupancy mask: bond b occupied iff word b < floor(p 2^32)."""
    out = np.empty(n, np.uint8)
    _L().gen_bernoulli_mask(seed & (2**64 - 1), stream, first, n, float(p), _p(out))
    return out


def mix_seed(base: int, k: int) -> int:
    return int(_L().gen_mix_seed(base & (2**64 - 1), k))


def permutation(seed: int, n: int, stream: int = STREAM_PERM) -> np.ndarray:
    out = np.empty(n, np.int32)
    _L().gen_permutation(seed & (2**64 - 1), stream, n, _p(out))
    return out


# ---------------------------------------------------------------- structures

def honeycomb_edges(L: int):
    m = 3 * L * L
    src, dst = np.empty(m, np.int32), np.empty(m, np.int32)
    _L().gen_honeycomb_edges(L, _p(src), _p(dst))
    return src, dst


def honeycomb_csr(L: int):
    row_ptr, col = np.empty(2 * L * L + 1, np.int32), np.empty(3 * L * L, np.int32)
    _L().gen_honeycomb_csr(L, _p(row_ptr), _p(col))
    return row_ptr, col


def triangle_edges(L: int):
    m = 3 * L * L
    src, dst = np.empty(m, np.int32), np.empty(m, np.int32)
    _L().gen_triangle_edges(L, _p(src), _p(dst))
    return src, dst


def triangle_csr(L: int):
    row_ptr, col = np.empty(L * L + 1, np.int32), np.empty(3 * L * L, np.int32)
    _L().gen_triangle_csr(L, _p(row_ptr), _p(col))
    return row_ptr, col


def cayley_size(shells: int) -> int:
    return int(_L().gen_cayley_size(shells))


def cayley_tree(shells: int):
    n = cayley_size(shells)
    src, dst = np.empty(n - 1, np.int32), np.empty(n - 1, np.int32)
    _L().gen_cayley_tree(shells, _p(src), _p(dst))
    return src, dst


def random_regular(n: int, z: int, seed: int):
    """Simple random z-regular graph on n sites (configuration model + repairs)."""
    m = n * z // 2
    src, dst = np.empty(m, np.int32), np.empty(m, np.int32)
    r = _L().gen_random_regular(n, z, seed & (2**64 - 1), _p(src), _p(dst))
    if r < 0:
        raise ValueError(f"random_regular(n={n}, z={z}) failed ({r})")
    return src, dst


def randomize_positions(src: np.ndarray, dst: np.ndarray, n: int, seed: int):
    """The paper's "random position": relabel sites by a uniform permutation,
    then shuffle the edge order and each edge's orientation (in place)."""
    perm = permutation(seed, n, STREAM_PERM)
    lib = _L()
    lib.gen_apply_permutation(len(src), _p(perm), _p(src), _p(dst))
    lib.gen_shuffle_edges(seed & (2**64 - 1), STREAM_EDGE_ORDER, len(src), _p(src), _p(dst))
    lib.gen_random_orientation(seed & (2**64 - 1), STREAM_ORIENT, len(src), _p(src), _p(dst))
    return src, dst


def y_wrap_bonds_honeycomb(L: int) -> np.ndarray:
    """bool mask of the bonds A(x,0)-B(x,L-1) that close the torus in y."""
    mask = np.zeros(3 * L * L, bool)
    mask[2:3 * L:3] = True  # bond 3c+2 of the cells c = x in row y = 0
    return mask


def y_wrap_bonds_triangle(L: int) -> np.ndarray:
    """bool mask of the bonds from row L-1 to row 0."""
    mask = np.zeros(3 * L * L, bool)
    base = 3 * (L - 1) * L
    mask[base + 1::3] = True
    mask[base + 2::3] = True
    return mask


# ---------------------------------------------------------------- workloads

@dataclass
class EdgeGraph:
    n_sites: int
    src: np.ndarray
    dst: np.ndarray
    occ: np.ndarray
    name: str = ""
    p: float = 1.0


@dataclass
class CsrGraph:
    n_sites: int
    row_ptr: np.ndarray
    col: np.ndarray
    occ: np.ndarray
    name: str = ""
    p: float = 1.0


def honeycomb_realization(L: int, p: float, seed: int) -> EdgeGraph:
    """Bond percolation on the periodic honeycomb lattice (2L^2 sites), edge list."""
    src, dst = honeycomb_edges(L)
    return EdgeGraph(2 * L * L, src, dst, bernoulli(seed, len(src), p), f"honeycomb L={L}", p)


def triangle_realization(L: int, p: float, seed: int) -> EdgeGraph:
    src, dst = triangle_edges(L)
    return EdgeGraph(L * L, src, dst, bernoulli(seed, len(src), p), f"triangle L={L}", p)


def triangle_csr_realization(L: int, p: float, seed: int) -> CsrGraph:
    """Bond percolation on the periodic triangle lattice (L^2 sites), half-CSR."""
    row_ptr, col = triangle_csr(L)
    return CsrGraph(L * L, row_ptr, col, bernoulli(seed, len(col), p), f"triangle-csr L={L}", p)


def bethe_random_regular(n: int, z: int, p: float, seed: int) -> EdgeGraph:
    """Random z-regular graph in random position (ids permuted, edges shuffled)."""
    src, dst = random_regular(n, z, seed)
    randomize_positions(src, dst, n, seed)
    return EdgeGraph(n, src, dst, bernoulli(seed, len(src), p), f"random {z}-regular N={n}", p)


def cayley_realization(shells: int, p: float, seed: int, random_position: bool) -> EdgeGraph:
    n = cayley_size(shells)
    src, dst = cayley_tree(shells)
    if random_position:
        randomize_positions(src, dst, n, seed)
    name = f"cayley G={shells} {'random' if random_position else 'standard'}"
    return EdgeGraph(n, src, dst, bernoulli(seed, len(src), p), name, p)


def ell_from_edges(n: int, src: np.ndarray, dst: np.ndarray, occ: np.ndarray | None, z_max: int,
                   pad: int = -1):
    """The paper's padded, column-major neighbour list of an undirected bond
    list (section 3): every bond (a, b) is entered in both a's and b's list
    with the same occupancy, in bond order, unused slots `pad`.  Returns
    (nn, occ_ell), both of shape (z_max, n): row k is slot k of every site
    (occ_ell is None when occ is).  Raises ValueError when a site has more
    than z_max neighbours."""
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    nn = np.empty((z_max, n), np.int32)
    occ_ell = None if occ is None else np.empty((z_max, n), np.uint8)
    o = None if occ is None else np.ascontiguousarray(occ, np.uint8)
    if _L().gen_ell_from_edges(n, len(src), _p(src), _p(dst), None if o is None else _p(o), z_max, pad,
                               _p(nn), None if occ_ell is None else _p(occ_ell)) != 0:
        raise ValueError(f"a site has more than z_max = {z_max} neighbours")
    return nn, occ_ell


# the five workloads of the measurement plan
CONFIG1 = dict(kind="honeycomb", L=256, p=0.6527, seed=1)
CONFIG2 = dict(kind="triangle-csr", L=8192, p=0.3473, seed=2)
CONFIG3 = dict(kind="random-regular", n=1 << 24, z=3, ps=(0.45, 0.5, 0.55), seed=3)


@dataclass
class InstanceSpec:
    kind: str  # "honeycomb" | "triangle"
    L: int
    p: float
    seed: int

    @property
    def n_sites(self) -> int:
        return (2 if self.kind == "honeycomb" else 1) * self.L * self.L

    @property
    def n_bonds(self) -> int:
        return 3 * self.L * self.L


BATCH_LS = (64, 128, 256, 512, 1024)


def batch_specs(k: int, base_seed: int, ls=BATCH_LS, width: float = 0.05):
    """k instance specs: lattice type 50/50, L uniform over `ls`,
    p uniform in [p_c - width, p_c + width], seed = mix(base, i)."""
    u = uniform(base_seed, STREAM_SPEC, 3 * k).reshape(k, 3)
    specs = []
    for i in range(k):
        kind = "honeycomb" if u[i, 0] < 0.5 else "triangle"
        L = ls[min(int(u[i, 1] * len(ls)), len(ls) - 1)]
        pc = PC_HONEYCOMB if kind == "honeycomb" else PC_TRIANGLE
        p = pc - width + 2 * width * u[i, 2]
        specs.append(InstanceSpec(kind, L, float(p), mix_seed(base_seed, i)))
    return specs


def batch_offsets(specs):
    site_off = np.zeros(len(specs) + 1, np.int64)
    bond_off = np.zeros(len(specs) + 1, np.int64)
    site_off[1:] = np.cumsum([s.n_sites for s in specs])
    bond_off[1:] = np.cumsum([s.n_bonds for s in specs])
    return site_off, bond_off


def fill_instance(spec: InstanceSpec, src: np.ndarray, dst: np.ndarray, occ: np.ndarray):
    """Write one instance (instance-local ids) into preallocated views."""
    lib = _L()
    if spec.kind == "honeycomb":
        lib.gen_honeycomb_edges(spec.L, _p(src), _p(dst))
    else:
        lib.gen_triangle_edges(spec.L, _p(src), _p(dst))
    lib.gen_bernoulli_mask(spec.seed & (2**64 - 1), STREAM_OCC, 0, len(occ), spec.p, _p(occ))


def batch_arrays(specs):
    """Concatenated edge lists of a batch (host numpy)."""
    site_off, bond_off = batch_offsets(specs)
    m = int(bond_off[-1])
    src, dst, occ = np.empty(m, np.int32), np.empty(m, np.int32), np.empty(m, np.uint8)
    for i, s in enumerate(specs):
        a, b = int(bond_off[i]), int(bond_off[i + 1])
        fill_instance(s, src[a:b], dst[a:b], occ[a:b])
    return site_off, bond_off, src, dst, occ


@dataclass
class Request:
    rid: int
    arrival: float  # seconds from the start of the trace
    z: int
    n_sites: int
    p: float
    seed: int


def request_trace(count: int, rate: float, base_seed: int, n_min: float = 1e3, n_max: float = 1e7,
                  zs=(3, 4, 6), width: float = 0.02):
    """Poisson arrivals at `rate` per second; z uniform over `zs`, N log-uniform
    in [n_min, n_max] (even when z is odd), p uniform in 1/(z-1) +- width."""
    u = uniform(base_seed, STREAM_TRACE, 4 * count).reshape(count, 4)
    t = 0.0
    reqs = []
    for i in range(count):
        t += -math.log(1.0 - u[i, 0]) / rate
        z = zs[min(int(u[i, 1] * len(zs)), len(zs) - 1)]
        n = int(round(10 ** (math.log10(n_min) + (math.log10(n_max) - math.log10(n_min)) * u[i, 2])))
        n = max(n, z + 2)
        if (n * z) % 2:
            n += 1
        p = pc_bethe(z) - width + 2 * width * u[i, 3]
        reqs.append(Request(i, t, z, n, float(p), mix_seed(base_seed, i)))
    return reqs


def request_graph(r: Request) -> EdgeGraph:
    return bethe_random_regular(r.n_sites, r.z, r.p, r.seed)
