"""Connected-component labeling of occupied bonds on an AMD MI355X.

Thin ctypes binding of ``libccl.so`` (see ``include/ccl.h``).  Every step of
the labeling -- init, the Algorithm-1 merge, flatten, the batched persistent
kernel -- runs in the library's HIP kernels; this module only checks tensor
devices / dtypes / contiguity and passes raw pointers and the current HIP
stream.  PyTorch supplies device memory and streams.  There is no CPU fallback:
if the library is missing or fails to load, importing this package fails.
"""
from __future__ import annotations

import contextlib
import ctypes
import os

import numpy as np
import torch  # first: the library then binds to the HIP runtime torch loaded

__all__ = [
    "CclError", "label", "label_philox", "label_csr", "label_csr_philox", "label_ell", "csr_workspace_bytes",
    "philox_u32", "bernoulli", "cluster_ids", "cluster_ids_noalloc", "cluster_sizes", "size_histogram",
    "spans", "Plan",
    "Tuning",
    "label_batched_per_instance", "validate_edges", "validate_csr", "trace", "probe_copy", "probe_random",
    "library_path", "version",
]

_PKG = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_PKG, "libccl.so")

CCL_OK = 0
CCL_ERR_INDEX_OUT_OF_RANGE = 2


class CclError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.ccl_status_string(status).decode()
        hip = _lib.ccl_last_hip_error()
        super().__init__(f"{where}: {msg}" + (f" (hip error {hip})" if status == 4 else ""))
        self.status = status


class Tuning(ctypes.Structure):
    """ccl_tuning: zero fields take the library defaults."""
    _fields_ = [("block_threads", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("bonds_per_chunk", ctypes.c_int32), ("sites_per_chunk", ctypes.c_int32),
                ("small_sites", ctypes.c_int32), ("schedule", ctypes.c_int32)]

    FUSED = 1
    PHASED = 2
    TILED = 3

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _load():
    if not os.path.exists(library_path):
        raise ImportError(f"{library_path} is not built; run `python -m paper_1603_08357_amd.build`")
    lib = ctypes.CDLL(library_path)
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    st = ctypes.c_int
    sig = {
        "ccl_label": (st, [i64, i64, P, P, P, P, P]),
        "ccl_label_philox": (st, [i64, i64, P, P, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, P, P]),
        "ccl_label_csr_workspace_size": (sz, [i64, i64]),
        "ccl_label_csr": (st, [i64, i64, P, P, P, P, P, sz, P]),
        "ccl_label_csr_philox": (st, [i64, i64, P, P, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double,
                                      P, P, sz, P]),
        "ccl_label_csr_grid": (st, [i64, i64, i64, P, P, P, P, P, sz, P]),
        "ccl_label_csr_grid_philox": (st, [i64, i64, i64, P, P, ctypes.c_uint64, ctypes.c_uint32,
                                           ctypes.c_double, P, P, sz, P]),
        "ccl_label_ell": (st, [i64, i32, P, P, P, P]),
        "ccl_philox_u32": (st, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, i64, P, P]),
        "ccl_bernoulli": (st, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, i64, ctypes.c_double,
                               P, P]),
        "ccl_cluster_ids_workspace_size": (sz, [i64]),
        "ccl_cluster_ids": (st, [i64, P, P, P, P, sz, P]),
        "ccl_cluster_ids_noalloc_max_sites": (sz, []),
        "ccl_cluster_ids_noalloc": (st, [i64, P, P, P, P]),
        "ccl_cluster_sizes": (st, [i64, P, P, P]),
        "ccl_cluster_size_histogram": (st, [i64, P, i64, P, P]),
        "ccl_spans": (st, [i64, P, i64, P, i64, P, P, P, P]),
        "ccl_plan_create": (st, [i32, P, P, P, P]),
        "ccl_plan_destroy": (st, [P]),
        "ccl_plan_create_capacity": (st, [i32, i64, i64, P, P]),
        "ccl_plan_set_layout": (st, [P, i32, P, P, P]),
        "ccl_plan_get_tuning": (st, [P, P]),
        "ccl_plan_check": (st, [P, P]),
        "ccl_label_batched": (st, [P, P, P, P, P, P]),
        "ccl_label_batched_per_instance": (st, [i32, P, P, P, P, P, P, P]),
        "ccl_validate_edges": (st, [i64, i64, P, P, P, P]),
        "ccl_validate_csr": (st, [i64, P, P, i64, P, P]),
        "ccl_status_string": (ctypes.c_char_p, [st]),
        "ccl_last_hip_error": (ctypes.c_int, []),
        "ccl_version": (ctypes.c_int, []),
        "ccl_trace_enable": (st, [ctypes.c_int]),
        "ccl_trace_count": (ctypes.c_int, []),
        "ccl_trace_get": (st, [ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                               ctypes.POINTER(ctypes.c_float)]),
        "ccl_probe_copy": (st, [P, P, sz, P]),
        "ccl_probe_random": (st, [P, i64, i64, i32, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def version() -> int:
    return _lib.ccl_version()


def _check(status: int, where: str):
    if status != CCL_OK:
        raise CclError(status, where)


def _dev_ptr(t, dtype, name, n=None, device=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return ctypes.c_void_p(t.data_ptr()) if t.numel() else None


def _stream(stream, device):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def label(src: torch.Tensor, dst: torch.Tensor, n_sites: int, occ: torch.Tensor | None = None,
          out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Min-site-index cluster labels of an edge list (int32 GPU tensors)."""
    dev = src.device
    m = src.numel()
    ps = _dev_ptr(src, torch.int32, "src", None, dev)
    pd = _dev_ptr(dst, torch.int32, "dst", m, dev)
    po = _dev_ptr(occ, torch.uint8, "occ", m, dev)
    if out is None:
        out = torch.empty(n_sites, dtype=torch.int32, device=dev)
    pl = _dev_ptr(out, torch.int32, "out", n_sites, dev)
    with torch.cuda.device(dev):
        _check(_lib.ccl_label(n_sites, m, ps, pd, po, pl, _stream(stream, dev)), "ccl_label")
    return out


def label_philox(src: torch.Tensor, dst: torch.Tensor, n_sites: int, seed: int, stream_id: int, p: float,
                 out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """label with bond b occupied when word b of the Philox stream
    (seed, stream_id) is below floor(p 2^32), drawn inside the merge kernel:
    the labels of label(src, dst, n_sites, bernoulli(seed, stream_id, len(src), p))."""
    dev = src.device
    m = src.numel()
    ps = _dev_ptr(src, torch.int32, "src", None, dev)
    pd = _dev_ptr(dst, torch.int32, "dst", m, dev)
    if out is None:
        out = torch.empty(n_sites, dtype=torch.int32, device=dev)
    pl = _dev_ptr(out, torch.int32, "out", n_sites, dev)
    with torch.cuda.device(dev):
        _check(_lib.ccl_label_philox(n_sites, m, ps, pd, seed, stream_id, float(p), pl, _stream(stream, dev)),
               "ccl_label_philox")
    return out


def label_ell(nn: torch.Tensor, occ: torch.Tensor | None = None, out: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
    """Min-site-index cluster labels from the paper's padded neighbour list:
    `nn` is int32 of shape (z_max, n_sites), row k holding neighbour k of
    every site (the column-major list, entries outside [0, n_sites) are
    padding); `occ` is uint8 of the same shape or None (all occupied)."""
    if nn.dim() != 2:
        raise ValueError("nn must have shape (z_max, n_sites)")
    dev = nn.device
    z, n = nn.shape
    pn = _dev_ptr(nn, torch.int32, "nn", None, dev)
    po = _dev_ptr(occ, torch.uint8, "occ", nn.numel(), dev)
    if occ is not None and occ.shape != nn.shape:
        raise ValueError("occ must have the shape of nn")
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=dev)
    pl = _dev_ptr(out, torch.int32, "out", n, dev)
    with torch.cuda.device(dev):
        _check(_lib.ccl_label_ell(n, z, pn, po, pl, _stream(stream, dev)), "ccl_label_ell")
    return out


def philox_u32(seed: int, stream_id: int, n: int, first: int = 0, out: torch.Tensor | None = None,
               device=None, stream=None) -> torch.Tensor:
    """Words first .. first+n-1 of Philox4x32-10 stream `stream_id` under
    `seed`, drawn on the GPU (int32 tensor holding the uint32 bits)."""
    dev = torch.device(device) if device is not None else (out.device if out is not None
                                                          else torch.device("cuda", torch.cuda.current_device()))
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=dev)
    po = _dev_ptr(out, torch.int32, "out", n, dev)
    with torch.cuda.device(dev):
        _check(_lib.ccl_philox_u32(seed, stream_id, first, n, po, _stream(stream, dev)), "ccl_philox_u32")
    return out


def bernoulli(seed: int, stream_id: int, n: int, p: float, first: int = 0,
              out: torch.Tensor | None = None, device=None, stream=None) -> torch.Tensor:
    """Bond occupancy drawn on the GPU: out[i] = 1 when word first+i of the
    Philox stream is below floor(p 2^32) (uint8 tensor)."""
    dev = torch.device(device) if device is not None else (out.device if out is not None
                                                          else torch.device("cuda", torch.cuda.current_device()))
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=dev)
    po = _dev_ptr(out, torch.uint8, "out", n, dev)
    with torch.cuda.device(dev):
        _check(_lib.ccl_bernoulli(seed, stream_id, first, n, float(p), po, _stream(stream, dev)),
               "ccl_bernoulli")
    return out


def cluster_ids(labels: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """Sequential cluster ids of a finished labeling (the k-th smallest
    cluster minimum gets id k) and the number of clusters, a 1-element int32
    GPU tensor (read it when the stream is done)."""
    dev = labels.device
    n = labels.numel()
    pl = _dev_ptr(labels, torch.int32, "labels", None, dev)
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=dev)
    po = _dev_ptr(out, torch.int32, "out", n, dev)
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty(max(int(_lib.ccl_cluster_ids_workspace_size(n)), 4), dtype=torch.uint8, device=dev)
    with torch.cuda.device(dev):
        _check(_lib.ccl_cluster_ids(n, pl, po, _dev_ptr(count, torch.int32, "count"),
                                    _dev_ptr(ws, torch.uint8, "ws"), ws.numel(), _stream(stream, dev)),
               "ccl_cluster_ids")
    return out, count


def cluster_ids_noalloc(labels: torch.Tensor, out: torch.Tensor, count: torch.Tensor, stream=None):
    """cluster_ids into caller-provided `out` (int32, like labels) and `count`
    (1-element int32) through ccl_cluster_ids_noalloc: no device memory is
    allocated, by the library or here, so the call can be captured in a HIP
    graph.  Calls that overlap on one device race (they share the library's
    fixed workspace)."""
    dev = labels.device
    n = labels.numel()
    pl = _dev_ptr(labels, torch.int32, "labels", None, dev)
    po = _dev_ptr(out, torch.int32, "out", n, dev)
    pc = _dev_ptr(count, torch.int32, "count", 1, dev)
    with torch.cuda.device(dev):
        _check(_lib.ccl_cluster_ids_noalloc(n, pl, po, pc, _stream(stream, dev)), "ccl_cluster_ids_noalloc")
    return out, count


def cluster_sizes(labels: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """sizes[r] = number of sites labelled r (zero unless r is a cluster minimum)."""
    dev = labels.device
    n = labels.numel()
    pl = _dev_ptr(labels, torch.int32, "labels", None, dev)
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=dev)
    po = _dev_ptr(out, torch.int32, "out", n, dev)
    with torch.cuda.device(dev):
        _check(_lib.ccl_cluster_sizes(n, pl, po, _stream(stream, dev)), "ccl_cluster_sizes")
    return out


def size_histogram(sizes: torch.Tensor, n_bins: int, out: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
    """n_s from cluster_sizes' output: out[s] = number of clusters of s sites
    (int64; the last bin holds every cluster of n_bins - 1 sites or more)."""
    dev = sizes.device
    n = sizes.numel()
    ps = _dev_ptr(sizes, torch.int32, "sizes", None, dev)
    if out is None:
        out = torch.empty(n_bins, dtype=torch.int64, device=dev)
    po = _dev_ptr(out, torch.int64, "out", n_bins, dev)
    with torch.cuda.device(dev):
        _check(_lib.ccl_cluster_size_histogram(n, ps, n_bins, po, _stream(stream, dev)),
               "ccl_cluster_size_histogram")
    return out


def spans(labels: torch.Tensor, sites_a: torch.Tensor, sites_b: torch.Tensor, stream=None) -> torch.Tensor:
    """1-element int32 GPU tensor: 1 when one cluster holds a site of sites_a
    and one of sites_b (the spanning test of section 4)."""
    dev = labels.device
    n = labels.numel()
    pl = _dev_ptr(labels, torch.int32, "labels", None, dev)
    pa = _dev_ptr(sites_a, torch.int32, "sites_a", None, dev)
    pb = _dev_ptr(sites_b, torch.int32, "sites_b", None, dev)
    flags = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
    res = torch.empty(1, dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        _check(_lib.ccl_spans(n, pl, sites_a.numel(), pa, sites_b.numel(), pb,
                              _dev_ptr(flags, torch.uint8, "flags"), _dev_ptr(res, torch.int32, "res"),
                              _stream(stream, dev)), "ccl_spans")
    return res


def csr_workspace_bytes(n_sites: int, n_bonds: int) -> int:
    """Workspace ccl_label_csr needs (0 for a graph of one 65536-site tile)."""
    return int(_lib.ccl_label_csr_workspace_size(n_sites, n_bonds))


def _csr_args(row_ptr, col, out, workspace):
    dev = row_ptr.device
    n = row_ptr.numel() - 1
    if n < 0:
        raise ValueError("row_ptr must hold n_sites + 1 entries")
    m = col.numel()
    prp = _dev_ptr(row_ptr, torch.int32, "row_ptr", None, dev)
    pc = _dev_ptr(col, torch.int32, "col", None, dev)
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=dev)
    pl = _dev_ptr(out, torch.int32, "out", n, dev)
    need = csr_workspace_bytes(n, m)
    if workspace is None and need > 0:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    pw = _dev_ptr(workspace, torch.uint8, "workspace", None, dev)
    wbytes = workspace.numel() if workspace is not None else 0
    return dev, n, m, prp, pc, out, pl, pw, wbytes


def label_csr(row_ptr: torch.Tensor, col: torch.Tensor, occ: torch.Tensor | None = None,
              out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
              stream=None, grid_width: int = 0) -> torch.Tensor:
    """Min-site-index cluster labels of a CSR graph; n_sites = len(row_ptr) - 1,
    bonds row_ptr[0] .. row_ptr[n]-1 of col (len(col) bounds their count).
    `workspace` (uint8, >= csr_workspace_bytes(n, len(col)) bytes) is
    allocated when None.  `grid_width` > 0: the ids number a grid of that row
    length row by row, and the tiles follow it (ccl_label_csr_grid); the
    labels are the same for any value."""
    dev, n, m, prp, pc, out, pl, pw, wbytes = _csr_args(row_ptr, col, out, workspace)
    po = _dev_ptr(occ, torch.uint8, "occ", m, dev)
    with torch.cuda.device(dev):
        if grid_width:
            _check(_lib.ccl_label_csr_grid(n, m, int(grid_width), prp, pc, po, pl, pw, wbytes,
                                           _stream(stream, dev)), "ccl_label_csr_grid")
        else:
            _check(_lib.ccl_label_csr(n, m, prp, pc, po, pl, pw, wbytes, _stream(stream, dev)),
                   "ccl_label_csr")
    return out


def label_csr_philox(row_ptr: torch.Tensor, col: torch.Tensor, seed: int, stream_id: int, p: float,
                     out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                     stream=None, grid_width: int = 0) -> torch.Tensor:
    """label_csr with bond e occupied when word e of the Philox stream
    (seed, stream_id) is below floor(p 2^32), drawn inside the kernel: the
    labels of label_csr(row_ptr, col, bernoulli(seed, stream_id, len(col), p))."""
    dev, n, m, prp, pc, out, pl, pw, wbytes = _csr_args(row_ptr, col, out, workspace)
    with torch.cuda.device(dev):
        if grid_width:
            _check(_lib.ccl_label_csr_grid_philox(n, m, int(grid_width), prp, pc, seed, stream_id, float(p),
                                                  pl, pw, wbytes, _stream(stream, dev)),
                   "ccl_label_csr_grid_philox")
        else:
            _check(_lib.ccl_label_csr_philox(n, m, prp, pc, seed, stream_id, float(p), pl, pw, wbytes,
                                             _stream(stream, dev)), "ccl_label_csr_philox")
    return out


def _host_i64(a):
    a = np.ascontiguousarray(np.asarray(a.cpu() if isinstance(a, torch.Tensor) else a),
                             dtype=np.int64)
    return a, ctypes.c_void_p(a.ctypes.data)


class Plan:
    """A batched-labeling plan for one layout of instances (ccl_plan)."""

    def __init__(self, site_off, bond_off, tuning: Tuning | dict | None = None, device=None):
        so, pso = _host_i64(site_off)
        bo, pbo = _host_i64(bond_off)
        if so.shape != bo.shape or so.ndim != 1 or len(so) < 1:
            raise ValueError("site_off and bond_off must be 1-D with K+1 entries")
        if isinstance(tuning, dict):
            tuning = Tuning(**tuning)
        d = torch.device(device) if device is not None else torch.device("cuda")
        self.device = d if d.index is not None else torch.device("cuda", torch.cuda.current_device())
        self.n_inst = len(so) - 1
        self.total_sites = int(so[-1])
        self.total_bonds = int(bo[-1])
        self._site_off, self._bond_off = so, bo
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.ccl_plan_create(self.n_inst, pso, pbo,
                                        ctypes.byref(tuning) if tuning is not None else None,
                                        ctypes.byref(self._h)), "ccl_plan_create")

    @classmethod
    def with_capacity(cls, max_inst: int, max_sites: int, max_bonds: int,
                      tuning: Tuning | dict | None = None, device=None) -> "Plan":
        """A plan for many layouts (ccl_plan_create_capacity): give it each
        launch's layout with set_layout."""
        if isinstance(tuning, dict):
            tuning = Tuning(**tuning)
        self = cls.__new__(cls)
        d = torch.device(device) if device is not None else torch.device("cuda")
        self.device = d if d.index is not None else torch.device("cuda", torch.cuda.current_device())
        self.n_inst, self.total_sites, self.total_bonds = 0, 0, 0
        self._site_off = self._bond_off = np.zeros(1, np.int64)
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib.ccl_plan_create_capacity(int(max_inst), int(max_sites), int(max_bonds),
                                                 ctypes.byref(tuning) if tuning is not None else None,
                                                 ctypes.byref(self._h)), "ccl_plan_create_capacity")
        return self

    def set_layout(self, site_off, bond_off, stream=None) -> None:
        """The layout of the next launches of a capacity plan
        (ccl_plan_set_layout), uploaded on `stream`."""
        so, pso = _host_i64(site_off)
        bo, pbo = _host_i64(bond_off)
        if so.shape != bo.shape or so.ndim != 1 or len(so) < 1:
            raise ValueError("site_off and bond_off must be 1-D with K+1 entries")
        with torch.cuda.device(self.device):
            _check(_lib.ccl_plan_set_layout(self._h, len(so) - 1, pso, pbo, _stream(stream, self.device)),
                   "ccl_plan_set_layout")
        self.n_inst, self.total_sites, self.total_bonds = len(so) - 1, int(so[-1]), int(bo[-1])
        self._site_off, self._bond_off = so, bo

    @property
    def tuning(self) -> Tuning:
        t = Tuning()
        _check(_lib.ccl_plan_get_tuning(self._h, ctypes.byref(t)), "ccl_plan_get_tuning")
        return t

    def label(self, src, dst, occ=None, out=None, stream=None) -> torch.Tensor:
        dev = self.device
        ps = _dev_ptr(src, torch.int32, "src", self.total_bonds, dev)
        pd = _dev_ptr(dst, torch.int32, "dst", self.total_bonds, dev)
        po = _dev_ptr(occ, torch.uint8, "occ", self.total_bonds, dev)
        if out is None:
            out = torch.empty(self.total_sites, dtype=torch.int32, device=dev)
        pl = _dev_ptr(out, torch.int32, "out", self.total_sites, dev)
        with torch.cuda.device(dev):
            _check(_lib.ccl_label_batched(self._h, ps, pd, po, pl, _stream(stream, dev)),
                   "ccl_label_batched")
        return out

    def check(self) -> int:
        """Nonzero when a work item of the last launch gave up waiting."""
        v = ctypes.c_int32()
        with torch.cuda.device(self.device):
            _check(_lib.ccl_plan_check(self._h, ctypes.byref(v)), "ccl_plan_check")
        return v.value

    def close(self):
        if getattr(self, "_h", None):
            with torch.cuda.device(self.device):
                _lib.ccl_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def label_batched_per_instance(site_off, bond_off, src, dst, occ=None, out=None, stream=None):
    """One ccl_label call per instance (the baseline schedule)."""
    so, pso = _host_i64(site_off)
    bo, pbo = _host_i64(bond_off)
    dev = src.device
    ps = _dev_ptr(src, torch.int32, "src", int(bo[-1]), dev)
    pd = _dev_ptr(dst, torch.int32, "dst", int(bo[-1]), dev)
    po = _dev_ptr(occ, torch.uint8, "occ", int(bo[-1]), dev)
    if out is None:
        out = torch.empty(int(so[-1]), dtype=torch.int32, device=dev)
    pl = _dev_ptr(out, torch.int32, "out", int(so[-1]), dev)
    with torch.cuda.device(dev):
        _check(_lib.ccl_label_batched_per_instance(len(so) - 1, pso, pbo, ps, pd, po, pl,
                                                   _stream(stream, dev)),
               "ccl_label_batched_per_instance")
    return out


def validate_edges(src, dst, n_sites: int, stream=None) -> int:
    """Number of bonds with an end outside [0, n_sites) (synchronous)."""
    dev = src.device
    bad = ctypes.c_int64()
    st = _lib.ccl_validate_edges(n_sites, src.numel(), _dev_ptr(src, torch.int32, "src", None, dev),
                                 _dev_ptr(dst, torch.int32, "dst", src.numel(), dev),
                                 ctypes.byref(bad), _stream(stream, dev))
    if st not in (CCL_OK, CCL_ERR_INDEX_OUT_OF_RANGE):
        _check(st, "ccl_validate_edges")
    return bad.value


def validate_csr(row_ptr, col, stream=None) -> int:
    dev = row_ptr.device
    bad = ctypes.c_int64()
    st = _lib.ccl_validate_csr(row_ptr.numel() - 1, _dev_ptr(row_ptr, torch.int32, "row_ptr", None, dev),
                               _dev_ptr(col, torch.int32, "col", None, dev), col.numel(),
                               ctypes.byref(bad), _stream(stream, dev))
    if st not in (CCL_OK, CCL_ERR_INDEX_OUT_OF_RANGE):
        _check(st, "ccl_validate_csr")
    return bad.value


@contextlib.contextmanager
def trace():
    """Per-kernel durations of every library launch inside the block:
    ``with trace() as rec: ...`` then ``rec`` holds (kernel, ms) pairs."""
    rec = []
    _check(_lib.ccl_trace_enable(1), "ccl_trace_enable")
    try:
        yield rec
    finally:
        n = _lib.ccl_trace_count()
        name, ms = ctypes.c_char_p(), ctypes.c_float()
        for i in range(max(n, 0)):
            _check(_lib.ccl_trace_get(i, ctypes.byref(name), ctypes.byref(ms)), "ccl_trace_get")
            rec.append((name.value.decode(), float(ms.value)))
        _lib.ccl_trace_enable(0)


def probe_copy(src: torch.Tensor, dst: torch.Tensor, stream=None):
    """Plain streaming copy (traffic-counter calibration)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() >= nbytes
    _check(_lib.ccl_probe_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                               nbytes, _stream(stream, src.device)), "ccl_probe_copy")


def probe_random(table: torch.Tensor, n_ops: int, mode: int, stream=None):
    """ccl_probe_random on an int32 GPU table (mode 0 gather, 1 atomicMin
    discarded, 2 atomicMin used, 3 dependent chase, 4 fill for mode 3)."""
    pt = _dev_ptr(table, torch.int32, "table", None, table.device)
    sink = torch.zeros(1, dtype=torch.int32, device=table.device)
    with torch.cuda.device(table.device):
        _check(_lib.ccl_probe_random(pt, table.numel(), int(n_ops), int(mode),
                                     ctypes.c_void_p(sink.data_ptr()), _stream(stream, table.device)),
               "ccl_probe_random")
