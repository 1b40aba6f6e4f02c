"""The C-ABI library loads on a machine without a GPU, exports every function
include/ccl.h declares, and rejects bad arguments on the host before any HIP
call (no compute call runs here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccl.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(ccl_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1603_08357_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    import paper_1603_08357_amd as ccl
    return ccl._lib


def test_header_parses():
    names = declared_functions()
    for must in ("ccl_label", "ccl_label_csr", "ccl_label_batched", "ccl_plan_create",
                 "ccl_validate_edges", "ccl_status_string"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1603_08357_amd import library_path
    out = subprocess.run(["nm", "-D", "--defined-only", library_path], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        getattr(lib, n)


def test_header_compiles_as_plain_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "ccl.h"\nint main(void){return ccl_version()>0?0:1;}\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    "-c", str(src), "-o", str(tmp_path / "t.o")], check=True)


def test_status_strings(lib):
    for code in range(7):
        assert lib.ccl_status_string(code).startswith(b"CCL_")
    assert lib.ccl_version() == 100


def test_host_side_argument_errors(lib):
    INVALID = 1
    assert lib.ccl_label(-1, 0, None, None, None, None, None) == INVALID
    assert lib.ccl_label(2**31, 0, None, None, None, None, None) == INVALID
    assert lib.ccl_label(5, 3, None, None, None, ctypes.c_void_p(64), None) == INVALID
    assert lib.ccl_label(5, 0, None, None, None, None, None) == INVALID  # labels NULL
    assert lib.ccl_label(0, 0, None, None, None, None, None) == 0  # nothing to do
    # bonds but no sites: no valid id exists
    assert lib.ccl_label(0, 2, ctypes.c_void_p(64), ctypes.c_void_p(128), None,
                         ctypes.c_void_p(256), None) == INVALID
    # labels overlapping src
    assert lib.ccl_label(10, 10, ctypes.c_void_p(4096), ctypes.c_void_p(8192), None,
                         ctypes.c_void_p(4096 + 8), None) == INVALID
    # CSR: > one tile needs a workspace of the right size and alignment
    n, m = 100_000, 300_000
    n_tiles = (n + 65535) // 65536
    assert lib.ccl_label_csr_workspace_size(n, m) == (n_tiles * 8 + 255) // 256 * 256 + 8 * m
    assert lib.ccl_label_csr_workspace_size(65536, 10**6) == 0  # one tile: none
    assert lib.ccl_label_csr_workspace_size(65537, 0) > 0
    assert lib.ccl_label_csr_workspace_size(0, 0) == 0
    need = lib.ccl_label_csr_workspace_size(n, m)
    args = (n, m, ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 24), None, ctypes.c_void_p(1 << 28))
    assert lib.ccl_label_csr(*args, None, 0, None) == INVALID
    assert lib.ccl_label_csr(*args, ctypes.c_void_p(1 << 33), need - 8, None) == INVALID
    assert lib.ccl_label_csr(*args, ctypes.c_void_p((1 << 33) + 4), need, None) == INVALID
    assert lib.ccl_label_csr(-3, 0, None, None, None, None, None, 0, None) == INVALID
    assert lib.ccl_label_csr(5, -1, None, None, None, None, None, 0, None) == INVALID
    assert lib.ccl_label_csr(0, 0, None, None, None, None, None, 0, None) == 0


def test_plan_argument_errors(lib):
    INVALID = 1
    plan = ctypes.c_void_p()
    so = (ctypes.c_int64 * 3)(0, 10, 5)  # decreasing
    bo = (ctypes.c_int64 * 3)(0, 4, 8)
    assert lib.ccl_plan_create(2, so, bo, None, ctypes.byref(plan)) == INVALID
    so = (ctypes.c_int64 * 3)(1, 10, 20)  # does not start at 0
    assert lib.ccl_plan_create(2, so, bo, None, ctypes.byref(plan)) == INVALID
    assert lib.ccl_plan_create(-1, so, bo, None, ctypes.byref(plan)) == INVALID
    assert lib.ccl_plan_create(1, None, None, None, ctypes.byref(plan)) == INVALID
    assert lib.ccl_label_batched(None, None, None, None, None, None) == INVALID
    assert lib.ccl_plan_destroy(None) == 0
    # capacity plans: negative limits and a missing plan are refused on the host
    lib.ccl_plan_create_capacity.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.c_void_p, ctypes.c_void_p]
    lib.ccl_plan_set_layout.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]
    assert lib.ccl_plan_create_capacity(-1, 10, 10, None, ctypes.byref(plan)) == INVALID
    assert lib.ccl_plan_create_capacity(4, -1, 10, None, ctypes.byref(plan)) == INVALID
    assert lib.ccl_plan_create_capacity(4, 10, 10, None, None) == INVALID
    assert lib.ccl_plan_set_layout(None, 2, so, bo, None) == INVALID


def test_probe_argument_errors(lib):
    INVALID = 1
    P = ctypes.c_void_p
    lib.ccl_probe_random.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, P, P]
    assert lib.ccl_probe_random(None, 16, 16, 0, P(64), None) == INVALID
    assert lib.ccl_probe_random(P(64), 0, 16, 0, P(128), None) == INVALID
    assert lib.ccl_probe_random(P(64), 1 << 31, 16, 0, P(128), None) == INVALID
    assert lib.ccl_probe_random(P(64), 16, -1, 0, P(128), None) == INVALID
    assert lib.ccl_probe_random(P(64), 16, 16, 5, P(128), None) == INVALID
    assert lib.ccl_probe_random(P(64), 16, 16, 0, None, None) == INVALID


def test_validation_argument_errors(lib):
    INVALID = 1
    bad = ctypes.c_int64()
    assert lib.ccl_validate_edges(-1, 0, None, None, ctypes.byref(bad), None) == INVALID
    assert lib.ccl_validate_edges(5, 3, None, None, ctypes.byref(bad), None) == INVALID
    assert lib.ccl_validate_edges(5, 0, None, None, ctypes.byref(bad), None) == 0
    assert bad.value == 0
    assert lib.ccl_validate_csr(5, None, None, 0, ctypes.byref(bad), None) == INVALID


def test_more_host_side_argument_errors(lib):
    """The neighbour-list path, the statistics and the device generator
    reject bad arguments on the host."""
    INVALID = 1
    P = ctypes.c_void_p
    # ccl_label_ell: negative sizes, missing pointers, oversized list, aliasing
    assert lib.ccl_label_ell(-1, 3, P(64), None, P(4096), None) == INVALID
    assert lib.ccl_label_ell(10, -1, P(64), None, P(4096), None) == INVALID
    assert lib.ccl_label_ell(10, 3, None, None, P(4096), None) == INVALID
    assert lib.ccl_label_ell(10, 3, P(64), None, None, None) == INVALID
    assert lib.ccl_label_ell(1 << 30, 1 << 11, P(64), None, P(1 << 40), None) == INVALID
    assert lib.ccl_label_ell(10, 3, P(4096), None, P(4096 + 8), None) == INVALID
    assert lib.ccl_label_ell(0, 3, None, None, None, None) == 0
    # ccl_cluster_ids: workspace size and alignment, aliasing
    n = 10_000
    need = lib.ccl_cluster_ids_workspace_size(n)
    assert need == 4 * ((n + 4095) // 4096) and lib.ccl_cluster_ids_workspace_size(0) == 0
    lab, ids, cnt, ws = P(1 << 20), P(1 << 24), P(1 << 28), P(1 << 32)
    assert lib.ccl_cluster_ids(n, lab, ids, cnt, ws, need - 4, None) == INVALID
    assert lib.ccl_cluster_ids(n, lab, ids, cnt, P((1 << 32) + 2), need, None) == INVALID
    assert lib.ccl_cluster_ids(n, lab, lab, cnt, ws, need, None) == INVALID
    assert lib.ccl_cluster_ids(n, lab, ids, None, ws, need, None) == INVALID
    assert lib.ccl_cluster_ids(-1, lab, ids, cnt, ws, need, None) == INVALID
    # ccl_cluster_sizes / ccl_spans
    assert lib.ccl_cluster_sizes(n, lab, lab, None) == INVALID
    assert lib.ccl_cluster_sizes(n, None, ids, None) == INVALID
    assert lib.ccl_spans(n, lab, 4, None, 4, P(64), P(1 << 36), P(1 << 38), None) == INVALID
    assert lib.ccl_spans(n, lab, -1, P(64), 4, P(64), P(1 << 36), P(1 << 38), None) == INVALID
    assert lib.ccl_spans(n, lab, 4, P(64), 4, P(64), P(1 << 36), None, None) == INVALID
    assert lib.ccl_spans(0, None, 1, P(64), 1, P(64), None, P(1 << 38), None) == INVALID
    # device generator: size overflow, missing output, NaN probability
    assert lib.ccl_philox_u32(1, 0, 2**64 - 2, 10, P(64), None) == INVALID
    assert lib.ccl_philox_u32(1, 0, 0, 10, None, None) == INVALID
    assert lib.ccl_philox_u32(1, 0, 0, -1, P(64), None) == INVALID
    assert lib.ccl_philox_u32(1, 0, 0, 0, None, None) == 0
    assert lib.ccl_bernoulli(1, 0, 0, 10, float("nan"), P(64), None) == INVALID
    assert lib.ccl_bernoulli(1, 0, 0, 10, 0.5, None, None) == INVALID
    # ccl_label_philox: NaN probability, then ccl_label's own checks
    assert lib.ccl_label_philox(10, 5, P(64), P(128), 1, 0, float("nan"), P(4096), None) == INVALID
    assert lib.ccl_label_philox(-1, 5, P(64), P(128), 1, 0, 0.5, P(4096), None) == INVALID
    assert lib.ccl_label_philox(10, 5, None, P(128), 1, 0, 0.5, P(4096), None) == INVALID
    assert lib.ccl_label_philox(10, 5, P(4096), P(128), 1, 0, 0.5, P(4096 + 8), None) == INVALID
    assert lib.ccl_label_philox(0, 0, None, None, 1, 0, 0.5, None, None) == 0
    # ccl_label_csr_philox: NaN probability, then ccl_label_csr's own checks
    rp, col, lab = P(1 << 20), P(1 << 24), P(1 << 28)
    assert lib.ccl_label_csr_philox(10, 30, rp, col, 1, 0, float("nan"), lab, None, 0, None) == INVALID
    assert lib.ccl_label_csr_philox(-1, 30, rp, col, 1, 0, 0.5, lab, None, 0, None) == INVALID
    assert lib.ccl_label_csr_philox(10, 30, None, col, 1, 0, 0.5, lab, None, 0, None) == INVALID
    assert lib.ccl_label_csr_philox(10, 30, rp, col, 1, 0, 0.5, rp, None, 0, None) == INVALID
    assert lib.ccl_label_csr_philox(1 << 20, 1 << 22, rp, col, 1, 0, 0.5, lab, None, 0, None) == INVALID
    assert lib.ccl_label_csr_philox(0, 0, None, None, 1, 0, 0.5, None, None, 0, None) == 0
