"""ccl_cluster_ids_noalloc (the entry point that allocates no device memory,
its workspace in the library's fixed device array) against ccl_cluster_ids
(caller workspace) through the C ABI: two calls in a row on one device, the
second smaller, so the second runs on the array the first left behind."""
import ctypes
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CCL_ERR_INVALID_VALUE = 1
CCL_ERR_TOO_LARGE = 6


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ccl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1603_08357_amd as lib
    return lib


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _ids_with_workspace(lib, labels, stream):
    n = labels.numel()
    ids = torch.full((n,), -3, dtype=torch.int32, device="cuda")
    count = torch.full((1,), -3, dtype=torch.int32, device="cuda")
    wsb = int(lib.ccl_cluster_ids_workspace_size(n))
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    st = lib.ccl_cluster_ids(n, _p(labels), _p(ids), _p(count), _p(ws), wsb, ctypes.c_void_p(stream.cuda_stream))
    assert st == 0, st
    return ids, count


def _ids_noalloc(lib, labels, stream):
    n = labels.numel()
    ids = torch.full((n,), -3, dtype=torch.int32, device="cuda")
    count = torch.full((1,), -3, dtype=torch.int32, device="cuda")
    st = lib.ccl_cluster_ids_noalloc(n, _p(labels), _p(ids), _p(count), ctypes.c_void_p(stream.cuda_stream))
    assert st == 0, st
    return ids, count


def test_noalloc_matches_workspace_entry_point(ccl):
    lib = ccl._lib
    assert lib.ccl_cluster_ids_noalloc_max_sites() == 2**31 - 1
    stream = torch.cuda.current_stream()
    # two labelings: 1,002,001 sites (ragged against the 4096-site spans), then 5,000
    big = gen.triangle_csr_realization(1001, 0.3473, 71)
    lab_big = oracle.label_csr(big.n_sites, big.row_ptr, big.col, big.occ)
    small = gen.bethe_random_regular(5000, 3, 0.45, 72)
    lab_small = oracle.label_edges(small.n_sites, small.src, small.dst, small.occ)
    for name, lab in (("1002001 sites", lab_big), ("5000 sites", lab_small)):
        _say(f"ccl_cluster_ids_noalloc {name}")
        d = torch.from_numpy(lab).cuda()
        want_ids, want_count = _ids_with_workspace(lib, d, stream)
        got_ids, got_count = _ids_noalloc(lib, d, stream)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got_ids.cpu().numpy(), want_ids.cpu().numpy())
        assert int(got_count.item()) == int(want_count.item())
        ids_o, count_o = oracle.cluster_ids(lab)
        np.testing.assert_array_equal(got_ids.cpu().numpy(), ids_o)
        assert int(got_count.item()) == count_o


def test_noalloc_host_side_errors(ccl):
    lib = ccl._lib
    null = ctypes.c_void_p(0)
    x = torch.zeros(4, dtype=torch.int32, device="cuda")
    assert lib.ccl_cluster_ids_noalloc(2**31, _p(x), _p(x), _p(x), null) == CCL_ERR_TOO_LARGE
    assert lib.ccl_cluster_ids_noalloc(-1, _p(x), _p(x), _p(x), null) == CCL_ERR_INVALID_VALUE
    assert lib.ccl_cluster_ids_noalloc(4, null, _p(x), _p(x), null) == CCL_ERR_INVALID_VALUE
    assert lib.ccl_cluster_ids_noalloc(0, null, null, null, null) == 0
