"""GPU parity: labels from libccl.so (through the C ABI) must equal the CPU
oracle's bit for bit -- the labeling is integer and its result unique (each
cluster labelled by its minimum site number), so no tolerance applies."""
import itertools
import sys

import numpy as np
import pytest

import gen
import oracle
from conftest import read_golden
from test_oracle import check_invariants, load_cases

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ccl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1603_08357_amd as lib
    return lib


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_edges(ccl, n, src, dst, occ=None):
    _say(f"ccl_label n={n} m={len(src)} occ={'none' if occ is None else 'mask'}")
    out = ccl.label(dev(src), dev(dst), n, None if occ is None else dev(occ))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def gpu_csr(ccl, row_ptr, col, occ=None, grid_width=0):
    _say(f"ccl_label_csr n={len(row_ptr) - 1} m={len(col)} grid_width={grid_width}")
    out = ccl.label_csr(dev(row_ptr), dev(col), None if occ is None else dev(occ), grid_width=grid_width)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def gpu_ell(ccl, nn, occ=None):
    _say(f"ccl_label_ell n={nn.shape[1]} z_max={nn.shape[0]}")
    out = ccl.label_ell(dev(nn), None if occ is None else dev(occ))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def oracle_ell(nn, occ=None):
    z, n = nn.shape
    return oracle.label_ell(n, z, nn.ravel(), None if occ is None else occ.ravel())


# ------------------------------------------------------------ small graphs

@pytest.mark.parametrize("case", load_cases(), ids=lambda c: c["name"])
def test_hand_worked_cases(ccl, case):
    b = case["bonds"]
    src = np.array([x[0] for x in b], np.int32)
    dst = np.array([x[1] for x in b], np.int32)
    occ = np.array([x[2] for x in b], np.uint8)
    assert gpu_edges(ccl, case["n"], src, dst, occ).tolist() == case["expect"]


def test_exhaustive_k5(ccl):
    pairs = list(itertools.combinations(range(5), 2))
    s = np.array([p[0] for p in pairs], np.int32)
    d = np.array([p[1] for p in pairs], np.int32)
    ds, dd = dev(s), dev(d)
    _say("exhaustive K5 (1024 masks)")
    for mask in range(1 << len(pairs)):
        occ = np.array([(mask >> j) & 1 for j in range(len(pairs))], np.uint8)
        got = ccl.label(ds if mask & 1 else dd, dd if mask & 1 else ds, 5, dev(occ)).cpu().numpy()
        want = oracle.label_edges(5, s, d, occ)
        assert got.tolist() == want.tolist(), mask


@pytest.mark.parametrize("n,m,seed", [(1, 0, 0), (1, 5, 1), (2, 1, 2), (7, 3, 3), (63, 40, 4),
                                      (65, 200, 5), (1000, 999, 6), (4099, 6000, 7),
                                      (100_003, 150_001, 8), (1_000_001, 700_001, 9)])
def test_random_multigraphs(ccl, n, m, seed):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    occ = (rng.random(m) < 0.6).astype(np.uint8)
    got = gpu_edges(ccl, n, src, dst, occ)
    np.testing.assert_array_equal(got, oracle.label_edges(n, src, dst, occ))
    check_invariants(got, n, src, dst, occ)


def test_empty_and_degenerate(ccl):
    e = np.zeros(0, np.int32)
    assert gpu_edges(ccl, 1, e, e).tolist() == [0]
    np.testing.assert_array_equal(gpu_edges(ccl, 1000, e, e), np.arange(1000))
    out = ccl.label(torch.zeros(0, dtype=torch.int32, device="cuda"),
                    torch.zeros(0, dtype=torch.int32, device="cuda"), 0)
    assert out.numel() == 0
    src, dst = gen.triangle_edges(33)
    np.testing.assert_array_equal(gpu_edges(ccl, 33 * 33, src, dst, np.zeros(len(src), np.uint8)),
                                  np.arange(33 * 33))
    assert not gpu_edges(ccl, 33 * 33, src, dst).any()  # NULL mask: all occupied


@pytest.mark.parametrize("shift", [0, 1, 2, 3])
def test_small_and_unaligned_label_arrays(ccl, shift):
    """Label arrays of 1-3 sites (fewer than one 16-byte group) and label
    views starting 4, 8 or 12 bytes into an allocation (the unaligned
    init and flatten paths), on the edge list, the neighbour list and CSR.
    The view ends at the end of its allocation, so a read past it would
    leave the buffer."""
    rng = np.random.default_rng(60 + shift)
    for n in (1, 2, 3, 5, 7, 1000, 70_001):
        m = 3 * n
        src = rng.integers(0, n, m).astype(np.int32)
        dst = rng.integers(0, n, m).astype(np.int32)
        occ = (rng.random(m) < 0.4).astype(np.uint8)
        want = oracle.label_edges(n, src, dst, occ)
        _say(f"small/unaligned n={n} shift={shift}")
        buf = torch.full((n + shift,), -5, dtype=torch.int32, device="cuda")
        out = buf[shift:]
        ccl.label(dev(src), dev(dst), n, dev(occ), out=out)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), want)
        assert (buf[:shift].cpu().numpy() == -5).all()
        nn, occ_ell = gen.ell_from_edges(n, src, dst, occ, int(np.bincount(
            np.concatenate([src, dst]), minlength=n).max()))
        buf.fill_(-5)
        ccl.label_ell(dev(nn), dev(occ_ell), out=out)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), want)
        order = np.argsort(src, kind="stable")
        row_ptr = np.zeros(n + 1, np.int32)
        np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
        buf.fill_(-5)
        ws = torch.empty(max(ccl.csr_workspace_bytes(n, m), 8), dtype=torch.uint8, device="cuda")
        ccl.label_csr(dev(row_ptr), dev(dst[order]), dev(occ[order]), out=out, workspace=ws)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), want)


# ------------------------------------------------------------ workloads

def test_config1_honeycomb_l256(ccl):
    """Honeycomb L=256 periodic, p = 0.6527, edge list."""
    g = gen.honeycomb_realization(256, 0.6527, 1)
    got = gpu_edges(ccl, g.n_sites, g.src, g.dst, g.occ)
    np.testing.assert_array_equal(got, oracle.label_edges(g.n_sites, g.src, g.dst, g.occ))
    check_invariants(got, g.n_sites, g.src, g.dst, g.occ)


@pytest.mark.parametrize("L,p", [(181, 0.3473), (257, 0.3473), (300, 0.1736), (300, 0.5209),
                                 (512, 0.3473), (700, 0.3473)])
def test_triangle_csr_multi_tile(ccl, L, p):
    """One tile (L=181), several 65536-site tiles and ragged last tiles."""
    g = gen.triangle_csr_realization(L, p, L)
    got = gpu_csr(ccl, g.row_ptr, g.col, g.occ)
    np.testing.assert_array_equal(got, oracle.label_csr(g.n_sites, g.row_ptr, g.col, g.occ))


@pytest.mark.parametrize("p", [0.3473, 0.1736, 0.5209])
def test_config2_triangle_l8192_csr(ccl, p):
    """Full size: triangle L=8192 periodic (67,108,864 sites), half-CSR, with
    slab tiles and with grid tiles (grid width 8192, the configuration the
    benchmark times)."""
    g = gen.triangle_csr_realization(8192, p, 2)
    want = oracle.label_csr(g.n_sites, g.row_ptr, g.col, g.occ)
    np.testing.assert_array_equal(gpu_csr(ccl, g.row_ptr, g.col, g.occ), want)
    np.testing.assert_array_equal(gpu_csr(ccl, g.row_ptr, g.col, g.occ, grid_width=8192), want)


def rect_triangle_csr(w, h, n=None):
    """Half-CSR of a w x h periodic triangular lattice (site y*w + x, forward
    bonds to (x+1, y), (x, y+1), (x+1, y+1)); with n < w*h only the first n
    sites, bonds to the missing ones dropped (non-affine rows at the end)."""
    y, x = np.divmod(np.arange(w * h, dtype=np.int64), w)
    nb = np.stack([y * w + (x + 1) % w, ((y + 1) % h) * w + x, ((y + 1) % h) * w + (x + 1) % w], 1)
    n = w * h if n is None else n
    nb = nb[:n]
    keep = nb < n
    deg = keep.sum(1)
    row_ptr = np.zeros(n + 1, np.int32)
    np.cumsum(deg, out=row_ptr[1:])
    return row_ptr, nb[keep].astype(np.int32)


@pytest.mark.parametrize("w,h,cut", [(8192, 40, 0), (8192, 40, 8192 - 100), (6004, 33, 0), (6004, 33, 5),
                                     (12288, 36, 0), (4100, 37, 4100), (2052, 70, 0), (4104, 96, 0),
                                     (8192, 33, 8192 - 100)])
def test_csr_grid_tiles(ccl, w, h, cut):
    """Grid tiles (32 rows x 2048 columns) on rectangular lattices: ragged
    tile columns (w not a multiple of 2048) and tile rows (h not a multiple of
    32), a partial last grid row whose missing sites make the last rows
    non-affine (the row path), a tile with no site, no mask, a device-drawn
    mask, and an occupancy view one byte off 4-byte alignment.  The flatten's
    32 x 512 windows are ragged the same way (w not a multiple of 512), and
    with h = 33 and a last row of 100 sites most windows of the last window
    row hold no site at all."""
    n = w * h - cut
    row_ptr, col = rect_triangle_csr(w, h, n)
    occ = gen.bernoulli(w + h, len(col), 0.3473)
    want = oracle.label_csr(n, row_ptr, col, occ)
    np.testing.assert_array_equal(gpu_csr(ccl, row_ptr, col, occ, grid_width=w), want)
    np.testing.assert_array_equal(gpu_csr(ccl, row_ptr, col, None, grid_width=w),
                                  oracle.label_csr(n, row_ptr, col, None))
    _say(f"grid tiles w={w} h={h} cut={cut}: drawn occupancy and an unaligned mask view")
    out = ccl.label_csr_philox(dev(row_ptr), dev(col), w + h, gen.STREAM_OCC, 0.3473, grid_width=w)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), want)
    buf = torch.zeros(len(occ) + 1, dtype=torch.uint8, device="cuda")
    buf[1:] = dev(occ)
    out = ccl.label_csr(dev(row_ptr), dev(col), buf[1:], grid_width=w)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), want)
    # labels written through a view 4 bytes off 16-byte alignment (the
    # flatten then takes its per-site form instead of the 16-byte windows)
    lab = torch.full((n + 1,), -1, dtype=torch.int32, device="cuda")
    ccl.label_csr(dev(row_ptr), dev(col), dev(occ), out=lab[1:], grid_width=w)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(lab[1:].cpu().numpy(), want)
    assert int(lab[0].item()) == -1


def test_csr_grid_any_graph(ccl):
    """The grid width changes only the tiling: ragged degrees and random
    columns (never affine) give the oracle's labels for any width."""
    rng = np.random.default_rng(12)
    n = 300_000
    deg = rng.integers(0, 7, n)
    rp = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    c = rng.integers(0, n, rp[-1]).astype(np.int32)
    o = (rng.random(rp[-1]) < 0.25).astype(np.uint8)
    want = oracle.label_csr(n, rp, c, o)
    for w in (4100, 8192, 10000, 15000):
        np.testing.assert_array_equal(gpu_csr(ccl, rp, c, o, grid_width=w), want)
    # a lattice numbered row by row, labelled with a wrong width
    row_ptr, col = rect_triangle_csr(8192, 24)
    occ = gen.bernoulli(9, len(col), 0.5)
    want = oracle.label_csr(8192 * 24, row_ptr, col, occ)
    for w in (4104, 8200, 12288):
        np.testing.assert_array_equal(gpu_csr(ccl, row_ptr, col, occ, grid_width=w), want)


def test_csr_forms(ccl):
    # honeycomb half-CSR: every second row empty
    L = 200
    row_ptr, col = gen.honeycomb_csr(L)
    occ = gen.bernoulli(4, len(col), 0.6527)
    np.testing.assert_array_equal(gpu_csr(ccl, row_ptr, col, occ),
                                  oracle.label_csr(2 * L * L, row_ptr, col, occ))
    # ragged degrees, random columns, both orientations listed
    rng = np.random.default_rng(11)
    n = 150_001
    deg = rng.integers(0, 9, n)
    rp = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    c = rng.integers(0, n, rp[-1]).astype(np.int32)
    o = (rng.random(rp[-1]) < 0.3).astype(np.uint8)
    np.testing.assert_array_equal(gpu_csr(ccl, rp, c, o), oracle.label_csr(n, rp, c, o))
    np.testing.assert_array_equal(gpu_csr(ccl, rp, c, None), oracle.label_csr(n, rp, c, None))
    # a single tile needs no workspace
    small = gen.triangle_csr_realization(100, 0.4, 5)
    out = ccl.label_csr(dev(small.row_ptr), dev(small.col), dev(small.occ),
                        workspace=torch.empty(8, dtype=torch.uint8, device="cuda"))
    np.testing.assert_array_equal(out.cpu().numpy(),
                                  oracle.label_csr(small.n_sites, small.row_ptr, small.col, small.occ))


def test_csr_almost_affine(ccl):
    """Tiles whose bond count is 3 per row although row_ptr is not affine: the
    affine reading is verified while it streams and such a tile starts over
    on the row path.  Tile 0 and the partial last tile are affine, tile 1
    alternates degrees 2 and 4, tile 2 differs in one pair of rows only."""
    T = 65536
    n = 3 * T + 1000
    deg = np.full(n, 3, dtype=np.int64)
    deg[T:2 * T:2], deg[T + 1:2 * T:2] = 2, 4
    deg[2 * T + 10], deg[2 * T + 11] = 2, 4
    rp = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    rng = np.random.default_rng(23)
    m = int(rp[-1])
    site = np.repeat(np.arange(n), deg)
    c = (site + rng.integers(-300, 301, m)) % n
    far = rng.random(m) < 0.05
    c[far] = rng.integers(0, n, int(far.sum()))
    c = c.astype(np.int32)
    o = (rng.random(m) < 0.45).astype(np.uint8)
    np.testing.assert_array_equal(gpu_csr(ccl, rp, c, o), oracle.label_csr(n, rp, c, o))
    np.testing.assert_array_equal(gpu_csr(ccl, rp, c, None), oracle.label_csr(n, rp, c, None))


# ------------------------------------------------- occupancy on the device

def test_device_philox_matches_the_host_generator(ccl):
    """The device's Philox4x32-10 against the published known-answer vector
    whose counter fits the stream layout (all zeros), then word for word and
    bit for bit against the host generator (itself pinned to all the
    published vectors) for unaligned ranges, several streams and seeds."""
    row = read_golden("philox4x32_10_kat.txt")[0]
    assert row[:6] == ["00000000"] * 6
    want = [int(x, 16) for x in row[6:10]]
    got = ccl.philox_u32(0, 0, 4).cpu().numpy().view(np.uint32).tolist()
    assert got == want
    for seed, stream, first, n in ((0, 0, 0, 4096), (gen.mix_seed(7, 3), 3, 5, 1001),
                                   (2**64 - 1, 2**32 - 1, 2**40 + 3, 777)):
        _say(f"philox seed={seed} stream={stream} first={first} n={n}")
        got = ccl.philox_u32(seed, stream, n, first=first).cpu().numpy().view(np.uint32)
        np.testing.assert_array_equal(got, gen.u32(seed, stream, n, first))
    for p in (0.0, 1.0, 0.3473, 0.6527, 1e-9):
        for first, n in ((0, 100_003), (7, 4099)):
            got = ccl.bernoulli(11, gen.STREAM_OCC, n, p, first=first).cpu().numpy()
            np.testing.assert_array_equal(got, gen.bernoulli(11, n, p, first=first))
    # the headline workload's mask, drawn on the device, labels identically
    g = gen.triangle_csr_realization(700, 0.3473, 2)
    occ_dev = ccl.bernoulli(2, gen.STREAM_OCC, len(g.col), 0.3473)
    np.testing.assert_array_equal(occ_dev.cpu().numpy(), g.occ)
    lab = ccl.label_csr(dev(g.row_ptr), dev(g.col), occ_dev)
    np.testing.assert_array_equal(lab.cpu().numpy(), oracle.label_csr(g.n_sites, g.row_ptr, g.col, g.occ))


def _fused(ccl, rp, c, seed, p):
    _say(f"ccl_label_csr_philox n={len(rp) - 1} m={len(c)} e0={int(rp[0])} seed={seed} p={p}")
    out = ccl.label_csr_philox(dev(rp), dev(c), seed, gen.STREAM_OCC, p)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_csr_with_drawn_occupancy(ccl):
    """The tile kernel drawing bond e's occupancy as word e of the Philox
    stream labels exactly as the host-drawn mask does: the affine path over
    several tiles and a ragged last tile, tiles whose first bond is not a
    multiple of four (row_ptr[0] = 1..3, so the four-bond draws straddle two
    Philox blocks), the row path (ragged degrees, rows longer than the ones
    kept in registers) and the limits p = 0, p = 1."""
    g = gen.triangle_csr_realization(700, 0.3473, 2)
    for p in (0.3473, 0.0, 1.0, 1e-9):
        occ = gen.bernoulli(2, len(g.col), p)
        np.testing.assert_array_equal(_fused(ccl, g.row_ptr, g.col, 2, p),
                                      oracle.label_csr(g.n_sites, g.row_ptr, g.col, occ))
    rp0, c0 = gen.triangle_csr(300)
    for e0 in (1, 2, 3):
        rp = (rp0 + e0).astype(np.int32)
        c = np.concatenate([np.full(e0, 7, np.int32), c0]).astype(np.int32)
        occ = gen.bernoulli(5, len(c), 0.3473)
        np.testing.assert_array_equal(_fused(ccl, rp, c, 5, 0.3473),
                                      oracle.label_csr(len(rp) - 1, rp, c, occ))
    rng = np.random.default_rng(31)
    n = 150_001
    deg = rng.integers(0, 13, n)
    deg[::997] = 40
    rp = np.concatenate([[3], 3 + np.cumsum(deg)]).astype(np.int32)
    c = rng.integers(0, n, int(rp[-1])).astype(np.int32)
    for p in (0.2, 0.05):
        occ = gen.bernoulli(9, len(c), p)
        np.testing.assert_array_equal(_fused(ccl, rp, c, 9, p), oracle.label_csr(n, rp, c, occ))
    with pytest.raises(ccl.CclError) as e:
        ccl.label_csr_philox(dev(g.row_ptr), dev(g.col), 2, gen.STREAM_OCC, float("nan"))
    assert e.value.status == 1


# ------------------------------------------------------- cluster statistics

def _gpu_stats(ccl, lab_t, top, bot):
    ids, count = ccl.cluster_ids(lab_t)
    sizes = ccl.cluster_sizes(lab_t)
    sp = ccl.spans(lab_t, dev(top), dev(bot))
    torch.cuda.synchronize()
    return ids.cpu().numpy(), int(count.item()), sizes.cpu().numpy(), bool(sp.item())


def test_cluster_statistics(ccl):
    """Sequential ids, sizes at the cluster minima and the spanning test
    against the oracle: triangle cylinders (open top and bottom) below, at
    and above the threshold, a multi-tile CSR labeling, and degenerate
    labelings."""
    L = 256
    n = L * L
    src, dst = gen.triangle_edges(L)
    wrap = gen.y_wrap_bonds_triangle(L)
    top = np.arange(L, dtype=np.int32)
    bot = np.arange(n - L, n, dtype=np.int32)
    seen = set()
    for p in (0.30, 0.3473, 0.40):
        occ = gen.bernoulli(41, len(src), p)
        occ[wrap] = 0
        lab = oracle.label_edges(n, src, dst, occ)
        _say(f"cluster statistics triangle L={L} p={p}")
        lab_t = dev(lab)
        ids, count, sizes, sp = _gpu_stats(ccl, lab_t, top, bot)
        want_ids, want_count = oracle.cluster_ids(lab)
        np.testing.assert_array_equal(ids, want_ids)
        assert count == want_count
        np.testing.assert_array_equal(sizes, oracle.sizes_by_minimum(lab))
        assert sp == oracle.spans(lab, top, bot)
        seen.add(sp)
    assert seen == {False, True}  # both outcomes occur
    g = gen.triangle_csr_realization(700, 0.3473, 3)
    lab_t = ccl.label_csr(dev(g.row_ptr), dev(g.col), dev(g.occ))
    lab = lab_t.cpu().numpy()
    ids, count, sizes, _ = _gpu_stats(ccl, lab_t, top, bot)
    np.testing.assert_array_equal(ids, oracle.cluster_ids(lab)[0])
    np.testing.assert_array_equal(sizes, oracle.sizes_by_minimum(lab))
    # isolated sites; one cluster; one site; empty site sets
    for lab in (np.arange(5000, dtype=np.int32), np.zeros(70000, np.int32), np.zeros(1, np.int32)):
        ids, count, sizes, sp = _gpu_stats(ccl, dev(lab), np.zeros(1, np.int32), np.zeros(1, np.int32))
        np.testing.assert_array_equal(ids, oracle.cluster_ids(lab)[0])
        assert count == oracle.cluster_ids(lab)[1]
        np.testing.assert_array_equal(sizes, oracle.sizes_by_minimum(lab))
        assert sp
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    assert ccl.spans(dev(np.arange(10, dtype=np.int32)), e, dev(np.arange(3, dtype=np.int32))).item() == 0
    # labels and site ids outside [0, N) are skipped: ids -1, no size, no flag
    # (N not a multiple of 8: the last lane of a span holds fewer sites)
    n = 9003
    lab = np.arange(n, dtype=np.int32)
    lab[[5, 4097, 8999]] = [n + 5, -3, 2**31 - 1]
    valid = lab == np.arange(n)
    ids, count, sizes, _ = _gpu_stats(ccl, dev(lab), np.zeros(1, np.int32), np.zeros(1, np.int32))
    np.testing.assert_array_equal(ids, np.where(valid, np.cumsum(valid) - 1, -1))
    assert count == int(valid.sum())
    np.testing.assert_array_equal(sizes, valid.astype(np.int32))
    a = dev(np.array([-1, n, 0, 5], np.int32))
    assert ccl.spans(dev(lab), a, dev(np.array([n + 100, 0], np.int32))).item() == 1
    assert ccl.spans(dev(lab), a, dev(np.array([n + 100, -7, 5], np.int32))).item() == 0
    # labels that are not 16-byte aligned (a view one element in) and a ragged
    # length: the statistics read them element by element
    g = gen.triangle_csr_realization(97, 0.3473, 4)
    want = oracle.label_csr(g.n_sites, g.row_ptr, g.col, g.occ)
    buf = dev(np.concatenate([[0], want]).astype(np.int32))
    view = buf[1:]
    assert view.data_ptr() % 16 != 0
    ids, count, sizes, _ = _gpu_stats(ccl, view, np.zeros(1, np.int32), np.zeros(1, np.int32))
    np.testing.assert_array_equal(ids, oracle.cluster_ids(want)[0])
    np.testing.assert_array_equal(sizes, oracle.sizes_by_minimum(want))


# ------------------------------------------- the paper's neighbour-list path

def test_ell_lattices_and_trees(ccl):
    """ccl_label_ell (steps (i)-(iv) of section 3 on the padded column-major
    neighbour list) against the oracle: a triangle lattice (z = 6) with and
    without a mask, Cayley trees in standard and random position (z = 3),
    and a random 3-regular graph."""
    g = gen.triangle_realization(96, 0.3473, 12)
    nn, oe = gen.ell_from_edges(g.n_sites, g.src, g.dst, g.occ, 6)
    np.testing.assert_array_equal(gpu_ell(ccl, nn, oe), oracle_ell(nn, oe))
    np.testing.assert_array_equal(gpu_ell(ccl, nn), oracle_ell(nn))
    for rp in (False, True):
        t = gen.cayley_realization(14, 0.75, 8, rp)
        nn, oe = gen.ell_from_edges(t.n_sites, t.src, t.dst, t.occ, 3)
        got = gpu_ell(ccl, nn, oe)
        np.testing.assert_array_equal(got, oracle_ell(nn, oe))
        assert len(np.unique(got)) == t.n_sites - int(t.occ.sum())  # a forest
    r = gen.bethe_random_regular(1 << 18, 3, 0.5, 4)
    nn, oe = gen.ell_from_edges(r.n_sites, r.src, r.dst, r.occ, 3)
    np.testing.assert_array_equal(gpu_ell(ccl, nn, oe), oracle_ell(nn, oe))


def test_ell_ragged_padding_and_degenerate(ccl):
    # ragged lists with padding (-1), duplicates and self entries, each bond
    # listed at both ends with one occupancy
    rng = np.random.default_rng(31)
    n, m = 20000, 45000
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    occ = (rng.random(m) < 0.55).astype(np.uint8)
    z = int(np.bincount(np.concatenate([src, dst]), minlength=n).max())
    nn, oe = gen.ell_from_edges(n, src, dst, occ, z + 2)
    got = gpu_ell(ccl, nn, oe)
    np.testing.assert_array_equal(got, oracle_ell(nn, oe))
    np.testing.assert_array_equal(got, oracle.label_edges(n, src, dst, occ))
    # z_max = 0, all padding, one site
    np.testing.assert_array_equal(gpu_ell(ccl, np.zeros((0, 1000), np.int32)), np.arange(1000))
    np.testing.assert_array_equal(gpu_ell(ccl, np.full((4, 777), -1, np.int32)), np.arange(777))
    assert gpu_ell(ccl, np.zeros((1, 1), np.int32)).tolist() == [0]
    out = ccl.label_ell(torch.zeros((3, 0), dtype=torch.int32, device="cuda"))
    assert out.numel() == 0


def test_ell_argument_errors(ccl):
    import ctypes

    lib = ccl._lib
    lab = torch.empty(16, dtype=torch.int32, device="cuda")
    nn = torch.zeros(16, dtype=torch.int32, device="cuda")
    P = ctypes.c_void_p
    s = P(torch.cuda.current_stream().cuda_stream)
    INVALID = 1  # CCL_ERR_INVALID_VALUE
    assert lib.ccl_label_ell(16, -1, P(nn.data_ptr()), None, P(lab.data_ptr()), s) == INVALID
    assert lib.ccl_label_ell(16, 1, None, None, P(lab.data_ptr()), s) == INVALID
    assert lib.ccl_label_ell(16, 1, P(nn.data_ptr()), None, None, s) == INVALID
    assert lib.ccl_label_ell(1 << 31, 1, P(nn.data_ptr()), None, P(lab.data_ptr()), s) == INVALID
    assert lib.ccl_label_ell(1 << 30, (1 << 31) - 1, P(nn.data_ptr()), None, P(lab.data_ptr()), s) == \
        INVALID
    # labels overlapping the list
    assert lib.ccl_label_ell(16, 1, P(nn.data_ptr()), None, P(nn.data_ptr()), s) == INVALID
    with pytest.raises(ValueError):
        ccl.label_ell(nn)  # not two-dimensional


@pytest.mark.parametrize("p", [0.45, 0.5, 0.55])
def test_config3_random_3_regular(ccl, p):
    """Bethe substitute: random 3-regular N = 2^24, random position."""
    g = gen.bethe_random_regular(1 << 24, 3, p, 3)
    got = gpu_edges(ccl, g.n_sites, g.src, g.dst, g.occ)
    np.testing.assert_array_equal(got, oracle.label_edges(g.n_sites, g.src, g.dst, g.occ))


@pytest.mark.parametrize("random_position", [False, True])
def test_cayley_tree(ccl, random_position):
    g = gen.cayley_realization(18, 0.75, 6, random_position)
    got = gpu_edges(ccl, g.n_sites, g.src, g.dst, g.occ)
    np.testing.assert_array_equal(got, oracle.label_edges(g.n_sites, g.src, g.dst, g.occ))
    assert len(np.unique(got)) == g.n_sites - int(g.occ.sum())


# ------------------------------------------------------------ adversarial

def test_star_hub_last(ccl):
    """Every union hits one root: 10^6 leaves, hub = N - 1."""
    n = 1_000_001
    leaves = np.arange(n - 1, dtype=np.int32)
    hub = np.full(n - 1, n - 1, np.int32)
    occ = (leaves % 7 != 3).astype(np.uint8)
    got = gpu_edges(ccl, n, hub, leaves, occ)
    np.testing.assert_array_equal(got, oracle.label_edges(n, hub, leaves, occ))


def test_descending_path_1e7(ccl):
    n = 10_000_000
    src = np.arange(n - 1, 0, -1, dtype=np.int32)
    dst = src - 1
    got = gpu_edges(ccl, n, src, dst)
    assert not got.any()


def test_complete_graph_k2000(ccl):
    k = 2000
    iu = np.triu_indices(k, 1)
    src, dst = iu[1].astype(np.int32), iu[0].astype(np.int32)
    rng = np.random.default_rng(2)
    perm = rng.permutation(k).astype(np.int32)
    got = gpu_edges(ccl, k, perm[src], perm[dst])
    assert not got.any()


def test_duplicated_bonds(ccl):
    g = gen.honeycomb_realization(64, 0.6, 7)
    reps = 1000
    src = np.tile(g.src, reps)
    dst = np.tile(g.dst, reps)
    occ = np.tile(g.occ, reps)
    got = gpu_edges(ccl, g.n_sites, src, dst, occ)
    np.testing.assert_array_equal(got, oracle.label_edges(g.n_sites, g.src, g.dst, g.occ))


def test_repeat_runs_identical(ccl):
    g = gen.triangle_csr_realization(1024, 0.3473, 12)
    want = oracle.label_csr(g.n_sites, g.row_ptr, g.col, g.occ)
    rp, c, o = dev(g.row_ptr), dev(g.col), dev(g.occ)
    out = torch.empty(g.n_sites, dtype=torch.int32, device="cuda")
    ws = torch.empty(ccl.csr_workspace_bytes(g.n_sites, len(g.col)), dtype=torch.uint8, device="cuda")
    _say("csr repeat x50")
    for _ in range(50):
        ccl.label_csr(rp, c, o, out=out, workspace=ws)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), want)


# ------------------------------------------------------------ batches

def _batch(specs):
    site_off, bond_off, src, dst, occ = gen.batch_arrays(specs)
    return site_off, bond_off, src, dst, occ


BATCH_TUNINGS = [None, dict(schedule=2, small_sites=-1),
                 dict(schedule=2, block_threads=256, blocks_per_cu=2, bonds_per_chunk=4096,
                      sites_per_chunk=2048),
                 dict(schedule=1), dict(schedule=1, small_sites=-1, bonds_per_chunk=8192,
                                        sites_per_chunk=4096),
                 dict(schedule=3), dict(schedule=3, small_sites=-1, sites_per_chunk=4096)]


@pytest.mark.parametrize("tuning", BATCH_TUNINGS, ids=lambda t: str(t))
def test_batched_matches_oracle(ccl, tuning):
    specs = gen.batch_specs(96, base_seed=21, ls=(8, 16, 64, 128, 256))
    specs.append(gen.InstanceSpec("triangle", 1, 0.3, 5))  # one site, three self-loops
    site_off, bond_off, src, dst, occ = _batch(specs)
    want = oracle.label_batched(site_off, bond_off, src, dst, occ)
    plan = ccl.Plan(site_off, bond_off, tuning)
    _say(f"batched K={len(specs)} sites={site_off[-1]} tuning={plan.tuning.as_dict()}")
    out = plan.label(dev(src), dev(dst), dev(occ))
    torch.cuda.synchronize()
    assert plan.check() == 0
    np.testing.assert_array_equal(out.cpu().numpy(), want)
    # second launch on the same plan and buffers
    out2 = plan.label(dev(src), dev(dst), dev(occ))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out2.cpu().numpy(), want)
    # the per-instance schedule gives the same labels
    base = ccl.label_batched_per_instance(site_off, bond_off, dev(src), dev(dst), dev(occ))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(base.cpu().numpy(), want)
    plan.close()


def test_batched_with_empty_instances(ccl):
    site_off = np.array([0, 0, 5, 5, 105], np.int64)
    bond_off = np.array([0, 0, 0, 3, 3 + 150], np.int64)
    rng = np.random.default_rng(3)
    src = np.concatenate([np.zeros(3), rng.integers(0, 100, 150)]).astype(np.int32)
    dst = np.concatenate([np.zeros(3), rng.integers(0, 100, 150)]).astype(np.int32)
    occ = (rng.random(153) < 0.5).astype(np.uint8)
    # instance 2 has bonds but no sites: rejected
    with pytest.raises(ccl.CclError):
        ccl.Plan(site_off, bond_off)
    bond_off = np.array([0, 0, 0, 0, 150], np.int64)
    src, dst, occ = src[3:], dst[3:], occ[3:]
    want = oracle.label_batched(site_off, bond_off, src, dst, occ)
    plan = ccl.Plan(site_off, bond_off)
    out = plan.label(dev(src), dev(dst), dev(occ))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), want)


@pytest.mark.parametrize("schedule", [1, 2, 3])
def test_batched_graph_replay(ccl, schedule):
    """Capture the batched launch in a HIP graph, replay it several times with
    eager work in between, and check every replay."""
    specs = gen.batch_specs(40, base_seed=5, ls=(16, 64, 128))
    site_off, bond_off, src, dst, occ = _batch(specs)
    want = oracle.label_batched(site_off, bond_off, src, dst, occ)
    plan = ccl.Plan(site_off, bond_off, dict(schedule=schedule))
    ds, dd, do = dev(src), dev(dst), dev(occ)
    out = torch.empty(int(site_off[-1]), dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.label(ds, dd, do, out=out, stream=s)  # warm-up outside the graph
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    _say("batched graph capture")
    with torch.cuda.graph(g, stream=s):
        plan.label(ds, dd, do, out=out, stream=s)
    for r in range(4):
        out.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), want, err_msg=f"replay {r}")
        assert plan.check() == 0


def test_monte_carlo_graph_replay(ccl):
    """One Monte-Carlo realization -- occupancy drawn on the device, CSR
    labeling, sequential ids, sizes, spanning test -- captured in a HIP graph
    and replayed with eager work and synchronizations in between; every
    replay must give the eager results, which equal the oracle's."""
    L, p, seed = 300, 0.3473, 13
    row_ptr, col = gen.triangle_csr(L)
    n, m = L * L, len(col)
    rp, dc = dev(row_ptr), dev(col)
    occ = torch.empty(m, dtype=torch.uint8, device="cuda")
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = torch.empty(max(ccl.csr_workspace_bytes(n, m), 8), dtype=torch.uint8, device="cuda")
    top = dev(np.arange(L, dtype=np.int32))
    bot = dev(np.arange(n - L, n, dtype=np.int32))
    s = torch.cuda.Stream()

    def realization():
        ccl.bernoulli(seed, gen.STREAM_OCC, m, p, out=occ, stream=s)
        ccl.label_csr(rp, dc, occ, out=lab, workspace=ws, stream=s)
        ids, count = ccl.cluster_ids(lab, stream=s)
        sizes = ccl.cluster_sizes(lab, stream=s)
        sp = ccl.spans(lab, top, bot, stream=s)
        return ids, count, sizes, sp

    host_occ = gen.bernoulli(seed, m, p)
    want_lab = oracle.label_csr(n, row_ptr, col, host_occ)
    want_ids, want_count = oracle.cluster_ids(want_lab)
    with torch.cuda.stream(s):
        eager = realization()
    torch.cuda.synchronize()
    eager = [t.cpu().numpy() for t in eager]
    np.testing.assert_array_equal(lab.cpu().numpy(), want_lab)
    np.testing.assert_array_equal(eager[0], want_ids)
    assert int(eager[1][0]) == want_count
    np.testing.assert_array_equal(eager[2], oracle.sizes_by_minimum(want_lab))
    g = torch.cuda.CUDAGraph()
    _say("monte-carlo graph capture")
    with torch.cuda.graph(g, stream=s):
        captured = realization()
    for r in range(3):
        lab.fill_(-7)
        occ.fill_(9)
        for t in captured:
            t.fill_(-5)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(lab.cpu().numpy(), want_lab, err_msg=f"replay {r}")
        for got, ref in zip(captured, eager):
            np.testing.assert_array_equal(got.cpu().numpy(), ref, err_msg=f"replay {r}")


def test_edges_with_drawn_occupancy(ccl):
    """The edge-list merge drawing bond b's occupancy as word b of the Philox
    stream labels exactly as the host-drawn mask does: a small honeycomb
    (one bond per lane), a triangle lattice of 5.9 M bonds (four bonds per
    lane, 16-byte loads) and a random 3-regular graph, plus p = 0 and 1."""
    for g, seed in ((gen.honeycomb_realization(256, 0.6527, 1), 1),
                    (gen.triangle_realization(1400, 0.3473, 6), 6),
                    (gen.bethe_random_regular(1 << 18, 3, 0.5, 8), 8)):
        for p in (g.p, 0.0, 1.0):
            occ = gen.bernoulli(seed, len(g.src), p)
            _say(f"ccl_label_philox {g.name} m={len(g.src)} p={p}")
            out = ccl.label_philox(dev(g.src), dev(g.dst), g.n_sites, seed, gen.STREAM_OCC, p)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(), oracle.label_edges(g.n_sites, g.src, g.dst, occ))
    with pytest.raises(ccl.CclError) as e:
        ccl.label_philox(dev(g.src), dev(g.dst), g.n_sites, 1, 0, float("nan"))
    assert e.value.status == 1


def test_drawn_occupancy_graph_replay(ccl):
    """The realization with its occupancy drawn inside the tile kernel
    (ccl_label_csr_philox) and its cluster sizes, captured in a HIP graph and
    replayed with eager work in between: every replay gives the oracle's
    labels for the host generator's mask."""
    L, p, seed = 300, 0.3473, 17
    row_ptr, col = gen.triangle_csr(L)
    n, m = L * L, len(col)
    rp, dc = dev(row_ptr), dev(col)
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = torch.empty(max(ccl.csr_workspace_bytes(n, m), 8), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()

    def realization():
        ccl.label_csr_philox(rp, dc, seed, gen.STREAM_OCC, p, out=lab, workspace=ws, stream=s)
        return ccl.cluster_sizes(lab, stream=s)

    want_lab = oracle.label_csr(n, row_ptr, col, gen.bernoulli(seed, m, p))
    want_sizes = oracle.sizes_by_minimum(want_lab)
    with torch.cuda.stream(s):
        sizes = realization()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(lab.cpu().numpy(), want_lab)
    np.testing.assert_array_equal(sizes.cpu().numpy(), want_sizes)
    g = torch.cuda.CUDAGraph()
    _say("drawn-occupancy graph capture")
    with torch.cuda.graph(g, stream=s):
        captured = realization()
    for r in range(3):
        lab.fill_(-7)
        captured.fill_(-5)
        ws.fill_(0xAB)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(lab.cpu().numpy(), want_lab, err_msg=f"replay {r}")
        np.testing.assert_array_equal(captured.cpu().numpy(), want_sizes, err_msg=f"replay {r}")


# ------------------------------------------------------------ checks & errors

def test_validate(ccl):
    src = dev(np.array([0, 1, 5, -1, 2], np.int32))
    dst = dev(np.array([1, 2, 0, 0, 9], np.int32))
    assert ccl.validate_edges(src, dst, 5) == 3
    assert ccl.validate_edges(src[:2], dst[:2], 5) == 0
    rp = dev(np.array([0, 2, 1, 4], np.int32))
    col = dev(np.array([1, 2, 3, 0], np.int32))
    assert ccl.validate_csr(rp, col) == 2  # one decreasing step, one id == n
    g = gen.triangle_csr_realization(50, 0.3, 1)
    assert ccl.validate_csr(dev(g.row_ptr), dev(g.col)) == 0


def test_argument_errors(ccl):
    e = dev(np.zeros(4, np.int32))
    with pytest.raises(ccl.CclError):  # labels alias an input
        ccl.label(e, e, 4, out=e)
    g = gen.triangle_csr_realization(300, 0.3, 1)
    assert ccl.csr_workspace_bytes(g.n_sites, len(g.col)) > 8  # 90000 sites: two tiles
    with pytest.raises(ccl.CclError):  # workspace too small
        ccl.label_csr(dev(g.row_ptr), dev(g.col), dev(g.occ),
                      workspace=torch.empty(8, dtype=torch.uint8, device="cuda"))
    small = gen.triangle_csr_realization(200, 0.3, 1)  # one tile: no workspace needed
    assert ccl.csr_workspace_bytes(small.n_sites, len(small.col)) == 0


# ------------------------------------------------------------ serving & autotune

def test_serving_mixed_equals_alone(ccl):
    """Requests of mixed sizes served concurrently give each request the
    labels it gets alone, and those equal the oracle's."""
    from paper_1603_08357_amd.serving import GpuExecutor, Job, Scheduler

    reqs = gen.request_trace(40, rate=2000.0, base_seed=17, n_max=200_000)
    jobs = []
    for r in reqs:
        g = gen.request_graph(r)
        jobs.append(Job(r.rid, r.arrival, g.n_sites, g.src, g.dst, g.occ))
    bad = Job(999, jobs[5].arrival, 10, np.array([0, 11], np.int32), np.array([1, 2], np.int32),
              np.ones(2, np.uint8))
    jobs.insert(6, bad)
    ex = GpuExecutor(n_streams=4, max_sites=max(j.n_sites for j in jobs))
    budget = 3 * max(j.bytes for j in jobs if j is not bad)
    sch = Scheduler(ex, budget, max_slots=4)
    _say(f"serving {len(jobs)} requests")
    done = sch.serve(jobs)
    assert len(done) == len(jobs)
    assert bad.status == "rejected"
    assert sch.peak_used <= budget and sch.peak_running > 1
    for j in jobs:
        if j is bad:
            continue
        assert j.status == "done"
        alone = gpu_edges(ccl, j.n_sites, j.src, j.dst, j.occ)
        np.testing.assert_array_equal(j.labels, alone)
        np.testing.assert_array_equal(j.labels, oracle.label_edges(j.n_sites, j.src, j.dst, j.occ))


def test_serving_ticks_under_a_binding_budget(ccl):
    """All requests present at once, a budget that holds about a third of
    them and small tick limits: small requests ride in batched ticks (one
    ccl_label_batched launch of a capacity plan per tick), the budget is
    what bounds the work in flight, and every result equals the oracle's."""
    from paper_1603_08357_amd.serving import GpuExecutor, Job, Scheduler

    reqs = gen.request_trace(90, rate=1e9, base_seed=23, n_max=300_000)
    jobs = []
    for r in reqs:
        g = gen.request_graph(r)
        jobs.append(Job(r.rid, 0.0, g.n_sites, g.src, g.dst, g.occ))
    jobs.append(Job(1000, 0.0, 0, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.uint8)))
    jobs.append(Job(1001, 0.0, 7, np.zeros(0, np.int32), np.zeros(0, np.int32), None))
    ex = GpuExecutor(n_streams=3, max_sites=max(j.n_sites for j in jobs), tick_sites=1 << 15, tick_jobs=12,
                     tick_total_sites=1 << 18, tick_total_bonds=1 << 20)
    budget = sum(j.bytes for j in jobs) // 3
    sch = Scheduler(ex, budget, max_slots=64)
    _say(f"serving {len(jobs)} requests, budget {budget} bytes")
    done = sch.serve(jobs)
    assert len(done) == len(jobs) and all(j.status == "done" for j in jobs)
    assert sch.ticks > 0 and sch.peak_used <= budget and sch.peak_used > budget // 2
    assert sum(j.batched > 1 for j in jobs) > 10
    for j in jobs:
        np.testing.assert_array_equal(j.labels, oracle.label_edges(j.n_sites, j.src, j.dst, j.occ),
                                      err_msg=f"request {j.rid} ({j.n_sites} sites, tick of {j.batched})")
        assert j.t_kernel_ms >= 0 and j.t_h2d_ms >= 0


@pytest.mark.parametrize("schedule", [3, 2, 1])
def test_capacity_plan_takes_a_layout_per_launch(ccl, schedule):
    """One capacity plan, five layouts set and launched back to back on one
    stream with no synchronization in between (each layout's tables are
    uploaded behind the previous launch); every batch equals the oracle.
    Layouts beyond the plan's limits and a plan made for one layout are
    refused."""
    plan = ccl.Plan.with_capacity(48, 2_000_000, 6_000_000, dict(schedule=schedule))
    stream = torch.cuda.Stream()
    cases = []
    for k, (count, seed, ls) in enumerate(((40, 1, (16, 64, 128)), (3, 2, (512,)), (48, 3, (16, 64, 256)),
                                           (1, 4, (64,)), (17, 5, (128, 256)))):
        specs = gen.batch_specs(count, base_seed=seed, ls=ls)
        so, bo, src, dst, occ = _batch(specs)
        cases.append((so, bo, dev(src), dev(dst), dev(occ), oracle.label_batched(so, bo, src, dst, occ)))
    torch.cuda.synchronize()
    outs = []
    _say(f"capacity plan, schedule {schedule}: {len(cases)} layouts back to back")
    for so, bo, src, dst, occ, _ in cases:
        plan.set_layout(so, bo, stream=stream)
        outs.append(plan.label(src, dst, occ, stream=stream))
    torch.cuda.synchronize()
    for k, (case, out) in enumerate(zip(cases, outs)):
        np.testing.assert_array_equal(out.cpu().numpy(), case[5], err_msg=f"layout {k}")
    assert plan.check() == 0
    big = gen.batch_specs(49, base_seed=6, ls=(16,))
    so, bo = gen.batch_offsets(big)
    with pytest.raises(ccl.CclError) as e:
        plan.set_layout(so, bo)  # 49 instances > 48
    assert e.value.status == 6
    so, bo = gen.batch_offsets(gen.batch_specs(2, base_seed=7, ls=(1024,)))
    with pytest.raises(ccl.CclError) as e:
        plan.set_layout(so, bo)  # 2^21 sites > 2,000,000
    assert e.value.status == 6
    plan.close()
    fixed = ccl.Plan(*gen.batch_offsets(gen.batch_specs(2, base_seed=8, ls=(16,))))
    with pytest.raises(ccl.CclError) as e:
        fixed.set_layout(*gen.batch_offsets(gen.batch_specs(2, base_seed=8, ls=(16,))))
    assert e.value.status == 1
    fixed.close()


def test_autotune_picks_a_correct_tuning(ccl, tmp_path, monkeypatch):
    from paper_1603_08357_amd import autotune
    monkeypatch.setenv("CCL_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    specs = gen.batch_specs(64, base_seed=8, ls=(16, 64, 128, 256))
    site_off, bond_off, src, dst, occ = _batch(specs)
    want = oracle.label_batched(site_off, bond_off, src, dst, occ)
    space = {"block_threads": (256, 512), "blocks_per_cu": (2, 4), "bonds_per_chunk": (16384,),
             "sites_per_chunk": (16384,), "small_sites": (0, -1), "schedule": (3, 2, 1)}
    _say("autotune 24 candidates")
    best = autotune.tune(site_off, bond_off, dev(src), dev(dst), dev(occ), space=space, reps=2)
    assert (tmp_path / "cache.json").exists()
    again = autotune.tune(site_off, bond_off, dev(src), dev(dst), dev(occ), space=space)
    assert again == best  # served from the cache
    plan = ccl.Plan(site_off, bond_off, best)
    out = plan.label(dev(src), dev(dst), dev(occ))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), want)
# ------------------------------------------------------------ concurrency

def test_concurrent_streams_match_oracle(ccl):
    """Edge-list, multi-tile CSR (slabs and grid tiles), neighbour-list (the
    paper's schedule) and batched-plan jobs (tiled schedule) in flight on
    eight streams at once: every result equals
    the oracle's.  (A merge-step compression store landing after the flatten's
    final root store showed up only under concurrent kernels; every label
    store of the labeling kernels is device-scope for that reason.)  Stops at
    the first mismatch."""
    jobs = []
    for i, (n, z, p) in enumerate([(300_000, 3, 0.5), (200_000, 4, 0.33), (150_000, 6, 0.2)]):
        g = gen.bethe_random_regular(n, z, p, 40 + i)
        jobs.append(("edges", g, oracle.label_edges(g.n_sites, g.src, g.dst, g.occ)))
    for L, p in [(300, 0.3473), (512, 0.5209)]:
        g = gen.triangle_csr_realization(L, p, L)
        jobs.append(("csr", g, oracle.label_csr(g.n_sites, g.row_ptr, g.col, g.occ)))
    g = gen.triangle_csr_realization(2176, 0.3473, 5)  # grid tiles: rows wider than a tile
    jobs.append(("csr_grid", g, oracle.label_csr(g.n_sites, g.row_ptr, g.col, g.occ)))
    e = gen.bethe_random_regular(250_000, 3, 0.55, 47)
    nn, occ_ell = gen.ell_from_edges(e.n_sites, e.src, e.dst, e.occ, 3)
    jobs.append(("ell", (nn, occ_ell), oracle.label_edges(e.n_sites, e.src, e.dst, e.occ)))
    specs = gen.batch_specs(24, base_seed=48, ls=(16, 64, 128, 256))
    site_off, bond_off, bsrc, bdst, bocc = _batch(specs)
    jobs.append(("batched", (site_off, bond_off, bsrc, bdst, bocc),
                 oracle.label_batched(site_off, bond_off, bsrc, bdst, bocc)))
    S = 8
    streams = [torch.cuda.Stream() for _ in range(S)]
    bufs = []
    for kind, g, want in jobs:
        ws = None
        if kind == "edges":
            ins = (dev(g.src), dev(g.dst), dev(g.occ))
        elif kind in ("csr", "csr_grid"):
            ins = (dev(g.row_ptr), dev(g.col), dev(g.occ))
            ws = [torch.empty(max(ccl.csr_workspace_bytes(g.n_sites, len(g.col)), 8), dtype=torch.uint8,
                              device="cuda") for _ in range(S)]
        elif kind == "ell":
            ins = (dev(g[0]), dev(g[1]))
        else:  # one plan per stream: a plan may be in flight on one stream at a time
            ins = (dev(g[2]), dev(g[3]), dev(g[4]))
            ws = [ccl.Plan(g[0], g[1]) for _ in range(S)]
        outs = [torch.empty(len(want), dtype=torch.int32, device="cuda") for _ in range(S)]
        bufs.append((ins, ws, outs))
    torch.cuda.synchronize()
    _say(f"concurrent: {len(jobs)} jobs (edge list, CSR slabs and grid tiles, neighbour list, batched) x {S} streams")
    for it in range(40):
        picks = []
        for s in range(S):
            gi = (it + s) % len(jobs)
            kind, g, _ = jobs[gi]
            ins, ws, outs = bufs[gi]
            with torch.cuda.stream(streams[s]):
                if kind == "edges":
                    ccl.label(ins[0], ins[1], g.n_sites, ins[2], out=outs[s], stream=streams[s])
                elif kind == "csr":
                    ccl.label_csr(ins[0], ins[1], ins[2], out=outs[s], workspace=ws[s], stream=streams[s])
                elif kind == "csr_grid":
                    ccl.label_csr(ins[0], ins[1], ins[2], out=outs[s], workspace=ws[s], stream=streams[s],
                                  grid_width=2176)
                elif kind == "ell":
                    ccl.label_ell(ins[0], ins[1], out=outs[s], stream=streams[s])
                else:
                    ws[s].label(ins[0], ins[1], ins[2], out=outs[s], stream=streams[s])
            picks.append((s, gi))
        for s, gi in picks:
            streams[s].synchronize()
            kind = jobs[gi][0]
            np.testing.assert_array_equal(bufs[gi][2][s].cpu().numpy(), jobs[gi][2],
                                          err_msg=f"iteration {it}, stream {s}, {kind} job")
            if kind == "batched":
                assert bufs[gi][1][s].check() == 0
    for (kind, _, _), (_, ws, _) in zip(jobs, bufs):
        if kind == "batched":
            for plan in ws:
                plan.close()


@pytest.mark.parametrize("L,p", [(512, 0.3473), (700, 0.5209), (8192, 0.3473)])
def test_cluster_size_histogram(ccl, L, p):
    """n_s on the GPU (ccl_cluster_sizes then ccl_cluster_size_histogram)
    equals the oracle's histogram element by element: bins held in LDS,
    bins past the LDS range (global atomics), a last bin that collects every
    larger cluster, and a sizes view that is not 16-byte aligned."""
    g = gen.triangle_csr_realization(L, p, 90 + L)
    lab = oracle.label_csr(g.n_sites, g.row_ptr, g.col, g.occ)
    dl = dev(lab)
    sizes = ccl.cluster_sizes(dl)
    for n_bins in (2, 3, 100, 9000, g.n_sites + 1):
        _say(f"size histogram L={L} p={p} bins={n_bins}")
        got = ccl.size_histogram(sizes, n_bins)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), oracle.size_histogram(lab, n_bins))
    buf = torch.zeros(g.n_sites + 1, dtype=torch.int32, device="cuda")
    buf[1:] = sizes
    got = ccl.size_histogram(buf[1:], 50)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), oracle.size_histogram(lab, 50))
    empty = ccl.size_histogram(torch.zeros(0, dtype=torch.int32, device="cuda"), 4)
    torch.cuda.synchronize()
    assert empty.cpu().tolist() == [0, 0, 0, 0]



@pytest.mark.parametrize("small_sites", [0, -1])
def test_batched_tiled_any_bond_order(ccl, small_sites):
    """The tiled schedule on instances whose bonds are not ordered by src
    (shuffled lattices: a tile's range then holds bonds of other tiles, which
    are joined as leaving bonds), random multigraphs with far more leaving
    bonds than a tile's list holds (the range is read again), instances of one
    tile, of several tiles and empty ones; every label equals the oracle's."""
    rng = np.random.default_rng(77 + small_sites)
    parts = []
    for L in (100, 300, 400):
        s_, d_ = gen.triangle_edges(L)
        o_ = gen.bernoulli(L, len(s_), 0.45)
        perm = rng.permutation(len(s_))
        parts.append((L * L, s_[perm], d_[perm], o_[perm]))
        parts.append((L * L, s_, d_, o_))
    for n, m in ((150_001, 400_000), (70_000, 10), (5, 0), (0, 0)):
        parts.append((n, rng.integers(0, max(n, 1), m).astype(np.int32), rng.integers(0, max(n, 1), m).astype(np.int32),
                      (rng.random(m) < 0.5).astype(np.uint8)))
    site_off = np.concatenate([[0], np.cumsum([p_[0] for p_ in parts])]).astype(np.int64)
    bond_off = np.concatenate([[0], np.cumsum([len(p_[1]) for p_ in parts])]).astype(np.int64)
    src = np.concatenate([p_[1] for p_ in parts]).astype(np.int32)
    dst = np.concatenate([p_[2] for p_ in parts]).astype(np.int32)
    occ = np.concatenate([p_[3] for p_ in parts]).astype(np.uint8)
    want = oracle.label_batched(site_off, bond_off, src, dst, occ)
    plan = ccl.Plan(site_off, bond_off, dict(schedule=3, small_sites=small_sites))
    _say(f"tiled batch K={len(parts)} sites={site_off[-1]} small_sites={small_sites}")
    for rep in range(2):
        out = plan.label(dev(src), dev(dst), dev(occ))
        torch.cuda.synchronize()
        assert plan.check() == 0
        np.testing.assert_array_equal(out.cpu().numpy(), want, err_msg=f"launch {rep}")
    out = plan.label(dev(src), dev(dst), None)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), oracle.label_batched(site_off, bond_off, src, dst, None))
    plan.close()


def test_probes_stay_in_bounds_and_do_their_work(ccl):
    """The copy probe copies; the random-access probe's fill mode writes only
    in-range indices (its dependent-chase mode follows them), and its
    atomicMin mode lowers entries to op numbers below n_ops."""
    n = 1 << 20
    src = torch.arange(3 * n, dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    ccl.probe_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    table = torch.empty(n, dtype=torch.int32, device="cuda")
    ccl.probe_random(table, 0, 4)  # fill: table[i] is a pseudo-random index in [0, n)
    torch.cuda.synchronize()
    t = table.cpu().numpy()
    assert t.min() >= 0 and t.max() < n and len(np.unique(t)) > n // 2
    for mode in (0, 3):  # gather, dependent chase: read only
        ccl.probe_random(table, 8 * n, mode)
    torch.cuda.synchronize()
    assert np.array_equal(table.cpu().numpy(), t)
    table.fill_(2**31 - 1)
    ops = 4 * n
    ccl.probe_random(table, ops, 1)  # atomicMin with the op number
    torch.cuda.synchronize()
    t = table.cpu().numpy()
    hit = t != 2**31 - 1
    assert hit.sum() > n // 2 and t[hit].max() < ops and t[hit].min() >= 0
