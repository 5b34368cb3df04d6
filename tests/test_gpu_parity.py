"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle, on seeded inputs."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import bf16_round, cast_inputs, cast_vals, oracle_ttmc_rounded, rel_fro

pytestmark = pytest.mark.gpu

TOL_Y = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-2}


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_10638_amd as tk_mod
    tk_mod.load_library()
    return tk_mod


def to_dev(coords, vals):
    return (torch.from_numpy(np.ascontiguousarray(coords, dtype=np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(vals, dtype=np.float64)).cuda())


def dev_list(U):
    return [torch.from_numpy(np.ascontiguousarray(u, dtype=np.float64)).cuda() for u in U]


def make(tk, w, dtype, fat_rule=True, memo=True):
    c, v = to_dev(w.coords, w.vals)
    return tk.tucker_init(c, v, w.dims, w.ranks, dtype=dtype, fat_rule=fat_rule, memo=memo)


def with_duplicates(w, k=37, seed=0):
    rng = np.random.default_rng(seed)
    pick = rng.choice(w.nnz, size=min(k, w.nnz), replace=False)
    c = np.concatenate([w.coords, w.coords[:, pick]], axis=1)
    v = np.concatenate([w.vals, rng.standard_normal(pick.size)])
    perm = rng.permutation(c.shape[1])
    return c[:, perm], v[perm]


# ------------------------------------------------------------------------------------------
# Layout (bit-exact)
# ------------------------------------------------------------------------------------------

def check_csf(tk, ctx, coords, vals, dtype):
    cc, cv = oracle.coalesce(coords, vals, ctx.dims)
    info = tk.tucker_get_info(ctx)
    assert info["nnz"] == cv.size
    for mode in range(ctx.order):
        exp = oracle.csf(cc, cv, mode)
        got = tk.tucker_get_csf(ctx, mode)
        assert info["rows"][mode] == exp["rows"].size
        np.testing.assert_array_equal(got["rows"].cpu().numpy(), exp["rows"])
        np.testing.assert_array_equal(got["ptr"].cpu().numpy(), exp["ptr"])
        np.testing.assert_array_equal(got["idx"].cpu().numpy(), exp["idx"])
        gv = got["vals"].cpu().numpy()
        if dtype == "f64":
            np.testing.assert_array_equal(gv, exp["vals"])
        elif dtype == "f32":
            np.testing.assert_array_equal(gv, exp["vals"].astype(np.float32))
        else:
            np.testing.assert_array_equal(gv, bf16_round(exp["vals"]))
    assert abs(info["normx2"] - float(cv @ cv)) <= 1e-12 * max(1.0, float(cv @ cv))


def test_csf_table1(tk):
    lines = [l.split() for l in open("tests/golden/table1_coo.txt") if l.strip() and not l.startswith("#")]
    arr = np.array([[float(x) for x in r] for r in lines])
    coords = (arr[:, :4].T - 1).astype(np.int32)
    vals = arr[:, 4]
    c, v = to_dev(coords, vals)
    ctx = tk.tucker_init(c, v, [5, 5, 5, 5], [1, 1, 1, 1], dtype="f64")
    check_csf(tk, ctx, coords, vals, "f64")
    got = tk.tucker_get_csf(ctx, 3)
    assert got["rows"].cpu().tolist() == [0, 3, 4]
    assert got["ptr"].cpu().tolist() == [0, 1, 2, 4]
    assert got["vals"].cpu().tolist() == [2.0, 5.0, 7.5, 4.0]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("dims", [[40, 300, 200], [30, 20, 25, 12]])
def test_csf_bit_exact_with_duplicates(tk, dtype, dims):
    w = synth.small_uniform(5, dims, [2] * len(dims), 6000)
    coords, vals = with_duplicates(w)
    c, v = to_dev(coords, vals)
    ctx = tk.tucker_init(c, v, dims, [2] * len(dims), dtype=dtype)
    check_csf(tk, ctx, coords, vals, dtype)
    # determinism: a second build gives identical bits
    ctx2 = tk.tucker_init(c, v, dims, [2] * len(dims), dtype=dtype)
    for mode in range(len(dims)):
        a, b = tk.tucker_get_csf(ctx, mode), tk.tucker_get_csf(ctx2, mode)
        for k in a:
            assert torch.equal(a[k], b[k])


def test_range_error(tk):
    coords = np.array([[0, 1], [0, 7]], dtype=np.int32)
    c, v = to_dev(coords, np.ones(2))
    with pytest.raises(tk.TuckerError) as e:
        tk.tucker_init(c, v, [4, 5], [1, 1])
    assert e.value.status == 2


# ------------------------------------------------------------------------------------------
# TTMc
# ------------------------------------------------------------------------------------------

TTMC_CASES = [
    # dims, ranks, nnz   (several chunks, rows split across chunks, ragged tails, empty rows)
    ([40, 300, 200], [16, 16, 16], 20000),     # order-3 MFMA path, long rows (split)
    ([500, 80, 60], [10, 10, 10], 12000),      # R = 10 (padded tile), empty rows in mode 0
    ([64, 48, 32], [8, 8, 8], 3000),
    ([30, 20, 25, 12], [3, 4, 2, 3], 5000),    # order 4, fiber-factored (short fibers)
    ([12, 10, 9, 8, 7], [2, 3, 2, 2, 2], 2500),  # order 5, fiber-factored (3 inner modes)
    ([400, 300, 60, 9], [8, 8, 8, 8], 30000),  # order 4, K = 512: 64 inner columns, R_f = 8, long fibers
    ([50, 40, 30, 20], [4, 12, 12, 16], 20000),  # order 4: 144-192 inner columns, R_f = 16 or 12
    ([20, 18, 16, 14], [20, 3, 4, 5], 8000),   # inner rank > 16 for some modes: generic path
    ([300, 250], [6, 6], 4000),                # order 2 (SpMM); R_1 <= K_1 = R_2 forces equal ranks
    ([50, 40, 30], [20, 3, 17], 4000),         # R > 16: generic path for order 3
    ([6, 5, 5, 4, 4, 3], [2, 2, 2, 2, 2, 2], 1500),              # order 6: generic path
    ([4, 4, 4, 3, 3, 3, 3, 3], [2, 2, 2, 2, 2, 2, 2, 2], 3000),  # order 8 (the compiled maximum)
]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("case", range(len(TTMC_CASES)))
def test_ttmc_parity(tk, dtype, case):
    dims, ranks, nnz = TTMC_CASES[case]
    w = synth.small_uniform(100 + case, dims, ranks, nnz)
    ctx = make(tk, w, dtype)
    Ud = dev_list(w.U_init)
    for mode in range(len(dims)):
        Y = tk.ttmc_mode(ctx, mode, Ud).double().cpu().numpy()
        Yo = oracle.ttmc(w.coords, w.vals, dims, ranks, mode, w.U_init)
        err = rel_fro(Y, Yo)
        assert err <= TOL_Y[dtype], (mode, err)
        # same rounded inputs: only the accumulation differs
        Yc = oracle_ttmc_rounded(w.coords, w.vals, dims, ranks, mode, w.U_init, dtype)
        assert rel_fro(Y, Yc) <= (1e-13 if dtype == "f64" else 2e-6), (mode, rel_fro(Y, Yc))


def long_row_case(seed):
    """Mode 0 with rows of very different lengths averaging well over 256 entries: long rows
    that span several chunks, and runs of 1-4 entry rows, so that up to four rows start inside
    one 16-entry group."""
    rng = np.random.default_rng(seed)
    dims, ranks = [120, 400, 300], [16, 12, 10]
    lens = np.zeros(dims[0], dtype=np.int64)
    lens[::7] = rng.integers(1500, 4000, size=lens[::7].size)
    short = np.setdiff1d(np.arange(dims[0]), np.arange(0, dims[0], 7))
    lens[short[: 60]] = rng.integers(1, 5, size=60)   # the rest stay empty
    coords = []
    for i, n in enumerate(lens):
        if n == 0:
            continue
        keys = rng.choice(dims[1] * dims[2], size=int(n), replace=False)
        coords.append(np.stack([np.full(n, i), keys // dims[2], keys % dims[2]]))
    coords = np.concatenate(coords, axis=1).astype(np.int32)
    vals = rng.standard_normal(coords.shape[1])
    U = [synth.gaussian_qr(rng, d, r) for d, r in zip(dims, ranks)]
    return dims, ranks, coords, vals, U


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_ttmc_long_rows(tk, dtype):
    dims, ranks, coords, vals, U = long_row_case(21)
    ctx = tk.tucker_init(*to_dev(coords, vals), dims, ranks, dtype=dtype)
    info = tk.tucker_get_info(ctx)
    assert info["nnz"] >= 256 * info["rows"][0]
    Ud = dev_list(U)
    Y = tk.ttmc_mode(ctx, 0, Ud)
    Y2 = tk.ttmc_mode(ctx, 0, Ud)
    assert torch.equal(Y, Y2)   # deterministic
    Y = Y.double().cpu().numpy()
    Yo = oracle.ttmc(coords, vals, dims, ranks, 0, U)
    assert rel_fro(Y, Yo) <= TOL_Y[dtype]
    Yc = oracle_ttmc_rounded(coords, vals, dims, ranks, 0, U, dtype)
    assert rel_fro(Y, Yc) <= 2e-6
    # rows: every non-empty row matches on its own (short rows next to long ones), empty rows are 0
    lens = np.bincount(coords[0], minlength=dims[0])
    for i in np.flatnonzero(lens):
        assert rel_fro(Y[i], Yc[i]) <= 2e-5, (i, lens[i])
    assert np.all(Y[lens == 0] == 0)


def fibered_case(seed, dims, ranks, nnz, fibers_per_row, a=1.2):
    """Order-3 nonzeros whose rows (Zipf-distributed lengths) draw their first other-mode index
    from a few values per row, so that fibers (i_n, i_f) hold many nonzeros, next to rows of one
    to three nonzeros (the structure of the recommendation-shaped workload)."""
    rng = np.random.default_rng(seed)
    i0 = synth.zipf_index(rng, dims[0], a, 3 * nnz)
    fsel = rng.integers(0, fibers_per_row, size=i0.size)
    i1 = (i0 * 7919 + fsel * 104729) % dims[1]
    i2 = rng.integers(0, dims[2], size=i0.size)
    key = (i0 * dims[1] + i1) * dims[2] + i2
    _, first = np.unique(key, return_index=True)
    first = np.sort(first)[:nnz]
    coords = np.stack([i0[first], i1[first], i2[first]]).astype(np.int32)
    vals = np.exp(rng.standard_normal(coords.shape[1]))
    U = [synth.gaussian_qr(rng, d, r) for d, r in zip(dims, ranks)]
    return coords, vals, U


TTMC3_KERNEL_CASES = [
    # dims, ranks, nnz, fibers per row
    ([3000, 400, 300], [10, 10, 10], 60000, 3),    # long fibers, Zipf rows (hot rows split over chunks)
    ([5000, 300, 200], [16, 16, 16], 40000, 2),    # full 16 x 16 tiles
    ([2000, 500, 90], [7, 12, 5], 30000, 5),       # R_f != R_in, odd ranks
    ([800, 60, 700], [4, 12, 3], 25000, 1),        # one fiber per row in mode 0
    ([9000, 9000, 50], [10, 10, 10], 20000, 40),   # mostly short rows and one-nonzero fibers
]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("case", range(len(TTMC3_KERNEL_CASES)))
def test_ttmc3_skewed_rows_and_fibers(tk, dtype, case):
    """The order-3 MFMA kernel against the oracle on every mode, on Zipf-shaped tensors with long
    and short fibers, hot rows cut across pieces next to one-nonzero rows, and several rows opening
    inside one batch; deterministic across calls; empty rows are zero."""
    dims, ranks, nnz, fpr = TTMC3_KERNEL_CASES[case]
    coords, vals, U = fibered_case(200 + case, dims, ranks, nnz, fpr)
    ctx = tk.tucker_init(*to_dev(coords, vals), dims, ranks, dtype=dtype)
    Ud = dev_list(U)
    for mode in range(3):
        Yt = tk.ttmc_mode(ctx, mode, Ud)
        assert torch.equal(Yt, tk.ttmc_mode(ctx, mode, Ud))
        Y = Yt.double().cpu().numpy()
        Yo = oracle.ttmc(coords, vals, dims, ranks, mode, U)
        assert rel_fro(Y, Yo) <= TOL_Y[dtype], (mode, rel_fro(Y, Yo))
        Yc = oracle_ttmc_rounded(coords, vals, dims, ranks, mode, U, dtype)
        assert rel_fro(Y, Yc) <= 2e-6, (mode, rel_fro(Y, Yc))
        lens = np.bincount(coords[mode], minlength=dims[mode])
        assert np.all(Y[lens == 0] == 0)
        rows = np.flatnonzero(lens)
        worst = max(rel_fro(Y[i], Yc[i]) for i in rows[:: max(1, rows.size // 200)])
        assert worst <= 2e-5, (mode, worst)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ttmc_degenerate(tk, dtype):
    # a single nonzero; all nonzeros in one row; rank-1 factors
    dims, ranks = [7, 6, 5], [1, 1, 1]
    coords = np.array([[3], [2], [4]], dtype=np.int32)
    w = synth.small_uniform(7, dims, ranks, 1)
    ctx = tk.tucker_init(*to_dev(coords, np.array([2.5])), dims, ranks, dtype=dtype)
    for mode in range(3):
        Y = tk.ttmc_mode(ctx, mode, dev_list(w.U_init)).double().cpu().numpy()
        Yo = oracle.ttmc(coords, np.array([2.5]), dims, ranks, mode, w.U_init)
        assert rel_fro(Y, Yo) < TOL_Y[dtype]
    rng = np.random.default_rng(3)
    dims, ranks = [4, 100, 100], [4, 16, 16]
    keys = rng.choice(100 * 100, size=5000, replace=False)
    coords = np.stack([np.full(5000, 2), keys // 100, keys % 100]).astype(np.int32)
    vals = rng.standard_normal(5000)
    U = [synth.gaussian_qr(rng, d, r) for d, r in zip(dims, ranks)]
    ctx = tk.tucker_init(*to_dev(coords, vals), dims, ranks, dtype=dtype)
    Y = tk.ttmc_mode(ctx, 0, dev_list(U)).double().cpu().numpy()
    Yo = oracle.ttmc(coords, vals, dims, ranks, 0, U)
    assert rel_fro(Y, Yo) < TOL_Y[dtype]
    assert np.all(Y[[0, 1, 3]] == 0)


def test_ttmc_empty_tensor(tk):
    dims, ranks = [5, 6, 7], [2, 2, 2]
    c = torch.zeros((3, 0), dtype=torch.int32, device="cuda")
    v = torch.zeros(0, dtype=torch.float64, device="cuda")
    ctx = tk.tucker_init(c, v, dims, ranks, dtype="f32")
    U = dev_list([np.ones((d, r)) for d, r in zip(dims, ranks)])
    for mode in range(3):
        Y = torch.full((dims[mode], 4), 7.0, dtype=torch.float32, device="cuda")
        tk.ttmc_mode(ctx, mode, U, Y)
        assert torch.count_nonzero(Y).item() == 0


# ------------------------------------------------------------------------------------------
# QRP, core, sweeps, reconstruct
# ------------------------------------------------------------------------------------------

def qrp_case(tk, dtype, dims, ranks, mode, nnz, seed, fat_rule=True):
    w = synth.small_uniform(seed, dims, ranks, nnz)
    ctx = make(tk, w, dtype, fat_rule)
    Yo = oracle.ttmc(w.coords, w.vals, dims, ranks, mode, w.U_init)
    yt = torch.float64 if dtype == "f64" else torch.float32
    Yd = torch.from_numpy(Yo).to(yt).cuda().contiguous()
    U, piv = tk.qrp_update(ctx, mode, Yd)
    Ue, pe = oracle.factor(Yd.double().cpu().numpy(), ranks[mode], fat_rule=fat_rule)
    return U.cpu().numpy(), piv.cpu().numpy(), Ue, pe


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", [
    ([3000, 40, 30], [12, 8, 8], 0, 20000),   # tall, Gram route (K = 64)
    ([2000, 60, 50], [16, 16, 16], 0, 30000), # tall, Gram route (K = 256)
    ([4000, 40, 40], [24, 32, 32], 0, 40000), # tall, Gram route, K = 1024, R > 16, L^T in memory
    ([3000, 40, 40], [20, 16, 16], 0, 40000), # tall, Gram route, K = 256, 16 < R <= 32: L in LDS
    ([200, 40, 30], [8, 8, 8], 0, 5000),      # small, Gram route
    ([3000, 10, 10], [10, 10, 10], 0, 30000), # Gram route, K = 100: two column blocks, ragged tile
    ([2003, 16, 8], [6, 16, 8], 0, 20000),    # Gram route, K = 128, ragged last row chunk
    ([2500, 8, 9], [9, 8, 9], 0, 20000),      # Gram route, K = 72: second block one live tile
    ([1000, 3, 3], [4, 3, 3], 0, 3000),       # Gram route, K = 9: one partly live tile
    ([400, 40, 40], [34, 6, 6], 0, 8000),     # R > 32: Householder route
    ([1500, 60, 50], [8, 40, 30], 0, 30000),  # K = 1200 > 1024: Householder route
    ([20, 30, 25, 40], [5, 4, 4, 4], 0, 6000),  # fat (K = 64 > 20): Householder on Y Y^T
    ([110, 20, 20, 20], [5, 5, 5, 5], 0, 30000),  # fat, Y Y^T 110 x 110: one workgroup, arrays in LDS
    ([200, 20, 20, 20], [6, 6, 6, 6], 0, 40000),  # fat, Y Y^T 200 x 200: beyond the LDS limit, global memory
])
def test_qrp_parity(tk, dtype, case):
    dims, ranks, mode, nnz = case
    U, piv, Ue, pe = qrp_case(tk, dtype, dims, ranks, mode, nnz, seed=200)
    assert piv.tolist() == pe.tolist()
    np.testing.assert_allclose(U, Ue, atol=1e-10)
    np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)


def test_qrp_rank_deficient_fallback(tk):
    """Y of rank 3 with R = 5: the Gram route detects the deficiency and the Householder kernel
    runs on the device.  Columns past the rank are set by round-off (parity unpinned); the first
    3 pivots, the rank-3 subspace and orthonormality are checked."""
    rng = np.random.default_rng(4)
    dims, ranks = [3000, 10, 10], [5, 8, 8]
    w = synth.small_uniform(9, dims, ranks, 100)
    ctx = make(tk, w, "f64")
    Y = rng.standard_normal((3000, 3)) @ rng.standard_normal((3, 64))
    U, piv = tk.qrp_update(ctx, 0, torch.from_numpy(Y).cuda())
    U = U.cpu().numpy()
    Ue, pe = oracle.factor(Y, 5)
    assert piv.cpu().numpy()[:3].tolist() == pe[:3].tolist()
    np.testing.assert_allclose(U.T @ U, np.eye(5), atol=1e-12)
    np.testing.assert_allclose(U[:, :3] @ (U[:, :3].T @ Y), Y, atol=1e-9 * np.abs(Y).max())


def test_qrp_fallback_grid_rank_deficient(tk):
    """As above with a Y of 5,000 x 64 entries (past the size at which the Householder QRP runs on
    the whole grid): the fallback after the Gram route's breakdown on the grid-wide kernel."""
    rng = np.random.default_rng(5)
    dims, ranks = [5000, 8, 8], [5, 8, 8]
    w = synth.small_uniform(9, dims, ranks, 100)
    ctx = make(tk, w, "f64")
    Y = rng.standard_normal((5000, 3)) @ rng.standard_normal((3, 64))
    U, piv = tk.qrp_update(ctx, 0, torch.from_numpy(Y).cuda())
    U = U.cpu().numpy()
    Ue, pe = oracle.factor(Y, 5)
    assert piv.cpu().numpy()[:3].tolist() == pe[:3].tolist()
    np.testing.assert_allclose(U.T @ U, np.eye(5), atol=1e-12)
    np.testing.assert_allclose(U[:, :3] @ (U[:, :3].T @ Y), Y, atol=1e-9 * np.abs(Y).max())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_qrp_fallback_grid_dominant_direction(tk, dtype):
    """A full-rank Y whose leading direction is 1e7 times the rest (the shape HOOI reaches on a
    tensor with a large mean): the Gram's Schur complements fall under 1e-12 of its diagonal, so
    the Gram route hands over to the grid-wide Householder QRP on Y, whose pivots, factor and
    pivot gaps match the oracle's."""
    rng = np.random.default_rng(6)
    m, K, R = 5000, 512, 8
    dims, ranks = [m, 8, 64], [R, 8, 64]
    w = synth.small_uniform(9, dims, ranks, 100)
    ctx = make(tk, w, dtype)
    Y = rng.standard_normal((m, K)) + 1e7 * np.outer(rng.random(m), rng.random(K))
    if dtype == "f32":
        Y = Y.astype(np.float32).astype(np.float64)
    yt = torch.float64 if dtype == "f64" else torch.float32
    U, piv = tk.qrp_update(ctx, 0, torch.from_numpy(Y).to(yt).cuda())
    Ue, pe, ge = oracle.factor(Y, R, gaps=True)
    assert piv.cpu().numpy().tolist() == pe.tolist()
    # the columns after the first are set by the small part of Y: error about eps * 1e7 * ||Y|| / sigma
    np.testing.assert_allclose(U.cpu().numpy(), Ue, atol=1e-7)
    np.testing.assert_allclose(np.array(tk.qrp_gaps(ctx, 0)), ge, rtol=1e-5, atol=1e-8)


def test_qrp_fat_grid(tk):
    """Fat Y (600 x 1000): the Householder QRP of Y Y^T (600 x 600) on the grid-wide kernel,
    pivots, factor and gaps against the oracle."""
    dims, ranks = [600, 40, 25], [8, 40, 25]
    w = synth.small_uniform(210, dims, ranks, 30000)
    ctx = make(tk, w, "f64")
    Yo = oracle.ttmc(w.coords, w.vals, dims, ranks, 0, w.U_init)
    U, piv = tk.qrp_update(ctx, 0, torch.from_numpy(Yo).cuda())
    Ue, pe, ge = oracle.factor(Yo, 8, fat_rule=True, gaps=True)
    assert piv.cpu().numpy().tolist() == pe.tolist()
    np.testing.assert_allclose(U.cpu().numpy(), Ue, atol=1e-10)
    np.testing.assert_allclose(np.array(tk.qrp_gaps(ctx, 0)), ge, rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("K", [64, 256])
def test_qrp_tied_norms(tk, K):
    """Columns 3 and 7 of Y have exactly equal norms (7 is 3 with half its entries negated) and the
    largest norm, so the first pivot is a tie: as in Householder QRP with column swaps, the lower
    position wins on both sides; later steps then split the pair."""
    rng = np.random.default_rng(12)
    dims, ranks = [2000, 8, K // 8], [12, 8, K // 8]
    w = synth.small_uniform(9, dims, ranks, 100)
    ctx = make(tk, w, "f64")
    Y = rng.standard_normal((2000, K))
    Y[:, 3] *= 3.0
    Y[:, 7] = Y[:, 3]
    Y[::2, 7] *= -1.0
    assert np.sum(Y[:, 3] ** 2) == np.sum(Y[:, 7] ** 2)
    U, piv = tk.qrp_update(ctx, 0, torch.from_numpy(Y).cuda())
    Ue, pe = oracle.factor(Y, 12)
    assert pe[0] == 3
    assert piv.cpu().numpy().tolist() == pe.tolist()
    np.testing.assert_allclose(U.cpu().numpy(), Ue, atol=1e-10)


@pytest.mark.parametrize("K,R", [(64, 12), (256, 16), (192, 24)])
def test_qrp_pivot_gaps(tk, K, R):
    """tucker_qrp_gaps after qrp_update equals the oracle's per-step gaps on the same Y (a near
    tie included); a tie gives 0; the fat-matrix route (Householder on Y Y^T) records the gaps of
    that matrix; the global-memory Cholesky route (K * 32 doubles above 64 KB) and a mode without
    a QRP give NaN."""
    rng = np.random.default_rng(K + R)
    dims, ranks = [2000, 8, K // 8], [R, 8, K // 8]
    w = synth.small_uniform(9, dims, ranks, 100)
    ctx = make(tk, w, "f64")
    assert all(np.isnan(tk.qrp_gaps(ctx, 1)))
    Y = rng.standard_normal((2000, K)) * np.linspace(1.0, 2.0, K)
    Y[:, 5] = Y[:, 2] * (1.0 + 1e-7)
    _, piv = tk.qrp_update(ctx, 0, torch.from_numpy(Y).cuda())
    g = tk.qrp_gaps(ctx, 0)
    _, pe, ge = oracle.factor(Y, R, gaps=True)
    assert piv.cpu().tolist() == pe.tolist()
    np.testing.assert_allclose(g, ge, atol=1e-10)
    Y[:, 7] = Y[:, K - 1]
    Y[::2, 7] *= -1.0
    Y[:, K - 1] *= 5.0
    Y[:, 7] *= 5.0
    tk.qrp_update(ctx, 0, torch.from_numpy(Y).cuda())
    assert tk.qrp_gaps(ctx, 0)[0] <= 1e-15
    # the fat-matrix route: Householder QRP of Y Y^T
    wf = synth.small_uniform(10, [20, 30, 30], [5, 6, 6], 2000)
    ctxf = make(tk, wf, "f64")
    Yf = rng.standard_normal((20, 36))
    _, pf = tk.qrp_update(ctxf, 0, torch.from_numpy(Yf).cuda())
    _, pfe, gfe = oracle.factor(Yf, 5, gaps=True)
    assert pf.cpu().tolist() == pfe.tolist()
    np.testing.assert_allclose(tk.qrp_gaps(ctxf, 0), gfe, atol=1e-10)
    wl = synth.small_uniform(11, [2000, 8, 40], [24, 8, 40], 100)
    ctxl = make(tk, wl, "f64")
    _, pl = tk.qrp_update(ctxl, 0, torch.from_numpy(rng.standard_normal((2000, 320))).cuda())
    assert all(np.isnan(tk.qrp_gaps(ctxl, 0)))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("svd", [False, True])
def test_hosvd_init_parity(tk, dtype, svd):
    """hosvd_init (sketch of every unfolding with the caller's Gaussian test factors, then QRP or
    SVD) against the oracle's hosvd_sketch on the same test factors: QRP factors to 1e-10 (FP64) /
    subspaces to 1e-5 (FP32 TTMc); SVD subspaces to 1e-9 (FP64) / 1e-5 (FP32); orthonormal
    columns.  Test factors are inputs: the library draws no random numbers."""
    dims, ranks = [300, 250, 200], [8, 6, 5]
    coords, vals, _, _ = synth.support_low_rank(41, dims, [60, 50, 40], ranks)
    vals = vals + 1e-3 * np.random.default_rng(43).standard_normal(vals.size) * np.abs(vals).mean()
    rng = np.random.default_rng(42)
    Omega = [rng.standard_normal((d, r)) for d, r in zip(dims, ranks)]
    ctx = tk.tucker_init(*to_dev(coords, vals), dims, ranks, dtype=dtype)
    Od = dev_list(Omega)
    U = [u.cpu().numpy() for u in tk.hosvd_init(ctx, Od, svd=svd)]
    Uo = oracle.hosvd_sketch(coords, vals, dims, ranks, Omega, svd=svd)
    for n in range(3):
        np.testing.assert_allclose(U[n].T @ U[n], np.eye(ranks[n]), atol=1e-12)
        sub = np.linalg.norm(U[n] @ U[n].T - Uo[n] @ Uo[n].T)
        if dtype == "f64" and not svd:
            np.testing.assert_allclose(U[n], Uo[n], atol=1e-10)
        else:
            assert sub <= (1e-9 if dtype == "f64" else 1e-5), (n, sub)
    # the test factors are left as they were
    for n in range(3):
        assert np.array_equal(Omega[n], Od[n].cpu().numpy())


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_hooi_order2_image(tk, dtype, tol):
    """Order 2 (no Kronecker product: the TTMc is a sparse-times-dense product), the image-shaped
    130 x 150 matrix of the retinal case, ranks 30 x 30, 12 sweeps: every fit within the tolerance
    of the oracle's, the final factors spanning the oracle's subspaces."""
    w = synth.image_like()
    Uo, Go, fo, _ = oracle.hooi(w.coords, w.vals, w.dims, w.ranks, w.U_init, w.sweeps)
    ctx = make(tk, w, dtype)
    U = dev_list(w.U_init)
    fits = [tk.hooi_sweep(ctx, U, sync_fit=True)[1] for _ in range(w.sweeps)]
    np.testing.assert_allclose(fits, fo, rtol=tol, atol=0)
    assert all(b >= a - 1e-12 for a, b in zip(fits, fits[1:]))   # monotone on this input
    for n in range(2):
        Un = U[n].cpu().numpy()
        assert np.linalg.norm(Un @ Un.T - Uo[n] @ Uo[n].T) <= (1e-9 if dtype == "f64" else 1e-4)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_core_fit_parity(tk, dtype):
    dims, ranks = [300, 200, 150], [8, 6, 5]
    w = synth.small_uniform(300, dims, ranks, 8000)
    ctx = make(tk, w, dtype)
    Yo = oracle.ttmc(w.coords, w.vals, dims, ranks, 2, w.U_init)
    yt = torch.float64 if dtype == "f64" else torch.float32
    Yd = torch.from_numpy(Yo).to(yt).cuda()
    G, fit = tk.core_fit(ctx, Yd, torch.from_numpy(w.U_init[2]).cuda())
    Ge = oracle.core(Yd.double().cpu().numpy(), w.U_init[2], ranks)
    assert rel_fro(G.cpu().numpy(), Ge) < 1e-13
    fe = oracle.fit(float(w.vals @ w.vals), Ge)
    assert abs(fit.item() - fe) < 1e-12


def test_hooi_sweeps_f64_200cube(tk):
    """The FP64 workload (200^3, 20,000 nnz, ranks 8, 5 sweeps): fits, factors and core match."""
    w = synth.hooi_small_f64(1)
    Uo, Go, fo, po = oracle.hooi(w.coords, w.vals, w.dims, w.ranks, w.U_init, w.sweeps)
    ctx = make(tk, w, "f64")
    U = dev_list(w.U_init)
    fits = []
    for _ in range(w.sweeps):
        G, f = tk.hooi_sweep(ctx, U, sync_fit=True)
        fits.append(f)
    np.testing.assert_allclose(fits, fo, rtol=1e-12, atol=0)
    for k in range(3):
        np.testing.assert_allclose(U[k].cpu().numpy(), Uo[k], atol=1e-10)
    assert rel_fro(G.cpu().numpy(), Go) < 1e-10


def test_hooi_run_stopping_rule(tk):
    """hooi_run: the sweeps are exactly those of repeated hooi_sweep calls, it stops at the first
    sweep whose fit changed by at most tol, and the fit sequence matches the oracle's."""
    w = synth.hooi_small_f64(1)
    tol = 1e-4   # reached at the 9th sweep on this tensor
    ctx = make(tk, w, "f64")
    U = dev_list(w.U_init)
    G, fits = tk.hooi_run(ctx, U, max_sweeps=20, tol=tol)
    assert 2 <= len(fits) < 20
    ctx2 = make(tk, w, "f64")
    U2 = dev_list(w.U_init)
    ref = [tk.hooi_sweep(ctx2, U2, sync_fit=True)[1] for _ in range(len(fits))]
    assert fits == ref
    for s in range(1, len(fits) - 1):
        assert abs(fits[s] - fits[s - 1]) > tol
    assert abs(fits[-1] - fits[-2]) <= tol
    _, _, fo, _ = oracle.hooi(w.coords, w.vals, w.dims, w.ranks, w.U_init, len(fits))
    np.testing.assert_allclose(fits, fo, rtol=1e-12, atol=0)
    with pytest.raises(tk.TuckerError) as e:
        tk.hooi_run(ctx, U, max_sweeps=0, tol=tol)
    assert e.value.status == 1


def test_hooi_sweeps_lowrank_small_f32(tk):
    """Order-3 low-rank + noise (the large FP32 workload's recipe at a small size): sweep fits match
    the FP64 oracle within 1e-5 relative; factors span the same subspaces."""
    w = synth.lowrank_f32(seed=12, dims=(3000, 2500, 2000), nnz=200000, R=16, noise=1e-3, sweeps=3)
    Uo, Go, fo, _ = oracle.hooi(w.coords, w.vals, w.dims, w.ranks, w.U_init, w.sweeps)
    ctx = make(tk, w, "f32")
    U = dev_list(w.U_init)
    fits = [tk.hooi_sweep(ctx, U, sync_fit=True)[1] for _ in range(w.sweeps)]
    rel = np.abs(np.array(fits) - fo) / np.abs(fo)
    assert np.all(rel <= 1e-5), (fits, fo)
    for k in range(3):
        P = U[k].cpu().numpy()
        assert np.linalg.norm(P @ P.T - Uo[k] @ Uo[k].T) < 1e-4


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("bf16", 1e-2)])
def test_hooi_sweeps_skewed_small(tk, dtype, tol):
    """Recommendation-shaped recipe (Zipf(1.2) modes 1-2, log-normal values, ranks 10) at a small
    size: sweep fits match the FP64 oracle within 1e-5 (FP32) / 1e-2 (BF16 operands) relative."""
    w = synth.skewed(seed=14, dims=(20000, 5000, 365), nnz=300000, R=10, dtype=dtype, sweeps=3)
    Uo, Go, fo, _ = oracle.hooi(w.coords, w.vals, w.dims, w.ranks, w.U_init, w.sweeps)
    ctx = make(tk, w, dtype)
    U = dev_list(w.U_init)
    fits = [tk.hooi_sweep(ctx, U, sync_fit=True)[1] for _ in range(w.sweeps)]
    rel = np.abs(np.array(fits) - fo) / np.abs(fo)
    assert np.all(rel <= tol), (fits, fo)


def test_hooi_order4_f32(tk):
    w = synth.order4(seed=13, dims=(400, 300, 60, 20), nnz=30000, R=4, sweeps=2)
    Uo, Go, fo, _ = oracle.hooi(w.coords, w.vals, w.dims, w.ranks, w.U_init, w.sweeps)
    ctx = make(tk, w, "f32")
    U = dev_list(w.U_init)
    fits = [tk.hooi_sweep(ctx, U, sync_fit=True)[1] for _ in range(w.sweeps)]
    np.testing.assert_allclose(fits, fo, rtol=1e-5)


# The last two modes' TTMc with shared fiber sums: (dims, ranks, nnz, what it exercises)
MEMO_CASES = [
    ([400, 300, 60, 9], [8, 8, 8, 8], 30000, "64 inner columns, about 55 nonzeros per fiber"),
    ([200, 150, 3, 2], [4, 5, 3, 2], 40000, "6 fibers of about 6,700 nonzeros, cut by chunk starts"),
    ([50, 40, 30, 20], [4, 12, 12, 16], 20000, "48 inner columns, R_{N-2} = 12, R_{N-1} = 16"),
    ([12, 10, 9, 8, 7], [2, 3, 2, 2, 2], 2500, "order 5: three inner modes"),
    ([30, 20, 500, 400], [3, 3, 4, 5], 20000, "mostly one-nonzero fibers"),
]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("case", range(len(MEMO_CASES)), ids=[c[3][:28] for c in MEMO_CASES])
def test_ttmc_memo_pair(tk, dtype, case):
    """Y_(N-2) with U and Y_(N-1) with U_{N-2} replaced (the second from the first's fiber sums)
    against the oracle's TTMc of each mode."""
    dims, ranks, nnz, _ = MEMO_CASES[case]
    w = synth.small_uniform(300 + case, dims, ranks, nnz)
    N = len(dims)
    a, b = N - 2, N - 1
    ctx = make(tk, w, dtype)
    rng = np.random.default_rng(400 + case)
    Unext = rng.standard_normal((dims[a], ranks[a]))
    Ya, Yb = tk.ttmc_memo_pair(ctx, dev_list(w.U_init), torch.from_numpy(Unext).cuda())
    U2 = list(w.U_init)
    U2[a] = Unext
    for Y, mode, U in ((Ya, a, w.U_init), (Yb, b, U2)):
        Y = Y.double().cpu().numpy()
        Yo = oracle.ttmc(w.coords, w.vals, dims, ranks, mode, U)
        assert rel_fro(Y, Yo) <= TOL_Y[dtype], (mode, rel_fro(Y, Yo))
        Yc = oracle_ttmc_rounded(w.coords, w.vals, dims, ranks, mode, U, dtype)
        assert rel_fro(Y, Yc) <= (1e-13 if dtype == "f64" else 2e-6), (mode, rel_fro(Y, Yc))
    # the fiber table is kept: a second call with other factors gives their products
    Unext2 = rng.standard_normal((dims[a], ranks[a]))
    _, Yb2 = tk.ttmc_memo_pair(ctx, dev_list(w.U_init), torch.from_numpy(Unext2).cuda())
    U2[a] = Unext2
    Yo = oracle.ttmc(w.coords, w.vals, dims, ranks, b, U2)
    assert rel_fro(Yb2.double().cpu().numpy(), Yo) <= TOL_Y[dtype]


def test_ttmc_memo_pair_unsupported(tk):
    """Order 3 has no fiber kernel: the C ABI refuses the call before any launch (the binding
    refuses it before calling)."""
    import ctypes
    from paper_2010_10638_amd import binding
    w = synth.small_uniform(320, [30, 20, 10], [3, 3, 3], 500)
    ctx = make(tk, w, "f32")
    U = dev_list(w.U_init)
    with pytest.raises(ValueError):
        tk.ttmc_memo_pair(ctx, U, U[1])
    Y = torch.empty(1 << 12, dtype=torch.float32, device="cuda")
    up = (ctypes.c_void_p * 3)(*[u.data_ptr() for u in U])
    st = binding.load_library().ttmc_memo_pair(ctx.handle, up, ctypes.c_void_p(U[1].data_ptr()),
                                               ctypes.c_void_p(Y.data_ptr()), ctypes.c_void_p(Y.data_ptr()), None)
    assert st == binding.TK_ERR_UNSUPPORTED


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_hooi_sweeps_memo(tk, dtype, tol):
    """Sweeps whose last two modes share the fiber sums (about 55 nonzeros per fiber) against the
    oracle's fits, and against the same sweeps without the sharing."""
    w = synth.small_uniform(330, [400, 300, 60, 9], [8, 8, 8, 8], 30000, sweeps=3)
    Uo, Go, fo, _ = oracle.hooi(w.coords, w.vals, w.dims, w.ranks, w.U_init, w.sweeps)
    fits = {}
    for memo in (True, False):
        ctx = make(tk, w, dtype, memo=memo)
        U = dev_list(w.U_init)
        fits[memo] = [tk.hooi_sweep(ctx, U, sync_fit=True)[1] for _ in range(w.sweeps)]
        np.testing.assert_allclose(fits[memo], fo, rtol=tol)
    np.testing.assert_allclose(fits[True], fits[False], rtol=tol)


def test_reconstruct_parity(tk):
    rng = np.random.default_rng(500)
    dims, ranks = [60, 50, 40, 30], [3, 4, 2, 5]
    w = synth.small_uniform(500, dims, ranks, 100)
    ctx = make(tk, w, "f64")
    G = rng.standard_normal(ranks)
    U = [rng.standard_normal((d, r)) for d, r in zip(dims, ranks)]
    coords = np.stack([rng.integers(0, d, 5000) for d in dims]).astype(np.int32)
    out = tk.reconstruct(ctx, torch.from_numpy(G).cuda(), dev_list(U), torch.from_numpy(coords).cuda())
    np.testing.assert_allclose(out.cpu().numpy(), oracle.reconstruct(G, U, coords), rtol=1e-13, atol=1e-13)
