"""GPU parity of the SVD factor update (standard HOOI, paper Alg. 1) against the oracle's LAPACK SVD,
through the C ABI, with both eigensolvers of the library: its own subspace iteration ("own", which
must converge on these cases: tucker_svd_info >= 0) and rocSOLVER's dsyevd ("lib").  Singular
vectors are compared after the library's sign convention (largest-magnitude entry of each column
positive, first one on ties) is applied to the oracle's."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_10638_amd as tk_mod
    tk_mod.load_library()
    return tk_mod


def signed(U):
    U = np.array(U, dtype=np.float64, copy=True)
    for r in range(U.shape[1]):
        i = int(np.argmax(np.abs(U[:, r])))
        if U[i, r] < 0:
            U[:, r] = -U[:, r]
    return U


def make(tk, w, dtype, svd=False, solver="own"):
    c = torch.from_numpy(np.ascontiguousarray(w.coords, dtype=np.int32)).cuda()
    v = torch.from_numpy(np.ascontiguousarray(w.vals, dtype=np.float64)).cuda()
    return tk.tucker_init(c, v, w.dims, w.ranks, dtype=dtype, svd=svd, svd_lib=(solver == "lib"))


def check_solver(tk, ctx, solver):
    steps = tk.svd_info(ctx)
    if solver == "own":
        assert steps >= 0, "subspace iteration fell back to the library solver"
    else:
        assert steps == -1


@pytest.mark.parametrize("solver", ["own", "lib"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", [
    ([3000, 40, 30], [12, 8, 8], 0, 20000),        # tall, K = 64
    ([2000, 60, 50], [16, 16, 16], 0, 30000),      # tall, K = 256
    ([900, 30, 40], [24, 16, 20], 0, 30000),       # tall, K = 320, R = 24
    ([20, 30, 25, 40], [5, 4, 4, 4], 0, 6000),     # fat (K = 64 > 20): eigenvectors of Y Y^T
    ([3000, 32, 32], [16, 32, 32], 0, 20000),      # K = 1024: block orthonormalised in global memory
    ([300, 3, 3], [8, 3, 3], 0, 2000),             # K = 9: block = whole space, odd (padded Jacobi)
    ([500, 20, 20], [1, 4, 4], 0, 5000),           # R = 1
])
def test_svd_update_parity(tk, dtype, case, solver):
    dims, ranks, mode, nnz = case
    w = synth.small_uniform(300, dims, ranks, nnz)
    ctx = make(tk, w, dtype, solver=solver)
    Yo = oracle.ttmc(w.coords, w.vals, dims, ranks, mode, w.U_init)
    yt = torch.float64 if dtype == "f64" else torch.float32
    Yd = torch.from_numpy(Yo).to(yt).cuda().contiguous()
    U = tk.svd_update(ctx, mode, Yd).cpu().numpy()
    check_solver(tk, ctx, solver)
    Ue = signed(oracle.svd_factor(Yd.double().cpu().numpy(), ranks[mode]))
    np.testing.assert_allclose(U, Ue, atol=1e-9)
    np.testing.assert_allclose(U.T @ U, np.eye(ranks[mode]), atol=1e-10)


@pytest.mark.parametrize("solver", ["own", "lib"])
def test_svd_update_planted_low_rank(tk, solver):
    """Y_(n) of a tensor with planted Tucker structure (the bench tensor's kind, smaller): a wide
    gap after the R-th singular value, K_n = 256."""
    w = synth.lowrank_f32(seed=8, dims=(2000, 300, 300), nnz=200_000, R=16)
    ctx = make(tk, w, "f32", solver=solver)
    Yo = oracle.ttmc(w.coords, w.vals, w.dims, w.ranks, 0, w.U_init)
    Yd = torch.from_numpy(Yo).float().cuda().contiguous()
    U = tk.svd_update(ctx, 0, Yd).cpu().numpy()
    check_solver(tk, ctx, solver)
    Ue = signed(oracle.svd_factor(Yd.double().cpu().numpy(), 16))
    np.testing.assert_allclose(U, Ue, atol=1e-9)


@pytest.mark.parametrize("solver", ["own", "lib"])
def test_svd_hooi_sweeps_f64(tk, solver):
    """SVD-HOOI sweeps: fits match the oracle's and never decrease (each mode step maximises
    ||U_n^T Y_(n)|| exactly, which is what makes the fit monotone for the SVD variant)."""
    dims, ranks = [120, 100, 80], [6, 5, 4]
    w = synth.small_uniform(31, dims, ranks, 15000)
    Uo, Go, fo = oracle.hooi_svd(w.coords, w.vals, dims, ranks, w.U_init, 5)
    ctx = make(tk, w, "f64", svd=True, solver=solver)
    U = [torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in w.U_init]
    fits = []
    for _ in range(5):
        G, f = tk.hooi_sweep(ctx, U, sync_fit=True)
        fits.append(f)
    check_solver(tk, ctx, solver)
    np.testing.assert_allclose(fits, fo, rtol=1e-10, atol=0)
    assert all(b >= a - 1e-13 for a, b in zip(fits, fits[1:])), fits
    for k in range(3):
        np.testing.assert_allclose(U[k].cpu().numpy(), signed(Uo[k]), atol=1e-9)
    # the core depends on the factors' signs; its norm (hence the fit) does not
    assert abs(np.linalg.norm(G.cpu().numpy()) - np.linalg.norm(Go)) <= 1e-10 * np.linalg.norm(Go)


def test_svd_update_fat_wide_rank(tk):
    """Fat Y_(n) (K = 64 > I = 40) with R = 34: past the subspace iteration's R <= 32, so dsyevd
    serves it (tucker_svd_info = -1), and the signs are fixed one column per workgroup."""
    dims, ranks = [40, 8, 8], [34, 8, 8]
    w = synth.small_uniform(77, dims, ranks, 2000)
    ctx = make(tk, w, "f64")
    Yo = oracle.ttmc(w.coords, w.vals, dims, ranks, 0, w.U_init)
    Yd = torch.from_numpy(Yo).cuda().contiguous()
    U = tk.svd_update(ctx, 0, Yd).cpu().numpy()
    assert tk.svd_info(ctx) == -1
    np.testing.assert_allclose(U, signed(oracle.svd_factor(Yo, 34)), atol=1e-9)


def test_svd_unsupported_shape(tk):
    """R_n > 32 on a tall Y has no Gram route: refused with TK_ERR_UNSUPPORTED."""
    w = synth.small_uniform(5, [400, 40, 40], [34, 6, 6], 8000)
    ctx = make(tk, w, "f64")
    Y = torch.zeros((400, 36), dtype=torch.float64, device="cuda")
    with pytest.raises(tk.TuckerError) as e:
        tk.svd_update(ctx, 0, Y)
    assert e.value.status == 5


def test_hooi_run_svd(tk):
    """hooi_run on a context with the SVD update: fits match the oracle's SVD-HOOI sweeps, never
    decrease, and the run stops at the first sweep whose fit changed by at most tol."""
    dims, ranks = [120, 100, 80], [6, 5, 4]
    w = synth.small_uniform(32, dims, ranks, 15000)
    tol = 5e-5   # the fit changes by 4.5e-5 at the 7th sweep on this tensor
    ctx = make(tk, w, "f64", svd=True)
    U = [torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in w.U_init]
    G, fits = tk.hooi_run(ctx, U, max_sweeps=12, tol=tol)
    assert len(fits) == 7, fits
    check_solver(tk, ctx, "own")
    _, _, fo = oracle.hooi_svd(w.coords, w.vals, dims, ranks, w.U_init, len(fits))
    np.testing.assert_allclose(fits, fo, rtol=1e-10, atol=0)
    assert all(b >= a - 1e-13 for a, b in zip(fits, fits[1:])), fits
    for s in range(1, len(fits) - 1):
        assert abs(fits[s] - fits[s - 1]) > tol
    assert abs(fits[-1] - fits[-2]) <= tol
