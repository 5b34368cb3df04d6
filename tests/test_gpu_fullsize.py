"""Parity at the full sizes of the workloads, in the configuration bench.py times.

The oracle cannot redo whole passes at these sizes, so the checks are ones it can afford: rows of
Y_(n) sampled and recomputed by the oracle from the nonzeros of those rows only; the QRP of the
GPU's own Y_(n) (pivot decisions in FP64 on identical input); the core and fit from the GPU's
Y_(N) and U_N; completion gradient rows sampled the same way, and the identity
<dL/dU_n, U_n> = <dL/dG, G> (the model is linear in each factor and in the core), which holds at
any size."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import cast_inputs, cast_vals, rel_fro

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_10638_amd as tk_mod
    tk_mod.load_library()
    return tk_mod


def sample_rows(rng, coords, mode, k):
    present = np.unique(coords[mode])
    return np.sort(rng.choice(present, size=min(k, present.size), replace=False))


def rows_by_oracle(w, mode, rows, U, dtype):
    """Rows `rows` of Y_(mode) from the nonzeros in those rows only (FP64 oracle)."""
    keep = np.isin(w.coords[mode], rows)
    c = w.coords[:, keep]
    v = w.vals[keep]
    Yo = oracle.ttmc(c, v, w.dims, w.ranks, mode, U)[rows]
    Yc = oracle.ttmc(c, cast_vals(v, dtype), w.dims, w.ranks, mode, cast_inputs(U, dtype))[rows]
    return Yo, Yc


def check_sampled_ttmc(tk, ctx, w, dtype, tol, seed):
    rng = np.random.default_rng(seed)
    Ud = [torch.from_numpy(u).cuda() for u in w.U_init]
    for mode in range(len(w.dims)):
        Y = tk.ttmc_mode(ctx, mode, Ud)
        rows = sample_rows(rng, w.coords, mode, 24)
        Yg = Y[torch.from_numpy(rows).cuda()].double().cpu().numpy()
        Yo, Yc = rows_by_oracle(w, mode, rows, w.U_init, dtype)
        assert rel_fro(Yg, Yo) <= tol, (mode, rel_fro(Yg, Yo))
        assert rel_fro(Yg, Yc) <= (2e-6 if dtype != "f64" else 1e-13), (mode, rel_fro(Yg, Yc))
        # rows without nonzeros are zero
        empty = np.setdiff1d(np.arange(min(w.dims[mode], 2000)), np.unique(w.coords[mode]))
        if empty.size:
            assert torch.count_nonzero(Y[torch.from_numpy(empty).cuda()]).item() == 0
        del Y


def test_lowrank_10000cube_fullsize(tk):
    """10,000^3, 10M nonzeros, ranks 16, FP32 TTMc / FP64 QRP (the bench workload)."""
    w = synth.lowrank_f32()
    c = torch.from_numpy(w.coords.astype(np.int32)).cuda()
    v = torch.from_numpy(w.vals).cuda()
    ctx = tk.tucker_init(c, v, w.dims, w.ranks, dtype="f32")
    del c, v
    check_sampled_ttmc(tk, ctx, w, "f32", 1e-5, seed=11)
    # QRP and core on the GPU's own Y_(n): identical input, pivot decisions in FP64 on both sides
    Ud = [torch.from_numpy(u).cuda() for u in w.U_init]
    for mode in range(3):
        Y = tk.ttmc_mode(ctx, mode, Ud)
        U, piv = tk.qrp_update(ctx, mode, Y)
        Ue, pe = oracle.factor(Y.double().cpu().numpy(), w.ranks[mode])
        assert piv.cpu().numpy().tolist() == pe.tolist()
        np.testing.assert_allclose(U.cpu().numpy(), Ue, atol=1e-10)
        Ud[mode] = U
    G, fit = tk.core_fit(ctx, Y, Ud[2])
    Go = oracle.core(Y.double().cpu().numpy(), Ud[2].cpu().numpy(), w.ranks)
    assert rel_fro(G.cpu().numpy(), Go) <= 1e-12
    normx2 = float(np.dot(w.vals.astype(np.float32).astype(np.float64), w.vals.astype(np.float32).astype(np.float64)))
    assert abs(float(fit.item()) - oracle.fit(normx2, Go)) <= 1e-9


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("bf16", 1e-2)])
def test_order4_fullsize(tk, dtype, tol):
    """Order 4, 50,000 x 50,000 x 5,000 x 100, 20M nonzeros, ranks 8 (K = 512, fiber-factored)."""
    w = synth.order4(dtype=dtype)
    c = torch.from_numpy(w.coords.astype(np.int32)).cuda()
    v = torch.from_numpy(w.vals).cuda()
    ctx = tk.tucker_init(c, v, w.dims, w.ranks, dtype=dtype)
    del c, v
    check_sampled_ttmc(tk, ctx, w, dtype, tol, seed=12)


def test_completion_fullsize(tk):
    """Completion, 100,000 x 100,000 x 1,000, 30M observed entries, ranks 16, FP32."""
    w = synth.completion()
    c = torch.from_numpy(w.coords.astype(np.int32)).cuda()
    v = torch.from_numpy(w.vals).cuda()
    ctx = tk.tucker_init(c, v, w.dims, w.ranks, dtype="f32")
    del c, v
    G = torch.from_numpy(w.G_init).float().cuda()
    U = [torch.from_numpy(u).float().cuda() for u in w.U_init]
    loss, gG, gU = tk.ttmc_adjoint(ctx, G, U)
    torch.cuda.synchronize()
    assert np.isfinite(loss.item()) and loss.item() > 0
    # <gU_n, U_n> = <gG, G> for every n
    ref = float((gG.double() * G.double()).sum())
    for n in range(3):
        got = float((gU[n].double() * U[n].double()).sum())
        assert abs(got - ref) <= 1e-4 * abs(ref), (n, got, ref)
    # sampled gradient rows: only the entries of those rows contribute
    rng = np.random.default_rng(13)
    r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    Gh, Uh = r32(w.G_init), [r32(u) for u in w.U_init]
    for n in range(3):
        rows = sample_rows(rng, w.coords, n, 8)
        keep = np.isin(w.coords[n], rows)
        _, _, gUo = oracle.completion(Gh, Uh, w.coords[:, keep], r32(w.vals[keep]), w.dims)
        scale = keep.sum() / w.nnz    # the oracle divides by the subset size
        got = gU[n][torch.from_numpy(rows).cuda()].double().cpu().numpy()
        assert rel_fro(got, gUo[n][rows] * scale) <= 1e-5, n
