"""Tucker completion through the adjoint TTMc (C ABI ttmc_adjoint and the autograd Function),
against the FP64 oracle's loss and gradients (which the CPU tests pin to finite differences)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import rel_fro

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_10638_amd as tk_mod
    tk_mod.load_library()
    return tk_mod


def instance(seed, dims, ranks, nnz):
    """Uniform random entries (values U(0,1)); parameters at an independent random point."""
    w = synth.small_uniform(seed, dims, ranks, nnz)
    rng = np.random.default_rng(seed + 1000)
    G = rng.standard_normal(tuple(ranks))
    U = [rng.standard_normal((d, r)) / np.sqrt(r) for d, r in zip(dims, ranks)]
    return w, G, U


def run(tk, w, G, U, dtype):
    tt = torch.float64 if dtype == "f64" else torch.float32
    c = torch.from_numpy(np.ascontiguousarray(w.coords, dtype=np.int32)).cuda()
    v = torch.from_numpy(np.ascontiguousarray(w.vals, dtype=np.float64)).cuda()
    ctx = tk.tucker_init(c, v, w.dims, w.ranks, dtype=dtype)
    Gd = torch.from_numpy(G).to(tt).cuda()
    Ud = [torch.from_numpy(u).to(tt).cuda() for u in U]
    loss, gG, gU = tk.ttmc_adjoint(ctx, Gd, Ud)
    torch.cuda.synchronize()
    return ctx, float(loss.item()), gG.double().cpu().numpy(), [g.double().cpu().numpy() for g in gU]


CASES = [
    ([30, 30, 30], [16, 16, 16], 2000),     # the gradient-check instance (MFMA TTMc path)
    ([200, 150, 120], [8, 6, 5], 6000),     # unequal ranks, order 3
    ([20, 18, 16, 14], [3, 4, 2, 3], 3000), # order 4 (generic TTMc)
    ([300, 250], [6, 6], 4000),             # order 2
    ([60, 50, 40], [20, 3, 17], 4000),      # R > 16 (generic TTMc path for order 3)
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_adjoint_f64_matches_oracle(tk, case):
    dims, ranks, nnz = CASES[case]
    w, G, U = instance(700 + case, dims, ranks, nnz)
    _, loss, gG, gU = run(tk, w, G, U, "f64")
    lo, gGo, gUo = oracle.completion(G, U, w.coords, w.vals, dims)
    assert abs(loss - lo) <= 1e-12 * abs(lo)
    assert rel_fro(gG, gGo) <= 1e-11
    for n in range(len(dims)):
        assert rel_fro(gU[n], gUo[n]) <= 1e-11, n


@pytest.mark.parametrize("case", [0, 1])
def test_adjoint_f32_within_1e5(tk, case):
    dims, ranks, nnz = CASES[case]
    w, G, U = instance(800 + case, dims, ranks, nnz)
    _, loss, gG, gU = run(tk, w, G, U, "f32")
    # the oracle on the FP32-rounded inputs: only the FP32 arithmetic differs
    r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    lo, gGo, gUo = oracle.completion(r32(G), [r32(u) for u in U], w.coords, r32(w.vals), dims)
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    assert rel_fro(gG, gGo) <= 1e-5
    for n in range(len(dims)):
        assert rel_fro(gU[n], gUo[n]) <= 1e-5, n


# FP32 order-3 instances on which every mode takes the matrix-core TTMc, so the residuals are
# formed inside it: (dims, ranks, nnz, what the layout exercises)
FUSED_CASES = [
    ([16, 400, 400], [16, 16, 16], 30000, "rows of ~1,900 entries cut into pieces (carry slots)"),
    ([20000, 50, 40], [16, 5, 9], 8000, "rows of 1-3 entries: tiles and batches spanning many rows"),
    ([700, 900, 64], [7, 16, 3], 50000, "unequal ranks below 16 (zero-padded blocks), ragged rows"),
    ([40, 40, 24], [8, 16, 8], 38400, "every coordinate observed (no padding in any row)"),
]


def fused_instance(case):
    dims, ranks, nnz, _ = FUSED_CASES[case]
    rng = np.random.default_rng(850 + case)
    if nnz == int(np.prod(dims)):
        coords = np.stack(np.unravel_index(np.arange(nnz), dims)).astype(np.int32)
    else:
        coords = np.stack([rng.integers(0, d, nnz) for d in dims]).astype(np.int32)
    vals = rng.standard_normal(nnz)
    vals[::7] = 0.0                      # observed zeros are entries like any other
    coords, vals = oracle.coalesce(coords, vals, dims)
    w = synth.Workload("fused", dims, ranks, np.ascontiguousarray(coords), vals, None)
    G = rng.standard_normal(tuple(ranks))
    U = [rng.standard_normal((d, r)) / np.sqrt(r) for d, r in zip(dims, ranks)]
    return w, G, U


@pytest.mark.parametrize("case", range(len(FUSED_CASES)), ids=[c[3].split(":")[0][:24] for c in FUSED_CASES])
def test_adjoint_f32_residual_form(tk, case):
    """The residual-in-TTMc path (order 3, FP32, every mode on the matrix-core kernel) against the
    oracle on the FP32-rounded inputs: loss and every gradient within 1e-5."""
    w, G, U = fused_instance(case)
    for n in range(3):
        assert tk.ttmc_kernel(w.dims, w.ranks, "f32", n) == "order3"
    _, loss, gG, gU = run(tk, w, G, U, "f32")
    r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    lo, gGo, gUo = oracle.completion(r32(G), [r32(u) for u in U], w.coords, r32(w.vals), w.dims)
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    assert rel_fro(gG, gGo) <= 1e-5
    for n in range(3):
        assert rel_fro(gU[n], gUo[n]) <= 1e-5, n


def test_adjoint_f32_repeated_calls_agree(tk):
    """Two calls on one context give bit-identical results (fixed summation order)."""
    w, G, U = fused_instance(1)
    ctx, l1, gG1, gU1 = run(tk, w, G, U, "f32")
    Gd = torch.from_numpy(G).float().cuda()
    Ud = [torch.from_numpy(u).float().cuda() for u in U]
    l2, gG2, gU2 = tk.ttmc_adjoint(ctx, Gd, Ud)
    assert float(l2.item()) == l1
    assert np.array_equal(gG2.double().cpu().numpy(), gG1)
    for a, b in zip(gU2, gU1):
        assert np.array_equal(a.double().cpu().numpy(), b)


def test_adjoint_duplicates_and_zero_residual(tk):
    """Duplicates are summed at init (|Omega| counts distinct entries); values equal to the model
    give a zero loss and zero gradients."""
    dims, ranks = [40, 30, 20], [4, 3, 5]
    w, G, U = instance(901, dims, ranks, 1500)
    xh = oracle.reconstruct(G, U, w.coords)
    half = xh / 2
    c = np.concatenate([w.coords, w.coords], axis=1)
    v = np.concatenate([half, xh - half])
    w2 = synth.Workload("dup", dims, ranks, c, v, U)
    _, loss, gG, gU = run(tk, w2, G, U, "f64")
    assert abs(loss) <= 1e-28
    assert np.abs(gG).max() <= 1e-14 and max(np.abs(g).max() for g in gU) <= 1e-14


def test_adjoint_empty(tk):
    dims, ranks = [10, 9, 8], [2, 3, 2]
    w = synth.Workload("empty", dims, ranks, np.zeros((3, 0), np.int32), np.zeros(0), [np.ones((d, r)) for d, r in zip(dims, ranks)])
    _, loss, gG, gU = run(tk, w, np.ones(ranks), w.U_init, "f64")
    assert loss == 0.0 and not gG.any() and not any(g.any() for g in gU)


def test_adjoint_dtype_mismatch(tk):
    """The binding refuses tensors of the wrong type; the C ABI refuses a dtype argument that
    differs from the context's (before any launch)."""
    import ctypes
    from paper_2010_10638_amd import binding
    dims, ranks = [10, 9, 8], [2, 3, 2]
    w, G, U = instance(902, dims, ranks, 100)
    ctx, *_ = run(tk, w, G, U, "f64")
    with pytest.raises(TypeError):
        tk.ttmc_adjoint(ctx, torch.from_numpy(G).float().cuda(), [torch.from_numpy(u).float().cuda() for u in U])
    Gd = torch.from_numpy(G).cuda()
    Ud = [torch.from_numpy(u).cuda() for u in U]
    gG, gU, loss = torch.empty_like(Gd), [torch.empty_like(u) for u in Ud], torch.empty(1, dtype=torch.float64, device="cuda")
    up = (ctypes.c_void_p * 3)(*[u.data_ptr() for u in Ud])
    gp = (ctypes.c_void_p * 3)(*[g.data_ptr() for g in gU])
    st = binding.load_library().ttmc_adjoint(ctx.handle, binding.TK_F32, ctypes.c_void_p(Gd.data_ptr()), up,
                                             ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(gG.data_ptr()), gp, None)
    assert st == binding.TK_ERR_ARG


def test_autograd_gradcheck(tk):
    """torch.autograd.gradcheck of the Function on the FP64 30^3 / 2,000-entry instance (R = 16)."""
    w, G, U = instance(700, [30, 30, 30], [16, 16, 16], 2000)
    c = torch.from_numpy(w.coords.astype(np.int32)).cuda()
    v = torch.from_numpy(w.vals).cuda()
    ctx = tk.tucker_init(c, v, w.dims, w.ranks, dtype="f64")
    params = [torch.from_numpy(G).cuda().requires_grad_()] + [torch.from_numpy(u).cuda().requires_grad_() for u in U]
    f = lambda g, *us: tk.completion_loss(ctx, g, us)
    assert torch.autograd.gradcheck(f, params, eps=1e-6, atol=1e-8, rtol=1e-5, fast_mode=True)


def test_adam_decreases_loss(tk):
    """A few Adam steps on a planted completion instance (FP32): the loss falls monotonically at
    first and ends well below its start."""
    w = synth.completion(dims=(2000, 1500, 300), nnz=200_000, R=8, noise=1e-2)
    c = torch.from_numpy(w.coords.astype(np.int32)).cuda()
    v = torch.from_numpy(w.vals).cuda()
    ctx = tk.tucker_init(c, v, w.dims, w.ranks, dtype="f32")
    G = torch.from_numpy(w.G_init).float().cuda().requires_grad_()
    U = [torch.from_numpy(u).float().cuda().requires_grad_() for u in w.U_init]
    opt = torch.optim.Adam([G] + U, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    losses = []
    for _ in range(60):
        opt.zero_grad()
        loss = tk.completion_loss(ctx, G, U)
        loss.backward()
        opt.step()
        losses.append(float(loss.item()))
    assert all(b < a for a, b in zip(losses[:10], losses[1:11]))
    assert losses[-1] < 0.5 * losses[0]
