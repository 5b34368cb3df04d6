"""The allocation-free entry point core_fit_static, called through the C ABI, against core_fit."""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_10638_amd as tk_mod
    tk_mod.load_library()
    return tk_mod


def last_mode_inputs(tk, seed, dims, ranks, nnz, dtype):
    """Y_(N) and U_N of one sweep's last mode (TTMc + QRP on the GPU) and the context's ||X||^2."""
    w = synth.small_uniform(seed, dims, ranks, nnz)
    c = torch.from_numpy(w.coords).cuda()
    v = torch.from_numpy(w.vals).cuda()
    ctx = tk.tucker_init(c, v, dims, ranks, dtype=dtype)
    U = [torch.from_numpy(u).cuda() for u in w.U_init]
    n = len(dims) - 1
    Y = tk.ttmc_mode(ctx, n, U)
    U[n], _ = tk.qrp_update(ctx, n, Y)
    return ctx, Y, U[n], tk.tucker_get_info(ctx)["normx2"]


def call_static(lib, Y, U, normx2, G, fit):
    ytype = 0 if Y.dtype == torch.float64 else 1
    I, K = Y.shape
    R = U.shape[1]
    st = lib.core_fit_static(ytype, I, R, K, ctypes.c_void_p(Y.data_ptr()), ctypes.c_void_p(U.data_ptr()),
                             ctypes.c_double(normx2), ctypes.c_void_p(G.data_ptr()),
                             ctypes.c_void_p(fit.data_ptr()),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_core_fit_static_matches_core_fit(tk, dtype):
    """Two calls in a row on one device, the second with a smaller input: each matches core_fit
    (the same kernels; the slab split may differ, so FP64 results agree to rounding)."""
    lib = tk.load_library()
    for seed, dims, ranks, nnz in [(71, [300, 250, 4000], [8, 12, 16], 60000), (72, [90, 80, 70], [4, 5, 6], 3000)]:
        ctx, Y, U, normx2 = last_mode_inputs(tk, seed, dims, ranks, nnz, dtype)
        G_ref, fit_ref = tk.core_fit(ctx, Y, U)
        R, K = U.shape[1], Y.shape[1]
        G = torch.full((R * K,), float("nan"), dtype=torch.float64, device="cuda")
        fit = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        assert call_static(lib, Y, U, normx2, G, fit) == 0
        torch.cuda.synchronize()
        np.testing.assert_allclose(G.cpu().numpy(), G_ref.reshape(-1).cpu().numpy(), rtol=1e-13, atol=1e-13)
        assert abs(fit.item() - fit_ref.item()) <= 1e-12 * max(1.0, abs(fit_ref.item()))


def test_core_fit_static_rejects_oversize(tk):
    """R * K above the static scratch is refused on the host (no launch)."""
    lib = tk.load_library()
    Y = torch.zeros((2, 4096), dtype=torch.float32, device="cuda")
    U = torch.zeros((2, 512), dtype=torch.float64, device="cuda")
    G = torch.zeros(1, dtype=torch.float64, device="cuda")
    fit = torch.zeros(1, dtype=torch.float64, device="cuda")
    assert call_static(lib, Y, U, 1.0, G, fit) == 5
    assert b"static scratch" in lib.tucker_last_error()
