"""ctypes binding of libsptucker.so: same entry points as include/sptucker.h, taking torch tensors.

Argument marshalling only: every step of the decomposition runs in the HIP library.  The library
must be built (``python paper_2010_10638_amd/build.py`` or ``__graft_entry__.build()``); loading
fails loudly otherwise - there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libsptucker.so")

TK_OK, TK_ERR_ARG, TK_ERR_RANGE, TK_ERR_OOM, TK_ERR_HIP, TK_ERR_UNSUPPORTED = range(6)
TK_F64, TK_F32, TK_BF16 = 0, 1, 2
TK_FLAG_NO_FAT_RULE = 0x1
TK_FLAG_SVD = 0x2
TK_FLAG_SVD_LIB = 0x4
TK_FLAG_NO_MEMO = 0x8
DTYPES = {"f64": TK_F64, "f32": TK_F32, "bf16": TK_BF16}
_STATUS = {1: "TK_ERR_ARG", 2: "TK_ERR_RANGE", 3: "TK_ERR_OOM", 4: "TK_ERR_HIP", 5: "TK_ERR_UNSUPPORTED"}

EXPORTS = ("tucker_init", "tucker_get_info", "tucker_get_csf", "ttmc_mode", "ttmc_memo_pair", "qrp_update", "svd_update",
           "tucker_svd_info", "tucker_qrp_gaps", "tucker_ttmc_kernel", "core_fit", "core_fit_static",
           "hosvd_init", "hooi_sweep", "hooi_run", "reconstruct", "ttmc_adjoint", "tucker_profile", "tucker_profile_read", "tucker_free",
           "tucker_last_error")


class TuckerError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsptucker.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP library first "
                          "(python paper_2010_10638_amd/build.py)")
    lib = ctypes.CDLL(path)
    P, I, I64, U32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32
    lib.tucker_init.argtypes = [ctypes.POINTER(P), I, P, P, I64, P, P, I, U32, P]
    lib.tucker_get_info.argtypes = [P, P, P, P, P]
    lib.tucker_get_csf.argtypes = [P, I, P, P, P, P, P]
    lib.ttmc_mode.argtypes = [P, I, P, P, P]
    lib.ttmc_memo_pair.argtypes = [P, P, P, P, P, P]
    lib.qrp_update.argtypes = [P, I, P, P, P, P]
    lib.svd_update.argtypes = [P, I, P, P, P]
    lib.tucker_svd_info.argtypes = [P, P]
    lib.tucker_qrp_gaps.argtypes = [P, I, P]
    lib.tucker_ttmc_kernel.argtypes = [I, P, P, I, I, P]
    lib.core_fit.argtypes = [P, P, P, P, P, P]
    lib.core_fit_static.argtypes = [I, I64, ctypes.c_int32, I64, P, P, ctypes.c_double, P, P, P]
    lib.hooi_sweep.argtypes = [P, P, P, P, P, P]
    lib.hosvd_init.argtypes = [P, P, P, I, P]
    lib.hooi_run.argtypes = [P, P, P, I, ctypes.c_double, P, P, P]
    lib.reconstruct.argtypes = [P, P, P, I64, P, P, P]
    lib.ttmc_adjoint.argtypes = [P, I, P, P, P, P, P, P]
    lib.tucker_profile.argtypes = [P, I]
    lib.tucker_profile_read.argtypes = [P, P, P, P, P, P]
    lib.tucker_free.argtypes = [P]
    lib.tucker_free.restype = None
    lib.tucker_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("tucker_free", "tucker_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != TK_OK:
        msg = load_library().tucker_last_error().decode(errors="replace")
        raise TuckerError(status, msg)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str, shape=None, numel=None):
    """Device pointer of a contiguous CUDA tensor of the given dtype.  shape / numel: what the
    library will read or write through the pointer; a mismatch raises ValueError before any call
    into the library (a wrong-sized buffer would otherwise be an out-of-bounds device access)."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(int(x) for x in shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if numel is not None and t.numel() != int(numel):
        raise ValueError(f"{name} must hold {int(numel)} values, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _ptrs(mats, ctx, skip=None, name="U"):
    """Host array of the N factor pointers; U[k] must be float64 I_k x R_k (U[skip] is not read)."""
    n = ctx.order
    if len(mats) != n:
        raise ValueError(f"{name} must hold {n} factors")
    arr = (ctypes.c_void_p * n)()
    for k in range(n):
        if k == skip:
            arr[k] = None
            continue
        arr[k] = _dev(mats[k], torch.float64, f"{name}[{k}]", shape=(ctx.dims[k], ctx.ranks[k])).value
    return arr


class Ctx:
    """Handle returned by tucker_init; holds the shapes needed to marshal later calls."""

    def __init__(self, handle, dims, ranks, dtype):
        self.handle = ctypes.c_void_p(handle)
        self.dims = [int(d) for d in dims]
        self.ranks = [int(r) for r in ranks]
        self.dtype = dtype
        self.order = len(self.dims)

    def K(self, mode: int) -> int:
        k = 1
        for t, r in enumerate(self.ranks):
            if t != mode:
                k *= r
        return k

    @property
    def ytype(self):
        return torch.float64 if self.dtype == "f64" else torch.float32

    def __del__(self):
        if getattr(self, "handle", None) is not None and self.handle.value and _lib is not None:
            _lib.tucker_free(self.handle)
            self.handle = ctypes.c_void_p(None)


def tucker_init(coords: torch.Tensor, vals: torch.Tensor, dims, ranks, dtype: str = "f32",
                fat_rule: bool = True, svd: bool = False, svd_lib: bool = False, memo: bool = True) -> Ctx:
    """coords: int32 [N, nnz] (0-based), vals: float64 [nnz], both on the GPU.  svd: hooi_sweep
    updates the factors by svd_update instead of qrp_update.  svd_lib: svd_update uses rocSOLVER's
    dsyevd for every eigenproblem instead of the library's own subspace iteration.  memo=False:
    hooi_sweep forms every mode's TTMc from the nonzeros (no sums shared by the last two modes)."""
    lib = load_library()
    N = len(dims)
    if coords.dim() != 2 or coords.shape[0] != N:
        raise ValueError("coords must be [N, nnz]")
    nnz = int(coords.shape[1])
    if vals.numel() != nnz:
        raise ValueError("vals must have nnz entries")
    d = (ctypes.c_int64 * N)(*[int(x) for x in dims])
    r = (ctypes.c_int32 * N)(*[int(x) for x in ranks])
    h = ctypes.c_void_p()
    flags = ((0 if fat_rule else TK_FLAG_NO_FAT_RULE) | (TK_FLAG_SVD if svd else 0)
             | (TK_FLAG_SVD_LIB if svd_lib else 0) | (0 if memo else TK_FLAG_NO_MEMO))
    cp = _dev(coords, torch.int32, "coords") if nnz else None
    vp = _dev(vals, torch.float64, "vals") if nnz else None
    _check(lib.tucker_init(ctypes.byref(h), N, d, r, nnz, cp, vp, DTYPES[dtype], flags, _stream()))
    return Ctx(h.value, dims, ranks, dtype)


def tucker_get_info(ctx: Ctx) -> dict:
    lib = load_library()
    nnz = ctypes.c_int64()
    rows = (ctypes.c_int64 * ctx.order)()
    chunks = (ctypes.c_int64 * ctx.order)()
    nx2 = ctypes.c_double()
    _check(lib.tucker_get_info(ctx.handle, ctypes.byref(nnz), rows, chunks, ctypes.byref(nx2)))
    return dict(nnz=nnz.value, rows=list(rows), chunks=list(chunks), normx2=nx2.value)


def tucker_get_csf(ctx: Ctx, mode: int) -> dict:
    info = tucker_get_info(ctx)
    S, D, N = info["rows"][mode], info["nnz"], ctx.order
    dev = torch.device("cuda")
    rows = torch.empty(max(S, 1), dtype=torch.int32, device=dev)
    ptr = torch.empty(S + 1, dtype=torch.int64, device=dev)
    idx = torch.empty((N - 1, max(D, 1)), dtype=torch.int32, device=dev)
    vt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.int16}[ctx.dtype]
    vals = torch.empty(max(D, 1), dtype=vt, device=dev)
    _check(load_library().tucker_get_csf(ctx.handle, mode, ctypes.c_void_p(rows.data_ptr()),
                                         ctypes.c_void_p(ptr.data_ptr()), ctypes.c_void_p(idx.data_ptr()),
                                         ctypes.c_void_p(vals.data_ptr()), _stream()))
    return dict(rows=rows[:S], ptr=ptr, idx=idx[:, :D], vals=vals[:D])


def ttmc_mode(ctx: Ctx, mode: int, U, Y: torch.Tensor | None = None) -> torch.Tensor:
    if Y is None:
        Y = torch.empty((ctx.dims[mode], ctx.K(mode)), dtype=ctx.ytype, device="cuda")
    _mode_ok(ctx, mode)
    yp = _dev(Y, ctx.ytype, "Y", shape=(ctx.dims[mode], ctx.K(mode)))
    _check(load_library().ttmc_mode(ctx.handle, mode, _ptrs(U, ctx, skip=mode), yp, _stream()))
    return Y


def ttmc_memo_pair(ctx: Ctx, U, U_next: torch.Tensor):
    """(Y_a, Y_b): the TTMc of mode N-2 with U and of mode N-1 with U[N-2] replaced by U_next, the
    second from the first's fiber sums (order >= 4)."""
    N = ctx.order
    if N < 4:
        raise ValueError("ttmc_memo_pair needs order >= 4")
    a, b = N - 2, N - 1
    Ya = torch.empty((ctx.dims[a], ctx.K(a)), dtype=ctx.ytype, device="cuda")
    Yb = torch.empty((ctx.dims[b], ctx.K(b)), dtype=ctx.ytype, device="cuda")
    un = _dev(U_next, torch.float64, "U_next", shape=(ctx.dims[a], ctx.ranks[a]))
    _check(load_library().ttmc_memo_pair(ctx.handle, _ptrs(U, ctx, skip=a), un,
                                         _dev(Ya, ctx.ytype, "Y_a"), _dev(Yb, ctx.ytype, "Y_b"), _stream()))
    return Ya, Yb


def qrp_update(ctx: Ctx, mode: int, Y: torch.Tensor, U_out: torch.Tensor | None = None,
               piv: torch.Tensor | None = None):
    if U_out is None:
        U_out = torch.empty((ctx.dims[mode], ctx.ranks[mode]), dtype=torch.float64, device="cuda")
    if piv is None:
        piv = torch.empty(ctx.ranks[mode], dtype=torch.int32, device="cuda")
    _mode_ok(ctx, mode)
    _check(load_library().qrp_update(ctx.handle, mode, _dev(Y, ctx.ytype, "Y", shape=(ctx.dims[mode], ctx.K(mode))),
                                     _dev(U_out, torch.float64, "U_out", shape=(ctx.dims[mode], ctx.ranks[mode])),
                                     _dev(piv, torch.int32, "piv", numel=ctx.ranks[mode]), _stream()))
    return U_out, piv


def svd_update(ctx: Ctx, mode: int, Y: torch.Tensor, U_out: torch.Tensor | None = None):
    if U_out is None:
        U_out = torch.empty((ctx.dims[mode], ctx.ranks[mode]), dtype=torch.float64, device="cuda")
    _mode_ok(ctx, mode)
    _check(load_library().svd_update(ctx.handle, mode, _dev(Y, ctx.ytype, "Y", shape=(ctx.dims[mode], ctx.K(mode))),
                                     _dev(U_out, torch.float64, "U_out", shape=(ctx.dims[mode], ctx.ranks[mode])),
                                     _stream()))
    return U_out


def svd_info(ctx: Ctx) -> int:
    """Rayleigh-Ritz steps the library's subspace iteration took in the last svd_update (beyond the
    first), or -1 when rocSOLVER's dsyevd served it."""
    v = ctypes.c_int(0)
    _check(load_library().tucker_svd_info(ctx.handle, ctypes.byref(v)))
    return v.value


TTMC_KERNELS = {0: "generic", 1: "order3", 2: "fiber"}


def ttmc_kernel(dims, ranks, dtype: str, mode: int) -> str:
    """Which TTMc kernel runs for `mode` of a tensor of this shape ("generic", "order3" or
    "fiber"); host-only."""
    N = len(dims)
    d = (ctypes.c_int64 * N)(*[int(x) for x in dims])
    r = (ctypes.c_int32 * N)(*[int(x) for x in ranks])
    k = ctypes.c_int()
    _check(load_library().tucker_ttmc_kernel(N, d, r, DTYPES[dtype], int(mode), ctypes.byref(k)))
    return TTMC_KERNELS[k.value]


def qrp_gaps(ctx: Ctx, mode: int):
    """Relative pivot gaps of the mode's last QRP (list of R_mode floats; NaN: not recorded)."""
    _mode_ok(ctx, mode)
    g = (ctypes.c_double * ctx.ranks[mode])()
    _check(load_library().tucker_qrp_gaps(ctx.handle, mode, g))
    return [g[j] for j in range(ctx.ranks[mode])]


def core_fit(ctx: Ctx, Y_last: torch.Tensor, U_last: torch.Tensor, G: torch.Tensor | None = None,
             fit: torch.Tensor | None = None):
    if G is None:
        G = torch.empty(ctx.ranks, dtype=torch.float64, device="cuda")
    if fit is None:
        fit = torch.empty(1, dtype=torch.float64, device="cuda")
    n = ctx.order - 1
    _check(load_library().core_fit(ctx.handle, _dev(Y_last, ctx.ytype, "Y_last", shape=(ctx.dims[n], ctx.K(n))),
                                   _dev(U_last, torch.float64, "U_last", shape=(ctx.dims[n], ctx.ranks[n])),
                                   _dev(G, torch.float64, "G", numel=_prod(ctx.ranks)),
                                   _dev(fit, torch.float64, "fit", numel=1), _stream()))
    return G, fit


def core_fit_static(Y_last: torch.Tensor, U_last: torch.Tensor, normx2: float, G: torch.Tensor | None = None,
                    fit: torch.Tensor | None = None):
    """core_fit without a context or allocation (static per-device scratch).  Y_last: I x K float32
    or float64; U_last: I x R float64; G: R * K float64 values (C-order as core_fit's)."""
    if Y_last.dim() != 2 or U_last.dim() != 2 or Y_last.shape[0] != U_last.shape[0]:
        raise ValueError("Y_last must be I x K and U_last I x R")
    I, K = (int(x) for x in Y_last.shape)
    R = int(U_last.shape[1])
    ytype = {torch.float64: TK_F64, torch.float32: TK_F32}.get(Y_last.dtype)
    if ytype is None:
        raise TypeError("Y_last must be float32 or float64")
    if G is None:
        G = torch.empty(R * K, dtype=torch.float64, device="cuda")
    if fit is None:
        fit = torch.empty(1, dtype=torch.float64, device="cuda")
    _check(load_library().core_fit_static(ytype, I, R, K, _dev(Y_last, Y_last.dtype, "Y_last"),
                                          _dev(U_last, torch.float64, "U_last"), float(normx2),
                                          _dev(G, torch.float64, "G", numel=R * K), _dev(fit, torch.float64, "fit", numel=1),
                                          _stream()))
    return G, fit


def hosvd_init(ctx: Ctx, Omega, svd: bool = False, U_out=None):
    """HOSVD-style initial factors from a Kronecker-structured random sketch of every unfolding:
    Omega[k] (float64 I_k x R_k, the caller's random test factors) -> U_out[k] (QRP of the
    sketch, or its leading left singular vectors with svd=True)."""
    if U_out is None:
        U_out = [torch.empty((ctx.dims[k], ctx.ranks[k]), dtype=torch.float64, device="cuda")
                 for k in range(ctx.order)]
    _check(load_library().hosvd_init(ctx.handle, _ptrs(Omega, ctx, name="Omega"), _ptrs(U_out, ctx, name="U_out"),
                                     int(bool(svd)), _stream()))
    return U_out


def hooi_sweep(ctx: Ctx, U, G: torch.Tensor | None = None, fit: torch.Tensor | None = None,
               sync_fit: bool = False):
    """One sweep; U (list of float64 CUDA tensors) is updated in place.  Returns (G, fit) where fit
    is a device tensor, or a Python float when sync_fit."""
    if G is None:
        G = torch.empty(ctx.ranks, dtype=torch.float64, device="cuda")
    if fit is None:
        fit = torch.empty(1, dtype=torch.float64, device="cuda")
    host = ctypes.c_double()
    _check(load_library().hooi_sweep(ctx.handle, _ptrs(U, ctx), _dev(G, torch.float64, "G", numel=_prod(ctx.ranks)),
                                     _dev(fit, torch.float64, "fit", numel=1),
                                     ctypes.byref(host) if sync_fit else None, _stream()))
    return G, (host.value if sync_fit else fit)


def hooi_run(ctx: Ctx, U, max_sweeps: int, tol: float, G: torch.Tensor | None = None):
    """Sweeps until |fit_s - fit_{s-1}| <= tol or max_sweeps; U is updated in place.  Returns
    (G, fits) with one fit per sweep run."""
    if G is None:
        G = torch.empty(ctx.ranks, dtype=torch.float64, device="cuda")
    fits = (ctypes.c_double * max(int(max_sweeps), 1))()   # max_sweeps < 1 is the library's TK_ERR_ARG
    done = ctypes.c_int()
    _check(load_library().hooi_run(ctx.handle, _ptrs(U, ctx), _dev(G, torch.float64, "G", numel=_prod(ctx.ranks)),
                                   int(max_sweeps),
                                   float(tol), fits, ctypes.byref(done), _stream()))
    return G, [fits[i] for i in range(done.value)]


def reconstruct(ctx: Ctx, G: torch.Tensor, U, coords: torch.Tensor, out: torch.Tensor | None = None):
    if coords.dim() != 2 or coords.shape[0] != ctx.order:
        raise ValueError(f"coords must be [{ctx.order}, m]")
    m = int(coords.shape[1])
    if out is None:
        out = torch.empty(m, dtype=torch.float64, device="cuda")
    if m == 0:
        return out
    _check(load_library().reconstruct(ctx.handle, _dev(G, torch.float64, "G", numel=_prod(ctx.ranks)),
                                      _ptrs(U, ctx), m, _dev(coords, torch.int32, "coords"),
                                      _dev(out, torch.float64, "out", numel=m), _stream()))
    return out


def ttmc_adjoint(ctx: Ctx, G: torch.Tensor, U, loss=None, gG=None, gU=None):
    """Loss and gradients of the sampled-entry Tucker model over ctx's entries (completion).

    G: [R_1, ..., R_N] and U[k]: [I_k, R_k], in the context's TTMc type (float32 for an "f32"
    context, float64 for "f64").  Returns (loss [1], gG like G, [gU_k like U_k])."""
    lib = load_library()
    if ctx.dtype not in ("f32", "f64"):
        raise TuckerError(TK_ERR_UNSUPPORTED, "ttmc_adjoint needs an f32 or f64 context")
    dt = ctx.ytype
    N = ctx.order
    if loss is None:
        loss = torch.empty(1, dtype=dt, device="cuda")
    if gG is None:
        gG = torch.empty(ctx.ranks, dtype=dt, device="cuda")
    if gU is None:
        gU = [torch.empty((ctx.dims[k], ctx.ranks[k]), dtype=dt, device="cuda") for k in range(N)]
    for k in range(N):
        if tuple(U[k].shape) != (ctx.dims[k], ctx.ranks[k]) or tuple(gU[k].shape) != (ctx.dims[k], ctx.ranks[k]):
            raise ValueError(f"U[{k}] / gU[{k}] must be {ctx.dims[k]} x {ctx.ranks[k]}")
    if len(U) != N or len(gU) != N:
        raise ValueError(f"U / gU must hold {N} factors")
    if G.numel() != gG.numel() or G.numel() != _prod(ctx.ranks):
        raise ValueError("G / gG must hold prod(ranks) values")
    if loss.numel() != 1:
        raise ValueError("loss must hold one value")
    up = (ctypes.c_void_p * N)(*[_dev(U[k], dt, f"U[{k}]").value for k in range(N)])
    gp = (ctypes.c_void_p * N)(*[_dev(gU[k], dt, f"gU[{k}]").value for k in range(N)])
    _check(lib.ttmc_adjoint(ctx.handle, DTYPES[ctx.dtype], _dev(G, dt, "G"), up, _dev(loss, dt, "loss"),
                            _dev(gG, dt, "gG"), gp, _stream()))
    return loss, gG, gU


def _mode_ok(ctx: Ctx, mode: int):
    if not 0 <= int(mode) < ctx.order:
        raise ValueError(f"mode must be in [0, {ctx.order})")


def _prod(xs):
    p = 1
    for x in xs:
        p *= int(x)
    return p


def tucker_profile(ctx: Ctx, capacity: int):
    _check(load_library().tucker_profile(ctx.handle, int(capacity)))


def tucker_profile_read(ctx: Ctx) -> dict:
    N = ctx.order
    tt = (ctypes.c_double * N)()
    tk = (ctypes.c_double * N)()
    qq = (ctypes.c_double * N)()
    cc = ctypes.c_double()
    ns = ctypes.c_int64()
    _check(load_library().tucker_profile_read(ctx.handle, tt, tk, qq, ctypes.byref(cc), ctypes.byref(ns)))
    return dict(ttmc_ms=list(tt), ttmc_kernel_ms=list(tk), qrp_ms=list(qq), core_ms=cc.value, sweeps=ns.value)


def tucker_free(ctx: Ctx):
    if ctx.handle.value:
        load_library().tucker_free(ctx.handle)
        ctx.handle = ctypes.c_void_p(None)
