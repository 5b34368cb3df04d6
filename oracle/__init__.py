"""Plain CPU oracle for sparse Tucker HOOI (FP64).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2010_10638_amd``) and never imports it.

The arithmetic lives in ``oracle.c`` (plain loops, FP64, input order).  This module only marshals
numpy arrays into it, plus three definitions that are a library primitive applied once:

* :func:`coalesce` and :func:`csf` - the mode-sorted layout, defined by a stable lexicographic
  sort (``numpy.lexsort``) of the coordinate tuples;
* :func:`svd_factor` - the SVD factor update of standard HOOI (paper Alg. 1), via LAPACK;

and, in numpy, the order-3 TTMc with BF16 matrix-core operands (:func:`ttmc_bf16_operands`:
each product x a rounded once to BF16, then one matrix product per row) and the BF16 rounding
it uses (:func:`bf16_nearest`, written from the definition of round to nearest, ties to even).

Pins (tests/test_oracle_pins.py) tie every function here to something other than itself.  The
completion loss/gradient is pinned by central finite differences and by the zero-residual case.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_LIB_DIR, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into oracle/_build/liboracle.so (plain -O2, no -ffast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        os.makedirs(_LIB_DIR, exist_ok=True)
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.orc_ttmc.argtypes = [ctypes.c_int, P, P, I64, P, P, ctypes.c_int, P, P]
        lib.orc_ttmc_threads.argtypes = [ctypes.c_int, P, P, I64, P, P, ctypes.c_int, P, P, ctypes.c_int]
        lib.orc_qrp.argtypes = [I64, I64, P, ctypes.c_int, P, P, P]
        lib.orc_factor.argtypes = [I64, I64, P, ctypes.c_int, ctypes.c_int, P, P, P]
        lib.orc_core.argtypes = [I64, I64, ctypes.c_int, P, P, P]
        lib.orc_fit.argtypes = [ctypes.c_double, P, I64]
        lib.orc_fit.restype = ctypes.c_double
        lib.orc_hooi.argtypes = [ctypes.c_int, P, P, I64, P, P, P, ctypes.c_int, ctypes.c_int, P, P, P,
                                 ctypes.c_int]
        lib.orc_reconstruct.argtypes = [ctypes.c_int, P, P, P, I64, P, P]
        lib.orc_completion.argtypes = [ctypes.c_int, P, P, P, P, I64, P, P, P, P, P]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ptr_array(mats):
    arr = (ctypes.c_void_p * len(mats))(*[m.ctypes.data for m in mats])
    return arr


def _check(st: int, what: str):
    if st != 0:
        raise RuntimeError(f"oracle {what} failed with status {st}")


def _prep(coords, vals, dims, ranks):
    coords = np.ascontiguousarray(coords, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    dims = np.ascontiguousarray(dims, dtype=np.int64)
    ranks = np.ascontiguousarray(ranks, dtype=np.int32)
    assert coords.ndim == 2 and coords.shape[0] == dims.size and coords.shape[1] == vals.size
    return coords, vals, dims, ranks


def kron_cols(ranks, mode) -> int:
    return int(np.prod([r for t, r in enumerate(ranks) if t != mode], dtype=np.int64))


def ttmc(coords, vals, dims, ranks, mode: int, U, threads: int = 1) -> np.ndarray:
    """Y_(mode) = X_(mode) (kron_{t != mode} U_t), Kronecker columns with the last mode fastest
    (Alg. 2, per-nonzero update of Sec. III-C).  threads > 1: the rows are split over that many
    host threads, each row still summed in input order (bit-identical; for timing only)."""
    coords, vals, dims, ranks = _prep(coords, vals, dims, ranks)
    U = [np.ascontiguousarray(u, dtype=np.float64) for u in U]
    Y = np.empty((int(dims[mode]), kron_cols(ranks, mode)), dtype=np.float64)
    if threads > 1:
        st = _load().orc_ttmc_threads(dims.size, _p(dims), _p(ranks), vals.size, _p(coords), _p(vals), mode,
                                      _ptr_array(U), _p(Y), int(threads))
    else:
        st = _load().orc_ttmc(dims.size, _p(dims), _p(ranks), vals.size, _p(coords), _p(vals), mode,
                              _ptr_array(U), _p(Y))
    _check(st, "ttmc")
    return Y


def bf16_nearest(x) -> np.ndarray:
    """Nearest BF16 number to each FP64 value (8 significant bits, halves to even), as FP64.

    From the definition: with x = m 2^e, 0.5 <= |m| < 1 (frexp), the BF16 numbers near x are the
    multiples of 2^(e-8); x / 2^(e-8) is exact and numpy.round takes halves to the even integer.
    For finite inputs of normal BF16 magnitude (no overflow or subnormal handling)."""
    x = np.asarray(x, dtype=np.float64)
    _, e = np.frexp(x)
    q = np.ldexp(1.0, e - 8)
    return np.where(x == 0, 0.0, np.round(x / q) * q)


def ttmc_bf16_operands(coords, vals, dims, ranks, mode: int, U) -> np.ndarray:
    """Order-3 TTMc with BF16 matrix-core operands: Y_(n)(i_n, :) = sum_p bf16(x_p a_p) kron b_p,
    where a_p and b_p are the rows U_s(i_s, :) and U_t(i_t, :) of the two other modes s < t, the
    product x_p a_p is formed exactly and rounded once to the nearest BF16 number (the reading
    the BF16 form of the Alg. 2 TTMc takes on matrix cores), and everything else is FP64.  Values
    and factors are taken as given (callers pass them already rounded to BF16).  Plain numpy: one
    (R_s x nnz_row) @ (nnz_row x R_t) product per row, flattened with t fastest."""
    coords = np.asarray(coords)
    vals = np.asarray(vals, dtype=np.float64)
    if coords.shape[0] != 3:
        raise ValueError("the BF16-operand TTMc is the order-3 form")
    s, t = [k for k in range(3) if k != mode]
    A = np.asarray(U[s], dtype=np.float64)[coords[s]]
    B = np.asarray(U[t], dtype=np.float64)[coords[t]]
    P = bf16_nearest(vals[:, None] * A)
    Y = np.zeros((int(dims[mode]), int(ranks[s]) * int(ranks[t])))
    order = np.argsort(coords[mode], kind="stable")
    rows = coords[mode][order]
    cut = np.flatnonzero(np.diff(rows)) + 1
    for seg in np.split(order, cut):
        if seg.size:
            Y[coords[mode][seg[0]]] = (P[seg].T @ B[seg]).ravel()
    return Y


def qrp(A, R: int, gaps: bool = False):
    """First R columns of Q and the pivots of Householder QRP (Sec. III-D), R steps; with gaps,
    also the relative gap between the largest and second largest trailing norm at each step."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    Q = np.empty((m, R), dtype=np.float64)
    piv = np.empty(R, dtype=np.int32)
    g = np.empty(R, dtype=np.float64)
    _check(_load().orc_qrp(m, n, _p(A), R, _p(Q), _p(piv), _p(g) if gaps else None), "qrp")
    return (Q, piv, g) if gaps else (Q, piv)


def factor(Y, R: int, fat_rule: bool = True, gaps: bool = False):
    """U_n <- QRP(Y_(n), R_n), with Y Y^T in place of a fat Y when fat_rule (Sec. III-D); with
    gaps, also the per-step relative pivot gaps."""
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    I, K = Y.shape
    U = np.empty((I, R), dtype=np.float64)
    piv = np.empty(R, dtype=np.int32)
    g = np.empty(R, dtype=np.float64)
    _check(_load().orc_factor(I, K, _p(Y), R, int(fat_rule), _p(U), _p(piv), _p(g) if gaps else None), "factor")
    return (U, piv, g) if gaps else (U, piv)


def core(Y_last, U_last, ranks) -> np.ndarray:
    """G with G_(N) = U_N^T Y_(N), returned as an N-way array (C order)."""
    Y_last = np.ascontiguousarray(Y_last, dtype=np.float64)
    U_last = np.ascontiguousarray(U_last, dtype=np.float64)
    I, K = Y_last.shape
    R = U_last.shape[1]
    G = np.empty(K * R, dtype=np.float64)
    _check(_load().orc_core(I, K, R, _p(Y_last), _p(U_last), _p(G)), "core")
    return G.reshape(tuple(int(r) for r in ranks))


def fit(normX2: float, G) -> float:
    G = np.ascontiguousarray(G, dtype=np.float64).ravel()
    return float(_load().orc_fit(float(normX2), _p(G), G.size))


def hooi(coords, vals, dims, ranks, U_init, sweeps: int, fat_rule: bool = True, threads: int = 1):
    """Alg. 2 sweeps.  Returns (U list, G, fits[sweeps], pivots[sweeps, N, maxR]).  threads > 1
    runs the TTMc row-partitioned on that many host threads (same results)."""
    coords, vals, dims, ranks = _prep(coords, vals, dims, ranks)
    U = [np.array(u, dtype=np.float64, order="C", copy=True) for u in U_init]
    N = dims.size
    G = np.empty(int(np.prod(ranks, dtype=np.int64)), dtype=np.float64)
    fits = np.empty(sweeps, dtype=np.float64)
    maxR = int(ranks.max())
    pivs = np.full((sweeps, N, maxR), -1, dtype=np.int32)
    _check(_load().orc_hooi(N, _p(dims), _p(ranks), vals.size, _p(coords), _p(vals), _ptr_array(U),
                            sweeps, int(fat_rule), _p(G), _p(fits), _p(pivs), int(threads)), "hooi")
    return U, G.reshape(tuple(int(r) for r in ranks)), fits, pivs


def reconstruct(G, U, coords) -> np.ndarray:
    """Model value at each sampled coordinate, summing over every core entry."""
    coords = np.ascontiguousarray(coords, dtype=np.int32)
    G = np.ascontiguousarray(G, dtype=np.float64)
    U = [np.ascontiguousarray(u, dtype=np.float64) for u in U]
    ranks = np.array(G.shape, dtype=np.int32)
    m = coords.shape[1]
    out = np.empty(m, dtype=np.float64)
    _check(_load().orc_reconstruct(len(U), _p(ranks), _p(G), _ptr_array(U), m, _p(coords), _p(out)),
           "reconstruct")
    return out


def completion(G, U, coords, vals, dims):
    """Sampled-entry loss sum(e^2)/(2|Omega|) and its gradients (dG, [dU_n])."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    U = [np.ascontiguousarray(u, dtype=np.float64) for u in U]
    ranks = np.array(G.shape, dtype=np.int32)
    coords, vals, dims, ranks = _prep(coords, vals, dims, ranks)
    gG = np.empty_like(G)
    gU = [np.empty_like(u) for u in U]
    loss = np.zeros(1, dtype=np.float64)
    _check(_load().orc_completion(len(U), _p(dims), _p(ranks), _p(G), _ptr_array(U), vals.size,
                                  _p(coords), _p(vals), _p(loss), _p(gG), _ptr_array(gU)),
           "completion")
    return float(loss[0]), gG, gU


# ---------------------------------------------------------------------------------------------
# Layout definitions (integer work: compared bit-exactly with the device builder).
# ---------------------------------------------------------------------------------------------

def coalesce(coords, vals, dims):
    """Distinct coordinates with duplicate values summed in input order.

    Returned in ascending lexicographic order of (i_1, ..., i_N)."""
    coords = np.asarray(coords, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    N, nnz = coords.shape
    if nnz == 0:
        return coords.astype(np.int32), vals.copy()
    order = np.lexsort(coords[::-1])  # stable; primary key i_1
    c = coords[:, order]
    v = vals[order]
    new = np.ones(nnz, dtype=bool)
    new[1:] = np.any(c[:, 1:] != c[:, :-1], axis=0)
    heads = np.flatnonzero(new)
    bounds = np.append(heads, nnz)
    out_v = v[heads].copy()
    for h in np.flatnonzero(np.diff(bounds) > 1):  # sequential sum per run, in input order
        s = v[bounds[h]]
        for q in range(bounds[h] + 1, bounds[h + 1]):
            s += v[q]
        out_v[h] = s
    return c[:, heads].astype(np.int32), out_v


def sort_modes(N: int, mode: int):
    """Key order of the mode-n sorted layout.

    Order <= 3: (i_n, other modes ascending).  Order >= 4: (i_n, i_f, remaining others ascending)
    where the fiber mode f is the last mode other than n, so that nonzeros sharing (i_n, i_f)
    are adjacent."""
    others = [t for t in range(N) if t != mode]
    if N >= 4:
        return [mode, others[-1]] + others[:-1]
    return [mode] + others


def csf(coords, vals, mode: int):
    """Mode-sorted layout of already-coalesced nonzeros.

    Returns dict(rows int32[S], ptr int64[S+1], idx int32[N-1, nnz] (other modes ascending),
    vals float64[nnz], order int64[nnz] (position in the input list))."""
    coords = np.asarray(coords, dtype=np.int64)
    N, nnz = coords.shape
    keys = sort_modes(N, mode)
    order = np.lexsort([coords[k] for k in reversed(keys)])
    c = coords[:, order]
    rows, counts = np.unique(c[mode], return_counts=True)
    ptr = np.zeros(rows.size + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(counts)
    others = [t for t in range(N) if t != mode]
    return dict(rows=rows.astype(np.int32), ptr=ptr, idx=c[others].astype(np.int32),
                vals=np.asarray(vals, dtype=np.float64)[order], order=order)


# ---------------------------------------------------------------------------------------------
# SVD factor update (standard HOOI, Alg. 1): used only by pins.
# ---------------------------------------------------------------------------------------------

def svd_factor(Y, R: int) -> np.ndarray:
    """First R left singular vectors of Y (LAPACK)."""
    u, _, _ = np.linalg.svd(np.asarray(Y, dtype=np.float64), full_matrices=False)
    return np.ascontiguousarray(u[:, :R])


def hosvd_sketch(coords, vals, dims, ranks, Omega, svd: bool = False):
    """HOSVD-style initial factors (Alg. 1's start) from a sketch: for each mode n independently,
    Y = X_(n) (kron_{k != n} Omega_k) by the TTMc, then U_n = QRP(Y, R_n) (the factor update of
    Alg. 2) or the leading R_n left singular vectors of Y (LAPACK)."""
    out = []
    for n in range(len(dims)):
        Y = ttmc(coords, vals, dims, ranks, n, Omega)
        out.append(svd_factor(Y, int(ranks[n])) if svd else factor(Y, int(ranks[n]))[0])
    return out


def hooi_svd(coords, vals, dims, ranks, U_init, sweeps: int):
    """Alg. 2 sweeps with the QRP replaced by the SVD of Alg. 1.  Returns (U, G, fits)."""
    U = [np.array(u, dtype=np.float64, copy=True) for u in U_init]
    normX2 = float(np.dot(vals, vals))
    N = len(dims)
    fits = np.empty(sweeps)
    G = None
    for s in range(sweeps):
        for n in range(N):
            Y = ttmc(coords, vals, dims, ranks, n, U)
            U[n] = svd_factor(Y, int(ranks[n]))
            if n == N - 1:
                G = core(Y, U[n], ranks)
        fits[s] = fit(normX2, G)
    return U, G, fits
