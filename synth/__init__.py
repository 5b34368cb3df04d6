"""Seeded synthetic inputs for the sparse Tucker workloads.

This module only draws inputs: coordinates, values, planted models and initial factors.  It holds
none of the decomposition's arithmetic and is shared, unchanged, by the oracle side and the GPU
side, so both always receive identical arrays.  The one piece of algebra here is the evaluation
of a *planted* Tucker model at the sampled coordinates, which produces input values for the
low-rank workloads; it is written with numpy matmuls and is not used to check any result.

Every workload is defined by its seed; sub-streams for coordinates, values, the planted model and
the initial factors come from ``numpy.random.SeedSequence(seed).spawn(4)`` with the PCG64 generator.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    dims: list
    ranks: list
    coords: np.ndarray          # int32 [N, nnz], 0-based, distinct
    vals: np.ndarray            # float64 [nnz]
    U_init: list                # float64 [I_k, R_k] per mode
    sweeps: int = 1
    dtype: str = "f64"          # TTMc arithmetic: "f64", "f32" or "bf16"
    G_init: np.ndarray | None = None   # completion workloads only
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.vals.size)

    @property
    def order(self) -> int:
        return len(self.dims)


def streams(seed: int):
    """Four independent PCG64 generators: coordinates, values, model, init."""
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(4)]


def gaussian_qr(rng, I: int, R: int) -> np.ndarray:
    """Random orthonormal I x R matrix: Q factor of an I x R standard Gaussian matrix."""
    q, _ = np.linalg.qr(rng.standard_normal((I, R)))
    return np.ascontiguousarray(q)


def _unravel(keys: np.ndarray, dims) -> np.ndarray:
    out = np.empty((len(dims), keys.size), dtype=np.int32)
    rem = keys.copy()
    for t in range(len(dims) - 1, -1, -1):
        out[t] = rem % dims[t]
        rem //= dims[t]
    return out


def _ravel(cols, dims) -> np.ndarray:
    key = np.zeros(cols[0].size, dtype=np.int64)
    for t, d in enumerate(dims):
        key = key * np.int64(d) + cols[t].astype(np.int64)
    return key


def _distinct_in_draw_order(draw, nnz: int, batch: int) -> np.ndarray:
    """Keep drawing batches of linear keys until nnz distinct ones exist; return the first nnz
    distinct keys in the order they were first drawn."""
    keys = np.empty(0, dtype=np.int64)
    while True:
        keys = np.concatenate([keys, draw(batch)])
        uniq, first = np.unique(keys, return_index=True)
        if uniq.size >= nnz:
            first.sort()
            return keys[first[:nnz]]
        keys = keys[np.sort(first)]


def uniform_coords(rng, dims, nnz: int) -> np.ndarray:
    """nnz distinct coordinates, each drawn uniformly over the index space."""
    total = int(np.prod(np.array(dims, dtype=np.float64)))
    if nnz == 0:
        return np.zeros((len(dims), 0), dtype=np.int32)
    if total <= 2 ** 31:
        keys = rng.choice(total, size=nnz, replace=False).astype(np.int64)
        return _unravel(keys, dims)

    def draw(b):
        return _ravel([rng.integers(0, d, size=b, dtype=np.int64) for d in dims], dims)

    keys = _distinct_in_draw_order(draw, nnz, nnz + nnz // 50 + 1024)
    return _unravel(keys, dims)


def zipf_index(rng, I: int, a: float, size: int) -> np.ndarray:
    """Bounded Zipf: P(k) proportional to k^-a for k = 1..I, returned as index k-1 (hot rows first)."""
    w = np.arange(1, I + 1, dtype=np.float64) ** (-a)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(size)
    return np.minimum(np.searchsorted(cdf, u, side="right"), I - 1).astype(np.int64)


def planted_values(coords, G, factors, batch: int = 1 << 18) -> np.ndarray:
    """Planted model G x_1 F_1 x_2 F_2 x_3 F_3 evaluated at order-3 coordinates (input synthesis)."""
    assert len(factors) == 3
    R1, R2, R3 = G.shape
    G1 = G.reshape(R1, R2 * R3)
    nnz = coords.shape[1]
    out = np.empty(nnz, dtype=np.float64)
    for s in range(0, nnz, batch):
        e = min(nnz, s + batch)
        T = (factors[0][coords[0, s:e]] @ G1).reshape(e - s, R2, R3)
        T = np.einsum("pbc,pc->pb", T, factors[2][coords[2, s:e]])
        out[s:e] = np.einsum("pb,pb->p", T, factors[1][coords[1, s:e]])
    return out


# ---------------------------------------------------------------------------------------------
# The five workloads.  Sizes follow the configurations this build is measured on.
# ---------------------------------------------------------------------------------------------

def hooi_small_f64(seed: int = 1) -> Workload:
    """Order-3 200x200x200, 20,000 distinct uniform coordinates, values U(0,1), ranks 8x8x8,
    Gaussian-QR init, 5 sweeps, FP64 throughout (the paper's 200^3 synthetic shape)."""
    rc, rv, _, ri = streams(seed)
    dims, ranks = [200, 200, 200], [8, 8, 8]
    coords = uniform_coords(rc, dims, 20000)
    vals = rv.random(coords.shape[1])
    U = [gaussian_qr(ri, d, r) for d, r in zip(dims, ranks)]
    return Workload("hooi_200cube_r8_f64", dims, ranks, coords, vals, U, sweeps=5, dtype="f64")


def lowrank_f32(seed: int = 2, dims=(10000, 10000, 10000), nnz: int = 10_000_000, R: int = 16,
                noise: float = 1e-3, sweeps: int = 10) -> Workload:
    """Order-3 entries sampled uniformly from a Tucker tensor with N(0,1) core R^3 and Gaussian-QR
    factors, plus N(0, noise) (standard deviation); ranks R; FP32 TTMc, FP64 QRP."""
    rc, rv, rm, ri = streams(seed)
    dims = list(dims)
    ranks = [R] * 3
    coords = uniform_coords(rc, dims, nnz)
    G = rm.standard_normal((R, R, R))
    F = [gaussian_qr(rm, d, R) for d in dims]
    vals = planted_values(coords, G, F) + noise * rv.standard_normal(coords.shape[1])
    U = [gaussian_qr(ri, d, R) for d in dims]
    name = "lowrank_%dx%dx%d_nnz%d_r%d_f32" % (dims[0], dims[1], dims[2], nnz, R)
    return Workload(name, dims, ranks, coords, vals, U, sweeps=sweeps, dtype="f32")


def skewed(seed: int = 3, dims=(500000, 100000, 365), nnz: int = 50_000_000, R: int = 10,
           a: float = 1.2, dtype: str = "bf16", sweeps: int = 5) -> Workload:
    """Recommendation-shaped order-3 tensor: Zipf(a) indices on modes 1-2 (hot rows first),
    uniform on mode 3, log-normal(0,1) values, nnz distinct coordinates kept in first-draw order."""
    rc, rv, _, ri = streams(seed)
    dims = list(dims)

    def draw(b):
        i1 = zipf_index(rc, dims[0], a, b)
        i2 = zipf_index(rc, dims[1], a, b)
        i3 = rc.integers(0, dims[2], size=b, dtype=np.int64)
        return _ravel([i1, i2, i3], dims)

    # one batch of 2.6 x nnz draws normally holds nnz distinct coordinates (about 60% of Zipf
    # draws collide at these sizes); the loop tops up otherwise
    keys = _distinct_in_draw_order(draw, nnz, max(1024, int(2.6 * nnz)))
    coords = _unravel(keys, dims)
    vals = np.exp(rv.standard_normal(nnz))
    U = [gaussian_qr(ri, d, R) for d in dims]
    name = "zipf_%dx%dx%d_nnz%d_r%d_%s" % (dims[0], dims[1], dims[2], nnz, R, dtype)
    return Workload(name, dims, [R] * 3, coords, vals, U, sweeps=sweeps, dtype=dtype)


def order4(seed: int = 4, dims=(50000, 50000, 5000, 100), nnz: int = 20_000_000, R: int = 8,
           dtype: str = "f32", sweeps: int = 5) -> Workload:
    """Order-4 tensor with uniform distinct coordinates, values U(0,1), ranks R^4."""
    rc, rv, _, ri = streams(seed)
    dims = list(dims)
    coords = uniform_coords(rc, dims, nnz)
    vals = rv.random(coords.shape[1])
    U = [gaussian_qr(ri, d, R) for d in dims]
    name = "order4_%s_nnz%d_r%d_%s" % ("x".join(map(str, dims)), nnz, R, dtype)
    return Workload(name, dims, [R] * 4, coords, vals, U, sweeps=sweeps, dtype=dtype)


def completion(seed: int = 5, dims=(100000, 100000, 1000), nnz: int = 30_000_000, R: int = 16,
               noise: float = 1e-2, dtype: str = "f32") -> Workload:
    """Observed entries of a planted rank-R^3 Tucker model (core N(0,1), factor entries
    N(0, 1/R)) plus N(0, noise); initial core N(0,1) and factors N(0, 1/R) from a separate stream."""
    rc, rv, rm, ri = streams(seed)
    dims = list(dims)
    coords = uniform_coords(rc, dims, nnz)
    G = rm.standard_normal((R, R, R))
    F = [rm.standard_normal((d, R)) / np.sqrt(R) for d in dims]
    vals = planted_values(coords, G, F) + noise * rv.standard_normal(coords.shape[1])
    U = [ri.standard_normal((d, R)) / np.sqrt(R) for d in dims]
    G0 = ri.standard_normal((R, R, R))
    name = "completion_%dx%dx%d_nnz%d_r%d_%s" % (dims[0], dims[1], dims[2], nnz, R, dtype)
    return Workload(name, dims, [R] * 3, coords, vals, U, dtype=dtype, G_init=G0)


def image_like(seed: int = 6, shape=(130, 150), R=(30, 30), sweeps: int = 12, dtype: str = "f64") -> Workload:
    """Order-2 sparse matrix shaped like a thresholded fundus photograph (the retinal-image case
    of Sec. IV-C, whose data is not available): a smooth radial background, a few dark blobs and
    bright vessel-like curves branching from one point, intensities in [0, 1]; pixels below a
    threshold are dropped (about half remain).  Ranks 30 x 30 (a rank above the other mode's rank
    would exceed K_n = R_other), Gaussian-QR init, 12 sweeps."""
    rc, rv, rm, ri = streams(seed)
    H, W = shape
    yy, xx = np.meshgrid(np.arange(H) / H, np.arange(W) / W, indexing="ij")
    img = 0.55 * np.exp(-((yy - 0.5) ** 2 + (xx - 0.5) ** 2) / 0.18)
    for _ in range(5):                                   # darker spots
        cy, cx, r = rm.random(), rm.random(), 0.02 + 0.05 * rm.random()
        img -= 0.2 * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * r * r))
    oy, ox = 0.45 + 0.1 * rm.random(), 0.35 + 0.1 * rm.random()
    for _ in range(9):                                   # vessels: bent curves from the disc
        ang = rm.uniform(0, 2 * np.pi)
        bend = rm.uniform(-1.5, 1.5)
        t = np.linspace(0, 0.7, 400)
        cy = oy + t * np.sin(ang + bend * t)
        cx = ox + t * np.cos(ang + bend * t)
        for py, px in zip(cy, cx):
            img += 0.004 * np.exp(-((yy - py) ** 2 + (xx - px) ** 2) / (2 * 0.006 ** 2))
    img = np.clip(img + 0.03 * rv.standard_normal(img.shape), 0.0, 1.0)
    keep = img > np.quantile(img, 0.5)
    coords = np.stack(np.nonzero(keep)).astype(np.int32)
    vals = img[keep].astype(np.float64)
    U = [gaussian_qr(ri, d, r) for d, r in zip(shape, R)]
    return Workload("image_%dx%d_r%d_%s" % (H, W, R[0], dtype), list(shape), list(R), coords, vals, U,
                    sweeps=sweeps, dtype=dtype)


# ---------------------------------------------------------------------------------------------
# Small structured inputs used by the pins.
# ---------------------------------------------------------------------------------------------

def small_uniform(seed: int, dims, ranks, nnz: int, dtype: str = "f64", sweeps: int = 1) -> Workload:
    rc, rv, _, ri = streams(seed)
    coords = uniform_coords(rc, list(dims), nnz)
    vals = rv.random(coords.shape[1])
    U = [gaussian_qr(ri, d, r) for d, r in zip(dims, ranks)]
    return Workload("small", list(dims), list(ranks), coords, vals, U, sweeps=sweeps, dtype=dtype)


def support_low_rank(seed: int, dims, support, ranks):
    """Exact multilinear-rank tensor with a sparse support: factor F_k is nonzero only on a random
    row subset S_k (|S_k| = support[k]), so X = G x_k F_k has nnz = prod |S_k| and rank <= ranks.
    Returns (coords, vals, G, F)."""
    rc, _, rm, _ = streams(seed)
    N = len(dims)
    S = [np.sort(rc.choice(d, size=s, replace=False)) for d, s in zip(dims, support)]
    F = []
    for d, s, r, Sk in zip(dims, support, ranks, S):
        f = np.zeros((d, r))
        f[Sk] = rm.standard_normal((s, r))
        F.append(f)
    G = rm.standard_normal(tuple(ranks))
    grids = np.meshgrid(*S, indexing="ij")
    coords = np.stack([g.ravel() for g in grids]).astype(np.int32)
    dense = G
    for k in range(N):
        dense = np.tensordot(dense, F[k][S[k]], axes=([0], [1]))
    vals = dense.reshape(-1).copy()  # C order of the meshgrid: last mode fastest, matches coords
    return coords, vals, G, F


def pmm_tensor(M: int, K: int, N: int):
    """Binary parallel-matrix-multiplication tensor (Sec. IV-C): mode 1 indexes A (M x K, row
    major), mode 2 indexes B (K x N, row major), mode 3 indexes C (M x N, column major); one unit
    entry per scalar product a_mk * b_kn accumulated into c_mn.  nnz = M K N."""
    m, k, n = np.meshgrid(np.arange(M), np.arange(K), np.arange(N), indexing="ij")
    i1 = (m * K + k).ravel()
    i2 = (k * N + n).ravel()
    i3 = (n * M + m).ravel()
    coords = np.stack([i1, i2, i3]).astype(np.int32)
    return coords, np.ones(coords.shape[1]), [M * K, K * N, M * N]
