"""Pins for the FP64 CPU oracle: each check ties an oracle routine to something other than itself
(a dense brute-force definition, a LAPACK or scipy routine, a closed form, an invariant, or a
value written out by hand from the paper's Table I)."""
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_from_coo(coords, vals, dims):
    X = np.zeros(dims)
    np.add.at(X, tuple(np.asarray(coords, dtype=np.int64)), vals)
    return X


def dense_chain(X, U, mode):
    """X x_t U_t^T for every t != mode, by tensordot on the dense array, then unfolded with the
    other modes ascending and the last fastest."""
    N = X.ndim
    T = X
    for t in range(N):
        if t == mode:
            continue
        T = np.moveaxis(np.tensordot(T, U[t], axes=([t], [0])), -1, t)
    return np.moveaxis(T, mode, 0).reshape(X.shape[mode], -1)


def random_tensor(seed, dims, nnz, ranks):
    w = synth.small_uniform(seed, dims, ranks, nnz)
    rng = np.random.default_rng(seed + 1000)
    w.vals = rng.standard_normal(w.nnz)
    return w


# ------------------------------------------------------------------------------------------
# TTMc
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("dims,ranks,nnz", [
    ([7, 6, 5], [2, 3, 2], 40),
    ([9, 4, 6], [3, 4, 5], 100),
    ([5, 4, 3, 6], [2, 3, 2, 3], 70),
    ([4, 3, 5, 2, 3], [2, 2, 3, 2, 1], 60),
    ([8, 6], [3, 4], 20),
])
def test_ttmc_equals_dense_chain(dims, ranks, nnz):
    """Sparse TTMc (Alg. 2) equals the dense chain of TTMs of Eq. (power iteration), every mode."""
    w = random_tensor(11, dims, nnz, ranks)
    X = dense_from_coo(w.coords, w.vals, dims)
    for n in range(len(dims)):
        Y = oracle.ttmc(w.coords, w.vals, dims, ranks, n, w.U_init)
        np.testing.assert_allclose(Y, dense_chain(X, w.U_init, n), rtol=0, atol=1e-13)


def test_ttmc_order2_is_spmm():
    """Order 2 reduces to a sparse-times-dense product (scipy.sparse), both modes."""
    w = random_tensor(12, [30, 20], 90, [4, 5])
    A = scipy.sparse.coo_matrix((w.vals, (w.coords[0], w.coords[1])), shape=(30, 20)).tocsr()
    np.testing.assert_allclose(oracle.ttmc(w.coords, w.vals, w.dims, w.ranks, 0, w.U_init),
                               A @ w.U_init[1], atol=1e-13)
    np.testing.assert_allclose(oracle.ttmc(w.coords, w.vals, w.dims, w.ranks, 1, w.U_init),
                               A.T @ w.U_init[0], atol=1e-13)


def test_ttmc_kronecker_column_order():
    """Column c of Y_(1) for a single nonzero equals a[i] * b[j] with c = R3 * i + j (the
    Kronecker-product listing of Sec. III-C): last mode fastest."""
    a = np.array([[1.0, 2.0]])
    b = np.array([[3.0, 5.0, 7.0]])
    U = [np.ones((1, 1)), a, b]
    Y = oracle.ttmc(np.zeros((3, 1), np.int32), np.array([1.0]), [1, 1, 1], [1, 2, 3], 0, U)
    assert Y.ravel().tolist() == [3.0, 5.0, 7.0, 6.0, 10.0, 14.0]


def test_ttmc_linear_and_duplicates():
    """Linear in the values; duplicate coordinates act as their sum."""
    w = random_tensor(13, [6, 7, 8], 50, [2, 3, 2])
    Y1 = oracle.ttmc(w.coords, w.vals, w.dims, w.ranks, 1, w.U_init)
    Y3 = oracle.ttmc(w.coords, 3.0 * w.vals, w.dims, w.ranks, 1, w.U_init)
    np.testing.assert_allclose(Y3, 3.0 * Y1, atol=1e-13)
    c = np.concatenate([w.coords, w.coords], axis=1)
    v = np.concatenate([0.25 * w.vals, 0.75 * w.vals])
    np.testing.assert_allclose(oracle.ttmc(c, v, w.dims, w.ranks, 1, w.U_init), Y1, atol=1e-13)
    cc, cv = oracle.coalesce(c, v, w.dims)
    np.testing.assert_allclose(oracle.ttmc(cc, cv, w.dims, w.ranks, 1, w.U_init), Y1, atol=1e-13)


@pytest.mark.parametrize("threads", [2, 3, 8, 64])
def test_ttmc_threads_bit_identical(threads):
    """The host-threaded TTMc (CPU-baseline timing) gives exactly orc_ttmc's result in every mode,
    including more threads than non-empty rows and a skewed row distribution; the threaded sweep
    gives the same fits and factors."""
    w = random_tensor(14, [40, 30, 9], 3000, [4, 3, 5])
    c = w.coords.copy()
    c[0, : 1500] = 3                              # one hot row holding half the nonzeros
    cc, cv = oracle.coalesce(c, w.vals, w.dims)
    for n in range(3):
        Y1 = oracle.ttmc(cc, cv, w.dims, w.ranks, n, w.U_init)
        Yt = oracle.ttmc(cc, cv, w.dims, w.ranks, n, w.U_init, threads=threads)
        assert np.array_equal(Y1, Yt)
    U1, G1, f1, p1 = oracle.hooi(cc, cv, w.dims, w.ranks, w.U_init, 2)
    Ut, Gt, ft, pt = oracle.hooi(cc, cv, w.dims, w.ranks, w.U_init, 2, threads=threads)
    assert np.array_equal(f1, ft) and np.array_equal(G1, Gt) and np.array_equal(p1, pt)
    assert all(np.array_equal(a, b) for a, b in zip(U1, Ut))


def test_bf16_nearest_matches_torch():
    """The oracle's BF16 rounding equals torch's CPU bfloat16 conversion (round to nearest, ties
    to even) on values over many binades and on exact halfway cases of both parities."""
    import torch
    rng = np.random.default_rng(5)
    x = (rng.standard_normal(20000) * np.exp2(rng.integers(-20, 20, 20000))).astype(np.float32).astype(np.float64)
    # halfway cases: a BF16 number plus half its unit in the last place
    b = torch.from_numpy(x[:5000]).to(torch.bfloat16).to(torch.float64).numpy()
    _, e = np.frexp(b)
    ties = b + np.ldexp(1.0, e - 9)
    x = np.concatenate([x, ties, [0.0, 1.0, -1.0]])
    ref = torch.from_numpy(x).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.bf16_nearest(x), ref)


def test_ttmc_bf16_operands_exact_products_equal_ttmc():
    """With power-of-two values and BF16 factors every product x a is a BF16 number, so the
    BF16-operand TTMc equals the plain TTMc (which pins its contraction and column order)."""
    rng = np.random.default_rng(8)
    dims, ranks = [9, 7, 6], [3, 4, 2]
    w = random_tensor(21, dims, 120, ranks)
    vals = np.exp2(rng.integers(-3, 4, w.nnz)) * np.sign(rng.standard_normal(w.nnz))
    U = [oracle.bf16_nearest(u) for u in w.U_init]
    for n in range(3):
        np.testing.assert_allclose(oracle.ttmc_bf16_operands(w.coords, vals, dims, ranks, n, U),
                                   oracle.ttmc(w.coords, vals, dims, ranks, n, U), rtol=0, atol=1e-14)


def test_ttmc_bf16_operands_brute_force():
    """Against a loop over nonzeros with torch's BF16 rounding of x a: Y[i_n] += kron(bf16(x a), b);
    and the rounding is within its bound of the plain TTMc (8 significant bits:
    |bf16(v) - v| <= 2^-8 |v|)."""
    import torch
    dims, ranks = [6, 5, 7], [2, 3, 4]
    w = random_tensor(23, dims, 60, ranks)
    U = [oracle.bf16_nearest(u) for u in w.U_init]
    vals = oracle.bf16_nearest(w.vals)
    for n in range(3):
        s, t = [k for k in range(3) if k != n]
        Y = np.zeros((dims[n], ranks[s] * ranks[t]))
        for p in range(w.nnz):
            a = U[s][w.coords[s, p]] * vals[p]
            a = torch.from_numpy(a).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
            Y[w.coords[n, p]] += np.kron(a, U[t][w.coords[t, p]])
        got = oracle.ttmc_bf16_operands(w.coords, vals, dims, ranks, n, U)
        np.testing.assert_allclose(got, Y, rtol=0, atol=1e-14)
        plain = oracle.ttmc(w.coords, vals, dims, ranks, n, U)
        assert np.abs(got - plain).max() > 0
        bound = np.zeros_like(plain)
        np.add.at(bound, w.coords[n], 2.0 ** -8 * np.abs(np.einsum("pi,pj->pij", U[s][w.coords[s]] * vals[:, None],
                                                                    U[t][w.coords[t]]).reshape(w.nnz, -1)))
        assert np.all(np.abs(got - plain) <= bound + 1e-15)


# ------------------------------------------------------------------------------------------
# QRP
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,R", [(40, 12, 5), (64, 64, 8), (300, 64, 8), (25, 25, 25), (50, 7, 7)])
def test_qrp_matches_lapack(m, n, R):
    """Householder QRP (Sec. III-D) equals LAPACK dgeqp3/dorgqr on generic input: same pivots,
    same Q columns (both use v = x + sgn(x_0)||x|| e_1)."""
    rng = np.random.default_rng(m * 1000 + n)
    A = rng.standard_normal((m, n)) * rng.uniform(0.1, 10.0, size=n)
    Q, piv = oracle.qrp(A, R)
    Ql, Rl, Pl = scipy.linalg.qr(A, pivoting=True, mode="economic")
    assert piv.tolist() == Pl[:R].tolist()
    # LAPACK leaves the last reflector out when its sub-column is empty (a 1-row x, m = R); the
    # textbook reflector then flips that column's sign.  Compare columns up to that single case.
    for j in range(R):
        s = 1.0 if (j < m - 1) else np.sign(Q[:, j] @ Ql[:, j])
        np.testing.assert_allclose(Q[:, j], s * Ql[:, j], atol=1e-12)


def test_qrp_pivot_gaps_from_projections():
    """The oracle's per-step pivot gaps equal those from the definition: at step j the trailing
    squared norm of column c is ||a_c||^2 - ||Q_j^T a_c||^2 with Q_j the first j columns of Q (LAPACK
    pivoted QR); the gap is (largest - second largest) / largest over the columns not yet chosen."""
    rng = np.random.default_rng(31)
    A = rng.standard_normal((200, 24)) * np.linspace(1.0, 3.0, 24)
    A[:, 7] = A[:, 3] * 1.0000001            # a near tie
    R = 10
    _, piv, gaps = oracle.qrp(A, R, gaps=True)
    Q, _, P = scipy.linalg.qr(A, pivoting=True, mode="economic")
    assert piv.tolist() == P[:R].tolist()
    chosen = []
    for j in range(R):
        Qj = Q[:, :j]
        norms = (A * A).sum(axis=0) - ((Qj.T @ A) ** 2).sum(axis=0)
        cand = np.array([c for c in range(A.shape[1]) if c not in chosen])
        v = np.sort(norms[cand])[::-1]
        assert abs(gaps[j] - (v[0] - v[1]) / v[0]) <= 1e-9, j
        chosen.append(P[j])


def test_qrp_invariants():
    """Q^T Q = I; R = Q^T A P is upper triangular with non-increasing |r_jj|; A P[:, :R] = Q R11."""
    rng = np.random.default_rng(7)
    A = rng.standard_normal((80, 30)) @ np.diag(np.linspace(5, 0.1, 30))
    R = 10
    Q, piv = oracle.qrp(A, R)
    np.testing.assert_allclose(Q.T @ Q, np.eye(R), atol=1e-13)
    Rm = Q.T @ A[:, piv]
    np.testing.assert_allclose(np.tril(Rm, -1), 0, atol=1e-12)
    d = np.abs(np.diag(Rm))
    assert np.all(d[:-1] >= d[1:] - 1e-12)
    np.testing.assert_allclose(Q @ Rm, A[:, piv], atol=1e-12)
    # truncation: the first R columns of a longer run are identical
    Q2, piv2 = oracle.qrp(A, 20)
    assert piv2[:R].tolist() == piv.tolist()
    np.testing.assert_allclose(Q2[:, :R], Q, atol=1e-14)


def test_qrp_rank_revealing_on_low_rank():
    """On an exactly rank-r matrix the first r pivoted columns span its column space."""
    rng = np.random.default_rng(8)
    A = rng.standard_normal((60, 4)) @ rng.standard_normal((4, 20))
    Q, _ = oracle.qrp(A, 4)
    np.testing.assert_allclose(Q @ (Q.T @ A), A, atol=1e-12)


def test_fat_rule_uses_gram():
    """A Y with more columns than rows goes through QRP of Y Y^T (Sec. III-D)."""
    rng = np.random.default_rng(9)
    Y = rng.standard_normal((12, 40))
    U, piv = oracle.factor(Y, 5, fat_rule=True)
    Q, p2 = oracle.qrp(Y @ Y.T, 5)
    np.testing.assert_allclose(U, Q, atol=1e-13)
    assert piv.tolist() == p2.tolist()
    U2, _ = oracle.factor(Y, 5, fat_rule=False)
    Q2, _ = scipy.linalg.qr(Y, pivoting=True, mode="economic")[0:2]
    np.testing.assert_allclose(np.abs(U2), np.abs(Q2[:, :5]), atol=1e-12)


# ------------------------------------------------------------------------------------------
# Core, fit, reconstruct, sweeps
# ------------------------------------------------------------------------------------------

def test_core_and_fit_against_dense():
    """G = X x_1 U_1^T ... x_N U_N^T (Eq. TTM_G) from the last chain product; fit formula equals the
    directly computed residual for orthonormal factors."""
    w = random_tensor(21, [9, 8, 7], 120, [3, 4, 2])
    X = dense_from_coo(w.coords, w.vals, w.dims)
    U = w.U_init
    Y = oracle.ttmc(w.coords, w.vals, w.dims, w.ranks, 2, U)
    G = oracle.core(Y, U[2], w.ranks)
    Gd = np.einsum("ijk,ia,jb,kc->abc", X, U[0], U[1], U[2])
    np.testing.assert_allclose(G, Gd, atol=1e-13)
    Xh = np.einsum("abc,ia,jb,kc->ijk", G, U[0], U[1], U[2])
    direct = np.linalg.norm(X - Xh) / np.linalg.norm(X)
    f = oracle.fit(float(w.vals @ w.vals), G)
    assert abs((1.0 - f) - direct) < 1e-7


def test_reconstruct_against_dense():
    rng = np.random.default_rng(22)
    dims, ranks = [6, 5, 4, 3], [2, 3, 2, 2]
    G = rng.standard_normal(ranks)
    U = [rng.standard_normal((d, r)) for d, r in zip(dims, ranks)]
    Xh = np.einsum("abcd,ia,jb,kc,ld->ijkl", G, *U)
    coords = np.stack([rng.integers(0, d, 50) for d in dims]).astype(np.int32)
    np.testing.assert_allclose(oracle.reconstruct(G, U, coords), Xh[tuple(coords)], atol=1e-13)


def test_exact_low_rank_reconstructs_to_roundoff():
    """A support-restricted tensor of exact multilinear rank is recovered to round-off: direct
    residual ~1e-15, factors orthonormal, the projectors onto the true column spaces match."""
    dims, ranks = [60, 60, 60], [4, 5, 3]
    coords, vals, Gt, F = synth.support_low_rank(31, dims, [20, 20, 20], ranks)
    rng = np.random.default_rng(32)
    U0 = [synth.gaussian_qr(rng, d, r) for d, r in zip(dims, ranks)]
    U, G, fits, _ = oracle.hooi(coords, vals, dims, ranks, U0, sweeps=3)
    Xh = oracle.reconstruct(G, U, coords)
    assert np.linalg.norm(Xh - vals) / np.linalg.norm(vals) < 1e-13
    for k in range(3):
        np.testing.assert_allclose(U[k].T @ U[k], np.eye(ranks[k]), atol=1e-13)
        Qt, _ = np.linalg.qr(F[k])
        np.testing.assert_allclose(U[k] @ U[k].T, Qt @ Qt.T, atol=1e-12)
    assert fits[-1] > 1.0 - 1e-7   # the fit formula itself has a sqrt(eps) floor


def test_core_identity_any_size():
    """sum_p x_p * xhat_p = ||G||^2 because G = X x_k U_k^T with orthonormal U."""
    w = synth.hooi_small_f64(1)
    U, G, fits, _ = oracle.hooi(w.coords, w.vals, w.dims, w.ranks, w.U_init, sweeps=1)
    xh = oracle.reconstruct(G, U, w.coords)
    assert abs(w.vals @ xh - np.sum(G * G)) < 1e-10 * np.sum(G * G)


@pytest.mark.parametrize("svd", [False, True])
def test_hosvd_sketch_recovers_exact_low_rank_spaces(svd):
    """On a tensor of exact multilinear rank (sparse support), the sketched HOSVD start (TTMc with
    Gaussian test factors, then QRP or SVD of each sketch) spans exactly the column space of each
    factor (projectors equal to round-off), and one HOOI sweep from it reconstructs X to round-off."""
    dims, support, ranks = [40, 35, 30], [12, 10, 9], [4, 5, 3]
    coords, vals, G, F = synth.support_low_rank(5, dims, support, ranks)
    rng = np.random.default_rng(6)
    Omega = [rng.standard_normal((d, r)) for d, r in zip(dims, ranks)]
    U = oracle.hosvd_sketch(coords, vals, dims, ranks, Omega, svd=svd)
    for n in range(3):
        Qf, _ = np.linalg.qr(F[n])
        assert np.linalg.norm(U[n] @ U[n].T - Qf @ Qf.T) <= 1e-12 * 10
        assert np.linalg.norm(U[n].T @ U[n] - np.eye(ranks[n])) <= 1e-12
    Uh, Gh, fits, _ = oracle.hooi(coords, vals, dims, ranks, U, 1)
    xhat = oracle.reconstruct(Gh, Uh, coords)
    assert np.linalg.norm(xhat - vals) <= 1e-12 * np.linalg.norm(vals)


def test_first_factor_init_is_unused():
    """Mode 1 of the first sweep reads only U_2..U_N (Alg. 2), so U_1's init cannot matter."""
    w = random_tensor(41, [10, 9, 8], 150, [3, 3, 3])
    U_a = [u.copy() for u in w.U_init]
    U_b = [u.copy() for u in w.U_init]
    U_b[0] = synth.gaussian_qr(np.random.default_rng(5), 10, 3)
    ra = oracle.hooi(w.coords, w.vals, w.dims, w.ranks, U_a, sweeps=2)
    rb = oracle.hooi(w.coords, w.vals, w.dims, w.ranks, U_b, sweeps=2)
    np.testing.assert_array_equal(ra[2], rb[2])
    np.testing.assert_array_equal(ra[1], rb[1])


def test_svd_hooi_fit_is_monotone():
    """With the SVD update (Alg. 1) each mode step maximises ||G|| for fixed other factors, so the
    fit never decreases across sweeps."""
    for seed in range(8):
        w = random_tensor(50 + seed, [12, 11, 10], 300, [3, 2, 3])
        _, _, fits = oracle.hooi_svd(w.coords, w.vals, w.dims, w.ranks, w.U_init, sweeps=6)
        assert np.all(np.diff(fits) >= -1e-12), fits


def test_qrp_and_svd_agree_on_low_rank_plus_noise():
    """Table II: Tucker with QRP loses no accuracy against Tucker with SVD on low-rank tensors.
    With a support-restricted low-rank tensor plus small noise the two errors agree closely."""
    dims, ranks = [50, 50, 50], [4, 4, 4]
    coords, vals, _, _ = synth.support_low_rank(61, dims, [15, 15, 15], ranks)
    vals = vals + 1e-9 * np.random.default_rng(62).standard_normal(vals.size)
    U0 = [synth.gaussian_qr(np.random.default_rng(63 + k), d, r) for k, (d, r) in enumerate(zip(dims, ranks))]
    Uq, Gq, _, _ = oracle.hooi(coords, vals, dims, ranks, U0, sweeps=3)
    Us, Gs, _ = oracle.hooi_svd(coords, vals, dims, ranks, U0, sweeps=3)
    eq = np.linalg.norm(oracle.reconstruct(Gq, Uq, coords) - vals) / np.linalg.norm(vals)
    es = np.linalg.norm(oracle.reconstruct(Gs, Us, coords) - vals) / np.linalg.norm(vals)
    assert eq < 1e-9 and es < 1e-9
    assert abs(eq - es) < 0.05 * es


def test_pmm_tensor_closed_forms():
    """Parallel-matrix-multiplication tensor of Sec. IV-C (M = N = K = 5, 25^3, nnz 125): every
    unfolding has X_(n) X_(n)^T = 5 I, so ||X||^2 = 125 and any rank-(5,5,5) fit is at most
    1 - sqrt(0.8).  Three sweeps make 125 * 3 * 3 = 1125 Kronecker products, as the paper counts."""
    coords, vals, dims = synth.pmm_tensor(5, 5, 5)
    assert vals.size == 125 and dims == [25, 25, 25]
    assert abs(vals.size / np.prod(dims) - 8e-3) < 1e-12
    X = dense_from_coo(coords, vals, dims)
    for n in range(3):
        Xn = np.moveaxis(X, n, 0).reshape(25, -1)
        np.testing.assert_array_equal(Xn @ Xn.T, 5 * np.eye(25))
    rng = np.random.default_rng(70)
    U0 = [synth.gaussian_qr(rng, 25, 5) for _ in range(3)]
    _, G, fits, _ = oracle.hooi(coords, vals, dims, [5, 5, 5], U0, sweeps=3)
    assert np.all(fits <= 1.0 - np.sqrt(0.8) + 1e-12)
    assert np.all(fits > 0)
    assert vals.size * 3 * 3 == 1125


# ------------------------------------------------------------------------------------------
# Completion gradient
# ------------------------------------------------------------------------------------------

def _loss_only(G, U, coords, vals):
    e = oracle.reconstruct(G, U, coords) - vals
    return float(e @ e) / (2 * vals.size)


def test_completion_gradient_finite_differences_exhaustive():
    rng = np.random.default_rng(80)
    dims, ranks = [6, 5, 4], [2, 3, 2]
    coords = synth.uniform_coords(rng, dims, 40)
    vals = rng.standard_normal(40)
    G = rng.standard_normal(ranks)
    U = [rng.standard_normal((d, r)) for d, r in zip(dims, ranks)]
    loss, gG, gU = oracle.completion(G, U, coords, vals, dims)
    assert abs(loss - _loss_only(G, U, coords, vals)) < 1e-14
    h = 1e-6
    for idx in np.ndindex(*ranks):
        Gp, Gm = G.copy(), G.copy()
        Gp[idx] += h
        Gm[idx] -= h
        fd = (_loss_only(Gp, U, coords, vals) - _loss_only(Gm, U, coords, vals)) / (2 * h)
        assert abs(fd - gG[idx]) < 1e-8
    for n in range(3):
        for idx in np.ndindex(*U[n].shape):
            Up = [u.copy() for u in U]
            Um = [u.copy() for u in U]
            Up[n][idx] += h
            Um[n][idx] -= h
            fd = (_loss_only(G, Up, coords, vals) - _loss_only(G, Um, coords, vals)) / (2 * h)
            assert abs(fd - gU[n][idx]) < 1e-8


def test_completion_gradient_30cube_directional():
    """The 30^3 / 2,000-entry / rank-16 instance: directional finite difference along a random
    direction in every parameter at once, plus 12 single coordinates."""
    w = synth.completion(seed=6, dims=(30, 30, 30), nnz=2000, R=16, dtype="f64")
    G, U = w.G_init, w.U_init
    loss, gG, gU = oracle.completion(G, U, w.coords, w.vals, w.dims)
    rng = np.random.default_rng(81)
    dG = rng.standard_normal(G.shape)
    dU = [rng.standard_normal(u.shape) for u in U]
    h = 1e-6
    lp = _loss_only(G + h * dG, [u + h * d for u, d in zip(U, dU)], w.coords, w.vals)
    lm = _loss_only(G - h * dG, [u - h * d for u, d in zip(U, dU)], w.coords, w.vals)
    fd = (lp - lm) / (2 * h)
    an = np.sum(gG * dG) + sum(np.sum(g * d) for g, d in zip(gU, dU))
    assert abs(fd - an) < 1e-6 * max(1.0, abs(an))
    for _ in range(12):
        n = int(rng.integers(0, 3))
        i = (int(rng.integers(0, 30)), int(rng.integers(0, 16)))
        Up = [u.copy() for u in U]
        Um = [u.copy() for u in U]
        Up[n][i] += h
        Um[n][i] -= h
        fd = (_loss_only(G, Up, w.coords, w.vals) - _loss_only(G, Um, w.coords, w.vals)) / (2 * h)
        assert abs(fd - gU[n][i]) < 1e-6 * max(1.0, abs(fd))


def test_completion_zero_residual_zero_gradient():
    rng = np.random.default_rng(82)
    dims, ranks = [7, 6, 5], [2, 2, 3]
    G = rng.standard_normal(ranks)
    U = [rng.standard_normal((d, r)) for d, r in zip(dims, ranks)]
    coords = synth.uniform_coords(rng, dims, 60)
    vals = oracle.reconstruct(G, U, coords)
    loss, gG, gU = oracle.completion(G, U, coords, vals, dims)
    assert loss < 1e-28
    assert np.abs(gG).max() < 1e-14
    assert max(np.abs(g).max() for g in gU) < 1e-14


# ------------------------------------------------------------------------------------------
# Mode-sorted layout
# ------------------------------------------------------------------------------------------

def _read_table1():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_coo.txt")) if not l.startswith("#")]
    arr = np.array([[float(x) for x in r] for r in rows if r])
    coords = (arr[:, :4].T.astype(np.int64) - 1).astype(np.int32)  # 1-based -> 0-based
    return coords, arr[:, 4]


def test_table1_csf_golden():
    coords, vals = _read_table1()
    assert coords.shape == (4, 4)
    expect = {}
    for line in open(os.path.join(GOLDEN, "table1_csf.txt")):
        if line.startswith("#") or not line.strip():
            continue
        m, r, p, v = [s.split() for s in line.split("|")]
        expect[int(m[0])] = ([int(x) for x in r], [int(x) for x in p], [float(x) for x in v])
    for mode in range(4):
        c = oracle.csf(coords, vals, mode)
        rows, ptr, v = expect[mode]
        assert c["rows"].tolist() == rows
        assert c["ptr"].tolist() == ptr
        assert c["vals"].tolist() == v


def test_csf_invariants():
    """Any input order gives the same layout; ptr differences equal the per-row counts; the sort
    key is (i_n, i_f, rest) for order 4 and (i_n, rest) for order 3."""
    for dims in ([9, 8, 7], [6, 5, 4, 3]):
        w = random_tensor(90, dims, 100, [2] * len(dims))
        rng = np.random.default_rng(91)
        perm = rng.permutation(w.nnz)
        for mode in range(len(dims)):
            a = oracle.csf(w.coords, w.vals, mode)
            b = oracle.csf(w.coords[:, perm], w.vals[perm], mode)
            for k in ("rows", "ptr", "idx", "vals"):
                np.testing.assert_array_equal(a[k], b[k])
            counts = np.bincount(w.coords[mode], minlength=dims[mode])
            np.testing.assert_array_equal(np.diff(a["ptr"]), counts[a["rows"]])
            keys = oracle.sort_modes(len(dims), mode)
            full = np.empty((len(dims), w.nnz), dtype=np.int64)
            others = [t for t in range(len(dims)) if t != mode]
            full[mode] = np.repeat(a["rows"], np.diff(a["ptr"]))
            for j, t in enumerate(others):
                full[t] = a["idx"][j]
            tup = [tuple(full[k][p] for k in keys) for p in range(w.nnz)]
            assert tup == sorted(tup)


def test_coalesce_sums_in_input_order():
    coords = np.array([[0, 1, 0, 0], [2, 2, 2, 1]], dtype=np.int32)
    vals = np.array([1e16, 3.0, 1.0, 5.0])
    c, v = oracle.coalesce(coords, vals, [2, 3])
    assert c.tolist() == [[0, 0, 1], [1, 2, 2]]
    assert v.tolist() == [5.0, 1e16 + 1.0, 3.0]
