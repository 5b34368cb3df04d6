/*
 * Plain FP64 CPU oracle for sparse Tucker decomposition by HOOI with QR column pivoting.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library.  It shares no code, header, table or helper with the GPU library,
 * and nothing in the GPU library may call it.
 *
 * Every routine is the definition written out, in input order, with no blocking, fusion or
 * reordering.  Arrays are row-major.  Coordinates are 0-based, stored structure-of-arrays:
 * coords[t * nnz + p] is the mode-t index of nonzero p.
 *
 * Kronecker column order (paper Alg. 2 and the Kronecker-product listing of Sec. III-C, which
 * index the product of two rows a (length R2) and b (length R3) as c = R3 * i + j): the other
 * modes are taken in ascending order and the LAST one varies fastest.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_OOM 3

static int64_t kron_len(int N, const int32_t* ranks, int skip)
{
    int64_t K = 1;
    for (int t = 0; t < N; ++t)
        if (t != skip) K *= ranks[t];
    return K;
}

/*
 * Sparse TTMc, paper Alg. 2 (inner loop over nonzeros) and the per-nonzero Kronecker update of
 * Sec. III-C: for each nonzero x at (i_1..i_N),
 *     Y_(n)(i_n, :) += x * (U_t1(i_t1, :) kron U_t2(i_t2, :) kron ...),  t ascending, t != n.
 * Y is dims[mode] x K_n with K_n = prod_{t != mode} ranks[t]; U[t] is dims[t] x ranks[t].
 */
int orc_ttmc(int N, const int64_t* dims, const int32_t* ranks, int64_t nnz,
             const int32_t* coords, const double* vals, int mode,
             const double* const* U, double* Y)
{
    if (N < 1 || mode < 0 || mode >= N) return ORC_ERR_ARG;
    const int64_t K = kron_len(N, ranks, mode);
    memset(Y, 0, (size_t)(dims[mode] * K) * sizeof(double));
    double* kr = (double*)malloc((size_t)K * sizeof(double));
    double* tmp = (double*)malloc((size_t)K * sizeof(double));
    if (!kr || !tmp) { free(kr); free(tmp); return ORC_ERR_OOM; }
    for (int64_t p = 0; p < nnz; ++p) {
        int64_t len = 1;
        kr[0] = vals[p];
        for (int t = 0; t < N; ++t) {
            if (t == mode) continue;
            const int64_t R = ranks[t];
            const double* row = U[t] + (int64_t)coords[(int64_t)t * nnz + p] * R;
            /* kr <- kr kron row : new[a * R + b] = kr[a] * row[b] */
            for (int64_t a = 0; a < len; ++a)
                for (int64_t b = 0; b < R; ++b)
                    tmp[a * R + b] = kr[a] * row[b];
            double* sw = kr; kr = tmp; tmp = sw;
            len *= R;
        }
        double* y = Y + (int64_t)coords[(int64_t)mode * nnz + p] * K;
        for (int64_t c = 0; c < K; ++c) y[c] += kr[c];
    }
    free(kr);
    free(tmp);
    return ORC_OK;
}

/*
 * The same TTMc on several host threads (used to time the CPU baseline on all cores; the
 * arithmetic is orc_ttmc's).  The rows of Y_(n) are cut into nthreads ranges holding about equal
 * numbers of nonzeros; each thread walks every nonzero in input order and applies only those whose
 * row lies in its range.  Each row therefore receives the additions of orc_ttmc in the same order,
 * so the result is bit-identical to orc_ttmc for any thread count.
 */
int orc_ttmc_threads(int N, const int64_t* dims, const int32_t* ranks, int64_t nnz,
                     const int32_t* coords, const double* vals, int mode,
                     const double* const* U, double* Y, int nthreads)
{
    if (N < 1 || mode < 0 || mode >= N || nthreads < 1) return ORC_ERR_ARG;
    const int64_t K = kron_len(N, ranks, mode);
    const int64_t I = dims[mode];
    const int32_t* rowidx = coords + (int64_t)mode * nnz;
    /* row ranges of about nnz / nthreads nonzeros each: bounds[k] .. bounds[k + 1] */
    int64_t* count = (int64_t*)calloc((size_t)I + 1, sizeof(int64_t));
    int64_t* bounds = (int64_t*)malloc((size_t)(nthreads + 1) * sizeof(int64_t));
    if (!count || !bounds) { free(count); free(bounds); return ORC_ERR_OOM; }
    for (int64_t p = 0; p < nnz; ++p) count[rowidx[p]] += 1;
    bounds[0] = 0;
    int64_t acc = 0, row = 0;
    for (int k = 1; k < nthreads; ++k) {
        const int64_t target = nnz * k / nthreads;
        while (row < I && acc + count[row] <= target) acc += count[row++];
        bounds[k] = row;
    }
    bounds[nthreads] = I;
    int status = ORC_OK;
#pragma omp parallel num_threads(nthreads)
    {
        const int k = omp_get_thread_num();
        const int64_t lo = bounds[k], hi = bounds[k + 1];
        double* kr = (double*)malloc((size_t)K * sizeof(double));
        double* tmp = (double*)malloc((size_t)K * sizeof(double));
        if (!kr || !tmp) {
#pragma omp atomic write
            status = ORC_ERR_OOM;
        } else {
            memset(Y + lo * K, 0, (size_t)((hi - lo) * K) * sizeof(double));
            for (int64_t p = 0; p < nnz; ++p) {
                const int64_t i = rowidx[p];
                if (i < lo || i >= hi) continue;
                int64_t len = 1;
                kr[0] = vals[p];
                for (int t = 0; t < N; ++t) {
                    if (t == mode) continue;
                    const int64_t R = ranks[t];
                    const double* rw = U[t] + (int64_t)coords[(int64_t)t * nnz + p] * R;
                    for (int64_t a = 0; a < len; ++a)
                        for (int64_t b = 0; b < R; ++b)
                            tmp[a * R + b] = kr[a] * rw[b];
                    double* sw = kr; kr = tmp; tmp = sw;
                    len *= R;
                }
                double* y = Y + i * K;
                for (int64_t c = 0; c < K; ++c) y[c] += kr[c];
            }
        }
        free(kr);
        free(tmp);
    }
    free(count);
    free(bounds);
    return status;
}

/*
 * Householder QR with column pivoting (Sec. III-D), stopped after R steps.
 * A is m x n.  At step j the squared norms of the trailing sub-columns A[j:, c], c >= j, are
 * recomputed exactly; the first column of largest norm is swapped to position j (Businger-Golub
 * pivoting, giving |r_11| >= |r_22| >= ...).  The reflector is the textbook one:
 *     x = A[j:, j],  v = x + sgn(x_0) ||x|| e_1  (sgn(0) = +1),  H_j = I - 2 v v^T / (v^T v),
 * with H_j = I when x = 0.  Only the first R reflectors are formed, so this equals the first R
 * steps of the full factorization.  Output: Q[:, :R] = H_0 H_1 ... H_{R-1} [I_R; 0] (m x R),
 * piv[j] = original index of the column placed at position j, and (if gaps is not NULL) gaps[j] =
 * the relative gap between the largest and the second largest trailing squared norm at step j.
 */
int orc_qrp(int64_t m, int64_t n, const double* A_in, int R, double* Q, int32_t* piv, double* gaps)
{
    if (R < 1 || R > m || R > n) return ORC_ERR_ARG;
    double* A = (double*)malloc((size_t)(m * n) * sizeof(double));
    double* V = (double*)calloc((size_t)(m * R), sizeof(double)); /* column j holds v_j in rows j.. */
    double* beta = (double*)calloc((size_t)R, sizeof(double));
    double* w = (double*)malloc((size_t)n * sizeof(double));
    int32_t* perm = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!A || !V || !beta || !w || !perm) {
        free(A); free(V); free(beta); free(w); free(perm);
        return ORC_ERR_OOM;
    }
    memcpy(A, A_in, (size_t)(m * n) * sizeof(double));
    for (int64_t c = 0; c < n; ++c) perm[c] = (int32_t)c;

    for (int j = 0; j < R; ++j) {
        /* pivot: first column of largest trailing norm */
        int64_t p = j;
        double best = -1.0, second = -1.0;
        for (int64_t c = j; c < n; ++c) {
            double s = 0.0;
            for (int64_t i = j; i < m; ++i) s += A[i * n + c] * A[i * n + c];
            if (s > best) { second = best; best = s; p = c; }
            else if (s > second) second = s;
        }
        /* relative gap to the runner-up (1 when there is none, 0 for a tie) */
        if (gaps) gaps[j] = (second < 0.0) ? 1.0 : (best > 0.0 ? (best - second) / best : 0.0);
        if (p != j) {
            for (int64_t i = 0; i < m; ++i) {
                double t = A[i * n + j]; A[i * n + j] = A[i * n + p]; A[i * n + p] = t;
            }
            int32_t t = perm[j]; perm[j] = perm[p]; perm[p] = t;
        }
        /* reflector from x = A[j:, j] */
        double alpha = 0.0;
        for (int64_t i = j; i < m; ++i) alpha += A[i * n + j] * A[i * n + j];
        alpha = sqrt(alpha);
        if (alpha == 0.0) { beta[j] = 0.0; continue; }
        double vv = 0.0;
        for (int64_t i = j; i < m; ++i) {
            double v = A[i * n + j];
            if (i == j) v += (v >= 0.0 ? 1.0 : -1.0) * alpha;
            V[i * R + j] = v;
            vv += v * v;
        }
        beta[j] = 2.0 / vv;
        /* A[j:, j:] -= v * (beta * v^T A[j:, j:]) */
        for (int64_t c = j; c < n; ++c) {
            double s = 0.0;
            for (int64_t i = j; i < m; ++i) s += V[i * R + j] * A[i * n + c];
            w[c] = beta[j] * s;
        }
        for (int64_t i = j; i < m; ++i)
            for (int64_t c = j; c < n; ++c) A[i * n + c] -= V[i * R + j] * w[c];
    }
    /* Q[:, :R] = H_0 ... H_{R-1} [I_R; 0], applying the reflectors right to left */
    memset(Q, 0, (size_t)(m * R) * sizeof(double));
    for (int j = 0; j < R; ++j) Q[(int64_t)j * R + j] = 1.0;
    for (int j = R - 1; j >= 0; --j) {
        if (beta[j] == 0.0) continue;
        for (int c = 0; c < R; ++c) {
            double s = 0.0;
            for (int64_t i = j; i < m; ++i) s += V[i * R + j] * Q[i * R + c];
            s *= beta[j];
            for (int64_t i = j; i < m; ++i) Q[i * R + c] -= V[i * R + j] * s;
        }
    }
    if (piv)
        for (int j = 0; j < R; ++j) piv[j] = perm[j];
    free(A); free(V); free(beta); free(w); free(perm);
    return ORC_OK;
}

/*
 * Factor update U_n <- QRP(Y_(n), R_n) (Alg. 2).  With the fat-matrix rule of Sec. III-D, a Y
 * with more columns than rows is replaced by the square Y Y^T before the QRP.
 */
int orc_factor(int64_t I, int64_t K, const double* Y, int R, int fat_rule, double* U, int32_t* piv, double* gaps)
{
    if (fat_rule && K > I) {
        double* A = (double*)malloc((size_t)(I * I) * sizeof(double));
        if (!A) return ORC_ERR_OOM;
        for (int64_t a = 0; a < I; ++a)
            for (int64_t b = 0; b < I; ++b) {
                double s = 0.0;
                for (int64_t c = 0; c < K; ++c) s += Y[a * K + c] * Y[b * K + c];
                A[a * I + b] = s;
            }
        int st = orc_qrp(I, I, A, R, U, piv, gaps);
        free(A);
        return st;
    }
    return orc_qrp(I, K, Y, R, U, piv, gaps);
}

/*
 * Core tensor from the last mode's chain product (Alg. 2, the step after the mode loop, and the
 * unfolded form G_(N) = U_N^T Y_(N) of Sec. III-B).  G is stored C-order (last index fastest), so
 * G[r_1..r_{N-1}, r_N] sits at c * R_N + r_N where c is the Kronecker column of (r_1..r_{N-1}).
 */
int orc_core(int64_t I_N, int64_t K_N, int R_N, const double* Y_N, const double* U_N, double* G)
{
    for (int64_t c = 0; c < K_N; ++c)
        for (int r = 0; r < R_N; ++r) {
            double s = 0.0;
            for (int64_t i = 0; i < I_N; ++i) s += U_N[i * R_N + r] * Y_N[i * K_N + c];
            G[c * R_N + r] = s;
        }
    return ORC_OK;
}

/* fit = 1 - ||X - X_hat|| / ||X||, using ||X - X_hat||^2 = ||X||^2 - ||G||^2 for orthonormal U. */
double orc_fit(double normX2, const double* G, int64_t size)
{
    double g2 = 0.0;
    for (int64_t i = 0; i < size; ++i) g2 += G[i] * G[i];
    double r2 = normX2 - g2;
    if (r2 < 0.0) r2 = 0.0;
    return 1.0 - sqrt(r2) / sqrt(normX2);
}

/*
 * Sparse Tucker sweeps (Alg. 2): for s in 1..sweeps, for n = 1..N: Y_(n) by TTMc with the current
 * factors (Gauss-Seidel: modes before n already updated this sweep), U_n <- QRP(Y_(n), R_n); after
 * the mode loop G from the last Y and fit.  U (N pointers) is updated in place.  fits[s] receives
 * the fit after sweep s; pivs (optional, sweeps x N x maxR) the pivot lists.  nthreads > 1 runs
 * the TTMc on that many host threads (orc_ttmc_threads: the same result).
 */
int orc_hooi(int N, const int64_t* dims, const int32_t* ranks, int64_t nnz,
             const int32_t* coords, const double* vals, double* const* U, int sweeps,
             int fat_rule, double* G, double* fits, int32_t* pivs, int nthreads)
{
    int maxR = 0;
    int64_t maxY = 0;
    for (int n = 0; n < N; ++n) {
        if (ranks[n] > maxR) maxR = ranks[n];
        int64_t y = dims[n] * kron_len(N, ranks, n);
        if (y > maxY) maxY = y;
    }
    double* Y = (double*)malloc((size_t)maxY * sizeof(double));
    if (!Y) return ORC_ERR_OOM;
    double normX2 = 0.0;
    for (int64_t p = 0; p < nnz; ++p) normX2 += vals[p] * vals[p];
    int64_t gsize = kron_len(N, ranks, -1);
    for (int s = 0; s < sweeps; ++s) {
        for (int n = 0; n < N; ++n) {
            int st = nthreads > 1
                ? orc_ttmc_threads(N, dims, ranks, nnz, coords, vals, n, (const double* const*)U, Y, nthreads)
                : orc_ttmc(N, dims, ranks, nnz, coords, vals, n, (const double* const*)U, Y);
            if (st) { free(Y); return st; }
            int32_t* pv = pivs ? pivs + ((int64_t)s * N + n) * maxR : NULL;
            st = orc_factor(dims[n], kron_len(N, ranks, n), Y, ranks[n], fat_rule, U[n], pv, NULL);
            if (st) { free(Y); return st; }
            if (n == N - 1) orc_core(dims[n], kron_len(N, ranks, n), ranks[n], Y, U[n], G);
        }
        if (fits) fits[s] = orc_fit(normX2, G, gsize);
    }
    free(Y);
    return ORC_OK;
}

/* Value of the Tucker model G x_1 U_1 ... x_N U_N at one coordinate, summed over every core entry. */
static double model_at(int N, const int32_t* ranks, const double* G, const double* const* U,
                       const int32_t* idx, int skip, int32_t* r)
{
    int64_t size = kron_len(N, ranks, -1);
    double s = 0.0;
    for (int t = 0; t < N; ++t) r[t] = 0;
    for (int64_t g = 0; g < size; ++g) {
        /* r = mixed-radix digits of g, last mode fastest */
        int64_t rem = g;
        for (int t = N - 1; t >= 0; --t) { r[t] = (int32_t)(rem % ranks[t]); rem /= ranks[t]; }
        double term = G[g];
        for (int t = 0; t < N; ++t)
            if (t != skip) term *= U[t][(int64_t)idx[t] * ranks[t] + r[t]];
        s += term;
    }
    return s;
}

/* Sampled reconstruction: out[p] = (G x_1 U_1 ... x_N U_N)(i_1(p), ..., i_N(p)). */
int orc_reconstruct(int N, const int32_t* ranks, const double* G, const double* const* U,
                    int64_t m, const int32_t* coords, double* out)
{
    int32_t idx[16], r[16];
    if (N > 16) return ORC_ERR_ARG;
    for (int64_t p = 0; p < m; ++p) {
        for (int t = 0; t < N; ++t) idx[t] = coords[(int64_t)t * m + p];
        out[p] = model_at(N, ranks, G, U, idx, -1, r);
    }
    return ORC_OK;
}

/*
 * Sampled-entry Tucker completion loss and its gradient, from the definitions:
 *   e_p = x_hat_p - x_p,  L = sum_p e_p^2 / (2 |Omega|),
 *   dL/dG[r]        = (1/|Omega|) sum_p e_p prod_k U_k(i_k, r_k),
 *   dL/dU_n(i, r_n) = (1/|Omega|) sum_{p: i_n = i} e_p sum_{r without r_n} G[r] prod_{k != n} U_k(i_k, r_k).
 * Every sum runs over all core entries per nonzero.  gU[n] (dims[n] x ranks[n]) and gG are overwritten.
 */
int orc_completion(int N, const int64_t* dims, const int32_t* ranks, const double* G,
                   const double* const* U, int64_t nnz, const int32_t* coords, const double* vals,
                   double* loss, double* gG, double* const* gU)
{
    int32_t idx[16], r[16];
    if (N > 16 || nnz < 1) return ORC_ERR_ARG;
    int64_t size = kron_len(N, ranks, -1);
    memset(gG, 0, (size_t)size * sizeof(double));
    for (int n = 0; n < N; ++n) memset(gU[n], 0, (size_t)(dims[n] * ranks[n]) * sizeof(double));
    const double inv = 1.0 / (double)nnz;
    double L = 0.0;
    for (int64_t p = 0; p < nnz; ++p) {
        for (int t = 0; t < N; ++t) idx[t] = coords[(int64_t)t * nnz + p];
        double e = model_at(N, ranks, G, U, idx, -1, r) - vals[p];
        L += e * e;
        for (int64_t g = 0; g < size; ++g) {
            int64_t rem = g;
            for (int t = N - 1; t >= 0; --t) { r[t] = (int32_t)(rem % ranks[t]); rem /= ranks[t]; }
            double prod = 1.0;
            for (int t = 0; t < N; ++t) prod *= U[t][(int64_t)idx[t] * ranks[t] + r[t]];
            gG[g] += inv * e * prod;
            for (int n = 0; n < N; ++n) {
                double others = G[g];
                for (int t = 0; t < N; ++t)
                    if (t != n) others *= U[t][(int64_t)idx[t] * ranks[t] + r[t]];
                gU[n][(int64_t)idx[n] * ranks[n] + r[n]] += inv * e * others;
            }
        }
    }
    *loss = L * 0.5 * inv;
    return ORC_OK;
}
