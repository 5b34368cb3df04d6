// SVD factor update of standard HOOI (paper Alg. 1): U_n <- the R_n leading left singular vectors
// of Y_(n), in FP64, the alternative to the QRP of Alg. 2 (Sec. III-D compares the two).
//
// The singular vectors come from the eigendecomposition of a small symmetric FP64 matrix that the
// QRP path already forms on the device: for a tall Y_(n) (K_n <= I_n) the Gram matrix
// C = Y^T Y (K_n x K_n), whose eigenpairs (sigma_r^2, v_r) give u_r = Y v_r / sigma_r; for a fat
// Y_(n) the matrix Y Y^T (I_n x I_n), whose leading eigenvectors are the u_r themselves.  Only the
// R_n leading eigenpairs are needed.  They come from kernels of this file (Chebyshev-filtered
// subspace iteration with Rayleigh-Ritz projection, Zhou and Saad 2007: products with A over many
// workgroups, the small dense steps in one), stopped on a residual test that the host reads back
// after every outer step; when it does not converge, or the shape is outside its limits, or
// the context asks for it, rocSOLVER's divide-and-conquer dsyevd (a library primitive, all
// eigenpairs, ascending) is used instead.  Forming U and fixing signs are kernels of this file.
// Sign convention (singular
// vectors are defined up to sign): each column's entry of largest magnitude, the first one on
// ties, is made positive.  A zero singular value gives a zero column (rank deficiency; such
// columns are not determined by Y).
#include "internal.h"

#include <algorithm>
#include <type_traits>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

namespace tk {

namespace {

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// ---- R leading eigenpairs of a symmetric positive semidefinite n x n matrix A -------------------
// Block of b = min(n, R + min(R, 16)) vectors (stored with bs = b rounded up to 8 columns, the
// extra columns zero), in four n x bs row-major FP64 buffers.  One outer step:
//   Rayleigh-Ritz: P = A Z, H = Z^T P, H = S diag(theta) S^T (cyclic Jacobi), X = Z S, AX = P S,
//     Ritz values in decreasing order;
//   stop when ||AX_r - theta_r X_r|| <= tol theta_0 for every r < R;
//   else filter: Y = p_d(A) X with p_d the degree-d Chebyshev polynomial of the interval
//     [0, theta_{b-1}] (the part of the spectrum to damp), normalised to 1 at theta_0, run by the
//     three-term recurrence (one product with A per degree; the first one is AX); Z = orth(Y)
//     (classical Gram-Schmidt with one reorthogonalisation).
// The degree is the one that would bring the largest residual under the tolerance at the
// filter's growth rate for theta_r, capped so that p_d(theta_0) / p_d(theta_{R-1}) <= 1e12 (a
// larger spread swamps the lower Ritz directions in rounding error), and at kEigMaxDeg.
constexpr int kEigT = 1024;          // threads of the one-workgroup steps
constexpr int kRrT = 512;            // threads of the Rayleigh-Ritz step
constexpr int kEigMaxB = 48;         // block size limit (R <= 32)
constexpr int kEigMaxN = 1024;
constexpr int kEigKT = 32;           // rows of a staged LDS tile
constexpr int kEigMaxOuter = 30;
constexpr int kEigMaxDeg = 40;
constexpr double kEigTol = 2e-14;

// Reduction scratch of the Gram-Schmidt and residual steps.
struct OrthLds {
    double red[16][64];                 // per-group partial sums
    double hv[64];
};

struct EigLds {
    double H[kEigMaxB][kEigMaxB + 1];   // projected matrix, diagonalised in place
    double S[kEigMaxB][kEigMaxB + 1];   // its eigenvectors (columns)
    double t0[kEigKT][kEigMaxB];        // staged rows of a block
    double t1[kEigKT][kEigMaxB];
    OrthLds o;
    double theta[kEigMaxB];             // Ritz values, decreasing
    double res[kEigMaxB];
    double cs[kEigMaxB / 2], sn[kEigMaxB / 2];
    int pp[kEigMaxB / 2], qq[kEigMaxB / 2];
    int perm[kEigMaxB];                 // Jacobi index of the r-th largest Ritz value
    double ctl_c, ctl_e, ctl_tl;
    int ctl_state, ctl_deg;             // state: 1 converged, 0 filter, 2 plain power step
};


__device__ inline double eig_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sum over the workgroup, returned to every thread.
__device__ double eig_block_sum(double v, OrthLds& L) {
    v = eig_wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) L.red[threadIdx.x >> 6][0] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kEigT / 64; ++w) s += L.red[w][0];
    return s;
}

// Columns 0..b-1 of Y (n rows, row stride ld) made orthonormal in place: classical Gram-Schmidt,
// a second pass only when the first removed more than half of the column's squared norm (Kahan
// and Parlett's "twice is enough"); a column left with under 1e-8 of its norm is replaced by a
// unit vector and redone.  Y is in LDS or global memory.
__device__ void eig_orth(double* Y, int n, int b, int ld, OrthLds& L) {
    const int t = threadIdx.x, k = t & 63, g = t >> 6;
    for (int j = 0; j < b; ++j) {
        for (int attempt = 0; attempt < 4; ++attempt) {
            double before = 0.0, nn = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                double s = 0.0;
                if (k <= j) {
#pragma unroll 8
                    for (int i = g; i < n; i += 16) s = fma(Y[(int64_t)i * ld + k], Y[(int64_t)i * ld + j], s);
                }
                __syncthreads();
                L.red[g][k] = s;
                __syncthreads();
                if (t < 64) {
                    double h = 0.0;
                    for (int q = 0; q < 16; ++q) h += L.red[q][t];
                    L.hv[t] = h;
                }
                __syncthreads();
                if (pass == 0) before = L.hv[j];
                for (int i = t; i < n; i += kEigT) {
                    double v = Y[(int64_t)i * ld + j];
#pragma unroll 8
                    for (int q = 0; q < j; ++q) v = fma(-L.hv[q], Y[(int64_t)i * ld + q], v);
                    Y[(int64_t)i * ld + j] = v;
                }
                __syncthreads();
                double sq = 0.0;
                for (int i = t; i < n; i += kEigT) {
                    const double v = Y[(int64_t)i * ld + j];
                    sq = fma(v, v, sq);
                }
                nn = eig_block_sum(sq, L);
                if (pass == 0 && nn >= 0.5 * before) break;
            }
            if (nn > 1e-16 * before && nn > 0.0) {
                const double inv = 1.0 / sqrt(nn);
                for (int i = t; i < n; i += kEigT) Y[(int64_t)i * ld + j] *= inv;
                __syncthreads();
                break;
            }
            const int m = (j * 131 + attempt * 37 + 1) % n;
            for (int i = t; i < n; i += kEigT) Y[(int64_t)i * ld + j] = (i == m) ? 1.0 : 0.0;
            __syncthreads();
        }
    }
}

// Cyclic Jacobi on L.H (b x b, symmetric; for odd b a zero row and column b make the order
// m = b + 1 even) by the whole workgroup, accumulated into L.S, until the off-diagonal sum of
// squares is at most 1e-30 of the diagonal's.  A round-robin round holds m/2 disjoint rotations:
// threads k < m/2 compute them, then all threads apply them together as H <- J^T H J (a thread per
// 2 x 2 block: rows of one pair, columns of another) and S <- S J (a thread per row and pair); two
// barriers per round.
__device__ void eig_jacobi(EigLds& L, int b) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m = b + (b & 1);
    const int half = m / 2;
    for (int e = t; e < m * m; e += kRrT) L.S[e / m][e % m] = (e / m == e % m) ? 1.0 : 0.0;
    __syncthreads();
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int e = t; e < b * b; e += kRrT) {
            const double v = L.H[e / b][e % b];
            if (e / b == e % b) dia += v * v;
            else off += v * v;
        }
        off = eig_wave_sum(off);
        dia = eig_wave_sum(dia);
        if (lane == 0) {
            L.o.red[w][0] = off;
            L.o.red[w][1] = dia;
        }
        __syncthreads();
        off = 0.0;
        dia = 0.0;
        for (int q = 0; q < kRrT / 64; ++q) {
            off += L.o.red[q][0];
            dia += L.o.red[q][1];
        }
        __syncthreads();
        if (!(off > 1e-30 * dia)) break;
        for (int rnd = 0; rnd < m - 1; ++rnd) {
            if (t < half) {
                int p = (t == 0) ? m - 1 : (rnd + t) % (m - 1);
                int q = (t == 0) ? rnd : (rnd - t + (m - 1)) % (m - 1);
                if (p > q) { const int x = p; p = q; q = x; }
                double c = 1.0, sn = 0.0;
                const double hpq = L.H[p][q];
                if (hpq != 0.0) {
                    const double tau = (L.H[q][q] - L.H[p][p]) / (2.0 * hpq);
                    const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    sn = tt * c;
                }
                L.pp[t] = p;
                L.qq[t] = q;
                L.cs[t] = c;
                L.sn[t] = sn;
            }
            __syncthreads();
            for (int e = t; e < half * half; e += kRrT) {
                const int k1 = e / half, k2 = e % half;
                const int p1 = L.pp[k1], q1 = L.qq[k1], p2 = L.pp[k2], q2 = L.qq[k2];
                const double c1 = L.cs[k1], s1 = L.sn[k1], c2 = L.cs[k2], s2 = L.sn[k2];
                const double a = L.H[p1][p2], bb = L.H[p1][q2], cc = L.H[q1][p2], d = L.H[q1][q2];
                const double a1 = c1 * a - s1 * cc, b1 = c1 * bb - s1 * d;    // rows: J^T
                const double c1r = s1 * a + c1 * cc, d1 = s1 * bb + c1 * d;
                L.H[p1][p2] = c2 * a1 - s2 * b1;                                // columns: J
                L.H[p1][q2] = s2 * a1 + c2 * b1;
                L.H[q1][p2] = c2 * c1r - s2 * d1;
                L.H[q1][q2] = s2 * c1r + c2 * d1;
            }
            for (int e = t; e < half * m; e += kRrT) {
                const int k = e / m, j = e % m;
                const int p = L.pp[k], q = L.qq[k];
                const double c = L.cs[k], sn = L.sn[k];
                const double sp = L.S[j][p], sq = L.S[j][q];
                L.S[j][p] = c * sp - sn * sq;
                L.S[j][q] = sn * sp + c * sq;
            }
            __syncthreads();
        }
    }
}

// Rayleigh-Ritz on the orthonormal block Z with P = A Z: theta, X = Z S, AX = P S (decreasing).
__device__ void eig_rr(const double* Z, const double* P, double* X, double* AX, int n, int b, int bs,
                       EigLds& L) {
    const int t = threadIdx.x;
    constexpr int NE = (kEigMaxB * kEigMaxB + kRrT - 1) / kRrT;   // entries of H per thread
    double acc[NE];
#pragma unroll
    for (int m = 0; m < NE; ++m) acc[m] = 0.0;
    for (int i0 = 0; i0 < n; i0 += kEigKT) {
        __syncthreads();
        for (int e = t; e < kEigKT * bs; e += kRrT) {
            const int r = e / bs, c = e % bs;
            const bool v = i0 + r < n;
            L.t0[r][c] = v ? Z[(int64_t)(i0 + r) * bs + c] : 0.0;
            L.t1[r][c] = v ? P[(int64_t)(i0 + r) * bs + c] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < NE; ++m) {
            const int e = t + m * kRrT;
            if (e >= b * b) continue;
            const int a = e / b, c = e % b;
#pragma unroll
            for (int r = 0; r < kEigKT; ++r) acc[m] = fma(L.t0[r][a], L.t1[r][c], acc[m]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NE; ++m) {
        const int e = t + m * kRrT;
        if (e < b * b) L.H[e / b][e % b] = acc[m];
    }
    if (t < kEigMaxB) L.perm[t] = t < b ? t : 0;
    __syncthreads();
    for (int e = t; e < b * b; e += kRrT) {
        const int a = e / b, c = e % b;
        if (a < c) {
            const double v = 0.5 * (L.H[a][c] + L.H[c][a]);
            L.H[a][c] = v;
            L.H[c][a] = v;
        }
    }
    if ((b & 1) && t <= b) {   // odd b: a zero row and column b pair with the index left out
        L.H[b][t] = 0.0;
        L.H[t][b] = 0.0;
    }
    __syncthreads();
    eig_jacobi(L, b);
    __syncthreads();
    if (t < b) {
        const double v = L.H[t][t];
        int rank = 0;
        for (int q = 0; q < b; ++q) {
            const double w = L.H[q][q];
            rank += (w > v || (w == v && q < t)) ? 1 : 0;
        }
        if (rank < b) {
            L.perm[rank] = t;
            L.theta[rank] = v;
        }
    }
    __syncthreads();
    const int ng = bs >> 3;
    for (int item = t; item < n * ng; item += kRrT) {
        const int i = item / ng, c0 = (item % ng) * 8;
        double sx[8], sp[8];
        int pc[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            sx[j] = 0.0;
            sp[j] = 0.0;
            const int pj = L.perm[min(c0 + j, kEigMaxB - 1)];
            pc[j] = (c0 + j < b && pj >= 0 && pj < b) ? pj : -1;
        }
#pragma unroll 2
        for (int a = 0; a < b; ++a) {
            const double za = Z[(int64_t)i * bs + a], pa = P[(int64_t)i * bs + a];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const double s = pc[j] >= 0 ? L.S[a][pc[j]] : 0.0;
                sx[j] = fma(za, s, sx[j]);
                sp[j] = fma(pa, s, sp[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            X[(int64_t)i * bs + c0 + j] = sx[j];
            AX[(int64_t)i * bs + c0 + j] = sp[j];
        }
    }
    __syncthreads();
}

// Control block of one outer step, read back by the host: state 1 converged, 0 filter with
// degree deg on [c - e, c + e] normalised at tl, 2 plain power step (AX is the next block).
struct EigCtl {
    int32_t state, deg, pad0, pad1;
    double c, e, tl;
};

// Start block: the columns of A at its b largest diagonal entries (first index on ties).
__global__ __launch_bounds__(kEigT) void k_eig_start(const double* __restrict__ A, int n, int b, int bs,
                                                     double* __restrict__ Z) {
    __shared__ int sel[kEigMaxB];
    const int t = threadIdx.x;
    if (t < kEigMaxB) sel[t] = t < n ? t : 0;
    __syncthreads();
    if (t < n) {
        const double v = A[(int64_t)t * n + t];
        int rank = 0;
        for (int q = 0; q < n; ++q) {
            const double w = A[(int64_t)q * n + q];
            rank += (w > v || (w == v && q < t)) ? 1 : 0;
        }
        if (rank < b) sel[rank] = t;
    }
    __syncthreads();
    for (int e = t; e < n * bs; e += kEigT) {
        const int i = e / bs, c = e % bs;
        Z[e] = (c < b) ? A[(int64_t)sel[c] * n + i] : 0.0;
    }
}

// Orthonormalisation of a block: staged in LDS (row stride bs + 1) when it fits, else in place in
// global memory.
constexpr int kOrthLds = 18432;   // doubles: n (bs + 1) <= 18432 (144 KB)
__global__ __launch_bounds__(kEigT) void k_eig_orth_lds(double* Z, int n, int b, int bs) {
    __shared__ double Ys[kOrthLds];
    __shared__ OrthLds L;
    const int ld = bs + 1;
    for (int e = threadIdx.x; e < n * bs; e += kEigT) Ys[(e / bs) * ld + e % bs] = Z[e];
    __syncthreads();
    eig_orth(Ys, n, b, ld, L);
    for (int e = threadIdx.x; e < n * bs; e += kEigT) Z[e] = Ys[(e / bs) * ld + e % bs];
}

__global__ __launch_bounds__(kEigT) void k_eig_orth(double* Z, int n, int b, int bs) {
    __shared__ OrthLds L;
    eig_orth(Z, n, b, bs, L);
}

// out = alpha ((A Z) - shift Z) + beta prev, one workgroup per row i: thread t takes column
// t % bs and every (256 / bs)-th term of the contraction, partial sums added through LDS in a
// fixed order.  out may be prev, not Z.
constexpr int kMulT = 256;
__global__ __launch_bounds__(kMulT) void k_eig_mul(const double* __restrict__ A, int n, const double* Z, int bs,
                                                   double alpha, double shift, double beta, const double* prev,
                                                   double* out) {
    __shared__ double part[kMulT];
    const int i = blockIdx.x, t = threadIdx.x;
    const int ns = kMulT / bs;
    const int c = t % bs, sl = t / bs;
    double acc = 0.0;
    if (sl < ns) {
        const double* arow = A + (int64_t)i * n;
#pragma unroll 8
        for (int k = sl; k < n; k += ns) acc = fma(arow[k], Z[(int64_t)k * bs + c], acc);
    }
    part[t] = acc;
    __syncthreads();
    if (t >= bs) return;
    double v = 0.0;
    for (int q = 0; q < ns; ++q) v += part[q * bs + t];
    const int64_t idx = (int64_t)i * bs + t;
    v = alpha * (v - shift * Z[idx]);
    if (beta != 0.0) v += beta * prev[idx];
    out[idx] = v;
}

// Rayleigh-Ritz of one outer step (P = A Z given), the residual test and the next step's
// parameters (ctl).  Converged: V, lam receive the R leading pairs.  Filter: the first filtered
// block sig (AX - c X) / e is written over P.
__global__ __launch_bounds__(kRrT) void k_eig_rr(const double* Z, double* P, double* X, double* AX, int n, int R,
                                                  int b, int bs, double* __restrict__ V, double* __restrict__ lam,
                                                  EigCtl* __restrict__ ctl) {
    __shared__ EigLds L;
    const int t = threadIdx.x;
    eig_rr(Z, P, X, AX, n, b, bs, L);
    {
        const int r = t & 63, g = t >> 6;
        double s = 0.0;
        if (r < R) {
            const double th = L.theta[r];
            for (int i = g; i < n; i += kRrT / 64) {
                const double d = AX[(int64_t)i * bs + r] - th * X[(int64_t)i * bs + r];
                s = fma(d, d, s);
            }
        }
        L.o.red[g][r] = s;
        __syncthreads();
        if (t < R) {
            double q = 0.0;
            for (int w = 0; w < kRrT / 64; ++w) q += L.o.red[w][t];
            L.res[t] = sqrt(q);
        }
        __syncthreads();
    }
    if (t == 0) {
        const double th0 = L.theta[0];
        const double lim = kEigTol * fmax(th0, 0.0);
        bool conv = true;
        for (int r = 0; r < R; ++r) conv = conv && (L.res[r] <= lim);
        int state = conv ? 1 : 0, deg = 0;
        double c = 0.0, e = 0.0, tl = 0.0;
        const double hi = L.theta[b - 1];
        if (!conv) {
            if (!(hi > 0.0) || !(th0 > hi * (1.0 + 1e-12)) || b == n) {
                state = 2;
            } else {
                e = 0.5 * hi;
                c = 0.5 * hi;
                tl = (th0 - c) / e;
                deg = 2;
                for (int r = 0; r < R; ++r) {
                    const double q = fmax(L.res[r] / (0.5 * lim), 1.0);
                    const double tr = (L.theta[r] - c) / e;
                    if (!(tr > 1.0 + 1e-12)) {
                        deg = kEigMaxDeg;
                    } else {
                        const double d = ceil(acosh(q) / acosh(tr)) + 1.0;
                        deg = max(deg, (int)fmin(d, (double)kEigMaxDeg));
                    }
                }
                const double span = acosh(tl) - acosh(fmax((L.theta[R - 1] - c) / e, 1.0));
                if (span > 0.0) deg = min(deg, max(2, (int)fmin(log(1e12) / span, (double)kEigMaxDeg)));
                deg = min(deg, kEigMaxDeg);
            }
        }
        L.ctl_state = state;
        L.ctl_deg = deg;
        L.ctl_c = c;
        L.ctl_e = e;
        L.ctl_tl = tl;
        ctl->state = state;
        ctl->deg = deg;
        ctl->c = c;
        ctl->e = e;
        ctl->tl = tl;
    }
    __syncthreads();
    const int state = L.ctl_state;
    if (state == 1) {
        for (int e = t; e < R * n; e += kRrT) {
            const int r = e / n, i = e % n;
            V[e] = X[(int64_t)i * bs + r];
        }
        if (t < R) lam[t] = L.theta[t];
    } else if (state == 0) {
        const double c = L.ctl_c, e = L.ctl_e, sig = 1.0 / L.ctl_tl;
        for (int q = t; q < n * bs; q += kRrT) P[q] = sig * (AX[q] - c * X[q]) / e;
    }
}

// Eigenpair j of rank r: j = r when the solver returns them in decreasing order (desc), else
// j = n-1-r (ascending, all n of them); eigenvector j at V + j n.
__device__ inline int64_t eig_index(int r, int64_t n, int desc) { return desc ? r : n - 1 - r; }

// Tall case: U[i][r] = (sum_c Y[i][c] v_r[c]) / sqrt(lambda_r), c ascending.  A thread per row
// (RM >= R accumulators in registers); the eigenvectors are staged through LDS 64 entries at a
// time.
template <typename YT, int RM>
__global__ __launch_bounds__(128) void k_svd_left(const YT* __restrict__ Y, int64_t I, int K,
                                                  const double* __restrict__ V, const double* __restrict__ D,
                                                  int desc, int R, double* __restrict__ U) {
    __shared__ double vs[64][RM + 1];
    __shared__ double sq[RM];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * 128 + t;
    if (t < R) {
        const double lam = D[eig_index(t, K, desc)];
        sq[t] = (lam > 0.0) ? sqrt(lam) : 0.0;
    }
    double acc[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) acc[r] = 0.0;
    for (int k0 = 0; k0 < K; k0 += 64) {
        __syncthreads();
        for (int e = t; e < 64 * RM; e += 128) {
            const int c = e / RM, r = e % RM;
            vs[c][r] = (r < R && k0 + c < K) ? V[eig_index(r, K, desc) * K + k0 + c] : 0.0;
        }
        __syncthreads();
        if (i < I) {
            const YT* y = Y + i * K + k0;
            const int kc = min(64, K - k0);
#pragma unroll 8
            for (int c = 0; c < kc; ++c) {
                const double yv = (double)y[c];
#pragma unroll
                for (int r = 0; r < RM; ++r) acc[r] = fma(yv, vs[c][r], acc[r]);
            }
        }
    }
    if (i >= I) return;
#pragma unroll
    for (int r = 0; r < RM; ++r)
        if (r < R) U[i * R + r] = (sq[r] > 0.0) ? acc[r] / sq[r] : 0.0;
}

// The same for FP32 Y, R <= 16, K % 16 == 0: a wave per 16 rows of Y on v_mfma_f64_16x16x4f64
// (FP64 sums), Y read once with 16-byte loads.  Lane l = 16 g + c loads columns
// 16 t + 4 g .. 16 t + 4 g + 3 of row c of the tile and of eigenvector c; the u-th of the four
// MFMAs of block t takes the u-th of them (lane l supplies A[c][g] and B[g][c]), so the
// contraction runs over the columns 16 t + 4 g + u.  Lane l holds D[g + 4 v][c] in result v.
typedef double svd_d4_t __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_svd_left_mfma(const float* __restrict__ Y, int64_t I, int K,
                                                       const double* __restrict__ V, const double* __restrict__ D,
                                                       int desc, int R, double* __restrict__ U) {
    const int lane = threadIdx.x & 63;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (row0 >= I) return;   // wave-uniform
    const int c = lane & 15, g = lane >> 4;
    const bool rok = row0 + c < I, vok = c < R;
    const float* y = Y + (rok ? row0 + c : 0) * (int64_t)K + 4 * g;
    const double* v = V + (vok ? eig_index(c, K, desc) : 0) * K + 4 * g;
    svd_d4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int t = 0; t < K; t += 16) {
        float4 yv = make_float4(0.f, 0.f, 0.f, 0.f);
        double2 v01 = make_double2(0.0, 0.0), v23 = make_double2(0.0, 0.0);
        if (rok) yv = *(const float4*)(y + t);
        if (vok) {
            v01 = *(const double2*)(v + t);
            v23 = *(const double2*)(v + t + 2);
        }
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)yv.x, v01.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)yv.y, v01.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)yv.z, v23.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)yv.w, v23.y, acc, 0, 0, 0);
    }
    if (!vok) return;
    const double lam = D[eig_index(c, K, desc)];
    const double sq = (lam > 0.0) ? sqrt(lam) : 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t r = row0 + g + 4 * q;
        if (r < I) U[r * R + c] = (sq > 0.0) ? acc[q] / sq : 0.0;
    }
}

// Fat case: U[i][r] = entry i of the r-th leading eigenvector of Y Y^T.
__global__ void k_svd_fat(const double* __restrict__ V, int64_t I, int desc, int R, double* __restrict__ U) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= I * R) return;
    const int64_t i = e / R;
    const int r = (int)(e % R);
    U[e] = V[eig_index(r, I, desc) * I + i];
}

// Sign convention: in each column the entry of largest magnitude (the first one on ties) made
// positive.  One workgroup of 1024 threads per column: a (value, row) reduction per wave by
// shuffles, then over the waves in order.
__global__ __launch_bounds__(1024) void k_svd_sign(double* __restrict__ U, int64_t I, int R) {
    __shared__ double s_v[16];
    __shared__ int64_t s_i[16];
    __shared__ int s_flip;
    const int r = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
    double best = -1.0;
    int64_t bi = 0;
    for (int64_t i = t; i < I; i += 1024) {
        const double v = fabs(U[i * R + r]);
        if (v > best) { best = v; bi = i; }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const double ov = __shfl_xor(best, o);
        const int64_t oi = __shfl_xor(bi, o);
        if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (lane == 0) { s_v[w] = best; s_i[w] = bi; }
    __syncthreads();
    if (t == 0) {
        double b = s_v[0];
        int64_t ii = s_i[0];
        for (int q = 1; q < 16; ++q)
            if (s_v[q] > b || (s_v[q] == b && s_i[q] < ii)) { b = s_v[q]; ii = s_i[q]; }
        s_flip = (U[ii * R + r] < 0.0) ? 1 : 0;
    }
    __syncthreads();
    if (s_flip)
        for (int64_t i = t; i < I; i += 1024) U[i * R + r] = -U[i * R + r];
}

template <typename YT>
int left_typed(const tk_ctx* ctx, int mode, const YT* Y, const double* V, const double* D, int desc,
               double* U, hipStream_t s) {
    const int64_t I = ctx->dims[mode];
    const int K = (int)ctx->mode[mode].K, R = ctx->ranks[mode];
    if (std::is_same<YT, float>::value && R <= 16 && K % 16 == 0 && ((uintptr_t)V % 16) == 0 &&
        ((uintptr_t)Y % 16) == 0)
        k_svd_left_mfma<<<cdiv(I, 64), 256, 0, s>>>((const float*)Y, I, K, V, D, desc, R, U);
    else if (R <= 8) k_svd_left<YT, 8><<<cdiv(I, 128), 128, 0, s>>>(Y, I, K, V, D, desc, R, U);
    else if (R <= 16) k_svd_left<YT, 16><<<cdiv(I, 128), 128, 0, s>>>(Y, I, K, V, D, desc, R, U);
    else k_svd_left<YT, 32><<<cdiv(I, 128), 128, 0, s>>>(Y, I, K, V, D, desc, R, U);
    TK_LAUNCH_CHECK("k_svd_left");
    return TK_OK;
}

}  // namespace

void free_svd_ws(tk_ctx* ctx) {
    void* ps[] = {ctx->svd_d, ctx->svd_e, ctx->svd_info, ctx->eig_ws};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    ctx->svd_d = ctx->svd_e = nullptr;
    ctx->svd_info = nullptr;
    ctx->eig_ws = nullptr;
    if (ctx->rb) (void)rocblas_destroy_handle((rocblas_handle)ctx->rb);
    ctx->rb = nullptr;
}

// Forms U from the R leading eigenpairs (V, D) of the mode's symmetric matrix, fixes the signs and
// refreshes the low-precision copy.
static int svd_finish(tk_ctx* ctx, int mode, const void* Y, const double* V, const double* D, int desc,
                      double* U, hipStream_t s) {
    const int64_t I = ctx->dims[mode];
    const int R = ctx->ranks[mode];
    int st = TK_OK;
    if (qrp_route(ctx, mode) == 2) {
        k_svd_fat<<<cdiv(I * R, 256), 256, 0, s>>>(V, I, desc, R, U);
        TK_LAUNCH_CHECK("k_svd_fat");
    } else if (ctx->dtype == TK_F64) {
        if ((st = left_typed<double>(ctx, mode, (const double*)Y, V, D, desc, U, s))) return st;
    } else {
        if ((st = left_typed<float>(ctx, mode, (const float*)Y, V, D, desc, U, s))) return st;
    }
    k_svd_sign<<<(unsigned)R, 1024, 0, s>>>(U, I, R);
    TK_LAUNCH_CHECK("k_svd_sign");
    return convert_factor(ctx, mode, U, s);
}

// The subspace iteration on A (n x n); returns 1 when it converged (V, D then hold the R leading
// eigenpairs, decreasing), 0 when the library solver has to be used, or a negative status on
// error.  The outer steps are driven from here: each reads the step's control block back (one
// synchronisation of the stream) and enqueues the filter's products with the scalars of the
// three-term recurrence.
static int eig_top(tk_ctx* ctx, const double* A, int n, int R, double** V, double** D, hipStream_t s) {
    const int b = std::min(n, R + std::min(R, 16));
    const int bs = (b + 7) / 8 * 8;
    if (R < 1 || R > 32 || n < 1 || n > kEigMaxN || b > kEigMaxB) return 0;
    const size_t nbuf = (size_t)kEigMaxN * kEigMaxB;
    static_assert(sizeof(EigCtl) <= 8 * sizeof(double), "control block slot");
    const size_t ndbl = 4 * nbuf + (size_t)32 * kEigMaxN + 32 + 8;
    if (!ctx->eig_ws) {
        if (hipMalloc((void**)&ctx->eig_ws, ndbl * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            ctx->eig_ws = nullptr;
            return -set_error(TK_ERR_OOM, "eigensolver workspace allocation failed");
        }
    }
    double* buf = ctx->eig_ws;
    double* Vd = ctx->eig_ws + 4 * nbuf;
    double* lam = Vd + (size_t)32 * kEigMaxN;
    EigCtl* ctl = (EigCtl*)(lam + 32);
    auto blk = [&](int q) { return buf + (size_t)q * nbuf; };
    auto mul = [&](const double* Zin, double alpha, double shift, double beta, const double* prev, double* out) {
        k_eig_mul<<<(unsigned)n, kMulT, 0, s>>>(A, n, Zin, bs, alpha, shift, beta, prev, out);
        return hipGetLastError() == hipSuccess;
    };
    const bool orth_lds = (int64_t)n * (bs + 1) <= kOrthLds;
    auto orth = [&](double* Zb) {
        if (orth_lds) k_eig_orth_lds<<<1, kEigT, 0, s>>>(Zb, n, b, bs);
        else k_eig_orth<<<1, kEigT, 0, s>>>(Zb, n, b, bs);
        return hipGetLastError() == hipSuccess;
    };
    k_eig_start<<<1, kEigT, 0, s>>>(A, n, b, bs, blk(0));
    if (hipGetLastError() != hipSuccess || !orth(blk(0))) return -set_error(TK_ERR_HIP, "k_eig_start launch failed");
    int iz = 0;
    for (int outer = 0; outer <= kEigMaxOuter; ++outer) {
        const int ip = (iz + 1) & 3, ix = (iz + 2) & 3, iax = (iz + 3) & 3;
        if (!mul(blk(iz), 1.0, 0.0, 0.0, nullptr, blk(ip))) return -set_error(TK_ERR_HIP, "k_eig_mul launch failed");
        k_eig_rr<<<1, kRrT, 0, s>>>(blk(iz), blk(ip), blk(ix), blk(iax), n, R, b, bs, Vd, lam, ctl);
        if (hipGetLastError() != hipSuccess) return -set_error(TK_ERR_HIP, "k_eig_rr launch failed");
        EigCtl h{};
        if (hipMemcpyAsync(&h, ctl, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return -set_error(TK_ERR_HIP, "eigensolver control read-back failed");
        if (h.state == 1) {
            ctx->eig_outer = outer;
            *V = Vd;
            *D = lam;
            return 1;
        }
        if (outer == kEigMaxOuter) break;
        if (h.state == 2) {
            iz = iax;
        } else {
            // Y0 = X, Y1 (written over P by k_eig_rr); Y_{k+1} = 2 sig' (A - c) Y_k / e - sig sig' Y_{k-1}
            int i0 = ix, i1 = ip;
            double sig = 1.0 / h.tl;
            for (int k = 1; k < h.deg; ++k) {
                const double sig2 = 1.0 / (2.0 * h.tl - sig);
                if (!mul(blk(i1), 2.0 * sig2 / h.e, h.c, -sig * sig2, blk(i0), blk(i0)))
                    return -set_error(TK_ERR_HIP, "k_eig_mul launch failed");
                std::swap(i0, i1);
                sig = sig2;
            }
            iz = i1;
        }
        if (!orth(blk(iz))) return -set_error(TK_ERR_HIP, "k_eig_orth launch failed");
    }
    ctx->eig_outer = -1;
    return 0;
}

int svd_run(tk_ctx* ctx, int mode, const void* Y, double* U, hipStream_t s) {
    double* A = nullptr;
    int n = 0;
    int st = gram_run(ctx, mode, Y, &A, &n, s);
    if (st) return st;
    if (!(ctx->flags & TK_FLAG_SVD_LIB)) {
        double *V = nullptr, *D = nullptr;
        const int got = eig_top(ctx, A, n, ctx->ranks[mode], &V, &D, s);
        if (got < 0) return -got;
        if (got == 1) return svd_finish(ctx, mode, Y, V, D, 1, U, s);
    }
    ctx->eig_outer = -1;
    if (!ctx->rb) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success)
            return set_error(TK_ERR_HIP, "rocblas_create_handle failed");
        ctx->rb = h;
    }
    if (!ctx->svd_d) {
        const size_t nb = (size_t)kMaxK * sizeof(double);
        hipError_t e1 = hipMalloc((void**)&ctx->svd_d, nb);
        hipError_t e2 = hipMalloc((void**)&ctx->svd_e, nb);
        hipError_t e3 = hipMalloc((void**)&ctx->svd_info, 16);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
            (void)hipGetLastError();
            free_svd_ws(ctx);
            return set_error(TK_ERR_OOM, "SVD workspace allocation failed");
        }
    }
    rocblas_handle h = (rocblas_handle)ctx->rb;
    if (rocblas_set_stream(h, s) != rocblas_status_success) return set_error(TK_ERR_HIP, "rocblas_set_stream failed");
    const rocblas_status rs = rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, n, A, n, ctx->svd_d,
                                               ctx->svd_e, ctx->svd_info);
    if (rs != rocblas_status_success) return set_error(TK_ERR_HIP, "rocsolver_dsyevd failed (status %d)", (int)rs);
    return svd_finish(ctx, mode, Y, A, ctx->svd_d, 0, U, s);
}

}  // namespace tk
