// U_n <- QRP(Y_(n), R_n) in FP64 (paper Alg. 2; Sec. III-D).
//
// Only the first R_n columns of Q are needed, and the first R_n pivot steps of a Householder QRP
// depend only on the column norms of the partly reduced matrix.  Two routes compute them:
//
// Route 0 (tall Y, K_n <= 1024, R_n <= 32) - one pass over Y instead of R_n passes:
//   1. C = Y^T Y in FP64 (v_mfma_f64_16x16x4; products of fp32 inputs are exact in FP64).
//   2. Pivoted Cholesky of C, R_n steps.  The Schur-complement diagonal equals the squared norm
//      of each trailing sub-column that the Householder QRP compares, so the pivot sequence is the
//      QRP's; the first maximum is taken over the physically swapped order, as in the textbook
//      algorithm.  R11 = the R_n x R_n leading block of the triangular factor.
//   3. Q1 = Y[:, piv] R11^{-1}, re-orthogonalised once (Cholesky of Q1^T Q1).
//   4. Householder signs: Q_house = Q1 S with s_j chosen, column by column, so that the LU
//      elimination (without pivoting) of the top R_n x R_n block of Q1 S - I has pivots <= -1 -
//      the reconstruction of Householder vectors from an orthonormal basis (Ballard et al.,
//      "Reconstructing Householder vectors from tall-skinny QR", 2014).  With the reflector
//      v = x + sgn(x_0) ||x|| e_1, the Householder Q satisfies exactly this condition.
//   A Cholesky breakdown or a pivot below 1e-12 of the largest diagonal (rank deficiency) sets a
//   device flag and the Householder kernel below runs instead, on the device, without a host sync.
//
// Route 1 (R_n > 32, K_n > 1024, fat Y without the fat rule, or the fallback) - eager textbook
// Householder QRP in one workgroup: exact trailing-norm recompute, first-maximum pivot,
// v = x + sgn(x_0)||x|| e_1.
// Route 2 (fat Y, K_n > I_n) - the same kernel on Y Y^T (I_n x I_n), as Sec. III-D prescribes.
#include <hip/hip_cooperative_groups.h>

#include "internal.h"

namespace tk {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <typename YT>
__device__ inline double yld(const YT* Y, int64_t i) { return (double)Y[i]; }

// ---- Route 0 -------------------------------------------------------------------------------

// The chunk loop of k_gram_rows for one pair shape (see there): LA / LB live 16-column tiles of
// the two panels; a diagonal pair stages one panel and reads both operands from it.  Each thread
// stages column cc of each panel for rows rw + 4k (k < 8) of a 32-row chunk; full chunks load from
// 32-bit byte offsets off a uniform base (off32: the whole Y below 4 GB), the last, partial chunk
// clamped loads.
template <typename YT, int LA, int LB, bool DIAG>
__device__ __attribute__((always_inline)) inline void gram_rows_loop(const YT* __restrict__ Y, int n, int bi, int bj,
                                                                     int64_t r0, int64_t r1, bool off32,
                                                                     YT (*As)[32][65], YT (*Bs)[32][65], d4_t* acc) {
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int kq = lane >> 4, c16 = lane & 15;
    const int cc = lane, rw = w;
    const bool oka = bi * 64 + cc < n, okb = bj * 64 + cc < n;
    const uint32_t ca = (uint32_t)(bi * 64 + (oka ? cc : 0)), cb = (uint32_t)(bj * 64 + (okb ? cc : 0));
    const uint32_t rowb = (uint32_t)n * (uint32_t)sizeof(YT);   // bytes per row of Y
    YT xa[8], xb[8];
    auto stage = [&](int64_t row0) __attribute__((always_inline)) {
        if (off32 && row0 + 32 <= r1) {
            const uint32_t o = (uint32_t)(row0 + rw) * rowb;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                xa[k] = *(const YT*)((const char*)Y + (o + 4u * (uint32_t)k * rowb + ca * (uint32_t)sizeof(YT)));
                if constexpr (!DIAG)
                    xb[k] = *(const YT*)((const char*)Y + (o + 4u * (uint32_t)k * rowb + cb * (uint32_t)sizeof(YT)));
            }
        } else {
            // clamped rows (the row past r1 repeats row r1 - 1 and is masked when staged)
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int64_t row = min(row0 + rw + 4 * k, r1 - 1);
                xa[k] = Y[row * n + ca];
                if constexpr (!DIAG) xb[k] = Y[row * n + cb];
            }
        }
    };
    stage(r0);
    int buf = 0;
    for (int64_t row0 = r0; row0 < r1; row0 += 32) {
        const bool full = row0 + 32 <= r1;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const bool rv = full || row0 + rw + 4 * k < r1;
            As[buf][rw + 4 * k][cc] = (rv && oka) ? xa[k] : YT(0);
            if constexpr (!DIAG) Bs[buf][rw + 4 * k][cc] = (rv && okb) ? xb[k] : YT(0);
        }
        __syncthreads();
        if (row0 + 32 < r1) stage(row0 + 32);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int rr = 8 * w + 4 * h + kq;
            double av[4], bv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (t < LA) av[t] = (double)As[buf][rr][16 * t + c16];
                if constexpr (!DIAG) {
                    if (t < LB) bv[t] = (double)Bs[buf][rr][16 * t + c16];
                } else {
                    bv[t] = av[t];
                }
            }
#define TK_GM(ti, tj)                                                                               \
    if constexpr ((ti) < LA && (tj) < LB && (!DIAG || (ti) <= (tj)))                                \
        acc[4 * (ti) + (tj)] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ti], bv[tj], acc[4 * (ti) + (tj)], 0, 0, 0);
            TK_GM(0, 0) TK_GM(0, 1) TK_GM(0, 2) TK_GM(0, 3)
            TK_GM(1, 0) TK_GM(1, 1) TK_GM(1, 2) TK_GM(1, 3)
            TK_GM(2, 0) TK_GM(2, 1) TK_GM(2, 2) TK_GM(2, 3)
            TK_GM(3, 0) TK_GM(3, 1) TK_GM(3, 2) TK_GM(3, 3)
#undef TK_GM
        }
        buf ^= 1;
    }
}

// Partial C = Y^T Y over one slab of rows for one upper pair (bi <= bj) of 64-column blocks.  Rows
// come in chunks of 32, staged through LDS in Y's precision (the next chunk's loads in flight
// during the current one); wave w takes the 4-row steps 2w and 2w+1 of
// each chunk and accumulates all 16 16x16 tiles of the pair for them, so that per step a lane
// reads 4 + 4 operands for up to 16 v_mfma_f64_16x16x4f64 (lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and holds D[l/16 + 4v][l%16] in result v).  Tiles that start at or past column n
// are skipped, and so are the lower tiles (ti > tj) of a diagonal pair, which reads its one panel
// once and writes the lower tiles as the mirror of the upper ones: on 100 columns 28 tile MFMAs
// per step instead of 48.  At the end the four waves' sums are added through LDS in wave order.
// blockIdx.x enumerates the upper block pairs, blockIdx.y the row slab; part[split] receives the
// n x n partial (entries of upper block pairs only).
template <typename YT>
__global__ __launch_bounds__(256, 2) void k_gram_rows(const YT* __restrict__ Y, int64_t m, int n,
                                                      int nb, int64_t slab, bool off32, double* __restrict__ part) {
    constexpr int kStage = 2 * 32 * 65 * (int)sizeof(YT);
    static_assert(2 * kStage >= 64 * 64 * (int)sizeof(double), "the reduction reuses the staging LDS");
    __shared__ __align__(16) char lds[2 * kStage];
    YT(*As)[32][65] = (YT(*)[32][65])lds;
    YT(*Bs)[32][65] = (YT(*)[32][65])(lds + kStage);
    int b = blockIdx.x, bi = 0;
    while (b >= nb - bi) { b -= nb - bi; ++bi; }
    const int bj = bi + b;
    const bool diag = bi == bj;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int kq = lane >> 4, c16 = lane & 15;
    // live tiles: bit 4 ti + tj
    unsigned live = 0;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
            if (64 * bi + 16 * ti < n && 64 * bj + 16 * tj < n && !(diag && ti > tj)) live |= 1u << (4 * ti + tj);
    const int64_t r0 = (int64_t)blockIdx.y * slab;
    const int64_t r1 = min(m, r0 + slab);
    d4_t acc[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] = d4_t{0, 0, 0, 0};
    // the chunk loop, compiled per pair shape: LA / LB live 16-column tiles in the two panels, and
    // a diagonal pair (one panel, upper tiles only)
    const int la = min(4, (n - 64 * bi + 15) / 16), lb = min(4, (n - 64 * bj + 15) / 16);
    if (diag) {
        switch (la) {
            case 1: gram_rows_loop<YT, 1, 1, true>(Y, n, bi, bj, r0, r1, off32, As, Bs, acc); break;
            case 2: gram_rows_loop<YT, 2, 2, true>(Y, n, bi, bj, r0, r1, off32, As, Bs, acc); break;
            case 3: gram_rows_loop<YT, 3, 3, true>(Y, n, bi, bj, r0, r1, off32, As, Bs, acc); break;
            default: gram_rows_loop<YT, 4, 4, true>(Y, n, bi, bj, r0, r1, off32, As, Bs, acc); break;
        }
    } else {   // bi < bj: the first panel is full
        switch (lb) {
            case 1: gram_rows_loop<YT, 4, 1, false>(Y, n, bi, bj, r0, r1, off32, As, Bs, acc); break;
            case 2: gram_rows_loop<YT, 4, 2, false>(Y, n, bi, bj, r0, r1, off32, As, Bs, acc); break;
            case 3: gram_rows_loop<YT, 4, 3, false>(Y, n, bi, bj, r0, r1, off32, As, Bs, acc); break;
            default: gram_rows_loop<YT, 4, 4, false>(Y, n, bi, bj, r0, r1, off32, As, Bs, acc); break;
        }
    }
    // the four waves' sums, added in wave order through LDS: red[tile][v][lane]
    __syncthreads();
    double* red = (double*)lds;
    for (int ww = 0; ww < 4; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int t = 0; t < 16; ++t)
                if (live & (1u << t))
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        double* r = red + (t * 4 + v) * 64 + lane;
                        *r = (ww == 0) ? acc[t][v] : *r + acc[t][v];
                    }
        }
        __syncthreads();
    }
    double* P = part + (int64_t)blockIdx.y * n * n;
    for (int e = threadIdx.x; e < 16 * 4 * 64; e += 256) {
        const int t = e >> 8, v = (e >> 6) & 3, l = e & 63;
        if (!(live & (1u << t))) continue;
        const int ti = t >> 2, tj = t & 3;
        const int i = bi * 64 + 16 * ti + (l >> 4) + 4 * v;
        const int j = bj * 64 + 16 * tj + (l & 15);
        if (i < n && j < n) {
            const double x = red[e];
            P[(int64_t)i * n + j] = x;
            if (diag && ti < tj) P[(int64_t)j * n + i] = x;
        }
    }
}

// Gram partials of Y (m x n) into part[nsplit][n][n]
template <typename YT>
void launch_gram_partial(const YT* Y, int64_t m, int n, int nb, int nsplit, int64_t slab, double* part,
                         hipStream_t s) {
    const dim3 g((unsigned)(nb * (nb + 1) / 2), (unsigned)nsplit);
    const bool off32 = (uint64_t)m * (uint64_t)n * sizeof(YT) < (1ull << 32);
    k_gram_rows<YT><<<g, 256, 0, s>>>(Y, m, n, nb, slab, off32, part);
}

// Sums the partials of entries in upper block pairs (bi <= bj) and writes both C[i][j] and its
// mirror C[j][i].  A workgroup of 4 waves takes 64 entries: wave w adds the splits w, w + 4, ... in order, and the
// four sums are added in wave order (every entry in the same order, so equal columns give equal
// sums).
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ part, int nsplit, int n,
                                                     double* __restrict__ C) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t nn = (int64_t)n * n;
    const int64_t e = (int64_t)blockIdx.x * 64 + lane;
    const bool ok = e < nn && ((int)(e / n) >> 6) <= ((int)(e % n) >> 6);
    red[w][lane] = (ok && w < nsplit) ? sum_strided(part + w * nn + e, (nsplit - w + 3) / 4, 4 * nn) : 0.0;
    __syncthreads();
    if (w == 0 && ok) {
        const double s = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        const int i = (int)(e / n), j = (int)(e % n);
        C[e] = s;
        if ((i >> 6) != (j >> 6)) C[(int64_t)j * n + i] = s;
    }
}

// Wave-wide maximum / minimum, the result in every lane: butterflies inside each row of 16 lanes
// through DPP (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror), then the
// four row results through readlane.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ inline double wave_max_f64(double v) {
    v = fmax(v, dpp_f64<0xB1>(v));
    v = fmax(v, dpp_f64<0x4E>(v));
    v = fmax(v, dpp_f64<0x141>(v));
    v = fmax(v, dpp_f64<0x140>(v));
    return fmax(fmax(wave_bcast(v, 15), wave_bcast(v, 31)), fmax(wave_bcast(v, 47), wave_bcast(v, 63)));
}
__device__ inline int wave_min_i32(int v) {
    v = min(v, __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(0, v, 0x140, 0xf, 0xf, false));
    return min(min(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31)),
               min(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63)));
}

// Pivoted Cholesky of C for R <= RM steps with L (R x n) in LDS: the decisions and arithmetic of
// k_pivchol below, with threads owning columns instead of positions.  Thread c keeps column c's
// Schur-complement diagonal and its current position (pivoting swaps positions; among equal
// maxima the lowest position wins).  Per step j, one barrier: each wave finds its candidate (the
// maximum diagonal over positions >= j, then the lowest position holding it, by DPP reductions)
// and posts it; after the barrier every thread picks the winner among the waves' candidates,
// swaps positions, reads row cs of C for its column and the pivot column of L (all RM rows at
// once, rows i >= j taken as zero, so the zero terms leave the sum unchanged), and writes its
// new entry of L.  R11 is gathered from the pivot columns of L and
// R11^{-1} formed by back substitution, thread c computing column c.
template <int RM>
__global__ __launch_bounds__(1024) void k_pivchol_cols(const double* __restrict__ C, int n, int R,
                                                       double* __restrict__ R11, double* __restrict__ Rinv,
                                                       int32_t* __restrict__ pivw, int32_t* __restrict__ flag,
                                                       double* __restrict__ gaps) {
    constexpr int kNone = 0x7fffffff;
    extern __shared__ double Ls[];              // [RM][n], row i = L[i][*] by column id
    __shared__ double s_v[2][16], s_d[2][16], s_v2[2][16];
    __shared__ int s_p[2][16], s_c[2][16];
    __shared__ double s_mx[16];
    __shared__ int s_piv[RM];
    __shared__ double sR[RM][RM + 1];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nw = (int)(blockDim.x >> 6);
    const bool valid = tid < n;
    for (int e = tid; e < RM * n; e += blockDim.x) Ls[e] = 0.0;
    double d = valid ? C[(int64_t)tid * n + tid] : -1.0;
    int pos = valid ? tid : kNone;
    {
        const double v = wave_max_f64(d);
        if (lane == 0) s_mx[wid] = v;
    }
    __syncthreads();
    double dmax0 = s_mx[0];
    for (int k = 1; k < nw; ++k) dmax0 = fmax(dmax0, s_mx[k]);
    bool bad = false;
    for (int j = 0; j < R; ++j) {
        const int b = j & 1;
        // the wave's candidate: maximum diagonal over positions >= j, lowest position holding it
        const bool cand = pos >= j && pos != kNone;
        const double v = cand ? d : -INFINITY;
        const double mx = wave_max_f64(v);
        const int lp = wave_min_i32((cand && v == mx) ? pos : kNone);
        // the wave's runner-up (equal to mx when the maximum is tied): the pivot gap of step j
        const double mx2 = wave_max_f64((cand && pos != lp) ? v : -INFINITY);
        if (lane == 0) s_v2[b][wid] = mx2;
        double touch = 0.0;
        if (lp != kNone) {
            const uint64_t h = __ballot(pos == lp);
            const int o = (int)__builtin_ctzll(h);
            const double dw = wave_bcast(d, o);
            if (lane == 0) { s_v[b][wid] = mx; s_p[b][wid] = lp; s_c[b][wid] = wid * 64 + o; s_d[b][wid] = dw; }
            // start fetching the candidate's row of C (one load per 32 bytes) while the waves
            // compare: the winner's row is then in this CU's cache when it is read below
            touch = C[(int64_t)(wid * 64 + o) * n + min(4 * lane, n - 1)];
        } else if (lane == 0) {
            s_v[b][wid] = -INFINITY; s_p[b][wid] = kNone; s_c[b][wid] = 0; s_d[b][wid] = 0.0;
        }
        __syncthreads();
        double bv = s_v[b][0];
        int bp = s_p[b][0], cs = s_c[b][0];
        double djj = s_d[b][0];
        int kw = 0;
        for (int k = 1; k < nw; ++k) {
            const double v2 = s_v[b][k];
            const int p2 = s_p[b][k];
            if (v2 > bv || (v2 == bv && p2 < bp)) { bv = v2; bp = p2; cs = s_c[b][k]; djj = s_d[b][k]; kw = k; }
        }
        if (tid == 0) {
            // relative gap between the chosen squared trailing norm and the largest other one
            double second = s_v2[b][kw];
            for (int k = 0; k < nw; ++k)
                if (k != kw) second = fmax(second, s_v[b][k]);
            gaps[j] = (second == -INFINITY) ? 1.0 : (bv > 0.0 ? (bv - second) / bv : 0.0);
        }
        if (bp == kNone) {
            // no comparable candidate (NaN): position j stays; its column and diagonal
            bp = j;
            const uint64_t h = __ballot(pos == j);
            if (h) {
                const int o = (int)__builtin_ctzll(h);
                s_c[b][0] = wid * 64 + o;   // one wave holds position j
                s_d[b][0] = wave_bcast(d, o);
            }
            __syncthreads();
            cs = s_c[b][0];
            djj = s_d[b][0];
        }
        if (pos == bp) pos = j;
        else if (pos == j) pos = bp;
        if (!(djj > 1e-12 * dmax0)) bad = true;
        const double ljj = bad ? 1.0 : sqrt(djj);
        double acc = C[(int64_t)cs * n + (valid ? tid : 0)];
        // rows i >= j read as zero (row j of the pivot column may already hold ljj)
        double lc[RM], lp2[RM];
#pragma unroll
        for (int i = 0; i < RM; ++i) {
            const double a0 = Ls[i * n + (valid ? tid : 0)];
            const double a1 = Ls[i * n + cs];
            lc[i] = (i < j) ? a0 : 0.0;
            lp2[i] = (i < j) ? a1 : 0.0;
        }
        if (tid == cs) {
            Ls[j * n + cs] = ljj;
        } else if (valid && pos > j) {
#pragma unroll
            for (int i = 0; i < RM; ++i) acc -= lc[i] * lp2[i];
            const double l = acc / ljj;
            Ls[j * n + tid] = l;
            d -= l * l;
        }
        asm volatile("" ::"v"(touch));   // keeps the prefetch (complete by now: loads retire in order)
    }
    if (pos < R) s_piv[pos] = tid;
    __syncthreads();
    for (int e = tid; e < R * R; e += blockDim.x) {
        const int i = e / R, jj = e % R;
        const double r = (i <= jj) ? Ls[i * n + s_piv[jj]] : 0.0;
        R11[e] = r;
        sR[i][jj] = r;
    }
    if (tid < R) pivw[tid] = s_piv[tid];
    __syncthreads();
    // column c of R11^{-1} in thread c: x_k = b_k / r_kk for k = c down to 0, removing each x_k
    // from the rows above it
    if (tid < R) {
        double bb[RM], x[RM];
#pragma unroll
        for (int i = 0; i < RM; ++i) {
            bb[i] = (i == tid) ? 1.0 : 0.0;
            x[i] = 0.0;
        }
#pragma unroll
        for (int k = RM - 1; k >= 0; --k) {
            if (k <= tid) {
                x[k] = bb[k] / sR[k][k];
#pragma unroll
                for (int i = 0; i < k; ++i) bb[i] -= sR[i][k] * x[k];
            }
        }
#pragma unroll
        for (int i = 0; i < RM; ++i)
            if (i < R) Rinv[i * R + tid] = (i <= tid) ? x[i] : 0.0;
    }
    if (tid == 0) *flag = bad ? 1 : 0;
}

// Pivoted Cholesky of C (n <= 1024), R steps, one workgroup of ceil(n/64) waves; thread t owns
// position t of the (physically swapped) column order and keeps that position's column id and
// Schur-complement diagonal in registers.  Per step: a block argmax (first maximum) of the
// diagonals at positions >= j, one barrier, then the swap of positions j and the winner done by
// the two threads involved, and the new row of L^T (entry (i, c) at i * n + c, indexed by column
// id) from one row of C (C is symmetric, so column cs is read as row cs).  Per-step LDS slots
// are double-buffered, so one barrier per step orders everything.  L lives in LDS when kLdsL.
// R11^{-1} is formed by column-oriented back substitution, one wave per column.
template <bool kLdsL>
__global__ __launch_bounds__(1024) void k_pivchol(const double* __restrict__ C, int n, int R,
                                                  double* __restrict__ Lg,
                                                  double* __restrict__ R11, double* __restrict__ Rinv,
                                                  int32_t* __restrict__ pivw, int32_t* __restrict__ flag) {
    extern __shared__ double Ls[];
    __shared__ double s_wv[2][16];
    __shared__ int s_wp[2][16];
    __shared__ int s_wc[2][16];
    __shared__ int s_jcol[2];
    __shared__ double s_jd[2];
    __shared__ double s_mx[16];
    __shared__ int s_piv[32];
    __shared__ double sR[32][33];
    double* L;
    if constexpr (kLdsL) L = Ls;
    else L = Lg;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nw = (int)(blockDim.x >> 6);
    int mycol = tid;
    double myd = (tid < n) ? C[(int64_t)tid * n + tid] : -1.0;
    double dmax0;
    {
        double v = myd;
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
        if (lane == 0) s_mx[wid] = v;
        __syncthreads();
        dmax0 = s_mx[0];
        for (int k = 1; k < nw; ++k) dmax0 = fmax(dmax0, s_mx[k]);
    }
    bool bad = false;
    for (int j = 0; j < R; ++j) {
        const int b = j & 1;
        if (tid == j) { s_jcol[b] = mycol; s_jd[b] = myd; }
        // wave argmax: the maximum value, then the lowest lane holding it (positions grow with lanes)
        const bool cand = tid >= j && tid < n;
        const double v = cand ? myd : -INFINITY;
        double mx = v;
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
        const uint64_t hold = __ballot(cand && v == mx);
        const int hl = hold ? (int)__builtin_ctzll(hold) : 0;
        const int hcol = __builtin_amdgcn_readlane(mycol, hl);
        if (lane == 0) {
            s_wv[b][wid] = hold ? mx : -INFINITY;
            s_wp[b][wid] = hold ? wid * 64 + hl : n;
            s_wc[b][wid] = hcol;
        }
        __syncthreads();
        double bv = s_wv[b][0];
        int bp = s_wp[b][0], bc = s_wc[b][0];
        for (int k = 1; k < nw; ++k) {
            const double v2 = s_wv[b][k];
            const int p2 = s_wp[b][k];
            if (v2 > bv || (v2 == bv && p2 < bp)) { bv = v2; bp = p2; bc = s_wc[b][k]; }
        }
        if (bp >= n) { bp = j; bc = s_jcol[b]; bv = s_jd[b]; }   // no comparable candidate (NaN)
        const int cs = bc;
        const double djj = bv;
        if (tid == bp && bp != j) { mycol = s_jcol[b]; myd = s_jd[b]; }
        if (tid == j) { mycol = cs; myd = djj; }
        if (!(djj > 1e-12 * dmax0)) bad = true;
        const double ljj = bad ? 1.0 : sqrt(djj);
        if (tid == j) L[(int64_t)j * n + cs] = ljj;
        if (tid > j && tid < n) {
            const int c = mycol;
            double acc = C[(int64_t)cs * n + c];
#pragma unroll 8
            for (int i = 0; i < j; ++i) acc -= L[(int64_t)i * n + c] * L[(int64_t)i * n + cs];
            const double l = acc / ljj;
            L[(int64_t)j * n + c] = l;
            myd -= l * l;
        }
    }
    if (tid < R) s_piv[tid] = mycol;
    __syncthreads();
    if (tid < R) pivw[tid] = mycol;
    for (int e = tid; e < R * R; e += blockDim.x) {
        const int i = e / R, jj = e % R;
        const double r = (i <= jj) ? L[(int64_t)i * n + s_piv[jj]] : 0.0;
        R11[e] = r;
        sR[i][jj] = r;
    }
    __syncthreads();
    // column c of R11^{-1}: lane i holds b_i; step k finalises x_k = b_k / r_kk and removes it
    for (int c = wid; c < R; c += nw) {
        double bi = (lane == c) ? 1.0 : 0.0;
        double xi = 0.0;
        for (int k = c; k >= 0; --k) {
            const double xk = wave_bcast(bi / sR[k][k], k);
            if (lane == k) xi = xk;
            if (lane < k) bi -= sR[lane][k] * xk;
        }
        if (lane < R) Rinv[lane * R + c] = (lane <= c) ? xi : 0.0;
    }
    if (tid == 0) *flag = bad ? 1 : 0;
}

// Q1 = Y[:, piv] R11^{-1} and the partial Gram Q1^T Q1 of the workgroup's 64 rows.  Four
// threads share a row (thread (r, g) forms q[r][c] for c = g, g + 4, ..., each as b times the
// precomputed upper-triangular inverse, so the R outputs of a row are independent sums), then one
// Gram entry per thread.  No flag check: after a breakdown the values are unused.
template <typename YT>
__global__ __launch_bounds__(256) void k_q1_gram(const YT* __restrict__ Y, int64_t m, int n, int R,
                                                 const int32_t* __restrict__ pivw,
                                                 const double* __restrict__ Rinv,
                                                 double* __restrict__ part2) {
    __shared__ double sRi[32 * 32];
    __shared__ int sp[32];
    __shared__ double q[64][33];
    const int tid = threadIdx.x;
    for (int e = tid; e < R * R; e += 256) sRi[e] = Rinv[e];
    if (tid < R) sp[tid] = pivw[tid];
    __syncthreads();
    const int r = tid >> 2, g = tid & 3;
    const int64_t row = (int64_t)blockIdx.x * 64 + r;
    // unconditional loads from clamped addresses (all in flight together), masked afterwards
    const int64_t rowc = row < m ? row : m - 1;
    double b[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) b[j] = yld(Y, rowc * n + sp[j < R ? j : 0]);
#pragma unroll
    for (int j = 0; j < 32; ++j) b[j] = (j < R && row < m) ? b[j] : 0.0;
    for (int c = g; c < R; c += 4) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 32; ++i)
            if (i <= c && i < R) acc += b[i] * sRi[i * R + c];
        q[r][c] = acc;
    }
    __syncthreads();
    const int nr = (int)min<int64_t>(64, m - (int64_t)blockIdx.x * 64);
    for (int pr = tid; pr < R * R; pr += 256) {
        const int a = pr / R, bb = pr % R;
        double acc = 0.0;
        for (int rr = 0; rr < nr; ++rr) acc += q[rr][a] * q[rr][bb];
        part2[(int64_t)blockIdx.x * R * R + pr] = acc;
    }
}

// G2[e] = sum over workgroups of part2[k][e], one workgroup per entry, fixed-order tree.
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, int nparts, int stride,
                                                      const int32_t* __restrict__ flag, double* __restrict__ out) {
    if (flag && *flag) return;
    __shared__ double red[256];
    const int e = blockIdx.x;
    double acc = 0.0;
    for (int k = threadIdx.x; k < nparts; k += 256) acc += part[(int64_t)k * stride + e];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[e] = red[0];
}

// Finishing algebra of route 0 in one wave, register-resident (RMAX >= R, RMAX in {8, 16, 32}):
//   Cholesky G2 = R2^T R2 (Gram of Q1; lane c holds column c, right-looking, broadcasts by
//   v_readlane);  M' = R11^{-1} R2^{-1} (lane i solves row i of M' R2 = R11^{-1});
//   T = Y[0:R, piv] M';  sign rule: LU of (T S - I) without pivoting with s_j chosen so that each
//   pivot is <= -1 (lane i holds row i of T);  M = M' S, so that U = Y[:, piv] M.
// A Cholesky breakdown sets the device flag (the gated Householder kernel then runs).
template <typename YT, int RMAX, bool kExact>
__global__ __launch_bounds__(64) void k_qrp_finish(const YT* __restrict__ Y, int n, int R_arg,
                                                   const int32_t* __restrict__ pivw,
                                                   const double* __restrict__ Rinv,
                                                   const double* __restrict__ G2in,
                                                   int32_t* __restrict__ flag, double* __restrict__ Mout,
                                                   int32_t* __restrict__ piv_out) {
    if (*flag) return;
    const int R = kExact ? RMAX : R_arg;     // kExact: R == RMAX, the guards below fold away
    __shared__ double sR2[RMAX][RMAX + 1];   // R2 (upper)
    __shared__ double sM[RMAX][RMAX + 1];    // M'
    const int lane = threadIdx.x;
    const bool live = lane < R;
    const int lr = live ? lane : 0;
    double w[RMAX], t[RMAX], yv[RMAX];
    // lane c: column c of G2; lane i: row i of R11^{-1} (t) and row i of Y[0:R, piv] (yv) - loads
    // in flight together
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        const int kk = k < R ? k : 0;
        w[k] = G2in[kk * R + lr];
        t[k] = Rinv[lr * R + kk];
        yv[k] = yld(Y, (int64_t)lr * n + pivw[kk]);
    }
    bool bad = false;
    // Cholesky, right-looking: after step j, w[j] of lane c is R2[j][c]
#pragma unroll
    for (int j = 0; j < RMAX; ++j) {
        if (j < R) {
            const double d = wave_bcast(w[j], j);
            if (!(d > 0.0)) bad = true;
            const double rjj = (d > 0.0) ? sqrt(d) : 1.0;
            const double r = (lane == j) ? rjj : ((lane > j) ? w[j] / rjj : 0.0);
            w[j] = r;
#pragma unroll
            for (int k = j + 1; k < RMAX; ++k)
                if (k < R) w[k] -= wave_bcast(r, k) * r;
        }
    }
#pragma unroll
    for (int k = 0; k < RMAX; ++k)
        if (live && k < R) sR2[k][lane] = w[k];
    __syncthreads();
    // row i of M' = row i of R11^{-1} times R2^{-1}: forward substitution over columns
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
        if (c < R) {
            double acc = t[c];
#pragma unroll
            for (int k = 0; k < c; ++k) acc -= t[k] * sR2[k][c];
            t[c] = acc / sR2[c][c];
        }
    }
#pragma unroll
    for (int c = 0; c < RMAX; ++c)
        if (live && c < R) sM[lane][c] = t[c];
    // row i of T = Y[0:R, piv] M' (t)
#pragma unroll
    for (int k = 0; k < RMAX; ++k) w[k] = yv[k];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < RMAX; ++k)
            if (k < R) acc += w[k] * sM[k][c];
        t[c] = acc;
    }
    // sign rule on the LU of T S - I (lane i holds row i)
    double sg[RMAX];
#pragma unroll
    for (int j = 0; j < RMAX; ++j) {
        sg[j] = 1.0;
        if (j < R) {
            sg[j] = (wave_bcast(t[j], j) >= 0.0) ? -1.0 : 1.0;
            t[j] *= sg[j];
            if (lane == j) t[j] -= 1.0;
            const double pv = wave_bcast(t[j], j);
            const double f = t[j] / pv;
#pragma unroll
            for (int c = j + 1; c < RMAX; ++c) {
                const double tjc = wave_bcast(t[c], j);
                if (c < R && lane > j) t[c] -= f * tjc;
            }
        }
    }
    if (live) {
#pragma unroll
        for (int c = 0; c < RMAX; ++c)
            if (c < R) Mout[lane * R + c] = sM[lane][c] * sg[c];
        if (piv_out) piv_out[lane] = pivw[lane];
    }
    if (lane == 0 && bad) *flag = 1;
}

// ---- Routes 1 and 2 ------------------------------------------------------------------------

// A = Y Y^T (I x I), FP64 accumulation.
template <typename YT>
__global__ void k_syrk_rows(const YT* __restrict__ Y, int I, int K, double* __restrict__ A) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)I * I) return;
    const int a = (int)(e / I), b = (int)(e % I);
    double s = 0.0;
    for (int c = 0; c < K; ++c) s += yld(Y, (int64_t)a * K + c) * yld(Y, (int64_t)b * K + c);
    A[e] = s;
}

// Y Y^T (I x I, FP64) for the fat rule, one wave per entry of the upper triangle: workgroup (x, y)
// takes row a = y and columns b = 4x + w >= a; lanes read consecutive columns of rows a and b
// (coalesced), the 64 partial sums are added by butterflies, and both A[a][b] and A[b][a] are
// written.
template <typename YT>
__global__ __launch_bounds__(256) void k_syrk_waves(const YT* __restrict__ Y, int I, int K, double* __restrict__ A) {
    const int lane = threadIdx.x & 63;
    const int a = blockIdx.y;
    const int b = 4 * blockIdx.x + (threadIdx.x >> 6);
    if (b < a || b >= I) return;
    const YT* ya = Y + (int64_t)a * K;
    const YT* yb = Y + (int64_t)b * K;
    double s = 0.0;
    for (int c = lane; c < K; c += 64) s += (double)ya[c] * (double)yb[c];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) {
        A[(int64_t)a * I + b] = s;
        A[(int64_t)b * I + a] = s;
    }
}

__device__ inline double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
    return s;
}

// Column sums  out(c) = sum_{i0 <= i < m} f(i, c)  for c in [c0, n), by one workgroup: lane l of
// every wave takes column c0 + 64 b + l of column block b (row-major A: coalesced rows), wave w
// the rows i0 + w, i0 + w + nw, ...; the per-wave partials are added in wave order.
// emit(c, s, valid) runs on the 64 lanes of wave 0 for every block (valid: c < n).
template <typename F, typename E>
__device__ __attribute__((always_inline)) inline void column_sums(int64_t i0, int64_t m, int c0, int n, double* part, F f, E emit) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = (int)(blockDim.x >> 6);
    for (int cb = c0; cb < n; cb += 64) {
        const int c = cb + lane;
        double sacc = 0.0;
        if (c < n)
            for (int64_t i = i0 + wv; i < m; i += nw) sacc += f(i, c);
        part[wv * 64 + lane] = sacc;
        __syncthreads();
        if (tid < 64) {
            double t = 0.0;
            for (int k = 0; k < nw; ++k) t += part[k * 64 + lane];
            emit(c, t, c < n);
        }
        __syncthreads();
    }
}

// Eager Householder QRP on A (m x n, FP64, in place), R steps, by one workgroup (any size up to
// 1024 threads), then Q[:, :R] = H_0 ... H_{R-1} [I; 0] into U (m x R) and the low-precision copy.
// f(i, c) for the entries e = tid, tid + nt, ... of a rows x cols block in row-major order, the
// (row, column) pair stepped incrementally after one division per thread
template <typename F>
__device__ __attribute__((always_inline)) inline void for_block(int64_t rows, int64_t cols, F f) {
    const int nt = (int)blockDim.x;
    if (rows <= 0 || cols <= 0) return;
    int64_t r = threadIdx.x / cols, c = threadIdx.x % cols;
    const int64_t dr = nt / cols, dc = nt % cols;
    for (; r < rows; r += dr, c += dc) {
        if (c >= cols) {
            c -= cols;
            ++r;
            if (r >= rows) break;
        }
        f(r, c);
    }
}

template <typename YT, typename LT>
__device__ __attribute__((always_inline)) void house_qrp_body(const YT* __restrict__ src, double* __restrict__ A, int64_t m, int n, int R,
                               double* __restrict__ V, double* __restrict__ w,
                               double* __restrict__ beta_s, int32_t* __restrict__ perm,
                               double* __restrict__ U, LT* __restrict__ Ulp, int ldlp,
                               int32_t* __restrict__ piv_out, double* __restrict__ gaps) {
    __shared__ double red[16];
    __shared__ double part[16 * 64];
    __shared__ double bestv, secondv;
    __shared__ int pbest;
    const int tid = threadIdx.x, nt = blockDim.x;
    if (src)
        for (int64_t e = tid; e < m * n; e += nt) A[e] = yld(src, e);
    for (int c = tid; c < n; c += nt) perm[c] = c;
    __syncthreads();
    for (int j = 0; j < R; ++j) {
        // trailing norms, exact recompute; first maximum (columns are met in ascending order)
        if (tid == 0) { bestv = -1.0; secondv = -1.0; pbest = n; }
        __syncthreads();
        column_sums(j, m, j, n, part, [&](int64_t i, int c) { const double x = A[i * n + c]; return x * x; },
                    [&](int c, double v, bool valid) {
                        // lanes of one block in order: wave-level first maximum, then against the best so far
                        double bv = valid ? v : -1.0;
                        int bp = valid ? c : n;
                        for (int o = 1; o < 64; o <<= 1) {
                            const double v2 = __shfl_xor(bv, o);
                            const int p2 = __shfl_xor(bp, o);
                            if (v2 > bv || (v2 == bv && p2 < bp)) { bv = v2; bp = p2; }
                        }
                        // the block's runner-up (the pivot gap)
                        double b2 = (valid && c != bp) ? v : -1.0;
                        for (int o = 1; o < 64; o <<= 1) b2 = fmax(b2, __shfl_xor(b2, o));
                        if ((threadIdx.x & 63) == 0) {
                            if (bv > bestv) { secondv = fmax(bestv, b2); bestv = bv; pbest = bp; }
                            else secondv = fmax(secondv, bv);
                        }
                    });
        if (tid == 0) {
            if (gaps)
                gaps[j] = (secondv < 0.0) ? 1.0 : (bestv > 0.0 ? (bestv - secondv) / bestv : 0.0);
            if (pbest >= n) pbest = j;   // no comparable norm (NaN): keep the column in place
            const int p0 = pbest;
            int t = perm[j]; perm[j] = perm[p0]; perm[p0] = t;
        }
        __syncthreads();
        const int p = pbest;
        if (p != j)
            for (int64_t i = tid; i < m; i += nt) {
                double t = A[i * n + j]; A[i * n + j] = A[i * n + p]; A[i * n + p] = t;
            }
        __syncthreads();
        double part1 = 0.0;
        for (int64_t i = j + tid; i < m; i += nt) part1 += A[i * n + j] * A[i * n + j];
        const double alpha = sqrt(block_sum(part1, red));
        if (alpha == 0.0) {
            if (tid == 0) beta_s[j] = 0.0;
            for (int64_t i = tid; i < m; i += nt) V[i * R + j] = 0.0;
            __syncthreads();
            continue;
        }
        const double x0 = A[(int64_t)j * n + j];
        part1 = 0.0;
        for (int64_t i = tid; i < m; i += nt) {
            double v = 0.0;
            if (i >= j) {
                v = A[i * n + j];
                if (i == j) v += (x0 >= 0.0 ? 1.0 : -1.0) * alpha;
            }
            V[i * R + j] = v;
            part1 += v * v;
        }
        const double vv = block_sum(part1, red);
        const double beta = 2.0 / vv;
        if (tid == 0) beta_s[j] = beta;
        __syncthreads();
        column_sums(j, m, j, n, part, [&](int64_t i, int c) { return V[i * R + j] * A[i * n + c]; },
                    [&](int c, double v, bool valid) { if (valid) w[c] = beta * v; });
        for_block(m - j, n - j, [&](int64_t r, int64_t cc) {
            const int64_t i = j + r;
            const int c = j + (int)cc;
            A[i * n + c] -= V[i * R + j] * w[c];
        });
        __syncthreads();
    }
    // Q = H_0 ... H_{R-1} [I; 0]
    for_block(m, R, [&](int64_t i, int64_t c) { U[i * R + c] = (i == c) ? 1.0 : 0.0; });
    __syncthreads();
    for (int j = R - 1; j >= 0; --j) {
        const double beta = beta_s[j];
        if (beta == 0.0) continue;
        column_sums(j, m, 0, R, part, [&](int64_t i, int c) { return V[i * R + j] * U[i * R + c]; },
                    [&](int c, double v, bool valid) { if (valid) w[c] = beta * v; });
        for_block(m - j, R, [&](int64_t r, int64_t c) {
            const int64_t i = j + r;
            U[i * R + c] -= V[i * R + j] * w[c];
        });
        __syncthreads();
    }
    for_block(m, ldlp, [&](int64_t i, int64_t c) {
        const int64_t e = i * ldlp + c;
        const double u = (c < R) ? U[i * R + c] : 0.0;
        if constexpr (sizeof(LT) == 8) Ulp[e] = u;
        else if constexpr (sizeof(LT) == 4) Ulp[e] = (float)u;
        else Ulp[e] = f32_to_bf16((float)u);
    });
    if (piv_out && tid < R) piv_out[tid] = perm[tid];
}

template <typename YT, typename LT>
__global__ __launch_bounds__(1024) void k_house_qrp(const YT* __restrict__ src, double* __restrict__ A, int64_t m, int n, int R,
                                                    double* __restrict__ V, double* __restrict__ w,
                                                    double* __restrict__ beta_s, int32_t* __restrict__ perm,
                                                    double* __restrict__ U, LT* __restrict__ Ulp, int ldlp,
                                                    int32_t* __restrict__ piv_out, double* __restrict__ gaps) {
    house_qrp_body<YT, LT>(src, A, m, n, R, V, w, beta_s, perm, U, Ulp, ldlp, piv_out, gaps);
}

// The same with every working array in LDS (dynamic shared memory, at most kHouseLdsBytes): the
// matrix (m n doubles, from Y = src or, for the fat rule, the Y Y^T already formed in A), the
// reflectors V (m R), w, the betas and the Q being formed (m R), which is copied to U at the end
constexpr size_t kHouseLdsBytes = 120 * 1024;

inline size_t house_lds_bytes(int64_t m, int n, int R) {
    return (size_t)(m * n + 2 * m * R + std::max(n, R) + R) * sizeof(double);
}

template <typename YT, typename LT>
__global__ __launch_bounds__(1024) void k_house_qrp_lds(const YT* __restrict__ src, const double* __restrict__ A,
                                                        int64_t m, int n, int R, int32_t* __restrict__ perm,
                                                        double* __restrict__ U, LT* __restrict__ Ulp, int ldlp,
                                                        int32_t* __restrict__ piv_out, double* __restrict__ gaps) {
    extern __shared__ double house_lds[];
    double* Al = house_lds;
    double* Vl = Al + m * n;
    double* wl = Vl + m * R;
    double* bl = wl + max(n, R);
    double* Ul = bl + R;
    for (int64_t e = threadIdx.x; e < m * n; e += blockDim.x) Al[e] = src ? yld(src, e) : A[e];
    __syncthreads();
    house_qrp_body<YT, LT>(nullptr, Al, m, n, R, Vl, wl, bl, perm, Ul, Ulp, ldlp, piv_out, gaps);
    __syncthreads();
    for (int64_t e = threadIdx.x; e < m * R; e += blockDim.x) U[e] = Ul[e];
}

// The same Householder QRP spread over the whole grid (cooperative launch, grid barriers between
// phases), for matrices too large for one workgroup to stream quickly.  Block b owns rows
// [b slab, (b+1) slab).  Per step j, two barriers:
//   1. each block: partial squared norms of columns j..n-1 over its rows >= j;      barrier
//   2. every block alike: the column totals (blocks added in order), first maximum and runner-up,
//      x0 = A[j][p] from a copy of row j that its owner made before the step; block 0 records the
//      swap in perm and the gap;
//   3. each block: swap columns j and p in its rows, v = its part of x + sgn(x0) alpha e_j, with
//      ||v||^2 = 2 alpha^2 + 2 |x0| alpha; partial v^T A over columns j..n-1;          barrier
//   4. every block alike: w = beta v^T A (totals as in 2), then A -= v w^T on its rows; the owner
//      of row j + 1 copies it.
// The two partial sets use separate buffers (a block can be writing one while another still reads
// the other).  Q = H_0 ... H_{R-1} [I; 0] in compact WY form after one more barrier, then the
// copies.  Every block takes every barrier (all loop bounds and branch conditions come from the
// same totals, added in the same order on each block), and with a flag the whole grid returns at
// once when it is clear.
namespace cg = cooperative_groups;

template <typename YT, typename LT>
struct HouseGridArgs {
    const YT* src;              // Y to copy into A, or null (A already filled)
    double* A;                  // m x n, row-major, in place
    int64_t m;
    int n, R;
    double* V;                  // m x R reflectors
    double* beta_s;             // R
    int32_t* perm;              // n
    double* U;                  // m x R
    LT* Ulp;
    int ldlp;
    int32_t* piv_out;           // R, or null
    double* gaps;               // R, or null
    const int32_t* flag;        // run only when *flag != 0, or null (always run)
    double* part;               // 2 x gridDim.x x max(n, R^2) partials (norms, v^T A)
    double* ctl;                // n: a copy of the row of A at the current step
    int64_t slab;               // rows per block
};

constexpr int kHouseGridT = 1024;

// out[c] for c in [c0, n): sum over the block's rows i in [lo, hi) of f(i, c).  The columns are
// taken W = min(1024, n - c0 rounded up to 64) at a time, thread t on column t % W and row slice
// t / W; each thread keeps four partial sums (rows taken in turn) so that four loads are in flight,
// added as (s0 + s1) + (s2 + s3); the slices are added in order through LDS.
template <typename F>
__device__ inline void slab_column_sums(int64_t lo, int64_t hi, int c0, int n, double* red, double* out, F f) {
    const int tid = threadIdx.x;
    for (int cb = c0; cb < n; cb += kHouseGridT) {
        const int W = min(kHouseGridT, (n - cb + 63) / 64 * 64);
        const int S = kHouseGridT / W;          // row slices (threads past S * W idle)
        const int col = tid % W, sl = tid / W;
        const int c = cb + col;
        double acc = 0.0;
        if (sl < S && c < n) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            int64_t i = lo + sl;
            const int64_t st = S;
            for (; i + 3 * st < hi; i += 4 * st) {
                s0 += f(i, c);
                s1 += f(i + st, c);
                s2 += f(i + 2 * st, c);
                s3 += f(i + 3 * st, c);
            }
            for (; i < hi; i += st) s0 += f(i, c);
            acc = (s0 + s1) + (s2 + s3);
        }
        red[tid] = acc;
        __syncthreads();
        if (sl == 0 && c < n) {
            double t = 0.0;
            for (int k = 0; k < S; ++k) t += red[k * W + col];
            out[c] = t;
        }
        __syncthreads();
    }
}

template <typename YT, typename LT>
__global__ __launch_bounds__(kHouseGridT) void k_house_qrp_grid(HouseGridArgs<YT, LT> a) {
    if (a.flag && *a.flag == 0) return;   // every block reads the same flag: all return together
    cg::grid_group grid = cg::this_grid();
    __shared__ double red[kHouseGridT];
    __shared__ double bv_s[kHouseGridT / 64], b2_s[kHouseGridT / 64];
    __shared__ int bp_s[kHouseGridT / 64];
    __shared__ double s_piv[3];             // pivot, its squared norm, x0
    __shared__ double s_T[kGramMaxR][kGramMaxR], s_M[kGramMaxR][kGramMaxR], s_G[kGramMaxR * kGramMaxR];
    extern __shared__ double tot[];   // this block's copy of the column totals (n values)
    const int tid = threadIdx.x, nb = gridDim.x, b = blockIdx.x;
    const int n = a.n, R = a.R;
    const int64_t m = a.m;
    const int64_t r0 = min(m, (int64_t)b * a.slab), r1 = min(m, r0 + a.slab);
    const int pw = max(n, R * R);
    double* mypart = a.part + (int64_t)b * pw;   // the Gram of V (after the steps)
    double* rowbuf = a.ctl;                 // row j of A as it stands before step j (n values)
    if (a.src)
        for (int64_t e = r0 * n + tid; e < r1 * n; e += kHouseGridT) a.A[e] = yld(a.src, e);
    if (b == 0)
        for (int c = tid; c < n; c += kHouseGridT) a.perm[c] = c;
    __syncthreads();
    if (r0 <= 0 && 0 < r1)
        for (int c = tid; c < n; c += kHouseGridT) rowbuf[c] = a.A[c];
    // column totals of a partials buffer, computed by every block alike (fixed order): thread t
    // takes columns c0 + t, c0 + t + 256, ...
    auto all_totals = [&](const double* part, int c0, double scale) __attribute__((always_inline)) {
        for (int c = c0 + tid; c < n; c += kHouseGridT) {
            double t = 0.0;
            for (int k = 0; k < nb; ++k) t += part[(int64_t)k * pw + c];
            tot[c] = scale * t;
        }
        __syncthreads();
    };
    double* const partA = a.part;                       // column norms
    double* const partB = a.part + (int64_t)nb * pw;    // v^T A
    for (int j = 0; j < R; ++j) {
        // 1. partial squared norms (this block's rows >= j)
        slab_column_sums(max(r0, (int64_t)j), r1, j, n, red, partA + (int64_t)b * pw, [&](int64_t i, int c) {
            const double x = a.A[i * n + c];
            return x * x;
        });
        grid.sync();
        // 2. every block: the column totals, the pivot (first maximum) and runner-up, the same on
        // each; x0 from the copy of row j
        all_totals(partA, j, 1.0);
        {
            double bv = -1.0, b2 = -1.0;
            int bp = n;
            for (int c = j + tid; c < n; c += kHouseGridT) {   // ascending: first maximum kept
                const double t = tot[c];
                if (t > bv) { b2 = fmax(b2, bv); bv = t; bp = c; }
                else b2 = fmax(b2, t);
            }
            for (int o = 1; o < 64; o <<= 1) {
                const double v2 = __shfl_xor(bv, o), s2 = __shfl_xor(b2, o);
                const int p2 = __shfl_xor(bp, o);
                const bool take = v2 > bv || (v2 == bv && p2 < bp);
                b2 = fmax(fmax(b2, s2), take ? bv : v2);
                if (take) { bv = v2; bp = p2; }
            }
            if ((tid & 63) == 0) { bv_s[tid >> 6] = bv; b2_s[tid >> 6] = b2; bp_s[tid >> 6] = bp; }
            __syncthreads();
            if (tid == 0) {
                double best = bv_s[0], second = b2_s[0];
                int pb = bp_s[0];
                for (int k = 1; k < kHouseGridT / 64; ++k) {
                    const bool take = bv_s[k] > best || (bv_s[k] == best && bp_s[k] < pb);
                    second = fmax(fmax(second, b2_s[k]), take ? best : bv_s[k]);
                    if (take) { best = bv_s[k]; pb = bp_s[k]; }
                }
                if (pb >= n) pb = j;   // no comparable norm (NaN): keep the column in place (alpha NaN)
                if (b == 0) {
                    if (a.gaps) a.gaps[j] = (second < 0.0) ? 1.0 : (best > 0.0 ? (best - second) / best : 0.0);
                    const int t = a.perm[j]; a.perm[j] = a.perm[pb]; a.perm[pb] = t;
                }
                s_piv[0] = (double)pb;
                s_piv[1] = best;
                s_piv[2] = rowbuf[pb];
            }
            __syncthreads();
        }
        // 3. swap, reflector, partial v^T A
        const int p = (int)s_piv[0];
        const double alpha = sqrt(s_piv[1]), x0 = s_piv[2];
        if (p != j)
            for (int64_t i = r0 + tid; i < r1; i += kHouseGridT) {
                const double t = a.A[i * n + j];
                a.A[i * n + j] = a.A[i * n + p];
                a.A[i * n + p] = t;
            }
        if (alpha == 0.0) {   // the same on every block
            if (b == 0 && tid == 0) a.beta_s[j] = 0.0;
            for (int64_t i = r0 + tid; i < r1; i += kHouseGridT) a.V[i * R + j] = 0.0;
            grid.sync();   // every block has read this step's copy of row j
            if (r0 <= j + 1 && j + 1 < r1)
                for (int c = tid; c < n; c += kHouseGridT) rowbuf[c] = a.A[(int64_t)(j + 1) * n + c];
            continue;
        }
        const double sg = (x0 >= 0.0 ? 1.0 : -1.0);
        for (int64_t i = r0 + tid; i < r1; i += kHouseGridT) {
            double v = 0.0;
            if (i >= j) {
                v = a.A[i * n + j];
                if (i == j) v += sg * alpha;
            }
            a.V[i * R + j] = v;
        }
        const double beta = 2.0 / (2.0 * alpha * alpha + 2.0 * fabs(x0) * alpha);
        if (b == 0 && tid == 0) a.beta_s[j] = beta;
        __syncthreads();
        slab_column_sums(max(r0, (int64_t)j), r1, j, n, red, partB + (int64_t)b * pw,
                         [&](int64_t i, int c) { return a.V[i * R + j] * a.A[i * n + c]; });
        grid.sync();
        // 4. every block: w = beta v^T A, then A -= v w^T on its rows >= j; the owner of row j + 1
        // copies it for step j + 1
        all_totals(partB, j, beta);
        for (int64_t i = max(r0, (int64_t)j); i < r1; ++i) {
            const double vi = a.V[i * R + j];
            for (int c = j + tid; c < n; c += kHouseGridT) a.A[i * n + c] -= vi * tot[c];
        }
        __syncthreads();   // the next step's column sums read these rows from other threads
        if (r0 <= j + 1 && j + 1 < r1)
            for (int c = tid; c < n; c += kHouseGridT) rowbuf[c] = a.A[(int64_t)(j + 1) * n + c];
    }
    // Q = H_0 ... H_{R-1} [I; 0] = [I; 0] - V T V_top^T (compact WY form: T upper triangular with
    // T_jj = beta_j, T[0:j, j] = -beta_j T[0:j, 0:j] (V[:, 0:j]^T v_j); V_top = the first R rows)
    slab_column_sums(r0, r1, 0, R * R, red, mypart,
                     [&](int64_t i, int c) { return a.V[i * R + c / R] * a.V[i * R + c % R]; });
    grid.sync();
    // every block: the Gram of V (blocks added in order), T and M = T V_top^T, the same on each
    for (int e = tid; e < R * R; e += kHouseGridT) {
        double g = 0.0;
        for (int k = 0; k < nb; ++k) g += a.part[(int64_t)k * pw + e];
        s_G[e] = g;
    }
    for (int e = tid; e < kGramMaxR * kGramMaxR; e += kHouseGridT) s_T[e / kGramMaxR][e % kGramMaxR] = 0.0;
    __syncthreads();
    for (int j = 0; j < R; ++j) {   // column j of T from columns 0..j-1 (thread i: entry i)
        const double bj = a.beta_s[j];
        if (tid < j) {
            double t = 0.0;
            for (int k = tid; k < j; ++k) t += s_T[tid][k] * s_G[k * R + j];
            s_T[tid][j] = -bj * t;
        } else if (tid == j) {
            s_T[j][j] = bj;
        }
        __syncthreads();
    }
    for (int e = tid; e < R * R; e += kHouseGridT) {
        const int r = e / R, c = e % R;
        double t = 0.0;
        for (int k = r; k < R; ++k) t += s_T[r][k] * a.V[(int64_t)c * R + k];   // V_top[c][k]
        s_M[r][c] = t;
    }
    __syncthreads();
    for (int64_t e = r0 * R + tid; e < r1 * R; e += kHouseGridT) {
        const int64_t i = e / R;
        const int c = (int)(e % R);
        double u = (i == c) ? 1.0 : 0.0;
        for (int k = 0; k < R; ++k) u -= a.V[i * R + k] * s_M[k][c];
        a.U[e] = u;
    }
    __syncthreads();
    for (int64_t e = r0 * a.ldlp + tid; e < r1 * a.ldlp; e += kHouseGridT) {
        const int64_t i = e / a.ldlp;
        const int c = (int)(e % a.ldlp);
        const double u = (c < R) ? a.U[i * R + c] : 0.0;
        if constexpr (sizeof(LT) == 8) a.Ulp[e] = u;
        else if constexpr (sizeof(LT) == 4) a.Ulp[e] = (float)u;
        else a.Ulp[e] = f32_to_bf16((float)u);
    }
    if (b == 0 && a.piv_out && tid < R) a.piv_out[tid] = a.perm[tid];
}

// U = Y[:, piv] M and its low-precision copy; ldlp consecutive threads share a row, one output
// column each (columns R..ldlp-1 of the copy are zeroed).
// After a breakdown (device flag set) workgroup 0 runs the Householder QRP on Y instead (small Y)
// or the grid-wide kernel launched after this one does (large Y), and the others exit.
template <typename YT, typename LT>
__global__ __launch_bounds__(1024) void k_form_u(const YT* __restrict__ Y, int64_t m, int n, int R,
                                                const int32_t* __restrict__ pivw,
                                                const double* __restrict__ M,
                                                const int32_t* __restrict__ flag,
                                                double* __restrict__ U, LT* __restrict__ Ulp, int ldlp,
                                                double* __restrict__ A, double* __restrict__ V,
                                                double* __restrict__ wv, double* __restrict__ beta_s,
                                                int32_t* __restrict__ perm, int32_t* __restrict__ piv_out,
                                                double* __restrict__ gaps, int fallback_here) {
    if (*flag) {   // fallback_here = 0: the grid-wide kernel, launched next, takes it
        if (fallback_here && blockIdx.x == 0)
            house_qrp_body<YT, LT>(Y, A, m, n, R, V, wv, beta_s, perm, U, Ulp, ldlp, piv_out, gaps);
        return;
    }
    __shared__ double sM[32 * 32];
    __shared__ int sp[32];
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) sM[e] = M[e];
    if (threadIdx.x < R) sp[threadIdx.x] = pivw[threadIdx.x];
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = g / ldlp;
    const int c = (int)(g % ldlp);
    if (row >= m) return;
    double u = 0.0;
    if (c < R)
        for (int j = 0; j < R; ++j) u += yld(Y, row * n + sp[j]) * sM[j * R + c];
    if (c < R) U[row * R + c] = u;
    if constexpr (sizeof(LT) == 8) Ulp[row * ldlp + c] = u;
    else if constexpr (sizeof(LT) == 4) Ulp[row * ldlp + c] = (float)u;
    else Ulp[row * ldlp + c] = f32_to_bf16((float)u);
}

struct QrpPlan {
    int route;
    int64_t m;       // rows of the QRP input
    int n;           // columns of the QRP input
    int R;
    int nb;          // 64-column blocks (route 0)
    int nsplit;      // row slabs of the Gram (route 0)
    int64_t slab;
    int nblk2;       // blocks of the Q1 Gram (route 0)
    int64_t rows2;
    // offsets into the FP64 workspace (in doubles)
    int64_t o_part, o_C, o_L, o_R11, o_Rinv, o_part2, o_G2, o_M, o_A, o_V, o_w, o_beta;
    bool grid;       // the Householder QRP (route 1/2, route-0 fallback) runs grid-wide
    int64_t o_hpart, o_hctl;
    int64_t total;
};

// Householder inputs of at least this many entries take the grid-wide kernel, with at least
// TK_HOUSE_ROWS rows per block
constexpr int64_t kHouseGridMin = 1 << 18;
constexpr int kHouseGridMaxB = 64;
#ifndef TK_HOUSE_ROWS
#define TK_HOUSE_ROWS 32
#endif

QrpPlan plan(const tk_ctx* ctx, int mode) {
    QrpPlan p{};
    const int64_t I = ctx->dims[mode];
    const int64_t K = ctx->mode[mode].K;
    const int R = ctx->ranks[mode];
    const bool fat = K > I;
    p.R = R;
    if (fat && !(ctx->flags & TK_FLAG_NO_FAT_RULE)) {
        p.route = 2;
        p.m = I;
        p.n = (int)I;
    } else {
        p.m = I;
        p.n = (int)K;
        p.route = (fat || R > kGramMaxR || K > 1024) ? 1 : 0;
    }
    int64_t off = 0;
    if (p.route == 0) {
        p.nb = (p.n + 63) / 64;
        const int64_t nn = (int64_t)p.n * p.n;
        int64_t cap = std::max<int64_t>(1, (int64_t)(32u << 20) / 8 / nn);  // <= 32 MB of partials
        const int64_t pairs = (int64_t)p.nb * (p.nb + 1) / 2;
        // one round of workgroups: two per compute unit (each stages 66 KB in LDS)
        const int64_t want = std::max<int64_t>(1, 2 * (int64_t)std::max(ctx->ncu, 1) / pairs);
        p.nsplit = (int)std::max<int64_t>(1, std::min<int64_t>({(p.m + 31) / 32, want, cap}));
        p.slab = ((p.m + p.nsplit - 1) / p.nsplit + 31) / 32 * 32;
        p.nsplit = (int)((p.m + p.slab - 1) / p.slab);
        p.rows2 = 64;
        p.nblk2 = (int)((p.m + 63) / 64);
        p.o_part = off; off += (int64_t)p.nsplit * nn;
        p.o_C = off; off += nn;
        p.o_L = off; off += (int64_t)p.n * R;
        p.o_R11 = off; off += (int64_t)R * R;
        p.o_Rinv = off; off += (int64_t)R * R;
        p.o_part2 = off; off += (int64_t)p.nblk2 * R * R;
        p.o_G2 = off; off += (int64_t)R * R;
        p.o_M = off; off += (int64_t)R * R;
    }
    // Householder workspace (route 1/2, and the route-0 fallback on Y)
    const int64_t hm = (p.route == 0) ? I : p.m;
    const int64_t hn = (p.route == 0) ? K : p.n;
    p.o_A = off; off += hm * hn;
    p.o_V = off; off += hm * R;
    p.o_w = off; off += std::max<int64_t>(hn, R);
    p.o_beta = off; off += R;
    p.grid = hm * hn >= kHouseGridMin && R <= kGramMaxR;
    if (p.grid) {
        p.o_hpart = off; off += 2 * (int64_t)kHouseGridMaxB * std::max<int64_t>(hn, (int64_t)R * R);
        p.o_hctl = off; off += hn;
    }
    p.total = off;
    return p;
}

// The grid-wide Householder QRP on (Y or A already filled); gated by flag when not null
template <typename YT, typename LT>
int launch_house_grid(const tk_ctx* ctx, const QrpPlan& p, const YT* src, double* W, int32_t* perm, double* U,
                      LT* Ulp, int ldlp, int32_t* piv, double* gaps, const int32_t* flag, hipStream_t s) {
    auto kern = k_house_qrp_grid<YT, LT>;
    const size_t shmem = (size_t)p.n * sizeof(double);   // the block's column totals
    static int occ = 0;   // blocks per CU at the largest totals array: asked once
    if (occ == 0)
        TK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)kern, kHouseGridT,
                                                            (size_t)TK_MAX_KCOLS * sizeof(double)));
    const int64_t want = std::min<int64_t>({(int64_t)kHouseGridMaxB, (int64_t)std::max(ctx->ncu, 1) * std::max(occ, 1),
                                            (p.m + TK_HOUSE_ROWS - 1) / TK_HOUSE_ROWS});
    const int nb = (int)std::max<int64_t>(1, want);
    HouseGridArgs<YT, LT> a{};
    a.src = src;
    a.A = W + p.o_A;
    a.m = p.m;
    a.n = p.n;
    a.R = p.R;
    a.V = W + p.o_V;
    a.beta_s = W + p.o_beta;
    a.perm = perm;
    a.U = U;
    a.Ulp = Ulp;
    a.ldlp = ldlp;
    a.piv_out = piv;
    a.gaps = gaps;
    a.flag = flag;
    a.part = W + p.o_hpart;
    a.ctl = W + p.o_hctl;
    a.slab = (p.m + nb - 1) / nb;
    void* args[] = {&a};
    TK_HIP(hipLaunchCooperativeKernel((const void*)kern, dim3((unsigned)nb), dim3(kHouseGridT), args, shmem, s));
    return TK_OK;
}

template <typename YT, typename LT>
int run_typed(tk_ctx* ctx, int mode, const YT* Y, double* U, int32_t* piv, hipStream_t s) {
    const QrpPlan p = plan(ctx, mode);
    double* W = ctx->ws.qrp;
    int32_t* flag = ctx->ws.qrp_int;            // [0] flag
    int32_t* pivw = ctx->ws.qrp_int + 16;       // [16 .. 16+R)
    int32_t* perm = ctx->ws.qrp_int + 64;       // Householder permutation, n entries
    LT* Ulp = (LT*)ctx->Ulp[mode];
    const int ldlp = ctx->ldU[mode];
    const int64_t I = ctx->dims[mode];
    const int64_t K = ctx->mode[mode].K;
    if (p.route == 0) {
        launch_gram_partial<YT>(Y, p.m, p.n, p.nb, p.nsplit, p.slab, W + p.o_part, s);
        TK_LAUNCH_CHECK("k_gram_partial");
        k_gram_reduce<<<cdiv((int64_t)p.n * p.n, 64), 256, 0, s>>>(W + p.o_part, p.nsplit, p.n, W + p.o_C);
        TK_LAUNCH_CHECK("k_gram_reduce");
        const size_t lsz = (size_t)p.n * p.R * sizeof(double);
        const unsigned nthr = (unsigned)std::max(64, (p.n + 63) / 64 * 64);
        double* gaps = ctx->qrp_gaps + (size_t)mode * kGramMaxR;
        if (p.R <= 16 && (size_t)p.n * 16 * sizeof(double) <= 64 * 1024)
            k_pivchol_cols<16><<<1, nthr, (size_t)p.n * 16 * sizeof(double), s>>>(W + p.o_C, p.n, p.R, W + p.o_R11,
                                                                              W + p.o_Rinv, pivw, flag, gaps);
        else if (p.R <= 32 && (size_t)p.n * 32 * sizeof(double) <= 64 * 1024)
            k_pivchol_cols<32><<<1, nthr, (size_t)p.n * 32 * sizeof(double), s>>>(W + p.o_C, p.n, p.R, W + p.o_R11,
                                                                              W + p.o_Rinv, pivw, flag, gaps);
        else {
            // this route does not record pivot gaps
            if (int st = fill_f64(gaps, kGramMaxR, NAN, s)) return st;
            if (lsz <= 64 * 1024)
                k_pivchol<true><<<1, nthr, lsz, s>>>(W + p.o_C, p.n, p.R, W + p.o_L, W + p.o_R11, W + p.o_Rinv, pivw, flag);
            else
                k_pivchol<false><<<1, nthr, 0, s>>>(W + p.o_C, p.n, p.R, W + p.o_L, W + p.o_R11, W + p.o_Rinv, pivw, flag);
        }
        TK_LAUNCH_CHECK("k_pivchol");
        k_q1_gram<YT><<<(unsigned)p.nblk2, 256, 0, s>>>(Y, p.m, p.n, p.R, pivw, W + p.o_Rinv, W + p.o_part2);
        TK_LAUNCH_CHECK("k_q1_gram");
        k_sum_partials<<<(unsigned)(p.R * p.R), 256, 0, s>>>(W + p.o_part2, p.nblk2, p.R * p.R, nullptr, W + p.o_G2);
        TK_LAUNCH_CHECK("k_sum_partials");
#define TK_FINISH(RM, EX) \
    k_qrp_finish<YT, RM, EX><<<1, 64, 0, s>>>(Y, p.n, p.R, pivw, W + p.o_Rinv, W + p.o_G2, flag, W + p.o_M, piv)
        if (p.R == 16) TK_FINISH(16, true);
        else if (p.R == 8) TK_FINISH(8, true);
        else if (p.R < 16) TK_FINISH(16, false);
        else if (p.R == 32) TK_FINISH(32, true);
        else TK_FINISH(32, false);
#undef TK_FINISH
        TK_LAUNCH_CHECK("k_qrp_finish");
        // U = Y[:, piv] M, or (flag set) the Householder fallback on Y in workgroup 0
        k_form_u<YT, LT><<<cdiv(p.m * ldlp, 1024), 1024, 0, s>>>(Y, p.m, p.n, p.R, pivw, W + p.o_M, flag, U, Ulp, ldlp,
                                                             W + p.o_A, W + p.o_V, W + p.o_w, W + p.o_beta, perm, piv,
                                                             gaps, p.grid ? 0 : 1);
        TK_LAUNCH_CHECK("k_form_u");
        if (p.grid) return launch_house_grid<YT, LT>(ctx, p, Y, W, perm, U, Ulp, ldlp, piv, gaps, flag, s);
        return TK_OK;
    }
    // Householder routes: gaps for the first kGramMaxR steps
    double* hgaps = ctx->qrp_gaps + (size_t)mode * kGramMaxR;
    if (p.R > kGramMaxR) {
        if (int st = fill_f64(hgaps, kGramMaxR, NAN, s)) return st;
        hgaps = nullptr;
    }
    if (p.route == 2) {
        if (I <= 65535) {
            k_syrk_waves<YT><<<dim3(cdiv(I, 4), (unsigned)I), 256, 0, s>>>(Y, (int)I, (int)K, W + p.o_A);
            TK_LAUNCH_CHECK("k_syrk_waves");
        } else {
            k_syrk_rows<YT><<<cdiv(I * I, 256), 256, 0, s>>>(Y, (int)I, (int)K, W + p.o_A);
            TK_LAUNCH_CHECK("k_syrk_rows");
        }
    }
    if (p.grid)
        return launch_house_grid<YT, LT>(ctx, p, p.route == 2 ? nullptr : Y, W, perm, U, Ulp, ldlp, piv, hgaps, nullptr, s);
    const size_t lbytes = house_lds_bytes(p.m, p.n, p.R);
    static int lds_ok = -1;   // whether the LDS kernel may take kHouseLdsBytes of dynamic LDS: asked once
    if (lds_ok < 0)
        lds_ok = hipFuncSetAttribute((const void*)k_house_qrp_lds<YT, LT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kHouseLdsBytes) == hipSuccess;
    if (lds_ok && lbytes <= kHouseLdsBytes) {
        k_house_qrp_lds<YT, LT><<<1, 1024, lbytes, s>>>(p.route == 2 ? nullptr : Y, W + p.o_A, p.m, p.n, p.R, perm, U,
                                                        Ulp, ldlp, piv, hgaps);
        TK_LAUNCH_CHECK("k_house_qrp_lds");
        return TK_OK;
    }
    k_house_qrp<YT, LT><<<1, 1024, 0, s>>>(p.route == 2 ? nullptr : Y, W + p.o_A, p.m, p.n, p.R, W + p.o_V, W + p.o_w,
                                           W + p.o_beta, perm, U, Ulp, ldlp, piv, hgaps);
    TK_LAUNCH_CHECK("k_house_qrp");
    return TK_OK;
}

}  // namespace

size_t qrp_workspace_bytes(const tk_ctx* ctx, int mode) { return (size_t)plan(ctx, mode).total * 8; }

int qrp_route(const tk_ctx* ctx, int mode) { return plan(ctx, mode).route; }

// The symmetric FP64 matrix the factor update of this mode works on: Y^T Y (K_n x K_n, the Gram
// kernels) when Y_(n) is tall, Y Y^T (I_n x I_n) when the fat rule applies; full storage in the
// QRP workspace.  Shapes without a Gram route (R_n > 32 or K_n > 1024 on a tall Y) are refused.
template <typename YT>
int gram_typed(tk_ctx* ctx, int mode, const YT* Y, double** A, int* n, hipStream_t s) {
    const QrpPlan p = plan(ctx, mode);
    double* W = ctx->ws.qrp;
    if (p.route == 0) {
        launch_gram_partial<YT>(Y, p.m, p.n, p.nb, p.nsplit, p.slab, W + p.o_part, s);
        TK_LAUNCH_CHECK("k_gram_partial");
        k_gram_reduce<<<cdiv((int64_t)p.n * p.n, 64), 256, 0, s>>>(W + p.o_part, p.nsplit, p.n, W + p.o_C);
        TK_LAUNCH_CHECK("k_gram_reduce");
        *A = W + p.o_C;
        *n = p.n;
        return TK_OK;
    }
    if (p.route == 2) {
        const int64_t I = ctx->dims[mode];
        if (I <= 65535) {
            k_syrk_waves<YT><<<dim3(cdiv(I, 4), (unsigned)I), 256, 0, s>>>(Y, (int)I, (int)ctx->mode[mode].K, W + p.o_A);
            TK_LAUNCH_CHECK("k_syrk_waves");
        } else {
            k_syrk_rows<YT><<<cdiv(I * I, 256), 256, 0, s>>>(Y, (int)I, (int)ctx->mode[mode].K, W + p.o_A);
            TK_LAUNCH_CHECK("k_syrk_rows");
        }
        *A = W + p.o_A;
        *n = (int)I;
        return TK_OK;
    }
    return set_error(TK_ERR_UNSUPPORTED, "mode %d: no Gram route for R_n = %d, K_n = %lld", mode, p.R,
                     (long long)ctx->mode[mode].K);
}

int gram_run(tk_ctx* ctx, int mode, const void* Y, double** A, int* n, hipStream_t s) {
    if (ctx->dtype == TK_F64) return gram_typed<double>(ctx, mode, (const double*)Y, A, n, s);
    return gram_typed<float>(ctx, mode, (const float*)Y, A, n, s);
}

int qrp_run(tk_ctx* ctx, int mode, const void* Y, double* U, int32_t* piv, hipStream_t s) {
    switch (ctx->dtype) {
        case TK_F64: return run_typed<double, double>(ctx, mode, (const double*)Y, U, piv, s);
        case TK_F32: return run_typed<float, float>(ctx, mode, (const float*)Y, U, piv, s);
        default: return run_typed<float, bf16_t>(ctx, mode, (const float*)Y, U, piv, s);
    }
}

}  // namespace tk
