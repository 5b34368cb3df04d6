// Tucker completion: loss and gradients of a sampled-entry Tucker model, built on the adjoint of
// the sparse TTMc (spec addition to the method of Alg. 2).
//
// For observed entries p in Omega with values x_p:
//   xhat_p = sum_r G[r] prod_k U_k(i_k, r_k),   e_p = xhat_p - x_p,   L = sum_p e_p^2 / (2 |Omega|)
//   dL/dU_n   = TTMc_n(E) G_(n)^T / |Omega|        (TTMc_n(E) = E_(n) kron_{k != n} U_k, I_n x K_n)
//   dL/dG_(N) = U_N^T TTMc_N(E) / |Omega|
// where E is the sparse tensor of residuals on the pattern of X.  The residuals are computed once,
// on mode 0's sorted stream: with W_0 = U_0 G_(0) (I_0 x K_0, dense), the model value of an entry
// is the dot product of row i_0 of W_0 with the entry's Kronecker row.  Every other mode gathers
// them into its own stream order through a position map built at the first call (both streams
// sorted by the same lexicographic coordinate key: the r-th entries are the same nonzero).  The
// residual values then replace the tensor values in the ordinary TTMc kernels (the adjoint reuses
// the forward kernels unchanged), and two small dense products give the gradients.  All sums have
// a fixed order: results are deterministic.
#include <hipcub/hipcub.hpp>

#include <type_traits>

#include "internal.h"
#include "atb.h"

namespace tk {

namespace {

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// rowid[q] = compressed row holding padded position q (binary search of the padded pointers)
__global__ void k_rowid(const int32_t* __restrict__ pptr, int64_t S, int64_t P, int32_t* __restrict__ rowid) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P) return;
    int64_t lo = 0, hi = S - 1;   // largest s with pptr[s] <= q
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (pptr[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    rowid[q] = (int32_t)lo;
}

// padded copy (I x ld, zero columns past R) of a factor given in the parameter type
template <typename IT, typename LT>
__global__ void k_factor_copy(const IT* __restrict__ U, int64_t I, int R, int ld, LT* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= I * ld) return;
    const int64_t i = e / ld;
    const int c = (int)(e % ld);
    out[e] = (c < R) ? (LT)U[i * R + c] : (LT)0;
}

struct Unfold {
    int32_t R[kMaxOrder];
    int N;
    int n;
    int64_t K;
    int64_t size;   // prod R
};

// Gn[r_n * K + c] = G[r_0, ..., r_{N-1}] (C order), c = the other modes' indices with the last
// fastest: the mode-n unfolding in the Kronecker column order of the TTMc
template <typename AT>
__global__ void k_unfold(Unfold u, const AT* __restrict__ G, AT* __restrict__ Gn) {
    const int64_t lin = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lin >= u.size) return;
    int64_t rest = lin;
    int digit[kMaxOrder];
    for (int t = u.N - 1; t >= 0; --t) {
        digit[t] = (int)(rest % u.R[t]);
        rest /= u.R[t];
    }
    int64_t c = 0;
    for (int t = 0; t < u.N; ++t)
        if (t != u.n) c = c * u.R[t] + digit[t];
    Gn[(int64_t)digit[u.n] * u.K + c] = G[lin];
}

// W[i][c] = sum_r U[i][r] Gn[r][c]   (r ascending)
template <typename AT>
__global__ void k_w(const AT* __restrict__ U, const AT* __restrict__ Gn, int64_t I, int R, int64_t K,
                    AT* __restrict__ W) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= I * K) return;
    const int64_t i = e / K, c = e % K;
    AT acc = 0;
    for (int r = 0; r < R; ++r) acc += U[i * R + r] * Gn[(int64_t)r * K + c];
    W[e] = acc;
}

// Fused form: W[i][16 ra + rb] = sum_r U[i][r] Gn[r][ra * Rb + rb] for ra < Ra, rb < Rb, zero
// elsewhere (r ascending).  Thread c of a block owns entry c of the 16 x 16 block; a block takes
// kW16Rows rows.  With R = RT known (RT > 0) the block first copies its rows of U into LDS
// (coalesced, one wait) and each thread keeps its column of Gn in registers; the products then
// read U from LDS at one address per wave.  RT = 0 is the plain loop for any R.
constexpr int kW16Rows = 64;

template <int RT>
__global__ __launch_bounds__(256) void k_w16(const float* __restrict__ U, const float* __restrict__ Gn, int64_t I,
                                             int R, int Ra, int Rb, float* __restrict__ W) {
    const int c = threadIdx.x, ra = c >> 4, rb = c & 15;
    const bool live = ra < Ra && rb < Rb;
    const int64_t K = (int64_t)Ra * Rb;
    const float* g = Gn + (live ? ra * Rb + rb : 0);
    const int64_t i0 = (int64_t)blockIdx.x * kW16Rows;
    const int64_t i1 = min(I, i0 + kW16Rows);
    if constexpr (RT > 0) {
        __shared__ float us[kW16Rows * RT];
        const int nflt = (int)(i1 - i0) * RT;
        for (int e = c; e < nflt; e += 256) us[e] = U[i0 * RT + e];
        float gr[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) gr[r] = g[(int64_t)r * K];
        __syncthreads();
        for (int64_t i = i0; i < i1; ++i) {
            const float* ur = us + (i - i0) * RT;
            float t = 0.f;
#pragma unroll
            for (int r = 0; r < RT; ++r) t += ur[r] * gr[r];
            W[i * 256 + c] = live ? t : 0.f;
        }
    } else {
        for (int64_t i = i0; i < i1; ++i) {
            const float* ur = U + i * R;
            float acc = 0.f;
            for (int r = 0; r < R; ++r) acc += ur[r] * g[(int64_t)r * K];
            W[i * 256 + c] = live ? acc : 0.f;
        }
    }
}

struct ResidArgs {
    const int32_t* rowid;
    const int32_t* rows;
    const int32_t* ptr;      // unpadded row pointers
    const int32_t* pptr;     // padded row pointers
    const int32_t* idx;      // [nm1][P]
    int64_t P;
    const void* val;
    const void* F[kMaxOrder - 1];
    int32_t ld[kMaxOrder - 1];
    int32_t R[kMaxOrder - 1];
    int32_t nm1;
    int64_t K;
    const void* W;
    void* e;                 // [P] residuals (pads: 0)
    double* part;            // per-block sum of e^2, or null
};

// One padded entry per thread: e = W(i_n, :) . kron_p - x_p (0 on pads), the Kronecker row walked
// in C order with an odometer that recomputes only the prefix products whose digit changed.
template <typename AT>
__global__ __launch_bounds__(256) void k_residual(ResidArgs a) {
    __shared__ double red[4];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e2 = 0.0;
    if (q < a.P) {
        const int s = a.rowid[q];
        const bool real = (q - a.pptr[s]) < (int64_t)(a.ptr[s + 1] - a.ptr[s]);
        AT ev = 0;
        if (real) {
            const int nm1 = a.nm1;
            const AT* rowp[kMaxOrder - 1];
            int r[kMaxOrder - 1];
            AT pre[kMaxOrder];
            for (int j = 0; j < nm1; ++j) {
                int32_t t = a.idx[(int64_t)j * a.P + q];
                if (j == 0) t &= kIndexMask;
                rowp[j] = (const AT*)a.F[j] + (int64_t)t * a.ld[j];
                r[j] = 0;
            }
            pre[0] = (AT)1;
            for (int j = 0; j < nm1; ++j) pre[j + 1] = pre[j] * rowp[j][0];
            const AT* w = (const AT*)a.W + (int64_t)a.rows[s] * a.K;
            AT xh = 0;
            for (int64_t c = 0; c < a.K; ++c) {
                xh += w[c] * pre[nm1];
                int j = nm1 - 1;
                while (j >= 0) {
                    if (++r[j] < a.R[j]) break;
                    r[j] = 0;
                    --j;
                }
                if (j < 0) break;
                for (int u = j; u < nm1; ++u) pre[u + 1] = pre[u] * rowp[u][r[u]];
            }
            ev = xh - ((const AT*)a.val)[q];
        }
        ((AT*)a.e)[q] = ev;
        e2 = (double)ev * (double)ev;
    }
    if (a.part) {
        for (int o = 32; o > 0; o >>= 1) e2 += __shfl_xor(e2, o);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e2;
        __syncthreads();
        if (threadIdx.x == 0) a.part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
    }
}

// Order 3 with R_a, R_b <= 16: the same residuals with the factor rows read by 16-byte loads and
// the W rows of the (few) compressed rows a workgroup's 256 positions touch staged in LDS; the
// model value of an entry is a^T M b with M = W(i_n, :) as an R_a x R_b matrix (K FMAs).  A
// workgroup spanning more than kResidRows rows reads M from global memory instead.
constexpr int kResidRows = 8;

template <typename AT>
__global__ __launch_bounds__(256) void k_residual3(ResidArgs a) {
    extern __shared__ __align__(16) unsigned char resid_lds[];
    AT* Ms = (AT*)resid_lds;                       // [kResidRows][K]
    __shared__ double red[4];
    const int64_t P = a.P;
    const int64_t b0 = (int64_t)blockIdx.x * 256;
    const int64_t q = b0 + threadIdx.x;
    const int64_t bl = min(P, b0 + 256) - 1;
    const int s_first = a.rowid[b0], s_last = a.rowid[bl];
    const int nr = s_last - s_first + 1;
    const int K = (int)a.K, Ra = a.R[0], Rb = a.R[1];
    const bool staged = nr <= kResidRows;
    if (staged) {
        for (int e = threadIdx.x; e < nr * K; e += 256) {
            const int r = e / K, c = e % K;
            Ms[e] = ((const AT*)a.W)[(int64_t)a.rows[s_first + r] * K + c];
        }
    }
    __syncthreads();
    double e2 = 0.0;
    if (q < P) {
        const int s = a.rowid[q];
        const bool real = (q - a.pptr[s]) < (int64_t)(a.ptr[s + 1] - a.ptr[s]);
        const int32_t ia = a.idx[q] & kIndexMask;
        const int32_t ib = a.idx[P + q];
        // factor rows: the whole padded row (16 columns), 16-byte loads
        constexpr int NV = 16 * (int)sizeof(AT) / 16;
        uint4 ra[NV], rb[NV];
        const uint4* pa = (const uint4*)((const AT*)a.F[0] + (int64_t)ia * a.ld[0]);
        const uint4* pb = (const uint4*)((const AT*)a.F[1] + (int64_t)ib * a.ld[1]);
#pragma unroll
        for (int v = 0; v < NV; ++v) { ra[v] = pa[v]; rb[v] = pb[v]; }
        const AT* av = (const AT*)ra;
        const AT* bv = (const AT*)rb;
        // a^T M b; instantiated per address space of M (LDS or global memory) and for R_b = 16
        // (row stride known: vector reads of M)
        auto model = [&](const AT* M, auto rb_const) {
            constexpr int RBC = decltype(rb_const)::value;
            const int ld = RBC ? RBC : Rb;
            AT xh = 0;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                if (i < Ra) {
                    AT t = 0;
#pragma unroll
                    for (int j = 0; j < 16; ++j)
                        if (RBC || j < Rb) t += M[i * ld + j] * bv[j];
                    xh += av[i] * t;
                }
            }
            return xh;
        };
        using RB16 = std::integral_constant<int, 16>;
        using RBN = std::integral_constant<int, 0>;
        const AT* Ml = Ms + (int64_t)(s - s_first) * K;
        const AT* Mg = (const AT*)a.W + (int64_t)a.rows[s] * K;
        AT xh;
        if (Rb == 16) xh = staged ? model(Ml, RB16{}) : model(Mg, RB16{});
        else xh = staged ? model(Ml, RBN{}) : model(Mg, RBN{});
        const AT ev = real ? xh - ((const AT*)a.val)[q] : AT(0);
        ((AT*)a.e)[q] = ev;
        e2 = (double)ev * (double)ev;
    }
    if (a.part) {
        for (int o = 32; o > 0; o >>= 1) e2 += __shfl_xor(e2, o);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e2;
        __syncthreads();
        if (threadIdx.x == 0) a.part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
    }
}

// gU[i][r] = scale * sum_c Y[i][c] Gn[r][c]   (c ascending, FP64 accumulation)
template <typename AT>
__global__ void k_gu(const AT* __restrict__ Y, const AT* __restrict__ Gn, int64_t I, int R, int64_t K,
                     double scale, AT* __restrict__ gU) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= I * R) return;
    const int64_t i = e / R;
    const int r = (int)(e % R);
    double acc = 0.0;
    for (int64_t c = 0; c < K; ++c) acc += (double)Y[i * K + c] * (double)Gn[(int64_t)r * K + c];
    gU[e] = (AT)(scale * acc);
}

// Same product, R <= 16: one thread per row i holds its R sums (FP64) and walks the row of Y with
// 16-byte loads; Gn sits in LDS (read by all lanes at the same address).
template <typename AT>
__global__ __launch_bounds__(256) void k_gu_rows(const AT* __restrict__ Y, const AT* __restrict__ Gn, int64_t I,
                                                 int R, int K, double scale, AT* __restrict__ gU) {
    extern __shared__ __align__(16) unsigned char gu_lds[];
    AT* G = (AT*)gu_lds;   // [R][K]
    for (int e = threadIdx.x; e < R * K; e += 256) G[e] = Gn[e];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= I) return;
    double acc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0;
    const AT* y = Y + i * K;
    constexpr int V = 16 / (int)sizeof(AT);   // values per 16-byte load
    for (int c0 = 0; c0 < K; c0 += V) {
        AT yv[V];
        *(uint4*)yv = *(const uint4*)(y + c0);
#pragma unroll
        for (int u = 0; u < V; ++u)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (r < R) acc[r] += (double)yv[u] * (double)G[r * K + c0 + u];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r)
        if (r < R) gU[i * R + r] = (AT)(scale * acc[r]);
}

// Same product for FP32, R <= 16, K % 16 == 0: a wave per 16 rows of Y on v_mfma_f64_16x16x4f64
// (FP32 inputs widened, FP64 sums), Y read once with 16-byte loads.  Lane l = 16 g + c loads
// columns 16 t + 4 g .. 16 t + 4 g + 3 of row c of the tile and of row c of Gn; the u-th of the
// four MFMAs of block t takes the u-th of them (lane l supplies A[c][g] and B[g][c]), so the
// contraction runs over the columns 16 t + 4 g + u.  Lane l holds D[g + 4 v][c] in result v.
__global__ __launch_bounds__(256) void k_gu_mfma(const float* __restrict__ Y, const float* __restrict__ Gn,
                                                 int64_t I, int R, int K, double scale, float* __restrict__ gU) {
    const int lane = threadIdx.x & 63;
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (row0 >= I) return;   // wave-uniform
    const int c = lane & 15, g = lane >> 4;
    const bool rok = row0 + c < I, gok = c < R;
    const float* y = Y + (rok ? row0 + c : 0) * (int64_t)K + 4 * g;
    const float* b = Gn + (int64_t)(gok ? c : 0) * K + 4 * g;
    atb_d4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int t = 0; t < K; t += 16) {
        float4 yv = make_float4(0.f, 0.f, 0.f, 0.f), bv = make_float4(0.f, 0.f, 0.f, 0.f);
        if (rok) yv = *(const float4*)(y + t);
        if (gok) bv = *(const float4*)(b + t);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)yv.x, (double)bv.x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)yv.y, (double)bv.y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)yv.z, (double)bv.z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)yv.w, (double)bv.w, acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t r = row0 + g + 4 * v;
        if (r < I && c < R) gU[r * R + c] = (float)(scale * acc[v]);
    }
}

// part[split][r][c] = sum_{i in slab} U[i][r] Y[i][c] on FP64 MFMA (same blocking as the core)
template <typename AT>
__global__ __launch_bounds__(256) void k_gg_partial(const AT* __restrict__ Y, const AT* __restrict__ U,
                                                    int64_t I, int K, int R, int64_t slab,
                                                    double* __restrict__ part) {
    __shared__ AT As[2][32][65];
    __shared__ AT Bs[2][32][65];
    const int b0 = blockIdx.x * 64, a0 = blockIdx.z * 64;
    const int64_t r0 = (int64_t)blockIdx.y * slab;
    const int64_t r1 = min(I, r0 + slab);
    atb_d4_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = atb_d4_t{0, 0, 0, 0};
    atb_block<AT, AT>(U, R, R, Y, K, K, r0, r1, a0, b0, As, Bs, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int kq = lane >> 4, c16 = lane & 15;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = a0 + 16 * w + kq + 4 * v;
            const int c = b0 + 16 * t + c16;
            if (r < R && c < K) part[((int64_t)blockIdx.y * R + r) * K + c] = acc[t][v];
        }
}

// gG[c * R + r] = scale * sum_split part[split][r][c]  (C order of the core: last mode = r)
template <typename AT>
__global__ void k_gg_reduce(const double* __restrict__ part, int nsplit, int K, int R, double scale,
                            AT* __restrict__ gG) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)K * R) return;
    const int r = (int)(e / K), c = (int)(e % K);
    gG[(int64_t)c * R + r] = (AT)(scale * sum_strided(part + (int64_t)r * K + c, nsplit, (int64_t)R * K));
}

// loss = scale * sum_k part[k]: 1024 threads sum contiguous slices in order, then a fixed tree
template <typename AT>
__global__ __launch_bounds__(1024) void k_loss(const double* __restrict__ part, int64_t n, double scale,
                                               AT* __restrict__ loss) {
    __shared__ double red[1024];
    const int64_t per = (n + 1023) / 1024;
    const int64_t b = (int64_t)threadIdx.x * per, e = min(n, b + per);
    red[threadIdx.x] = (e > b) ? sum_strided(part + b, (int)(e - b), 1) : 0.0;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (AT)(scale * red[0]);
}

template <typename AT>
__global__ void k_fill(AT* __restrict__ p, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = (AT)0;
}

// Lexicographic key (i_0, ..., i_{N-1}) of every padded position of mode m (padding: `pad`,
// which sorts after every real key), and the position itself as the sort value.
struct LexSpec {
    int64_t dims[kMaxOrder];
    int others[kMaxOrder - 1];
    int N, m;
};

__global__ void k_lex_keys(LexSpec ls, const int32_t* __restrict__ rowid, const int32_t* __restrict__ rows,
                           const int32_t* __restrict__ ptr, const int32_t* __restrict__ pptr,
                           const int32_t* __restrict__ idx, int64_t P, uint64_t pad, uint64_t* __restrict__ keys,
                           int32_t* __restrict__ pos) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P) return;
    const int s = rowid[q];
    pos[q] = (int32_t)q;
    if (q - pptr[s] >= (int64_t)ptr[s + 1] - ptr[s]) {
        keys[q] = pad;
        return;
    }
    int64_t c[kMaxOrder];
    c[ls.m] = rows[s];
    for (int j = 0; j < ls.N - 1; ++j) c[ls.others[j]] = idx[(int64_t)j * P + q] & kIndexMask;
    uint64_t key = 0;
    for (int t = 0; t < ls.N; ++t) key = key * (uint64_t)ls.dims[t] + (uint64_t)c[t];
    keys[q] = key;
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

// map[pos_n[r]] = pos_0[r] for the D real entries (the first D of both sorted orders)
__global__ void k_map(const int32_t* __restrict__ pos0, const int32_t* __restrict__ posn, int64_t D,
                      int32_t* __restrict__ map) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < D) map[posn[r]] = pos0[r];
}

// residuals of mode 0's stream into mode n's order (zero on padding)
template <typename AT>
__global__ void k_permute(const int32_t* __restrict__ map, int64_t P, const AT* __restrict__ e0, AT* __restrict__ en) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P) return;
    const int32_t src = map[q];
    en[q] = (src >= 0) ? e0[src] : (AT)0;
}

void gg_plan(int64_t I, int64_t K, int R, int& nsplit, int64_t& slab) {
    const int64_t cblocks = ((K + 63) / 64) * ((R + 63) / 64);
    nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(512 / std::max<int64_t>(cblocks, 1), (I + 127) / 128));
    slab = ((I + nsplit - 1) / nsplit + 31) / 32 * 32;
    nsplit = (int)((I + slab - 1) / slab);
}

int ensure_ws(tk_ctx* ctx, hipStream_t s) {
    CompletionWs& w = ctx->cws;
    if (w.ready) return TK_OK;
    const int N = ctx->N;
    const size_t at = ytype_size(ctx->dtype);
    bool fused = ctx->nnz > 0;
    for (int n = 0; n < N; ++n) fused = fused && ttmc_residual_form(ctx, n);
    int64_t maxP = 0, maxIK = 0, gn = 0, part = 1024;
    for (int n = 0; n < N; ++n) {
        const ModeLayout& ml = ctx->mode[n];
        maxP = std::max(maxP, ml.P);
        maxIK = std::max<int64_t>(maxIK, ctx->dims[n] * (fused ? 256 : ml.K));
        gn += (int64_t)ctx->ranks[n] * ml.K;
        part = std::max<int64_t>(part, fused ? ml.nchunks : (ml.P + 255) / 256);
        int ns;
        int64_t sl;
        gg_plan(ctx->dims[n], ml.K, ctx->ranks[n], ns, sl);
        part = std::max<int64_t>(part, (int64_t)ns * ctx->ranks[n] * ml.K);
    }
    auto alloc = [&](void** p, size_t bytes) -> int {
        hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 16));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return set_error(TK_ERR_OOM, "completion workspace: allocation of %zu bytes failed", bytes);
        }
        return TK_OK;
    };
    int st;
    if ((st = alloc(&w.W, (size_t)maxIK * at)) || (st = alloc(&w.Gn, (size_t)gn * at)) ||
        (st = alloc((void**)&w.part, (size_t)part * 8)))
        return st;
    if (fused) {   // the residuals never leave the TTMc kernel: no residual arrays, no position maps
        w.fused = true;
        w.ready = true;
        return TK_OK;
    }
    if ((st = alloc(&w.e, (size_t)maxP * at)) || (st = alloc(&w.e2, (size_t)maxP * at))) return st;
    for (int n = 0; n < N; ++n) {
        const ModeLayout& ml = ctx->mode[n];
        if ((st = alloc((void**)&w.rowid[n], (size_t)ml.P * 4))) return st;
        if (ml.P > 0) {
            k_rowid<<<cdiv(ml.P, 256), 256, 0, s>>>(ml.pptr, ml.S, ml.P, w.rowid[n]);
            TK_LAUNCH_CHECK("k_rowid");
        }
    }
    // position maps: mode 0's and mode n's padded streams sorted by the lexicographic key
    const int64_t D = ctx->nnz;
    if (D > 0 && N >= 2) {
        uint64_t prod = 1;
        for (int t = 0; t < N; ++t) prod *= (uint64_t)ctx->dims[t];   // < 2^63, checked at init
        int bits = 1;
        while (bits < 63 && ((prod >> bits) != 0)) ++bits;
        const uint64_t pad = (bits >= 64) ? ~0ull : ((1ull << bits) - 1);   // > every real key
        void *kin = nullptr, *kout = nullptr, *pin = nullptr, *pout = nullptr, *pos0 = nullptr, *tmp = nullptr;
        size_t tmp_bytes = 0;
        TK_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                                  (int32_t*)nullptr, (int32_t*)nullptr, (int)maxP, 0, bits, s));
        auto release = [&]() {
            (void)hipStreamSynchronize(s);
            void* ps[] = {kin, kout, pin, pout, pos0, tmp};
            for (void* p : ps)
                if (p) (void)hipFree(p);
        };
        if ((st = alloc(&kin, (size_t)maxP * 8)) || (st = alloc(&kout, (size_t)maxP * 8)) ||
            (st = alloc(&pin, (size_t)maxP * 4)) || (st = alloc(&pout, (size_t)maxP * 4)) ||
            (st = alloc(&pos0, (size_t)D * 4)) || (st = alloc(&tmp, tmp_bytes))) {
            release();
            return st;
        }
        for (int n = 0; n < N; ++n) {
            const ModeLayout& ml = ctx->mode[n];
            LexSpec ls{};
            ls.N = N;
            ls.m = n;
            for (int t = 0; t < N; ++t) ls.dims[t] = ctx->dims[t];
            for (int j = 0; j < N - 1; ++j) ls.others[j] = ml.others[j];
            k_lex_keys<<<cdiv(ml.P, 256), 256, 0, s>>>(ls, w.rowid[n], ml.rows, ml.ptr, ml.pptr, ml.idx, ml.P, pad,
                                                     (uint64_t*)kin, (int32_t*)pin);
            if (hipGetLastError() != hipSuccess) {
                release();
                return set_error(TK_ERR_HIP, "k_lex_keys launch failed");
            }
            size_t tb = tmp_bytes;
            if (hipcub::DeviceRadixSort::SortPairs(tmp, tb, (uint64_t*)kin, (uint64_t*)kout, (int32_t*)pin,
                                                   (int32_t*)pout, (int)ml.P, 0, bits, s) != hipSuccess) {
                release();
                return set_error(TK_ERR_HIP, "position-map sort failed");
            }
            if (n == 0) {
                if (hipMemcpyAsync(pos0, pout, (size_t)D * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) {
                    release();
                    return set_error(TK_ERR_HIP, "position-map copy failed");
                }
                continue;
            }
            if ((st = alloc((void**)&w.map[n], (size_t)ml.P * 4))) {
                release();
                return st;
            }
            k_fill_i32<<<cdiv(ml.P, 256), 256, 0, s>>>(w.map[n], ml.P, -1);
            k_map<<<cdiv(D, 256), 256, 0, s>>>((const int32_t*)pos0, (const int32_t*)pout, D, w.map[n]);
            if (hipGetLastError() != hipSuccess) {
                release();
                return set_error(TK_ERR_HIP, "k_map launch failed");
            }
        }
        release();
    }
    w.ready = true;
    return TK_OK;
}

// gU_n = scale * TTMc_n(E) G_(n)^T, and for the last mode gG = scale * U_N^T TTMc_N(E)
template <typename AT>
int gradients(const AT* Y, const AT* Gn, const AT* Un, int64_t I, int R, int64_t K, double scale, bool last,
              double* part, AT* gUn, AT* gG, hipStream_t s) {
    if (std::is_same<AT, float>::value && R <= 16 && K % 16 == 0) {
        k_gu_mfma<<<cdiv(I, 64), 256, 0, s>>>((const float*)Y, (const float*)Gn, I, R, (int)K, scale, (float*)gUn);
        TK_LAUNCH_CHECK("k_gu_mfma");
    } else if (R <= 16 && K % 4 == 0 && (size_t)R * K * sizeof(AT) <= 64 * 1024) {
        k_gu_rows<AT><<<cdiv(I, 256), 256, (size_t)R * K * sizeof(AT), s>>>(Y, Gn, I, R, (int)K, scale, gUn);
        TK_LAUNCH_CHECK("k_gu_rows");
    } else {
        k_gu<AT><<<cdiv(I * R, 256), 256, 0, s>>>(Y, Gn, I, R, K, scale, gUn);
        TK_LAUNCH_CHECK("k_gu");
    }
    if (last) {
        int nsplit;
        int64_t slab;
        gg_plan(I, K, R, nsplit, slab);
        dim3 grid(cdiv(K, 64), (unsigned)nsplit, cdiv(R, 64));
        k_gg_partial<AT><<<grid, 256, 0, s>>>(Y, Un, I, (int)K, R, slab, part);
        TK_LAUNCH_CHECK("k_gg_partial");
        k_gg_reduce<AT><<<cdiv(K * R, 256), 256, 0, s>>>(part, nsplit, (int)K, R, scale, gG);
        TK_LAUNCH_CHECK("k_gg_reduce");
    }
    return TK_OK;
}

// Order 3, FP32: per mode, W_n = U_n G_(n) in 16 x 16 blocks and the TTMc over the residuals
// computed inside the kernel (mode 0's pass also yields the per-chunk loss partials)
int adjoint_fused(tk_ctx* ctx, const float* G, const float* const* U, float* loss, float* gG, float* const* gU,
                  double scale, int64_t size, hipStream_t s) {
    CompletionWs& w = ctx->cws;
    const int N = ctx->N;
    float* Gn = (float*)w.Gn;
    int st;
    for (int n = 0; n < N; ++n) {
        const ModeLayout& ml = ctx->mode[n];
        const int64_t I = ctx->dims[n];
        const int R = ctx->ranks[n];
        Unfold u{};
        for (int t = 0; t < N; ++t) u.R[t] = ctx->ranks[t];
        u.N = N;
        u.n = n;
        u.K = ml.K;
        u.size = size;
        k_unfold<float><<<cdiv(size, 256), 256, 0, s>>>(u, G, Gn);
        TK_LAUNCH_CHECK("k_unfold");
        const int Ra = ctx->ranks[ml.others[0]], Rb = ctx->ranks[ml.others[1]];
        const unsigned wgrid = cdiv(I, kW16Rows);
        if (R == 16) k_w16<16><<<wgrid, 256, 0, s>>>(U[n], Gn, I, R, Ra, Rb, (float*)w.W);
        else k_w16<0><<<wgrid, 256, 0, s>>>(U[n], Gn, I, R, Ra, Rb, (float*)w.W);
        TK_LAUNCH_CHECK("k_w16");
        if ((st = ttmc_residual_run(ctx, n, ctx->ws.y, (const float*)w.W, n == 0 ? w.part : nullptr, s))) return st;
        if (n == 0) {
            // the loss partials are consumed before the last mode reuses the buffer
            k_loss<float><<<1, 1024, 0, s>>>(w.part, ml.nchunks, 0.5 * scale, loss);
            TK_LAUNCH_CHECK("k_loss");
        }
        if ((st = gradients<float>((const float*)ctx->ws.y, Gn, U[n], I, R, ml.K, scale, n == N - 1, w.part, gU[n],
                                   gG, s)))
            return st;
    }
    return TK_OK;
}

template <typename AT>
int adjoint_typed(tk_ctx* ctx, const AT* G, const AT* const* U, AT* loss, AT* gG, AT* const* gU, hipStream_t s) {
    const int N = ctx->N;
    int st;
    if (ctx->nnz == 0) {   // empty pattern: zero loss and gradients
        k_fill<AT><<<1, 64, 0, s>>>(loss, 1);
        int64_t size = 1;
        for (int t = 0; t < N; ++t) size *= ctx->ranks[t];
        k_fill<AT><<<cdiv(size, 256), 256, 0, s>>>(gG, size);
        for (int t = 0; t < N; ++t) {
            const int64_t n = ctx->dims[t] * ctx->ranks[t];
            k_fill<AT><<<cdiv(n, 256), 256, 0, s>>>(gU[t], n);
        }
        TK_LAUNCH_CHECK("k_fill");
        return TK_OK;
    }
    if ((st = ensure_ws(ctx, s))) return st;
    CompletionWs& w = ctx->cws;
    const double scale = 1.0 / (double)ctx->nnz;
    // low-precision factor copies read by the TTMc kernels (here in the parameter type)
    for (int t = 0; t < N; ++t) {
        const int64_t I = ctx->dims[t];
        k_factor_copy<AT, AT><<<cdiv(I * ctx->ldU[t], 256), 256, 0, s>>>(U[t], I, ctx->ranks[t], ctx->ldU[t],
                                                                          (AT*)ctx->Ulp[t]);
        TK_LAUNCH_CHECK("k_factor_copy");
    }
    int64_t size = 1;
    for (int t = 0; t < N; ++t) size *= ctx->ranks[t];
    AT* Gn = (AT*)w.Gn;
    if constexpr (std::is_same<AT, float>::value) {
        if (w.fused) return adjoint_fused(ctx, G, U, loss, gG, gU, scale, size, s);
    }
    int64_t nblk0 = 0;
    for (int n = 0; n < N; ++n) {
        const ModeLayout& ml = ctx->mode[n];
        const int64_t I = ctx->dims[n];
        const int R = ctx->ranks[n];
        const int64_t K = ml.K;
        Unfold u{};
        for (int t = 0; t < N; ++t) u.R[t] = ctx->ranks[t];
        u.N = N;
        u.n = n;
        u.K = K;
        u.size = size;
        k_unfold<AT><<<cdiv(size, 256), 256, 0, s>>>(u, G, Gn);
        TK_LAUNCH_CHECK("k_unfold");
        if (n > 0) {
            // the residuals of mode 0's stream, in mode n's order
            if (ml.P > 0) {
                k_permute<AT><<<cdiv(ml.P, 256), 256, 0, s>>>(w.map[n], ml.P, (const AT*)w.e, (AT*)w.e2);
                TK_LAUNCH_CHECK("k_permute");
            }
        } else if (ml.P > 0) {
            k_w<AT><<<cdiv(I * K, 256), 256, 0, s>>>(U[n], Gn, I, R, K, (AT*)w.W);
            TK_LAUNCH_CHECK("k_w");
            ResidArgs ra{};
            ra.rowid = w.rowid[n];
            ra.rows = ml.rows;
            ra.ptr = ml.ptr;
            ra.pptr = ml.pptr;
            ra.idx = ml.idx;
            ra.P = ml.P;
            ra.val = ml.val;
            for (int j = 0; j < N - 1; ++j) {
                const int t = ml.others[j];
                ra.F[j] = ctx->Ulp[t];
                ra.ld[j] = ctx->ldU[t];
                ra.R[j] = ctx->ranks[t];
            }
            ra.nm1 = N - 1;
            ra.K = K;
            ra.W = w.W;
            ra.e = w.e;
            ra.part = (n == 0) ? w.part : nullptr;
            if (N == 3 && ra.R[0] <= 16 && ra.R[1] <= 16 && ctx->ldU[ml.others[0]] == 16 &&
                ctx->ldU[ml.others[1]] == 16) {
                const size_t lds = (size_t)kResidRows * K * sizeof(AT);
                k_residual3<AT><<<cdiv(ml.P, 256), 256, lds, s>>>(ra);
                TK_LAUNCH_CHECK("k_residual3");
            } else {
                k_residual<AT><<<cdiv(ml.P, 256), 256, 0, s>>>(ra);
                TK_LAUNCH_CHECK("k_residual");
            }
            nblk0 = (ml.P + 255) / 256;
        }
        // TTMc_n(E): the forward kernels with the residuals in place of the values
        if ((st = ttmc_run(ctx, n, ctx->ws.y, s, nullptr, n == 0 ? w.e : w.e2))) return st;
        if (n == 0) {
            // the loss partials of mode 0 are consumed before the last mode reuses the buffer
            k_loss<AT><<<1, 1024, 0, s>>>(w.part, nblk0, 0.5 * scale, loss);
            TK_LAUNCH_CHECK("k_loss");
        }
        if ((st = gradients<AT>((const AT*)ctx->ws.y, Gn, U[n], I, R, K, scale, n == N - 1, w.part, gU[n], gG, s)))
            return st;
    }
    return TK_OK;
}

}  // namespace

void free_completion_ws(tk_ctx* ctx) {
    CompletionWs& w = ctx->cws;
    void* ps[] = {w.e, w.e2, w.W, w.Gn, w.part};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    for (int n = 0; n < kMaxOrder; ++n) {
        if (w.rowid[n]) (void)hipFree(w.rowid[n]);
        if (w.map[n]) (void)hipFree(w.map[n]);
    }
    w = CompletionWs{};
}

int adjoint_run(tk_ctx* ctx, const void* G, const void* const* U, void* loss, void* gG, void* const* gU,
                hipStream_t s) {
    if (ctx->dtype == TK_F64)
        return adjoint_typed<double>(ctx, (const double*)G, (const double* const*)U, (double*)loss, (double*)gG,
                                     (double* const*)gU, s);
    return adjoint_typed<float>(ctx, (const float*)G, (const float* const*)U, (float*)loss, (float*)gG,
                                (float* const*)gU, s);
}

}  // namespace tk
