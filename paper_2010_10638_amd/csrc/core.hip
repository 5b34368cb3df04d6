// Core tensor and fit (paper Alg. 2, the step after the mode loop; Sec. III-B unfolded form
// G_(N) = U_N^T Y_(N)), sampled reconstruction of the Tucker model, factor conversions.
#include <mutex>

#include "internal.h"
#include "atb.h"

namespace tk {

// Scratch of the allocation-free core/fit entry point (core_fit_static): the per-slab partial
// products of G_(N).  One copy per device, held until the process ends; calls on one device share it.
constexpr int64_t kCoreScratchDoubles = (int64_t)1 << 20;   // 8 MiB
static __device__ __align__(256) double scratch[kCoreScratchDoubles];

namespace {

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

__global__ void k_fill_zero(uint32_t* __restrict__ p, int64_t words) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < words;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0u;
}

__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = v;
}

template <typename LT>
__global__ void k_convert_factor(const double* __restrict__ U, int64_t I, int R, int ld, LT* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= I * ld) return;
    const int64_t i = e / ld;
    const int c = (int)(e % ld);
    const double u = (c < R) ? U[i * R + c] : 0.0;
    if constexpr (sizeof(LT) == 8) out[e] = u;
    else if constexpr (sizeof(LT) == 4) out[e] = (float)u;
    else out[e] = f32_to_bf16((float)u);
}

// part[split][r][c] = sum_{i in slab} U[i][r] * Y[i][c] for r in a 64-block of U's columns and
// c in a 64-block of Y's columns, on FP64 MFMA through LDS panels.
template <typename YT>
__global__ __launch_bounds__(256) void k_core_partial(const YT* __restrict__ Y, const double* __restrict__ U,
                                                      int64_t I, int K, int R, int64_t slab,
                                                      double* __restrict__ part) {
    __shared__ double As[2][32][65];
    __shared__ YT Bs[2][32][65];
    const int b0 = blockIdx.x * 64, a0 = blockIdx.z * 64;
    const int64_t r0 = (int64_t)blockIdx.y * slab;
    const int64_t r1 = min(I, r0 + slab);
    atb_d4_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = atb_d4_t{0, 0, 0, 0};
    atb_block<double, YT>(U, R, R, Y, K, K, r0, r1, a0, b0, As, Bs, acc);
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

// G[c * R + r] = sum_split part[split][r][c], summed in split order (thread e = r * K + c, so the
// partial reads are coalesced).
__global__ void k_core_reduce(const double* __restrict__ part, int nsplit, int K, int R,
                              double* __restrict__ G) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)K * R) return;
    const int r = (int)(e / K), c = (int)(e % K);
    G[(int64_t)c * R + r] = sum_strided(part + (int64_t)r * K + c, nsplit, (int64_t)R * K);
}

// ||G||^2 (fixed-order tree) and fit = 1 - sqrt(max(||X||^2 - ||G||^2, 0)) / ||X||.
__global__ __launch_bounds__(1024) void k_core_fit(const double* __restrict__ G, int64_t size, double normx2,
                                                   double* __restrict__ fit) {
    __shared__ double red[16];
    double g2 = 0.0;
    for (int64_t e = threadIdx.x; e < size; e += blockDim.x) g2 += G[e] * G[e];
    for (int o = 32; o > 0; o >>= 1) g2 += __shfl_xor(g2, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = g2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
        double r2 = normx2 - s;
        if (r2 < 0.0) r2 = 0.0;
        *fit = (normx2 > 0.0) ? 1.0 - sqrt(r2) / sqrt(normx2) : 0.0;
    }
}

struct ReconArgs {
    const double* U[kMaxOrder];
    int32_t R[kMaxOrder];
    int N;
    int64_t size;
};

// One thread per coordinate; the core is walked in C order (last index fastest) with an
// odometer that recomputes only the prefix products whose digit changed.
__global__ void k_reconstruct(ReconArgs a, const double* __restrict__ G, int64_t m,
                              const int32_t* __restrict__ coords, double* __restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    const double* row[kMaxOrder];
    int r[kMaxOrder];
    double pre[kMaxOrder + 1];
    const int N = a.N;
    for (int t = 0; t < N; ++t) {
        row[t] = a.U[t] + (int64_t)coords[(int64_t)t * m + p] * a.R[t];
        r[t] = 0;
    }
    pre[0] = 1.0;
    for (int t = 0; t < N; ++t) pre[t + 1] = pre[t] * row[t][0];
    double sum = 0.0;
    for (int64_t g = 0; g < a.size; ++g) {
        sum += G[g] * pre[N];
        int t = N - 1;
        while (t >= 0) {
            if (++r[t] < a.R[t]) break;
            r[t] = 0;
            --t;
        }
        if (t < 0) break;
        for (int u = t; u < N; ++u) pre[u + 1] = pre[u] * row[u][r[u]];
    }
    out[p] = sum;
}

}  // namespace

int fill_zero(void* p, size_t bytes, hipStream_t s) {
    const int64_t words = (int64_t)(bytes / 4);
    if (words == 0) return TK_OK;
    k_fill_zero<<<std::min<unsigned>(2048, cdiv(words, 256)), 256, 0, s>>>((uint32_t*)p, words);
    TK_LAUNCH_CHECK("k_fill_zero");
    return TK_OK;
}

int fill_f64(double* p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return TK_OK;
    k_fill_f64<<<cdiv(n, 256), 256, 0, s>>>(p, n, v);
    TK_LAUNCH_CHECK("k_fill_f64");
    return TK_OK;
}

int convert_factor(tk_ctx* ctx, int k, const double* U, hipStream_t s) {
    const int64_t I = ctx->dims[k];
    const int R = ctx->ranks[k], ld = ctx->ldU[k];
    const unsigned g = cdiv(I * ld, 256);
    if (ctx->dtype == TK_F64) k_convert_factor<double><<<g, 256, 0, s>>>(U, I, R, ld, (double*)ctx->Ulp[k]);
    else if (ctx->dtype == TK_F32) k_convert_factor<float><<<g, 256, 0, s>>>(U, I, R, ld, (float*)ctx->Ulp[k]);
    else k_convert_factor<bf16_t><<<g, 256, 0, s>>>(U, I, R, ld, (bf16_t*)ctx->Ulp[k]);
    TK_LAUNCH_CHECK("k_convert_factor");
    return TK_OK;
}

static void core_plan(const tk_ctx* ctx, int& nsplit, int64_t& slab) {
    const int n = ctx->N - 1;
    const int64_t I = ctx->dims[n];
    const int64_t K = ctx->mode[n].K;
    const int64_t cblocks = ((K + 63) / 64) * ((ctx->ranks[n] + 63) / 64);
    nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(512 / std::max<int64_t>(cblocks, 1), (I + 127) / 128));
    slab = ((I + nsplit - 1) / nsplit + 31) / 32 * 32;
    nsplit = (int)((I + slab - 1) / slab);
}

size_t core_workspace_bytes(const tk_ctx* ctx) {
    int nsplit;
    int64_t slab;
    core_plan(ctx, nsplit, slab);
    const int n = ctx->N - 1;
    return (size_t)nsplit * ctx->ranks[n] * ctx->mode[n].K * 8;
}

int core_run(tk_ctx* ctx, const void* Y, const double* U, double* G, double* fit, hipStream_t s) {
    const int n = ctx->N - 1;
    const int64_t I = ctx->dims[n];
    const int K = (int)ctx->mode[n].K;
    const int R = ctx->ranks[n];
    int nsplit;
    int64_t slab;
    core_plan(ctx, nsplit, slab);
    double* part = ctx->ws.qrp;   // the QRP of the last mode has finished with its workspace
    dim3 grid(cdiv(K, 64), (unsigned)nsplit, cdiv(R, 64));
    if (ctx->dtype == TK_F64)
        k_core_partial<double><<<grid, 256, 0, s>>>((const double*)Y, U, I, K, R, slab, part);
    else
        k_core_partial<float><<<grid, 256, 0, s>>>((const float*)Y, U, I, K, R, slab, part);
    TK_LAUNCH_CHECK("k_core_partial");
    k_core_reduce<<<cdiv((int64_t)K * R, 256), 256, 0, s>>>(part, nsplit, K, R, G);
    TK_LAUNCH_CHECK("k_core_reduce");
    if (fit) {
        k_core_fit<<<1, 1024, 0, s>>>(G, (int64_t)K * R, ctx->normx2, fit);
        TK_LAUNCH_CHECK("k_core_fit");
    }
    return TK_OK;
}

int64_t core_static_max_cols() { return kCoreScratchDoubles; }

// Device address of this device's copy of `scratch`, looked up once per device with that device
// current (the array's name is only a host-side stand-in).
static int core_scratch_address(double** out) {
    static std::mutex mu;
    static double* addr[64] = {};
    int dev = 0;
    TK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return set_error(TK_ERR_UNSUPPORTED, "device ordinal %d above 63", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        TK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_error(TK_ERR_HIP, "hipGetSymbolAddress returned a null address");
        addr[dev] = (double*)p;
    }
    *out = addr[dev];
    return TK_OK;
}

int core_static_run(int ytype, int64_t I, int R, int64_t K, const void* Y, const double* U, double normx2,
                    double* G, double* fit, hipStream_t s) {
    double* part = nullptr;
    int st = core_scratch_address(&part);
    if (st) return st;
    // slabs as in core_run, at most as many as the scratch holds
    const int64_t cblocks = ((K + 63) / 64) * ((R + 63) / 64);
    int64_t nsplit = std::max<int64_t>(1, std::min<int64_t>(512 / std::max<int64_t>(cblocks, 1), (I + 127) / 128));
    nsplit = std::max<int64_t>(1, std::min<int64_t>(nsplit, kCoreScratchDoubles / ((int64_t)R * K)));
    const int64_t slab = ((I + nsplit - 1) / nsplit + 31) / 32 * 32;
    nsplit = (I + slab - 1) / slab;
    dim3 grid(cdiv(K, 64), (unsigned)nsplit, cdiv(R, 64));
    if (ytype == TK_F64)
        k_core_partial<double><<<grid, 256, 0, s>>>((const double*)Y, U, I, (int)K, R, slab, part);
    else
        k_core_partial<float><<<grid, 256, 0, s>>>((const float*)Y, U, I, (int)K, R, slab, part);
    TK_LAUNCH_CHECK("k_core_partial");
    k_core_reduce<<<cdiv(K * R, 256), 256, 0, s>>>(part, (int)nsplit, (int)K, R, G);
    TK_LAUNCH_CHECK("k_core_reduce");
    if (fit) {
        k_core_fit<<<1, 1024, 0, s>>>(G, K * R, normx2, fit);
        TK_LAUNCH_CHECK("k_core_fit");
    }
    return TK_OK;
}

int reconstruct_run(tk_ctx* ctx, const double* G, const double* const* U, int64_t m,
                    const int32_t* coords, double* out, hipStream_t s) {
    if (m == 0) return TK_OK;
    ReconArgs a{};
    a.N = ctx->N;
    a.size = 1;
    for (int t = 0; t < ctx->N; ++t) {
        a.U[t] = U[t];
        a.R[t] = ctx->ranks[t];
        a.size *= ctx->ranks[t];
    }
    k_reconstruct<<<cdiv(m, 128), 128, 0, s>>>(a, G, m, coords, out);
    TK_LAUNCH_CHECK("k_reconstruct");
    return TK_OK;
}

}  // namespace tk
