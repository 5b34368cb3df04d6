// C ABI entry points (include/sptucker.h): argument validation, context lifetime, workspace
// sizing, and the sweep driver of Alg. 2.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.h"

namespace tk {

static thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int hip_error(hipError_t e, const char* what) {
    (void)hipGetLastError();
    return set_error(e == hipErrorOutOfMemory ? TK_ERR_OOM : TK_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int qrp_route(const tk_ctx* ctx, int mode);

namespace {

int dmalloc(void** p, size_t bytes) {
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return set_error(TK_ERR_OOM, "device allocation of %zu bytes failed", bytes);
    }
    return TK_OK;
}

void free_events(tk_ctx* c) {
    if (c->prof_ev) {
        const int per = 4 * c->N + 2;
        for (int i = 0; i < c->prof_cap * per; ++i)
            if (c->prof_ev[i]) (void)hipEventDestroy(c->prof_ev[i]);
        delete[] c->prof_ev;
    }
    c->prof_ev = nullptr;
    c->prof_cap = 0;
    c->prof_used = 0;
}

void free_ctx(tk_ctx* c) {
    if (!c) return;
    free_events(c);
    free_completion_ws(c);
    free_svd_ws(c);
    free_memo(c);
    for (int m = 0; m < kMaxOrder; ++m) {
        ModeLayout& ml = c->mode[m];
        void* ps[] = {ml.rows, ml.ptr, ml.pptr, ml.idx, ml.val, ml.chunk_ptr, ml.chunk_row, ml.chunk_slot, ml.split};
        for (void* p : ps)
            if (p) (void)hipFree(p);
        if (c->Ulp[m]) (void)hipFree(c->Ulp[m]);
    }
    void* ws[] = {c->ws.y, c->ws.carry, c->ws.qrp, c->ws.qrp_int, c->ws.scal, c->qrp_gaps};
    for (void* p : ws)
        if (p) (void)hipFree(p);
    delete c;
}

int check_ctx(const tk_ctx* c) {
    if (!c) return set_error(TK_ERR_ARG, "null context");
    return TK_OK;
}

int check_mode(const tk_ctx* c, int mode) {
    if (mode < 0 || mode >= c->N) return set_error(TK_ERR_ARG, "mode %d outside [0, %d)", mode, c->N);
    return TK_OK;
}

// Surface asynchronous faults of earlier work before enqueueing more.
int pending_error() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "earlier device work");
    return TK_OK;
}

}  // namespace
}  // namespace tk

using namespace tk;

extern "C" {

const char* tucker_last_error(void) { return tk::g_err; }

int tucker_init(tk_ctx** out, int order, const int64_t* dims, const int32_t* ranks, int64_t nnz,
                const int32_t* coords, const double* vals, int dtype, uint32_t flags, void* stream) {
    if (!out) return set_error(TK_ERR_ARG, "out is null");
    *out = nullptr;
    if (order < 2 || order > kMaxOrder) return set_error(TK_ERR_ARG, "order %d outside [2, %d]", order, kMaxOrder);
    if (!dims || !ranks) return set_error(TK_ERR_ARG, "dims/ranks is null");
    if (dtype != TK_F64 && dtype != TK_F32 && dtype != TK_BF16) return set_error(TK_ERR_ARG, "bad dtype %d", dtype);
    if (nnz < 0) return set_error(TK_ERR_ARG, "negative nnz");
    if (nnz >= (int64_t)1 << 31) return set_error(TK_ERR_UNSUPPORTED, "nnz %lld >= 2^31", (long long)nnz);
    if (nnz > 0 && (!coords || !vals)) return set_error(TK_ERR_ARG, "coords/vals is null");
    if (flags & ~(TK_FLAG_NO_FAT_RULE | TK_FLAG_SVD | TK_FLAG_SVD_LIB | TK_FLAG_NO_MEMO))
        return set_error(TK_ERR_ARG, "unknown flags 0x%x", flags);
    double log2prod = 0.0;
    for (int t = 0; t < order; ++t) {
        if (dims[t] < 1) return set_error(TK_ERR_ARG, "dims[%d] = %lld < 1", t, (long long)dims[t]);
        if (dims[t] >= ((int64_t)1 << 31)) return set_error(TK_ERR_UNSUPPORTED, "dims[%d] >= 2^31", t);
        if (ranks[t] < 1 || ranks[t] > dims[t])
            return set_error(TK_ERR_ARG, "ranks[%d] = %d outside [1, I_%d = %lld]", t, ranks[t], t, (long long)dims[t]);
        log2prod += std::log2((double)dims[t]);
    }
    if (log2prod >= 62.999) return set_error(TK_ERR_UNSUPPORTED, "prod(dims) must be below 2^63");
    for (int n = 0; n < order; ++n) {
        int64_t K = 1;
        for (int t = 0; t < order; ++t)
            if (t != n) K *= ranks[t];
        if (K > kMaxK) return set_error(TK_ERR_UNSUPPORTED, "K_%d = %lld exceeds %d", n, (long long)K, kMaxK);
        if (ranks[n] > K) return set_error(TK_ERR_ARG, "ranks[%d] = %d exceeds K_%d = %lld", n, ranks[n], n, (long long)K);
    }
    int st = pending_error();
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    tk_ctx* c = new tk_ctx();
    c->N = order;
    c->dtype = dtype;
    c->flags = flags;
    for (int t = 0; t < order; ++t) {
        c->dims[t] = dims[t];
        c->ranks[t] = ranks[t];
    }
    (void)hipGetDevice(&c->device);
    st = build_layout(c, coords, vals, nnz, s);
    if (st) { free_ctx(c); return st; }
    // factor copies and workspaces
    size_t ybytes = 0, cbytes = 0, qbytes = core_workspace_bytes(c);
    int64_t maxn = 0;
    // factor copies: 16 columns (a multiple of 16 above 16), except order >= 4 with every rank
    // <= 8, whose fiber-factored TTMc gathers 8-column rows (half the bytes and cache footprint)
    for (int t = 0; t < order; ++t) {
        c->ldU[t] = factor_ld(order, ranks, t);
        if ((st = dmalloc(&c->Ulp[t], (size_t)dims[t] * c->ldU[t] * dtype_size(dtype)))) { free_ctx(c); return st; }
        if ((st = fill_zero(c->Ulp[t], (size_t)dims[t] * c->ldU[t] * dtype_size(dtype), s))) { free_ctx(c); return st; }
        const ModeLayout& ml = c->mode[t];
        ybytes = std::max(ybytes, (size_t)dims[t] * ml.K * ytype_size(dtype));
        cbytes = std::max(cbytes, (size_t)ml.ncarry * ml.K * ytype_size(dtype));
        qbytes = std::max(qbytes, qrp_workspace_bytes(c, t));
        maxn = std::max<int64_t>(maxn, std::max<int64_t>(ml.K, dims[t]));
    }
    c->ws.y_bytes = ybytes;
    c->ws.carry_bytes = cbytes;
    c->ws.qrp_bytes = qbytes;
    c->ws.qrp_int_bytes = (size_t)(64 + maxn) * 4;
    if ((st = dmalloc(&c->ws.y, ybytes)) || (st = dmalloc(&c->ws.carry, cbytes)) ||
        (st = dmalloc((void**)&c->ws.qrp, qbytes)) || (st = dmalloc((void**)&c->ws.qrp_int, c->ws.qrp_int_bytes)) ||
        (st = dmalloc((void**)&c->ws.scal, 16 * sizeof(double))) ||
        (st = dmalloc((void**)&c->qrp_gaps, (size_t)order * kGramMaxR * sizeof(double)))) {
        free_ctx(c);
        return st;
    }
    if ((st = fill_f64(c->qrp_gaps, (int64_t)order * kGramMaxR, NAN, s))) { free_ctx(c); return st; }
    // the QRP flag and the completion ticket of the Q1 Gram start at zero
    if ((st = fill_zero(c->ws.qrp_int, c->ws.qrp_int_bytes, s))) { free_ctx(c); return st; }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) { free_ctx(c); return hip_error(e, "tucker_init"); }
    c->last_stream = s;
    *out = c;
    return TK_OK;
}

int tucker_get_info(const tk_ctx* ctx, int64_t* nnz_distinct, int64_t* rows, int64_t* chunks, double* normx2) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (nnz_distinct) *nnz_distinct = ctx->nnz;
    for (int m = 0; m < ctx->N; ++m) {
        if (rows) rows[m] = ctx->mode[m].S;
        if (chunks) chunks[m] = ctx->mode[m].nchunks;
    }
    if (normx2) *normx2 = ctx->normx2;
    return TK_OK;
}

int tucker_get_csf(tk_ctx* ctx, int mode, int32_t* rows, int64_t* ptr, int32_t* idx, void* vals, void* stream) {
    int st = check_ctx(ctx);
    if (st || (st = check_mode(ctx, mode))) return st;
    const ModeLayout& ml = ctx->mode[mode];
    hipStream_t s = (hipStream_t)stream;
    if (ml.S > 0 && !rows) return set_error(TK_ERR_ARG, "rows is null");
    if (!ptr) return set_error(TK_ERR_ARG, "ptr is null");
    if (ctx->nnz > 0 && (!idx || !vals)) return set_error(TK_ERR_ARG, "idx/vals is null");
    if (ml.S > 0) TK_HIP(hipMemcpyAsync(rows, ml.rows, (size_t)ml.S * 4, hipMemcpyDeviceToDevice, s));
    // widen the int32 row pointers on the host side of the copy (init-time data, small)
    std::vector<int32_t> h32((size_t)ml.S + 1);
    std::vector<int64_t> h64((size_t)ml.S + 1);
    TK_HIP(hipMemcpyAsync(h32.data(), ml.ptr, h32.size() * 4, hipMemcpyDeviceToHost, s));
    TK_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < h32.size(); ++i) h64[i] = h32[i];
    TK_HIP(hipMemcpyAsync(ptr, h64.data(), h64.size() * 8, hipMemcpyHostToDevice, s));
    if (ctx->nnz > 0 && (st = export_layout(ctx, mode, idx, vals, s))) return st;
    TK_HIP(hipStreamSynchronize(s));
    ctx->last_stream = s;
    return TK_OK;
}

int ttmc_mode(tk_ctx* ctx, int mode, const double* const* U, void* Y, void* stream) {
    int st = check_ctx(ctx);
    if (st || (st = check_mode(ctx, mode))) return st;
    if (!U || !Y) return set_error(TK_ERR_ARG, "U/Y is null");
    for (int t = 0; t < ctx->N; ++t)
        if (t != mode && !U[t]) return set_error(TK_ERR_ARG, "U[%d] is null", t);
    if ((st = pending_error())) return st;
    hipStream_t s = (hipStream_t)stream;
    for (int t = 0; t < ctx->N; ++t)
        if (t != mode && (st = convert_factor(ctx, t, U[t], s))) return st;
    st = ttmc_run(ctx, mode, Y, s);
    ctx->last_stream = s;
    return st;
}

int ttmc_memo_pair(tk_ctx* ctx, const double* const* U, const double* U_next, void* Y_a, void* Y_b, void* stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    const int N = ctx->N;
    if (!U || !U_next || !Y_a || !Y_b) return set_error(TK_ERR_ARG, "U/U_next/Y_a/Y_b is null");
    for (int t = 0; t < N; ++t)
        if (t != N - 2 && !U[t]) return set_error(TK_ERR_ARG, "U[%d] is null", t);
    if ((st = pending_error())) return st;
    hipStream_t s = (hipStream_t)stream;
    if ((st = memo_build(ctx, s))) return st;
    if (ctx->memo.state != 1)
        return set_error(TK_ERR_UNSUPPORTED, "shared sums need order >= 4 and the fiber kernel on mode N-2");
    for (int t = 0; t < N; ++t)
        if (t != N - 2 && (st = convert_factor(ctx, t, U[t], s))) return st;
    if ((st = memo_first_run(ctx, Y_a, s))) return st;
    if ((st = convert_factor(ctx, N - 2, U_next, s))) return st;
    st = memo_last_run(ctx, Y_b, s);
    ctx->last_stream = s;
    return st;
}

int qrp_update(tk_ctx* ctx, int mode, const void* Y, double* U_out, int32_t* piv, void* stream) {
    int st = check_ctx(ctx);
    if (st || (st = check_mode(ctx, mode))) return st;
    if (!Y || !U_out) return set_error(TK_ERR_ARG, "Y/U_out is null");
    if ((st = pending_error())) return st;
    hipStream_t s = (hipStream_t)stream;
    st = qrp_run(ctx, mode, Y, U_out, piv, s);
    ctx->last_stream = s;
    return st;
}

int svd_update(tk_ctx* ctx, int mode, const void* Y, double* U_out, void* stream) {
    int st = check_ctx(ctx);
    if (st || (st = check_mode(ctx, mode))) return st;
    if (!Y || !U_out) return set_error(TK_ERR_ARG, "Y/U_out is null");
    if ((st = pending_error())) return st;
    hipStream_t s = (hipStream_t)stream;
    st = svd_run(ctx, mode, Y, U_out, s);
    ctx->last_stream = s;
    return st;
}

int tucker_ttmc_kernel(int order, const int64_t* dims, const int32_t* ranks, int dtype, int mode, int* kernel) {
    if (order < 2 || order > kMaxOrder) return set_error(TK_ERR_ARG, "order %d outside [2, %d]", order, kMaxOrder);
    if (!dims || !ranks || !kernel) return set_error(TK_ERR_ARG, "dims/ranks/kernel is null");
    if (dtype != TK_F64 && dtype != TK_F32 && dtype != TK_BF16) return set_error(TK_ERR_ARG, "unknown dtype %d", dtype);
    if (mode < 0 || mode >= order) return set_error(TK_ERR_ARG, "mode %d outside [0, %d)", mode, order);
    for (int t = 0; t < order; ++t)
        if (dims[t] < 1 || ranks[t] < 1) return set_error(TK_ERR_ARG, "dims and ranks must be positive");
    *kernel = ttmc_kernel_for(order, dims, ranks, dtype, mode);
    return TK_OK;
}

int tucker_qrp_gaps(tk_ctx* ctx, int mode, double* gaps) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (mode < 0 || mode >= ctx->N) return set_error(TK_ERR_ARG, "mode %d outside [0, %d)", mode, ctx->N);
    if (!gaps) return set_error(TK_ERR_ARG, "gaps is null");
    if ((st = pending_error())) return st;
    hipStream_t s = ctx->last_stream;
    const int R = ctx->ranks[mode];
    const int n = std::min(R, kGramMaxR);
    TK_HIP(hipMemcpyAsync(gaps, ctx->qrp_gaps + (size_t)mode * kGramMaxR, (size_t)n * sizeof(double),
                          hipMemcpyDeviceToHost, s));
    TK_HIP(hipStreamSynchronize(s));
    for (int j = n; j < R; ++j) gaps[j] = NAN;
    return TK_OK;
}

int tucker_svd_info(const tk_ctx* ctx, int* outer_steps) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!outer_steps) return set_error(TK_ERR_ARG, "outer_steps is null");
    *outer_steps = ctx->eig_outer;
    return TK_OK;
}

int core_fit(tk_ctx* ctx, const void* Y_last, const double* U_last, double* G, double* fit, void* stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!Y_last || !U_last || !G) return set_error(TK_ERR_ARG, "Y_last/U_last/G is null");
    if ((st = pending_error())) return st;
    hipStream_t s = (hipStream_t)stream;
    st = core_run(ctx, Y_last, U_last, G, fit, s);
    ctx->last_stream = s;
    return st;
}

int core_fit_static(int ytype, int64_t I, int32_t R, int64_t K, const void* Y_last, const double* U_last,
                    double normx2, double* G, double* fit, void* stream) {
    if (ytype != TK_F64 && ytype != TK_F32) return set_error(TK_ERR_ARG, "ytype must be TK_F64 or TK_F32");
    if (I < 1 || R < 1 || K < 1) return set_error(TK_ERR_ARG, "I, R and K must be positive");
    if (!Y_last || !U_last || !G) return set_error(TK_ERR_ARG, "Y_last/U_last/G is null");
    if (!(normx2 >= 0.0) || !std::isfinite(normx2)) return set_error(TK_ERR_ARG, "normx2 must be finite and >= 0");
    if ((int64_t)R * K > core_static_max_cols())
        return set_error(TK_ERR_UNSUPPORTED, "R * K = %lld exceeds the static scratch of %lld doubles",
                         (long long)((int64_t)R * K), (long long)core_static_max_cols());
    int st = pending_error();
    if (st) return st;
    return core_static_run(ytype, I, R, K, Y_last, U_last, normx2, G, fit, (hipStream_t)stream);
}

int hosvd_init(tk_ctx* ctx, const double* const* Omega, double* const* U_out, int use_svd, void* stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!Omega || !U_out) return set_error(TK_ERR_ARG, "Omega/U_out is null");
    for (int t = 0; t < ctx->N; ++t) {
        if (!Omega[t]) return set_error(TK_ERR_ARG, "Omega[%d] is null", t);
        if (!U_out[t]) return set_error(TK_ERR_ARG, "U_out[%d] is null", t);
        for (int k = 0; k < ctx->N; ++k)
            if ((const double*)U_out[t] == Omega[k]) return set_error(TK_ERR_ARG, "U_out[%d] aliases Omega[%d]", t, k);
    }
    if ((st = pending_error())) return st;
    hipStream_t s = (hipStream_t)stream;
    // every mode sketches with the caller's test factors only (not with the modes already done)
    for (int n = 0; n < ctx->N; ++n) {
        for (int t = 0; t < ctx->N; ++t)
            if (t != n && (st = convert_factor(ctx, t, Omega[t], s))) return st;
        if ((st = ttmc_run(ctx, n, ctx->ws.y, s))) return st;
        st = use_svd ? svd_run(ctx, n, ctx->ws.y, U_out[n], s) : qrp_run(ctx, n, ctx->ws.y, U_out[n], nullptr, s);
        if (st) return st;
    }
    ctx->last_stream = s;
    return TK_OK;
}

int hooi_sweep(tk_ctx* ctx, double* const* U, double* G, double* fit_dev, double* fit_host, void* stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (!U || !G) return set_error(TK_ERR_ARG, "U/G is null");
    for (int t = 0; t < ctx->N; ++t)
        if (!U[t]) return set_error(TK_ERR_ARG, "U[%d] is null", t);
    if ((st = pending_error())) return st;
    hipStream_t s = (hipStream_t)stream;
    // mode 0 reads U_1..U_{N-1}; U_0's copy is rewritten by its own QRP before any later use
    for (int t = 1; t < ctx->N; ++t)
        if ((st = convert_factor(ctx, t, U[t], s))) return st;
    double* fit = (fit_dev || !fit_host) ? fit_dev : ctx->ws.scal;
    // events: [ttmc start, ttmc end = qrp start] per mode, then qrp end of the last mode, core end,
    // then [main TTMc kernel start, end] per mode
    const int N = ctx->N;
    hipEvent_t* ev = nullptr;
    if (ctx->prof_ev && ctx->prof_used < ctx->prof_cap)
        ev = ctx->prof_ev + (size_t)(ctx->prof_used++) * (4 * N + 2);
    // modes N-2 and N-1 share the fiber sums of the first N-2 modes when the fibers of mode N-2
    // hold 4 or more nonzeros on average
    bool memo = false;
    if (N >= 4 && !(ctx->flags & TK_FLAG_NO_MEMO)) {
        if ((st = memo_build(ctx, s))) return st;
        memo = ctx->memo.state == 1 && ctx->memo.npieces * 4 <= ctx->mode[N - 2].P;
    }
    for (int n = 0; n < ctx->N; ++n) {
        if (ev) TK_HIP(hipEventRecord(ev[2 * n], s));
        hipEvent_t* evm = ev ? ev + 2 * N + 2 + 2 * n : nullptr;
        if (memo && n == N - 2) st = memo_first_run(ctx, ctx->ws.y, s, evm);
        else if (memo && n == N - 1) st = memo_last_run(ctx, ctx->ws.y, s, evm);
        else st = ttmc_run(ctx, n, ctx->ws.y, s, evm);
        if (st) return st;
        if (ev) TK_HIP(hipEventRecord(ev[2 * n + 1], s));
        st = (ctx->flags & TK_FLAG_SVD) ? svd_run(ctx, n, ctx->ws.y, U[n], s)
                                        : qrp_run(ctx, n, ctx->ws.y, U[n], nullptr, s);
        if (st) return st;
    }
    if (ev) TK_HIP(hipEventRecord(ev[2 * ctx->N], s));
    if ((st = core_run(ctx, ctx->ws.y, U[ctx->N - 1], G, fit, s))) return st;
    if (ev) TK_HIP(hipEventRecord(ev[2 * ctx->N + 1], s));
    ctx->last_stream = s;
    if (fit_host) {
        TK_HIP(hipMemcpyAsync(fit_host, fit, 8, hipMemcpyDeviceToHost, s));
        TK_HIP(hipStreamSynchronize(s));
    }
    return TK_OK;
}

int hooi_run(tk_ctx* ctx, double* const* U, double* G, int max_sweeps, double tol, double* fits_host,
             int* sweeps_done, void* stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (max_sweeps < 1) return set_error(TK_ERR_ARG, "max_sweeps %d < 1", max_sweeps);
    if (!(tol >= 0.0)) return set_error(TK_ERR_ARG, "tol must be >= 0");
    if (sweeps_done) *sweeps_done = 0;
    double prev = 0.0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        double f = 0.0;
        if ((st = hooi_sweep(ctx, U, G, nullptr, &f, stream))) return st;
        if (fits_host) fits_host[sw] = f;
        if (sweeps_done) *sweeps_done = sw + 1;
        if (sw >= 1 && fabs(f - prev) <= tol) break;
        prev = f;
    }
    return TK_OK;
}

int reconstruct(tk_ctx* ctx, const double* G, const double* const* U, int64_t m, const int32_t* coords,
                double* out, void* stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (m < 0) return set_error(TK_ERR_ARG, "negative m");
    if (m > 0 && (!G || !U || !coords || !out)) return set_error(TK_ERR_ARG, "null argument");
    for (int t = 0; m > 0 && t < ctx->N; ++t)
        if (!U[t]) return set_error(TK_ERR_ARG, "U[%d] is null", t);
    if ((st = pending_error())) return st;
    hipStream_t s = (hipStream_t)stream;
    st = reconstruct_run(ctx, G, U, m, coords, out, s);
    ctx->last_stream = s;
    return st;
}

int ttmc_adjoint(tk_ctx* ctx, int dtype, const void* G, const void* const* U, void* loss, void* gG,
                 void* const* gU, void* stream) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (ctx->dtype == TK_BF16) return set_error(TK_ERR_UNSUPPORTED, "ttmc_adjoint needs an FP32 or FP64 context");
    if (dtype != ctx->dtype)
        return set_error(TK_ERR_ARG, "dtype %d differs from the context's TTMc type %d", dtype, ctx->dtype);
    if (!G || !U || !loss || !gG || !gU) return set_error(TK_ERR_ARG, "null argument");
    for (int t = 0; t < ctx->N; ++t)
        if (!U[t] || !gU[t]) return set_error(TK_ERR_ARG, "U[%d] or gU[%d] is null", t, t);
    if ((st = pending_error())) return st;
    hipStream_t s = (hipStream_t)stream;
    st = adjoint_run(ctx, G, U, loss, gG, gU, s);
    ctx->last_stream = s;
    return st;
}

int tucker_profile(tk_ctx* ctx, int capacity) {
    int st = check_ctx(ctx);
    if (st) return st;
    if (capacity < 0) return set_error(TK_ERR_ARG, "negative capacity");
    if (ctx->last_stream || ctx->prof_ev) (void)hipStreamSynchronize(ctx->last_stream);
    free_events(ctx);
    if (capacity == 0) return TK_OK;
    const int per = 4 * ctx->N + 2;
    ctx->prof_ev = new hipEvent_t[(size_t)capacity * per]();
    ctx->prof_cap = capacity;
    for (int i = 0; i < capacity * per; ++i) TK_HIP(hipEventCreate(&ctx->prof_ev[i]));
    return TK_OK;
}

int tucker_profile_read(tk_ctx* ctx, double* ttmc_ms, double* ttmc_kernel_ms, double* qrp_ms, double* core_ms,
                        int64_t* sweeps) {
    int st = check_ctx(ctx);
    if (st) return st;
    const int N = ctx->N, per = 4 * N + 2;
    double tt[kMaxOrder] = {}, tk_[kMaxOrder] = {}, qq[kMaxOrder] = {}, cc = 0.0;
    for (int k = 0; k < ctx->prof_used; ++k) {
        hipEvent_t* ev = ctx->prof_ev + (size_t)k * per;
        TK_HIP(hipEventSynchronize(ev[2 * N + 1]));   // core end: the last event a sweep records
        float ms = 0.f;
        for (int n = 0; n < N; ++n) {
            TK_HIP(hipEventElapsedTime(&ms, ev[2 * n], ev[2 * n + 1]));
            tt[n] += ms;
            TK_HIP(hipEventElapsedTime(&ms, ev[2 * n + 1], (n + 1 < N) ? ev[2 * n + 2] : ev[2 * N]));
            qq[n] += ms;
            TK_HIP(hipEventElapsedTime(&ms, ev[2 * N + 2 + 2 * n], ev[2 * N + 3 + 2 * n]));
            tk_[n] += ms;
        }
        TK_HIP(hipEventElapsedTime(&ms, ev[2 * N], ev[2 * N + 1]));
        cc += ms;
    }
    for (int n = 0; n < N; ++n) {
        if (ttmc_ms) ttmc_ms[n] = tt[n];
        if (ttmc_kernel_ms) ttmc_kernel_ms[n] = tk_[n];
        if (qrp_ms) qrp_ms[n] = qq[n];
    }
    if (core_ms) *core_ms = cc;
    if (sweeps) *sweeps = ctx->prof_used;
    return TK_OK;
}

void tucker_free(tk_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->last_stream);
    free_ctx(ctx);
}

}  // extern "C"
