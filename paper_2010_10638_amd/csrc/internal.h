// Internal declarations shared by the library's translation units (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/sptucker.h"

namespace tk {

constexpr int kMaxOrder = TK_MAX_ORDER;
constexpr int kMaxK = TK_MAX_KCOLS;
#ifndef TK_CHUNK_WAVES_PER_CU
#define TK_CHUNK_WAVES_PER_CU 16
#endif
// TTMc work split: pieces of the nonzero stream per compute unit (one wave each)
constexpr int kChunkWavesPerCU = TK_CHUNK_WAVES_PER_CU;
constexpr int kPadR = 16;          // factor copies are padded to a multiple of 16 columns
constexpr int kGramMaxR = 32;      // Gram/Cholesky QRP route handles R_n up to this

// bf16 storage (upper half of an IEEE binary32)
typedef uint16_t bf16_t;

__host__ __device__ inline float bf16_to_f32(bf16_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __uint_as_float(((uint32_t)b) << 16);
#else
    uint32_t u = ((uint32_t)b) << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
#endif
}

// Round to nearest, ties to even (NaN kept quiet).
__host__ __device__ inline bf16_t f32_to_bf16(float f) {
    uint32_t u;
#if defined(__HIP_DEVICE_COMPILE__)
    u = __float_as_uint(f);
#else
    __builtin_memcpy(&u, &f, 4);
#endif
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (bf16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}

inline int pad_rank(int R) { return (R + kPadR - 1) / kPadR * kPadR; }
inline size_t dtype_size(int dt) { return dt == TK_F64 ? 8 : (dt == TK_F32 ? 4 : 2); }
inline size_t ytype_size(int dt) { return dt == TK_F64 ? 8 : 4; }

// Per-mode sorted layout and the chunk walk of the TTMc kernels.
// The sorted nonzeros of a mode are stored padded: row s occupies [pptr[s], pptr[s+1]), its
// ptr[s+1]-ptr[s] nonzeros followed by zero-valued entries (at the indices of the row's last
// nonzero) up to a multiple of 4, so that a 4-nonzero MFMA step never spans two rows.  Bit 31 of the first other-mode index marks the first
// entry of every row (kFirstOfRow); readers mask it off.
constexpr uint32_t kFirstOfRow = 0x80000000u;
constexpr int32_t kIndexMask = 0x7fffffff;

struct ModeLayout {
    int64_t S = 0;                  // distinct i_n
    int32_t* rows = nullptr;        // [S]      distinct i_n, ascending
    int32_t* ptr = nullptr;         // [S + 1]  row pointers into the unpadded order
    int32_t* pptr = nullptr;        // [S + 1]  row pointers into the padded stream (multiples of 4)
    int64_t P = 0;                  // padded stream length
    int32_t* idx = nullptr;         // [(N-1) * P] other-mode indices, modes ascending, SoA (padded)
    void* val = nullptr;            // [P] TTMc storage type (padded)
    int64_t K = 0;                  // prod_{t != n} R_t
    int others[kMaxOrder - 1];      // other modes, ascending
    int fiber_slot = -1;            // position of the fiber mode in others (order >= 4), else -1
    // chunk walk
    int64_t nchunks = 0;
    int32_t* chunk_ptr = nullptr;   // [nchunks + 1] first padded entry of each chunk (multiples of 4)
    int32_t* chunk_row = nullptr;   // [nchunks] compressed row holding the chunk's first nonzero
    int32_t* chunk_slot = nullptr;  // [nchunks] carry slot of a chunk that starts inside a row, else -1
    int64_t ncarry = 0;             // number of carry slots
    int64_t nsplit = 0;             // rows whose nonzeros span several chunks
    int32_t* split = nullptr;       // [nsplit * 3]: compressed row, first slot, last slot
    int32_t max_row_nnz = 0;
    // QRP route for this mode
    int qrp_route = 0;              // 0 = Gram/Cholesky, 1 = small Householder on Y, 2 = fat (Y Y^T)
};

struct Workspace {
    void* y = nullptr;              // Y_(n) of the sweep, max_n I_n * K_n entries of the Y type
    size_t y_bytes = 0;
    void* carry = nullptr;          // carry rows of split rows, max_n ncarry * K_n
    size_t carry_bytes = 0;
    double* qrp = nullptr;          // QRP / core scratch (FP64)
    size_t qrp_bytes = 0;
    int32_t* qrp_int = nullptr;     // pivots, flags
    size_t qrp_int_bytes = 0;
    double* scal = nullptr;         // small device scalars (fit when the caller gives none)
};

// pivot gaps of the last QRP of each mode: [N][kGramMaxR] relative gaps (NaN: not recorded)

// Completion (adjoint TTMc) workspace, allocated on the first ttmc_adjoint call
struct CompletionWs {
    bool ready = false;
    bool fused = false;              // residuals computed inside the TTMc (order 3, FP32): no e, e2, maps
    int32_t* rowid[kMaxOrder] = {};  // per mode: compressed row of every padded position
    void* e = nullptr;               // residuals on mode 0's padded stream (parameter type)
    void* e2 = nullptr;              // the same residuals on mode n's padded stream, n >= 1
    int32_t* map[kMaxOrder] = {};    // n >= 1: mode-0 padded position of every padded position of mode n (-1: pad)
    void* W = nullptr;               // U_n G_(n), max_n I_n x K_n (fused: max_n I_n x 256, 16 x 16 blocks)
    void* Gn = nullptr;              // mode-n unfolding of the core
    double* part = nullptr;          // loss and core-gradient partials
};

// Shared partial sums of the last two modes (order >= 4), built on first use by a sweep
struct MemoWs {
    int state = 0;                   // 0 not built, 1 built, -1 not applicable to the context
    int64_t npieces = 0;             // fiber pieces of mode N-2 (fibers cut by chunk starts)
    int Ks = 0;                      // inner columns: prod_{k < N-2} R_k
    int nsplit = 1;                  // waves per row of mode N-1
    int32_t* pid_base = nullptr;     // [nchunks of mode N-2] first piece of each chunk
    int32_t* pj = nullptr;           // [npieces] i_{N-2} of each piece, in perm order
    int32_t* perm = nullptr;         // [npieces] pieces ordered by i_{N-1} (stream order within)
    int32_t* rptr = nullptr;         // [I_{N-1} + 1] first position of each i_{N-1} in perm
    void* T = nullptr;               // [npieces][Ks] inner sums, TTMc arithmetic type
    void* part = nullptr;            // [I_{N-1}][nsplit][K_{N-1}] partial rows (nsplit > 1)
};

}  // namespace tk

struct tk_ctx {
    int N = 0;
    int dtype = TK_F64;
    uint32_t flags = 0;
    int64_t dims[tk::kMaxOrder] = {};
    int32_t ranks[tk::kMaxOrder] = {};
    int64_t nnz = 0;                 // distinct coordinates
    double normx2 = 0.0;
    tk::ModeLayout mode[tk::kMaxOrder];
    void* Ulp[tk::kMaxOrder] = {};   // factor copies in TTMc precision, I_k x ldU[k]
    int ldU[tk::kMaxOrder] = {};
    tk::Workspace ws;
    double* qrp_gaps = nullptr;      // [N * kGramMaxR] relative pivot gaps of each mode's last QRP
    tk::CompletionWs cws;
    tk::MemoWs memo;
    // SVD factor update: rocBLAS handle and eigen-solver workspace (allocated on first use)
    void* rb = nullptr;
    double* svd_d = nullptr;         // eigenvalues, TK_MAX_KCOLS
    double* svd_e = nullptr;         // off-diagonal workspace, TK_MAX_KCOLS
    int32_t* svd_info = nullptr;
    double* eig_ws = nullptr;        // one-workgroup eigensolver: blocks, eigenpairs, status
    int eig_outer = -1;              // its outer steps in the last SVD update (-1: library solver)
    hipStream_t last_stream = nullptr;
    int device = 0;
    int ncu = 0;                     // compute units of the device
    // region timing of hooi_sweep (tucker_profile)
    hipEvent_t* prof_ev = nullptr;   // [capacity][4N + 2]
    int prof_cap = 0;
    int prof_used = 0;
};

namespace tk {

int set_error(int code, const char* fmt, ...);
int hip_error(hipError_t e, const char* what);

#define TK_HIP(call)                                                  \
    do {                                                              \
        hipError_t e_ = (call);                                       \
        if (e_ != hipSuccess) return ::tk::hip_error(e_, #call);      \
    } while (0)

#define TK_LAUNCH_CHECK(what)                                         \
    do {                                                              \
        hipError_t e_ = hipGetLastError();                            \
        if (e_ != hipSuccess) return ::tk::hip_error(e_, what);       \
    } while (0)

// value of v in lane src (src wave-uniform), through two v_readlane (no LDS round trip)
__device__ inline double wave_bcast(double v, int src) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// sum_{k < cnt} p[k * stride], added in k order; the loads are issued eight at a time so they
// overlap (the order of the additions, hence the result, is that of the plain loop)
__device__ inline double sum_strided(const double* __restrict__ p, int cnt, int64_t stride) {
    double s = 0.0;
    int k = 0;
    for (; k + 8 <= cnt; k += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(k + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; k < cnt; ++k) s += p[(int64_t)k * stride];
    return s;
}

// Layout builder (build.hip)
int build_layout(tk_ctx* ctx, const int32_t* coords, const double* vals, int64_t nnz_in,
                 hipStream_t s);
// unpadded, flag-free copy of one mode's indices and values (tucker_get_csf)
int export_layout(tk_ctx* ctx, int mode, int32_t* idx_out, void* val_out, hipStream_t s);

// Conversions (core.hip)
int convert_factor(tk_ctx* ctx, int k, const double* U, hipStream_t s);
int fill_zero(void* p, size_t bytes, hipStream_t s);
int fill_f64(double* p, int64_t n, double v, hipStream_t s);   // a kernel, not a memset (graph-safe)

// TTMc (ttmc.hip): uses ctx->Ulp copies
// ev_main (optional, [2]): events recorded on s around the main TTMc kernel (fix-up excluded);
// val (optional): values on the mode's padded stream to use instead of the tensor's (same type)
// memo, pid_base (optional, fiber kernel only): also write the inner sum of every fiber piece to
// memo[piece][Ks] (pieces in stream order from pid_base[chunk])
int ttmc_run(tk_ctx* ctx, int mode, void* Y, hipStream_t s, hipEvent_t* ev_main = nullptr,
             const void* val = nullptr, void* memo = nullptr, const int32_t* pid_base = nullptr);
// columns of the factor copy of mode t (16, a multiple of 16 above, or 8 for order >= 4 with
// every rank <= 8) and the TTMc kernel a mode runs (enum tk_ttmc_kernel); host-only
int factor_ld(int N, const int32_t* ranks, int t);
int ttmc_kernel_for(int N, const int64_t* dims, const int32_t* ranks, int dtype, int mode);
// TTMc of mode n over the residuals e = xhat - x of the entries (padding: 0), xhat from W = the
// mode's rows of U_n G_(n) as zero-padded 16 x 16 blocks ([I_n][256], FP32); part (optional, one
// per chunk) receives the chunk's sum of e^2.  Order 3, FP32 context, the order-3 MFMA kernel only
// (ttmc_residual_form).
bool ttmc_residual_form(const tk_ctx* ctx, int mode);
int ttmc_residual_run(tk_ctx* ctx, int mode, void* Y, const float* W, double* part, hipStream_t s);
// Completion (completion.hip): loss and gradients over the context's entries, parameters in the
// context's TTMc type (FP32 or FP64)
int adjoint_run(tk_ctx* ctx, const void* G, const void* const* U, void* loss, void* gG, void* const* gU,
                hipStream_t s);
void free_completion_ws(tk_ctx* ctx);
// Shared partial sums of modes N-2 and N-1 (memo.hip): applicability, the layout (built once;
// state -1 when not applicable), mode N-2's TTMc that also writes the fiber sums, and mode N-1's
// TTMc from them with the current copy of U_{N-2}
bool memo_applicable(const tk_ctx* ctx);
int memo_build(tk_ctx* ctx, hipStream_t s);
void free_memo(tk_ctx* ctx);
int memo_first_run(tk_ctx* ctx, void* Y, hipStream_t s, hipEvent_t* ev_main = nullptr);
int memo_last_run(tk_ctx* ctx, void* Y, hipStream_t s, hipEvent_t* ev_main = nullptr);

// QRP (qrp.hip): Y -> U (FP64) and the low-precision copy ctx->Ulp[mode]
int qrp_run(tk_ctx* ctx, int mode, const void* Y, double* U, int32_t* piv, hipStream_t s);
// FP64 Y^T Y (tall) or Y Y^T (fat) of a mode in the QRP workspace: *A (n x n, full), *n
int gram_run(tk_ctx* ctx, int mode, const void* Y, double** A, int* n, hipStream_t s);
// SVD factor update (svd.hip): U <- leading R_n left singular vectors of Y_(n)
int svd_run(tk_ctx* ctx, int mode, const void* Y, double* U, hipStream_t s);
void free_svd_ws(tk_ctx* ctx);
size_t qrp_workspace_bytes(const tk_ctx* ctx, int mode);
int qrp_route(const tk_ctx* ctx, int mode);

// Core, fit, reconstruct (core.hip)
int core_run(tk_ctx* ctx, const void* Y, const double* U, double* G, double* fit, hipStream_t s);
size_t core_workspace_bytes(const tk_ctx* ctx);
// allocation-free core and fit on the library's static per-device scratch (R * K <= the returned bound)
int core_static_run(int ytype, int64_t I, int R, int64_t K, const void* Y, const double* U, double normx2,
                    double* G, double* fit, hipStream_t s);
int64_t core_static_max_cols();
int reconstruct_run(tk_ctx* ctx, const double* G, const double* const* U, int64_t m,
                    const int32_t* coords, double* out, hipStream_t s);

}  // namespace tk
