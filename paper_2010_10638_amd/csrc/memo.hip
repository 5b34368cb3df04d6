// TTMc of the last two modes with shared partial Kronecker sums (order >= 4).
//
// The reuse the method rests on (Sec. III-C: a Kronecker product is formed once for all nonzeros
// that share its indices) carried across two modes of a sweep.  Mode m = N-2 runs the fiber
// kernel with fiber mode N-1: for each fiber (i_m, i_{N-1}) it forms the inner sum
//   T(i_m, i_{N-1}, :) = sum_{nonzeros of the fiber} x kron_{k < N-2} U_k(i_k, :)      (Ks columns)
// and folds it with U_{N-1}(i_{N-1}, :) into Y_(m).  Mode N-1 needs the same inner sums folded the
// other way:
//   Y_(N-1)(i_{N-1}, c R_{N-2} + r) = sum_{i_m} T(i_m, i_{N-1}, c) U_{N-2}(i_m, r),
// a sum over fibers instead of nonzeros.  In a HOOI sweep the two modes are consecutive and only
// U_{N-2} changes between them (its own factor update), which this product takes in its new
// value; U_0..U_{N-3}, inside T, are unchanged.  So the fiber kernel of mode N-2 also writes T,
// one row per fiber piece (a fiber, or its part inside one chunk of the walk, numbered in stream
// order), and mode N-1's TTMc reads the pieces grouped by i_{N-1}.
//
// Layout, built at the first use: per chunk of mode N-2 the number of its first piece, per piece
// its i_{N-2}, and the pieces sorted by i_{N-1} (stable: stream order within) with row pointers.
// The product runs one wave per (row of mode N-1, split of its pieces): lane l owns inner columns
// l + 64 j and keeps the R_{N-2} sums of each; the splits' partial rows are added in split order,
// so the result is deterministic.
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "internal.h"

namespace tk {

namespace {

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

struct Tmp {
    void* p = nullptr;
    ~Tmp() { if (p) (void)hipFree(p); }
};

int dev_alloc(void** p, size_t bytes) {
    if (hipMalloc(p, std::max<size_t>(bytes, 16)) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return set_error(TK_ERR_OOM, "shared-sum TTMc: allocation of %zu bytes failed", bytes);
    }
    return TK_OK;
}

// flag[q] = 1 where a piece starts: the first entry, a row start, or a new fiber index
__global__ void k_piece_flags(const int32_t* __restrict__ idx0, const int32_t* __restrict__ fib, int64_t P,
                              int32_t* __restrict__ flag) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P) return;
    flag[q] = (q == 0 || idx0[q] < 0 || fib[q] != fib[q - 1]) ? 1 : 0;
}

// ... and where a chunk of the walk starts
__global__ void k_piece_chunks(const int32_t* __restrict__ chunk_ptr, int64_t nchunks, int64_t P,
                               int32_t* __restrict__ flag) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nchunks && chunk_ptr[c] < P) flag[chunk_ptr[c]] = 1;
}

// per piece: its i_{N-1} (sort key) and i_{N-2} (compressed row of the start, by binary search of
// the padded row pointers); per chunk: the number of its first piece
__global__ void k_piece_table(const int32_t* __restrict__ flag, const int32_t* __restrict__ pid,
                              const int32_t* __restrict__ fib, const int32_t* __restrict__ pptr,
                              const int32_t* __restrict__ rows, int64_t S, int64_t P, int32_t* __restrict__ key,
                              int32_t* __restrict__ pj, int32_t* __restrict__ iota) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= P || !flag[q]) return;
    int64_t lo = 0, hi = S - 1;   // largest s with pptr[s] <= q
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (pptr[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    const int32_t p = pid[q];
    key[p] = fib[q];
    pj[p] = rows[lo];
    iota[p] = p;
}

__global__ void k_chunk_base(const int32_t* __restrict__ chunk_ptr, const int32_t* __restrict__ pid,
                             int64_t nchunks, int64_t P, int32_t* __restrict__ base) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nchunks) base[c] = (chunk_ptr[c] < P) ? pid[chunk_ptr[c]] : 0;   // an empty chunk writes nothing
}

// pjs[k] = pj[perm[k]]: the i_{N-2} of the pieces in sorted order (one dependent load fewer)
__global__ void k_permute_pj(const int32_t* __restrict__ pj, const int32_t* __restrict__ perm, int64_t n,
                             int32_t* __restrict__ pjs) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) pjs[k] = pj[perm[k]];
}

// rptr[i] = first position of key i in the sorted keys (i = 0..I)
__global__ void k_key_ptr(const int32_t* __restrict__ sorted, int64_t n, int64_t I, int32_t* __restrict__ rptr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > I) return;
    int64_t lo = 0, hi = n;   // first k with sorted[k] >= i
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (sorted[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    rptr[i] = (int32_t)lo;
}

struct MemoRowArgs {
    const int32_t* perm;
    const int32_t* rptr;
    const int32_t* pj;   // i_{N-2} of the pieces in perm order
    const void* T;       // [pieces][Ks], arithmetic type
    const void* U;       // U_{N-2} copy, I x ld, storage type
    int32_t ld, R, Ks, nsplit;
    int64_t K;           // Ks * R
    void* out;           // Y (nsplit == 1) or the partial rows [I][nsplit][K]
};

template <typename AT, typename ST> __device__ inline AT to_at(const ST* p, int64_t i) {
    if constexpr (sizeof(ST) == 2) return (AT)bf16_to_f32(p[i]);
    else return (AT)p[i];
}

// one wave per (row, split); lane l owns inner columns l + 64 j (j < KSL), with R <= RF sums each.
// Pieces are taken eight at a time: their numbers, rows of U and rows of T are all requested
// before the products (a piece alone is a chain of three dependent loads).
constexpr int kMemoGroup = 8;

template <typename AT, typename ST, int KSL, int RF>
__global__ __launch_bounds__(64) void k_memo_rows(MemoRowArgs a) {
    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    const int sp = blockIdx.y;
    const int b0 = a.rptr[i], b1 = a.rptr[i + 1];
    const int len = (b1 - b0 + a.nsplit - 1) / a.nsplit;
    const int lo = min(b1, b0 + sp * len), hi = min(b1, lo + len);
    const AT* __restrict__ T = (const AT*)a.T;
    const ST* __restrict__ U = (const ST*)a.U;
    AT acc[KSL][RF];
#pragma unroll
    for (int j = 0; j < KSL; ++j)
#pragma unroll
        for (int r = 0; r < RF; ++r) acc[j][r] = AT(0);
    for (int k0 = lo; k0 < hi; k0 += kMemoGroup) {
        int p[kMemoGroup];
#pragma unroll
        for (int g = 0; g < kMemoGroup; ++g) p[g] = a.perm[min(k0 + g, hi - 1)];
        AT u[kMemoGroup][RF], t[kMemoGroup][KSL];
#pragma unroll
        for (int g = 0; g < kMemoGroup; ++g) {
            const bool live = k0 + g < hi;
            const ST* urow = U + (int64_t)a.pj[min(k0 + g, hi - 1)] * a.ld;
            // the factor copy's rows are ld >= RF values, 16-byte aligned: read them whole
            // (columns past R are zero in the copy)
            constexpr int NV = RF * (int)sizeof(ST) / 16;
            ST raw[RF];
#pragma unroll
            for (int v = 0; v < NV; ++v) ((uint4*)raw)[v] = ((const uint4*)urow)[v];
#pragma unroll
            for (int r = 0; r < RF; ++r) u[g][r] = live ? to_at<AT, ST>(raw, r) : AT(0);
#pragma unroll
            for (int j = 0; j < KSL; ++j) {
                const int cs = lane + 64 * j;
                t[g][j] = (cs < a.Ks) ? T[(int64_t)p[g] * a.Ks + cs] : AT(0);
            }
        }
        // pieces in order (the sum order of the plain loop)
#pragma unroll
        for (int g = 0; g < kMemoGroup; ++g)
#pragma unroll
            for (int j = 0; j < KSL; ++j)
#pragma unroll
                for (int r = 0; r < RF; ++r) acc[j][r] += t[g][j] * u[g][r];
    }
    AT* dst = (AT*)a.out + ((a.nsplit == 1) ? i * a.K : (i * a.nsplit + sp) * a.K);
#pragma unroll
    for (int j = 0; j < KSL; ++j) {
        const int cs = lane + 64 * j;
        if (cs < a.Ks) {
#pragma unroll
            for (int r = 0; r < RF; ++r)
                if (r < a.R) dst[(int64_t)cs * a.R + r] = acc[j][r];
        }
    }
}

template <typename AT>
__global__ void k_memo_reduce(const AT* __restrict__ part, int64_t I, int nsplit, int64_t K, AT* __restrict__ Y) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= I * K) return;
    const int64_t i = e / K, c = e % K;
    AT v = AT(0);
    for (int sp = 0; sp < nsplit; ++sp) v += part[(i * nsplit + sp) * K + c];
    Y[e] = v;
}

template <typename AT, typename ST, int KSL>
void launch_rows_r(const MemoRowArgs& a, int64_t I, hipStream_t s) {
    dim3 grid((unsigned)I, (unsigned)a.nsplit);
    if (a.R <= 8) k_memo_rows<AT, ST, KSL, 8><<<grid, 64, 0, s>>>(a);
    else k_memo_rows<AT, ST, KSL, 16><<<grid, 64, 0, s>>>(a);
}

template <typename AT, typename ST>
void launch_rows_t(const MemoRowArgs& a, int64_t I, hipStream_t s) {
    const int ksl = (a.Ks + 63) / 64;
    if (ksl <= 1) launch_rows_r<AT, ST, 1>(a, I, s);
    else if (ksl <= 2) launch_rows_r<AT, ST, 2>(a, I, s);
    else if (ksl <= 4) launch_rows_r<AT, ST, 4>(a, I, s);
    else launch_rows_r<AT, ST, 8>(a, I, s);
}

}  // namespace

bool memo_applicable(const tk_ctx* ctx) {
    const int N = ctx->N;
    if (N < 4) return false;
    const int m = N - 2;
    if (ctx->mode[m].nchunks == 0 || ctx->mode[m].fiber_slot != N - 2) return false;
    if (ttmc_kernel_for(N, ctx->dims, ctx->ranks, ctx->dtype, m) != TK_TTMC_FIBER) return false;
    int64_t Ks = 1;
    for (int k = 0; k < N - 2; ++k) Ks *= ctx->ranks[k];
    return Ks <= 512 && ctx->ranks[N - 2] <= 16;
}

int memo_build(tk_ctx* ctx, hipStream_t s) {
    MemoWs& w = ctx->memo;
    if (w.state != 0) return TK_OK;
    free_memo(ctx);   // what an earlier attempt that failed part-way left
    if (!memo_applicable(ctx)) {
        w.state = -1;
        return TK_OK;
    }
    const int N = ctx->N, m = N - 2;
    const ModeLayout& ml = ctx->mode[m];
    const int64_t P = ml.P, I = ctx->dims[N - 1];
    const int32_t* fib = ml.idx + (int64_t)ml.fiber_slot * P;
    Tmp flag, pid, key, keys_sorted, iota, tmp;
    int st;
    if ((st = dev_alloc(&flag.p, (size_t)P * 4)) || (st = dev_alloc(&pid.p, (size_t)P * 4))) return st;
    k_piece_flags<<<cdiv(P, 256), 256, 0, s>>>(ml.idx, fib, P, (int32_t*)flag.p);
    k_piece_chunks<<<cdiv(ml.nchunks, 256), 256, 0, s>>>(ml.chunk_ptr, ml.nchunks, P, (int32_t*)flag.p);
    TK_LAUNCH_CHECK("k_piece_flags");
    size_t scan_bytes = 0;
    TK_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (int32_t*)flag.p, (int32_t*)pid.p, (int)P, s));
    if ((st = dev_alloc(&tmp.p, scan_bytes))) return st;
    TK_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, scan_bytes, (int32_t*)flag.p, (int32_t*)pid.p, (int)P, s));
    int32_t last[2];
    TK_HIP(hipMemcpyAsync(&last[0], (int32_t*)pid.p + (P - 1), 4, hipMemcpyDeviceToHost, s));
    TK_HIP(hipMemcpyAsync(&last[1], (int32_t*)flag.p + (P - 1), 4, hipMemcpyDeviceToHost, s));
    TK_HIP(hipStreamSynchronize(s));
    const int64_t np = (int64_t)last[0] + last[1];
    int64_t Ks = 1;
    for (int k = 0; k < N - 2; ++k) Ks *= ctx->ranks[k];
    const size_t at = ytype_size(ctx->dtype);
    const int64_t K = ctx->mode[N - 1].K;
    const int nsplit = (int)std::max<int64_t>(1, std::min<int64_t>(64, (8192 + I - 1) / I));
    if ((st = dev_alloc((void**)&w.pid_base, (size_t)ml.nchunks * 4)) || (st = dev_alloc((void**)&w.pj, (size_t)np * 4)) ||
        (st = dev_alloc((void**)&w.perm, (size_t)np * 4)) || (st = dev_alloc((void**)&w.rptr, (size_t)(I + 1) * 4)) ||
        (st = dev_alloc(&w.T, (size_t)np * Ks * at)) ||
        (nsplit > 1 && (st = dev_alloc(&w.part, (size_t)I * nsplit * K * at))) ||
        (st = dev_alloc(&key.p, (size_t)np * 4)) || (st = dev_alloc(&keys_sorted.p, (size_t)np * 4)) ||
        (st = dev_alloc(&iota.p, (size_t)np * 4))) {
        free_memo(ctx);
        return st;
    }
    k_chunk_base<<<cdiv(ml.nchunks, 256), 256, 0, s>>>(ml.chunk_ptr, (const int32_t*)pid.p, ml.nchunks, P, w.pid_base);
    k_piece_table<<<cdiv(P, 256), 256, 0, s>>>((const int32_t*)flag.p, (const int32_t*)pid.p, fib, ml.pptr, ml.rows,
                                              ml.S, P, (int32_t*)key.p, w.pj, (int32_t*)iota.p);
    TK_LAUNCH_CHECK("k_piece_table");
    int bits = 1;
    while (bits < 31 && ((I - 1) >> bits) != 0) ++bits;
    size_t sort_bytes = 0;
    TK_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (int32_t*)key.p, (int32_t*)keys_sorted.p,
                                              (int32_t*)iota.p, w.perm, (int)np, 0, bits, s));
    Tmp tmp2;
    if ((st = dev_alloc(&tmp2.p, sort_bytes))) {
        free_memo(ctx);
        return st;
    }
    TK_HIP(hipcub::DeviceRadixSort::SortPairs(tmp2.p, sort_bytes, (int32_t*)key.p, (int32_t*)keys_sorted.p,
                                              (int32_t*)iota.p, w.perm, (int)np, 0, bits, s));
    k_key_ptr<<<cdiv(I + 1, 256), 256, 0, s>>>((const int32_t*)keys_sorted.p, np, I, w.rptr);
    TK_LAUNCH_CHECK("k_key_ptr");
    // the pieces' i_{N-2} in sorted order, over the unsorted table (no longer needed)
    k_permute_pj<<<cdiv(np, 256), 256, 0, s>>>(w.pj, w.perm, np, (int32_t*)key.p);
    TK_LAUNCH_CHECK("k_permute_pj");
    TK_HIP(hipMemcpyAsync(w.pj, key.p, (size_t)np * 4, hipMemcpyDeviceToDevice, s));
    TK_HIP(hipStreamSynchronize(s));   // the temporaries are freed on return
    w.npieces = np;
    w.Ks = (int)Ks;
    w.nsplit = nsplit;
    w.state = 1;
    return TK_OK;
}

void free_memo(tk_ctx* ctx) {
    MemoWs& w = ctx->memo;
    void* ps[] = {w.pid_base, w.pj, w.perm, w.rptr, w.T, w.part};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    w = MemoWs{};
}

int memo_first_run(tk_ctx* ctx, void* Y, hipStream_t s, hipEvent_t* ev_main) {
    MemoWs& w = ctx->memo;
    if (w.state != 1) return set_error(TK_ERR_UNSUPPORTED, "shared-sum TTMc: layout not built");
    return ttmc_run(ctx, ctx->N - 2, Y, s, ev_main, nullptr, w.T, w.pid_base);
}

int memo_last_run(tk_ctx* ctx, void* Y, hipStream_t s, hipEvent_t* ev_main) {
    MemoWs& w = ctx->memo;
    if (w.state != 1) return set_error(TK_ERR_UNSUPPORTED, "shared-sum TTMc: layout not built");
    const int N = ctx->N;
    const int64_t I = ctx->dims[N - 1];
    MemoRowArgs a{};
    a.perm = w.perm;
    a.rptr = w.rptr;
    a.pj = w.pj;
    a.T = w.T;
    a.U = ctx->Ulp[N - 2];
    a.ld = ctx->ldU[N - 2];
    a.R = ctx->ranks[N - 2];
    a.Ks = w.Ks;
    a.nsplit = w.nsplit;
    a.K = ctx->mode[N - 1].K;
    a.out = (w.nsplit == 1) ? Y : w.part;
    if (ev_main) TK_HIP(hipEventRecord(ev_main[0], s));
    if (ctx->dtype == TK_F64) launch_rows_t<double, double>(a, I, s);
    else if (ctx->dtype == TK_F32) launch_rows_t<float, float>(a, I, s);
    else launch_rows_t<float, bf16_t>(a, I, s);
    TK_LAUNCH_CHECK("k_memo_rows");
    if (w.nsplit > 1) {
        if (ctx->dtype == TK_F64)
            k_memo_reduce<double><<<cdiv(I * a.K, 256), 256, 0, s>>>((const double*)w.part, I, w.nsplit, a.K, (double*)Y);
        else
            k_memo_reduce<float><<<cdiv(I * a.K, 256), 256, 0, s>>>((const float*)w.part, I, w.nsplit, a.K, (float*)Y);
        TK_LAUNCH_CHECK("k_memo_reduce");
    }
    if (ev_main) TK_HIP(hipEventRecord(ev_main[1], s));
    return TK_OK;
}

}  // namespace tk
