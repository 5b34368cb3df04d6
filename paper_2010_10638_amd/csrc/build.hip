// Device builder of the per-mode sorted layout: validation, duplicate coalescing, one radix sort
// per mode on a 64-bit composite key, row pointers, and the nonzero chunk table walked by the
// TTMc kernels.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include <cmath>

#include "internal.h"

namespace tk {

namespace {

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

int dalloc(DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return set_error(TK_ERR_OOM, "device allocation of %zu bytes failed", bytes);
    }
    return TK_OK;
}

struct KeySpec {
    const int32_t* col[kMaxOrder];   // coordinate arrays in key order (most significant first)
    int64_t radix[kMaxOrder];        // dims in key order
    int n;
};

__global__ void k_keys_validate(const int32_t* __restrict__ coords, int64_t nnz, int N,
                                KeySpec spec, uint64_t* __restrict__ keys,
                                int32_t* __restrict__ iota, int32_t* __restrict__ bad) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnz) return;
    uint64_t key = 0;
    bool ok = true;
    for (int t = 0; t < N; ++t) {
        int32_t i = coords[(int64_t)t * nnz + p];
        bool in = (i >= 0) && ((int64_t)i < spec.radix[t]);
        ok = ok && in;
        key = key * (uint64_t)spec.radix[t] + (uint64_t)(in ? i : 0);
    }
    keys[p] = key;
    iota[p] = (int32_t)p;
    if (!ok) atomicOr(bad, 1);
}

__global__ void k_keys(int64_t n, KeySpec spec, uint64_t* __restrict__ keys,
                       int32_t* __restrict__ iota) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    uint64_t key = 0;
    for (int t = 0; t < spec.n; ++t) key = key * (uint64_t)spec.radix[t] + (uint64_t)spec.col[t][p];
    keys[p] = key;
    iota[p] = (int32_t)p;
}

__global__ void k_heads64(const uint64_t* __restrict__ keys, int64_t n, int32_t* __restrict__ h) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    h[q] = (q == 0 || keys[q] != keys[q - 1]) ? 1 : 0;
}

__global__ void k_heads32(const int32_t* __restrict__ v, int64_t n, int32_t* __restrict__ h) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    h[q] = (q == 0 || v[q] != v[q - 1]) ? 1 : 0;
}

// One thread per run of equal keys: sums the run's values in sorted (= input, the sort is
// stable) order and writes the distinct entry.
__global__ void k_coalesce(const int32_t* __restrict__ h, const int32_t* __restrict__ pos,
                           const int32_t* __restrict__ perm, int64_t n,
                           const int32_t* __restrict__ coords, const double* __restrict__ vals,
                           int N, int64_t D, int32_t* __restrict__ dcoords,
                           double* __restrict__ dvals) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n || !h[q]) return;
    int32_t src = perm[q];
    double s = vals[src];
    for (int64_t r = q + 1; r < n && !h[r]; ++r) s += vals[perm[r]];
    int64_t d = pos[q];
    dvals[d] = s;
    for (int t = 0; t < N; ++t) dcoords[(int64_t)t * D + d] = coords[(int64_t)t * n + src];
}

// Deterministic sum of squares: fixed grid, fixed per-thread element set, fixed tree.
__global__ void k_sumsq_partial(const double* __restrict__ v, int64_t n, double* __restrict__ part) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        s += v[i] * v[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_final(const double* __restrict__ part, int np, double* __restrict__ out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += 256) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

template <typename ST>
__device__ inline ST store_val(double v);
template <> __device__ inline double store_val<double>(double v) { return v; }
template <> __device__ inline float store_val<float>(double v) { return (float)v; }
template <> __device__ inline bf16_t store_val<bf16_t>(double v) { return f32_to_bf16((float)v); }

struct GatherSpec {
    const int32_t* other[kMaxOrder - 1];
    int nothers;
};

template <typename ST>
__global__ void k_gather_mode(const int32_t* __restrict__ perm, int64_t D,
                              const int32_t* __restrict__ rowsrc, GatherSpec g,
                              const double* __restrict__ dvals, int32_t* __restrict__ rowid,
                              int32_t* __restrict__ idx, ST* __restrict__ val) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= D) return;
    int32_t src = perm[q];
    rowid[q] = rowsrc[src];
    for (int j = 0; j < g.nothers; ++j) idx[(int64_t)j * D + q] = g.other[j][src];
    val[q] = store_val<ST>(dvals[src]);
}

// Scatter the sorted entry q (row s = the number of row heads up to q, minus one) to its padded
// slot pptr[s] + (q - ptr[s]); the first entry of a row gets the kFirstOfRow flag on idx[0].
template <typename ST>
__global__ void k_pad_scatter(const int32_t* __restrict__ h, const int32_t* __restrict__ pos, int64_t D,
                              const int32_t* __restrict__ ptr, const int32_t* __restrict__ pptr, int nothers,
                              const int32_t* __restrict__ idx_u, const ST* __restrict__ val_u, int64_t P,
                              int32_t* __restrict__ idx_p, ST* __restrict__ val_p) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= D) return;
    const int64_t s = pos[q] - (h[q] ? 0 : 1);
    const int64_t d = pptr[s] + (q - ptr[s]);
    for (int j = 0; j < nothers; ++j) {
        int32_t v = idx_u[(int64_t)j * D + q];
        if (j == 0 && h[q]) v = (int32_t)((uint32_t)v | kFirstOfRow);
        idx_p[(int64_t)j * P + d] = v;
    }
    val_p[d] = val_u[q];
    // the row's last nonzero also fills the row's padding: zero values at its own indices, so a
    // pad continues the last fiber of the row and gathers a factor row that is already cached
    if (q == (int64_t)ptr[s + 1] - 1) {
        for (int64_t e = d + 1; e < (int64_t)pptr[s + 1]; ++e) {
            for (int j = 0; j < nothers; ++j)
                idx_p[(int64_t)j * P + e] = idx_u[(int64_t)j * D + q];
            val_p[e] = ST(0);
        }
    }
}

template <typename ST>
__global__ void k_pad_fill(int nothers, int64_t P, int32_t* __restrict__ idx_p, ST* __restrict__ val_p) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P) return;
    for (int j = 0; j < nothers; ++j) idx_p[(int64_t)j * P + e] = 0;
    val_p[e] = ST(0);
}

__global__ void k_rows(const int32_t* __restrict__ h, const int32_t* __restrict__ pos,
                       const int32_t* __restrict__ rowid, int64_t D, int64_t S,
                       int32_t* __restrict__ rows, int32_t* __restrict__ ptr) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) ptr[S] = (int32_t)D;
    if (q >= D || !h[q]) return;
    rows[pos[q]] = rowid[q];
    ptr[pos[q]] = (int32_t)q;
}

inline unsigned blocks_for(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

int key_bits(const int64_t* dims, int N) {
    // number of bits of prod dims - 1
    unsigned __int128 prod = 1;
    for (int t = 0; t < N; ++t) prod *= (unsigned __int128)dims[t];
    unsigned __int128 maxkey = prod - 1;
    int bits = 0;
    while (maxkey > 0) { ++bits; maxkey >>= 1; }
    return std::max(bits, 1);
}

template <typename ST>
int launch_gather(const int32_t* perm, int64_t D, const int32_t* rowsrc, const GatherSpec& g,
                  const double* dvals, int32_t* rowid, int32_t* idx, void* val, hipStream_t s) {
    k_gather_mode<ST><<<blocks_for(D), 256, 0, s>>>(perm, D, rowsrc, g, dvals, rowid, idx, (ST*)val);
    TK_LAUNCH_CHECK("k_gather_mode");
    return TK_OK;
}

// Balanced chunking of the padded stream: C pieces of (nearly) equal length, each a multiple of
// 4 entries, cut anywhere - a piece may start inside a row.  The piece where a row starts owns it
// (writes Y_(n) directly); every later piece holding part of that row is a carrier whose partial
// row sum goes to a carry slot, added to the row by the fix-up pass in slot order.  Equal pieces
// give every wave the same work whatever the row-length distribution (skewed fibers included).
#ifndef TK_ROW_WEIGHT
#define TK_ROW_WEIGHT 32
#endif
constexpr int64_t kRowWeight = TK_ROW_WEIGHT;

void make_chunks(const std::vector<int32_t>& ptr, int64_t C, std::vector<int32_t>& cptr,
                 std::vector<int32_t>& crow, std::vector<int32_t>& cslot,
                 std::vector<int32_t>& split, int64_t& ncarry, int32_t& maxrow) {
    const int64_t S = (int64_t)ptr.size() - 1;
    const int64_t D = ptr[S];
    ncarry = 0;
    maxrow = 0;
    for (int64_t r = 0; r < S; ++r) maxrow = std::max<int32_t>(maxrow, ptr[r + 1] - ptr[r]);
    if (D == 0) {
        cptr.push_back(0);
        return;
    }
    const int64_t quads = D / 4;
    C = std::max<int64_t>(1, std::min<int64_t>(C, quads));
    // pieces of equal work: an entry weighs 1, a row start kRowWeight more (writing a finished row
    // and starting the next costs about that many entries' time), so that pieces full of short
    // rows are not the last to finish
    const double W = (double)D + (double)kRowWeight * (double)S;
    int64_t r = 0;            // row holding the current piece start
    int64_t open_row = -1;    // row with carry slots being collected
    for (int64_t k = 0; k < C; ++k) {
        // first quad boundary q (in row r) with q + kRowWeight * (r + 1) >= W k / C
        const double target = W * (double)k / (double)C;
        int64_t q = 0;
        if (k > 0) {
            while (r < S - 1 && (double)ptr[r + 1] + (double)kRowWeight * (double)(r + 2) <= target) ++r;
            const double qa = target - (double)kRowWeight * (double)(r + 1);
            q = std::max<int64_t>(ptr[r], ((int64_t)std::ceil(qa) + 3) / 4 * 4);
            if (q >= ptr[r + 1]) q = ptr[r + 1];
            if (q >= D) break;
        }
        if (!cptr.empty() && q <= cptr.back()) continue;
        while (ptr[r + 1] <= q) ++r;
        cptr.push_back((int32_t)q);
        crow.push_back((int32_t)r);
        if (ptr[r] == q) {
            cslot.push_back(-1);
        } else {
            if (open_row != r) {
                split.push_back((int32_t)r);
                split.push_back((int32_t)ncarry);
                split.push_back((int32_t)ncarry);
                open_row = r;
            } else {
                split.back() = (int32_t)ncarry;
            }
            cslot.push_back((int32_t)(ncarry++));
        }
    }
    cptr.push_back((int32_t)D);
}

template <typename T>
int upload(T** dst, const std::vector<T>& v, hipStream_t s) {
    size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
    hipError_t e = hipMalloc((void**)dst, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *dst = nullptr;
        return set_error(TK_ERR_OOM, "device allocation of %zu bytes failed", bytes);
    }
    if (!v.empty()) TK_HIP(hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return TK_OK;
}

// Padded entry e -> its unpadded position (row found by binary search of pptr); pads are skipped
// and the row flag is masked off.
template <typename ST>
__global__ void k_export(const int32_t* __restrict__ ptr, const int32_t* __restrict__ pptr, int64_t S, int64_t P,
                         int64_t D, int nothers, const int32_t* __restrict__ idx_p, const ST* __restrict__ val_p,
                         int32_t* __restrict__ idx_out, ST* __restrict__ val_out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P) return;
    int64_t lo = 0, hi = S;  // largest s with pptr[s] <= e
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        if (pptr[mid] <= e) lo = mid; else hi = mid;
    }
    const int64_t off = e - pptr[lo];
    if (off >= (int64_t)ptr[lo + 1] - ptr[lo]) return;
    const int64_t d = ptr[lo] + off;
    for (int j = 0; j < nothers; ++j) idx_out[(int64_t)j * D + d] = idx_p[(int64_t)j * P + e] & kIndexMask;
    val_out[d] = val_p[e];
}

}  // namespace

int export_layout(tk_ctx* ctx, int mode, int32_t* idx_out, void* val_out, hipStream_t s) {
    const ModeLayout& ml = ctx->mode[mode];
    if (ml.P == 0) return TK_OK;
    const unsigned g = blocks_for(ml.P);
    const int no = ctx->N - 1;
    if (ctx->dtype == TK_F64)
        k_export<double><<<g, 256, 0, s>>>(ml.ptr, ml.pptr, ml.S, ml.P, ctx->nnz, no, ml.idx, (const double*)ml.val,
                                           idx_out, (double*)val_out);
    else if (ctx->dtype == TK_F32)
        k_export<float><<<g, 256, 0, s>>>(ml.ptr, ml.pptr, ml.S, ml.P, ctx->nnz, no, ml.idx, (const float*)ml.val,
                                          idx_out, (float*)val_out);
    else
        k_export<bf16_t><<<g, 256, 0, s>>>(ml.ptr, ml.pptr, ml.S, ml.P, ctx->nnz, no, ml.idx, (const bf16_t*)ml.val,
                                           idx_out, (bf16_t*)val_out);
    TK_LAUNCH_CHECK("k_export");
    return TK_OK;
}

int build_layout(tk_ctx* ctx, const int32_t* coords, const double* vals, int64_t n, hipStream_t s) {
    const int N = ctx->N;
    const int bits = key_bits(ctx->dims, N);
    int st;
    DevBuf kin, kout, iin, iout, hbuf, pbuf, bad, tmp, dco, dva, rowid, part;
    size_t nn = (size_t)std::max<int64_t>(n, 1);
    if ((st = dalloc(kin, nn * 8)) || (st = dalloc(kout, nn * 8)) || (st = dalloc(iin, nn * 4)) ||
        (st = dalloc(iout, nn * 4)) || (st = dalloc(hbuf, nn * 4)) || (st = dalloc(pbuf, nn * 4)) ||
        (st = dalloc(bad, 16)) || (st = dalloc(rowid, nn * 4)) || (st = dalloc(part, 1040 * 8)))
        return st;
    size_t sort_bytes = 0, scan_bytes = 0;
    TK_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (uint64_t*)kin.p, (uint64_t*)kout.p,
                                              (int32_t*)iin.p, (int32_t*)iout.p, (int)nn, 0, bits, s));
    TK_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (int32_t*)hbuf.p, (int32_t*)pbuf.p,
                                            (int)nn, s));
    if ((st = dalloc(tmp, std::max(sort_bytes, scan_bytes)))) return st;
    size_t tmp_bytes = std::max(sort_bytes, scan_bytes);

    // 1. validate and key every entry in (i_1, ..., i_N) order
    KeySpec spec{};
    spec.n = N;
    for (int t = 0; t < N; ++t) spec.radix[t] = ctx->dims[t];
    TK_HIP(hipMemsetAsync(bad.p, 0, 4, s));
    int64_t D = 0;
    if (n > 0) {
        k_keys_validate<<<blocks_for(n), 256, 0, s>>>(coords, n, N, spec, (uint64_t*)kin.p,
                                                      (int32_t*)iin.p, (int32_t*)bad.p);
        TK_LAUNCH_CHECK("k_keys_validate");
        int32_t hbad = 0;
        TK_HIP(hipMemcpyAsync(&hbad, bad.p, 4, hipMemcpyDeviceToHost, s));
        TK_HIP(hipStreamSynchronize(s));
        if (hbad) return set_error(TK_ERR_RANGE, "a coordinate lies outside [0, I_k)");
        // 2. stable sort, find runs of equal coordinates, sum each run
        TK_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp_bytes, (uint64_t*)kin.p, (uint64_t*)kout.p,
                                                  (int32_t*)iin.p, (int32_t*)iout.p, (int)n, 0, bits, s));
        k_heads64<<<blocks_for(n), 256, 0, s>>>((uint64_t*)kout.p, n, (int32_t*)hbuf.p);
        TK_LAUNCH_CHECK("k_heads64");
        TK_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tmp_bytes, (int32_t*)hbuf.p, (int32_t*)pbuf.p,
                                                (int)n, s));
        int32_t last[2];
        TK_HIP(hipMemcpyAsync(&last[0], (int32_t*)pbuf.p + (n - 1), 4, hipMemcpyDeviceToHost, s));
        TK_HIP(hipMemcpyAsync(&last[1], (int32_t*)hbuf.p + (n - 1), 4, hipMemcpyDeviceToHost, s));
        TK_HIP(hipStreamSynchronize(s));
        D = (int64_t)last[0] + last[1];
    }
    ctx->nnz = D;
    size_t dd = (size_t)std::max<int64_t>(D, 1);
    if ((st = dalloc(dco, dd * 4 * N)) || (st = dalloc(dva, dd * 8))) return st;
    if (D > 0) {
        k_coalesce<<<blocks_for(n), 256, 0, s>>>((int32_t*)hbuf.p, (int32_t*)pbuf.p, (int32_t*)iout.p, n,
                                                 coords, vals, N, D, (int32_t*)dco.p, (double*)dva.p);
        TK_LAUNCH_CHECK("k_coalesce");
        unsigned nb = std::min<unsigned>(1024, blocks_for(D));
        k_sumsq_partial<<<nb, 256, 0, s>>>((double*)dva.p, D, (double*)part.p);
        TK_LAUNCH_CHECK("k_sumsq_partial");
        k_sum_final<<<1, 256, 0, s>>>((double*)part.p, (int)nb, (double*)part.p + 1032);
        TK_LAUNCH_CHECK("k_sum_final");
        TK_HIP(hipMemcpyAsync(&ctx->normx2, (double*)part.p + 1032, 8, hipMemcpyDeviceToHost, s));
    } else {
        ctx->normx2 = 0.0;
    }

    // 3. per mode: sort by the mode key, gather the SoA layout, row pointers, chunk table
    const int32_t* dc = (const int32_t*)dco.p;
    // chunk count: kChunkWavesPerCU resident waves per compute unit, pieces of at least 64 entries
    // (small tensors still spread over many waves; the walk is latency-bound there)
    int ncu = 0;
    TK_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    ctx->ncu = ncu;
    const int64_t nchunk_target =
        std::max<int64_t>(1, std::min<int64_t>((int64_t)std::max(ncu, 1) * kChunkWavesPerCU, D / 64));
    for (int m = 0; m < N; ++m) {
        ModeLayout& ml = ctx->mode[m];
        int no = 0;
        for (int t = 0; t < N; ++t)
            if (t != m) ml.others[no++] = t;
        int keyorder[kMaxOrder];
        int kk = 0;
        keyorder[kk++] = m;
        if (N >= 4) {
            ml.fiber_slot = no - 1;
            keyorder[kk++] = ml.others[no - 1];
            for (int j = 0; j < no - 1; ++j) keyorder[kk++] = ml.others[j];
        } else {
            ml.fiber_slot = -1;
            for (int j = 0; j < no; ++j) keyorder[kk++] = ml.others[j];
        }
        ml.K = 1;
        for (int j = 0; j < no; ++j) ml.K *= ctx->ranks[ml.others[j]];

        size_t vs = dtype_size(ctx->dtype);
        if (D == 0) {
            ml.S = 0;
            ml.P = 0;
            TK_HIP(hipMalloc((void**)&ml.idx, 16 * (N - 1)));
            TK_HIP(hipMalloc(&ml.val, 16));
            TK_HIP(hipMalloc((void**)&ml.rows, 16));
            TK_HIP(hipMalloc((void**)&ml.ptr, 16));
            TK_HIP(hipMalloc((void**)&ml.pptr, 16));
            TK_HIP(hipMemsetAsync(ml.ptr, 0, 4, s));
            TK_HIP(hipMemsetAsync(ml.pptr, 0, 4, s));
            ml.nchunks = 0;
            std::vector<int32_t> z{0};
            if ((st = upload(&ml.chunk_ptr, z, s))) return st;
            if ((st = upload(&ml.chunk_row, std::vector<int32_t>(), s))) return st;
            if ((st = upload(&ml.chunk_slot, std::vector<int32_t>(), s))) return st;
            if ((st = upload(&ml.split, std::vector<int32_t>(), s))) return st;
            continue;
        }
        KeySpec ks{};
        ks.n = N;
        for (int j = 0; j < N; ++j) {
            ks.col[j] = dc + (int64_t)keyorder[j] * D;
            ks.radix[j] = ctx->dims[keyorder[j]];
        }
        k_keys<<<blocks_for(D), 256, 0, s>>>(D, ks, (uint64_t*)kin.p, (int32_t*)iin.p);
        TK_LAUNCH_CHECK("k_keys");
        TK_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp_bytes, (uint64_t*)kin.p, (uint64_t*)kout.p,
                                                  (int32_t*)iin.p, (int32_t*)iout.p, (int)D, 0, bits, s));
        GatherSpec g{};
        g.nothers = no;
        for (int j = 0; j < no; ++j) g.other[j] = dc + (int64_t)ml.others[j] * D;
        const int32_t* rowsrc = dc + (int64_t)m * D;
        DevBuf idx_u, val_u;
        if ((st = dalloc(idx_u, dd * 4 * (N - 1))) || (st = dalloc(val_u, dd * vs))) return st;
        if (ctx->dtype == TK_F64)
            st = launch_gather<double>((int32_t*)iout.p, D, rowsrc, g, (double*)dva.p, (int32_t*)rowid.p, (int32_t*)idx_u.p, val_u.p, s);
        else if (ctx->dtype == TK_F32)
            st = launch_gather<float>((int32_t*)iout.p, D, rowsrc, g, (double*)dva.p, (int32_t*)rowid.p, (int32_t*)idx_u.p, val_u.p, s);
        else
            st = launch_gather<bf16_t>((int32_t*)iout.p, D, rowsrc, g, (double*)dva.p, (int32_t*)rowid.p, (int32_t*)idx_u.p, val_u.p, s);
        if (st) return st;
        k_heads32<<<blocks_for(D), 256, 0, s>>>((int32_t*)rowid.p, D, (int32_t*)hbuf.p);
        TK_LAUNCH_CHECK("k_heads32");
        TK_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tmp_bytes, (int32_t*)hbuf.p, (int32_t*)pbuf.p,
                                                (int)D, s));
        int32_t last[2];
        TK_HIP(hipMemcpyAsync(&last[0], (int32_t*)pbuf.p + (D - 1), 4, hipMemcpyDeviceToHost, s));
        TK_HIP(hipMemcpyAsync(&last[1], (int32_t*)hbuf.p + (D - 1), 4, hipMemcpyDeviceToHost, s));
        TK_HIP(hipStreamSynchronize(s));
        ml.S = (int64_t)last[0] + last[1];
        TK_HIP(hipMalloc((void**)&ml.rows, (size_t)ml.S * 4));
        TK_HIP(hipMalloc((void**)&ml.ptr, (size_t)(ml.S + 1) * 4));
        k_rows<<<blocks_for(D), 256, 0, s>>>((int32_t*)hbuf.p, (int32_t*)pbuf.p, (int32_t*)rowid.p, D,
                                             ml.S, ml.rows, ml.ptr);
        TK_LAUNCH_CHECK("k_rows");
        std::vector<int32_t> hptr((size_t)ml.S + 1);
        TK_HIP(hipMemcpyAsync(hptr.data(), ml.ptr, hptr.size() * 4, hipMemcpyDeviceToHost, s));
        TK_HIP(hipStreamSynchronize(s));
        std::vector<int32_t> hpptr((size_t)ml.S + 1);
        hpptr[0] = 0;
        for (int64_t r = 0; r < ml.S; ++r) {
            const int64_t len = (int64_t)hptr[r + 1] - hptr[r];
            const int64_t padded = (int64_t)hpptr[r] + (len + 3) / 4 * 4;
            if (padded >= ((int64_t)1 << 31)) return set_error(TK_ERR_UNSUPPORTED, "padded stream exceeds 2^31 entries");
            hpptr[r + 1] = (int32_t)padded;
        }
        ml.P = hpptr[ml.S];
        if ((st = upload(&ml.pptr, hpptr, s))) return st;
        TK_HIP(hipMalloc((void**)&ml.idx, (size_t)ml.P * 4 * (N - 1)));
        TK_HIP(hipMalloc(&ml.val, (size_t)ml.P * vs));
        {
            const unsigned gp = blocks_for(ml.P), gd = blocks_for(D);
            if (ctx->dtype == TK_F64) {
                k_pad_fill<double><<<gp, 256, 0, s>>>(N - 1, ml.P, ml.idx, (double*)ml.val);
                k_pad_scatter<double><<<gd, 256, 0, s>>>((int32_t*)hbuf.p, (int32_t*)pbuf.p, D, ml.ptr, ml.pptr, N - 1,
                                                         (int32_t*)idx_u.p, (const double*)val_u.p, ml.P, ml.idx, (double*)ml.val);
            } else if (ctx->dtype == TK_F32) {
                k_pad_fill<float><<<gp, 256, 0, s>>>(N - 1, ml.P, ml.idx, (float*)ml.val);
                k_pad_scatter<float><<<gd, 256, 0, s>>>((int32_t*)hbuf.p, (int32_t*)pbuf.p, D, ml.ptr, ml.pptr, N - 1,
                                                        (int32_t*)idx_u.p, (const float*)val_u.p, ml.P, ml.idx, (float*)ml.val);
            } else {
                k_pad_fill<bf16_t><<<gp, 256, 0, s>>>(N - 1, ml.P, ml.idx, (bf16_t*)ml.val);
                k_pad_scatter<bf16_t><<<gd, 256, 0, s>>>((int32_t*)hbuf.p, (int32_t*)pbuf.p, D, ml.ptr, ml.pptr, N - 1,
                                                         (int32_t*)idx_u.p, (const bf16_t*)val_u.p, ml.P, ml.idx, (bf16_t*)ml.val);
            }
            TK_LAUNCH_CHECK("k_pad_scatter");
        }
        std::vector<int32_t> cptr, crow, cslot, split;
        make_chunks(hpptr, nchunk_target, cptr, crow, cslot, split, ml.ncarry, ml.max_row_nnz);
        ml.nchunks = (int64_t)crow.size();
        ml.nsplit = (int64_t)split.size() / 3;
        if ((st = upload(&ml.chunk_ptr, cptr, s)) || (st = upload(&ml.chunk_row, crow, s)) ||
            (st = upload(&ml.chunk_slot, cslot, s)) || (st = upload(&ml.split, split, s)))
            return st;
    }
    TK_HIP(hipStreamSynchronize(s));
    return TK_OK;
}

}  // namespace tk
