// Shared FP64 MFMA building block: partial A^T B over a slab of rows, staged through LDS.
#pragma once

#include "internal.h"

namespace tk {

typedef double atb_d4_t __attribute__((ext_vector_type(4)));

// Partial products P = A[rows, a0:a0+64]^T B[rows, b0:b0+64] in FP64 over one slab of rows.
// Rows are consumed in chunks of 32: the block loads both 32 x 64 panels coalesced (the next
// chunk's loads are issued before the current chunk's MFMAs) into LDS in their own precision
// (FP32 panels take half the LDS of FP64 ones) and converts operands to FP64 as it reads them; wave w
// computes the 16 output rows a0+16w.. across the 64 output columns (4 tiles of
// v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and B[l/16][l%16] and holds
// D[l/16 + 4v][l%16] in result v).  Columns past na / nb read as zero.  Requires r0 < r1,
// a0 < na and b0 < nbc.
// Raw loads of one 32-row chunk: every load is issued unconditionally from a clamped (valid)
// address, so all 16 are in flight together; masking and the conversion to FP64 happen when the
// chunk is written to LDS, after the MFMAs of the previous chunk.
template <typename AT, typename BT>
__device__ inline void atb_stage(const AT* __restrict__ A, int lda, int na, const BT* __restrict__ B, int ldb,
                                 int nbc, int64_t row0, int64_t r1, int a0, int b0, AT* xa, BT* xb) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int e = threadIdx.x + 256 * k;
        const int rr = e >> 6, cc = e & 63;
        const int64_t row = min(row0 + rr, r1 - 1);
        xa[k] = A[row * lda + (a0 + cc < na ? a0 + cc : a0)];
        xb[k] = B[row * ldb + (b0 + cc < nbc ? b0 + cc : b0)];
    }
}

template <typename AT, typename BT>
__device__ void atb_block(const AT* __restrict__ A, int lda, int na, const BT* __restrict__ B, int ldb,
                          int nbc, int64_t r0, int64_t r1, int a0, int b0, AT (*As)[32][65],
                          BT (*Bs)[32][65], atb_d4_t* acc) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int kq = lane >> 4, c16 = lane & 15;
    // this thread's share of a chunk: column cc of each panel, rows rw + 4k (k < 8).  Full chunks
    // load from 32-bit byte offsets off a uniform base when both matrices' rows below r1 span less
    // than 4 GB; the last, partial chunk (and larger inputs) take the clamped loads above.
    const int cc = lane, rw = w;
    const bool oka = a0 + cc < na, okb = b0 + cc < nbc;
    const uint32_t ca = (uint32_t)(oka ? a0 + cc : a0) * (uint32_t)sizeof(AT);
    const uint32_t cb = (uint32_t)(okb ? b0 + cc : b0) * (uint32_t)sizeof(BT);
    const uint32_t rowa = (uint32_t)lda * (uint32_t)sizeof(AT), rowb = (uint32_t)ldb * (uint32_t)sizeof(BT);
    const bool off32 = (uint64_t)r1 * (uint64_t)lda * sizeof(AT) < (1ull << 32) &&
                       (uint64_t)r1 * (uint64_t)ldb * sizeof(BT) < (1ull << 32);
    AT xa[8];
    BT xb[8];
    auto stage = [&](int64_t row0) __attribute__((always_inline)) {
        if (off32 && row0 + 32 <= r1) {
            const uint32_t r = (uint32_t)(row0 + rw);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                xa[k] = *(const AT*)((const char*)A + ((r + 4u * (uint32_t)k) * rowa + ca));
                xb[k] = *(const BT*)((const char*)B + ((r + 4u * (uint32_t)k) * rowb + cb));
            }
        } else {
            atb_stage(A, lda, na, B, ldb, nbc, row0, r1, a0, b0, xa, xb);
        }
    };
    stage(r0);
    int buf = 0;
    for (int64_t row0 = r0; row0 < r1; row0 += 32) {
        if (row0 + 32 <= r1) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                As[buf][rw + 4 * k][cc] = oka ? xa[k] : AT(0);
                Bs[buf][rw + 4 * k][cc] = okb ? xb[k] : BT(0);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const bool rv = row0 + rw + 4 * k < r1;
                As[buf][rw + 4 * k][cc] = (rv && oka) ? xa[k] : AT(0);
                Bs[buf][rw + 4 * k][cc] = (rv && okb) ? xb[k] : BT(0);
            }
        }
        __syncthreads();
        if (row0 + 32 < r1) stage(row0 + 32);
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            const int rr = 4 * st + kq;
            const double av = (double)As[buf][rr][16 * w + c16];
#pragma unroll
            for (int t = 0; t < 4; ++t)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, (double)Bs[buf][rr][16 * t + c16], acc[t], 0, 0, 0);
        }
        buf ^= 1;
    }
}

}  // namespace tk
