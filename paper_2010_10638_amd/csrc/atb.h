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
    AT xa[8];
    BT xb[8];
    atb_stage(A, lda, na, B, ldb, nbc, r0, r1, a0, b0, xa, xb);
    int buf = 0;
    for (int64_t row0 = r0; row0 < r1; row0 += 32) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int e = threadIdx.x + 256 * k;
            const int rr = e >> 6, cc = e & 63;
            const bool rv = row0 + rr < r1;
            As[buf][rr][cc] = (rv && a0 + cc < na) ? xa[k] : AT(0);
            Bs[buf][rr][cc] = (rv && b0 + cc < nbc) ? xb[k] : BT(0);
        }
        __syncthreads();
        if (row0 + 32 < r1) atb_stage(A, lda, na, B, ldb, nbc, row0 + 32, r1, a0, b0, xa, xb);
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
