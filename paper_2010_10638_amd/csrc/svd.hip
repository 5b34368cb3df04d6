// SVD factor update of standard HOOI (paper Alg. 1): U_n <- the R_n leading left singular vectors
// of Y_(n), in FP64, the alternative to the QRP of Alg. 2 (Sec. III-D compares the two).
//
// The singular vectors come from the eigendecomposition of a small symmetric FP64 matrix that the
// QRP path already forms on the device: for a tall Y_(n) (K_n <= I_n) the Gram matrix
// C = Y^T Y (K_n x K_n), whose eigenpairs (sigma_r^2, v_r) give u_r = Y v_r / sigma_r; for a fat
// Y_(n) the matrix Y Y^T (I_n x I_n), whose leading eigenvectors are the u_r themselves.  The
// eigendecomposition is rocSOLVER's divide-and-conquer dsyevd (a library primitive, eigenvalues
// ascending); forming U and fixing signs are kernels of this file.  Sign convention (singular
// vectors are defined up to sign): each column's entry of largest magnitude, the first one on
// ties, is made positive.  A zero singular value gives a zero column (rank deficiency; such
// columns are not determined by Y).
#include "internal.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

namespace tk {

namespace {

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Tall case: U[i][r] = (sum_c Y[i][c] V[c][j]) / sqrt(lambda_j), j = K-1-r (descending
// eigenvalues); V column-major (eigenvector j at V + j K).  One thread per output entry (the
// lanes of a row read the same Y entries; the R eigenvector columns stay in cache), c ascending.
template <typename YT>
__global__ __launch_bounds__(256) void k_svd_left(const YT* __restrict__ Y, int64_t I, int K,
                                                  const double* __restrict__ V, const double* __restrict__ D,
                                                  int R, double* __restrict__ U) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= I * R) return;
    const int64_t i = e / R;
    const int r = (int)(e % R);
    const YT* y = Y + i * K;
    const double* v = V + (int64_t)(K - 1 - r) * K;
    double acc = 0.0;
    for (int c = 0; c < K; ++c) acc += (double)y[c] * v[c];
    const double lam = D[K - 1 - r];
    U[e] = (lam > 0.0) ? acc / sqrt(lam) : 0.0;
}

// Fat case: U[i][r] = eigenvector I-1-r of Y Y^T, entry i.
__global__ void k_svd_fat(const double* __restrict__ V, int64_t I, int R, double* __restrict__ U) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= I * R) return;
    const int64_t i = e / R;
    const int r = (int)(e % R);
    U[e] = V[(I - 1 - r) * I + i];
}

// One workgroup per column: the entry of largest magnitude (first one on ties) made positive.
__global__ __launch_bounds__(256) void k_svd_sign(double* __restrict__ U, int64_t I, int R) {
    __shared__ double s_v[256];
    __shared__ int64_t s_i[256];
    __shared__ int s_flip;
    const int r = blockIdx.x;
    double best = -1.0;
    int64_t bi = 0;
    for (int64_t i = threadIdx.x; i < I; i += blockDim.x) {
        const double v = fabs(U[i * R + r]);
        if (v > best) { best = v; bi = i; }
    }
    s_v[threadIdx.x] = best;
    s_i[threadIdx.x] = bi;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = s_v[0];
        int64_t ii = s_i[0];
        for (int t = 1; t < (int)blockDim.x; ++t)
            if (s_v[t] > b || (s_v[t] == b && s_i[t] < ii)) { b = s_v[t]; ii = s_i[t]; }
        s_flip = (U[ii * R + r] < 0.0) ? 1 : 0;
    }
    __syncthreads();
    if (s_flip)
        for (int64_t i = threadIdx.x; i < I; i += blockDim.x) U[i * R + r] = -U[i * R + r];
}

template <typename YT>
int left_typed(const tk_ctx* ctx, int mode, const YT* Y, const double* V, const double* D, double* U,
               hipStream_t s) {
    const int64_t I = ctx->dims[mode];
    const int K = (int)ctx->mode[mode].K, R = ctx->ranks[mode];
    k_svd_left<YT><<<cdiv(I * R, 256), 256, 0, s>>>(Y, I, K, V, D, R, U);
    TK_LAUNCH_CHECK("k_svd_left");
    return TK_OK;
}

}  // namespace

void free_svd_ws(tk_ctx* ctx) {
    void* ps[] = {ctx->svd_d, ctx->svd_e, ctx->svd_info};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    ctx->svd_d = ctx->svd_e = nullptr;
    ctx->svd_info = nullptr;
    if (ctx->rb) (void)rocblas_destroy_handle((rocblas_handle)ctx->rb);
    ctx->rb = nullptr;
}

int svd_run(tk_ctx* ctx, int mode, const void* Y, double* U, hipStream_t s) {
    double* A = nullptr;
    int n = 0;
    int st = gram_run(ctx, mode, Y, &A, &n, s);
    if (st) return st;
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
    const int64_t I = ctx->dims[mode];
    const int R = ctx->ranks[mode];
    if (qrp_route(ctx, mode) == 2) {
        k_svd_fat<<<cdiv(I * R, 256), 256, 0, s>>>(A, I, R, U);
        TK_LAUNCH_CHECK("k_svd_fat");
    } else if (ctx->dtype == TK_F64) {
        if ((st = left_typed<double>(ctx, mode, (const double*)Y, A, ctx->svd_d, U, s))) return st;
    } else {
        if ((st = left_typed<float>(ctx, mode, (const float*)Y, A, ctx->svd_d, U, s))) return st;
    }
    k_svd_sign<<<(unsigned)R, 256, 0, s>>>(U, I, R);
    TK_LAUNCH_CHECK("k_svd_sign");
    return convert_factor(ctx, mode, U, s);
}

}  // namespace tk
