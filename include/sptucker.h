/*
 * sptucker.h - C ABI of the MI355X (gfx950) sparse Tucker library.
 *
 * The library computes the hot path of sparse Tucker decomposition by higher-order orthogonal
 * iteration with QR column pivoting (Kaya-style sparse HOOI as stated in "Sparse Tucker Tensor
 * Decomposition on a Hybrid FPGA-CPU Platform", arXiv 2010.10638):
 *   - per mode n, the sparse tensor-times-matrix chain (TTMc) of Alg. 2:
 *       Y_(n)(i_n, :) += x * (U_t1(i_t1, :) kron U_t2(i_t2, :) kron ...)   over the nonzeros,
 *     other modes t != n ascending, the LAST one varying fastest (Sec. III-C, Kronecker listing);
 *   - U_n <- the first R_n columns of Q from a QR with column pivoting of Y_(n) (Sec. III-D),
 *     or of Y_(n) Y_(n)^T when Y_(n) has more columns than rows;
 *   - after the mode loop, the core G_(N) = U_N^T Y_(N) (Alg. 2; unfolded form in Sec. III-B);
 *   - the fit 1 - ||X - G x_1 U_1 ... x_N U_N|| / ||X||.
 *
 * Conventions for every entry point:
 *   - Plain C types only.  "device" pointers are HIP device memory (hipMalloc or a PyTorch CUDA
 *     tensor); "host" pointers are ordinary host memory.  Every pointer argument is owned by the
 *     caller; the library owns only what hangs off a tk_ctx and frees it in tucker_free.
 *   - stream is a hipStream_t passed as void* (NULL = the default stream).  Work is enqueued
 *     asynchronously on it; only the calls documented as synchronising wait for the device.
 *   - Every call on one context uses that context's scratch (factor copies, Y_(n), carry rows,
 *     QRP, SVD and completion workspaces).  Calls on the same context must therefore be ordered:
 *     issue them on one stream, or make each call's stream wait for the previous call's stream
 *     (an event) before the call.  Concurrent calls on one context race; different contexts are
 *     independent.
 *   - Indices are 0-based.  Modes are 0-based in the API (mode 0 is the paper's mode 1).
 *   - Matrices are row-major: U_k is I_k x R_k, Y_(n) is I_n x K_n with K_n = prod_{t != n} R_t.
 *   - The core G is stored C-order (last index fastest), R_1 x ... x R_N.
 *   - Return value: TK_OK or an error code; tucker_last_error() gives a message (thread-local).
 *     Arguments are validated before any launch.  A HIP failure, including an asynchronous
 *     fault of earlier work on the stream that surfaces during the call, returns TK_ERR_HIP.
 */
#ifndef SPTUCKER_H
#define SPTUCKER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tk_ctx tk_ctx;

enum tk_status {
    TK_OK = 0,
    TK_ERR_ARG = 1,          /* invalid argument (null pointer, bad mode, rank out of range, ...) */
    TK_ERR_RANGE = 2,        /* a coordinate lies outside [0, I_k) */
    TK_ERR_OOM = 3,          /* device allocation failed */
    TK_ERR_HIP = 4,          /* a HIP runtime call or kernel failed */
    TK_ERR_UNSUPPORTED = 5   /* valid input outside the library's compiled limits (TK_MAX_*) */
};

/* Arithmetic of the TTMc (the QRP, core and fit always run in FP64):
 *   TK_F64  - FP64 values, factors, products and accumulation; Y_(n) is double.
 *   TK_F32  - FP32 values and factor copies, FP32 products and accumulation; Y_(n) is float.
 *   TK_BF16 - BF16 values and factor copies and FP32 accumulation; Y_(n) is float.  Order 3
 *             (both other ranks <= 16) runs on the BF16 matrix instruction: x a is rounded
 *             once to BF16 (nearest, ties to even) and multiplied by b exactly in FP32.  Other
 *             orders take FP32 products (exact: a product of three bf16 numbers fits the fp32
 *             significand). */
enum tk_dtype { TK_F64 = 0, TK_F32 = 1, TK_BF16 = 2 };

/* tucker_init flags */
#define TK_FLAG_NO_FAT_RULE 0x1u     /* factor a fat Y_(n) directly instead of Y_(n) Y_(n)^T */
#define TK_FLAG_SVD         0x2u     /* hooi_sweep updates each factor by svd_update (Alg. 1) */
#define TK_FLAG_SVD_LIB     0x4u     /* svd_update: rocSOLVER dsyevd for every eigenproblem */
#define TK_FLAG_NO_MEMO     0x8u     /* hooi_sweep: every mode's TTMc from the nonzeros (no shared sums) */

#define TK_MAX_ORDER 8               /* 2 <= N <= TK_MAX_ORDER */
#define TK_MAX_KCOLS 4096            /* K_n = prod_{t != n} R_t must not exceed this */

/*
 * tucker_init - take a COO tensor and build the per-mode sorted layout (Alg. 2 input: the sparse
 * tensor and the ranks R_1..R_N; COO format of Sec. III-A / Table I).
 *   out     host   receives the new context
 *   order   N, 2..TK_MAX_ORDER
 *   dims    host   int64[N], I_k >= 1, with prod I_k < 2^63
 *   ranks   host   int32[N], 1 <= R_k <= I_k and R_k <= K_k (the QRP needs R_k columns)
 *   nnz     number of COO entries, 0 <= nnz < 2^31
 *   coords  device int32[N * nnz], structure of arrays: coords[k * nnz + p] = i_k of entry p
 *   vals    device double[nnz]
 *   dtype   enum tk_dtype for the TTMc
 *   flags   TK_FLAG_*
 * Duplicate coordinates are summed (in input order, FP64); explicit zeros are kept.  The inputs
 * are copied; the caller may free them after the call returns.  Synchronises the stream once (to
 * size the layout).  Errors: TK_ERR_ARG, TK_ERR_RANGE (no context is created), TK_ERR_OOM,
 * TK_ERR_UNSUPPORTED, TK_ERR_HIP.
 */
int tucker_init(tk_ctx** out, int order, const int64_t* dims, const int32_t* ranks, int64_t nnz,
                const int32_t* coords, const double* vals, int dtype, uint32_t flags, void* stream);

/*
 * tucker_get_info - sizes of the layout built by tucker_init (host outputs, any may be NULL):
 *   nnz_distinct  number of distinct coordinates
 *   rows          int64[N]: number of distinct i_n per mode (non-empty rows of Y_(n))
 *   chunks        int64[N]: number of nonzero chunks the TTMc kernels walk per mode
 *   normx2        ||X||_F^2 of the coalesced values (FP64)
 */
int tucker_get_info(const tk_ctx* ctx, int64_t* nnz_distinct, int64_t* rows, int64_t* chunks,
                    double* normx2);

/*
 * tucker_get_csf - copy the mode-sorted layout of one mode to caller device buffers.  The sort key
 * is (i_n, other modes ascending) for N <= 3 and (i_n, i_f, remaining others ascending) for
 * N >= 4, where the fiber mode f is the last mode other than n.
 *   rows  device int32[S]      distinct i_n, ascending (S = rows[mode] of tucker_get_info)
 *   ptr   device int64[S + 1]  row pointers into the sorted nonzeros
 *   idx   device int32[(N-1) * nnz_distinct], other-mode indices, other modes ascending (SoA)
 *   vals  device, nnz_distinct values in the TTMc storage type (double / float / bf16 bits)
 */
int tucker_get_csf(tk_ctx* ctx, int mode, int32_t* rows, int64_t* ptr, int32_t* idx, void* vals,
                   void* stream);

/*
 * ttmc_mode - Y_(n) = X_(n) (kron_{t != n} U_t): the nonzero loop of Alg. 2 for one mode, the
 * per-nonzero Kronecker update of Sec. III-C.
 *   mode  0..N-1
 *   U     host array of N device pointers to FP64 factors (I_k x R_k); U[mode] is not read
 *   Y     device, I_n x K_n row-major: double for TK_F64, float otherwise.  Every entry is written
 *         (rows without nonzeros are set to zero).
 * The factors are converted to the context's TTMc precision on the stream before the product.
 */
int ttmc_mode(tk_ctx* ctx, int mode, const double* const* U, void* Y, void* stream);

/*
 * ttmc_memo_pair - the TTMc of the last two modes with shared partial sums (order >= 4).  The
 * reuse of Sec. III-C (a Kronecker product formed once for the nonzeros sharing its indices)
 * carried across the modes N-2 and N-1, which follow each other in a sweep (Alg. 2): mode N-2's
 * fiber kernel forms, for every fiber (i_{N-2}, i_{N-1}), the inner sum
 * T = sum x kron_{k < N-2} U_k(i_k, :), and mode N-1's TTMc is then a sum over fibers,
 * Y_(N-1)(i_{N-1}, c R_{N-2} + r) = sum_{i_{N-2}} T(i_{N-2}, i_{N-1}, c) U_{N-2}(i_{N-2}, r).
 *   U       host array of N device pointers to FP64 factors (I_k x R_k); U[N-2] is not read
 *   U_next  device FP64 I_{N-2} x R_{N-2}: the U_{N-2} that the second product uses (in a sweep,
 *           mode N-2's updated factor)
 *   Y_a     device, I_{N-2} x K_{N-2}: TTMc of mode N-2 with U (as ttmc_mode)
 *   Y_b     device, I_{N-1} x K_{N-1}: TTMc of mode N-1 with U, U[N-2] replaced by U_next
 * Both in the context's Y type (double for TK_F64, float otherwise); every entry is written.
 * hooi_sweep runs modes N-2 and N-1 this way unless the context has TK_FLAG_NO_MEMO or mode
 * N-2's fibers hold fewer than 4 nonzeros on average.  The first call builds the fiber table
 * (kept by the context; the fiber sums take pieces x prod_{k<N-2} R_k values of the Y type).
 * Errors: TK_ERR_UNSUPPORTED below order 4, when mode N-2 does not run the fiber kernel
 * (tucker_ttmc_kernel), or prod_{k<N-2} R_k > 512 or R_{N-2} > 16; TK_ERR_ARG for null pointers;
 * TK_ERR_OOM.
 */
int ttmc_memo_pair(tk_ctx* ctx, const double* const* U, const double* U_next, void* Y_a, void* Y_b, void* stream);

/*
 * qrp_update - U_n <- QRP(Y_(n), R_n) (Alg. 2; Sec. III-D): the first R_n columns of Q of a QR
 * with column pivoting, in FP64.  When K_n > I_n (and TK_FLAG_NO_FAT_RULE is not set) the QRP is
 * taken of Y_(n) Y_(n)^T.  Q is the Householder one: column j has the sign that the reflector
 * v = x + sgn(x_0) ||x|| e_1 (sgn(0) = +1) gives it.
 *   Y     device I_n x K_n (double for TK_F64, float otherwise)
 *   U_out device double I_n x R_n
 *   piv   device int32[R_n] or NULL: original column index chosen at each pivot step
 * Also refreshes the context's low-precision copy of U_n used by hooi_sweep.
 */
int qrp_update(tk_ctx* ctx, int mode, const void* Y, double* U_out, int32_t* piv, void* stream);

/*
 * svd_update - U_n <- the R_n leading left singular vectors of Y_(n) (the SVD update of standard
 * HOOI, Alg. 1; Sec. III-D contrasts it with the QRP), in FP64.  Computed from the
 * eigendecomposition of Y_(n)^T Y_(n) (K_n <= I_n; columns Y v / sigma) or of Y_(n) Y_(n)^T
 * (fat rule), formed in FP64 on the device.  Columns are ordered by decreasing singular value;
 * each column's entry of largest magnitude (the first one on ties) is positive.  A zero singular
 * value gives a zero column.
 *   Y     device I_n x K_n (double for TK_F64, float otherwise)
 *   U_out device double I_n x R_n
 * The R_n leading eigenpairs come from a Chebyshev-filtered subspace iteration (order <= 1024,
 * R_n <= 32), stopped when every residual ||A v - lambda v|| <= 2e-14 lambda_max; the call reads
 * each outer step's residual test back (one synchronisation of the stream per step).  If it
 * does not converge within its step limit, if the shape is outside those limits, or if the
 * context was created with TK_FLAG_SVD_LIB, rocSOLVER's dsyevd computes all eigenpairs instead.
 * Shapes the QRP handles only by Householder (R_n > 32, or K_n > 1024 on a tall Y_(n), or a fat
 * Y_(n) with TK_FLAG_NO_FAT_RULE) return TK_ERR_UNSUPPORTED.  Also refreshes the context's
 * low-precision copy of U_n.
 */
int svd_update(tk_ctx* ctx, int mode, const void* Y, double* U_out, void* stream);

/*
 * tucker_svd_info - which eigensolver served the context's last svd_update (host output):
 *   outer_steps  Rayleigh-Ritz steps the subspace iteration took after the first (0 when the
 *                start block was already converged), or -1 when rocSOLVER's dsyevd computed the
 *                eigenpairs (no SVD update yet, TK_FLAG_SVD_LIB, shape outside the iteration's
 *                limits, or no convergence within its step limit)
 */
int tucker_svd_info(const tk_ctx* ctx, int* outer_steps);

/* The TTMc kernel a mode runs (tucker_ttmc_kernel). */
enum tk_ttmc_kernel {
    TK_TTMC_GENERIC = 0,   /* any order and K_n <= TK_MAX_KCOLS, vector ALU */
    TK_TTMC_ORDER3 = 1,    /* order 3, other ranks <= 16, factors below 2^31 bytes: matrix cores */
    TK_TTMC_FIBER = 2      /* order 4-5: fiber-factored (each fiber's row of the last other mode once) */
};

/*
 * tucker_ttmc_kernel - which TTMc kernel ttmc_mode / hooi_sweep run for a mode of a tensor of this
 * shape (host-only: no device, no context).  The order-3 matrix-core kernel forms its gather
 * offsets in 32 bits, so it is taken only while every other factor's copy stays below 2^31 bytes
 * (dims[t] x 16 columns x the TTMc type's size); larger factors take the generic kernel.
 *   kernel  host int, receives enum tk_ttmc_kernel
 * Errors: TK_ERR_ARG.
 */
int tucker_ttmc_kernel(int order, const int64_t* dims, const int32_t* ranks, int dtype, int mode, int* kernel);

/*
 * tucker_qrp_gaps - pivot gaps of the last QRP of a mode (qrp_update or a sweep): gaps[j] =
 * (d_j - d'_j) / d_j, where d_j is the squared norm of the trailing column chosen at step j of the
 * pivoted factorization (Sec. III-D compares these norms) and d'_j the largest squared norm among
 * the other candidates; 0 means a tie (decided by column position), small values mean that
 * rounding of Y_(n) can change the pivot.  NaN where the route used does not record them (the
 * Householder and fat-matrix routes, R_n > 32) or before the mode's first QRP.
 *   gaps  host double[R_mode]
 * Synchronises the stream of the context's last call.  Errors: TK_ERR_ARG, TK_ERR_HIP.
 */
int tucker_qrp_gaps(tk_ctx* ctx, int mode, double* gaps);

/*
 * core_fit - G_(N) = U_N^T Y_(N) (Alg. 2, the step after the mode loop) and the fit.
 *   Y_last device I_N x K_N (context Y type) computed with the final U_1..U_{N-1}
 *   U_last device double I_N x R_N (orthonormal columns)
 *   G      device double[prod R_k], C-order: G[r_1..r_{N-1}, r_N] = G_(N)[r_N, c(r_1..r_{N-1})]
 *   fit    device double scalar or NULL: 1 - sqrt(max(||X||^2 - ||G||^2, 0)) / ||X||
 */
int core_fit(tk_ctx* ctx, const void* Y_last, const double* U_last, double* G, double* fit,
             void* stream);

/*
 * core_fit_static - core_fit without a context and without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arithmetic and kernels as core_fit; the slab partials live in a static
 * per-device scratch array of the library (8 MiB per device, held until the process ends).
 *   ytype   TK_F64 or TK_F32: element type of Y_last
 *   I, R, K I_N, R_N, K_N; R * K must not exceed 2^20 (else TK_ERR_UNSUPPORTED, nothing launched)
 *   Y_last  device I x K (ytype), U_last device double I x R, G device double[R * K] (C-order as
 *           for core_fit), fit device double scalar or NULL, normx2 = ||X||^2 (host value)
 * Calls on the same device share the scratch: calls that overlap in time on one device (two
 * streams, two host threads) race and must be serialised by the caller.  Nothing in the scratch
 * needs clearing: every call overwrites the partials it reads.  Errors: TK_ERR_ARG,
 * TK_ERR_UNSUPPORTED, TK_ERR_HIP.
 */
int core_fit_static(int ytype, int64_t I, int32_t R, int64_t K, const void* Y_last, const double* U_last,
                    double normx2, double* G, double* fit, void* stream);

/*
 * hosvd_init - HOSVD-style initial factors (Alg. 1 starts HOOI from the leading left singular
 * vectors of every unfolding X_(n)), computed on a sketch: for each mode n independently,
 * Y_(n) = X_(n) (kron_{k != n} Omega_k) with the caller's random test factors Omega_k (a
 * Kronecker-structured random projection of the columns of X_(n), the TTMc of ttmc_mode), then
 * U_n <- QRP(Y_(n), R_n) (use_svd = 0, the factor update of Alg. 2) or its leading R_n left
 * singular vectors (use_svd != 0, as svd_update).  With Omega_k of full column rank the sketch
 * keeps the column space of X_(n) whenever rank(X_(n)) <= K_n.
 *   Omega  host array of N device pointers to double I_k x R_k (e.g. Gaussian; read only; Omega[n]
 *          is read for the other modes)
 *   U_out  host array of N device pointers to double I_k x R_k, written (must not alias Omega)
 * The context's factor copies and Y buffer are overwritten.  Errors: as ttmc_mode and
 * qrp_update / svd_update.
 */
int hosvd_init(tk_ctx* ctx, const double* const* Omega, double* const* U_out, int use_svd, void* stream);

/*
 * hooi_sweep - one sweep of Alg. 2: for n = 0..N-1, TTMc with the current factors then
 * U_n <- QRP(Y_(n), R_n) (modes updated in order, each using the factors already refreshed in this
 * sweep); then the core and the fit.  A context created with TK_FLAG_SVD updates the factors with
 * svd_update instead (Alg. 1), which synchronises the stream a few times per mode.
 *   U        host array of N device pointers to double I_k x R_k, read and overwritten
 *   G        device double[prod R_k] (C-order), overwritten
 *   fit_dev  device double scalar or NULL
 *   fit_host host double or NULL; when non-NULL the call synchronises the stream to return it
 * The Y_(n) buffers are owned by the context.
 */
int hooi_sweep(tk_ctx* ctx, double* const* U, double* G, double* fit_dev, double* fit_host,
               void* stream);

/*
 * hooi_run - the outer loop of Alg. 2 with a stopping rule (the paper iterates "until
 * convergence" without stating one; here: stop after sweep s >= 1 when |fit_s - fit_{s-1}| <= tol,
 * or after max_sweeps sweeps).  Each sweep is hooi_sweep; the stream is synchronised once per
 * sweep to read the fit.
 *   U, G        as for hooi_sweep
 *   max_sweeps  >= 1
 *   tol         >= 0 (0: run max_sweeps sweeps unless the fit repeats exactly)
 *   fits_host   host double[max_sweeps] or NULL: the fit after each sweep
 *   sweeps_done host int or NULL: the number of sweeps run
 */
int hooi_run(tk_ctx* ctx, double* const* U, double* G, int max_sweeps, double tol, double* fits_host,
             int* sweeps_done, void* stream);

/*
 * reconstruct - the Tucker model at sampled coordinates (paper Sec. III, the model
 * X ~ G x_1 U_1 ... x_N U_N):  out[p] = sum_r G[r] prod_k U_k(i_k(p), r_k), in FP64.
 *   G       device double[prod R_k] C-order
 *   U       host array of N device pointers to double I_k x R_k
 *   m       number of coordinates (0 allowed)
 *   coords  device int32[N * m] (SoA, 0-based; each must lie in [0, I_k) - not checked here)
 *   out     device double[m]
 */
int reconstruct(tk_ctx* ctx, const double* G, const double* const* U, int64_t m,
                const int32_t* coords, double* out, void* stream);

/*
 * ttmc_adjoint - loss and gradients of the sampled-entry Tucker model over the context's entries
 * (Tucker completion, built on the adjoint of the TTMc of Alg. 2).  With the model value
 * xhat_p = sum_r G[r] prod_k U_k(i_k, r_k) and the residual e_p = xhat_p - x_p of every entry p
 * of the context (|Omega| = distinct entries):
 *   loss  = sum_p e_p^2 / (2 |Omega|)
 *   gU_n  = E_(n) (kron_{k != n} U_k) G_(n)^T / |Omega|        (I_n x R_n)
 *   gG    = sum_p e_p kron_k U_k(i_k, :) / |Omega|             (C order, like G)
 *   dtype  TK_F32 or TK_F64: the type of G, U, loss, gG, gU; it must equal the context's TTMc
 *          type (a TK_BF16 context returns TK_ERR_UNSUPPORTED)
 *   G      device [prod R_k], C order (last mode fastest)
 *   U      host array of N device pointers, I_k x R_k row-major
 *   loss   device scalar
 *   gG     device [prod R_k], written
 *   gU     host array of N device pointers, I_k x R_k, written
 * Every pointer is caller-owned; the work is enqueued on `stream` without synchronisation,
 * except in the first call.  That call allocates the completion workspace, held until
 * tucker_free: the row of every padded position of each mode, the residuals in two stream orders,
 * U_0 G_(0), and for every mode n >= 1 a map from its padded positions to mode 0's.  It builds the
 * maps with radix sorts, synchronising the stream once to release their temporaries.  Sums run in
 * a fixed order, so the results are deterministic.  Errors: TK_ERR_ARG (null pointer, dtype mismatch),
 * TK_ERR_UNSUPPORTED, TK_ERR_OOM, TK_ERR_HIP.
 */
int ttmc_adjoint(tk_ctx* ctx, int dtype, const void* G, const void* const* U, void* loss, void* gG,
                 void* const* gU, void* stream);

/*
 * tucker_profile - start (capacity > 0) or stop (capacity = 0) timing the regions of hooi_sweep.
 * While on, each sweep records HIP events on its stream around every mode's TTMc (kernel and
 * split-row fix-up), every QRP and the core/fit; at most `capacity` sweeps are recorded.  The
 * events are created here, so recording adds no allocation to the sweep.  Errors: TK_ERR_ARG,
 * TK_ERR_HIP.
 */
int tucker_profile(tk_ctx* ctx, int capacity);

/*
 * tucker_profile_read - synchronise the recorded events and return the summed region times in
 * milliseconds since tucker_profile was switched on (host outputs, any may be NULL):
 *   ttmc_ms         double[N]  per-mode TTMc region (main kernel and split-row fix-up)
 *   ttmc_kernel_ms  double[N]  per-mode main TTMc kernel alone
 *   qrp_ms          double[N]  per-mode QRP time
 *   core_ms         double     core and fit
 *   sweeps          int64      sweeps recorded
 */
int tucker_profile_read(tk_ctx* ctx, double* ttmc_ms, double* ttmc_kernel_ms, double* qrp_ms, double* core_ms,
                        int64_t* sweeps);

/* tucker_free - synchronise the last stream used, release every context allocation.  NULL is ok. */
void tucker_free(tk_ctx* ctx);

/* tucker_last_error - message for the last non-OK status returned on this host thread. */
const char* tucker_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPTUCKER_H */
