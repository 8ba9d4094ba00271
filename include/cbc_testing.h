/*
 * cbc_testing.h -- kernel-level entry points of libcbc.so, used by the test suite to check single
 * steps of the compression on the GPU in isolation. They allocate their own scratch with hipMalloc
 * and synchronise the stream; they are not part of the production path.
 *
 * All matrices are row-major, interleaved complex (complex64 if the *_c128 flag is 0, complex128
 * otherwise), device pointers. Return values are cbc_status codes from cbc.h.
 */
#ifndef CBC_TESTING_H
#define CBC_TESTING_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* C (M x N) = op(A) op(B), op(X) = X, X^T, conj(X) or X^H by (trans, conj). A is stored M x K (or
 * K x M if transA), B is K x N (or N x K if transB). acc_fp64 selects FP64 MFMA accumulation,
 * otherwise FP32 MFMA. tile: -1 = the compression's policy (tile by shape, split reduction where it
 * would split), 0 = 32x32, 1 = 64x64, 2 = pipelined 64x64, 3 = pipelined 128x128 on eight waves
 * (FP32 accumulation; FP64 takes 2); other values are rejected. This is the contraction kernel of
 * every sweep. */
int cbc_test_gemm(int M, int N, int K, const void* A, int a_c128, int transA, int conjA,
                  const void* B, int b_c128, int transB, int conjB, void* C, int c_c128,
                  int acc_fp64, int tile, void* stream);

/* Timing of the same kernel on a plain row-major M x K by K x N product with buffers it allocates
 * itself (zero-filled): one untimed launch, then `reps` launches between two HIP events on the null
 * stream; *ms (host) receives the average milliseconds per launch. */
int cbc_test_gemm_time(int M, int N, int K, int a_c128, int b_c128, int c_c128, int acc_fp64,
                       int tile, int reps, float* ms);

/* Truncation eigensolve (Sec. III A: the joined leg is compressed, by a singular value decomposition,
 * realised on the FP64 Gram matrix): G (s x s complex128 Hermitian, overwritten) -> U (s x kmax
 * complex128, top eigenvectors as columns, zero beyond the kept count), lam (kmax doubles,
 * descending), kkeep (1 int), inv_sqrt_l0 (1 double). tstamp: nullptr, or 16 int64 device slots:
 * wall-clock stamps (100 MHz) of the start [0] and the ends of the tridiagonal reduction [1], the
 * eigenvalues [2] and the eigenvectors [3]; accumulated durations of the reduction's phases [4..6]
 * (and, for s > 128, [8..12]); the number of eigenvalue clusters [7]. */
int cbc_test_eig(void* G, int s, int kmax, double tol, void* U, void* lam, void* kkeep,
                 void* inv_sqrt_l0, void* tstamp, void* stream);

/* The same eigensolve with the reduction to tridiagonal form chosen for s > 128: reduction 0 is the
 * library's (two-stage: dense -> band of half-bandwidth 16 -> tridiagonal), 1 the one-stage
 * multi-workgroup Householder reduction (s <= 1536), which the library uses for single eager
 * instances; other values are
 * rejected. */
int cbc_test_eig_reduction(void* G, int s, int kmax, double tol, int reduction, void* U, void* lam,
                           void* kkeep, void* inv_sqrt_l0, void* tstamp, void* stream);

/* The same eigensolve with the call's report: status (1 int, device, must hold 0 = CBC_OK before
 * the call) receives a failure code, rec (one cbc_trunc_record, device) the truncation record
 * (node 7, sweep 2). force_timeout = 1 makes the first cross-workgroup wait of the multi-workgroup
 * reduction (s > 128) give up at once, so that the time-out path runs while every workgroup exits
 * normally: status then holds CBC_ETIMEOUT. */
int cbc_test_eig_report(void* G, int s, int kmax, double tol, int force_timeout, void* U, void* lam,
                        void* kkeep, void* inv_sqrt_l0, void* status, void* rec, void* stream);

/* One Cholesky + triangular inverse step of the QR on the parent leg (Sec. III A, Eq.
 * tt_cbc_qr_decomp, realised as Cholesky-QR): G (k x k complex128 Hermitian PSD, overwritten) ->
 * Cinv (k x k complex128, inverse of the lower Cholesky factor; zero rows and columns for dropped
 * pivots); shift_rel adds shift_rel * trace(G) to the diagonal first. ndrop (1 int) receives the
 * number of dropped pivots. tstamp: nullptr or 4 int64 device slots for wall-clock stamps (100 MHz)
 * at: start, factorised, inverted, written (LDS-resident sizes only). */
int cbc_test_chol_inv(void* G, int k, double shift_rel, double drop_rel, void* Cinv, void* ndrop,
                      void* tstamp, void* stream);

#ifdef __cplusplus
}
#endif
#endif
