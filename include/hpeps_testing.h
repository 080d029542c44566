/*
 * hpeps_testing.h -- kernel-level entry points of libhpeps used by the unit
 * parity tests (each exposes one stage of the randomized SVD of Alg. 4 on
 * its own).  Same conventions as hpeps.h: device pointers to dense
 * row-major arrays, batch instances stored back to back, dtype HPEPS_F64 or
 * HPEPS_C128 (complex as interleaved double pairs), work on the context's
 * stream, status codes returned, nothing synchronised.
 */
#ifndef HPEPS_TESTING_H
#define HPEPS_TESTING_H

#include "hpeps.h"

#ifdef __cplusplus
extern "C" {
#endif

/* C[b] = op(A[b]) @ B[b] with A [M,K] (trans_a = 0) or [K,M] read as its
 * (conjugate, for C128) transpose (trans_a = 1), B [K,N], C [M,N].  This is
 * the gathered MFMA GEMM every contraction of the library goes through. */
hpeps_status hpeps_test_gemm(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t batch, int64_t M,
                             int64_t N, int64_t K, int32_t trans_a, const void* A, const void* B,
                             void* C);

/* Orthonormal basis P [n,k] of range(Y) for Y [n,k] (CholeskyQR with the
 * shifted first pass and the conditional third pass, the "orthogonalize" of
 * Alg. 4).  Y is overwritten. */
hpeps_status hpeps_test_orthogonalize(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t batch, int64_t n,
                                      int64_t k, void* Y, void* P);

/* Reshape-avoiding orthogonalization (Alg. 5: Gram matrix, its
 * eigendecomposition, P = Y X Lambda^-1/2), in the two-pass form the
 * einsumsvd runs with HPEPS_ORTH_EIGH (first pass shifted): Q [n,k] to P and
 * R = Q^H Y [k,k] to R, Y [n,k] unchanged.  k <= 128, n >= k. */
hpeps_status hpeps_test_orthogonalize_eigh(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t batch, int64_t n,
                                           int64_t k, const void* Y, void* P, void* R);

/* Householder QR (the orthogonalization fallback for sketches flagged as
 * rank-deficient or very ill-conditioned; tall-skinny, one reduction level)
 * of every instance of Y [n,k] (unchanged): the orthonormal Q [n,k] to P and
 * the upper-triangular R [k,k] (zero below the diagonal) to R, each when
 * non-NULL, Y = Q R.  LAPACK's reflector convention (R's diagonal may be
 * negative; an exactly zero column gives tau = 0).  k <= 128, n >= k. */
hpeps_status hpeps_test_householder(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t batch, int64_t n,
                                    int64_t k, const void* Y, void* P, void* R);

/* Byte budget of one intermediate of an energy strip column (default 1 GiB):
 * larger column transfers run in chunks of the bottom-environment leg,
 * accumulated into the column's output (not while a gradient tape records).
 * Small budgets force the chunked path on small lattices. */
hpeps_status hpeps_test_strip_chunk_bytes(hpeps_ctx* ctx, int64_t bytes);

/* Reverse mode of the norm and energy gradients: on != 0 (the default)
 * checkpoints every zip-up row of the boundary passes (only its input
 * boundary is kept, the row is recomputed in the reverse walk); 0 records
 * every intermediate of every row instead.  Both give the same gradients. */
hpeps_status hpeps_test_checkpoint_rows(hpeps_ctx* ctx, int32_t on);

/* Small SVD stage: for the upper-triangular R [k,k] writes Z [k,k] (left
 * singular vectors of R^H, columns sorted by descending singular value) and
 * sigma [k] (double).  One-sided Jacobi. */
hpeps_status hpeps_test_small_svd(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t batch, int64_t k,
                                  const void* R, void* Z, double* sigma);

/* One application of the zip-up operator (see hpeps_einsumsvd_zipup): with
 * adjoint = 0, Y [rows,k] = A X for X [cols,k]; with adjoint = 1,
 * Y [cols,k] = A^* X for X [rows,k]. */
hpeps_status hpeps_test_zip_apply(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t batch,
                                  const int64_t dims[9], const void* V, const void* S,
                                  const void* T, const void* Bra, int64_t k, int32_t adjoint,
                                  const void* X, void* Y);

/* Forces the launch variant of every following GEMM of the context (tile
 * shape index 0..14, K-step multiple 1 or 2, split-K count or 0 for the
 * heuristic), so that the tests can cover each kernel instantiation;
 * tile = -1 returns to the normal selection.  Unknown or unsupported tile
 * indices fall back to the heuristic. */
hpeps_status hpeps_test_gemm_variant(hpeps_ctx* ctx, int32_t tile, int32_t kstep, int32_t split);

/* Forces the contraction order of the zip-up operator's two middle stages
 * for every following operator application of the context: 0 = chosen by
 * the cost model, 1 = bra stage then boundary stage (intermediate
 * [U,H,u,h,c,j]), 2 = boundary stage then bra stage (intermediate
 * [b,U,h,p,Y,G,j]).  Both orders compute the same product (Table II's
 * network, two contraction sequences). */
hpeps_status hpeps_test_zip_order(hpeps_ctx* ctx, int32_t order);

/* on = 0 sends every later real product with a short reduction (K <= 16,
 * N >= 72) or few rows (M <= 8, N >= 256) and suitably contiguous output
 * columns to the MFMA tile kernel instead of the store-bound short-reduction
 * kernel or the read-bound few-rows kernel; on != 0 restores the default.
 * All compute the same product (different summation order). */
hpeps_status hpeps_test_gemm_smallk(hpeps_ctx* ctx, int32_t on);

#ifdef __cplusplus
}
#endif
#endif /* HPEPS_TESTING_H */
