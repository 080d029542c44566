/*
 * hpeps.h -- C ABI of the MI355X (gfx950) PEPS contraction library.
 *
 * The library implements the bottleneck operation of two-dimensional
 * tensor-network (PEPS) simulation described in Pang, Hao, Dugad, Zhou,
 * Solomonik, "Efficient 2D Tensor Network Simulation of Quantum Systems"
 * (SC20): einsumsvd -- contract a tensor network and refactorize it into two
 * tensors joined by one truncated leg (Sec. II-C) -- computed by randomized
 * SVD on an implicit operator that is only applied through tensor
 * contractions (Alg. 4, Sec. IV-A), and the algorithms built on it:
 * boundary-MPS contraction with zip-up row absorption (Algs. 2-3, two-layer
 * form of Sec. III-B), expectation values with cached environments (Eq. 5,
 * Sec. IV-B) and QR-SVD two-site gate application for imaginary-time
 * evolution (Alg. 1, Eq. 4, Sec. II-D).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every tensor argument is a pointer to caller-owned DEVICE memory holding
 *    a dense row-major array in the leg order written next to it.  Element
 *    type is given by an hpeps_dtype (HPEPS_F64: double; HPEPS_C128: two
 *    doubles, real then imaginary).
 *  - PEPS site tensors have legs [u, d, l, r, p] (up, down, left, right,
 *    physical); legs on the open boundary have dimension 1.
 *  - Boundary-MPS tensors have legs [mL, x, X, mR]: left bond, the ket and
 *    bra legs that connect to the next row to be absorbed, right bond.
 *  - Two-site operators are G[out1, out2, in1, in2] (the index order of the
 *    two-qubit gate of Eq. 2); site 1 is the left (horizontal bond) or the
 *    upper (vertical bond) site.  One-site operators are O[out, in].
 *  - All work is enqueued on the context's stream.  Calls that return host
 *    scalars synchronise that stream; no other call does.  Outputs are
 *    untouched when a call returns an error before launching work.
 *  - The library owns only a workspace arena per context (device memory it
 *    allocates on first use and grows when a larger problem arrives).
 *  - Status codes are returned; no C++ exception crosses the ABI.  One
 *    context must not be used from two host threads at once.
 */
#ifndef HPEPS_H
#define HPEPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HPEPS_OK = 0,
  HPEPS_ERR_INVALID_ARG = 1,  /* null pointer, bad enum, non-positive size   */
  HPEPS_ERR_SHAPE = 2,        /* inconsistent leg dimensions                 */
  HPEPS_ERR_DTYPE = 3,        /* unsupported element type for this call      */
  HPEPS_ERR_ALLOC = 4,        /* device allocation failed / exceeds the cap  */
  HPEPS_ERR_HIP = 5,          /* a HIP runtime call failed                   */
  HPEPS_ERR_NUMERIC = 6,      /* non-finite values met in a factorization    */
  HPEPS_ERR_NOT_CONVERGED = 7,/* Jacobi SVD hit its sweep limit              */
  HPEPS_ERR_UNSUPPORTED = 8   /* size beyond what a kernel supports          */
} hpeps_status;

typedef enum { HPEPS_F64 = 0, HPEPS_C128 = 1, HPEPS_F32 = 2, HPEPS_BF16 = 3 } hpeps_dtype;

/* Where the singular values go in an einsumsvd; U = P Z (Alg. 4) is the
 * isometric left factor, V^* is computed as Sigma^-1 Z^* (P^* A) (row i has
 * relative error ~ 1e-16 * sigma_1 / sigma_i):
 *   CARRY  -> left U, right (Sigma / sigma_1) V^*, and log(sigma_1) is added
 *             to the log-scale accumulator (zip-up carry, see hpeps_peps_norm)
 *   RIGHT  -> left U, right Sigma V^*
 *   NONE   -> left U, right V^*
 *   LEFT   -> left U Sigma, right V^*
 *   SQRT   -> left U Sigma^1/2, right Sigma^1/2 V^* (the split of Alg. 1)
 * The adjoint calls support NONE and RIGHT.                                 */
typedef enum {
  HPEPS_ABSORB_CARRY = 0,
  HPEPS_ABSORB_RIGHT = 1,
  HPEPS_ABSORB_NONE = 2,
  HPEPS_ABSORB_LEFT = 3,
  HPEPS_ABSORB_SQRT = 4
} hpeps_absorb;

typedef struct hpeps_ctx hpeps_ctx;

/* Options of one randomized einsumsvd (Alg. 4).
 *  rank            m: number of singular triplets kept (m' = min(m, k)).
 *  oversample      p: sketch width k = min(m + p, rows, cols).
 *  power_iters     q: Alg. 4's iteration count.
 *  sketch_precision HPEPS_F64 | HPEPS_F32 | HPEPS_BF16: arithmetic of the
 *                  operator applications A X and A^* Y.  FP32 runs the
 *                  contractions on FP32 MFMA with FP32 accumulation; BF16
 *                  rounds the operands and the sketch panels to bfloat16 and
 *                  runs them on BF16 MFMA with FP32 accumulation (intermediate
 *                  stages stored in BF16, the panel fed to the orthogonalization
 *                  in FP64).  Orthogonalization, the small SVD and truncation
 *                  always run in FP64.  FP32 and BF16 are real-only.
 *  seed, stream_id select the sketch: element i of Omega (row-major over
 *                  (column multi-index, sketch column)) is
 *                  2 * (h_i >> 11) * 2^-53 - 1 with h_i = mix(base + (i+1) *
 *                  0x9E3779B97F4A7C15), base = mix(mix(seed) + stream_id) and
 *                  mix the SplitMix64 output function (Steele, Lea & Flood,
 *                  OOPSLA 2014).  Instance b of a batch uses stream_id + b.
 *  jacobi_max_sweeps cap on the one-sided Jacobi sweeps of the small SVD
 *                  (0 selects the default, 40).
 *  orth        how Alg. 4 orthogonalizes its panels.  HPEPS_ORTH_CHOLQR (0,
 *              the default): CholeskyQR with a shifted first pass, a second
 *              pass and a third one for flagged sketches, and a Householder
 *              fallback for numerically rank-deficient ones.  HPEPS_ORTH_EIGH
 *              (1): the reshape-avoiding orthogonalization of Alg. 5
 *              (Sec. V-C) in the same pass structure: per pass the Gram matrix
 *              G = Y^* Y, its eigendecomposition G = X Lambda X^* (from the
 *              Cholesky factor G = C^* C and the one-sided Jacobi SVD of C^*,
 *              accurate to eps kappa(Y)), and P = Y X Lambda^-1/2; the factor
 *              of the final projection is R = P^* Y.  Forward calls only: the
 *              adjoints differentiate the CholeskyQR path and reject 1.
 *  method      HPEPS_ESVD_IMPLICIT (0, the default): the randomized SVD of
 *              Alg. 4 on the implicit operator (IBMPS).  HPEPS_ESVD_EXPLICIT
 *              (1): the network is contracted into its matrix and factored by
 *              a dense truncated SVD (BMPS, Sec. III-B; Table II): the range
 *              basis is exact (the identity when rows <= cols, else the
 *              orthogonalized matrix), then the QR of the projection and the
 *              one-sided Jacobi SVD of its R factor.  oversample,
 *              power_iters, seed and stream_id are then unused;
 *              min(rows, cols) <= 128 (88 complex); FP64 / complex128 only;
 *              forward calls only.  Supported by hpeps_einsumsvd and the
 *              amplitude calls; the others reject it.                       */
enum { HPEPS_ORTH_CHOLQR = 0, HPEPS_ORTH_EIGH = 1 };
enum { HPEPS_ESVD_IMPLICIT = 0, HPEPS_ESVD_EXPLICIT = 1 };

typedef struct {
  int64_t rank;
  int64_t oversample;
  int32_t power_iters;
  int32_t sketch_precision;
  uint64_t seed;
  uint64_t stream_id;
  int32_t jacobi_max_sweeps;
  int32_t orth;           /* HPEPS_ORTH_CHOLQR (0) or HPEPS_ORTH_EIGH (1)     */
  int32_t method;         /* HPEPS_ESVD_IMPLICIT (0) or HPEPS_ESVD_EXPLICIT (1) */
  int32_t reserved;       /* must be 0                                        */
} hpeps_esvd_opts;

/* A strided dense tensor in device memory (the operands of hpeps_einsumsvd). */
typedef struct {
  const void* data;     /* device memory, caller-owned, dtype of the call        */
  int32_t ndim;         /* 1..8                                                  */
  int32_t conj;         /* nonzero: the operand enters complex-conjugated        */
  int64_t shape[8];
  int64_t strides[8];   /* element strides, >= 1 for every leg of extent > 1    */
} hpeps_tensor;

/* Diagnostics of the last einsumsvd-based call (host struct, filled after the
 * call's stream work completes when the call synchronises, else on the next
 * hpeps_get_info). */
typedef struct {
  int64_t rank_kept;        /* m'                                            */
  int64_t sketch_width;     /* k                                             */
  int32_t orth_extra_passes;/* CholeskyQR factorizations that needed a shift */
                            /* and a third pass (ill-conditioned sketches)   */
  int32_t jacobi_sweeps;    /* largest sweep count of any small SVD          */
  int32_t numeric_errors;   /* factorizations that met non-finite values     */
  int32_t not_converged;    /* small SVDs that hit the sweep cap             */
  int32_t orth_householder; /* flagged sketches whose orthogonalization (or  */
                            /* projected factor) was redone by Householder   */
                            /* QR (the fallback of Alg. 4's orthogonalize)   */
  int32_t reserved;
} hpeps_esvd_info;

/* ---- context ---------------------------------------------------------- */
hpeps_status hpeps_create(int device, hpeps_ctx** out);
hpeps_status hpeps_destroy(hpeps_ctx* ctx);
/* stream: a hipStream_t (passed as void*); NULL selects the null stream. */
hpeps_status hpeps_set_stream(hpeps_ctx* ctx, void* stream);
const char* hpeps_status_string(hpeps_status s);
const char* hpeps_last_error(hpeps_ctx* ctx);
/* Caps the workspace arena (bytes; 0 = no cap).  Calls that would need more
 * return HPEPS_ERR_ALLOC before launching anything. */
hpeps_status hpeps_set_workspace_limit(hpeps_ctx* ctx, int64_t bytes);
/* High-water mark of the workspace arena in bytes (device memory the
 * library's calls on this context had in use at once) since creation or the
 * last reset; reset != 0 restarts it from zero afterwards. */
hpeps_status hpeps_workspace_peak(hpeps_ctx* ctx, int64_t* bytes, int32_t reset);
/* Synchronises the stream and copies the diagnostics accumulated since the
 * last call of hpeps_get_info (or creation) to *info, then clears them. */
hpeps_status hpeps_get_info(hpeps_ctx* ctx, hpeps_esvd_info* info);

/* ---- live kernel timing ---------------------------------------------------
 * While profiling is on, every kernel launch of the context whose class name
 * contains `filter` (all launches when filter is NULL or "") is bracketed by
 * two HIP events on the context stream.  Class names:
 * "gemm_<prec>_<BM>x<BN>k<BK>" for the gathered MFMA GEMM with a BM x BN tile
 * and BK-deep K-steps (prec f64, c128, f32, bf16 with FP64 output; f32o32,
 * bf16o16 with FP32 / BF16 output), "chol_inv", "jacobi_svd".  hpeps_profile_read synchronises the stream,
 * writes up to max_entries aggregates (launch count, summed kernel time in
 * ms, summed algorithmic flops -- 2 M N K per product, times 4 for complex --
 * and summed algorithmic operand bytes) and clears the records; profiling
 * stays on until hpeps_profile_stop. */
typedef struct {
  char name[64];
  int64_t launches;
  double ms;
  double flops;
  double bytes;
} hpeps_profile_entry;
hpeps_status hpeps_profile_start(hpeps_ctx* ctx, const char* filter);
hpeps_status hpeps_profile_stop(hpeps_ctx* ctx);
/* on != 0: the GEMM class names of later launches carry the product's shape,
 * "gemm_<prec>_<BM>x<BN>k<BK>_M<M>_N<N>_K<K>_b<batch>", so that products of
 * one kernel variant with different shapes (and bounds) are timed apart;
 * on = 0 returns to the variant names. */
hpeps_status hpeps_profile_by_shape(hpeps_ctx* ctx, int32_t on);
hpeps_status hpeps_profile_read(hpeps_ctx* ctx, int32_t max_entries, hpeps_profile_entry* out,
                                int32_t* n_out);

/* ---- autotuner of the contraction kernels ----------------------------------
 * Each contraction runs as a gathered MFMA GEMM with a tile shape, a K-step
 * (16 or 32) and a split-K count.  By default a size heuristic chooses them.
 * With autotuning on, the first product of every new key (precision, M, N,
 * K, batch, operand layouts) times each variant on the call's own operands
 * and keeps the fastest; later products of that key reuse the choice.  The
 * tuning call synchronises the context stream.  Products that accumulate
 * into their output, whose output overlaps an input, or that are issued
 * during stream capture are never tuned (they use the heuristic).  Results
 * are the same whichever variant runs, up to floating-point summation order
 * (split-K partial sums). */
hpeps_status hpeps_autotune_enable(hpeps_ctx* ctx, int32_t on);
/* The tuned choices as JSON text {"gemm": {"<key>": [tile, kstep, split]}}.
 * Writes at most cap bytes, NUL-terminated, to buf (when buf is non-NULL);
 * *needed receives the full length + 1.  Host memory. */
hpeps_status hpeps_autotune_export(hpeps_ctx* ctx, char* buf, int64_t cap, int64_t* needed);
/* Merges choices from text written by hpeps_autotune_export (a context of
 * the same device type); HPEPS_ERR_INVALID_ARG on malformed text, in which
 * case nothing is merged. */
hpeps_status hpeps_autotune_import(hpeps_ctx* ctx, const char* json);

/* ---- sketch -------------------------------------------------------------
 * Writes the sketch Omega that an einsumsvd with (seed, stream_id) draws:
 * batch blocks of n*k values (block b uses stream_id + b), element i of a
 * block as documented for hpeps_esvd_opts, as double (dtype HPEPS_F64) or
 * rounded to nearest float (HPEPS_F32).  out: device memory. */
hpeps_status hpeps_sketch(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t n, int64_t k, int64_t batch,
                          uint64_t seed, uint64_t stream_id, void* out);

/* ---- einsumsvd of an arbitrary network (Sec. II-C, Alg. 4) --------------
 * The network is written as einsum subscripts over single-letter legs,
 * "<legs of op 0>,<legs of op 1>,...-><row legs>|<column legs>", e.g. the
 * zip-up network "axXbhH,buUc,uyhgp,UYHGp->axX|yYcgG".  Every leg either
 * joins exactly two operands (summed) or belongs to one operand and appears
 * once in the output.  The network is read as the matrix
 * A[(row legs), (column legs)] and factorized A ~ U diag(sigma) V^* by the
 * randomized SVD of Alg. 4 without forming A: the products A X and A^* Y
 * are sequences of pairwise contractions of the network with the k-column
 * sketch panel (next the operand sharing most legs with the running tensor),
 * each one gathered MFMA GEMM; orthogonalization, small SVD, canonical
 * phase, truncation and absorption are those of hpeps_einsumsvd_zipup.
 * Operands: n_ops strided tensors (hpeps_tensor; conj = read conjugated,
 * which is how a bra layer enters).  dtype HPEPS_F64 or HPEPS_C128;
 * opts->sketch_precision must be HPEPS_F64.  Outputs (device, caller-owned,
 * contiguous): U [row legs..., m'], sigma [m'] (may be NULL), R [m', column
 * legs...] per absorb as for the zip-up call; log_scale (device, one
 * double) is incremented by log(sigma_1) in the CARRY mode (may be NULL
 * otherwise).  m' = min(rank, k), k = min(rank + oversample, rows, cols)
 * (hpeps_einsumsvd_query returns rows, cols and m' without launching
 * anything).  Errors: INVALID_ARG for malformed subscripts (a leg used three
 * times, a repeated leg in one operand, no '|'), SHAPE for inconsistent
 * dimensions, DTYPE, UNSUPPORTED for k > 128 (88 complex). */
hpeps_status hpeps_einsumsvd(hpeps_ctx* ctx, hpeps_dtype dtype, const char* subscripts, int32_t n_ops,
                             const hpeps_tensor* ops, const hpeps_esvd_opts* opts, hpeps_absorb absorb,
                             void* U, double* sigma, void* R, double* log_scale);
hpeps_status hpeps_einsumsvd_query(hpeps_ctx* ctx, const char* subscripts, int32_t n_ops,
                                   const hpeps_tensor* ops, const hpeps_esvd_opts* opts, int64_t* rows,
                                   int64_t* cols, int64_t* rank_kept);

/* ---- adjoint of the network einsumsvd (reverse mode, Sec. II-C, Alg. 4) --
 * Gradients of a real loss of the outputs of hpeps_einsumsvd with respect
 * to every operand, for the same subscripts, operands and options (the
 * sketch is held fixed; the CholeskyQR orthogonalization, the small SVD and
 * the canonical phase are differentiated as computed).  dU [row legs...,
 * m'] and dR [m', column legs...] are the cotangents of U and R (device,
 * contiguous, the dtype of the call), dsigma [m'] that of sigma (device
 * double; NULL = 0).  broadening as for hpeps_einsumsvd_pair_backward (the
 * Lorentzian d / (d^2 + broadening * s_1^4), 0 = the exact derivative).
 * grads: n_ops device pointers (host array); grads[i]
 * receives the gradient of operand i, contiguous row-major over that
 * operand's subscript legs (its shape), overwritten; NULL skips operand i.
 * Complex gradients follow the conjugate-Wirtinger convention
 * (dL/dRe + i dL/dIm), which also holds for operands entered conjugated.
 * The k sketched singular values must be nonzero: the reverse walk uses
 * all k right singular vectors V = B Z Sigma^-1 of the projection, so a
 * network of exact rank below k = min(rank + oversample, rows, cols) gives
 * unbounded gradients (keep rank + oversample within the network's rank).
 * Absorb modes NONE and RIGHT (others UNSUPPORTED); method IMPLICIT and orth
 * CHOLQR only; errors otherwise as hpeps_einsumsvd. */
hpeps_status hpeps_einsumsvd_backward(hpeps_ctx* ctx, hpeps_dtype dtype, const char* subscripts, int32_t n_ops,
                                      const hpeps_tensor* ops, const hpeps_esvd_opts* opts, hpeps_absorb absorb,
                                      double broadening, const void* dU, const double* dsigma, const void* dR,
                                      void* const* grads);

/* ---- batched einsumsvd of an arbitrary network (Sec. II-C, Alg. 4) ------
 * `batch` independent instances of the network of hpeps_einsumsvd, each
 * factorized on its own.  Every operand has one more dimension than its
 * subscript term, the leading one, of extent `batch`; its stride is the
 * instance stride and must be at least one instance's extent (instances are
 * disjoint; a stride that does not meet this is SHAPE).  The subscripts
 * name only the per-instance legs.  Instance b draws its sketch from stream
 * opts->stream_id + b, so it equals hpeps_einsumsvd on that instance's
 * operands with stream_id + b.  Each product of the network runs once for
 * all instances (one batched gathered GEMM), and so does every later stage.
 * Outputs (device, caller-owned, contiguous): U [batch][row legs..., m'],
 * sigma [batch][m'] (may be NULL), R [batch][m'][column legs...];
 * log_scale [batch] for the CARRY mode.  batch < 1 is INVALID_ARG; other
 * errors as for hpeps_einsumsvd. */
hpeps_status hpeps_einsumsvd_batched(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t batch, const char* subscripts,
                                     int32_t n_ops, const hpeps_tensor* ops, const hpeps_esvd_opts* opts,
                                     hpeps_absorb absorb, void* U, double* sigma, void* R, double* log_scale);

/* ---- einsumsvd on the zip-up network (Alg. 3 inner step, Alg. 4) -------
 * One einsumsvd of boundary contraction: the carry V[a,x,X,b,h,H] of the
 * previous column, the boundary tensor S[b,u,U,c], the ket site
 * T[u,y,h,g,p] and the bra site Bra[U,Y,H,G,p] (used complex-conjugated;
 * NULL means Bra = T) define the implicit matrix
 *     A[(a,x,X), (y,Y,c,g,G)] = sum_{b,h,H,u,U,p} V S T conj(Bra),
 * which is never formed.  Randomized SVD A ~ U Sigma V^* with the options in
 * *opts; outputs:
 *     U      [batch][a, x, X, m']           left factor (isometry)
 *     sigma  [batch][m'] (device, double)   singular values, descending
 *     R      [batch][m', y, Y, c, g, G]     right factor per *absorb*
 *     log_scale [batch] (device, double)    incremented by log(sigma_1)
 *                                           when absorb == CARRY (may be
 *                                           NULL otherwise)
 * dims = {a, x, b, h, u, c, y, g, d}.  Tensors of instance i start at
 * i * (element count of one instance).  dtype: HPEPS_F64 or HPEPS_C128.
 * Errors: SHAPE if k = min(m+p, rows, cols) exceeds 128 (F64) / 88 (C128). */
hpeps_status hpeps_einsumsvd_zipup(hpeps_ctx* ctx, int64_t batch, hpeps_dtype dtype,
                                   const int64_t dims[9], const void* V, const void* S,
                                   const void* T, const void* Bra,
                                   const hpeps_esvd_opts* opts, hpeps_absorb absorb,
                                   void* U, double* sigma, void* R, double* log_scale);

/* ---- einsumsvd on the two-column pair network --------------------------
 * Two adjacent boundary tensors Bl[a,u,U,b], Br[b,v,V,c] (each [m,D,D,m]) and
 * two horizontally adjacent sites T1[u,x,1,h,p], T2[v,y,h,1,q] (outer
 * horizontal legs of dim 1; bra = conj(ket)) define
 *     A[(a,x,X), (y,Y,c)] = sum Bl Br T1 conj(T1) T2 conj(T2)      (Fig. 2b)
 * The carry sum_{u,U,p} Bl T1 conj(T1) is contracted exactly first, then the
 * randomized SVD runs as in hpeps_einsumsvd_zipup with g = G = 1.
 *     U [batch][m, D, D, m'], sigma [batch][m'], R [batch][m', D, D, m]
 * dims = {m, D, d}. */
hpeps_status hpeps_einsumsvd_pair(hpeps_ctx* ctx, int64_t batch, hpeps_dtype dtype,
                                  const int64_t dims[3], const void* Bl, const void* Br,
                                  const void* T1, const void* T2,
                                  const hpeps_esvd_opts* opts, hpeps_absorb absorb,
                                  void* U, double* sigma, void* R);

/* ---- adjoint of the pair einsumsvd (reverse mode) -------------------------
 * Vector-Jacobian product of hpeps_einsumsvd_pair with the sketch held fixed.
 * The paper differentiates nothing; this is the derivative of Alg. 4 as it
 * runs (every CholeskyQR and the small SVD differentiated), for optimizing
 * PEPS tensors against quantities built from the einsumsvd outputs.  Given
 * the cotangents of the outputs
 *     dU [batch][m, D, D, m'], dsigma [batch][m'] (device double; NULL = 0),
 *     dR [batch][m', D, D, m]
 * it writes the gradients of the real loss into gBl, gBr, gT1, gT2 (device,
 * caller-owned, the shapes of Bl, Br, T1, T2, overwritten); complex tensors
 * get the conjugate Wirtinger gradient dL/dRe + i dL/dIm.  The forward pass
 * is recomputed inside the call from the same inputs and opts (same sketch,
 * same outputs), then the reverse sweep runs on the GPU: truncated-SVD
 * backward, CholeskyQR backward of every orthogonalization, the adjoint of
 * every operator application, and the contraction of the operator cotangent
 * with the network for each tensor.  The 1 / (s_j^2 - s_i^2) factors of the
 * SVD backward are Lorentzian-broadened, d / (d^2 + broadening * s_1^4) with
 * d = s_j^2 - s_i^2 (0 where d = 0); broadening = 0 gives the exact
 * derivative, a small value (1e-12) bounds the gradient of (near-)degenerate
 * spectra.  The result is the exact derivative of the algorithm, the
 * canonical phase choice of the singular pairs included.
 *   absorb: HPEPS_ABSORB_NONE or RIGHT, as in the forward call; the
 *   sketch_precision of opts must be HPEPS_F64.  Workspace: a few times the
 *   forward call's (all panels of the power iteration are kept).
 * Errors: as hpeps_einsumsvd_pair; HPEPS_ERR_UNSUPPORTED for the CARRY mode,
 * HPEPS_ERR_DTYPE for a non-FP64 sketch, HPEPS_ERR_INVALID_ARG for a
 * negative broadening. */
hpeps_status hpeps_einsumsvd_pair_backward(hpeps_ctx* ctx, int64_t batch, hpeps_dtype dtype,
                                           const int64_t dims[3], const void* Bl, const void* Br,
                                           const void* T1, const void* T2,
                                           const hpeps_esvd_opts* opts, hpeps_absorb absorb,
                                           double broadening, const void* dU, const double* dsigma,
                                           const void* dR, void* gBl, void* gBr, void* gT1,
                                           void* gT2);

/* ---- PEPS and boundary-MPS containers ---------------------------------- */
typedef struct {
  int32_t nrow, ncol;
  int32_t dtype;              /* HPEPS_F64 or HPEPS_C128, all sites        */
  int32_t reserved;
  void* const* sites;         /* nrow*ncol device pointers, row-major      */
  const int64_t* shapes;      /* host, nrow*ncol*5: [u,d,l,r,p] per site   */
} hpeps_peps;

typedef struct {
  int32_t ncol;
  int32_t dtype;
  void* const* tensors;       /* ncol device pointers [mL, x, X, mR]       */
  int64_t* shapes;            /* host, ncol*4 (written for outputs)        */
  const int64_t* capacity;    /* host, ncol: element capacity of each      */
                              /* output buffer (NULL for inputs)           */
} hpeps_bmps;

typedef enum { HPEPS_L2R = 0, HPEPS_R2L = 1 } hpeps_direction;

/* ---- boundary_contract_row (ApproxApply, Alg. 3) ------------------------
 * Absorbs one PEPS row (ket row, bra row = NULL for conj(ket)) into the
 * boundary MPS *bnd (legs x/X of bnd connect to the up legs u/U of the row)
 * by the zip-up: the first column's carry is exact, every later column runs
 * one einsumsvd (ABSORB_CARRY).  dir selects the sweep direction.  The new
 * boundary (legs x/X = down legs of the row) goes to *out, whose buffers
 * the caller allocates; shapes are written to out->shapes.  *log_scale (host)
 * is incremented by the logarithms of all normalisation factors (the first
 * carry's Frobenius norm and every sigma_1).  Stream ids follow
 * opts->stream_id + column index.  Synchronises (returns a host scalar). */
hpeps_status hpeps_boundary_contract_row(hpeps_ctx* ctx, const hpeps_bmps* bnd,
                                         const hpeps_peps* ket, const hpeps_peps* bra,
                                         int32_t row, hpeps_direction dir,
                                         const hpeps_esvd_opts* opts, hpeps_bmps* out,
                                         double* log_scale);

/* ---- peps_norm (boundary MPS, Alg. 2) -----------------------------------
 * <bra|ket> (bra = NULL: <ket|ket>) of a two-layer PEPS network.  Site
 * tensors are rescaled to unit Frobenius norm, row 1 is the exact boundary,
 * rows 2..n-1 are absorbed by zip-ups whose direction alternates (L2R on the
 * 1st, 3rd, ... absorbed row), row n is contracted exactly.  The sketch of
 * the einsumsvd absorbing column j of row i uses stream_id
 * 1 + (i * ncol + j) (opts->stream_id is ignored).
 * Result: value = phase * exp(*log_norm); phase = {re, im} (host). */
hpeps_status hpeps_peps_norm(hpeps_ctx* ctx, const hpeps_peps* ket, const hpeps_peps* bra,
                             const hpeps_esvd_opts* opts, double* log_norm, double* phase);

/* ---- peps_amplitude (one-layer boundary MPS, Sec. III with Algs. 2-4) ----
 * <bits|psi>: every physical leg of the ket is fixed to bits[i*ncol + j]
 * (host, row-major over the sites, 0 <= bit < p), which leaves a one-layer
 * network of [u,d,l,r] slices (gathered into the workspace).
 * Row 1 is the exact boundary [l, d, r] (each tensor normalised), rows
 * 2..n-1 are absorbed by zip-ups whose direction alternates (L2R on the
 * 1st, 3rd, ... absorbed row): the first column's carry is exact, every
 * later column is one randomized einsumsvd of the network
 * "axbh,buc,uyhg->ax|ycg" (carry, boundary tensor, slice; rows (a,x),
 * columns (y,c,g)) with the options of opts (sketch_precision HPEPS_F64;
 * stream_id 1 + (i*ncol + j) for lattice row i, column j), row n is
 * contracted exactly.  Result (host): <bits|psi> = phase * exp(*log_abs),
 * phase = {re, im} of unit modulus; an exactly zero slice gives
 * *log_abs = -inf and phase = {0, 0}.  Errors: INVALID_ARG (bit out of
 * range, null pointers, bad options), SHAPE (inconsistent bonds), DTYPE
 * (sketch precision other than FP64), NUMERIC (a non-finite result, e.g. an
 * exactly zero boundary from nonzero slices).  Synchronises. */
hpeps_status hpeps_peps_amplitude(hpeps_ctx* ctx, const hpeps_peps* ket, const int32_t* bits,
                                  const hpeps_esvd_opts* opts, double* log_abs, double* phase);

/* ---- peps_amplitudes (the same for a batch of basis states) --------------
 * n_states basis states (1..65535), bits[t*nsites + i*ncol + j] (host); every
 * state's amplitude is computed exactly as by hpeps_peps_amplitude (same
 * sketch streams), all states in lockstep: their slices are gathered into
 * one batch and every kernel launch of the contraction carries the whole
 * batch.  Outputs (host): log_abs[n_states], phase[2*n_states].  A bit out of
 * range fails the whole call (INVALID_ARG) before any launch; a non-finite
 * amplitude of any state fails it with NUMERIC.  Synchronises. */
hpeps_status hpeps_peps_amplitudes(hpeps_ctx* ctx, const hpeps_peps* ket, int64_t n_states,
                                   const int32_t* bits, const hpeps_esvd_opts* opts, double* log_abs,
                                   double* phase);

/* ---- peps_energy (Eq. 5 with cached environments, Sec. IV-B) ------------
 * Terms: n_terms entries; term t acts on nsites[t] (1 or 2) sites given by
 * sites[4t .. 4t+3] = {i1, j1, i2, j2} (nearest neighbours, site 1 left of or
 * above site 2, or diagonal neighbours i2 = i1 + 1, j2 = j1 +- 1: the J2
 * pairs of Eq. 7); its operator (host memory, complex128 as interleaved
 * {re, im} pairs, [2,2] or [2,2,2,2]) starts op_offset[t] complex entries
 * into ops, i.e. at the double ops + 2 * op_offset[t]; the call reads up to
 * the end of the operator that ends last.  Every term value is
 * strip(term)/strip(id), where the strip is the exact contraction of the
 * cached top environment, the one (two, for vertical and diagonal terms) PEPS
 * rows of the term and the cached bottom environment; a diagonal term spans
 * two columns of its strip.  (hpeps_peps_energy_uncached and
 * hpeps_peps_energy_backward take nearest-neighbour terms only.)  Environments come from two full boundary passes
 * (top-down stream ids 1 + (i*ncol+j), bottom-up 1 + ((nrow+i)*ncol+j)).
 * Outputs (host): energy[2] = {re, im} of the sum, per_term[2*n_terms]
 * (may be NULL).  Synchronises. */
hpeps_status hpeps_peps_energy(hpeps_ctx* ctx, const hpeps_peps* ket, int32_t n_terms,
                               const int32_t* nsites, const int32_t* sites,
                               const double* ops, const int64_t* op_offset,
                               const hpeps_esvd_opts* opts, double* energy, double* per_term);

/* hpeps_peps_energy_uncached: Eq. 5 without the caching of Sec. IV-B, the
 * baseline the cached call is measured against.  Every term is its own full
 * boundary-MPS contraction <psi|H_t psi> / <psi|psi>, with H_t applied to the
 * ket exactly: a one-site operator on its site's physical leg; a two-site
 * operator G[P,Q,p,q] (out1, out2, in1, in2) by the elementary split
 * G = sum_{Q,q} G[:,Q,:,q] (x) |Q><q| -- site 1 takes G[:,Q,:,q], site 2
 * takes |Q><q|, and (Q, q) is appended to their shared bond (new index
 * (b, Q, q) row-major: the bond grows from D to D d^2) -- and the bra
 * zero-padded to the grown bond, which leaves the overlap unchanged.  Same
 * arguments and outputs as hpeps_peps_energy (a real PEPS takes real
 * operators only: HPEPS_ERR_DTYPE otherwise); n_terms + 1 contractions, all
 * with the stream ids of hpeps_peps_norm.  Synchronises. */
hpeps_status hpeps_peps_energy_uncached(hpeps_ctx* ctx, const hpeps_peps* ket, int32_t n_terms,
                                        const int32_t* nsites, const int32_t* sites,
                                        const double* ops, const int64_t* op_offset,
                                        const hpeps_esvd_opts* opts, double* energy, double* per_term);

/* hpeps_peps_trotter_expectation: the Trotter-Taylor estimate of Eq. 6,
 * <H> ~ (<psi| prod_j G_j |psi> / <psi|psi> - 1) / tau with G_j = e^{tau H_j}
 * supplied by the caller: n_gates nearest-neighbour gates, sites[4*j] =
 * (i1, j1, i2, j2) (site 1 left of / above site 2), gates (host, complex128
 * pairs) [n_gates][d,d,d,d] (out1, out2, in1, in2).  phi = prod_j G_j psi is
 * applied exactly, gate by gate in the order given (the elementary split of
 * hpeps_peps_energy_uncached: every bond a gate touches grows by d^2), and
 * <psi|phi> is one boundary contraction against the zero-padded psi, beside
 * the contraction of <psi|psi>.  Outputs (host): estimate[2] = {re, im},
 * ratio[2] = <psi|phi> / <psi|psi> (may be NULL).  Synchronises. */
hpeps_status hpeps_peps_trotter_expectation(hpeps_ctx* ctx, const hpeps_peps* ket, int32_t n_gates,
                                            const int32_t* sites, const double* gates, double tau,
                                            const hpeps_esvd_opts* opts, double* estimate, double* ratio);

/* ---- gradients of peps_norm / peps_energy (reverse mode) -----------------
 * The paper evaluates these quantities; it does not differentiate them.
 * These calls give their gradients with respect to every site tensor, for
 * variational optimisation of the PEPS: the forward contraction runs once
 * while a reverse-mode tape records every product, exact carry and
 * einsumsvd (with the FP64 sketch, same stream ids as the forward call), then
 * the tape is walked backwards on the GPU.  Each einsumsvd's adjoint
 * recomputes its own power iteration from the kept inputs (checkpoint and
 * recompute per einsumsvd; boundary tensors and carries stay in the
 * workspace).  The Frobenius and sigma_1 rescalings are constants of the
 * derivative: the energy is a ratio and log<psi|psi> a log-derivative, so
 * neither depends on them.  Derivatives of the canonical phase of every
 * singular pair are included.  broadening: Lorentzian width of the SVD
 * backward, as in hpeps_einsumsvd_pair_backward (0 = exact).
 *   grads: nrow*ncol device pointers (row-major over sites), each a
 *   caller-owned buffer with the shape and dtype of its site, overwritten
 *   with dL/dRe + i dL/dIm.  Workspace grows with the whole contraction
 *   (every boundary tensor, carry and strip intermediate is kept).
 * hpeps_peps_norm_backward: L = log<psi|psi> (bra = ket), value to
 *   *log_norm.
 * hpeps_peps_energy_backward: L = Re E with E the energy of
 *   hpeps_peps_energy (same term arguments), E to energy[2].
 * Both synchronise.  Errors as the forward calls; HPEPS_ERR_INVALID_ARG for
 * a null gradient pointer or a negative broadening. */
hpeps_status hpeps_peps_norm_backward(hpeps_ctx* ctx, const hpeps_peps* ket,
                                      const hpeps_esvd_opts* opts, double broadening,
                                      void* const* grads, double* log_norm);
hpeps_status hpeps_peps_energy_backward(hpeps_ctx* ctx, const hpeps_peps* ket, int32_t n_terms,
                                        const int32_t* nsites, const int32_t* sites,
                                        const double* ops, const int64_t* op_offset,
                                        const hpeps_esvd_opts* opts, double broadening,
                                        void* const* grads, double* energy);

/* ---- apply_two_site_gate (QR-SVD, Alg. 1 / Eq. 4) -----------------------
 * In place on two neighbouring sites of *peps: site (i,j) and its right
 * neighbour (axis 0) or lower neighbour (axis 1).  Each site is matricized
 * as (other legs) x (shared bond, p) and QR-factored (skipped when it has no
 * more rows than columns); Theta = G R1 R2 is decomposed by an exact SVD,
 * truncated to D' = min(max_rank, rows, cols), the kept singular values are
 * normalised to unit 2-norm and split as sqrt into both sides, and the Q
 * factors are multiplied back.  The site buffers must have room for the new
 * bond (capacity given in elements); the new shapes are written to
 * peps->shapes (which must then be writable: pass a non-const array).
 * sigma_out (device, may be NULL) receives the D' kept values.
 * Synchronises (returns the new bond on the host). */
/* ---- one-site operator (Eq. 3) --------------------------------------------
 * out[u,d,l,r,P] = sum_p G[P,p] site[u,d,l,r,p] for one site tensor of
 * shape dims[5] (row-major, device, dtype HPEPS_F64 or HPEPS_C128) and the
 * device d x d gate G (same dtype); out (device, same shape) may alias site.
 * Asynchronous on the context stream. */
hpeps_status hpeps_apply_one_site_gate(hpeps_ctx* ctx, hpeps_dtype dtype, const int64_t* dims,
                                       const void* site, const void* G, void* out);

hpeps_status hpeps_apply_two_site_gate(hpeps_ctx* ctx, hpeps_peps* peps,
                                       const int64_t* capacity, int32_t i, int32_t j,
                                       int32_t axis, const void* G, int64_t max_rank,
                                       int64_t* new_bond, double* sigma_out);

/* ---- apply_two_site_gate without allocation -----------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * update, arguments, layouts, results and errors as hpeps_apply_two_site_gate,
 * but every device buffer the call needs beyond the caller's sites, gate and
 * sigma_out (staging copies of the two sites, the dimension and bond tables, the
 * gate, the singular values) comes from a static
 * 1 MiB array in the library's device image, one per GPU, resolved when a
 * context is created on that GPU.  The call makes no hipMalloc / hipFree and
 * no allocating library call.  Sizes whose buffers exceed the static array
 * (2 max_rank^4 d doubles for the two sites plus small tables, 256-byte
 * aligned)
 * return HPEPS_ERR_ALLOC before anything is enqueued; every size the
 * QR-SVD kernel supports fits.  All calls on one GPU share that array: calls
 * that overlap in time on one GPU (from several host threads or contexts)
 * race and must be serialised by the caller.  Synchronises. */
hpeps_status hpeps_apply_two_site_gate_noalloc(hpeps_ctx* ctx, hpeps_peps* peps,
                                               const int64_t* capacity, int32_t i, int32_t j,
                                               int32_t axis, const void* G, int64_t max_rank,
                                               int64_t* new_bond, double* sigma_out);

/* ---- batched imaginary-time-evolution sweep (TEBD, Sec. II-D) -----------
 * A plan owns the evolving PEPS in a device arena of fixed capacity
 * max_rank per bond.  Each sweep applies the gate of every bond, layer by
 * layer (horizontal bonds at even then odd columns, vertical bonds at even
 * then odd rows), with one launch per layer in which every bond of the
 * layer is processed by its own workgroup; bond dimensions live in a device
 * table so the sweeps replay as one captured HIP graph.
 *  gates: n_gates device [2,2,2,2] operators (dtype of the plan);
 *  bond_gate: host, one gate index per bond in layer order (sizes of the
 *             layers: nrow*ceil((ncol-1)/2), nrow*floor((ncol-1)/2),
 *             ceil((nrow-1)/2)*ncol, floor((nrow-1)/2)*ncol).
 * The initial state is copied from *init (any bond dims <= max_rank). */
typedef struct hpeps_ite_plan hpeps_ite_plan;
hpeps_status hpeps_ite_plan_create(hpeps_ctx* ctx, const hpeps_peps* init,
                                   int32_t n_gates, const void* gates,
                                   const int32_t* bond_gate, int64_t max_rank,
                                   hpeps_ite_plan** out);
/* A plan over an arbitrary gate list (the TEBD sweep of a Hamiltonian with
 * further-neighbour terms, such as the diagonal J2 bonds of Eq. 7, or the
 * layers of a quantum circuit): n_ops operations, ops[6*t] = (kind, i1, j1,
 * i2, j2, gate): kind 2 applies the two-site gate gates2[gate] ([d,d,d,d],
 * out1, out2, in1, in2, FP64 host) to sites (i1, j1), (i2, j2) by the QR-SVD
 * update of Alg. 1 with bonds truncated to max_rank; kind 1 applies the
 * one-site gate gates1[gate] ([d,d], out, in, FP64 host) to site (i1, j1) as
 * in Eq. 3 (i2, j2 ignored).  Two-site gates on sites that are not nearest
 * neighbours run as SWAP chains (Sec. II-C): site 2's state is moved by SWAP
 * gates along its row to site 1's column, then along that column until it
 * neighbours site 1, the gate acts there (transposed when site 2 ends up
 * left of or above site 1), and the SWAPs are undone in reverse order; every
 * SWAP is itself a truncating QR-SVD update.  The operations are packed into
 * layers (each one in the first layer after the last one touching its
 * sites; one-site and two-site operations in separate layers), one launch
 * per layer, and a sweep runs the whole list; hpeps_ite_run,
 * hpeps_ite_spectra (two-site updates in layer order, SWAPs included),
 * hpeps_ite_get_state and hpeps_ite_plan_destroy take the plan.  d <= 8. */
hpeps_status hpeps_circuit_plan_create(hpeps_ctx* ctx, const hpeps_peps* init, int32_t n_gates2,
                                       const double* gates2, int32_t n_gates1, const double* gates1,
                                       int32_t n_ops, const int32_t* ops, int64_t max_rank,
                                       hpeps_ite_plan** out);
/* Number of layers of a plan's sweep and of its two-site updates (the rows
 * of hpeps_ite_spectra). */
hpeps_status hpeps_ite_plan_layers(hpeps_ite_plan* plan, int32_t* n_layers, int32_t* n_bonds);
/* Runs n_sweeps sweeps: use_graph = 1 replays the captured graph of the
 * layer launches, 0 issues the layer launches directly, 2 is the plain
 * form with one launch per bond (no graph; the baseline of the batched
 * forms).  All three compute the same updates; other values of use_graph
 * (and n_sweeps < 0) return INVALID_ARG. */
hpeps_status hpeps_ite_run(hpeps_ite_plan* plan, int32_t n_sweeps, int32_t use_graph);
/* Kept singular values of every bond update of the most recent sweep (Alg. 1
 * step: the truncated spectrum of Theta normalised to unit 2-norm), bond by
 * bond in layer order (the order of bond_gate), max_rank values per bond,
 * zero past the bond's new dimension: n_bonds * max_rank doubles copied to
 * the caller's device buffer out on the context stream (not synchronised).
 * Zeros before the first sweep. */
hpeps_status hpeps_ite_spectra(hpeps_ite_plan* plan, double* out);
/* Copies the current state out: shapes (host, nrow*ncol*5) and, when sites
 * is not NULL, the tensors into caller buffers (device pointers, each with
 * room for max_rank-bond shapes). Synchronises. */
hpeps_status hpeps_ite_get_state(hpeps_ite_plan* plan, int64_t* shapes, void* const* sites);
hpeps_status hpeps_ite_plan_destroy(hpeps_ite_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* HPEPS_H */
