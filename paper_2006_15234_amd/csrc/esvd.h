// einsumsvd internals shared by the ABI entry points and the boundary code.
#pragma once
#include <functional>
#include <utility>
#include "internal.h"

namespace hp {

// Leg dimensions of one zip-up einsumsvd: carry V[a,x,X,b,h,H], boundary
// S[b,u,U,c], ket T[u,y,h,g,p] and bra Bra[U,Y,H,G,p] (bra dims = ket dims).
struct ZipDims {
  int64_t a = 1, x = 1, b = 1, h = 1, u = 1, c = 1, y = 1, g = 1, d = 1;
  int64_t rows() const;
  int64_t cols() const;
  int64_t v_size() const;
  int64_t s_size() const;
  int64_t t_size() const;
};

// Element strides of every leg of the four operands (any permutation of the
// stored legs: mirrored sweeps are stride permutations) and the per-instance
// extents used for bounds checks and batch strides.
struct ZipLayout {
  int64_t V[6];  // a, x, X, b, h, H
  int64_t S[4];  // b, u, U, c
  int64_t T[5];  // u, y, h, g, p
  int64_t B[5];  // U, Y, H, G, p
  int64_t nV = 0, nS = 0, nT = 0, nB = 0;
  static ZipLayout row_major(const ZipDims& z);
};

struct ZipOperands {
  const void* V = nullptr;
  const void* S = nullptr;
  const void* T = nullptr;
  const void* Bra = nullptr;
};

struct ZipWork {
  void* W1 = nullptr;
  void* W2 = nullptr;
  void* W3 = nullptr;
};

struct OrthWork {
  double* G = nullptr;
  double* Rinv = nullptr;
  double* Racc = nullptr;
  int* flags = nullptr;
  int mode = HPEPS_ORTH_CHOLQR;  // or HPEPS_ORTH_EIGH (Alg. 5)
};

// Output placement of the two factors: U[(a,x,X), i] at Urows + Ucol(i),
// R[i, (y,Y,c,g,G)] at Rrow(i) + Rcols; extents per instance.
struct ZipOut {
  IndexMap Urows, Ucol, Rrow, Rcols;
  int64_t nU = 0, nR = 0;
  static ZipOut row_major(const ZipDims& z, int64_t mp);
};

// Contraction order of the middle two stages of an operator application.
// Classic: bra then boundary, through W2 [U,H,u,h,c,j] (D^4 m k values);
// BoundaryFirst: boundary then bra, through Z [b,U,h,p,Y,G,j] (m d D^3 k
// values for the pair network) at d D^5 m^2 k instead of d D^6 m k +
// D^4 m^2 k flops -- the smaller intermediate pays off where the stages are
// bound by HBM traffic rather than by MFMA work.  Auto asks zip_order.
enum class ZipOrder { Auto, Classic, BoundaryFirst };
ZipOrder zip_order(const Ctx& ctx, Prec prec, const ZipDims& z, int64_t k, int batch);
// element count of the W2 work buffer (large enough for either order)
int64_t zip_w2_elems(const ZipDims& z, int64_t k);

// A X (adjoint = false, X: cols x k) or A^* X (X: rows x k) for the zip-up
// operator; Y is written as double when y_f64 (F32 applies), else in the
// apply precision.  With Y == nullptr (classic order only) the last stage is
// skipped and the first three stages' results stay in w (forward: W1
// [u,h,p,Y,c,G,j], W2 [U,H,u,h,c,j], W3 [b,h,H,j]; adjoint: W3, W2 as
// forward, W1 [Y,G,p,u,h,c,j]).
void zip_apply(Ctx& ctx, Prec prec, const ZipDims& z, const ZipLayout& L, const ZipOperands& op,
               int batch, int64_t k, bool adjoint, const void* X, void* Y, bool y_f64,
               const ZipWork& w, ZipOrder order = ZipOrder::Auto);

void orthogonalize(Ctx& ctx, bool cplx, double* Y, double* P, int64_t n, int64_t k, int batch,
                   const OrthWork& w, double* Rt_inv = nullptr);
// R factor of the CholeskyQR of Y (accumulated over the passes) into w.Racc;
// S1, S2: n x k scratch panels
void cholqr_r(Ctx& ctx, bool cplx, const double* Y, double* S1, double* S2, int64_t n, int64_t k,
              int batch, const OrthWork& w);

int64_t sketch_width(int64_t m, int64_t p, int64_t rows, int64_t cols);

// A X (adj = false, X: cols x k) or A^* X (adj = true, X: rows x k) of an
// implicit operator, FP64 / complex128 panels, row-major per instance.
using ApplyFn = std::function<void(bool adj, const double* X, double* Y)>;
// Rank-k terms (L_t, R_t) of an operator cotangent Abar = sum_t L_t R_t^H.
using RankTerms = std::vector<std::pair<const double*, const double*>>;

struct ZipOut;
// Alg. 4 from the first product Y0 = A Omega on (orthogonalizations, power
// iterations, projection, small SVD, canonical phase, factors).
void rsvd_finish(Ctx& ctx, bool cplx, int64_t rows, int64_t cols, int64_t k, int64_t mp, int batch,
                 const hpeps_esvd_opts& o, hpeps_absorb absorb, const ZipOut& out, void* U, double* sigma,
                 void* R, double* log_scale, double* Y0, const ApplyFn& apply);
// Truncated SVD of explicit matrices (BMPS's einsumsvd): M = A^* as
// [batch][cols][rows] when rows <= cols, else M = A as [batch][rows][cols]
// (overwritten), whose projection A^* P adj_apply(true, P, out) computes.
// k = min(rows, cols) <= 128 (88 complex).
void dense_finish(Ctx& ctx, bool cplx, int64_t rows, int64_t cols, int64_t mp, int batch, const hpeps_esvd_opts& o,
                  hpeps_absorb absorb, const ZipOut& out, void* U, double* sigma, void* R, double* log_scale,
                  double* M, const ApplyFn& adj_apply);

// Randomized einsumsvd (Alg. 4) of the zip-up operator; operands are FP64 /
// complex128 device arrays (instances back to back with the extents of L).
void zip_esvd(Ctx& ctx, bool cplx, const ZipDims& z, const ZipLayout& L, const ZipOperands& op,
              int batch, const hpeps_esvd_opts& o, hpeps_absorb absorb, const ZipOut& out,
              void* U, double* sigma, void* R, double* log_scale);

// einsumsvd of an arbitrary network given by subscripts ("ab,bc->a|c"):
// rows are the open legs left of '|', columns those right of it; FP64 /
// complex128.  U [rows, m'] and R [m', cols] row-major.  batch 0: one
// network; batch >= 1: every operand has a leading instance dimension and
// the outputs are [batch][...] (sigma [batch][m'], log_scale [batch]).
void einsumsvd_network(Ctx& ctx, bool cplx, const char* subscripts, int n_ops, const hpeps_tensor* ops,
                       const hpeps_esvd_opts& o, hpeps_absorb absorb, void* U, double* sigma, void* R,
                       double* log_scale, int64_t batch = 0);
// Reverse mode of Alg. 4 up to the operator (see esvd_grad.hip): recomputes
// the forward pass through `apply` and appends the operator cotangent's
// rank-k terms to `terms` (buffers in the caller's workspace scope).
void rsvd_backward_terms(Ctx& ctx, bool cplx, int64_t rows, int64_t cols, int batch, const hpeps_esvd_opts& o,
                         hpeps_absorb absorb, double broadening, const ZipOut& out, const void* dU,
                         const double* dsigma, const void* dR, const ApplyFn& apply, RankTerms& terms);
// Adjoint of einsumsvd_network (batch 0: one network): gradients of every
// operand (grads[i] row-major over operand i's legs, [batch] first when
// batched; NULL skips it) for the output cotangents dU, dsigma, dR.
void einsumsvd_network_backward(Ctx& ctx, bool cplx, const char* subscripts, int n_ops, const hpeps_tensor* ops,
                                const hpeps_esvd_opts& o, hpeps_absorb absorb, double broadening, const void* dU,
                                const double* dsigma, const void* dR, void* const* grads, int64_t batch = 0);
void einsumsvd_query(const char* subscripts, int n_ops, const hpeps_tensor* ops, const hpeps_esvd_opts& o,
                     int64_t* rows, int64_t* cols, int64_t* rank);

// Exact carry V[a,x,X,b,h,H] = sum_{u,U,p} L[a,u,U,b] T[u,x,h,p] conj(Bra[U,X,H,p])
// (the left leg of T and Bra has dim 1 and is skipped); V is row-major.
struct CarryDims {
  int64_t a = 1, u = 1, b = 1, x = 1, h = 1, d = 1;
};
struct CarryLayout {
  int64_t L[4];  // a, u, U, b
  int64_t T[4];  // u, x, h, p
  int64_t B[4];  // U, X, H, p
  int64_t nL = 0, nT = 0, nB = 0;
  static CarryLayout row_major(const CarryDims& c);  // T, Bra stored [u,x,1,h,p]
};
void form_carry(Ctx& ctx, bool cplx, const CarryDims& cd, const CarryLayout& cl, const void* L,
                const void* T, const void* Bra, void* V, int batch);

// Adjoint of zip_esvd (FP64 / complex128 sketch): cotangents of U, sigma
// (NULL = 0) and R, stored with the placement of `out`, are turned into the
// gradients of V, S, T, Bra (layouts of L), ACCUMULATED into gV, gS, gT, gBra
// (gT and gBra may alias).  CARRY treats s_1 as a constant (the carry scale
// only moves the logarithmic accumulator).  broadening: Lorentzian width of
// the 1 / (s_j^2 - s_i^2) terms, relative to s_1^4.
void zip_esvd_backward(Ctx& ctx, bool cplx, const ZipDims& z, const ZipLayout& L,
                       const ZipOperands& op, int batch, const hpeps_esvd_opts& o,
                       hpeps_absorb absorb, double broadening, const ZipOut& out, const void* dU,
                       const double* dsigma, const void* dR, void* gV, void* gS, void* gT,
                       void* gBra);
// Adjoint of form_carry: cotangent gV (row-major V) accumulated into gL, gT,
// gBra (gT and gBra may alias).
void carry_backward(Ctx& ctx, bool cplx, const CarryDims& cd, const CarryLayout& cl, const void* Lm,
                    const void* T, const void* Bra, const void* gV, void* gL, void* gT, void* gBra,
                    int batch);

// workspace scope: everything allocated after mark() is reused after release
struct WsScope {
  Ctx& c;
  int chunk;
  int64_t off;
  explicit WsScope(Ctx& ctx);
  ~WsScope();
};

}  // namespace hp
