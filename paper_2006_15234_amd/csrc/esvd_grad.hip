// Adjoint (reverse mode) of the randomized einsumsvd of Alg. 4 with the
// sketch held fixed, and of the exact carry of the pair network.
//
// The forward pass is recomputed (checkpoint and recompute: nothing is kept
// between the forward call and this one) with every panel of Alg. 4 kept:
// P_0 .. P_q, Q_1 .. Q_q, the inverses of their total CholeskyQR factors,
// B = A^* P_q and the small SVD M = B^H = Z Sigma V^H.  The reverse sweep
// then runs:
//   * truncated-SVD backward of M (1 / (s_j^2 - s_i^2) Lorentzian-broadened
//     by a caller-chosen width relative to s_1^4, complex phase term on the
//     left vectors), giving Mbar;
//   * M = P^H A:        Abar += P Mbar,         Pbar += A Mbar^H;
//   * P = orth(Y):      Ybar = (Pbar + P copyltu(-Pbar^H P)) R^-H (copyltu with
//                       a real diagonal: R has a real positive diagonal);
//   * Y = A X:          Abar += Ybar X^H,       Xbar  = A^* Ybar;
//   * Z = A^* P:        Abar += P Zbar^H,       Pbar  = A Zbar;
// so the operator cotangent is a sum of 2q + 2 outer products of k-wide
// panels, Abar = sum_t L_t R_t^H, never formed.  Each term is turned into the
// gradients of the four tensors of the zip-up operator by contracting the
// network with one tensor removed: the panel R_t runs through the first three
// forward stages, L_t through the first three adjoint stages, and one GEMM
// per tensor joins them.  Gradients use the conjugate Wirtinger convention
// (dL/dRe + i dL/dIm of a real loss).  They are exact derivatives of the
// algorithm for losses that do not depend on the phase of the singular
// vectors (the canonical phase choice is not differentiated).
#include "esvd.h"
#include "tape.h"

namespace hp {
namespace {

enum class Op { N, H };

// C[b] = alpha op(A[b]) op(B[b]) (+ C[b]); op(A) is M x K, op(B) is K x N; every
// matrix row-major with the given row strides; Op::H is the conjugate transpose
// of the stored matrix (A stored K x M, B stored N x K).
void pg(Ctx& ctx, bool cplx, int batch, int64_t M, int64_t N, int64_t K, const void* A, Op oa,
        int64_t lda, int64_t sA, const void* B, Op ob, int64_t ldb, int64_t sB, void* C, int64_t ldc,
        int64_t sC, bool acc = false, const double* nscale = nullptr, int64_t nld = 0) {
  GemmDesc D;
  D.M = M;
  D.N = N;
  D.K = K;
  if (oa == Op::N) {
    D.Am.add(M, lda);
    D.Ak.add(K, 1);
  } else {
    D.Am.add(M, 1);
    D.Ak.add(K, lda);
  }
  if (ob == Op::N) {
    D.Bk.add(K, ldb);
    D.Bn.add(N, 1);
  } else {
    D.Bk.add(K, 1);
    D.Bn.add(N, ldb);
  }
  D.Cm.add(M, ldc);
  D.Cn.add(N, 1);
  GemmCall c;
  c.A = A;
  c.B = B;
  c.C = C;
  c.sA = sA;
  c.sB = sB;
  c.sC = sC;
  c.batch = batch;
  c.conjA = cplx && oa == Op::H;
  c.conjB = cplx && ob == Op::H;
  c.accumulate = acc;
  c.nscale = nscale;
  c.nscale_ld = nld;
  gemm(ctx, cplx ? Prec::C128 : Prec::F64, D, c);
}

void copy_dev(Ctx& ctx, void* dst, const void* src, int64_t bytes) {
  HP_CHECK_HIP(hipMemcpyAsync(dst, src, (size_t)bytes, hipMemcpyDeviceToDevice, ctx.stream));
}

// Ybar = (Pbar + P copyltu(-Pbar^H P)) Rt^-H for P = orth(Y), Y = P Rt (n x k)
void orth_backward(Ctx& ctx, bool cplx, int batch, int64_t n, int64_t k, const double* P,
                   const double* Rtinv, const double* Pbar, double* Ybar) {
  WsScope scope(ctx);
  const int es = cplx ? 2 : 1;
  double* Mk = ctx.ws<double>((int64_t)batch * k * k * es);
  double* W = ctx.ws<double>((int64_t)batch * n * k * es);
  pg(ctx, cplx, batch, k, k, n, Pbar, Op::H, k, n * k, P, Op::N, k, n * k, Mk, k, k * k);
  copyltu_neg(ctx, cplx, Mk, k, batch);
  copy_dev(ctx, W, Pbar, (int64_t)batch * n * k * es * 8);
  pg(ctx, cplx, batch, n, k, k, P, Op::N, k, n * k, Mk, Op::N, k, k * k, W, k, n * k, true);
  pg(ctx, cplx, batch, n, k, k, W, Op::N, k, n * k, Rtinv, Op::H, k, k * k, Ybar, k, n * k);
}

}  // namespace

// Gradients of the four zip-up tensors for one operator-cotangent term
// Abar += Lt Rt^H (Lt: rows x k, Rt: cols x k), accumulated into gV, gS, gT,
// gBra (layouts of L; a null target is skipped).  wL / wR: stage buffers of
// the adjoint / forward chains.
static void zip_vjp_term(Ctx& ctx, bool cplx, const ZipDims& z, const ZipLayout& L,
                         const ZipOperands& op, int batch, int64_t k, const double* Lt,
                         const double* Rt, const ZipWork& wL, const ZipWork& wR, void* gV, void* gS,
                         void* gT, void* gBra) {
  const Prec p = cplx ? Prec::C128 : Prec::F64;
  const int64_t a = z.a, x = z.x, b = z.b, h = z.h, u = z.u, c = z.c, y = z.y, g = z.g, d = z.d;
  const int64_t rows = z.rows(), cols = z.cols();
  // R through s1..s3, L through t4..t2
  zip_apply(ctx, p, z, L, op, batch, k, false, Rt, nullptr, true, wR, ZipOrder::Classic);
  zip_apply(ctx, p, z, L, op, batch, k, true, Lt, nullptr, true, wL, ZipOrder::Classic);
  // stage layouts (as in zip_apply)
  const int64_t nW1 = u * h * d * y * c * g * k, nW2 = u * h * u * h * c * k, nW3 = b * h * h * k;
  const int64_t w2j = 1, w2c = k, w2h = c * k, w2u = h * w2h, w2H = u * w2u, w2U = h * w2H;
  const int64_t w3j = 1, w3H = k, w3h = h * k, w3b = h * w3h;
  const int64_t w1j = 1, w1G = k, w1c = g * k, w1Y = c * w1c, w1p = y * w1Y, w1h = d * w1p, w1u = h * w1h;
  const int64_t v1j = 1, v1c = k, v1h = c * k, v1u = h * v1h, v1p = u * v1u, v1G = d * v1p, v1Y = g * v1G;
  const int64_t xj = 1, xG = k, xg = g * k, xc = g * xg, xY = c * xc, xy = y * xY;
  auto run = [&](GemmDesc& D, const void* A, int64_t nA, bool cA, const void* B, int64_t nB, bool cB,
                 void* C, int64_t nC) {
    GemmCall gc;
    gc.A = A;
    gc.B = B;
    gc.C = C;
    gc.sA = nA;
    gc.sB = nB;
    gc.sC = nC;
    gc.batch = batch;
    gc.conjA = cplx && cA;
    gc.conjB = cplx && cB;
    gc.accumulate = true;
    gemm(ctx, p, D, gc);
  };
  // gV[a,x,X,b,h,H] += sum_j L[axX, j] conj(W3R[b,h,H,j])
  if (gV) {
    GemmDesc D;
    D.M = rows; D.K = k; D.N = b * h * h;
    D.Am.add(rows, k);
    D.Ak.add(k, 1);
    D.Bk.add(k, w3j);
    D.Bn.add(b, w3b).add(h, w3h).add(h, w3H);
    D.Cm.add(a, L.V[0]).add(x, L.V[1]).add(x, L.V[2]);
    D.Cn.add(b, L.V[3]).add(h, L.V[4]).add(h, L.V[5]);
    run(D, Lt, rows * k, false, wR.W3, nW3, true, gV, L.nV);
  }
  // gS[b,u,U,c] += sum_{h,H,j} W3L[b,h,H,j] conj(W2R[U,H,u,h,c,j])
  if (gS) {
    GemmDesc D;
    D.M = b; D.K = h * h * k; D.N = u * u * c;
    D.Am.add(b, w3b);
    D.Ak.add(h, w3h).add(h, w3H).add(k, w3j);
    D.Bk.add(h, w2h).add(h, w2H).add(k, w2j);
    D.Bn.add(u, w2u).add(u, w2U).add(c, w2c);
    D.Cm.add(b, L.S[0]);
    D.Cn.add(u, L.S[1]).add(u, L.S[2]).add(c, L.S[3]);
    run(D, wL.W3, nW3, false, wR.W2, nW2, true, gS, L.nS);
  }
  // gT[u,y,h,g,p] += sum_{Y,G,c,j} W1L[Y,G,p,u,h,c,j] conj(R[y,Y,c,g,G,j])
  if (gT) {
    GemmDesc D;
    D.M = u * h * d; D.K = y * g * c * k; D.N = y * g;
    D.Am.add(u, v1u).add(h, v1h).add(d, v1p);
    D.Ak.add(y, v1Y).add(g, v1G).add(c, v1c).add(k, v1j);
    D.Bk.add(y, xY).add(g, xG).add(c, xc).add(k, xj);
    D.Bn.add(y, xy).add(g, xg);
    D.Cm.add(u, L.T[0]).add(h, L.T[2]).add(d, L.T[4]);
    D.Cn.add(y, L.T[1]).add(g, L.T[3]);
    run(D, wL.W1, nW1, false, Rt, cols * k, true, gT, L.nT);
  }
  // gBra[U,Y,H,G,p] += sum_{u,h,c,j} conj(W2L[U,H,u,h,c,j]) W1R[u,h,p,Y,c,G,j]
  if (gBra) {
    GemmDesc D;
    D.M = u * h; D.K = u * h * c * k; D.N = y * g * d;
    D.Am.add(u, w2U).add(h, w2H);
    D.Ak.add(u, w2u).add(h, w2h).add(c, w2c).add(k, w2j);
    D.Bk.add(u, w1u).add(h, w1h).add(c, w1c).add(k, w1j);
    D.Bn.add(y, w1Y).add(g, w1G).add(d, w1p);
    D.Cm.add(u, L.B[0]).add(h, L.B[2]);
    D.Cn.add(y, L.B[1]).add(g, L.B[3]).add(d, L.B[4]);
    run(D, wL.W2, nW2, true, wR.W1, nW1, false, gBra, L.nB);
  }
}

// Reverse mode of Alg. 4 up to the operator: the forward pass is recomputed
// through `apply` (A X for adj = false, A^* X for adj = true), keeping every
// panel, and then walked back through the factors, the canonical phase, the
// small SVD, the projection and the power iterations.  The cotangent of the
// operator comes out as a sum of rank-k terms Abar = sum_t L_t R_t^H (L_t
// rows x k, R_t cols x k per instance), appended to `terms`; their buffers
// live in the caller's workspace scope.
void rsvd_backward_terms(Ctx& ctx, bool cplx, int64_t rows, int64_t cols, int batch, const hpeps_esvd_opts& o,
                         hpeps_absorb absorb, double broadening, const ZipOut& out, const void* dU,
                         const double* dsigma, const void* dR, const ApplyFn& apply, RankTerms& terms) {
  HP_REQUIRE(broadening >= 0.0, HPEPS_ERR_INVALID_ARG, "broadening must be >= 0");
  HP_REQUIRE(o.sketch_precision == HPEPS_F64, HPEPS_ERR_DTYPE, "the adjoint runs in FP64 / complex128");
  HP_REQUIRE(o.orth == HPEPS_ORTH_CHOLQR, HPEPS_ERR_UNSUPPORTED, "the adjoint differentiates the CholeskyQR path");
  HP_REQUIRE(absorb == HPEPS_ABSORB_NONE || absorb == HPEPS_ABSORB_RIGHT || absorb == HPEPS_ABSORB_CARRY,
             HPEPS_ERR_UNSUPPORTED, "the adjoint supports the NONE, RIGHT and CARRY absorb modes");
  const int64_t k = sketch_width(o.rank, o.oversample, rows, cols);
  const int64_t mp = std::min<int64_t>(o.rank, k);
  HP_REQUIRE(k >= 1 && k <= (cplx ? 88 : 128), HPEPS_ERR_SHAPE, "sketch width out of range");
  const int es = cplx ? 2 : 1;
  const int64_t nb = batch, q = o.power_iters;
  const int max_sweeps = o.jacobi_max_sweeps > 0 ? o.jacobi_max_sweeps : 40;
  auto R_ = [&](int64_t n) { return ctx.ws<double>(nb * n * es); };

  // ---- forward recompute, keeping the panels
  OrthWork ow;
  ow.G = R_(k * k);
  ow.Rinv = R_(k * k);
  ow.Racc = R_(k * k);
  ow.flags = ctx.ws<int>(nb);
  double* Om = R_(cols * k);
  std::vector<double*> Ps(q + 1), Qs(q), RP(q + 1), RQ(q);
  for (auto& v : Ps) v = R_(rows * k);
  for (auto& v : Qs) v = R_(cols * k);
  for (auto& v : RP) v = R_(k * k);
  for (auto& v : RQ) v = R_(k * k);
  double* Xr = R_(rows * k);
  double* Xc = R_(cols * k);
  double* Xc2 = R_(cols * k);
  double* B = R_(cols * k);
  double* Z = R_(k * k);
  double* sig = ctx.ws<double>(nb * k);
  double* isig = ctx.ws<double>(nb * k);
  double* isig1 = ctx.ws<double>(nb);
  int* sweeps = ctx.ws<int>(nb);

  sketch(ctx, Om, false, cols, k, batch, o.seed, o.stream_id, cplx);
  apply(false, Om, Xr);
  orthogonalize(ctx, cplx, Xr, Ps[0], rows, k, batch, ow, RP[0]);
  for (int64_t i = 0; i < q; ++i) {
    apply(true, Ps[i], Xc);
    orthogonalize(ctx, cplx, Xc, Qs[i], cols, k, batch, ow, RQ[i]);
    apply(false, Qs[i], Xr);
    orthogonalize(ctx, cplx, Xr, Ps[i + 1], rows, k, batch, ow, RP[i + 1]);
  }
  apply(true, Ps[q], B);
  cholqr_r(ctx, cplx, B, Xc, Xc2, cols, k, batch, ow);
  jacobi_svd(ctx, cplx, ow.Racc, k, batch, max_sweeps, Z, sig, isig, isig1, nullptr, sweeps);
  double* Ut = R_(rows * mp);
  pg(ctx, cplx, batch, rows, mp, k, Ps[q], Op::N, k, rows * k, Z, Op::N, k, k * k, Ut, mp, rows * mp);
  gauge_fix(ctx, cplx, Ut, rows, mp, Z, k, batch);
  // all k right singular vectors of M: V = B Z Sigma^-1
  double* Vf = R_(cols * k);
  pg(ctx, cplx, batch, cols, k, k, B, Op::N, k, cols * k, Z, Op::N, k, k * k, Vf, k, cols * k, false,
     isig, k);

  // ---- cotangents of the outputs, gathered to row-major U [rows, m'] and
  // R [m', cols].  R row i is sc_i V[:, i]^H with sc_i = 1 (NONE), s_i
  // (RIGHT) or s_i / s_1 (CARRY, s_1 held constant: the carry scale only
  // moves the logarithmic accumulator, which carries no cotangent).
  double* dUr = R_(rows * mp);
  double* dRr = R_(mp * cols);
  gather2d(ctx, cplx, dU, out.nU, out.Urows, out.Ucol, dUr, batch);
  gather2d(ctx, cplx, dR, out.nR, out.Rrow, out.Rcols, dRr, batch);
  const double* s_r = absorb == HPEPS_ABSORB_NONE ? nullptr : sig;
  const double* rsc = absorb == HPEPS_ABSORB_CARRY ? isig1 : nullptr;
  if (cplx) {
    // the kept left vectors after the phase choice
    pg(ctx, cplx, batch, rows, mp, k, Ps[q], Op::N, k, rows * k, Z, Op::N, k, k * k, Ut, mp, rows * mp);
    gauge_backward(ctx, dUr, Ut, dRr, Vf, s_r, rsc, rows, cols, mp, k, batch);
  }
  double* Vbar = R_(cols * k);
  vbar_from_dr(ctx, cplx, dRr, s_r, rsc, cols, mp, k, batch, Vbar);
  double* sbar = ctx.ws<double>(nb * k);
  sigma_bar(ctx, cplx, dsigma, dRr, Vf, rsc, cols, mp, k, batch, absorb != HPEPS_ABSORB_NONE, sbar);
  double* Zbar = R_(k * k);
  fill_zero(ctx, Zbar, nb * k * k * es * 8);
  pg(ctx, cplx, batch, k, mp, rows, Ps[q], Op::H, k, rows * k, dUr, Op::N, mp, rows * mp, Zbar, k, k * k);
  double* Pbar = R_(rows * k);
  pg(ctx, cplx, batch, rows, k, mp, dUr, Op::N, mp, rows * mp, Z, Op::H, k, k * k, Pbar, k, rows * k);

  // ---- truncated-SVD backward of M = Z Sigma V^H
  double* ZZ = R_(k * k);
  double* VV = R_(k * k);
  double* G1H = R_(k * k);
  pg(ctx, cplx, batch, k, k, k, Z, Op::H, k, k * k, Zbar, Op::N, k, k * k, ZZ, k, k * k);
  pg(ctx, cplx, batch, k, k, cols, Vf, Op::H, k, cols * k, Vbar, Op::N, k, cols * k, VV, k, k * k);
  svd_bwd_core(ctx, cplx, ZZ, VV, sig, sbar, k, batch, broadening, G1H);
  // Mbar^H = (V G1^H + Vbar Sigma^-1) Z^H
  double* T1 = R_(cols * k);
  pg(ctx, cplx, batch, cols, k, k, Vf, Op::N, k, cols * k, G1H, Op::N, k, k * k, T1, k, cols * k);
  axpy_colscale(ctx, cplx, T1, Vbar, isig, cols, k, batch);

  // operator cotangent terms Abar += L_t R_t^H
  double* MbarH = R_(cols * k);
  pg(ctx, cplx, batch, cols, k, k, T1, Op::N, k, cols * k, Z, Op::H, k, k * k, MbarH, k, cols * k);
  terms.push_back({Ps[q], MbarH});
  apply(false, MbarH, Xr);
  axpy(ctx, Pbar, Xr, 1.0, nb * rows * k * es);

  // ---- reverse through the power iterations
  for (int64_t i = q; i >= 1; --i) {
    double* Yb = R_(rows * k);
    orth_backward(ctx, cplx, batch, rows, k, Ps[i], RP[i], Pbar, Yb);
    terms.push_back({Yb, Qs[i - 1]});
    apply(true, Yb, Xc);       // Qbar = A^* Ybar
    double* Zb = R_(cols * k);
    orth_backward(ctx, cplx, batch, cols, k, Qs[i - 1], RQ[i - 1], Xc, Zb);
    terms.push_back({Ps[i - 1], Zb});
    apply(false, Zb, Pbar);    // Pbar = A Zbar
  }
  double* Yb0 = R_(rows * k);
  orth_backward(ctx, cplx, batch, rows, k, Ps[0], RP[0], Pbar, Yb0);
  terms.push_back({Yb0, Om});

}

void zip_esvd_backward(Ctx& ctx, bool cplx, const ZipDims& z, const ZipLayout& L,
                       const ZipOperands& op, int batch, const hpeps_esvd_opts& o,
                       hpeps_absorb absorb, double broadening, const ZipOut& out, const void* dU,
                       const double* dsigma, const void* dR, void* gV, void* gS, void* gT,
                       void* gBra) {
  WsScope scope(ctx);
  const int64_t rows = z.rows(), cols = z.cols();
  const int64_t k = sketch_width(o.rank, o.oversample, rows, cols);
  HP_REQUIRE(k >= 1 && k <= (cplx ? 88 : 128), HPEPS_ERR_SHAPE, "sketch width out of range");
  const Prec p = cplx ? Prec::C128 : Prec::F64;
  const int es = cplx ? 2 : 1;
  const int64_t nb = batch;
  auto R_ = [&](int64_t n) { return ctx.ws<double>(nb * n * es); };
  ZipWork w;
  w.W1 = R_(z.u * z.h * z.d * z.y * z.c * z.g * k);
  w.W2 = R_(zip_w2_elems(z, k));
  w.W3 = R_(z.b * z.h * z.h * k);
  RankTerms terms;
  rsvd_backward_terms(ctx, cplx, rows, cols, batch, o, absorb, broadening, out, dU, dsigma, dR,
                      [&](bool adj, const double* X, double* Y) {
                        zip_apply(ctx, p, z, L, op, batch, k, adj, X, Y, true, w);
                      },
                      terms);

  // ---- tensor gradients (accumulated: gT and gBra may be one buffer)
  ZipWork wL, wR;
  wL.W1 = R_(z.u * z.h * z.d * z.y * z.c * z.g * k);
  wL.W2 = R_(z.u * z.h * z.u * z.h * z.c * k);
  wL.W3 = R_(z.b * z.h * z.h * k);
  wR = w;
  for (const auto& t : terms)
    zip_vjp_term(ctx, cplx, z, L, op, batch, k, t.first, t.second, wL, wR, gV, gS, gT, gBra);
}

// Gradients of the exact carry V[a,x,X,b,h,H] = sum_{u,U,p} L[a,u,U,b] T[u,x,h,p]
// conj(Bra[U,X,H,p]) for the cotangent gV (row-major V); accumulated into gL, gT,
// gBra (gT and gBra may be one buffer).
void carry_backward(Ctx& ctx, bool cplx, const CarryDims& cd, const CarryLayout& cl, const void* Lm,
                    const void* T, const void* Bra, const void* gV, void* gL, void* gT, void* gBra,
                    int batch) {
  WsScope scope(ctx);
  const int64_t a = cd.a, u = cd.u, b = cd.b, x = cd.x, h = cd.h, d = cd.d;
  const Prec p = cplx ? Prec::C128 : Prec::F64;
  const int es = cplx ? 2 : 1;
  const int64_t VH = 1, Vh = h, Vb = h * h, VX = b * Vb, Vx = x * VX, Va = x * Vx;
  const int64_t nV = a * x * x * b * h * h;
  // Y1[a,b,X,H,u,p] = sum_{x,h} gV[a,x,X,b,h,H] conj(T[u,x,h,p])
  const int64_t Y1p = 1, Y1u = d, Y1H = u * d, Y1X = h * Y1H, Y1b = x * Y1X, Y1a = b * Y1b;
  const int64_t nY1 = a * b * x * h * u * d;
  // Y2[x,X,h,H,u,U] = sum_{a,b} gV[a,x,X,b,h,H] conj(L[a,u,U,b])
  const int64_t Y2U = 1, Y2u = u, Y2H = u * u, Y2h = h * Y2H, Y2X = h * Y2h, Y2x = x * Y2X;
  const int64_t nY2 = x * x * h * h * u * u;
  double* Y1 = ctx.ws<double>((int64_t)batch * nY1 * es);
  double* Y2 = ctx.ws<double>((int64_t)batch * nY2 * es);
  auto run = [&](GemmDesc& D, const void* A, int64_t nA, bool cA, const void* B, int64_t nB, bool cB,
                 void* C, int64_t nC) {
    GemmCall gc;
    gc.A = A;
    gc.B = B;
    gc.C = C;
    gc.sA = nA;
    gc.sB = nB;
    gc.sC = nC;
    gc.batch = batch;
    gc.conjA = cplx && cA;
    gc.conjB = cplx && cB;
    gc.accumulate = C != Y1 && C != Y2;
    gemm(ctx, p, D, gc);
  };
  if (gL) {
    GemmDesc D;
    D.M = a * b * x * h; D.K = x * h; D.N = u * d;
    D.Am.add(a, Va).add(b, Vb).add(x, VX).add(h, VH);
    D.Ak.add(x, Vx).add(h, Vh);
    D.Bk.add(x, cl.T[1]).add(h, cl.T[2]);
    D.Bn.add(u, cl.T[0]).add(d, cl.T[3]);
    D.Cm.add(a, Y1a).add(b, Y1b).add(x, Y1X).add(h, Y1H);
    D.Cn.add(u, Y1u).add(d, Y1p);
    run(D, gV, nV, false, T, cl.nT, true, Y1, nY1);
  }
  // gL[a,u,U,b] += sum_{X,H,p} Y1[a,b,X,H,u,p] Bra[U,X,H,p]
  if (gL) {
    GemmDesc D;
    D.M = a * u * b; D.K = x * h * d; D.N = u;
    D.Am.add(a, Y1a).add(u, Y1u).add(b, Y1b);
    D.Ak.add(x, Y1X).add(h, Y1H).add(d, Y1p);
    D.Bk.add(x, cl.B[1]).add(h, cl.B[2]).add(d, cl.B[3]);
    D.Bn.add(u, cl.B[0]);
    D.Cm.add(a, cl.L[0]).add(u, cl.L[1]).add(b, cl.L[3]);
    D.Cn.add(u, cl.L[2]);
    run(D, Y1, nY1, false, Bra, cl.nB, false, gL, cl.nL);
  }
  if (gT || gBra) {
    GemmDesc D;
    D.M = x * x * h * h; D.K = a * b; D.N = u * u;
    D.Am.add(x, Vx).add(x, VX).add(h, Vh).add(h, VH);
    D.Ak.add(a, Va).add(b, Vb);
    D.Bk.add(a, cl.L[0]).add(b, cl.L[3]);
    D.Bn.add(u, cl.L[1]).add(u, cl.L[2]);
    D.Cm.add(x, Y2x).add(x, Y2X).add(h, Y2h).add(h, Y2H);
    D.Cn.add(u, Y2u).add(u, Y2U);
    run(D, gV, nV, false, Lm, cl.nL, true, Y2, nY2);
  }
  // gT[u,x,h,p] += sum_{U,X,H} Y2[x,X,h,H,u,U] Bra[U,X,H,p]
  if (gT) {
    GemmDesc D;
    D.M = u * x * h; D.K = u * x * h; D.N = d;
    D.Am.add(u, Y2u).add(x, Y2x).add(h, Y2h);
    D.Ak.add(u, Y2U).add(x, Y2X).add(h, Y2H);
    D.Bk.add(u, cl.B[0]).add(x, cl.B[1]).add(h, cl.B[2]);
    D.Bn.add(d, cl.B[3]);
    D.Cm.add(u, cl.T[0]).add(x, cl.T[1]).add(h, cl.T[2]);
    D.Cn.add(d, cl.T[3]);
    run(D, Y2, nY2, false, Bra, cl.nB, false, gT, cl.nT);
  }
  // gBra[U,X,H,p] += sum_{u,x,h} conj(Y2[x,X,h,H,u,U]) T[u,x,h,p]
  if (gBra) {
    GemmDesc D;
    D.M = u * x * h; D.K = u * x * h; D.N = d;
    D.Am.add(u, Y2U).add(x, Y2X).add(h, Y2H);
    D.Ak.add(u, Y2u).add(x, Y2x).add(h, Y2h);
    D.Bk.add(u, cl.T[0]).add(x, cl.T[1]).add(h, cl.T[2]);
    D.Bn.add(d, cl.T[3]);
    D.Cm.add(u, cl.B[0]).add(x, cl.B[1]).add(h, cl.B[2]);
    D.Cn.add(d, cl.B[3]);
    run(D, Y2, nY2, true, T, cl.nT, false, gBra, cl.nB);
  }
}

}  // namespace hp
