// einsumsvd by randomized SVD on the implicit zip-up operator (Alg. 4 on
// the network of Alg. 3's inner step, two-layer form of Sec. III-B).
//
// The operator A[(a,x,X),(y,Y,c,g,G)] = sum V[a,x,X,b,h,H] S[b,u,U,c]
// T[u,y,h,g,p] conj(Bra[U,Y,H,G,p]) is applied right to left as four
// gathered GEMMs (ket, bra, boundary, carry); its adjoint mirrors them.
// Per einsumsvd: sketch, q+1 forward and q+1 adjoint applications, a
// CholeskyQR orthogonalization after each, a CholeskyQR of B^* = A^* P to
// obtain the k x k factor R_B, a one-sided Jacobi SVD of R_B^H, and two
// factor products.  Every step is a kernel on the context stream; the only
// host work is the launch sequence.
#include <algorithm>
#include <cmath>

#include "esvd.h"
#include "tape.h"

namespace hp {

int64_t ZipDims::rows() const { return a * x * x; }
int64_t ZipDims::cols() const { return y * y * c * g * g; }
int64_t ZipDims::v_size() const { return a * x * x * b * h * h; }
int64_t ZipDims::s_size() const { return b * u * u * c; }
int64_t ZipDims::t_size() const { return u * y * h * g * d; }

ZipLayout ZipLayout::row_major(const ZipDims& z) {
  ZipLayout L;
  L.V[5] = 1; L.V[4] = z.h; L.V[3] = z.h * z.h; L.V[2] = z.b * L.V[3]; L.V[1] = z.x * L.V[2]; L.V[0] = z.x * L.V[1];
  L.S[3] = 1; L.S[2] = z.c; L.S[1] = z.u * z.c; L.S[0] = z.u * L.S[1];
  L.T[4] = 1; L.T[3] = z.d; L.T[2] = z.g * z.d; L.T[1] = z.h * L.T[2]; L.T[0] = z.y * L.T[1];
  for (int i = 0; i < 5; ++i) L.B[i] = L.T[i];
  L.nV = z.v_size();
  L.nS = z.s_size();
  L.nT = L.nB = z.t_size();
  return L;
}

ZipOut ZipOut::row_major(const ZipDims& z, int64_t mp) {
  ZipOut o;
  const int64_t rows = z.rows(), cols = z.cols();
  o.Urows.add(rows, mp);
  o.Ucol.add(mp, 1);
  o.Rrow.add(mp, cols);
  o.Rcols.add(cols, 1);
  o.nU = rows * mp;
  o.nR = mp * cols;
  return o;
}

CarryLayout CarryLayout::row_major(const CarryDims& c) {
  CarryLayout L;
  L.L[3] = 1; L.L[2] = c.b; L.L[1] = c.u * c.b; L.L[0] = c.u * L.L[1];
  // [u, x, 1, h, p]
  L.T[3] = 1; L.T[2] = c.d; L.T[1] = c.h * c.d; L.T[0] = c.x * L.T[1];
  for (int i = 0; i < 4; ++i) L.B[i] = L.T[i];
  L.nL = c.a * c.u * c.u * c.b;
  L.nT = L.nB = c.u * c.x * c.h * c.d;
  return L;
}

WsScope::WsScope(Ctx& ctx) : c(ctx), chunk(ctx.ws_chunk()), off(ctx.ws_offset()) {}
WsScope::~WsScope() {
  if (!tape_keeps_workspace(c)) c.ws_restore(chunk, off);
}

// ---------------------------------------------------------------------------
// operator applications

int64_t zip_w2_elems(const ZipDims& z, int64_t k) {
  const int64_t w2 = z.u * z.h * z.u * z.h * z.c * k;           // [U,H,u,h,c,j]
  const int64_t zz = z.b * z.u * z.h * z.d * z.y * z.g * k;     // [b,U,h,p,Y,G,j]
  return std::max(w2, zz);
}

// Time model of one product: the larger of its MFMA time (an effective rate
// per precision, scaled down when a tile dimension is below 16) and its HBM
// time (every operand element moved once at 3.2 TB/s, the rate the gathered
// GEMM sustains on these streaming shapes; 41 TF/s FP64 on the MFMA-bound
// ones).
static double stage_time(Prec prec, int64_t M, int64_t N, int64_t K, int64_t elems, int batch) {
  const bool cplx = prec == Prec::C128;
  const double rate = prec == Prec::BF16 ? 200e12 : prec == Prec::F32 ? 80e12 : 40e12;
  const double elt = prec == Prec::BF16 ? 2 : prec == Prec::F32 ? 4 : cplx ? 16 : 8;
  const double fill = std::min<double>(1.0, (double)std::min(M, N) / 16.0);
  const double flops = 2.0 * M * N * K * (cplx ? 4 : 1) * batch;
  return std::max(flops / (rate * fill), elems * elt * batch / 3.2e12);
}

ZipOrder zip_order(const Ctx& ctx, Prec prec, const ZipDims& z, int64_t k, int batch) {
  if (ctx.zip_order_force == 1) return ZipOrder::Classic;
  if (ctx.zip_order_force == 2) return ZipOrder::BoundaryFirst;
  const int64_t b = z.b, h = z.h, u = z.u, c = z.c, y = z.y, g = z.g, d = z.d;
  const int64_t nW1 = u * h * d * y * c * g * k, nW2 = u * h * u * h * c * k, nW3 = b * h * h * k;
  const int64_t nZ = b * u * h * d * y * g * k, nS = b * u * u * c, nB = u * y * h * g * d;
  const double classic = stage_time(prec, u * h, u * h * c * k, y * g * d, nW1 + nW2 + nB, batch) +
                         stage_time(prec, b, h * h * k, u * u * c, nW2 + nW3 + nS, batch);
  const double bfirst = stage_time(prec, b * u, h * d * y * g * k, u * c, nW1 + nZ + nS, batch) +
                        stage_time(prec, h, b * h * k, u * y * g * d, nZ + nW3 + nB, batch);
  return bfirst < 0.9 * classic ? ZipOrder::BoundaryFirst : ZipOrder::Classic;
}

void zip_apply(Ctx& ctx, Prec prec, const ZipDims& z, const ZipLayout& L, const ZipOperands& op,
               int batch, int64_t k, bool adjoint, const void* X, void* Y, bool y_f64,
               const ZipWork& w, ZipOrder order) {
  const int64_t a = z.a, x = z.x, b = z.b, h = z.h, u = z.u, c = z.c, y = z.y, g = z.g, d = z.d;
  if (order == ZipOrder::Auto) order = zip_order(ctx, prec, z, k, batch);
  HP_REQUIRE(Y || order == ZipOrder::Classic, HPEPS_ERR_INVALID_ARG,
             "kept stage results exist in the classic order only");
  const bool bfirst = order == ZipOrder::BoundaryFirst;
  // Z[b,U,h,p,Y,G,j] (boundary-first order; shares the W2 buffer)
  const int64_t nZ = b * u * h * d * y * g * k;
  const int64_t zj = 1, zG = k, zY = g * k, zp = y * zY, zh = d * zp, zU = h * zh, zb = u * zU;
  const int64_t rows = z.rows(), cols = z.cols();
  const int64_t nW1 = u * h * d * y * c * g * k;  // [u,h,p,Y,c,G,j] or [Y,G,p,u,h,c,j]
  const int64_t nW2 = u * h * u * h * c * k;      // [U,H,u,h,c,j]
  const int64_t nW3 = b * h * h * k;              // [b,h,H,j]
  // W2 strides [U,H,u,h,c,j]
  const int64_t w2j = 1, w2c = k, w2h = c * k, w2u = h * w2h, w2H = u * w2u, w2U = h * w2H;
  // W3 strides [b,h,H,j]
  const int64_t w3j = 1, w3H = k, w3h = h * k, w3b = h * w3h;
  const bool f32 = prec == Prec::F32 || prec == Prec::BF16;  // narrow operands
  const int64_t *sV = L.V, *sS = L.S, *sT = L.T, *sB = L.B;

  auto call = [&](const GemmDesc& dsc, const void* A, int64_t nA, bool cA, const void* B, int64_t nB,
                  bool cB, void* C, int64_t nC, bool out_f64) {
    GemmCall gc;
    gc.A = A;
    gc.B = B;
    gc.C = C;
    gc.sA = nA;
    gc.sB = nB;
    gc.sC = nC;
    gc.batch = batch;
    gc.conjA = cA;
    gc.conjB = cB;
    gc.out_f64 = out_f64;
    gemm(ctx, prec, dsc, gc);
  };

  if (!adjoint) {
    // X[y,Y,c,g,G,j]
    const int64_t xj = 1, xG = k, xg = g * k, xc = g * xg, xY = c * xc, xy = y * xY;
    // W1 [u,h,p,Y,c,G,j] (classic) or [u,c,h,p,Y,G,j] (boundary first: the
    // next product then reads it as a plain row-major (u,c) x (h,p,Y,G,j) matrix)
    int64_t w1j = 1, w1G = k, w1c = g * k, w1Y = c * w1c, w1p = y * w1Y, w1h = d * w1p, w1u = h * w1h;
    if (bfirst) {
      w1Y = g * k;
      w1p = y * w1Y;
      w1h = d * w1p;
      w1c = h * w1h;
      w1u = c * w1c;
    }
    // s1: W1[u,h,p | Y,c,G,j] = sum_{y,g} T[u,y,h,g,p] X[y,Y,c,g,G,j]
    {
      GemmDesc D;
      D.M = u * h * d; D.K = y * g; D.N = y * c * g * k;
      D.Am.add(u, sT[0]).add(h, sT[2]).add(d, sT[4]);
      D.Ak.add(y, sT[1]).add(g, sT[3]);
      D.Bk.add(y, xy).add(g, xg);
      D.Bn.add(y, xY).add(c, xc).add(g, xG).add(k, xj);
      D.Cm.add(u, w1u).add(h, w1h).add(d, w1p);
      D.Cn.add(y, w1Y).add(c, w1c).add(g, w1G).add(k, w1j);
      call(D, op.T, L.nT, false, X, cols * k, false, w.W1, nW1, false);
    }
    if (bfirst) {
      // s2': Z[b,U | h,p,Y,G,j] = sum_{u,c} S[b,u,U,c] W1[u,h,p,Y,c,G,j]
      {
        GemmDesc D;
        D.M = b * u; D.K = u * c; D.N = h * d * y * g * k;
        D.Am.add(b, sS[0]).add(u, sS[2]);
        D.Ak.add(u, sS[1]).add(c, sS[3]);
        D.Bk.add(u, w1u).add(c, w1c);
        D.Bn.add(h, w1h).add(d, w1p).add(y, w1Y).add(g, w1G).add(k, w1j);
        D.Cm.add(b, zb).add(u, zU);
        D.Cn.add(h, zh).add(d, zp).add(y, zY).add(g, zG).add(k, zj);
        call(D, op.S, L.nS, false, w.W1, nW1, false, w.W2, nZ, false);
      }
      // s3': W3[H | b,h,j] = sum_{U,Y,G,p} conj(Bra[U,Y,H,G,p]) Z[b,U,h,p,Y,G,j]
      {
        GemmDesc D;
        D.M = h; D.K = u * y * g * d; D.N = b * h * k;
        D.Am.add(h, sB[2]);
        D.Ak.add(u, sB[0]).add(y, sB[1]).add(g, sB[3]).add(d, sB[4]);
        D.Bk.add(u, zU).add(y, zY).add(g, zG).add(d, zp);
        D.Bn.add(b, zb).add(h, zh).add(k, zj);
        D.Cm.add(h, w3H);
        D.Cn.add(b, w3b).add(h, w3h).add(k, w3j);
        call(D, op.Bra, L.nB, true, w.W2, nZ, false, w.W3, nW3, false);
      }
    }
    // s2: W2[U,H | u,h,c,j] = sum_{Y,G,p} conj(Bra[U,Y,H,G,p]) W1[u,h,p,Y,c,G,j]
    if (!bfirst) {
      GemmDesc D;
      D.M = u * h; D.K = y * g * d; D.N = u * h * c * k;
      D.Am.add(u, sB[0]).add(h, sB[2]);
      D.Ak.add(y, sB[1]).add(g, sB[3]).add(d, sB[4]);
      D.Bk.add(y, w1Y).add(g, w1G).add(d, w1p);
      D.Bn.add(u, w1u).add(h, w1h).add(c, w1c).add(k, w1j);
      D.Cm.add(u, w2U).add(h, w2H);
      D.Cn.add(u, w2u).add(h, w2h).add(c, w2c).add(k, w2j);
      call(D, op.Bra, L.nB, true, w.W1, nW1, false, w.W2, nW2, false);
    }
    // s3: W3[b | h,H,j] = sum_{u,U,c} S[b,u,U,c] W2[U,H,u,h,c,j]
    if (!bfirst) {
      GemmDesc D;
      D.M = b; D.K = u * u * c; D.N = h * h * k;
      D.Am.add(b, sS[0]);
      D.Ak.add(u, sS[1]).add(u, sS[2]).add(c, sS[3]);
      D.Bk.add(u, w2u).add(u, w2U).add(c, w2c);
      D.Bn.add(h, w2h).add(h, w2H).add(k, w2j);
      D.Cm.add(b, w3b);
      D.Cn.add(h, w3h).add(h, w3H).add(k, w3j);
      call(D, op.S, L.nS, false, w.W2, nW2, false, w.W3, nW3, false);
    }
    // s4: Y[a,x,X | j] = sum_{b,h,H} V[a,x,X,b,h,H] W3[b,h,H,j]
    if (Y) {
      GemmDesc D;
      D.M = rows; D.K = b * h * h; D.N = k;
      D.Am.add(a, sV[0]).add(x, sV[1]).add(x, sV[2]);
      D.Ak.add(b, sV[3]).add(h, sV[4]).add(h, sV[5]);
      D.Bk.add(b, w3b).add(h, w3h).add(h, w3H);
      D.Bn.add(k, w3j);
      D.Cm.add(rows, k);
      D.Cn.add(k, 1);
      call(D, op.V, L.nV, false, w.W3, nW3, false, Y, rows * k, y_f64 || !f32);
    }
  } else {
    // t4: W3[b,h,H | j] = sum_{a,x,X} conj(V[a,x,X,b,h,H]) P[a,x,X,j]
    {
      GemmDesc D;
      D.M = b * h * h; D.K = rows; D.N = k;
      D.Am.add(b, sV[3]).add(h, sV[4]).add(h, sV[5]);
      D.Ak.add(a, sV[0]).add(x, sV[1]).add(x, sV[2]);
      D.Bk.add(rows, k);
      D.Bn.add(k, 1);
      D.Cm.add(b, w3b).add(h, w3h).add(h, w3H);
      D.Cn.add(k, w3j);
      call(D, op.V, L.nV, true, X, rows * k, false, w.W3, nW3, false);
    }
    // t3: W2[u,U,c | h,H,j] = sum_b conj(S[b,u,U,c]) W3[b,h,H,j]   (W2 stored [U,H,u,h,c,j])
    if (!bfirst) {
      GemmDesc D;
      D.M = u * u * c; D.K = b; D.N = h * h * k;
      D.Am.add(u, sS[1]).add(u, sS[2]).add(c, sS[3]);
      D.Ak.add(b, sS[0]);
      D.Bk.add(b, w3b);
      D.Bn.add(h, w3h).add(h, w3H).add(k, w3j);
      D.Cm.add(u, w2u).add(u, w2U).add(c, w2c);
      D.Cn.add(h, w2h).add(h, w2H).add(k, w2j);
      call(D, op.S, L.nS, true, w.W3, nW3, false, w.W2, nW2, false);
    }
    // t2: W1[Y,G,p | u,h,c,j] = sum_{U,H} Bra[U,Y,H,G,p] W2[U,H,u,h,c,j]
    // W1 [Y,G,p,u,h,c,j] (classic) or [u,c,h,p,Y,G,j] (boundary first: written
    // by contiguous rows of the (u,c) x (h,p,Y,G,j) product)
    int64_t v1j = 1, v1c = k, v1h = c * k, v1u = h * v1h, v1p = u * v1u, v1G = d * v1p, v1Y = g * v1G;
    if (bfirst) {
      v1G = k;
      v1Y = g * k;
      v1p = y * v1Y;
      v1h = d * v1p;
      v1c = h * v1h;
      v1u = c * v1c;
    }
    if (bfirst) {
      // t3': Z[U,Y,G,p | b,h,j] = sum_H Bra[U,Y,H,G,p] W3[b,h,H,j]   (Z stored [b,U,h,p,Y,G,j])
      {
        GemmDesc D;
        D.M = u * y * g * d; D.K = h; D.N = b * h * k;
        D.Am.add(u, sB[0]).add(y, sB[1]).add(g, sB[3]).add(d, sB[4]);
        D.Ak.add(h, sB[2]);
        D.Bk.add(h, w3H);
        D.Bn.add(b, w3b).add(h, w3h).add(k, w3j);
        D.Cm.add(u, zU).add(y, zY).add(g, zG).add(d, zp);
        D.Cn.add(b, zb).add(h, zh).add(k, zj);
        call(D, op.Bra, L.nB, false, w.W3, nW3, false, w.W2, nZ, false);
      }
      // t2': W1[u,c | h,p,Y,G,j] = sum_{b,U} conj(S[b,u,U,c]) Z[b,U,h,p,Y,G,j]
      {
        GemmDesc D;
        D.M = u * c; D.K = b * u; D.N = h * d * y * g * k;
        D.Am.add(u, sS[1]).add(c, sS[3]);
        D.Ak.add(b, sS[0]).add(u, sS[2]);
        D.Bk.add(b, zb).add(u, zU);
        D.Bn.add(h, zh).add(d, zp).add(y, zY).add(g, zG).add(k, zj);
        D.Cm.add(u, v1u).add(c, v1c);
        D.Cn.add(h, v1h).add(d, v1p).add(y, v1Y).add(g, v1G).add(k, v1j);
        call(D, op.S, L.nS, true, w.W2, nZ, false, w.W1, nW1, false);
      }
    } else {
      GemmDesc D;
      D.M = y * g * d; D.K = u * h; D.N = u * h * c * k;
      D.Am.add(y, sB[1]).add(g, sB[3]).add(d, sB[4]);
      D.Ak.add(u, sB[0]).add(h, sB[2]);
      D.Bk.add(u, w2U).add(h, w2H);
      D.Bn.add(u, w2u).add(h, w2h).add(c, w2c).add(k, w2j);
      D.Cm.add(y, v1Y).add(g, v1G).add(d, v1p);
      D.Cn.add(u, v1u).add(h, v1h).add(c, v1c).add(k, v1j);
      call(D, op.Bra, L.nB, false, w.W2, nW2, false, w.W1, nW1, false);
    }
    // t1: Z[y,g | Y,c,G,j] = sum_{u,h,p} conj(T[u,y,h,g,p]) W1[Y,G,p,u,h,c,j]
    if (Y) {
      const int64_t oj = 1, oG = k, og = g * k, oc = g * og, oY = c * oc, oy = y * oY;
      GemmDesc D;
      D.M = y * g; D.K = u * h * d; D.N = y * c * g * k;
      D.Am.add(y, sT[1]).add(g, sT[3]);
      D.Ak.add(u, sT[0]).add(h, sT[2]).add(d, sT[4]);
      D.Bk.add(u, v1u).add(h, v1h).add(d, v1p);
      D.Bn.add(y, v1Y).add(c, v1c).add(g, v1G).add(k, v1j);
      D.Cm.add(y, oy).add(g, og);
      D.Cn.add(y, oY).add(c, oc).add(g, oG).add(k, oj);
      call(D, op.T, L.nT, true, w.W1, nW1, false, Y, cols * k, y_f64 || !f32);
    }
  }
}

// ---------------------------------------------------------------------------
// P = Y R^-1 for n x k Y (batch stride n k), optional pass-through flags
static void apply_rinv(Ctx& ctx, bool cplx, const double* Y, int64_t n, int64_t k, int batch,
                       const double* Rinv, double* P, const int* copy_flags) {
  GemmDesc D;
  D.M = n; D.K = k; D.N = k;
  D.Am.add(n, k);
  D.Ak.add(k, 1);
  D.Bk.add(k, k);
  D.Bn.add(k, 1);
  D.Cm.add(n, k);
  D.Cn.add(k, 1);
  GemmCall c;
  c.A = Y;
  c.B = Rinv;
  c.C = P;
  c.sA = c.sC = n * k;
  c.sB = k * k;
  c.batch = batch;
  c.copy_if_zero = copy_flags;
  gemm(ctx, cplx ? Prec::C128 : Prec::F64, D, c);
}

// Rt <- Rt * Rinv (k x k, upper triangular, per instance); the product is
// formed in the scratch S and copied back
static void chain_rinv(Ctx& ctx, bool cplx, double* Rt, const double* Rinv, double* S, int64_t k,
                       int batch) {
  GemmDesc D;
  D.M = k; D.K = k; D.N = k;
  D.Am.add(k, k);
  D.Ak.add(k, 1);
  D.Bk.add(k, k);
  D.Bn.add(k, 1);
  D.Cm.add(k, k);
  D.Cn.add(k, 1);
  GemmCall c;
  c.A = Rt;
  c.B = Rinv;
  c.C = S;
  c.sA = c.sB = c.sC = k * k;
  c.batch = batch;
  gemm(ctx, cplx ? Prec::C128 : Prec::F64, D, c);
  HP_CHECK_HIP(hipMemcpyAsync(Rt, S, (size_t)batch * k * k * (cplx ? 16 : 8), hipMemcpyDeviceToDevice,
                              ctx.stream));
}

// One pass of the reshape-avoiding orthogonalization (Alg. 5) on the Gram
// matrix G = Y^H Y already in w.G: its eigendecomposition G = X Lambda X^*,
// then P = Y X Lambda^-1/2.  The eigendecomposition is taken from the
// Cholesky factor, G = C^H C (the CholeskyQR factor step of the same pass,
// with its shift and flags), and the one-sided Jacobi SVD of
// C^H = X Sigma W^*: X are G's eigenvectors and Lambda = Sigma^2, accurate to
// eps kappa(C) = eps kappa(Y).  (A one-sided Jacobi on G itself works with
// kappa(G)^2 = kappa(Y)^4: its vectors, and with them P's orthogonality,
// would carry errors of order eps kappa(Y)^3.)  copy_flags: instances whose
// flag is 0 get P = Y (the skipped third pass).
static void eigh_pass(Ctx& ctx, bool cplx, const double* Y, double* P, int64_t n, int64_t k, int batch,
                      const OrthWork& w, int pass, const int* copy_flags) {
  WsScope scope(ctx);
  const int es = cplx ? 2 : 1;
  double* C = ctx.ws<double>((int64_t)batch * k * k * es);
  double* X = ctx.ws<double>((int64_t)batch * k * k * es);
  double* sig = ctx.ws<double>((int64_t)batch * k);
  double* isig = ctx.ws<double>((int64_t)batch * k);
  double* isig1 = ctx.ws<double>(batch);
  int* sweeps = ctx.ws<int>(batch);
  chol_inv(ctx, cplx, w.G, n, k, batch, pass, w.Rinv, C, w.flags, true);
  jacobi_svd(ctx, cplx, C, k, batch, 40, X, sig, isig, isig1, nullptr, sweeps);
  GemmDesc D;
  D.M = n; D.K = k; D.N = k;
  D.Am.add(n, k);
  D.Ak.add(k, 1);
  D.Bk.add(k, k);
  D.Bn.add(k, 1);
  D.Cm.add(n, k);
  D.Cn.add(k, 1);
  GemmCall c;
  c.A = Y;
  c.B = X;
  c.C = P;
  c.sA = c.sC = n * k;
  c.sB = k * k;
  c.batch = batch;
  c.nscale = isig;
  c.nscale_ld = k;
  c.copy_if_zero = copy_flags;
  gemm(ctx, cplx ? Prec::C128 : Prec::F64, D, c);
  stats_reduce(ctx, nullptr, sweeps, batch, ctx.stats_dev);
}

// Alg. 5 in the pass structure of the CholeskyQR path: pass 1 (shifted when
// ill-conditioned), pass 2, the Householder fallback for numerically
// rank-deficient sketches (whose weak and null directions no Gram-based
// factorization resolves), pass 3 for flagged instances.  Y is left intact;
// Y2 is a scratch panel of Y's size.
static void orthogonalize_eigh(Ctx& ctx, bool cplx, const double* Y, double* P, double* Y2, int64_t n, int64_t k,
                               int batch, const OrthWork& w) {
  HP_REQUIRE(!ctx.tape, HPEPS_ERR_UNSUPPORTED, "the Gram-eigendecomposition orthogonalization has no adjoint");
  gram(ctx, cplx, Y, n, k, batch, w.G, nullptr);
  eigh_pass(ctx, cplx, Y, P, n, k, batch, w, 1, nullptr);
  gram(ctx, cplx, P, n, k, batch, w.G, nullptr);
  eigh_pass(ctx, cplx, P, Y2, n, k, batch, w, 2, nullptr);
  householder_qr(ctx, cplx, Y, n, k, batch, w.flags, FLAG_RANK_DEFICIENT, Y2, nullptr);
  gram(ctx, cplx, Y2, n, k, batch, w.G, w.flags);
  eigh_pass(ctx, cplx, Y2, P, n, k, batch, w, 3, w.flags);
  stats_reduce(ctx, w.flags, nullptr, batch, ctx.stats_dev);
}

// Orthonormal basis of range(Y): result in P; Y is overwritten unless the
// Householder fallback may run.  Rt_inv (optional, k x k per instance)
// receives the inverse of the total factor R with Y = P R (the product of
// the passes' inverses).
void orthogonalize(Ctx& ctx, bool cplx, double* Y, double* P, int64_t n, int64_t k, int batch,
                   const OrthWork& w, double* Rt_inv) {
  if (w.mode == HPEPS_ORTH_EIGH) {
    HP_REQUIRE(!Rt_inv, HPEPS_ERR_UNSUPPORTED, "the Gram-eigendecomposition orthogonalization has no adjoint");
    WsScope scope(ctx);
    double* Y2 = ctx.ws<double>((int64_t)batch * n * k * (cplx ? 2 : 1));
    orthogonalize_eigh(ctx, cplx, Y, P, Y2, n, k, batch, w);
    return;
  }
  WsScope scope(ctx);
  // (no fallback under a tape, recording or suspended: the reverse walk
  // differentiates, and a checkpointed row recomputes, the CholeskyQR path)
  const bool fallback = !Rt_inv && !ctx.tape;
  double* S = Rt_inv ? ctx.ws<double>((int64_t)batch * k * k * (cplx ? 2 : 1)) : nullptr;
  // second-pass output: a scratch panel when the fallback may need Y intact
  double* Y2 = fallback ? ctx.ws<double>((int64_t)batch * n * k * (cplx ? 2 : 1)) : Y;
  gram(ctx, cplx, Y, n, k, batch, w.G, nullptr);
  chol_inv(ctx, cplx, w.G, n, k, batch, 1, w.Rinv, nullptr, w.flags);
  apply_rinv(ctx, cplx, Y, n, k, batch, w.Rinv, P, nullptr);
  if (Rt_inv)
    HP_CHECK_HIP(hipMemcpyAsync(Rt_inv, w.Rinv, (size_t)batch * k * k * (cplx ? 16 : 8),
                                hipMemcpyDeviceToDevice, ctx.stream));
  gram(ctx, cplx, P, n, k, batch, w.G, nullptr);
  chol_inv(ctx, cplx, w.G, n, k, batch, 2, w.Rinv, nullptr, w.flags);
  apply_rinv(ctx, cplx, P, n, k, batch, w.Rinv, Y2, nullptr);
  if (Rt_inv) chain_rinv(ctx, cplx, Rt_inv, w.Rinv, S, k, batch);
  // sketches whose second-pass Gram breaks down are numerically
  // rank-deficient: a Gram-based factorization cannot resolve their weak and
  // null directions, so the Householder QR of the original Y replaces the
  // second pass's output (the third pass then leaves it unchanged to
  // rounding).  Not while differentiating: the adjoint of the
  // orthogonalization is the CholeskyQR one.
  if (fallback) householder_qr(ctx, cplx, Y, n, k, batch, w.flags, FLAG_RANK_DEFICIENT, Y2, nullptr);
  // third pass: the Gram only of flagged instances (the factor step writes
  // the identity for the others without reading G); a recording tape keeps
  // every Gram
  gram(ctx, cplx, Y2, n, k, batch, w.G, taping(ctx) ? nullptr : w.flags);
  chol_inv(ctx, cplx, w.G, n, k, batch, 3, w.Rinv, nullptr, w.flags);
  apply_rinv(ctx, cplx, Y2, n, k, batch, w.Rinv, P, w.flags);
  if (Rt_inv) chain_rinv(ctx, cplx, Rt_inv, w.Rinv, S, k, batch);
  stats_reduce(ctx, w.flags, nullptr, batch, ctx.stats_dev);
}

// R factor of the CholeskyQR of Y (accumulated over the passes) into Racc.
void cholqr_r(Ctx& ctx, bool cplx, const double* Y, double* S1, double* S2, int64_t n,
                     int64_t k, int batch, const OrthWork& w) {
  if (w.mode == HPEPS_ORTH_EIGH) {
    // Y = Q R with Q = S2 and R = Q^H Y (exact to rounding once Q is
    // orthonormal with range(Q) = range(Y))
    orthogonalize_eigh(ctx, cplx, Y, S2, S1, n, k, batch, w);
    GemmDesc D;
    D.M = k; D.K = n; D.N = k;
    D.Am.add(k, 1);
    D.Ak.add(n, k);
    D.Bk.add(n, k);
    D.Bn.add(k, 1);
    D.Cm.add(k, k);
    D.Cn.add(k, 1);
    GemmCall c;
    c.A = S2;
    c.B = Y;
    c.C = w.Racc;
    c.sA = c.sB = n * k;
    c.sC = k * k;
    c.batch = batch;
    c.conjA = true;
    gemm(ctx, cplx ? Prec::C128 : Prec::F64, D, c);
    return;
  }
  gram(ctx, cplx, Y, n, k, batch, w.G, nullptr);
  chol_inv(ctx, cplx, w.G, n, k, batch, 1, w.Rinv, w.Racc, w.flags);
  apply_rinv(ctx, cplx, Y, n, k, batch, w.Rinv, S1, nullptr);
  gram(ctx, cplx, S1, n, k, batch, w.G, nullptr);
  chol_inv(ctx, cplx, w.G, n, k, batch, 2, w.Rinv, w.Racc, w.flags);
  apply_rinv(ctx, cplx, S1, n, k, batch, w.Rinv, S2, w.flags);
  gram(ctx, cplx, S2, n, k, batch, w.G, taping(ctx) ? nullptr : w.flags);
  chol_inv(ctx, cplx, w.G, n, k, batch, 3, w.Rinv, w.Racc, w.flags);
  // rank-deficient panels: R of the Householder QR of Y (kept unchanged above)
  if (!ctx.tape) householder_qr(ctx, cplx, Y, n, k, batch, w.flags, FLAG_RANK_DEFICIENT, nullptr, w.Racc);
  stats_reduce(ctx, w.flags, nullptr, batch, ctx.stats_dev);
}

// ---------------------------------------------------------------------------

int64_t sketch_width(int64_t m, int64_t p, int64_t rows, int64_t cols) {
  return std::min(m + p, std::min(rows, cols));
}

// The end of Alg. 4 from an orthonormal basis P of the range (Xr1, rows x k
// per instance) and the projection B^* = A^* P (Xc0, cols x k): the R factor
// of B^*, the small SVD, the canonical phase and the two factors.  Neither
// panel is modified.
static void project_svd(Ctx& ctx, bool cplx, int64_t rows, int64_t cols, int64_t k, int64_t mp, int batch,
                        const hpeps_esvd_opts& o, hpeps_absorb absorb, const ZipOut& out, void* U, double* sigma,
                        void* R, double* log_scale, const double* Xr1, const double* Xc0) {
  WsScope scope(ctx);
  const int es = cplx ? 2 : 1;
  const int64_t nb = batch;
  const int max_sweeps = o.jacobi_max_sweeps > 0 ? o.jacobi_max_sweeps : 40;
  double* Xc1 = ctx.ws<double>(nb * cols * k * es);
  double* Xc2 = ctx.ws<double>(nb * cols * k * es);
  OrthWork ow;
  ow.G = ctx.ws<double>(nb * k * k * es);
  ow.Rinv = ctx.ws<double>(nb * k * k * es);
  ow.Racc = ctx.ws<double>(nb * k * k * es);
  ow.flags = ctx.ws<int>(nb);
  ow.mode = o.orth;
  double* Z = ctx.ws<double>(nb * k * k * es);
  double* sig = ctx.ws<double>(nb * k);
  double* isig = ctx.ws<double>(nb * k);
  double* isig1 = ctx.ws<double>(nb);
  int* sweeps = ctx.ws<int>(nb);
  cholqr_r(ctx, cplx, Xc0, Xc1, Xc2, cols, k, batch, ow);          // R_B in Racc
  jacobi_svd(ctx, cplx, ow.Racc, k, batch, max_sweeps, Z, sig, isig, isig1,
             absorb == HPEPS_ABSORB_CARRY ? log_scale : nullptr, sweeps);
  stats_reduce(ctx, nullptr, sweeps, batch, ctx.stats_dev);

  const Prec p64 = cplx ? Prec::C128 : Prec::F64;
  // canonical phase of the kept singular pairs: U = P Z is formed once in a
  // row-major scratch, Z's columns are rotated, then the factors are formed
  {
    double* Ut = ctx.ws<double>(nb * rows * mp * es);
    GemmDesc D;
    D.M = rows; D.K = k; D.N = mp;
    D.Am.add(rows, k);
    D.Ak.add(k, 1);
    D.Bk.add(k, k);
    D.Bn.add(mp, 1);
    D.Cm.add(rows, mp);
    D.Cn.add(mp, 1);
    GemmCall c;
    c.A = Xr1;
    c.B = Z;
    c.C = Ut;
    c.sA = rows * k;
    c.sB = k * k;
    c.sC = rows * mp;
    c.batch = batch;
    gemm(ctx, p64, D, c);
    gauge_fix(ctx, cplx, Ut, rows, mp, Z, k, batch);
  }
  // sigma^1/2 and sigma^-1/2 for the SQRT split
  double* sq = nullptr;
  double* isq = nullptr;
  if (absorb == HPEPS_ABSORB_SQRT) {
    sq = ctx.ws<double>(nb * k);
    isq = ctx.ws<double>(nb * k);
    sqrt_pair(ctx, sig, nb * k, sq, isq);
  }
  // U = P Z[:, :m'] (times Sigma or Sigma^1/2 for LEFT / SQRT)
  {
    GemmDesc D;
    D.M = rows; D.K = k; D.N = mp;
    D.Am.add(rows, k);
    D.Ak.add(k, 1);
    D.Bk.add(k, k);
    D.Bn.add(mp, 1);
    D.Cm = out.Urows;
    D.Cn = out.Ucol;
    GemmCall c;
    c.A = Xr1;
    c.B = Z;
    c.C = U;
    c.sA = rows * k;
    c.sB = k * k;
    c.sC = out.nU;
    c.batch = batch;
    if (absorb == HPEPS_ABSORB_LEFT || absorb == HPEPS_ABSORB_SQRT) {
      c.nscale = absorb == HPEPS_ABSORB_LEFT ? sig : sq;
      c.nscale_ld = k;
    }
    gemm(ctx, p64, D, c);
  }
  // right factor: (B^* Z[:, :m'])^H, scaled per *absorb*
  {
    GemmDesc D;
    D.M = cols; D.K = k; D.N = mp;
    D.Am.add(cols, k);
    D.Ak.add(k, 1);
    D.Bk.add(k, k);
    D.Bn.add(mp, 1);
    D.Cm = out.Rcols;
    D.Cn = out.Rrow;
    GemmCall c;
    c.A = Xc0;
    c.B = Z;
    c.C = R;
    c.sA = cols * k;
    c.sB = k * k;
    c.sC = out.nR;
    c.batch = batch;
    c.conjC = cplx;
    if (absorb == HPEPS_ABSORB_CARRY) c.scale = isig1;
    if (absorb == HPEPS_ABSORB_NONE || absorb == HPEPS_ABSORB_LEFT || absorb == HPEPS_ABSORB_SQRT) {
      c.nscale = absorb == HPEPS_ABSORB_SQRT ? isq : isig;
      c.nscale_ld = k;
    }
    gemm(ctx, p64, D, c);
  }
  if (sigma) copy_sigma(ctx, sig, k, mp, batch, sigma);
}

// Alg. 4 after the first product: Y0 = A Omega (rows x k per instance) is
// orthogonalized, the q power iterations and the projection B^* = A^* P run
// through `apply` (A X for adj = false, A^* X for adj = true; FP64 /
// complex128 panels), then project_svd finishes.  Y0 is overwritten.
void rsvd_finish(Ctx& ctx, bool cplx, int64_t rows, int64_t cols, int64_t k, int64_t mp, int batch,
                 const hpeps_esvd_opts& o, hpeps_absorb absorb, const ZipOut& out, void* U, double* sigma,
                 void* R, double* log_scale, double* Xr0, const ApplyFn& apply) {
  WsScope scope(ctx);
  const int es = cplx ? 2 : 1;
  const int64_t nb = batch;
  HP_REQUIRE(o.orth == HPEPS_ORTH_CHOLQR || o.orth == HPEPS_ORTH_EIGH, HPEPS_ERR_INVALID_ARG, "unknown orth mode");
  HP_REQUIRE(o.method == HPEPS_ESVD_IMPLICIT || o.method == HPEPS_ESVD_EXPLICIT, HPEPS_ERR_INVALID_ARG,
             "unknown einsumsvd method");
  HP_REQUIRE(o.method == HPEPS_ESVD_IMPLICIT, HPEPS_ERR_UNSUPPORTED,
             "this entry point runs the implicit (randomized) einsumsvd only");
  double* Xc0 = ctx.ws<double>(nb * cols * k * es);
  double* Xc1 = ctx.ws<double>(nb * cols * k * es);
  double* Xr1 = ctx.ws<double>(nb * rows * k * es);
  OrthWork ow;
  ow.G = ctx.ws<double>(nb * k * k * es);
  ow.Rinv = ctx.ws<double>(nb * k * k * es);
  ow.Racc = ctx.ws<double>(nb * k * k * es);
  ow.flags = ctx.ws<int>(nb);
  ow.mode = o.orth;
  orthogonalize(ctx, cplx, Xr0, Xr1, rows, k, batch, ow);          // P in Xr1
  for (int it = 0; it < o.power_iters; ++it) {
    apply(true, Xr1, Xc0);
    orthogonalize(ctx, cplx, Xc0, Xc1, cols, k, batch, ow);        // Q in Xc1
    apply(false, Xc1, Xr0);
    orthogonalize(ctx, cplx, Xr0, Xr1, rows, k, batch, ow);        // P in Xr1
  }
  apply(true, Xr1, Xc0);                                           // B^* = A^* P
  project_svd(ctx, cplx, rows, cols, k, mp, batch, o, absorb, out, U, sigma, R, log_scale, Xr1, Xc0);
}

// Truncated SVD of explicit matrices (the einsumsvd of BMPS, Sec. III-B:
// the network contracted into its matrix, then a dense SVD).  The range
// basis is exact instead of sketched: for rows <= cols, P = I and
// B^* = A^* is M itself ([batch][cols][rows]); otherwise M = A
// ([batch][rows][cols], overwritten) is orthogonalized to P and
// B^* = A^* P comes from adj_apply.  The dense SVD is then the QR of B^*
// and the one-sided Jacobi SVD of its R factor.
void dense_finish(Ctx& ctx, bool cplx, int64_t rows, int64_t cols, int64_t mp, int batch, const hpeps_esvd_opts& o,
                  hpeps_absorb absorb, const ZipOut& out, void* U, double* sigma, void* R, double* log_scale,
                  double* M, const ApplyFn& adj_apply) {
  WsScope scope(ctx);
  const int es = cplx ? 2 : 1;
  const int64_t nb = batch;
  const int64_t k = std::min(rows, cols);
  HP_REQUIRE(o.orth == HPEPS_ORTH_CHOLQR || o.orth == HPEPS_ORTH_EIGH, HPEPS_ERR_INVALID_ARG, "unknown orth mode");
  HP_REQUIRE(!ctx.tape, HPEPS_ERR_UNSUPPORTED, "the explicit einsumsvd has no adjoint");
  HP_REQUIRE(k >= 1 && k <= (cplx ? 88 : 128), HPEPS_ERR_SHAPE,
             "explicit einsumsvd: min(rows, cols) must be <= 128 (88 complex)");
  HP_REQUIRE(mp >= 1 && mp <= k, HPEPS_ERR_SHAPE, "kept rank out of range");
  if (rows <= cols) {
    double* P = ctx.ws<double>(nb * rows * rows * es);
    fill_identity(ctx, P, rows, batch, cplx);
    project_svd(ctx, cplx, rows, cols, k, mp, batch, o, absorb, out, U, sigma, R, log_scale, P, M);
    return;
  }
  double* P = ctx.ws<double>(nb * rows * k * es);
  double* Bs = ctx.ws<double>(nb * cols * k * es);
  OrthWork ow;
  ow.G = ctx.ws<double>(nb * k * k * es);
  ow.Rinv = ctx.ws<double>(nb * k * k * es);
  ow.Racc = ctx.ws<double>(nb * k * k * es);
  ow.flags = ctx.ws<int>(nb);
  ow.mode = o.orth;
  orthogonalize(ctx, cplx, M, P, rows, k, batch, ow);
  adj_apply(true, P, Bs);
  project_svd(ctx, cplx, rows, cols, k, mp, batch, o, absorb, out, U, sigma, R, log_scale, P, Bs);
}

void zip_esvd(Ctx& ctx, bool cplx, const ZipDims& z, const ZipLayout& L, const ZipOperands& op64,
              int batch, const hpeps_esvd_opts& o, hpeps_absorb absorb, const ZipOut& out,
              void* U, double* sigma, void* R, double* log_scale) {
  if (taping(ctx)) {
    HP_REQUIRE(!sigma, HPEPS_ERR_UNSUPPORTED, "tape: singular values are not a differentiable output");
    tape_zip(ctx, cplx, z, L, op64, batch, o, absorb, out, U, R);
  }
  TapeSuspend unrecorded(ctx);
  WsScope scope(ctx);
  const int64_t rows = z.rows(), cols = z.cols();
  const int64_t k = sketch_width(o.rank, o.oversample, rows, cols);
  const int64_t mp = std::min<int64_t>(o.rank, k);
  HP_REQUIRE(k >= 1, HPEPS_ERR_SHAPE, "empty einsumsvd");
  HP_REQUIRE(k <= (cplx ? 88 : 128), HPEPS_ERR_SHAPE, "sketch width k exceeds the small-SVD limit");
  const bool f32 = o.sketch_precision == HPEPS_F32;
  const bool bf16 = o.sketch_precision == HPEPS_BF16;
  const bool narrow = f32 || bf16;
  HP_REQUIRE(!(narrow && cplx), HPEPS_ERR_DTYPE, "FP32 and BF16 sketches are real-only");
  HP_REQUIRE(o.sketch_precision == HPEPS_F64 || narrow, HPEPS_ERR_DTYPE,
             "sketch precision must be F64, F32 or BF16");
  HP_REQUIRE(out.Urows.size() == rows && out.Ucol.size() == mp && out.Rrow.size() == mp &&
                 out.Rcols.size() == cols,
             HPEPS_ERR_SHAPE, "output layout does not match the factor shapes");
  const Prec prec = cplx ? Prec::C128 : (f32 ? Prec::F32 : (bf16 ? Prec::BF16 : Prec::F64));
  const int es = cplx ? 2 : 1;  // doubles per element
  ctx.last_rank = mp;
  ctx.last_k = k;

  // workspace
  const int64_t nb = batch;
  double* Xc0 = ctx.ws<double>(nb * cols * k * es);  // the sketch
  double* Xr0 = ctx.ws<double>(nb * rows * k * es);  // A Omega
  const int64_t esz = f32 ? 4 : (bf16 ? 2 : 8 * es);  // bytes per intermediate element
  ZipWork w;
  w.W1 = ctx.ws_alloc(nb * z.u * z.h * z.d * z.y * z.c * z.g * k * esz);
  w.W2 = ctx.ws_alloc(nb * zip_w2_elems(z, k) * esz);
  w.W3 = ctx.ws_alloc(nb * z.b * z.h * z.h * k * esz);

  // operands in the apply precision
  ZipOperands op = op64;
  float* xin32 = nullptr;
  void* xin16 = nullptr;
  if (bf16) {
    void* parts[4];
    const void* src[4] = {op64.V, op64.S, op64.T, op64.Bra};
    const int64_t cnt[4] = {L.nV, L.nS, L.nT, L.nB};
    for (int i = 0; i < 4; ++i) {
      parts[i] = ctx.ws_alloc(nb * cnt[i] * 2);
      convert_f64_to_bf16(ctx, (const double*)src[i], parts[i], nb * cnt[i]);
    }
    op.V = parts[0];
    op.S = parts[1];
    op.T = parts[2];
    op.Bra = parts[3];
    xin16 = ctx.ws_alloc(nb * std::max(rows, cols) * k * 2);
  }
  if (f32) {
    float* V32 = ctx.ws<float>(nb * L.nV);
    float* S32 = ctx.ws<float>(nb * L.nS);
    float* T32 = ctx.ws<float>(nb * L.nT);
    float* B32 = ctx.ws<float>(nb * L.nB);
    convert_f64_to_f32(ctx, (const double*)op64.V, V32, nb * L.nV);
    convert_f64_to_f32(ctx, (const double*)op64.S, S32, nb * L.nS);
    convert_f64_to_f32(ctx, (const double*)op64.T, T32, nb * L.nT);
    convert_f64_to_f32(ctx, (const double*)op64.Bra, B32, nb * L.nB);
    op.V = V32;
    op.S = S32;
    op.T = T32;
    op.Bra = B32;
    xin32 = ctx.ws<float>(nb * std::max(rows, cols) * k);
  }
  auto apply = [&](bool adj, const double* X, double* Y) {
    const void* xin = X;
    if (f32) {
      convert_f64_to_f32(ctx, X, xin32, nb * (adj ? rows : cols) * k);
      xin = xin32;
    }
    if (bf16) {
      convert_f64_to_bf16(ctx, X, xin16, nb * (adj ? rows : cols) * k);
      xin = xin16;
    }
    zip_apply(ctx, prec, z, L, op, batch, k, adj, xin, Y, true, w);
  };

  // Alg. 4
  if (f32) {
    sketch(ctx, xin32, true, cols, k, batch, o.seed, o.stream_id);
    zip_apply(ctx, prec, z, L, op, batch, k, false, xin32, Xr0, true, w);
  } else if (bf16) {
    sketch(ctx, Xc0, false, cols, k, batch, o.seed, o.stream_id);
    apply(false, Xc0, Xr0);
  } else {
    sketch(ctx, Xc0, false, cols, k, batch, o.seed, o.stream_id, cplx);
    zip_apply(ctx, prec, z, L, op, batch, k, false, Xc0, Xr0, true, w);
  }
  rsvd_finish(ctx, cplx, rows, cols, k, mp, batch, o, absorb, out, U, sigma, R, log_scale, Xr0, apply);
}

// ---------------------------------------------------------------------------
// exact carry of one column: V[a,x,X,b,h,H] = sum_{u,U,p} L[a,u,U,b] T[u,x,h,p] conj(Bra[U,X,H,p])
void form_carry(Ctx& ctx, bool cplx, const CarryDims& cd, const CarryLayout& cl, const void* L,
                const void* T, const void* Bra, void* V, int batch) {
  tape_carry(ctx, cplx, cd, cl, L, T, Bra, V, batch);
  TapeSuspend unrecorded(ctx);
  WsScope scope(ctx);
  const int64_t a = cd.a, u = cd.u, b = cd.b, x = cd.x, h = cd.h, d = cd.d;
  const Prec p = cplx ? Prec::C128 : Prec::F64;
  const int es = cplx ? 2 : 1;
  // X1[a,U,b,x,h,p]
  const int64_t Xp = 1, Xh = d, Xx = h * d, Xb = x * Xx, XU = b * Xb, Xa = u * XU;
  // V[a,x,X,b,h,H]
  const int64_t VH = 1, Vh = h, Vb = h * h, VX = b * Vb, Vx = x * VX, Va = x * Vx;
  const int64_t nX1 = a * u * b * x * h * d, nV = a * x * x * b * h * h;
  double* X1 = ctx.ws<double>((int64_t)batch * nX1 * es);
  {
    GemmDesc D;
    D.M = a * u * b; D.K = u; D.N = x * h * d;
    D.Am.add(a, cl.L[0]).add(u, cl.L[2]).add(b, cl.L[3]);
    D.Ak.add(u, cl.L[1]);
    D.Bk.add(u, cl.T[0]);
    D.Bn.add(x, cl.T[1]).add(h, cl.T[2]).add(d, cl.T[3]);
    D.Cm.add(a, Xa).add(u, XU).add(b, Xb);
    D.Cn.add(x, Xx).add(h, Xh).add(d, Xp);
    GemmCall c;
    c.A = L;
    c.B = T;
    c.C = X1;
    c.sA = cl.nL;
    c.sB = cl.nT;
    c.sC = nX1;
    c.batch = batch;
    gemm(ctx, p, D, c);
  }
  {
    GemmDesc D;
    D.M = a * b * x * h; D.K = u * d; D.N = x * h;
    D.Am.add(a, Xa).add(b, Xb).add(x, Xx).add(h, Xh);
    D.Ak.add(u, XU).add(d, Xp);
    D.Bk.add(u, cl.B[0]).add(d, cl.B[3]);
    D.Bn.add(x, cl.B[1]).add(h, cl.B[2]);
    D.Cm.add(a, Va).add(b, Vb).add(x, Vx).add(h, Vh);
    D.Cn.add(x, VX).add(h, VH);
    GemmCall c;
    c.A = X1;
    c.B = Bra;
    c.C = V;
    c.sA = nX1;
    c.sB = cl.nB;
    c.sC = nV;
    c.batch = batch;
    c.conjB = cplx;
    gemm(ctx, p, D, c);
  }
}

}  // namespace hp
