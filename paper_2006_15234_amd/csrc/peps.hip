// Boundary-MPS contraction of two-layer PEPS networks (Algs. 2-3).
//
// * The first row is absorbed exactly (its boundary bond is the ket bond
//   times the bra bond).
// * Every later row but the last is absorbed by the zip-up: the first
//   column's carry is contracted exactly, every later column runs one
//   randomized einsumsvd whose isometric left factor becomes the finished
//   boundary tensor and whose right factor Sigma/sigma_1 V^* is the next carry.
// * The sweep direction alternates between rows.  A right-to-left sweep is
//   the left-to-right sweep of the mirrored lattice; mirroring only permutes
//   the strides handed to the gathered GEMMs (no data is moved), and the
//   factors are written straight into the canonical [mL, x, X, mR] layout.
// * The last row is contracted exactly into a scalar.
// All normalisation factors are accumulated as logarithms on the device.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "peps.h"
#include <memory>

#include "tape.h"

namespace hp {

namespace {
std::vector<int64_t> rm(const std::vector<int64_t>& d) { return rm_strides(d); }
}  // namespace

SiteView orient_site(const DevTensor& t, Side side, Dir dir) {
  HP_REQUIRE(t.dims.size() == 5, HPEPS_ERR_SHAPE, "site tensors have 5 legs");
  const auto s = rm(t.dims);
  const int up = side == kTop ? 0 : 1, down = side == kTop ? 1 : 0;
  const int left = dir == kL2R ? 2 : 3, right = dir == kL2R ? 3 : 2;
  const int roles[5] = {up, down, left, right, 4};
  SiteView v;
  v.p = t.p;
  for (int i = 0; i < 5; ++i) {
    v.n[i] = t.dims[roles[i]];
    v.s[i] = s[roles[i]];
  }
  v.extent = t.size();
  return v;
}

BndView orient_bnd(const DevTensor& t, Dir dir) {
  HP_REQUIRE(t.dims.size() == 4, HPEPS_ERR_SHAPE, "boundary tensors have 4 legs");
  const auto s = rm(t.dims);
  const int roles[4] = {dir == kL2R ? 0 : 3, 1, 2, dir == kL2R ? 3 : 0};
  BndView v;
  v.p = t.p;
  for (int i = 0; i < 4; ++i) {
    v.n[i] = t.dims[roles[i]];
    v.s[i] = s[roles[i]];
  }
  v.extent = t.size();
  return v;
}

void first_row_boundary(Ctx& ctx, bool cplx, const std::vector<SiteView>& ket,
                        const std::vector<SiteView>& bra, std::vector<DevTensor>& out,
                        double* log_dev) {
  const Prec p = cplx ? Prec::C128 : Prec::F64;
  for (size_t j = 0; j < ket.size(); ++j) {
    const SiteView &T = ket[j], &B = bra[j];
    HP_REQUIRE(T.n[0] == 1 && B.n[0] == 1, HPEPS_ERR_SHAPE, "first-row sites must have outer legs of dim 1");
    HP_REQUIRE(T.n[4] == B.n[4], HPEPS_ERR_SHAPE, "ket/bra physical dims differ");
    const int64_t l = T.n[2], x = T.n[1], r = T.n[3], L = B.n[2], X = B.n[1], R = B.n[3], d = T.n[4];
    DevTensor& o = out[j];
    HP_REQUIRE(o.size() == l * L * x * X * r * R, HPEPS_ERR_SHAPE, "first-row output buffer size");
    const int64_t sR = 1, sr = R, sX = r * R, sx = X * sX, sL = x * sx, sl = L * sL;
    GemmDesc D;
    D.M = l * x * r; D.K = d; D.N = L * X * R;
    D.Am.add(l, T.s[2]).add(x, T.s[1]).add(r, T.s[3]);
    D.Ak.add(d, T.s[4]);
    D.Bk.add(d, B.s[4]);
    D.Bn.add(L, B.s[2]).add(X, B.s[1]).add(R, B.s[3]);
    D.Cm.add(l, sl).add(x, sx).add(r, sr);
    D.Cn.add(L, sL).add(X, sX).add(R, sR);
    GemmCall c;
    c.A = T.p;
    c.B = B.p;
    c.C = o.p;
    c.sA = T.extent;
    c.sB = B.extent;
    c.sC = o.size();
    c.conjB = cplx;
    gemm(ctx, p, D, c);
    normalize(ctx, cplx, o.p, o.size(), 1, log_dev);
  }
}

std::vector<std::array<int64_t, 4>> absorb_shapes(const std::vector<BndView>& bnd,
                                                  const std::vector<SiteView>& ket, int64_t m,
                                                  int64_t p) {
  const size_t n = ket.size();
  std::vector<std::array<int64_t, 4>> sh(n);
  int64_t a = bnd[0].n[0], x = ket[0].n[1], b = bnd[0].n[3], h = ket[0].n[3];
  for (size_t j = 1; j < n; ++j) {
    const int64_t y = ket[j].n[1], c = bnd[j].n[3], g = ket[j].n[3];
    const int64_t rows = a * x * x, cols = y * y * c * g * g;
    const int64_t k = sketch_width(m, p, rows, cols);
    const int64_t mp = std::min(m, k);
    sh[j - 1] = {a, x, x, mp};
    a = mp;
    x = y;
    b = c;
    h = g;
  }
  sh[n - 1] = {a, x, x, b * h * h};
  return sh;
}

void absorb_row(Ctx& ctx, bool cplx, const std::vector<BndView>& bnd,
                const std::vector<SiteView>& ket, const std::vector<SiteView>& bra, Dir dir,
                const hpeps_esvd_opts& o, const std::vector<uint64_t>& stream_ids,
                std::vector<DevTensor>& out, double* log_dev) {
  const size_t n = ket.size();
  const int es = cplx ? 2 : 1;
  HP_REQUIRE(bnd.size() == n && bra.size() == n && out.size() == n && stream_ids.size() == n,
             HPEPS_ERR_SHAPE, "row lengths differ");
  for (size_t j = 0; j < n; ++j) {
    HP_REQUIRE(bnd[j].n[1] == ket[j].n[0] && bnd[j].n[2] == bra[j].n[0], HPEPS_ERR_SHAPE,
               "boundary legs do not match the row's up legs");
    for (int q = 0; q < 5; ++q)
      HP_REQUIRE(ket[j].n[q] == bra[j].n[q], HPEPS_ERR_SHAPE, "bra and ket shapes differ");
    if (j > 0) {
      HP_REQUIRE(bnd[j].n[0] == bnd[j - 1].n[3], HPEPS_ERR_SHAPE, "boundary bonds do not chain");
      HP_REQUIRE(ket[j].n[2] == ket[j - 1].n[3], HPEPS_ERR_SHAPE, "site bonds do not chain");
    }
  }
  HP_REQUIRE(bnd[0].n[0] == 1 && bnd[n - 1].n[3] == 1 && ket[0].n[2] == 1 && ket[n - 1].n[3] == 1,
             HPEPS_ERR_SHAPE, "open boundary legs must have dim 1");
  const auto shapes = absorb_shapes(bnd, ket, o.rank, o.oversample);

  // carry buffers (row-major V[a,x,X,b,h,H])
  int64_t maxv = 0;
  {
    int64_t a = bnd[0].n[0], x = ket[0].n[1], b = bnd[0].n[3], h = ket[0].n[3];
    maxv = a * x * x * b * h * h;
    for (size_t j = 1; j < n; ++j) {
      const int64_t mp = shapes[j - 1][3];
      a = mp;
      x = ket[j].n[1];
      b = bnd[j].n[3];
      h = ket[j].n[3];
      maxv = std::max(maxv, a * x * x * b * h * h);
    }
  }
  WsScope scope(ctx);
  double* carry[2] = {ctx.ws<double>(maxv * es), ctx.ws<double>(maxv * es)};

  // first column: exact carry
  {
    CarryDims cd;
    cd.a = bnd[0].n[0]; cd.u = ket[0].n[0]; cd.b = bnd[0].n[3];
    cd.x = ket[0].n[1]; cd.h = ket[0].n[3]; cd.d = ket[0].n[4];
    CarryLayout cl;
    for (int q = 0; q < 4; ++q) cl.L[q] = bnd[0].s[q];
    const int tr[4] = {0, 1, 3, 4};  // u, x(down), h(right), p
    for (int q = 0; q < 4; ++q) {
      cl.T[q] = ket[0].s[tr[q]];
      cl.B[q] = bra[0].s[tr[q]];
    }
    cl.nL = bnd[0].extent;
    cl.nT = ket[0].extent;
    cl.nB = bra[0].extent;
    form_carry(ctx, cplx, cd, cl, bnd[0].p, ket[0].p, bra[0].p, carry[0], 1);
    const int64_t nv = cd.a * cd.x * cd.x * cd.b * cd.h * cd.h;
    normalize(ctx, cplx, carry[0], nv, 1, log_dev);
    if (n == 1) {
      // a one-column row has no einsumsvd: the exact carry is the boundary
      // ([1, x, X, 1] in either direction)
      out[0].dims = {cd.a, cd.x, cd.x, cd.b * cd.h * cd.h};
      HP_CHECK_HIP(hipMemcpyAsync(out[0].p, carry[0], nv * es * sizeof(double), hipMemcpyDeviceToDevice,
                                  ctx.stream));
      tape_copy(ctx, cplx, out[0].p, carry[0], nv);
      return;
    }
  }
  int cur = 0;
  int64_t a = bnd[0].n[0], x = ket[0].n[1], b = bnd[0].n[3], h = ket[0].n[3];
  for (size_t j = 1; j < n; ++j) {
    ZipDims z;
    z.a = a; z.x = x; z.b = b; z.h = h;
    z.u = ket[j].n[0]; z.c = bnd[j].n[3]; z.y = ket[j].n[1]; z.g = ket[j].n[3]; z.d = ket[j].n[4];
    ZipLayout L = ZipLayout::row_major(z);
    for (int q = 0; q < 4; ++q) L.S[q] = bnd[j].s[q];
    for (int q = 0; q < 5; ++q) {
      L.T[q] = ket[j].s[q];
      L.B[q] = bra[j].s[q];
    }
    L.nS = bnd[j].extent;
    L.nT = ket[j].extent;
    L.nB = bra[j].extent;
    const int64_t mp = shapes[j - 1][3];
    const int64_t rows = z.rows(), cols = z.cols();
    ZipOut zo;
    // finished tensor of sweep position j-1, oriented [a, x, X, mp]
    DevTensor& U = out[j - 1];
    if (dir == kL2R) {
      U.dims = {a, x, x, mp};
      zo.Urows.add(a, x * x * mp).add(x, x * mp).add(x, mp);
      zo.Ucol.add(mp, 1);
    } else {
      U.dims = {mp, x, x, a};
      zo.Urows.add(a, 1).add(x, x * a).add(x, a);
      zo.Ucol.add(mp, x * x * a);
    }
    zo.nU = rows * mp;
    void* Rp;
    if (j + 1 < n) {
      zo.Rrow.add(mp, cols);
      zo.Rcols.add(cols, 1);
      zo.nR = mp * cols;
      Rp = carry[1 - cur];
    } else {
      DevTensor& last = out[n - 1];
      const int64_t y = z.y, cgg = z.c * z.g * z.g;
      if (dir == kL2R) {
        last.dims = {mp, y, y, cgg};
        zo.Rrow.add(mp, cols);
        zo.Rcols.add(cols, 1);
      } else {
        last.dims = {cgg, y, y, mp};
        // cgg == 1 at the end of a row: element (i, y, Y) at y Y mp + Y mp + i
        zo.Rrow.add(mp, 1);
        zo.Rcols.add(y, y * mp).add(y, mp).add(cgg, 1);
      }
      zo.nR = mp * cols;
      Rp = last.p;
    }
    hpeps_esvd_opts oj = o;
    oj.stream_id = stream_ids[j];
    // a recording tape needs every carry kept: no ping-pong reuse
    if (taping(ctx) && j + 1 < n) Rp = carry[1 - cur] = ctx.ws<double>(maxv * es);
    ZipOperands op{carry[cur], bnd[j].p, ket[j].p, bra[j].p};
    zip_esvd(ctx, cplx, z, L, op, 1, oj, HPEPS_ABSORB_CARRY, zo, U.p, nullptr, Rp, log_dev);
    cur = 1 - cur;
    a = mp;
    x = z.y;
    b = z.c;
    h = z.g;
  }
}

void absorb_row_recorded(Ctx& ctx, bool cplx, const std::vector<BndView>& bnd,
                         const std::vector<SiteView>& ket, const std::vector<SiteView>& bra, Dir dir,
                         const hpeps_esvd_opts& o, const std::vector<uint64_t>& stream_ids,
                         std::vector<DevTensor>& out, double* log_dev) {
  if (!taping(ctx) || !ctx.checkpoint_rows) {
    absorb_row(ctx, cplx, bnd, ket, bra, dir, o, stream_ids, out, log_dev);
    return;
  }
  {
    TapeSuspend unrecorded(ctx);  // the row's workspace is released at its end
    absorb_row(ctx, cplx, bnd, ket, bra, dir, o, stream_ids, out, log_dev);
  }
  auto w = std::make_shared<RowCheckpoint>();
  w->cplx = cplx;
  w->bnd = bnd;
  w->ket = ket;
  w->bra = bra;
  w->dir = dir;
  w->o = o;
  w->sids = stream_ids;
  w->out = out;
  TapeOp op;
  op.kind = TapeOp::ROW;
  op.row = w;
  ctx.tape->record(op);
}

void row_backward(Ctx& ctx, const RowCheckpoint& r, Tape& main, double broadening) {
  const int es = r.cplx ? 2 : 1;
  bool any = false;
  for (const auto& t : r.out) any = any || main.grad_if_live(t.p);
  if (!any) return;
  // the inputs that carry gradients; their adjoints in the main tape are
  // allocated before the recompute's scope (they outlive it)
  std::vector<std::pair<const void*, int64_t>> ins;
  auto add = [&](const void* p, int64_t n) {
    if (!main.depends(p)) return;
    for (auto& e : ins)
      if (e.first == p) {
        e.second = std::max(e.second, n);
        return;
      }
    ins.push_back({p, n});
  };
  for (const auto& b : r.bnd) add(b.p, b.extent);
  for (const auto& t : r.ket) add(t.p, t.extent);
  for (const auto& t : r.bra) add(t.p, t.extent);
  std::vector<double*> gmain;
  for (auto& e : ins) gmain.push_back(main.grad(ctx, e.first));
  WsScope scope(ctx);
  std::vector<DevTensor> out2 = r.out;
  for (auto& t : out2) t.p = ctx.ws<double>(t.size() * es);
  double* logd = ctx.ws<double>(1);
  fill_zero(ctx, logd, sizeof(double));
  Tape sub(r.cplx);
  for (auto& e : ins) sub.mark_input(e.first, e.second);
  ctx.tape = &sub;
  try {
    absorb_row(ctx, r.cplx, r.bnd, r.ket, r.bra, r.dir, r.o, r.sids, out2, logd);
  } catch (...) {
    ctx.tape = nullptr;
    throw;
  }
  ctx.tape = nullptr;
  for (size_t q = 0; q < r.out.size(); ++q) {
    const double* g = main.grad_if_live(r.out[q].p);
    if (g && sub.depends(out2[q].p))
      HP_CHECK_HIP(hipMemcpyAsync(sub.grad(ctx, out2[q].p), g, out2[q].size() * es * sizeof(double),
                                  hipMemcpyDeviceToDevice, ctx.stream));
  }
  sub.backward(ctx, broadening);
  for (size_t i = 0; i < ins.size(); ++i) {
    const double* g = sub.grad_if_live(ins[i].first);
    if (g) axpy(ctx, gmain[i], g, 1.0, ins[i].second * es);
  }
}

void contract_last_row(Ctx& ctx, bool cplx, const std::vector<BndView>& bnd,
                       const std::vector<SiteView>& ket, const std::vector<SiteView>& bra,
                       double* result_dev, double* log_dev, double** final_E) {
  const Prec pr = cplx ? Prec::C128 : Prec::F64;
  const int es = cplx ? 2 : 1;
  const size_t n = ket.size();
  int64_t maxe = 1, max1 = 1, max2 = 1;
  for (size_t j = 0; j < n; ++j) {
    HP_REQUIRE(ket[j].n[1] == 1 && bra[j].n[1] == 1, HPEPS_ERR_SHAPE, "last-row sites must have down legs of dim 1");
    HP_REQUIRE(bnd[j].n[1] == ket[j].n[0] && bnd[j].n[2] == bra[j].n[0], HPEPS_ERR_SHAPE,
               "boundary legs do not match the last row");
    const int64_t b = bnd[j].n[0], u = bnd[j].n[1], c = bnd[j].n[3], h = ket[j].n[2], g = ket[j].n[3];
    maxe = std::max(maxe, std::max(b * h * h, c * g * g));
    max1 = std::max(max1, h * h * u * u * c);
    max2 = std::max(max2, h * u * c * g * ket[j].n[4]);
  }
  WsScope scope(ctx);
  double* E[2] = {ctx.ws<double>(maxe * es), ctx.ws<double>(maxe * es)};
  double* X1 = ctx.ws<double>(max1 * es);
  double* X2 = ctx.ws<double>(max2 * es);
  fill_value(ctx, E[0], 1, 1.0, cplx);
  int cur = 0;
  for (size_t j = 0; j < n; ++j) {
    if (taping(ctx)) {  // a recording tape keeps every intermediate
      E[1 - cur] = ctx.ws<double>(maxe * es);
      X1 = ctx.ws<double>(max1 * es);
      X2 = ctx.ws<double>(max2 * es);
    }
    const BndView& S = bnd[j];
    const SiteView &T = ket[j], &B = bra[j];
    const int64_t b = S.n[0], u = S.n[1], U = S.n[2], c = S.n[3];
    const int64_t h = T.n[2], H = B.n[2], g = T.n[3], G = B.n[3], d = T.n[4];
    HP_REQUIRE(h * H == (j == 0 ? 1 : h * H), HPEPS_ERR_SHAPE, "bond mismatch");
    // e1: X1[h,H,u,U,c] = sum_b E[b,h,H] S[b,u,U,c]
    {
      GemmDesc D;
      D.M = h * H; D.K = b; D.N = u * U * c;
      D.Am.add(h, H).add(H, 1);
      D.Ak.add(b, h * H);
      D.Bk.add(b, S.s[0]);
      D.Bn.add(u, S.s[1]).add(U, S.s[2]).add(c, S.s[3]);
      D.Cm.add(h * H, u * U * c);
      D.Cn.add(u * U * c, 1);
      GemmCall gc;
      gc.A = E[cur]; gc.B = S.p; gc.C = X1;
      gc.sA = b * h * H; gc.sB = S.extent; gc.sC = h * H * u * U * c;
      gemm(ctx, pr, D, gc);
    }
    // e2: X2[H,U,c,g,p] = sum_{h,u} X1[h,H,u,U,c] T[u,1,h,g,p]
    {
      GemmDesc D;
      D.M = H * U * c; D.K = h * u; D.N = g * d;
      D.Am.add(H, u * U * c).add(U, c).add(c, 1);
      D.Ak.add(h, H * u * U * c).add(u, U * c);
      D.Bk.add(h, T.s[2]).add(u, T.s[0]);
      D.Bn.add(g, T.s[3]).add(d, T.s[4]);
      D.Cm.add(H * U * c, g * d);
      D.Cn.add(g * d, 1);
      GemmCall gc;
      gc.A = X1; gc.B = T.p; gc.C = X2;
      gc.sA = h * H * u * U * c; gc.sB = T.extent; gc.sC = H * U * c * g * d;
      gemm(ctx, pr, D, gc);
    }
    // e3: E'[c,g,G] = sum_{H,U,p} X2[H,U,c,g,p] conj(Bra[U,1,H,G,p])
    {
      GemmDesc D;
      D.M = c * g; D.K = H * U * d; D.N = G;
      D.Am.add(c, g * d).add(g, d);
      D.Ak.add(H, U * c * g * d).add(U, c * g * d).add(d, 1);
      D.Bk.add(H, B.s[2]).add(U, B.s[0]).add(d, B.s[4]);
      D.Bn.add(G, B.s[3]);
      D.Cm.add(c * g, G);
      D.Cn.add(G, 1);
      GemmCall gc;
      gc.A = X2; gc.B = B.p; gc.C = E[1 - cur];
      gc.sA = H * U * c * g * d; gc.sB = B.extent; gc.sC = c * g * G;
      gc.conjB = cplx;
      gemm(ctx, pr, D, gc);
    }
    cur = 1 - cur;
    normalize(ctx, cplx, E[cur], c * g * G, 1, log_dev);
  }
  // the last E is a single element; normalize divided it by |E|, so recover
  // the mantissa as phase only: result = E (unit modulus) and log holds |E|
  copy_scalar(ctx, E[cur], cplx, result_dev);
  if (final_E) *final_E = E[cur];
}

Lattice lattice_from_abi(const hpeps_peps* p) {
  HP_REQUIRE(p && p->nrow >= 1 && p->ncol >= 1 && p->sites && p->shapes, HPEPS_ERR_INVALID_ARG,
             "bad PEPS descriptor");
  HP_REQUIRE(p->dtype == HPEPS_F64 || p->dtype == HPEPS_C128, HPEPS_ERR_DTYPE, "PEPS dtype F64 or C128");
  Lattice L;
  L.nrow = p->nrow;
  L.ncol = p->ncol;
  L.cplx = p->dtype == HPEPS_C128;
  for (int i = 0; i < p->nrow; ++i)
    for (int j = 0; j < p->ncol; ++j) {
      const int q = i * p->ncol + j;
      DevTensor t;
      t.p = p->sites[q];
      HP_REQUIRE(t.p, HPEPS_ERR_INVALID_ARG, "null site pointer");
      t.dims.assign(p->shapes + 5 * q, p->shapes + 5 * q + 5);
      for (auto dd : t.dims) HP_REQUIRE(dd >= 1, HPEPS_ERR_SHAPE, "site dims must be >= 1");
      HP_REQUIRE(t.dims[0] == 1 || i > 0, HPEPS_ERR_SHAPE, "top legs must have dim 1");
      HP_REQUIRE(t.dims[1] == 1 || i < p->nrow - 1, HPEPS_ERR_SHAPE, "bottom legs must have dim 1");
      HP_REQUIRE(t.dims[2] == 1 || j > 0, HPEPS_ERR_SHAPE, "left legs must have dim 1");
      HP_REQUIRE(t.dims[3] == 1 || j < p->ncol - 1, HPEPS_ERR_SHAPE, "right legs must have dim 1");
      L.sites.push_back(t);
    }
  for (int i = 0; i < L.nrow; ++i)
    for (int j = 0; j < L.ncol; ++j) {
      if (j + 1 < L.ncol)
        HP_REQUIRE(L.at(i, j).dims[3] == L.at(i, j + 1).dims[2], HPEPS_ERR_SHAPE, "horizontal bond mismatch");
      if (i + 1 < L.nrow)
        HP_REQUIRE(L.at(i, j).dims[1] == L.at(i + 1, j).dims[0], HPEPS_ERR_SHAPE, "vertical bond mismatch");
      HP_REQUIRE(L.at(i, j).dims[4] == L.at(0, 0).dims[4], HPEPS_ERR_SHAPE, "physical dims differ");
    }
  return L;
}

void write_site_grads(Ctx& ctx, const Tape& tape, const Lattice& K, void* const* grads) {
  const int es = K.cplx ? 2 : 1;
  for (size_t q = 0; q < K.sites.size(); ++q) {
    const int64_t bytes = K.sites[q].size() * es * (int64_t)sizeof(double);
    const double* g = tape.grad_if_live(K.sites[q].p);
    if (g)
      HP_CHECK_HIP(hipMemcpyAsync(grads[q], g, bytes, hipMemcpyDeviceToDevice, ctx.stream));
    else
      fill_zero(ctx, grads[q], bytes);
  }
}

Lattice normalized_copy(Ctx& ctx, const Lattice& L, double* log_dev) {
  Lattice out = L;
  const int es = L.cplx ? 2 : 1;
  for (auto& t : out.sites) {
    double* p = ctx.ws<double>(t.size() * es);
    HP_CHECK_HIP(hipMemcpyAsync(p, t.p, t.size() * es * sizeof(double), hipMemcpyDeviceToDevice, ctx.stream));
    tape_copy(ctx, L.cplx, p, t.p, t.size());
    normalize(ctx, L.cplx, p, t.size(), 1, log_dev);
    t.p = p;
  }
  return out;
}

void boundary_pass(Ctx& ctx, const Lattice& ket, const Lattice& bra, Side side,
                   const hpeps_esvd_opts& o, int upto, std::vector<std::vector<DevTensor>>& envs,
                   double* log_dev) {
  const int nrow = ket.nrow, ncol = ket.ncol;
  const bool cplx = ket.cplx;
  const int es = cplx ? 2 : 1;
  auto orow = [&](int t) { return side == kTop ? t : nrow - 1 - t; };
  envs.clear();
  {
    std::vector<SiteView> kv, bv;
    std::vector<DevTensor> out(ncol);
    for (int j = 0; j < ncol; ++j) {
      kv.push_back(orient_site(ket.at(orow(0), j), side, kL2R));
      bv.push_back(orient_site(bra.at(orow(0), j), side, kL2R));
      out[j].dims = {kv[j].n[2] * bv[j].n[2], kv[j].n[1], bv[j].n[1], kv[j].n[3] * bv[j].n[3]};
      out[j].p = ctx.ws<double>(out[j].size() * es);
    }
    first_row_boundary(ctx, cplx, kv, bv, out, log_dev);
    envs.push_back(out);
  }
  for (int t = 1; t < upto; ++t) {
    const int r = orow(t);
    const Dir dir = (t % 2 == 1) ? kL2R : kR2L;
    std::vector<BndView> bnd;
    std::vector<SiteView> kv, bv;
    std::vector<uint64_t> sids;
    for (int q = 0; q < ncol; ++q) {
      const int col = dir == kL2R ? q : ncol - 1 - q;
      bnd.push_back(orient_bnd(envs.back()[col], dir));
      kv.push_back(orient_site(ket.at(r, col), side, dir));
      bv.push_back(orient_site(bra.at(r, col), side, dir));
      sids.push_back(1 + ((uint64_t)(side * nrow + r) * ncol + col));
    }
    const auto shapes = absorb_shapes(bnd, kv, o.rank, o.oversample);
    std::vector<DevTensor> out(ncol);
    for (int q = 0; q < ncol; ++q) {
      int64_t sz = 1;
      for (auto v : shapes[q]) sz *= v;
      out[q].p = ctx.ws<double>(sz * es);
    }
    absorb_row_recorded(ctx, cplx, bnd, kv, bv, dir, o, sids, out, log_dev);
    std::vector<DevTensor> env(ncol);
    for (int q = 0; q < ncol; ++q) env[dir == kL2R ? q : ncol - 1 - q] = out[q];
    envs.push_back(env);
  }
}

}  // namespace hp

// ---------------------------------------------------------------------------
// ABI

namespace {
template <class F>
hpeps_status guard_p(hpeps_ctx* ctx, F&& f) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  try {
    ctx->impl->ws_reset();
    f(*ctx->impl);
    return HPEPS_OK;
  } catch (const hp::Error& e) {
    ctx->impl->tape = nullptr;
    ctx->impl->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->impl->tape = nullptr;
    ctx->impl->last_error = "host allocation failed";
    return HPEPS_ERR_ALLOC;
  } catch (...) {
    ctx->impl->tape = nullptr;
    ctx->impl->last_error = "unknown error";
    return HPEPS_ERR_INVALID_ARG;
  }
}

void check_opts_p(const hpeps_esvd_opts* o) {
  HP_REQUIRE(o, HPEPS_ERR_INVALID_ARG, "opts is NULL");
  HP_REQUIRE(o->rank >= 1 && o->oversample >= 0 && o->power_iters >= 0 && o->jacobi_max_sweeps >= 0,
             HPEPS_ERR_INVALID_ARG, "bad einsumsvd options");
}
// <bra|ket> by boundary MPS: dev[0] += log scale, dev[1..2] = phase; the
// final unit-modulus mantissa buffer is returned through final_E.
void norm_run(hp::Ctx& c, const hp::Lattice& K, const hp::Lattice& B, const hpeps_esvd_opts& o, double* dev,
              double** final_E) {
  HP_REQUIRE(B.nrow == K.nrow && B.ncol == K.ncol && B.cplx == K.cplx, HPEPS_ERR_SHAPE,
             "bra and ket lattices differ");
  for (size_t q = 0; q < K.sites.size(); ++q)
    for (int e = 0; e < 5; ++e)
      HP_REQUIRE(K.sites[q].dims[e] == B.sites[q].dims[e], HPEPS_ERR_SHAPE, "bra and ket shapes differ");
  hp::fill_value(c, dev, 1, 0.0, false);
  // the bra layer is rescaled separately even when it is the ket itself:
  // both layers' norms enter <bra|ket>
  hp::Lattice Kn = hp::normalized_copy(c, K, dev);
  hp::Lattice Bn = hp::normalized_copy(c, B, dev);
  std::vector<hp::BndView> bv;
  std::vector<hp::SiteView> kv, brv;
  std::vector<std::vector<hp::DevTensor>> envs;
  std::vector<hp::DevTensor> triv;
  if (K.nrow == 1) {
    const int es = K.cplx ? 2 : 1;
    for (int j = 0; j < K.ncol; ++j) {
      hp::DevTensor t;
      t.dims = {1, 1, 1, 1};
      t.p = c.ws<double>(es);
      hp::fill_value(c, (double*)t.p, 1, 1.0, K.cplx);
      triv.push_back(t);
    }
    for (int j = 0; j < K.ncol; ++j) bv.push_back(hp::orient_bnd(triv[j], hp::kL2R));
  } else {
    hp::boundary_pass(c, Kn, Bn, hp::kTop, o, K.nrow - 1, envs, dev);
    for (int j = 0; j < K.ncol; ++j) bv.push_back(hp::orient_bnd(envs.back()[j], hp::kL2R));
  }
  for (int j = 0; j < K.ncol; ++j) {
    kv.push_back(hp::orient_site(Kn.at(K.nrow - 1, j), hp::kTop, hp::kL2R));
    brv.push_back(hp::orient_site(Bn.at(K.nrow - 1, j), hp::kTop, hp::kL2R));
  }
  hp::contract_last_row(c, K.cplx, bv, kv, brv, dev + 1, dev, final_E);
}
}  // namespace

namespace hp {
void norm_lattices(Ctx& c, const Lattice& ket, const Lattice& bra, const hpeps_esvd_opts& o, double* dev) {
  norm_run(c, ket, bra, o, dev, nullptr);
}
}  // namespace hp

extern "C" {

hpeps_status hpeps_boundary_contract_row(hpeps_ctx* ctx, const hpeps_bmps* bnd, const hpeps_peps* ket,
                                         const hpeps_peps* bra, int32_t row, hpeps_direction dir,
                                         const hpeps_esvd_opts* opts, hpeps_bmps* out,
                                         double* log_scale) {
  return guard_p(ctx, [&](hp::Ctx& c) {
    check_opts_p(opts);
    HP_REQUIRE(bnd && out && log_scale && out->tensors && out->shapes && out->capacity,
               HPEPS_ERR_INVALID_ARG, "null argument");
    HP_REQUIRE(dir == HPEPS_L2R || dir == HPEPS_R2L, HPEPS_ERR_INVALID_ARG, "bad direction");
    hp::Lattice K = hp::lattice_from_abi(ket);
    hp::Lattice B = bra ? hp::lattice_from_abi(bra) : K;
    HP_REQUIRE(row >= 0 && row < K.nrow && B.nrow == K.nrow && B.ncol == K.ncol, HPEPS_ERR_INVALID_ARG,
               "bad row index");
    HP_REQUIRE(B.cplx == K.cplx, HPEPS_ERR_DTYPE, "bra and ket dtypes differ");
    const int n = K.ncol;
    HP_REQUIRE(bnd->ncol == n && out->ncol == n, HPEPS_ERR_SHAPE, "boundary length differs from the row");
    HP_REQUIRE(bnd->dtype == ket->dtype && out->dtype == ket->dtype, HPEPS_ERR_DTYPE, "dtype mismatch");
    const hp::Dir d = dir == HPEPS_L2R ? hp::kL2R : hp::kR2L;
    std::vector<hp::BndView> bv;
    std::vector<hp::SiteView> kv, brv;
    std::vector<uint64_t> sids;
    for (int q = 0; q < n; ++q) {
      const int col = d == hp::kL2R ? q : n - 1 - q;
      hp::DevTensor t;
      t.p = bnd->tensors[col];
      t.dims.assign(bnd->shapes + 4 * col, bnd->shapes + 4 * col + 4);
      bv.push_back(hp::orient_bnd(t, d));
      kv.push_back(hp::orient_site(K.at(row, col), hp::kTop, d));
      brv.push_back(hp::orient_site(B.at(row, col), hp::kTop, d));
      sids.push_back(opts->stream_id + col);
    }
    const auto shapes = hp::absorb_shapes(bv, kv, opts->rank, opts->oversample);
    std::vector<hp::DevTensor> res(n);
    for (int q = 0; q < n; ++q) {
      const int col = d == hp::kL2R ? q : n - 1 - q;
      int64_t sz = 1;
      for (auto v : shapes[q]) sz *= v;
      HP_REQUIRE(out->tensors[col] && out->capacity[col] >= sz, HPEPS_ERR_SHAPE,
                 "output buffer too small for column " + std::to_string(col));
      res[q].p = out->tensors[col];
    }
    double* log_dev = c.ws<double>(1);
    hp::fill_value(c, log_dev, 1, 0.0, false);
    hp::absorb_row(c, K.cplx, bv, kv, brv, d, *opts, sids, res, log_dev);
    for (int q = 0; q < n; ++q) {
      const int col = d == hp::kL2R ? q : n - 1 - q;
      for (int e = 0; e < 4; ++e) out->shapes[4 * col + e] = res[q].dims[e];
    }
    double h = 0;
    HP_CHECK_HIP(hipMemcpyAsync(&h, log_dev, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    HP_CHECK_HIP(hipStreamSynchronize(c.stream));
    *log_scale += h;
  });
}

hpeps_status hpeps_peps_norm(hpeps_ctx* ctx, const hpeps_peps* ket, const hpeps_peps* bra,
                             const hpeps_esvd_opts* opts, double* log_norm, double* phase) {
  return guard_p(ctx, [&](hp::Ctx& c) {
    check_opts_p(opts);
    HP_REQUIRE(log_norm && phase, HPEPS_ERR_INVALID_ARG, "null output");
    hp::Lattice K = hp::lattice_from_abi(ket);
    hp::Lattice B = bra ? hp::lattice_from_abi(bra) : K;
    double* dev = c.ws<double>(4);  // log, result re/im
    norm_run(c, K, B, *opts, dev, nullptr);
    double h[3];
    HP_CHECK_HIP(hipMemcpyAsync(h, dev, sizeof(h), hipMemcpyDeviceToHost, c.stream));
    HP_CHECK_HIP(hipStreamSynchronize(c.stream));
    HP_REQUIRE(std::isfinite(h[0]) && std::isfinite(h[1]) && std::isfinite(h[2]), HPEPS_ERR_NUMERIC,
               "non-finite norm");
    *log_norm = h[0];
    phase[0] = h[1];
    phase[1] = h[2];
  });
}

hpeps_status hpeps_peps_norm_backward(hpeps_ctx* ctx, const hpeps_peps* ket, const hpeps_esvd_opts* opts,
                                      double broadening, void* const* grads, double* log_norm) {
  return guard_p(ctx, [&](hp::Ctx& c) {
    check_opts_p(opts);
    HP_REQUIRE(grads && log_norm, HPEPS_ERR_INVALID_ARG, "null argument");
    HP_REQUIRE(broadening >= 0.0, HPEPS_ERR_INVALID_ARG, "broadening must be >= 0");
    hp::Lattice K = hp::lattice_from_abi(ket);
    for (size_t q = 0; q < K.sites.size(); ++q) HP_REQUIRE(grads[q], HPEPS_ERR_INVALID_ARG, "null gradient pointer");
    double* dev = c.ws<double>(4);
    hp::Tape tape(K.cplx);
    for (auto& s : K.sites) tape.mark_input(s.p, s.size());
    double* E = nullptr;
    c.tape = &tape;
    norm_run(c, K, K, *opts, dev, &E);
    c.tape = nullptr;
    // d log|E| / dE (conjugate Wirtinger) = E / |E|^2 = E: the final mantissa
    // has unit modulus after its rescaling
    HP_CHECK_HIP(hipMemcpyAsync(tape.grad(c, E), E, (K.cplx ? 2 : 1) * sizeof(double), hipMemcpyDeviceToDevice,
                                c.stream));
    tape.backward(c, broadening);
    hp::write_site_grads(c, tape, K, grads);
    double h = 0;
    HP_CHECK_HIP(hipMemcpyAsync(&h, dev, sizeof(double), hipMemcpyDeviceToHost, c.stream));
    HP_CHECK_HIP(hipStreamSynchronize(c.stream));
    HP_REQUIRE(std::isfinite(h), HPEPS_ERR_NUMERIC, "non-finite norm");
    *log_norm = h;
  });
}

}  // extern "C"
