// Kernel-level entry points for the unit parity tests (include/hpeps_testing.h).
#include "../../include/hpeps_testing.h"
#include "esvd.h"

namespace {
template <class F>
hpeps_status guard_t(hpeps_ctx* ctx, F&& f) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  try {
    ctx->impl->ws_reset();
    f(*ctx->impl);
    return HPEPS_OK;
  } catch (const hp::Error& e) {
    ctx->impl->last_error = e.msg;
    return e.code;
  } catch (...) {
    ctx->impl->last_error = "unknown error";
    return HPEPS_ERR_INVALID_ARG;
  }
}
bool cplx_of(hpeps_dtype t) {
  HP_REQUIRE(t == HPEPS_F64 || t == HPEPS_C128, HPEPS_ERR_DTYPE, "dtype must be F64 or C128");
  return t == HPEPS_C128;
}
}  // namespace

extern "C" {

hpeps_status hpeps_test_gemm(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t batch, int64_t M, int64_t N,
                             int64_t K, int32_t trans_a, const void* A, const void* B, void* C) {
  return guard_t(ctx, [&](hp::Ctx& c) {
    const bool cplx = cplx_of(dtype);
    HP_REQUIRE(A && B && C && batch >= 1 && M >= 1 && N >= 1 && K >= 1, HPEPS_ERR_INVALID_ARG,
               "bad gemm arguments");
    hp::GemmDesc d;
    d.M = M; d.N = N; d.K = K;
    if (trans_a) {
      d.Am.add(M, 1);
      d.Ak.add(K, M);
    } else {
      d.Am.add(M, K);
      d.Ak.add(K, 1);
    }
    d.Bk.add(K, N);
    d.Bn.add(N, 1);
    d.Cm.add(M, N);
    d.Cn.add(N, 1);
    hp::GemmCall g;
    g.A = A; g.B = B; g.C = C;
    g.sA = M * K; g.sB = K * N; g.sC = M * N;
    g.batch = (int)batch;
    g.conjA = cplx && trans_a;
    hp::gemm(c, cplx ? hp::Prec::C128 : hp::Prec::F64, d, g);
  });
}

hpeps_status hpeps_test_orthogonalize(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t batch, int64_t n,
                                      int64_t k, void* Y, void* P) {
  return guard_t(ctx, [&](hp::Ctx& c) {
    const bool cplx = cplx_of(dtype);
    HP_REQUIRE(Y && P && batch >= 1 && n >= k && k >= 1 && k <= 128, HPEPS_ERR_INVALID_ARG,
               "bad orthogonalize arguments");
    const int es = cplx ? 2 : 1;
    hp::OrthWork w;
    w.G = c.ws<double>(batch * k * k * es);
    w.Rinv = c.ws<double>(batch * k * k * es);
    w.Racc = c.ws<double>(batch * k * k * es);
    w.flags = c.ws<int>(batch);
    hp::orthogonalize(c, cplx, (double*)Y, (double*)P, n, k, (int)batch, w);
  });
}

hpeps_status hpeps_test_orthogonalize_eigh(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t batch, int64_t n,
                                           int64_t k, const void* Y, void* P, void* R) {
  return guard_t(ctx, [&](hp::Ctx& c) {
    const bool cplx = cplx_of(dtype);
    HP_REQUIRE(Y && P && R && batch >= 1 && n >= k && k >= 1 && k <= 128, HPEPS_ERR_INVALID_ARG,
               "bad orthogonalize arguments");
    const int es = cplx ? 2 : 1;
    hp::OrthWork w;
    w.G = c.ws<double>(batch * k * k * es);
    w.Rinv = c.ws<double>(batch * k * k * es);
    w.Racc = (double*)R;
    w.flags = c.ws<int>(batch);
    w.mode = HPEPS_ORTH_EIGH;
    double* S1 = c.ws<double>(batch * n * k * es);
    hp::cholqr_r(c, cplx, (const double*)Y, S1, (double*)P, n, k, (int)batch, w);
  });
}

hpeps_status hpeps_test_householder(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t batch, int64_t n, int64_t k,
                                    const void* Y, void* P, void* R) {
  return guard_t(ctx, [&](hp::Ctx& c) {
    const bool cplx = cplx_of(dtype);
    HP_REQUIRE(Y && (P || R) && batch >= 1 && n >= k && k >= 1 && k <= 128, HPEPS_ERR_INVALID_ARG,
               "bad Householder arguments");
    hp::householder_qr(c, cplx, (const double*)Y, n, k, (int)batch, nullptr, 0, (double*)P, (double*)R);
  });
}

hpeps_status hpeps_test_strip_chunk_bytes(hpeps_ctx* ctx, int64_t bytes) {
  if (!ctx || bytes < 1) return HPEPS_ERR_INVALID_ARG;
  ctx->impl->strip_chunk_bytes = bytes;
  return HPEPS_OK;
}

hpeps_status hpeps_test_checkpoint_rows(hpeps_ctx* ctx, int32_t on) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  ctx->impl->checkpoint_rows = on != 0;
  return HPEPS_OK;
}

hpeps_status hpeps_test_small_svd(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t batch, int64_t k,
                                  const void* R, void* Z, double* sigma) {
  return guard_t(ctx, [&](hp::Ctx& c) {
    const bool cplx = cplx_of(dtype);
    HP_REQUIRE(R && Z && sigma && batch >= 1 && k >= 1, HPEPS_ERR_INVALID_ARG, "bad svd arguments");
    double* isig = c.ws<double>(batch * k);
    double* isig1 = c.ws<double>(batch);
    int* sweeps = c.ws<int>(batch);
    hp::jacobi_svd(c, cplx, (const double*)R, k, (int)batch, 40, (double*)Z, sigma, isig, isig1,
                   nullptr, sweeps);
    hp::stats_reduce(c, nullptr, sweeps, (int)batch, c.stats_dev);
  });
}

hpeps_status hpeps_test_zip_apply(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t batch,
                                  const int64_t dims[9], const void* V, const void* S,
                                  const void* T, const void* Bra, int64_t k, int32_t adjoint,
                                  const void* X, void* Y) {
  return guard_t(ctx, [&](hp::Ctx& c) {
    const bool cplx = cplx_of(dtype);
    HP_REQUIRE(dims && V && S && T && X && Y && k >= 1, HPEPS_ERR_INVALID_ARG, "bad apply arguments");
    hp::ZipDims z;
    z.a = dims[0]; z.x = dims[1]; z.b = dims[2]; z.h = dims[3]; z.u = dims[4];
    z.c = dims[5]; z.y = dims[6]; z.g = dims[7]; z.d = dims[8];
    const int es = cplx ? 2 : 1;
    hp::ZipWork w;
    w.W1 = c.ws<double>(batch * z.u * z.h * z.d * z.y * z.c * z.g * k * es);
    w.W2 = c.ws<double>(batch * hp::zip_w2_elems(z, k) * es);
    w.W3 = c.ws<double>(batch * z.b * z.h * z.h * k * es);
    hp::ZipOperands op{V, S, T, Bra ? Bra : T};
    hp::zip_apply(c, cplx ? hp::Prec::C128 : hp::Prec::F64, z, hp::ZipLayout::row_major(z), op,
                  (int)batch, k, adjoint != 0, X, Y, true, w);
  });
}

hpeps_status hpeps_test_zip_order(hpeps_ctx* ctx, int32_t order) {
  if (!ctx || order < 0 || order > 2) return HPEPS_ERR_INVALID_ARG;
  ctx->impl->zip_order_force = order;
  return HPEPS_OK;
}

hpeps_status hpeps_test_gemm_smallk(hpeps_ctx* ctx, int32_t on) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  ctx->impl->smallk = on != 0;
  return HPEPS_OK;
}

hpeps_status hpeps_test_gemm_variant(hpeps_ctx* ctx, int32_t tile, int32_t kstep, int32_t split) {
  if (!ctx || split < 0) return HPEPS_ERR_INVALID_ARG;
  ctx->impl->gemm_force = hp::GemmVariant{tile < 0 ? -1 : tile, kstep, split};
  return HPEPS_OK;
}

}  // extern "C"
