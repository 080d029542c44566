// extern "C" entry points of libhpeps (see include/hpeps.h).
#include <cstring>
#include <new>

#include "esvd.h"
#include "peps.h"

namespace {

template <class F>
hpeps_status guard(hpeps_ctx* ctx, F&& f) {
  try {
    f();
    return HPEPS_OK;
  } catch (const hp::Error& e) {
    if (ctx) ctx->impl->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->impl->last_error = "host allocation failed";
    return HPEPS_ERR_ALLOC;
  } catch (...) {
    if (ctx) ctx->impl->last_error = "unknown error";
    return HPEPS_ERR_INVALID_ARG;
  }
}

void check_opts(const hpeps_esvd_opts* o) {
  HP_REQUIRE(o, HPEPS_ERR_INVALID_ARG, "opts is NULL");
  HP_REQUIRE(o->rank >= 1, HPEPS_ERR_INVALID_ARG, "rank must be >= 1");
  HP_REQUIRE(o->oversample >= 0, HPEPS_ERR_INVALID_ARG, "oversample must be >= 0");
  HP_REQUIRE(o->power_iters >= 0, HPEPS_ERR_INVALID_ARG, "power_iters must be >= 0");
  HP_REQUIRE(o->jacobi_max_sweeps >= 0, HPEPS_ERR_INVALID_ARG, "jacobi_max_sweeps must be >= 0");
}

bool is_cplx(hpeps_dtype t) {
  HP_REQUIRE(t == HPEPS_F64 || t == HPEPS_C128, HPEPS_ERR_DTYPE, "tensors must be F64 or C128");
  return t == HPEPS_C128;
}

}  // namespace

extern "C" {

const char* hpeps_status_string(hpeps_status s) {
  switch (s) {
    case HPEPS_OK: return "ok";
    case HPEPS_ERR_INVALID_ARG: return "invalid argument";
    case HPEPS_ERR_SHAPE: return "shape mismatch";
    case HPEPS_ERR_DTYPE: return "unsupported dtype";
    case HPEPS_ERR_ALLOC: return "allocation failed";
    case HPEPS_ERR_HIP: return "HIP runtime error";
    case HPEPS_ERR_NUMERIC: return "non-finite values";
    case HPEPS_ERR_NOT_CONVERGED: return "not converged";
    case HPEPS_ERR_UNSUPPORTED: return "unsupported size";
  }
  return "unknown status";
}

hpeps_status hpeps_create(int device, hpeps_ctx** out) {
  if (!out) return HPEPS_ERR_INVALID_ARG;
  *out = nullptr;
  hpeps_ctx* c = new (std::nothrow) hpeps_ctx{nullptr};
  if (!c) return HPEPS_ERR_ALLOC;
  hpeps_status st = guard(nullptr, [&] { c->impl = new hp::Ctx(device); });
  if (st != HPEPS_OK) {
    delete c;
    return st;
  }
  *out = c;
  return HPEPS_OK;
}

hpeps_status hpeps_destroy(hpeps_ctx* ctx) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  delete ctx->impl;
  delete ctx;
  return HPEPS_OK;
}

hpeps_status hpeps_set_stream(hpeps_ctx* ctx, void* stream) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  ctx->impl->stream = (hipStream_t)stream;
  return HPEPS_OK;
}

const char* hpeps_last_error(hpeps_ctx* ctx) { return ctx ? ctx->impl->last_error.c_str() : ""; }

hpeps_status hpeps_set_workspace_limit(hpeps_ctx* ctx, int64_t bytes) {
  if (!ctx || bytes < 0) return HPEPS_ERR_INVALID_ARG;
  ctx->impl->ws_limit = bytes;
  return HPEPS_OK;
}

hpeps_status hpeps_workspace_peak(hpeps_ctx* ctx, int64_t* bytes, int32_t reset) {
  if (!ctx || !bytes) return HPEPS_ERR_INVALID_ARG;
  *bytes = ctx->impl->ws_peak;
  if (reset) ctx->impl->ws_peak = 0;
  return HPEPS_OK;
}

hpeps_status hpeps_get_info(hpeps_ctx* ctx, hpeps_esvd_info* info) {
  if (!ctx || !info) return HPEPS_ERR_INVALID_ARG;
  return guard(ctx, [&] {
    hp::Ctx& c = *ctx->impl;
    int h[8];
    HP_CHECK_HIP(hipMemcpyAsync(h, c.stats_dev, sizeof(h), hipMemcpyDeviceToHost, c.stream));
    HP_CHECK_HIP(hipStreamSynchronize(c.stream));
    HP_CHECK_HIP(hipMemsetAsync(c.stats_dev, 0, sizeof(h), c.stream));
    info->rank_kept = c.last_rank;
    info->sketch_width = c.last_k;
    info->orth_extra_passes = h[0];
    info->jacobi_sweeps = h[1];
    info->numeric_errors = h[2];
    info->not_converged = h[3];
    info->orth_householder = h[4];
    info->reserved = 0;
  });
}

hpeps_status hpeps_autotune_enable(hpeps_ctx* ctx, int32_t on) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  ctx->impl->autotune = on != 0;
  return HPEPS_OK;
}

hpeps_status hpeps_autotune_export(hpeps_ctx* ctx, char* buf, int64_t cap, int64_t* needed) {
  if (!ctx || !needed || (buf && cap <= 0)) return HPEPS_ERR_INVALID_ARG;
  return guard(ctx, [&] {
    const std::string s = hp::autotune_export(*ctx->impl);
    *needed = (int64_t)s.size() + 1;
    if (buf) {
      const int64_t n = std::min<int64_t>(cap - 1, (int64_t)s.size());
      memcpy(buf, s.data(), (size_t)n);
      buf[n] = '\0';
    }
  });
}

hpeps_status hpeps_autotune_import(hpeps_ctx* ctx, const char* json) {
  if (!ctx || !json) return HPEPS_ERR_INVALID_ARG;
  return guard(ctx, [&] { hp::autotune_import(*ctx->impl, json); });
}

hpeps_status hpeps_profile_start(hpeps_ctx* ctx, const char* filter) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  ctx->impl->prof_on = true;
  ctx->impl->prof_filter = filter ? filter : "";
  return HPEPS_OK;
}

hpeps_status hpeps_profile_by_shape(hpeps_ctx* ctx, int32_t on) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  ctx->impl->prof_shapes = on != 0;
  return HPEPS_OK;
}

hpeps_status hpeps_profile_stop(hpeps_ctx* ctx) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  ctx->impl->prof_on = false;
  return HPEPS_OK;
}

hpeps_status hpeps_profile_read(hpeps_ctx* ctx, int32_t max_entries, hpeps_profile_entry* out,
                                int32_t* n_out) {
  if (!ctx || !n_out || (max_entries > 0 && !out)) return HPEPS_ERR_INVALID_ARG;
  return guard(ctx, [&] {
    auto agg = ctx->impl->prof_read();
    int32_t n = 0;
    for (auto& a : agg) {
      if (a.launches == 0) continue;
      if (n < max_entries) {
        std::memset(out[n].name, 0, sizeof(out[n].name));
        std::strncpy(out[n].name, a.name.c_str(), sizeof(out[n].name) - 1);
        out[n].launches = a.launches;
        out[n].ms = a.ms;
        out[n].flops = a.flops;
        out[n].bytes = a.bytes;
      }
      ++n;
    }
    *n_out = n;
  });
}

hpeps_status hpeps_sketch(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t n, int64_t k, int64_t batch,
                          uint64_t seed, uint64_t stream_id, void* out) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  return guard(ctx, [&] {
    HP_REQUIRE(out && n >= 1 && k >= 1 && batch >= 1 && batch < 65536, HPEPS_ERR_INVALID_ARG,
               "bad sketch arguments");
    HP_REQUIRE(dtype == HPEPS_F64 || dtype == HPEPS_F32, HPEPS_ERR_DTYPE, "sketch dtype F64 or F32");
    hp::sketch(*ctx->impl, out, dtype == HPEPS_F32, n, k, (int)batch, seed, stream_id);
  });
}

hpeps_status hpeps_einsumsvd(hpeps_ctx* ctx, hpeps_dtype dtype, const char* subscripts, int32_t n_ops,
                             const hpeps_tensor* ops, const hpeps_esvd_opts* opts, hpeps_absorb absorb,
                             void* U, double* sigma, void* R, double* log_scale) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  return guard(ctx, [&] {
    check_opts(opts);
    const bool cplx = is_cplx(dtype);
    HP_REQUIRE(U && R, HPEPS_ERR_INVALID_ARG, "null output");
    HP_REQUIRE(absorb >= HPEPS_ABSORB_CARRY && absorb <= HPEPS_ABSORB_SQRT, HPEPS_ERR_INVALID_ARG,
               "bad absorb mode");
    HP_REQUIRE(absorb != HPEPS_ABSORB_CARRY || log_scale, HPEPS_ERR_INVALID_ARG,
               "the CARRY mode needs log_scale");
    hp::Ctx& c = *ctx->impl;
    c.ws_reset();
    hp::einsumsvd_network(c, cplx, subscripts, n_ops, ops, *opts, absorb, U, sigma, R, log_scale);
  });
}

hpeps_status hpeps_einsumsvd_batched(hpeps_ctx* ctx, hpeps_dtype dtype, int64_t batch, const char* subscripts,
                                     int32_t n_ops, const hpeps_tensor* ops, const hpeps_esvd_opts* opts,
                                     hpeps_absorb absorb, void* U, double* sigma, void* R, double* log_scale) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  return guard(ctx, [&] {
    check_opts(opts);
    const bool cplx = is_cplx(dtype);
    HP_REQUIRE(batch >= 1, HPEPS_ERR_INVALID_ARG, "batch must be >= 1");
    HP_REQUIRE(U && R, HPEPS_ERR_INVALID_ARG, "null output");
    HP_REQUIRE(absorb >= HPEPS_ABSORB_CARRY && absorb <= HPEPS_ABSORB_SQRT, HPEPS_ERR_INVALID_ARG,
               "bad absorb mode");
    HP_REQUIRE(absorb != HPEPS_ABSORB_CARRY || log_scale, HPEPS_ERR_INVALID_ARG,
               "the CARRY mode needs log_scale");
    hp::Ctx& c = *ctx->impl;
    c.ws_reset();
    hp::einsumsvd_network(c, cplx, subscripts, n_ops, ops, *opts, absorb, U, sigma, R, log_scale, batch);
  });
}

hpeps_status hpeps_einsumsvd_backward(hpeps_ctx* ctx, hpeps_dtype dtype, const char* subscripts, int32_t n_ops,
                                      const hpeps_tensor* ops, const hpeps_esvd_opts* opts, hpeps_absorb absorb,
                                      double broadening, const void* dU, const double* dsigma, const void* dR,
                                      void* const* grads) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  return guard(ctx, [&] {
    check_opts(opts);
    const bool cplx = is_cplx(dtype);
    HP_REQUIRE(absorb == HPEPS_ABSORB_NONE || absorb == HPEPS_ABSORB_RIGHT, HPEPS_ERR_UNSUPPORTED,
               "the adjoint supports the NONE and RIGHT absorb modes");
    hp::Ctx& c = *ctx->impl;
    c.ws_reset();
    hp::einsumsvd_network_backward(c, cplx, subscripts, n_ops, ops, *opts, absorb, broadening, dU, dsigma, dR,
                                   grads);
  });
}

hpeps_status hpeps_einsumsvd_query(hpeps_ctx* ctx, const char* subscripts, int32_t n_ops,
                                   const hpeps_tensor* ops, const hpeps_esvd_opts* opts, int64_t* rows,
                                   int64_t* cols, int64_t* rank_kept) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  return guard(ctx, [&] {
    check_opts(opts);
    hp::einsumsvd_query(subscripts, n_ops, ops, *opts, rows, cols, rank_kept);
  });
}

hpeps_status hpeps_einsumsvd_zipup(hpeps_ctx* ctx, int64_t batch, hpeps_dtype dtype,
                                   const int64_t dims[9], const void* V, const void* S,
                                   const void* T, const void* Bra, const hpeps_esvd_opts* opts,
                                   hpeps_absorb absorb, void* U, double* sigma, void* R,
                                   double* log_scale) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  return guard(ctx, [&] {
    check_opts(opts);
    const bool cplx = is_cplx(dtype);
    HP_REQUIRE(dims && V && S && T && U && sigma && R, HPEPS_ERR_INVALID_ARG, "null argument");
    HP_REQUIRE(batch >= 1 && batch < 65536, HPEPS_ERR_INVALID_ARG, "batch out of range");
    HP_REQUIRE(absorb >= HPEPS_ABSORB_CARRY && absorb <= HPEPS_ABSORB_SQRT, HPEPS_ERR_INVALID_ARG,
               "bad absorb mode");
    for (int i = 0; i < 9; ++i) HP_REQUIRE(dims[i] >= 1, HPEPS_ERR_SHAPE, "dims must be >= 1");
    hp::ZipDims z;
    z.a = dims[0]; z.x = dims[1]; z.b = dims[2]; z.h = dims[3]; z.u = dims[4];
    z.c = dims[5]; z.y = dims[6]; z.g = dims[7]; z.d = dims[8];
    hp::ZipOperands op{V, S, T, Bra ? Bra : T};
    hp::Ctx& c = *ctx->impl;
    c.ws_reset();
    const int64_t k = hp::sketch_width(opts->rank, opts->oversample, z.rows(), z.cols());
    hp::zip_esvd(c, cplx, z, hp::ZipLayout::row_major(z), op, (int)batch, *opts, absorb,
                 hp::ZipOut::row_major(z, std::min<int64_t>(opts->rank, k)), U, sigma, R, log_scale);
  });
}

hpeps_status hpeps_einsumsvd_pair(hpeps_ctx* ctx, int64_t batch, hpeps_dtype dtype,
                                  const int64_t dims[3], const void* Bl, const void* Br,
                                  const void* T1, const void* T2, const hpeps_esvd_opts* opts,
                                  hpeps_absorb absorb, void* U, double* sigma, void* R) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  return guard(ctx, [&] {
    check_opts(opts);
    const bool cplx = is_cplx(dtype);
    HP_REQUIRE(dims && Bl && Br && T1 && T2 && U && sigma && R, HPEPS_ERR_INVALID_ARG, "null argument");
    HP_REQUIRE(batch >= 1 && batch < 65536, HPEPS_ERR_INVALID_ARG, "batch out of range");
    HP_REQUIRE(absorb >= HPEPS_ABSORB_CARRY && absorb <= HPEPS_ABSORB_SQRT, HPEPS_ERR_INVALID_ARG,
               "bad absorb mode");
    const int64_t m = dims[0], D = dims[1], d = dims[2];
    HP_REQUIRE(m >= 1 && D >= 1 && d >= 1, HPEPS_ERR_SHAPE, "dims must be >= 1");
    hp::Ctx& c = *ctx->impl;
    c.ws_reset();
    const int es = cplx ? 2 : 1;
    // exact carry over the left column: V[a,x,X,b,h,H]
    hp::CarryDims cd;
    cd.a = m; cd.u = D; cd.b = m; cd.x = D; cd.h = D; cd.d = d;
    double* V = c.ws<double>(batch * m * D * D * m * D * D * es);
    hp::form_carry(c, cplx, cd, hp::CarryLayout::row_major(cd), Bl, T1, T1, V, (int)batch);
    hp::ZipDims z;
    z.a = m; z.x = D; z.b = m; z.h = D; z.u = D; z.c = m; z.y = D; z.g = 1; z.d = d;
    hp::ZipOperands op{V, Br, T2, T2};
    const int64_t k = hp::sketch_width(opts->rank, opts->oversample, z.rows(), z.cols());
    hp::zip_esvd(c, cplx, z, hp::ZipLayout::row_major(z), op, (int)batch, *opts, absorb,
                 hp::ZipOut::row_major(z, std::min<int64_t>(opts->rank, k)), U, sigma, R, nullptr);
  });
}

hpeps_status hpeps_einsumsvd_pair_backward(hpeps_ctx* ctx, int64_t batch, hpeps_dtype dtype,
                                           const int64_t dims[3], const void* Bl, const void* Br,
                                           const void* T1, const void* T2,
                                           const hpeps_esvd_opts* opts, hpeps_absorb absorb,
                                           double broadening, const void* dU, const double* dsigma,
                                           const void* dR, void* gBl, void* gBr, void* gT1,
                                           void* gT2) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  return guard(ctx, [&] {
    check_opts(opts);
    const bool cplx = is_cplx(dtype);
    HP_REQUIRE(dims && Bl && Br && T1 && T2 && dU && dR && gBl && gBr && gT1 && gT2,
               HPEPS_ERR_INVALID_ARG, "null argument");
    HP_REQUIRE(batch >= 1 && batch < 65536, HPEPS_ERR_INVALID_ARG, "batch out of range");
    HP_REQUIRE(absorb == HPEPS_ABSORB_NONE || absorb == HPEPS_ABSORB_RIGHT, HPEPS_ERR_UNSUPPORTED,
               "the adjoint supports the NONE and RIGHT absorb modes");
    const int64_t m = dims[0], D = dims[1], d = dims[2];
    HP_REQUIRE(m >= 1 && D >= 1 && d >= 1, HPEPS_ERR_SHAPE, "dims must be >= 1");
    hp::Ctx& c = *ctx->impl;
    c.ws_reset();
    const int es = cplx ? 2 : 1;
    hp::CarryDims cd;
    cd.a = m; cd.u = D; cd.b = m; cd.x = D; cd.h = D; cd.d = d;
    const hp::CarryLayout cl = hp::CarryLayout::row_major(cd);
    const int64_t nV = m * D * D * m * D * D, nT = D * D * D * d;
    double* V = c.ws<double>(batch * nV * es);
    hp::form_carry(c, cplx, cd, cl, Bl, T1, T1, V, (int)batch);
    hp::ZipDims z;
    z.a = m; z.x = D; z.b = m; z.h = D; z.u = D; z.c = m; z.y = D; z.g = 1; z.d = d;
    hp::ZipOperands op{V, Br, T2, T2};
    double* gV = c.ws<double>(batch * nV * es);
    hp::fill_zero(c, gV, batch * nV * es * 8);
    const int64_t nB = m * D * D * m;
    hp::fill_zero(c, gBl, batch * nB * es * 8);
    hp::fill_zero(c, gBr, batch * nB * es * 8);
    hp::fill_zero(c, gT1, batch * nT * es * 8);
    hp::fill_zero(c, gT2, batch * nT * es * 8);
    const int64_t k = hp::sketch_width(opts->rank, opts->oversample, z.rows(), z.cols());
    // T2 serves as ket and bra: both gradients accumulate into gT2 (same for T1)
    hp::zip_esvd_backward(c, cplx, z, hp::ZipLayout::row_major(z), op, (int)batch, *opts, absorb,
                          broadening, hp::ZipOut::row_major(z, std::min<int64_t>(opts->rank, k)), dU,
                          dsigma, dR, gV, gBr, gT2, gT2);
    hp::carry_backward(c, cplx, cd, cl, Bl, T1, T1, gV, gBl, gT1, gT1, (int)batch);
  });
}

}  // extern "C"
