// Amplitudes <bits|psi> of a PEPS by the boundary-MPS contraction of a
// one-layer network (Sec. III: the amplitude network has one layer fewer
// than the <psi|psi> network of the IBMPS; Algs. 2-3 with Alg. 4).
// * Fixing every physical leg to its bit leaves the slices A[u,d,l,r] =
//   T[u,d,l,r,bit], gathered per basis state into [state, u, d, l, r].
// * Row 1 is the exact boundary ([l, d, r] per column, normalised).
// * Rows 2..n-1 are absorbed by the zip-up, left to right on the 1st, 3rd,
//   ... absorbed row and right to left on the others: the first column's
//   carry C[a,x,b,h] = sum_u S[a,u,b] A[u,x,1,h] is exact (normalised), every
//   later column is one randomized einsumsvd of the network
//   C[a,x,b,h] S[b,u,c] A[u,y,h,g] read as rows (a,x) x columns (y,c,g): the
//   isometric U [a,x,m'] is the finished boundary tensor and
//   (Sigma / sigma_1) V^* [m',y,c,g] the next carry.  A right-to-left sweep
//   reads every tensor through mirrored strides.
// * Row n is contracted exactly column by column.
// Every normalisation factor and sigma_1 enters a device-side log.
// Basis states share every shape, so a call takes a batch of them and runs
// the zip-ups in lockstep: every launch carries all states (the slices are
// gathered per state; the sketch of a column is shared, as its stream id is).
#include <cmath>
#include <initializer_list>
#include <string>
#include <vector>

#include "contract.h"
#include "esvd.h"
#include "peps.h"

namespace hp {
namespace {

// A batch of one-layer tensors: instance i at p + i * zs (elements), leg dims
// and strides in lattice orientation (boundary tensors [left, x, right],
// slices [u, d, l, r]).
template <int N>
struct View {
  const void* p = nullptr;
  int64_t n[N], s[N];
  int64_t zs = 0;
};
using Bnd = View<3>;
using Slc = View<4>;

// Sweep-frame legs: a boundary tensor as (a, x, b) = (behind, down, ahead),
// a slice as (u, y, h, g) = (up, down, behind, ahead).
Bnd orient(const Bnd& t, Dir dir) {
  if (dir == kL2R) return t;
  Bnd o = t;
  o.n[0] = t.n[2]; o.s[0] = t.s[2];
  o.n[2] = t.n[0]; o.s[2] = t.s[0];
  return o;
}
Slc orient(const Slc& t, Dir dir) {
  if (dir == kL2R) return t;
  Slc o = t;
  o.n[2] = t.n[3]; o.s[2] = t.s[3];
  o.n[3] = t.n[2]; o.s[3] = t.s[2];
  return o;
}

// The view with the state leg Z in front.
template <int N>
TView tvz(const View<N>& v, const char* legs, int nb, bool conj = false) {
  std::vector<int64_t> d{nb}, st{v.zs};
  for (int i = 0; i < N; ++i) {
    d.push_back(v.n[i]);
    st.push_back(v.s[i]);
  }
  return tview(v.p, std::string("Z") + legs, d, st, (int64_t)nb * v.zs, conj);
}
template <int N>
View<N> contiguous(void* p, std::initializer_list<int64_t> dims) {
  View<N> v;
  v.p = p;
  int i = 0;
  for (auto d : dims) v.n[i++] = d;
  int64_t st = 1;
  for (int q = N - 1; q >= 0; --q) {
    v.s[q] = st;
    st *= v.n[q];
  }
  v.zs = st;
  return v;
}

// Storage of one zip-up: the new boundary tensors go to `store` (slot j of
// lattice column j holds nb * cap_u elements), the carries alternate between
// carries[0] and carries[1] (nb * cap_c elements each); every other buffer
// of a column lives in a workspace scope, so the footprint does not grow
// with the lattice.
struct RowBuffers {
  double* store;
  int64_t cap_u;
  double* carries[2];
  int64_t cap_c;
};

// One zip-up (Alg. 3) of the slices `row` into the boundary `bnd` (both by
// lattice column), all states at once; out receives the new boundary.
void absorb_row(Ctx& ctx, bool cplx, int nb, const std::vector<Bnd>& bnd, const std::vector<Slc>& row, Dir dir,
                const hpeps_esvd_opts& o, int lattice_row, const RowBuffers& rb, std::vector<Bnd>& out,
                double* logs) {
  const int n = (int)row.size();
  const int es = cplx ? 2 : 1;
  auto col = [&](int q) { return dir == kL2R ? q : n - 1 - q; };
  auto slot = [&](int j) { return rb.store + (int64_t)j * nb * rb.cap_u * es; };
  // first column: exact carry [a, x, b, h] (a = h_left = 1)
  const Bnd S0 = orient(bnd[col(0)], dir);
  const Slc A0 = orient(row[col(0)], dir);
  HP_REQUIRE(S0.n[0] == 1 && A0.n[2] == 1, HPEPS_ERR_SHAPE, "open boundary legs must have dim 1");
  HP_REQUIRE(S0.n[1] == A0.n[0], HPEPS_ERR_SHAPE, "row and boundary legs do not chain");
  int64_t a = 1, x = A0.n[1], b = S0.n[2], h = A0.n[3];
  HP_REQUIRE(x * b * h <= (n == 1 ? rb.cap_u : rb.cap_c), HPEPS_ERR_SHAPE, "carry exceeds its buffer");
  // a one-column row has no einsumsvd: the exact carry is the boundary
  double* carry = n == 1 ? slot(0) : rb.carries[0];
  int cur = 0;
  contract2(ctx, cplx, tvz(S0, "auc", nb), tvz(A0, "uyhg", nb), "Zayhcg", carry, nb * x * b * h);
  normalize(ctx, cplx, carry, x * b * h, nb, logs);
  if (n == 1) {
    out[0] = contiguous<3>(carry, {1, x, b * h});
    return;
  }
  for (int q = 1; q < n; ++q) {
    WsScope scope(ctx);
    const Bnd S = orient(bnd[col(q)], dir);
    const Slc A = orient(row[col(q)], dir);
    HP_REQUIRE(S.n[0] == b && A.n[2] == h && S.n[1] == A.n[0], HPEPS_ERR_SHAPE, "row and boundary legs do not chain");
    const int64_t u = A.n[0], y = A.n[1], c = S.n[2], g = A.n[3];
    const int64_t rows = a * x, cols = y * c * g;
    const bool dense = o.method == HPEPS_ESVD_EXPLICIT;
    const int64_t k = dense ? std::min(rows, cols) : sketch_width(o.rank, o.oversample, rows, cols);
    const int64_t mp = std::min<int64_t>(o.rank, k);
    HP_REQUIRE(k >= 1 && k <= (cplx ? 88 : 128), HPEPS_ERR_SHAPE, "sketch width k out of range");
    HP_REQUIRE(rows * mp <= rb.cap_u && mp * cols <= (q + 1 < n ? rb.cap_c : rb.cap_u), HPEPS_ERR_SHAPE,
               "einsumsvd factors exceed their buffers");
    ctx.last_rank = mp;
    ctx.last_k = k;
    const View<4> Cv = contiguous<4>(carry, {a, x, b, h});
    const int64_t w1 = nb * u * h * c * k, w2 = nb * b * h * k;
    double* W1 = ctx.ws<double>(w1 * es);
    double* W2 = ctx.ws<double>(w2 * es);
    // A X: slice over (y, g), boundary tensor over (u, c), carry over (b, h);
    // X is the shared sketch (no state leg) or a panel [Z, y, c, g, k]
    auto fwd = [&](const double* X, bool per_state, double* Y) {
      const TView Xv = per_state ? tview_rm(X, "Zycgk", {nb, y, c, g, k}) : tview_rm(X, "ycgk", {y, c, g, k});
      contract2(ctx, cplx, tvz(A, "uyhg", nb), Xv, "Zuhck", W1, w1);
      contract2(ctx, cplx, tvz(S, "buc", nb), tview_rm(W1, "Zuhck", {nb, u, h, c, k}), "Zbhk", W2, w2);
      contract2(ctx, cplx, tvz(Cv, "axbh", nb), tview_rm(W2, "Zbhk", {nb, b, h, k}), "Zaxk", Y, nb * rows * k);
    };
    // A^* Y: the mirror stages on the conjugated operands
    auto adj = [&](const double* X, double* Y) {
      contract2(ctx, cplx, tvz(Cv, "axbh", nb, true), tview_rm(X, "Zaxk", {nb, a, x, k}), "Zbhk", W2, w2);
      contract2(ctx, cplx, tvz(S, "buc", nb, true), tview_rm(W2, "Zbhk", {nb, b, h, k}), "Zuchk", W1, w1);
      contract2(ctx, cplx, tvz(A, "uyhg", nb, true), tview_rm(W1, "Zuchk", {nb, u, c, h, k}), "Zycgk", Y,
                nb * cols * k);
    };
    ZipOut zo;
    zo.Urows.add(rows, mp);
    zo.Ucol.add(mp, 1);
    zo.Rrow.add(mp, cols);
    zo.Rcols.add(cols, 1);
    zo.nU = rows * mp;
    zo.nR = mp * cols;
    double* U = slot(col(q - 1));
    double* R = q + 1 < n ? rb.carries[1 - cur] : slot(col(q));
    if (dense) {
      // BMPS: the matrix of the network, A [Z,(a,x),(y,c,g)] or, when it is
      // wide, A^* [Z,(y,c,g),(a,x)] (every operand conjugated), then its
      // dense truncated SVD
      const bool wide = rows <= cols;
      double* Wt = ctx.ws<double>(nb * a * x * h * u * c * es);
      double* M = ctx.ws<double>(nb * rows * cols * es);
      contract2(ctx, cplx, tvz(Cv, "axbh", nb, wide), tvz(S, "buc", nb, wide), "Zaxhuc", Wt,
                nb * a * x * h * u * c);
      contract2(ctx, cplx, tview_rm(Wt, "Zaxhuc", {nb, a, x, h, u, c}), tvz(A, "uyhg", nb, wide),
                wide ? "Zycgax" : "Zaxycg", M, nb * rows * cols);
      dense_finish(ctx, cplx, rows, cols, mp, nb, o, HPEPS_ABSORB_CARRY, zo, U, nullptr, R, logs, M,
                   [&](bool, const double* P, double* Bs) {
                     contract2(ctx, cplx, tview_rm(M, "Zaxycg", {nb, a, x, y, c, g}, cplx),
                               tview_rm(P, "Zaxk", {nb, a, x, k}), "Zycgk", Bs, nb * cols * k);
                   });
    } else {
      double* Om = ctx.ws<double>(cols * k * es);
      sketch(ctx, Om, false, cols, k, 1, o.seed, 1 + ((uint64_t)lattice_row * n + col(q)), cplx);
      double* Y0 = ctx.ws<double>(nb * rows * k * es);
      fwd(Om, false, Y0);
      rsvd_finish(ctx, cplx, rows, cols, k, mp, nb, o, HPEPS_ABSORB_CARRY, zo, U, nullptr, R, logs, Y0,
                  [&](bool adjoint, const double* X, double* Y) {
                    if (adjoint)
                      adj(X, Y);
                    else
                      fwd(X, true, Y);
                  });
    }
    // U [a, x, mp] in the sweep frame: lattice [left, x, right]
    Bnd uv;
    uv.p = U;
    uv.zs = rows * mp;
    if (dir == kL2R) {
      uv.n[0] = a; uv.n[1] = x; uv.n[2] = mp;
      uv.s[0] = x * mp; uv.s[1] = mp; uv.s[2] = 1;
    } else {
      uv.n[0] = mp; uv.n[1] = x; uv.n[2] = a;
      uv.s[0] = 1; uv.s[1] = mp; uv.s[2] = x * mp;
    }
    out[col(q - 1)] = uv;
    if (q + 1 < n) {
      carry = R;
      cur = 1 - cur;
      a = mp; x = y; b = c; h = g;
    } else {
      // the last carry [mp, y, c*g = 1] is the last boundary tensor
      Bnd l;
      l.p = R;
      l.zs = mp * cols;
      if (dir == kL2R) {
        l.n[0] = mp; l.n[1] = y; l.n[2] = c * g;
        l.s[0] = y; l.s[1] = 1; l.s[2] = 1;
      } else {
        l.n[0] = c * g; l.n[1] = y; l.n[2] = mp;
        l.s[0] = 1; l.s[1] = 1; l.s[2] = y;
      }
      out[col(q)] = l;
    }
  }
}

// Exact contraction of the boundary with the last row (down legs 1): the
// unit-modulus mantissas (one per state) are returned, the logs go to logs.
double* last_row(Ctx& ctx, bool cplx, int nb, const std::vector<Bnd>& bnd, const std::vector<Slc>& row,
                 double* logs) {
  const int es = cplx ? 2 : 1;
  double* E = ctx.ws<double>(nb * es);
  fill_value(ctx, E, nb, 1.0, cplx);
  int64_t b = 1, h = 1;
  for (size_t j = 0; j < row.size(); ++j) {
    const Bnd& S = bnd[j];
    const Slc& A = row[j];
    HP_REQUIRE(A.n[1] == 1, HPEPS_ERR_SHAPE, "last-row sites must have down legs of dim 1");
    HP_REQUIRE(S.n[0] == b && A.n[2] == h && S.n[1] == A.n[0], HPEPS_ERR_SHAPE, "row and boundary legs do not chain");
    const int64_t u = S.n[1], c = S.n[2], g = A.n[3];
    const View<2> Ev = contiguous<2>(E, {b, h});
    double* X1 = ctx.ws<double>(nb * h * u * c * es);
    contract2(ctx, cplx, tvz(Ev, "bh", nb), tvz(S, "buc", nb), "Zhuc", X1, nb * h * u * c);
    double* En = ctx.ws<double>(nb * c * g * es);
    contract2(ctx, cplx, tview_rm(X1, "Zhuc", {nb, h, u, c}), tvz(A, "udhg", nb), "Zcdg", En, nb * c * g);
    normalize(ctx, cplx, En, c * g, nb, logs);
    E = En;
    b = c;
    h = g;
  }
  return E;
}

// out[t, e] = T[e * P + bit_t] (es doubles per element) for state t (one
// block per state); flags[t * nsites + site] = the slice has a nonzero.
__global__ void gather_slices_kernel(const double* T, long long vol, int P, const int* bits, int nsites, int site,
                                     int es, double* out, int* flags) {
  const int t = blockIdx.x;
  const int bit = bits[(long long)t * nsites + site];
  double* o = out + (long long)t * vol * es;
  int any = 0;
  for (long long e = threadIdx.x; e < vol; e += blockDim.x)
    for (int q = 0; q < es; ++q) {
      const double v = T[(e * P + bit) * es + q];
      o[e * es + q] = v;
      any |= v != 0.0;
    }
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) flags[(long long)t * nsites + site] = any;
}

template <class F>
hpeps_status guard_a(hpeps_ctx* ctx, F&& f) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  try {
    ctx->impl->ws_reset();
    f(*ctx->impl);
    return HPEPS_OK;
  } catch (const Error& e) {
    ctx->impl->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->impl->last_error = "host allocation failed";
    return HPEPS_ERR_ALLOC;
  } catch (...) {
    ctx->impl->last_error = "unknown error";
    return HPEPS_ERR_INVALID_ARG;
  }
}

void amplitudes(Ctx& c, const hpeps_peps* ket, int64_t n_states, const int32_t* bits, const hpeps_esvd_opts* opts,
                double* log_abs, double* phase) {
  HP_REQUIRE(opts && bits && log_abs && phase, HPEPS_ERR_INVALID_ARG, "null argument");
  HP_REQUIRE(n_states >= 1 && n_states <= 65535, HPEPS_ERR_INVALID_ARG, "n_states must be in 1..65535");
  HP_REQUIRE(opts->rank >= 1 && opts->oversample >= 0 && opts->power_iters >= 0 && opts->jacobi_max_sweeps >= 0,
             HPEPS_ERR_INVALID_ARG, "bad einsumsvd options");
  HP_REQUIRE(opts->sketch_precision == HPEPS_F64, HPEPS_ERR_DTYPE, "amplitudes run in FP64 / complex128");
  HP_REQUIRE(opts->method == HPEPS_ESVD_IMPLICIT || opts->method == HPEPS_ESVD_EXPLICIT, HPEPS_ERR_INVALID_ARG,
             "unknown einsumsvd method");
  const Lattice K = lattice_from_abi(ket);
  const bool cplx = K.cplx;
  const int es = cplx ? 2 : 1;
  const int nrow = K.nrow, ncol = K.ncol, nsites = nrow * ncol;
  const int nb = (int)n_states;
  for (int64_t t = 0; t < n_states; ++t)
    for (int q = 0; q < nsites; ++q) {
      const int32_t bit = bits[t * nsites + q];
      HP_REQUIRE(bit >= 0 && bit < K.sites[q].dims[4], HPEPS_ERR_INVALID_ARG,
                 "bit out of range of the physical dimension");
    }
  int* dbits = c.ws<int>(n_states * nsites);
  int* flags = c.ws<int>(n_states * nsites);
  HP_CHECK_HIP(hipMemcpyAsync(dbits, bits, (size_t)n_states * nsites * sizeof(int32_t), hipMemcpyHostToDevice,
                              c.stream));
  // slices gathered per state: [Z, u, d, l, r]
  std::vector<std::vector<Slc>> layer(nrow, std::vector<Slc>(ncol));
  for (int i = 0; i < nrow; ++i)
    for (int j = 0; j < ncol; ++j) {
      const DevTensor& T = K.at(i, j);
      const int P = (int)T.dims[4];
      const int64_t vol = T.size() / P;
      double* g = c.ws<double>(n_states * vol * es);
      gather_slices_kernel<<<nb, 256, 0, c.stream>>>((const double*)T.p, vol, P, dbits, nsites, i * ncol + j, es,
                                                     g, flags);
      HP_CHECK_HIP(hipGetLastError());
      layer[i][j] = contiguous<4>(g, {T.dims[0], T.dims[1], T.dims[2], T.dims[3]});
    }
  double* logs = c.ws<double>(n_states);
  fill_value(c, logs, n_states, 0.0, false);
  // zip-up storage: boundary tensors [left, x, right] of at most M x Dm x M
  // elements and carries [a, x, b, h] of at most M x Dm x M x Dm, with Dm
  // the largest site dimension and M = max(rank, Dm) (the first boundary's
  // bonds are site bonds); two boundary rows and two carries are live at once
  int64_t Dm = 1;
  for (const auto& t : K.sites)
    for (int q = 0; q < 4; ++q) Dm = std::max<int64_t>(Dm, t.dims[q]);
  const int64_t M = std::max<int64_t>(opts->rank, Dm);
  RowBuffers rbuf[2];
  for (auto& r : rbuf) {
    r.cap_u = M * Dm * M;
    r.cap_c = M * Dm * M * Dm;
    r.store = nrow > 2 ? c.ws<double>((int64_t)ncol * n_states * r.cap_u * es) : nullptr;
  }
  if (nrow > 2) {
    rbuf[0].carries[0] = rbuf[1].carries[0] = c.ws<double>(n_states * rbuf[0].cap_c * es);
    rbuf[0].carries[1] = rbuf[1].carries[1] = c.ws<double>(n_states * rbuf[0].cap_c * es);
  }
  std::vector<Bnd> bnd(ncol);
  if (nrow == 1) {
    double* one = c.ws<double>(n_states * es);
    fill_value(c, one, n_states, 1.0, cplx);
    for (int j = 0; j < ncol; ++j) bnd[j] = contiguous<3>(one, {1, 1, 1});
  } else {
    // row 1: each slice [1, d, l, r] read as [l, d, r], normalised in place
    for (int j = 0; j < ncol; ++j) {
      const Slc& A = layer[0][j];
      HP_REQUIRE(A.n[0] == 1, HPEPS_ERR_SHAPE, "top legs must have dim 1");
      normalize(c, cplx, const_cast<void*>(A.p), A.zs, nb, logs);
      Bnd v;
      v.p = A.p;
      v.zs = A.zs;
      v.n[0] = A.n[2]; v.s[0] = A.s[2];
      v.n[1] = A.n[1]; v.s[1] = A.s[1];
      v.n[2] = A.n[3]; v.s[2] = A.s[3];
      bnd[j] = v;
    }
    for (int t = 1; t < nrow - 1; ++t) {
      std::vector<Bnd> nbnd(ncol);
      absorb_row(c, cplx, nb, bnd, layer[t], t % 2 == 1 ? kL2R : kR2L, *opts, t, rbuf[t % 2], nbnd, logs);
      bnd = nbnd;
    }
  }
  const double* E = last_row(c, cplx, nb, bnd, layer[nrow - 1], logs);
  std::vector<double> hl(n_states), he(n_states * es);
  std::vector<int> hf(n_states * nsites);
  HP_CHECK_HIP(hipMemcpyAsync(hl.data(), logs, hl.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  HP_CHECK_HIP(hipMemcpyAsync(he.data(), E, he.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  HP_CHECK_HIP(hipMemcpyAsync(hf.data(), flags, hf.size() * sizeof(int), hipMemcpyDeviceToHost, c.stream));
  HP_CHECK_HIP(hipStreamSynchronize(c.stream));
  for (int64_t t = 0; t < n_states; ++t) {
    bool zero = false;
    for (int q = 0; q < nsites; ++q) zero = zero || !hf[t * nsites + q];
    if (zero) {
      // an exactly zero slice makes the amplitude exactly zero
      log_abs[t] = -INFINITY;
      phase[2 * t] = phase[2 * t + 1] = 0.0;
      continue;
    }
    const double re = he[t * es], im = cplx ? he[t * es + 1] : 0.0;
    HP_REQUIRE(std::isfinite(hl[t]) && std::isfinite(re) && std::isfinite(im), HPEPS_ERR_NUMERIC,
               "non-finite amplitude");
    log_abs[t] = hl[t];
    phase[2 * t] = re;
    phase[2 * t + 1] = im;
  }
}

}  // namespace
}  // namespace hp

extern "C" hpeps_status hpeps_peps_amplitudes(hpeps_ctx* ctx, const hpeps_peps* ket, int64_t n_states,
                                              const int32_t* bits, const hpeps_esvd_opts* opts, double* log_abs,
                                              double* phase) {
  return hp::guard_a(ctx, [&](hp::Ctx& c) { hp::amplitudes(c, ket, n_states, bits, opts, log_abs, phase); });
}

extern "C" hpeps_status hpeps_peps_amplitude(hpeps_ctx* ctx, const hpeps_peps* ket, const int32_t* bits,
                                             const hpeps_esvd_opts* opts, double* log_abs, double* phase) {
  return hp::guard_a(ctx, [&](hp::Ctx& c) { hp::amplitudes(c, ket, 1, bits, opts, log_abs, phase); });
}
