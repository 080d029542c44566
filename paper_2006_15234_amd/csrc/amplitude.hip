// Amplitudes <bits|psi> of a PEPS by the boundary-MPS contraction of a
// one-layer network (Sec. III: the amplitude network has one layer fewer
// than the <psi|psi> network of the IBMPS; Algs. 2-3 with Alg. 4).
// * Fixing every physical leg to its bit leaves the slices A[u,d,l,r] =
//   T[u,d,l,r,bit]: strided views of the sites, nothing is copied.
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
#include <cmath>
#include <initializer_list>
#include <string>
#include <vector>

#include "contract.h"
#include "esvd.h"
#include "peps.h"

namespace hp {
namespace {

// A one-layer tensor: leg dims and element strides in lattice orientation
// (boundary tensors [left, x, right]; slices [u, d, l, r]).
template <int N>
struct View {
  const void* p = nullptr;
  int64_t n[N], s[N];
  int64_t extent = 0;
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

template <int N>
TView tv(const View<N>& v, const char* legs) {
  return tview(v.p, legs, std::vector<int64_t>(v.n, v.n + N), std::vector<int64_t>(v.s, v.s + N), v.extent);
}
template <int N>
hpeps_tensor ht(const View<N>& v) {
  hpeps_tensor t{};
  t.data = v.p;
  t.ndim = N;
  for (int i = 0; i < N; ++i) {
    t.shape[i] = v.n[i];
    t.strides[i] = v.s[i];
  }
  return t;
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
  v.extent = st;
  return v;
}

constexpr const char* kZip1 = "axbh,buc,uyhg->ax|ycg";

// One zip-up (Alg. 3) of the slices `row` into the boundary `bnd` (both by
// lattice column); out receives the new boundary by lattice column.
void absorb_row1(Ctx& ctx, bool cplx, const std::vector<Bnd>& bnd, const std::vector<Slc>& row, Dir dir,
                 const hpeps_esvd_opts& o, int lattice_row, std::vector<Bnd>& out, double* log_dev) {
  const int n = (int)row.size();
  const int es = cplx ? 2 : 1;
  auto col = [&](int q) { return dir == kL2R ? q : n - 1 - q; };
  // first column: exact carry [a, x, b, h] (a = h_left = 1)
  const Bnd S0 = orient(bnd[col(0)], dir);
  const Slc A0 = orient(row[col(0)], dir);
  HP_REQUIRE(S0.n[0] == 1 && A0.n[2] == 1, HPEPS_ERR_SHAPE, "open boundary legs must have dim 1");
  int64_t a = 1, x = A0.n[1], b = S0.n[2], h = A0.n[3];
  double* carry = ctx.ws<double>(x * b * h * es);
  contract2(ctx, cplx, tv(S0, "auc"), tv(A0, "uyhg"), "ayhcg", carry, x * b * h);
  normalize(ctx, cplx, carry, x * b * h, 1, log_dev);
  if (n == 1) {
    out[0] = contiguous<3>(carry, {1, x, b * h});
    return;
  }
  for (int q = 1; q < n; ++q) {
    const Bnd S = orient(bnd[col(q)], dir);
    const Slc A = orient(row[col(q)], dir);
    HP_REQUIRE(S.n[0] == b && A.n[2] == h && S.n[1] == A.n[0], HPEPS_ERR_SHAPE, "row and boundary legs do not chain");
    const int64_t y = A.n[1], c = S.n[2], g = A.n[3];
    View<4> Cview = contiguous<4>(carry, {a, x, b, h});
    const hpeps_tensor ops[3] = {ht(Cview), ht(S), ht(A)};
    hpeps_esvd_opts oq = o;
    oq.stream_id = 1 + ((uint64_t)lattice_row * n + col(q));
    int64_t rows = 0, cols = 0, mp = 0;
    einsumsvd_query(kZip1, 3, ops, oq, &rows, &cols, &mp);
    double* U = ctx.ws<double>(rows * mp * es);
    double* R = ctx.ws<double>(mp * cols * es);
    einsumsvd_network(ctx, cplx, kZip1, 3, ops, oq, HPEPS_ABSORB_CARRY, U, nullptr, R, log_dev);
    // U [a, x, mp] in the sweep frame: lattice [left, x, right]
    Bnd u;
    u.p = U;
    u.extent = rows * mp;
    if (dir == kL2R) {
      u.n[0] = a; u.n[1] = x; u.n[2] = mp;
      u.s[0] = x * mp; u.s[1] = mp; u.s[2] = 1;
    } else {
      u.n[0] = mp; u.n[1] = x; u.n[2] = a;
      u.s[0] = 1; u.s[1] = mp; u.s[2] = x * mp;
    }
    out[col(q - 1)] = u;
    if (q + 1 < n) {
      carry = R;
      a = mp; x = y; b = c; h = g;
    } else {
      // the last carry [mp, y, c*g = 1] is the last boundary tensor
      Bnd l;
      l.p = R;
      l.extent = mp * y;
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
// unit-modulus mantissa goes to result_dev, the logs to log_dev.
void last_row1(Ctx& ctx, bool cplx, const std::vector<Bnd>& bnd, const std::vector<Slc>& row, double* result_dev,
               double* log_dev) {
  const int es = cplx ? 2 : 1;
  double* E = ctx.ws<double>(es);
  fill_value(ctx, E, 1, 1.0, cplx);
  int64_t b = 1, h = 1;
  for (size_t j = 0; j < row.size(); ++j) {
    const Bnd& S = bnd[j];
    const Slc& A = row[j];
    HP_REQUIRE(A.n[1] == 1, HPEPS_ERR_SHAPE, "last-row sites must have down legs of dim 1");
    HP_REQUIRE(S.n[0] == b && A.n[2] == h && S.n[1] == A.n[0], HPEPS_ERR_SHAPE, "row and boundary legs do not chain");
    const int64_t u = S.n[1], c = S.n[2], g = A.n[3];
    View<2> Ev = contiguous<2>(E, {b, h});
    double* X1 = ctx.ws<double>(h * u * c * es);
    contract2(ctx, cplx, tv(Ev, "bh"), tv(S, "buc"), "huc", X1, h * u * c);
    View<3> Xv = contiguous<3>(X1, {h, u, c});
    double* En = ctx.ws<double>(c * g * es);
    contract2(ctx, cplx, tv(Xv, "huc"), tv(A, "udhg"), "cdg", En, c * g);
    normalize(ctx, cplx, En, c * g, 1, log_dev);
    E = En;
    b = c;
    h = g;
  }
  copy_scalar(ctx, E, cplx, result_dev);
}

// flags[q] = 1 when slice q has a nonzero element (element e of slice q at
// (e * P + bit) in the site's storage, es doubles per element).
struct SliceRef {
  const double* p;
  long long n;
  int P, bit;
};
__global__ void slice_nonzero_kernel(const SliceRef* refs, int es, int* flags) {
  const SliceRef r = refs[blockIdx.x];
  int any = 0;
  for (long long e = threadIdx.x; e < r.n; e += blockDim.x)
    for (int c = 0; c < es; ++c) any |= r.p[(e * r.P + r.bit) * es + c] != 0.0;
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) flags[blockIdx.x] = any;
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

}  // namespace
}  // namespace hp

extern "C" hpeps_status hpeps_peps_amplitude(hpeps_ctx* ctx, const hpeps_peps* ket, const int32_t* bits,
                                             const hpeps_esvd_opts* opts, double* log_abs, double* phase) {
  using namespace hp;
  return guard_a(ctx, [&](Ctx& c) {
    HP_REQUIRE(opts && bits && log_abs && phase, HPEPS_ERR_INVALID_ARG, "null argument");
    HP_REQUIRE(opts->rank >= 1 && opts->oversample >= 0 && opts->power_iters >= 0 && opts->jacobi_max_sweeps >= 0,
               HPEPS_ERR_INVALID_ARG, "bad einsumsvd options");
    HP_REQUIRE(opts->sketch_precision == HPEPS_F64, HPEPS_ERR_DTYPE, "amplitudes run in FP64 / complex128");
    const Lattice K = lattice_from_abi(ket);
    const bool cplx = K.cplx;
    const int es = cplx ? 2 : 1;
    const int nrow = K.nrow, ncol = K.ncol;
    // slices as strided views of the sites
    std::vector<std::vector<Slc>> layer(nrow, std::vector<Slc>(ncol));
    std::vector<SliceRef> refs;
    for (int i = 0; i < nrow; ++i)
      for (int j = 0; j < ncol; ++j) {
        const DevTensor& T = K.at(i, j);
        const int P = (int)T.dims[4], bit = bits[i * ncol + j];
        HP_REQUIRE(bit >= 0 && bit < P, HPEPS_ERR_INVALID_ARG, "bit out of range of the physical dimension");
        const auto st = rm_strides(T.dims);
        Slc& v = layer[i][j];
        v.p = (const double*)T.p + (int64_t)bit * es;
        for (int q = 0; q < 4; ++q) {
          v.n[q] = T.dims[q];
          v.s[q] = st[q];
        }
        v.extent = T.size() - bit;
        refs.push_back(SliceRef{(const double*)T.p, T.size() / P, P, bit});
      }
    // an exactly zero slice makes the amplitude exactly zero
    {
      SliceRef* d_refs = c.ws<SliceRef>((int64_t)refs.size());
      int* flags = c.ws<int>((int64_t)refs.size());
      HP_CHECK_HIP(hipMemcpyAsync(d_refs, refs.data(), refs.size() * sizeof(SliceRef), hipMemcpyHostToDevice,
                                  c.stream));
      slice_nonzero_kernel<<<(unsigned)refs.size(), 256, 0, c.stream>>>(d_refs, es, flags);
      HP_CHECK_HIP(hipGetLastError());
      std::vector<int> h(refs.size());
      HP_CHECK_HIP(hipMemcpyAsync(h.data(), flags, h.size() * sizeof(int), hipMemcpyDeviceToHost, c.stream));
      HP_CHECK_HIP(hipStreamSynchronize(c.stream));
      for (int f : h)
        if (!f) {
          *log_abs = -INFINITY;
          phase[0] = phase[1] = 0.0;
          return;
        }
    }
    double* dev = c.ws<double>(4);  // log, mantissa re/im
    fill_value(c, dev, 1, 0.0, false);
    std::vector<Bnd> bnd(ncol);
    if (nrow == 1) {
      double* one = c.ws<double>(es);
      fill_value(c, one, 1, 1.0, cplx);
      for (int j = 0; j < ncol; ++j) bnd[j] = contiguous<3>(one, {1, 1, 1});
    } else {
      // row 1: [l, d, r] copies of the slices (u = 1), normalised
      double* one = c.ws<double>(es);
      fill_value(c, one, 1, 1.0, cplx);
      const View<1> onev = contiguous<1>(one, {1});
      for (int j = 0; j < ncol; ++j) {
        const Slc& A = layer[0][j];
        HP_REQUIRE(A.n[0] == 1, HPEPS_ERR_SHAPE, "top legs must have dim 1");
        const int64_t l = A.n[2], d = A.n[1], r = A.n[3];
        double* B = c.ws<double>(l * d * r * es);
        contract2(c, cplx, tv(A, "udlr"), tv(onev, "u"), "ldr", B, l * d * r);
        normalize(c, cplx, B, l * d * r, 1, dev);
        bnd[j] = contiguous<3>(B, {l, d, r});
      }
      for (int t = 1; t < nrow - 1; ++t) {
        std::vector<Bnd> nb(ncol);
        absorb_row1(c, cplx, bnd, layer[t], t % 2 == 1 ? kL2R : kR2L, *opts, t, nb, dev);
        bnd = nb;
      }
    }
    last_row1(c, cplx, bnd, layer[nrow - 1], dev + 1, dev);
    double hres[3];
    HP_CHECK_HIP(hipMemcpyAsync(hres, dev, sizeof(hres), hipMemcpyDeviceToHost, c.stream));
    HP_CHECK_HIP(hipStreamSynchronize(c.stream));
    HP_REQUIRE(std::isfinite(hres[0]) && std::isfinite(hres[1]) && std::isfinite(hres[2]), HPEPS_ERR_NUMERIC,
               "non-finite amplitude");
    *log_abs = hres[0];
    phase[0] = hres[1];
    phase[1] = hres[2];
  });
}
