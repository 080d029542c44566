// Host-side AddressSanitizer / UndefinedBehaviorSanitizer run of the C ABI.
// Built by build.sh with the library's host code instrumented (device code is
// not: -fsanitize only after -Xarch_host).  It first checks host <-> device
// copies and the stages of the randomized SVD against host arithmetic, then
// walks the entry points a user reaches first -- context, subscript parsing
// with malformed input, an einsumsvd of a small network, its batched form
// and its adjoint, the autotune JSON round trip with malformed input, a PEPS
// norm, an amplitude, an energy and the norm's gradient, an ITE plan in its
// three launch forms, the allocation-free gate update and the profiler --
// and checks every status.  Exit status 0 when every call returned what it
// should; a sanitizer report aborts with its own status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "hpeps.h"
#include "hpeps_testing.h"

static int g_fail = 0;
static void fail(int line, const char* what) {
  std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, line, what);
  ++g_fail;
}
#define CHECK(cond) \
  do {              \
    if (!(cond)) fail(__LINE__, #cond); \
  } while (0)
#define EXPECT(call, want)                                                                 \
  do {                                                                                     \
    const hpeps_status st_ = (call);                                                       \
    if (st_ != (want)) {                                                                   \
      std::fprintf(stderr, "%s:%d: %s returned %d (%s), expected %d\n", __FILE__, __LINE__, \
                   #call, (int)st_, hpeps_status_string(st_), (int)(want));                \
      ++g_fail;                                                                            \
    }                                                                                      \
  } while (0)

static double* dev_copy(const std::vector<double>& h) {
  double* d = nullptr;
  if (hipMalloc(&d, h.size() * sizeof(double)) != hipSuccess) std::abort();
  if (hipMemcpy(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) std::abort();
  return d;
}

static std::vector<double> randn(size_t n, std::mt19937_64& g) {
  std::normal_distribution<double> nd;
  std::vector<double> v(n);
  for (auto& x : v) x = nd(g);
  return v;
}

static hpeps_esvd_opts opts(int64_t rank) {
  hpeps_esvd_opts o;
  std::memset(&o, 0, sizeof(o));
  o.rank = rank;
  o.oversample = 4;
  o.power_iters = 1;
  o.sketch_precision = HPEPS_F64;
  o.seed = 1;
  o.stream_id = 1;
  return o;
}

// a random nrow x ncol PEPS of bond D (open edges of dimension 1), d = 2
struct Lattice {
  int nrow, ncol;
  std::vector<int64_t> shapes;
  std::vector<void*> sites;
  hpeps_peps view() const { return hpeps_peps{nrow, ncol, HPEPS_F64, 0, sites.data(), shapes.data()}; }
};

static Lattice make_lattice(int nrow, int ncol, int64_t D, std::mt19937_64& g) {
  Lattice L{nrow, ncol, {}, {}};
  for (int i = 0; i < nrow; ++i)
    for (int j = 0; j < ncol; ++j) {
      const int64_t sh[5] = {i > 0 ? D : 1, i < nrow - 1 ? D : 1, j > 0 ? D : 1, j < ncol - 1 ? D : 1, 2};
      size_t n = 1;
      for (int a = 0; a < 5; ++a) {
        L.shapes.push_back(sh[a]);
        n *= (size_t)sh[a];
      }
      L.sites.push_back(dev_copy(randn(n, g)));
    }
  return L;
}

// Host -> device -> host round trip of n doubles through host memory `h` (a
// sanitizer heap block, a stack array or pinned memory); true when every value
// comes back.
static bool round_trip(double* h, double* back, int n, const char* kind) {
  for (int i = 0; i < n; ++i) h[i] = 1.0 + i;
  double* d = nullptr;
  if (hipMalloc(&d, n * sizeof(double)) != hipSuccess) std::abort();
  const hipError_t e1 = hipMemcpy(d, h, n * sizeof(double), hipMemcpyHostToDevice);
  for (int i = 0; i < n; ++i) back[i] = -1.0;
  const hipError_t e2 = hipMemcpy(back, d, n * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  int bad = 0;
  for (int i = 0; i < n; ++i) bad += back[i] != 1.0 + i;
  std::fprintf(stderr, "round trip via %s: copy status %d %d, %d of %d values wrong (first back %g)\n", kind,
               (int)e1, (int)e2, bad, n, back[0]);
  return e1 == hipSuccess && e2 == hipSuccess && bad == 0;
}

static std::vector<double> host_copy(const double* d, size_t n) {
  std::vector<double> h(n);
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(h.data(), d, n * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    std::abort();
  return h;
}

// largest |Q^T Q - I| of a row-major n x k panel
static double orth_error(const std::vector<double>& Q, int n, int k) {
  double e = 0;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      double g = 0;
      for (int r = 0; r < n; ++r) g += Q[r * k + i] * Q[r * k + j];
      e = std::max(e, std::fabs(g - (i == j)));
    }
  return e;
}

// The stages of the randomized SVD one by one on small inputs, each checked
// on the host: the product, CholeskyQR, Householder QR of a rank-deficient
// panel and the small SVD.
static void check_stages(hpeps_ctx* ctx, std::mt19937_64& g) {
  const int M = 6, K = 5, N = 7;
  const std::vector<double> hA = randn(M * K, g), hB = randn(K * N, g);
  double *A = dev_copy(hA), *B = dev_copy(hB), *C = nullptr;
  if (hipMalloc(&C, M * N * sizeof(double)) != hipSuccess) std::abort();
  for (int smallk = 1; smallk >= 0; --smallk) {
    EXPECT(hpeps_test_gemm_smallk(ctx, smallk), HPEPS_OK);
    EXPECT(hpeps_test_gemm(ctx, HPEPS_F64, 1, M, N, K, 0, A, B, C), HPEPS_OK);
    const std::vector<double> hC = host_copy(C, M * N);
    double e = 0;
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < N; ++j) {
        double v = 0;
        for (int t = 0; t < K; ++t) v += hA[i * K + t] * hB[t * N + j];
        e = std::max(e, std::fabs(v - hC[i * N + j]));
      }
    std::fprintf(stderr, "stage gemm (smallk %d): max error %g\n", smallk, e);
    CHECK(e < 1e-12);
  }
  EXPECT(hpeps_test_gemm_smallk(ctx, 1), HPEPS_OK);
  // a full-rank 6 x 6 panel through CholeskyQR, then the rank-5 product
  // A (B's first six columns) through Householder QR
  const int n = 6;
  double *Y = dev_copy(randn(n * n, g)), *P = nullptr, *R = nullptr;
  if (hipMalloc(&P, n * n * sizeof(double)) != hipSuccess || hipMalloc(&R, n * n * sizeof(double)) != hipSuccess)
    std::abort();
  EXPECT(hpeps_test_orthogonalize(ctx, HPEPS_F64, 1, n, n, Y, P), HPEPS_OK);
  double e = orth_error(host_copy(P, n * n), n, n);
  std::fprintf(stderr, "stage CholeskyQR: orthogonality error %g\n", e);
  CHECK(e < 1e-12);
  std::vector<double> hY(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0;
      for (int t = 0; t < K; ++t) v += hA[i * K + t] * hB[t * N + j];
      hY[i * n + j] = v;
    }
  double* Yd = dev_copy(hY);
  EXPECT(hpeps_test_householder(ctx, HPEPS_F64, 1, n, n, Yd, P, R), HPEPS_OK);
  const std::vector<double> hP = host_copy(P, n * n), hR = host_copy(R, n * n);
  double rec = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0;
      for (int t = 0; t < n; ++t) v += hP[i * n + t] * hR[t * n + j];
      rec = std::max(rec, std::fabs(v - hY[i * n + j]));
    }
  e = orth_error(hP, n, n);
  std::fprintf(stderr, "stage Householder (rank 5): orthogonality error %g, reconstruction error %g\n", e, rec);
  CHECK(e < 1e-12 && rec < 1e-12);
  // small SVD of that R: the singular values of Y
  double *Z = nullptr, *sig = nullptr;
  if (hipMalloc(&Z, n * n * sizeof(double)) != hipSuccess || hipMalloc(&sig, n * sizeof(double)) != hipSuccess)
    std::abort();
  EXPECT(hpeps_test_small_svd(ctx, HPEPS_F64, 1, n, R, Z, sig), HPEPS_OK);
  const std::vector<double> hs = host_copy(sig, n);
  double fro2 = 0, s2 = 0;
  for (double v : hY) fro2 += v * v;
  for (double v : hs) s2 += v * v;
  std::fprintf(stderr, "stage small SVD: sigma %g .. %g, |sum sigma^2 - |Y|_F^2| %g\n", hs[0], hs[n - 1],
               std::fabs(s2 - fro2));
  CHECK(std::fabs(s2 - fro2) < 1e-10 * fro2 && hs[0] >= hs[n - 1]);
  for (double* p : {A, B, C, Y, P, R, Yd, Z, sig}) (void)hipFree(p);
}

int main() {
  {
    std::vector<double> h(64), back(64);
    double hs[64], bs[64];
    double *ph = nullptr, *pb = nullptr;
    if (hipHostMalloc(&ph, 64 * sizeof(double)) != hipSuccess || hipHostMalloc(&pb, 64 * sizeof(double)) != hipSuccess)
      std::abort();
    CHECK(round_trip(h.data(), back.data(), 64, "heap"));
    CHECK(round_trip(hs, bs, 64, "stack"));
    CHECK(round_trip(ph, pb, 64, "pinned"));
    (void)hipHostFree(ph);
    (void)hipHostFree(pb);
  }
  for (int s = 0; s <= 9; ++s) CHECK(hpeps_status_string((hpeps_status)s) != nullptr);
  hpeps_ctx* ctx = nullptr;
  EXPECT(hpeps_create(0, &ctx), HPEPS_OK);
  if (!ctx) return 1;
  std::mt19937_64 g(12345);
  check_stages(ctx, g);

  // ---- subscripts: one well-formed network and malformed ones ----
  const int64_t a = 6, b = 5, c = 7;
  double* A = dev_copy(randn(a * b, g));
  double* B = dev_copy(randn(b * c, g));
  hpeps_tensor ops[2];
  std::memset(ops, 0, sizeof(ops));
  ops[0].data = A;
  ops[0].ndim = 2;
  ops[0].shape[0] = a;
  ops[0].shape[1] = b;
  ops[0].strides[0] = b;
  ops[0].strides[1] = 1;
  ops[1].data = B;
  ops[1].ndim = 2;
  ops[1].shape[0] = b;
  ops[1].shape[1] = c;
  ops[1].strides[0] = c;
  ops[1].strides[1] = 1;
  const hpeps_esvd_opts o3 = opts(3);
  int64_t rows = 0, cols = 0, kept = 0;
  EXPECT(hpeps_einsumsvd_query(ctx, "ab,bc->a|c", 2, ops, &o3, &rows, &cols, &kept), HPEPS_OK);
  CHECK(rows == a && cols == c && kept == 3);
  const char* bad[] = {"ab,bc->ac", "ab,bc->a|c|", "aa,bc->a|c", "ab,bc->a|b", "ab,bc,cd->a|d", "", "->|",
                       "ab,bc->a|cc", "ab,bc->a|x", "ab;bc->a|c"};
  for (const char* s : bad) {
    const hpeps_status st = hpeps_einsumsvd_query(ctx, s, 2, ops, &o3, &rows, &cols, &kept);
    if (st == HPEPS_OK) {
      std::fprintf(stderr, "malformed subscripts accepted: '%s'\n", s);
      ++g_fail;
    }
  }
  EXPECT(hpeps_einsumsvd_query(ctx, nullptr, 2, ops, &o3, &rows, &cols, &kept), HPEPS_ERR_INVALID_ARG);

  // ---- einsumsvd of the network ----
  double *U = nullptr, *R = nullptr, *sg = nullptr;
  if (hipMalloc(&U, a * 3 * sizeof(double)) != hipSuccess || hipMalloc(&R, 3 * c * sizeof(double)) != hipSuccess ||
      hipMalloc(&sg, 3 * sizeof(double)) != hipSuccess)
    std::abort();
  EXPECT(hpeps_einsumsvd(ctx, HPEPS_F64, "ab,bc->a|c", 2, ops, &o3, HPEPS_ABSORB_NONE, U, sg, R, nullptr),
         HPEPS_OK);
  double hs[3];
  if (hipMemcpy(hs, sg, sizeof(hs), hipMemcpyDeviceToHost) != hipSuccess) std::abort();
  for (double v : hs) CHECK(v > 0 && std::isfinite(v));
  hpeps_esvd_info info;
  EXPECT(hpeps_get_info(ctx, &info), HPEPS_OK);
  std::fprintf(stderr, "einsumsvd sigma %g %g %g  k %lld extra %d numeric %d householder %d sweeps %d\n", hs[0],
               hs[1], hs[2], (long long)info.sketch_width, info.orth_extra_passes, info.numeric_errors,
               info.orth_householder, info.jacobi_sweeps);

  // ---- batched form of the network: instance 1 equals the single call with stream_id + 1 ----
  {
    double* A2 = dev_copy(randn(2 * a * b, g));
    double* B2 = dev_copy(randn(2 * b * c, g));
    hpeps_tensor bops[2];
    std::memset(bops, 0, sizeof(bops));
    const int64_t bsh[2][3] = {{2, a, b}, {2, b, c}}, bst[2][3] = {{a * b, b, 1}, {b * c, c, 1}};
    bops[0].data = A2;
    bops[1].data = B2;
    for (int t = 0; t < 2; ++t) {
      bops[t].ndim = 3;
      for (int q = 0; q < 3; ++q) {
        bops[t].shape[q] = bsh[t][q];
        bops[t].strides[q] = bst[t][q];
      }
    }
    double *U2 = nullptr, *R2 = nullptr, *s2 = nullptr;
    if (hipMalloc(&U2, 2 * a * 3 * sizeof(double)) != hipSuccess ||
        hipMalloc(&R2, 2 * 3 * c * sizeof(double)) != hipSuccess || hipMalloc(&s2, 6 * sizeof(double)) != hipSuccess)
      std::abort();
    EXPECT(hpeps_einsumsvd_batched(ctx, HPEPS_F64, 2, "ab,bc->a|c", 2, bops, &o3, HPEPS_ABSORB_NONE, U2, s2, R2,
                                   nullptr),
           HPEPS_OK);
    hpeps_tensor one[2] = {ops[0], ops[1]};
    one[0].data = A2 + a * b;
    one[1].data = B2 + b * c;
    hpeps_esvd_opts o3b = o3;
    o3b.stream_id += 1;
    EXPECT(hpeps_einsumsvd(ctx, HPEPS_F64, "ab,bc->a|c", 2, one, &o3b, HPEPS_ABSORB_NONE, U, sg, R, nullptr),
           HPEPS_OK);
    const std::vector<double> sb = host_copy(s2, 6), s1 = host_copy(sg, 3);
    for (int i = 0; i < 3; ++i) CHECK(std::fabs(sb[3 + i] - s1[i]) <= 1e-12 * s1[0]);
    EXPECT(hpeps_einsumsvd_batched(ctx, HPEPS_F64, 0, "ab,bc->a|c", 2, bops, &o3, HPEPS_ABSORB_NONE, U2, s2, R2,
                                   nullptr),
           HPEPS_ERR_INVALID_ARG);
    bops[0].strides[0] = 0;  // overlapping instances
    EXPECT(hpeps_einsumsvd_batched(ctx, HPEPS_F64, 2, "ab,bc->a|c", 2, bops, &o3, HPEPS_ABSORB_NONE, U2, s2, R2,
                                   nullptr),
           HPEPS_ERR_SHAPE);
    for (double* p : {A2, B2, U2, R2, s2}) (void)hipFree(p);
  }

  // ---- adjoint of a network of full rank 6 = k (6 x 6 times 6 x 7) ----
  {
    double* A3 = dev_copy(randn(36, g));
    double* B3 = dev_copy(randn(42, g));
    hpeps_tensor ops3[2] = {ops[0], ops[1]};
    ops3[0].data = A3;
    ops3[0].shape[1] = 6;
    ops3[0].strides[0] = 6;
    ops3[1].data = B3;
    ops3[1].shape[0] = 6;
    double* dU3 = dev_copy(randn(6 * 3, g));
    double* dR3 = dev_copy(randn(3 * 7, g));
    double *g0 = nullptr, *g1 = nullptr;
    if (hipMalloc(&g0, 36 * sizeof(double)) != hipSuccess || hipMalloc(&g1, 42 * sizeof(double)) != hipSuccess)
      std::abort();
    void* gp[2] = {g0, g1};
    EXPECT(hpeps_einsumsvd_backward(ctx, HPEPS_F64, "ab,bc->a|c", 2, ops3, &o3, HPEPS_ABSORB_NONE, 0.0, dU3, nullptr,
                                    dR3, gp),
           HPEPS_OK);
    bool finite = true;
    for (double v : host_copy(g0, 36)) finite = finite && std::isfinite(v);
    for (double v : host_copy(g1, 42)) finite = finite && std::isfinite(v);
    CHECK(finite);
    EXPECT(hpeps_einsumsvd_backward(ctx, HPEPS_F64, "ab,bc->a|c", 2, ops3, &o3, HPEPS_ABSORB_CARRY, 0.0, dU3,
                                    nullptr, dR3, gp),
           HPEPS_ERR_UNSUPPORTED);
    for (double* p : {A3, B3, dU3, dR3, g0, g1}) (void)hipFree(p);
  }

  // ---- autotune JSON: export (size query, then the text) and imports ----
  int64_t need = 0;
  EXPECT(hpeps_autotune_export(ctx, nullptr, 0, &need), HPEPS_OK);
  std::vector<char> buf((size_t)need + 1);
  EXPECT(hpeps_autotune_export(ctx, buf.data(), (int64_t)buf.size(), &need), HPEPS_OK);
  EXPECT(hpeps_autotune_import(ctx, buf.data()), HPEPS_OK);
  EXPECT(hpeps_autotune_import(ctx, "{\"gemm\": {\"f64_M8_N8_K8_b1_a00_b00\": [0, 1, 1]}}"), HPEPS_OK);
  const char* bad_json[] = {"", "{", "{\"gemm\": ", "{\"gemm\": {\"k\": [1, 2]}}", "{\"gemm\": {\"k\": [99, 1, 1]}}",
                            "{\"gemm\": {\"k\": [0, 1, -2]}}", "[]", "{\"other\": {}}"};
  for (const char* s : bad_json) {
    if (hpeps_autotune_import(ctx, s) == HPEPS_OK) {
      std::fprintf(stderr, "malformed autotune JSON accepted: '%s'\n", s);
      ++g_fail;
    }
  }

  // ---- PEPS norm (3 x 3, bond 2) and a bad option ----
  Lattice L = make_lattice(3, 3, 2, g);
  const hpeps_peps P = L.view();
  const hpeps_esvd_opts o4 = opts(4);
  double ln = 0, ph[2] = {0, 0};
  EXPECT(hpeps_peps_norm(ctx, &P, nullptr, &o4, &ln, ph), HPEPS_OK);
  CHECK(std::isfinite(ln));
  hpeps_esvd_opts obad = o4;
  obad.rank = 0;
  EXPECT(hpeps_peps_norm(ctx, &P, nullptr, &obad, &ln, ph), HPEPS_ERR_INVALID_ARG);

  // ---- amplitude <0...0|psi> and a bit out of range ----
  {
    std::vector<int32_t> bits(9, 0);
    double la = 0, aph[2] = {0, 0};
    EXPECT(hpeps_peps_amplitude(ctx, &P, bits.data(), &o4, &la, aph), HPEPS_OK);
    CHECK(std::isfinite(la) && std::isfinite(aph[0]) && std::isfinite(aph[1]));
    bits[4] = 2;
    EXPECT(hpeps_peps_amplitude(ctx, &P, bits.data(), &o4, &la, aph), HPEPS_ERR_INVALID_ARG);
  }

  // ---- energy of a ZZ bond and a one-site X; a term on non-neighbours ----
  {
    std::vector<double> zz(32, 0.0), xop(8, 0.0), ops_h;
    const double zs[2] = {1.0, -1.0};
    for (int a2 = 0; a2 < 2; ++a2)
      for (int b2 = 0; b2 < 2; ++b2) zz[2 * ((a2 * 2 + b2) * 4 + a2 * 2 + b2)] = zs[a2] * zs[b2];
    xop[2 * 1] = xop[2 * 2] = 1.0;  // X = [[0, 1], [1, 0]] as complex pairs
    ops_h.insert(ops_h.end(), zz.begin(), zz.end());
    ops_h.insert(ops_h.end(), xop.begin(), xop.end());
    const int32_t nsites[2] = {2, 1};
    int32_t sites[8] = {0, 0, 0, 1, 1, 1, 0, 0};
    const int64_t off[2] = {0, 16};  // in complex entries: the X operator follows the 16 of ZZ
    double e[2] = {0, 0}, per[4] = {0, 0, 0, 0};
    EXPECT(hpeps_peps_energy(ctx, &P, 2, nsites, sites, ops_h.data(), off, &o4, e, per), HPEPS_OK);
    CHECK(std::isfinite(e[0]) && std::fabs(e[0] - (per[0] + per[2])) <= 1e-10 * (1 + std::fabs(e[0])));
    sites[2] = 2;
    sites[3] = 2;  // (0,0) with (2,2): not neighbours
    CHECK(hpeps_peps_energy(ctx, &P, 2, nsites, sites, ops_h.data(), off, &o4, e, per) != HPEPS_OK);
  }

  // ---- gradient of log<psi|psi> with respect to every site; a null gradient pointer ----
  {
    std::vector<void*> gr(9, nullptr);
    std::vector<size_t> gn(9, 1);
    for (int t = 0; t < 9; ++t) {
      for (int q = 0; q < 5; ++q) gn[t] *= (size_t)L.shapes[5 * t + q];
      if (hipMalloc(&gr[t], gn[t] * sizeof(double)) != hipSuccess) std::abort();
    }
    double lg = 0;
    EXPECT(hpeps_peps_norm_backward(ctx, &P, &o4, 0.0, gr.data(), &lg), HPEPS_OK);
    CHECK(std::isfinite(lg));
    std::fprintf(stderr, "log<psi|psi>: norm %.15g, norm_backward %.15g\n", ln, lg);
    bool fin = true;
    for (int t = 0; t < 9; ++t)
      for (double v : host_copy((const double*)gr[t], gn[t])) fin = fin && std::isfinite(v);
    CHECK(fin);
    void* keep = gr[4];
    gr[4] = nullptr;
    EXPECT(hpeps_peps_norm_backward(ctx, &P, &o4, 0.0, gr.data(), &lg), HPEPS_ERR_INVALID_ARG);
    gr[4] = keep;
    for (void* q : gr) (void)hipFree(q);
  }

  // ---- ITE plan: graph, direct layers, one launch per bond ----
  Lattice I = make_lattice(3, 4, 1, g);
  const hpeps_peps PI = I.view();
  std::vector<double> gate(16, 0.0);
  for (int e = 0; e < 4; ++e) gate[e * 5] = 1.0;
  gate[0] = 0.9;
  gate[15] = 0.9;
  gate[6] = 0.1;
  gate[9] = 0.1;
  double* dG = dev_copy(gate);
  const int nbonds = 3 * 3 + 2 * 4;
  std::vector<int32_t> bond_gate(nbonds, 0);
  hpeps_ite_plan* plan = nullptr;
  EXPECT(hpeps_ite_plan_create(ctx, &PI, 1, dG, bond_gate.data(), 4, &plan), HPEPS_OK);
  if (plan) {
    EXPECT(hpeps_ite_run(plan, 2, 1), HPEPS_OK);
    EXPECT(hpeps_ite_run(plan, 1, 0), HPEPS_OK);
    EXPECT(hpeps_ite_run(plan, 1, 2), HPEPS_OK);
    EXPECT(hpeps_ite_run(plan, 1, 7), HPEPS_ERR_INVALID_ARG);
    int32_t nl = 0, nb = 0;
    EXPECT(hpeps_ite_plan_layers(plan, &nl, &nb), HPEPS_OK);
    CHECK(nl == 4 && nb == nbonds);
    std::vector<int64_t> shp(3 * 4 * 5);
    EXPECT(hpeps_ite_get_state(plan, shp.data(), nullptr), HPEPS_OK);
    EXPECT(hpeps_ite_plan_destroy(plan), HPEPS_OK);
  }
  EXPECT(hpeps_ite_plan_create(ctx, &PI, 1, dG, bond_gate.data(), 0, &plan), HPEPS_ERR_INVALID_ARG);

  // ---- allocation-free gate update on a copy of the lattice with room for bond 4 ----
  Lattice W = make_lattice(3, 4, 2, g);
  std::vector<int64_t> cap(12);
  for (int s = 0; s < 12; ++s) {
    cap[s] = 4 * 4 * 4 * 4 * 2;
    double* big = nullptr;
    if (hipMalloc(&big, cap[s] * sizeof(double)) != hipSuccess) std::abort();
    size_t n = 1;
    for (int t = 0; t < 5; ++t) n *= (size_t)W.shapes[5 * s + t];
    if (hipMemcpy(big, W.sites[s], n * sizeof(double), hipMemcpyDeviceToDevice) != hipSuccess) std::abort();
    (void)hipFree(W.sites[s]);
    W.sites[s] = big;
  }
  hpeps_peps PW{3, 4, HPEPS_F64, 0, W.sites.data(), W.shapes.data()};
  int64_t nbond = 0;
  double* sig = nullptr;
  if (hipMalloc(&sig, 4 * sizeof(double)) != hipSuccess) std::abort();
  EXPECT(hpeps_apply_two_site_gate_noalloc(ctx, &PW, cap.data(), 1, 1, 0, dG, 4, &nbond, sig), HPEPS_OK);
  EXPECT(hpeps_apply_two_site_gate(ctx, &PW, cap.data(), 1, 2, 1, dG, 4, &nbond, sig), HPEPS_OK);
  EXPECT(hpeps_apply_two_site_gate(ctx, &PW, cap.data(), 1, 3, 0, dG, 4, &nbond, sig), HPEPS_ERR_INVALID_ARG);

  // ---- profiler ----
  EXPECT(hpeps_profile_start(ctx, nullptr), HPEPS_OK);
  EXPECT(hpeps_einsumsvd(ctx, HPEPS_F64, "ab,bc->a|c", 2, ops, &o3, HPEPS_ABSORB_RIGHT, U, sg, R, nullptr),
         HPEPS_OK);
  std::vector<hpeps_profile_entry> ent(64);
  int32_t nent = 0;
  EXPECT(hpeps_profile_read(ctx, (int32_t)ent.size(), ent.data(), &nent), HPEPS_OK);
  CHECK(nent >= 1);
  EXPECT(hpeps_profile_stop(ctx), HPEPS_OK);

  EXPECT(hpeps_destroy(ctx), HPEPS_OK);
  for (auto* p : {A, B, U, R, sg, dG, sig}) (void)hipFree(p);
  for (auto* L2 : {&L, &I, &W})
    for (void* p : L2->sites) (void)hipFree(p);
  if (g_fail) std::fprintf(stderr, "%d check(s) failed\n", g_fail);
  else std::printf("host sanitizer driver: all checks passed\n");
  return g_fail ? 1 : 0;
}
