// Householder QR of tall panels: the fallback of Alg. 4's "orthogonalize"
// for sketches that the first CholeskyQR pass flags (breakdown, or a
// Cholesky diagonal spanning more than 1e7, i.e. a numerically
// rank-deficient or very ill-conditioned panel).
//
// A Gram-based factorization cannot resolve the directions of such a panel
// below the square root of the unit roundoff: the basis it returns for the
// weak and null directions keeps components in range(Y) far above rounding,
// and the next operator application turns them into spurious singular
// values.  Householder QR is backward stable for any conditioning (Y + E =
// Q R with ||E|| = O(u ||Y||) and Q orthonormal to rounding), which is the
// property the randomized SVD needs: its result depends only on the range
// of each panel up to rounding (basis invariance).
//
// Tall-skinny QR in one reduction level: the n rows are split into nblk
// blocks of at least 2k rows; one workgroup factors each block (Householder
// reflectors in a column-major copy, its k x k R); one workgroup per
// instance factors the stacked R's and forms their Q explicitly; one
// workgroup per block then applies its reflectors to its k rows of that Q
// padded with zeros, which gives the block's rows of the panel's Q.
// Reflectors follow the LAPACK convention (H = I - tau v v^H, v_j = 1,
// beta = -sign(Re alpha) ||x||, tau = 0 for a column that is already zero
// below the diagonal).  The basis Q may differ from another QR's by a
// unitary k x k factor (and in the null directions of a rank-deficient
// panel); only its range enters the randomized SVD.
// Instances whose flag lacks the requested bit return at once.
#include <algorithm>
#include <cmath>

#include "dpp.h"
#include "esvd.h"

namespace hp {

namespace {

constexpr int kHhThreads = 256;
constexpr int kHhWaves = kHhThreads / 64;
constexpr int kHhMaxK = 128;

struct V2 {
  double re, im;
};

template <bool CPLX>
struct E2 {
  static constexpr int es = CPLX ? 2 : 1;
  static __device__ __forceinline__ V2 ld(const double* p, long long i) {
    if constexpr (CPLX) return {p[2 * i], p[2 * i + 1]};
    else return {p[i], 0.0};
  }
  static __device__ __forceinline__ void st(double* p, long long i, V2 v) {
    if constexpr (CPLX) {
      p[2 * i] = v.re;
      p[2 * i + 1] = v.im;
    } else {
      p[i] = v.re;
    }
  }
  // conj(a) * b
  static __device__ __forceinline__ V2 cjmul(V2 a, V2 b) {
    if constexpr (CPLX) return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
    else return {a.re * b.re, 0.0};
  }
  static __device__ __forceinline__ V2 mul(V2 a, V2 b) {
    if constexpr (CPLX) return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    else return {a.re * b.re, 0.0};
  }
  // a - b * c
  static __device__ __forceinline__ V2 fnms(V2 a, V2 b, V2 c) {
    if constexpr (CPLX) return {a.re - (b.re * c.re - b.im * c.im), a.im - (b.re * c.im + b.im * c.re)};
    else return {a.re - b.re * c.re, 0.0};
  }
  static __device__ __forceinline__ V2 add(V2 a, V2 b) {
    if constexpr (CPLX) return {a.re + b.re, a.im + b.im};
    else return {a.re + b.re, 0.0};
  }
  static __device__ __forceinline__ V2 cj(V2 a) { return {a.re, -a.im}; }
};

// In-place Householder QR of the rows x k column-major matrix A (column c
// at A + c * ld, element offsets in scalars of the type): afterwards the
// upper triangle holds R (R[j][c] at column c, row j) and column j below the
// diagonal holds v_j[r] (r > j); tau[j] receives tau_j.  rows >= k.  All
// kHhThreads threads of the workgroup take part.
template <bool CPLX>
__device__ void hh_factor(double* A, long long ld, int rows, int k, double* tau, V2* sh_s, V2* sh_g) {
  using E = E2<CPLX>;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int j = 0; j < k; ++j) {
    const double* Aj = A + (long long)j * ld * E::es;
    // s_l = sum_{r > j} conj(A[r, j]) A[r, l] for l >= j (s_j = ||x||^2)
    for (int l = j + wv; l < k; l += kHhWaves) {
      const double* Al = A + (long long)l * ld * E::es;
      V2 acc = {0.0, 0.0};
      for (int r = j + 1 + lane; r < rows; r += 64) acc = E::add(acc, E::cjmul(E::ld(Aj, r), E::ld(Al, r)));
      acc.re = wave_sum(acc.re);
      if constexpr (CPLX) acc.im = wave_sum(acc.im);
      if (lane == 0) sh_s[l] = acc;
    }
    __syncthreads();
    // the reflector (every thread computes the same scalars)
    const V2 alpha = E::ld(Aj, j);
    const double xn2 = sh_s[j].re;
    V2 tj = {0.0, 0.0}, scale = {0.0, 0.0};
    double beta = alpha.re;
    const bool skip = xn2 == 0.0 && (!CPLX || alpha.im == 0.0);
    if (!skip) {
      const double nrm = sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn2);
      beta = -copysign(nrm, alpha.re);
      tj = {(beta - alpha.re) / beta, -alpha.im / beta};
      // scale = 1 / (alpha - beta)
      const double dr = alpha.re - beta, di = alpha.im;
      const double den = dr * dr + di * di;
      scale = {dr / den, -di / den};
    }
    // g_l = conj(tau) (v^H A[:, l]), v^H A[:, l] = A[j, l] + conj(scale) s_l
    for (int l = j + 1 + tid; l < k; l += kHhThreads) {
      const V2 c = E::add(E::ld(A + (long long)l * ld * E::es, j), E::cjmul(scale, sh_s[l]));
      sh_g[l] = E::cjmul(tj, c);
    }
    if (tid == 0) E::st(tau, j, tj);
    __syncthreads();
    // A[:, l] -= g_l v (rows >= j, columns > j); column j becomes v / R[j, j]
    if (!skip) {
      for (int r = j + tid; r < rows; r += kHhThreads) {
        const V2 v = r == j ? V2{1.0, 0.0} : E::mul(scale, E::ld(Aj, r));
        for (int l = j + 1; l < k; ++l) {
          double* Al = A + (long long)l * ld * E::es;
          E::st(Al, r, E::fnms(E::ld(Al, r), sh_g[l], v));
        }
        E::st(const_cast<double*>(Aj), r, r == j ? V2{beta, 0.0} : v);
      }
    }
    __syncthreads();
  }
}

// B <- H_0 H_1 ... H_{nref-1} B for the reflectors of hh_factor (column j of
// W below the diagonal, tau) and the rows x ncols column-major B.  With
// form_q, B starts as [I; 0] and column l < j is still e_l when H_j is
// applied, so only columns l >= j are touched.
template <bool CPLX>
__device__ void hh_apply(const double* W, long long ldw, const double* tau, int nref, double* B, long long ldb,
                         int rows, int ncols, bool form_q, V2* sh_g) {
  using E = E2<CPLX>;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int j = nref - 1; j >= 0; --j) {
    const double* Wj = W + (long long)j * ldw * E::es;
    const V2 tj = E::ld(tau, j);
    if (tj.re == 0.0 && tj.im == 0.0) continue;  // H_j = I (uniform)
    const int l0 = form_q ? j : 0;
    // g_l = tau (v^H B[:, l])
    for (int l = l0 + wv; l < ncols; l += kHhWaves) {
      const double* Bl = B + (long long)l * ldb * E::es;
      V2 acc = {0.0, 0.0};
      for (int r = j + lane; r < rows; r += 64) {
        const V2 v = r == j ? V2{1.0, 0.0} : E::ld(Wj, r);
        acc = E::add(acc, E::cjmul(v, E::ld(Bl, r)));
      }
      acc.re = wave_sum(acc.re);
      if constexpr (CPLX) acc.im = wave_sum(acc.im);
      if (lane == 0) sh_g[l] = E::mul(tj, acc);
    }
    __syncthreads();
    for (int r = j + tid; r < rows; r += kHhThreads) {
      const V2 v = r == j ? V2{1.0, 0.0} : E::ld(Wj, r);
      for (int l = l0; l < ncols; ++l) {
        double* Bl = B + (long long)l * ldb * E::es;
        E::st(Bl, r, E::fnms(E::ld(Bl, r), sh_g[l], v));
      }
    }
    __syncthreads();
  }
}

__device__ __forceinline__ bool hh_active(const int* flags, int mask, int b) {
  return !flags || (flags[b] & mask) != 0;
}

// Block i of instance b: rows [n i / nblk, n (i + 1) / nblk) of Y (row-major
// n x k) are copied column-major into W (k columns of stride n) and factored;
// the block's R goes to rows [i k, (i + 1) k) of the stacked matrix Ws
// (column-major, nblk k rows).
template <bool CPLX>
__global__ __launch_bounds__(kHhThreads) void hh_block_factor_kernel(const double* Y, long long n, int k, int nblk,
                                                                     const int* flags, int mask, double* W,
                                                                     double* tau, double* Ws) {
  using E = E2<CPLX>;
  __shared__ V2 sh_s[kHhMaxK], sh_g[kHhMaxK];
  const int i = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  if (!hh_active(flags, mask, b)) return;
  const long long r0 = n * i / nblk, r1 = n * (i + 1) / nblk;
  const int rows = (int)(r1 - r0);
  const double* Yb = Y + (long long)b * n * k * E::es;
  double* Wb = W + (long long)b * n * k * E::es;
  for (long long e = tid; e < (long long)rows * k; e += kHhThreads) {
    const long long r = e / k;
    const int c = (int)(e - r * k);
    E::st(Wb, (long long)c * n + r0 + r, E::ld(Yb, (r0 + r) * k + c));
  }
  __syncthreads();
  double* taub = tau + ((long long)b * nblk + i) * k * E::es;
  hh_factor<CPLX>(Wb + r0 * E::es, n, rows, k, taub, sh_s, sh_g);
  const long long ls = (long long)nblk * k;
  double* Wsb = Ws + (long long)b * ls * k * E::es;
  for (int e = tid; e < k * k; e += kHhThreads) {
    const int c = e / k, r = e - c * k;
    const V2 v = r <= c ? E::ld(Wb, (long long)c * n + r0 + r) : V2{0.0, 0.0};
    E::st(Wsb, (long long)c * ls + (long long)i * k + r, v);
  }
}

// Per instance: QR of the stacked R's (nblk k x k, column-major in Ws, in
// place); R to Rout (row-major k x k, zero below the diagonal) when given;
// the explicit Q (column-major nblk k x k) to Qs when given.  Marks the
// instance with FLAG_HOUSEHOLDER.
template <bool CPLX>
__global__ __launch_bounds__(kHhThreads) void hh_stack_kernel(double* Ws, int k, int nblk, int* flags, int mask,
                                                              double* taus, double* Qs, double* Rout) {
  using E = E2<CPLX>;
  __shared__ V2 sh_s[kHhMaxK], sh_g[kHhMaxK];
  const int b = blockIdx.x, tid = threadIdx.x;
  if (!hh_active(flags, mask, b)) return;
  const int ls = nblk * k;
  double* Wsb = Ws + (long long)b * ls * k * E::es;
  double* tb = taus + (long long)b * k * E::es;
  hh_factor<CPLX>(Wsb, ls, ls, k, tb, sh_s, sh_g);
  if (Rout) {
    double* Rb = Rout + (long long)b * k * k * E::es;
    for (int e = tid; e < k * k; e += kHhThreads) {
      const int r = e / k, c = e - r * k;
      E::st(Rb, e, c >= r ? E::ld(Wsb, (long long)c * ls + r) : V2{0.0, 0.0});
    }
  }
  if (Qs) {
    double* Qb = Qs + (long long)b * ls * k * E::es;
    for (int e = tid; e < ls * k; e += kHhThreads) {
      const int c = e / ls, r = e - c * ls;
      E::st(Qb, e, V2{r == c ? 1.0 : 0.0, 0.0});
    }
    __syncthreads();
    hh_apply<CPLX>(Wsb, ls, tb, k, Qb, ls, ls, k, true, sh_g);
  }
  if (flags && tid == 0) flags[b] |= FLAG_HOUSEHOLDER;
}

// Block i: its rows of the panel's Q = H^(i) [Qs rows i k .. i k + k; 0],
// formed column-major in Eb and written row-major to P.
template <bool CPLX>
__global__ __launch_bounds__(kHhThreads) void hh_block_q_kernel(const double* W, long long n, int k, int nblk,
                                                                const double* tau, const double* Qs,
                                                                const int* flags, int mask, double* Ebuf,
                                                                double* P) {
  using E = E2<CPLX>;
  __shared__ V2 sh_g[kHhMaxK];
  const int i = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  if (!hh_active(flags, mask, b)) return;
  const long long r0 = n * i / nblk, r1 = n * (i + 1) / nblk;
  const int rows = (int)(r1 - r0);
  const long long ls = (long long)nblk * k;
  const double* Qb = Qs + (long long)b * ls * k * E::es;
  double* Eb = Ebuf + (long long)b * n * k * E::es + r0 * E::es;
  for (long long e = tid; e < (long long)rows * k; e += kHhThreads) {
    const int c = (int)(e / rows);
    const long long r = e - (long long)c * rows;
    E::st(Eb, (long long)c * n + r, r < k ? E::ld(Qb, (long long)c * ls + (long long)i * k + r) : V2{0.0, 0.0});
  }
  __syncthreads();
  const double* Wb = W + (long long)b * n * k * E::es + r0 * E::es;
  const double* taub = tau + ((long long)b * nblk + i) * k * E::es;
  hh_apply<CPLX>(Wb, n, taub, k, Eb, n, rows, k, false, sh_g);
  double* Pb = P + (long long)b * n * k * E::es;
  for (long long e = tid; e < (long long)rows * k; e += kHhThreads) {
    const long long r = e / k;
    const int c = (int)(e - r * k);
    E::st(Pb, (r0 + r) * k + c, E::ld(Eb, (long long)c * n + r));
  }
}

}  // namespace

int householder_blocks(int64_t n, int64_t k) {
  const int64_t nb = n / (2 * k);
  return (int)std::max<int64_t>(1, std::min<int64_t>(64, nb));
}

void householder_qr(Ctx& ctx, bool cplx, const double* Y, int64_t n, int64_t k, int batch, int* flags, int mask,
                    double* P, double* R) {
  HP_REQUIRE(k >= 1 && k <= kHhMaxK && n >= k, HPEPS_ERR_UNSUPPORTED, "Householder QR needs 1 <= k <= 128 and n >= k");
  HP_REQUIRE(n <= 0x7fffffffLL, HPEPS_ERR_UNSUPPORTED, "Householder QR panel rows above 2^31");
  WsScope scope(ctx);
  const int es = cplx ? 2 : 1;
  const int nblk = householder_blocks(n, k);
  const int64_t ls = (int64_t)nblk * k;
  double* W = ctx.ws<double>((int64_t)batch * n * k * es);
  double* tau = ctx.ws<double>((int64_t)batch * nblk * k * es);
  double* Ws = ctx.ws<double>((int64_t)batch * ls * k * es);
  double* taus = ctx.ws<double>((int64_t)batch * k * es);
  double* Qs = P ? ctx.ws<double>((int64_t)batch * ls * k * es) : nullptr;
  double* Eb = P ? ctx.ws<double>((int64_t)batch * n * k * es) : nullptr;
  const dim3 gb(nblk, batch);
  const int rec = ctx.prof_begin("householder");
  hipStream_t s = ctx.stream;
  if (cplx) {
    hh_block_factor_kernel<true><<<gb, kHhThreads, 0, s>>>(Y, n, (int)k, nblk, flags, mask, W, tau, Ws);
    hh_stack_kernel<true><<<batch, kHhThreads, 0, s>>>(Ws, (int)k, nblk, flags, mask, taus, Qs, R);
    if (P) hh_block_q_kernel<true><<<gb, kHhThreads, 0, s>>>(W, n, (int)k, nblk, tau, Qs, flags, mask, Eb, P);
  } else {
    hh_block_factor_kernel<false><<<gb, kHhThreads, 0, s>>>(Y, n, (int)k, nblk, flags, mask, W, tau, Ws);
    hh_stack_kernel<false><<<batch, kHhThreads, 0, s>>>(Ws, (int)k, nblk, flags, mask, taus, Qs, R);
    if (P) hh_block_q_kernel<false><<<gb, kHhThreads, 0, s>>>(W, n, (int)k, nblk, tau, Qs, flags, mask, Eb, P);
  }
  HP_CHECK_HIP(hipGetLastError());
  ctx.prof_end(rec, 0.0, 0.0);
}

}  // namespace hp
