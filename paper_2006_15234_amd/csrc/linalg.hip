// Small dense kernels of the randomized SVD (Alg. 4): sketch generation,
// Gram matrices, CholeskyQR factor/inverse with an automatic shift, the
// one-sided Jacobi SVD of the k x k projected factor, and helpers.
//
// Orthogonalization (Alg. 4 "orthogonalize") runs through a small Gram
// matrix, as in the paper's reshape-avoiding orthogonalization (Alg. 5),
// but factors it by Cholesky instead of an eigendecomposition:
//   pass 1:  G = Y^H Y, R = chol(G) (retried with the shift of shifted
//            CholeskyQR -- Fukaya, Kannan, Nakatsukasa, Zhang, Yamamoto,
//            SIAM J. Sci. Comput. 42 (2020) -- when it breaks down or the
//            factor is too ill-conditioned), P1 = Y R^-1
//   pass 2:  the same on P1 (CholeskyQR2, Yamamoto et al. 2015)
//   pass 3:  only for sketches flagged in pass 1.
// Every small factorization runs in one 1024-thread workgroup per instance
// with the k x k matrix resident in LDS (up to 128 KB of the 160 KB).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "dpp.h"
#include "internal.h"

namespace hp {

namespace {

struct cd {
  double re, im;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cconj(cd a) { return {a.re, -a.im}; }

template <bool CPLX>
struct S;
template <>
struct S<false> {
  using T = double;
  static __device__ __forceinline__ double re(double x) { return x; }
  static __device__ __forceinline__ double abs2(double x) { return x * x; }
  static __device__ __forceinline__ double mul(double a, double b) { return a * b; }
  static __device__ __forceinline__ double conjmul(double a, double b) { return a * b; }  // conj(a)*b
  static __device__ __forceinline__ double conj(double a) { return a; }
  static __device__ __forceinline__ double scale(double a, double s) { return a * s; }
  static __device__ __forceinline__ double zero() { return 0.0; }
  static __device__ __forceinline__ double one() { return 1.0; }
  static __device__ __forceinline__ double sub(double a, double b) { return a - b; }
  static __device__ __forceinline__ double add(double a, double b) { return a + b; }
  static __device__ __forceinline__ bool finite(double a) { return isfinite(a); }
};
template <>
struct S<true> {
  using T = cd;
  static __device__ __forceinline__ double re(cd x) { return x.re; }
  static __device__ __forceinline__ double abs2(cd x) { return x.re * x.re + x.im * x.im; }
  static __device__ __forceinline__ cd mul(cd a, cd b) { return cmul(a, b); }
  static __device__ __forceinline__ cd conjmul(cd a, cd b) { return cmul(cconj(a), b); }
  static __device__ __forceinline__ cd conj(cd a) { return cconj(a); }
  static __device__ __forceinline__ cd scale(cd a, double s) { return {a.re * s, a.im * s}; }
  static __device__ __forceinline__ cd zero() { return {0.0, 0.0}; }
  static __device__ __forceinline__ cd one() { return {1.0, 0.0}; }
  static __device__ __forceinline__ cd sub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
  static __device__ __forceinline__ cd add(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
  static __device__ __forceinline__ bool finite(cd a) { return isfinite(a.re) && isfinite(a.im); }
};

constexpr int kSmallThreads = 1024;

// ---------------------------------------------------------------------------
// sketch generator (SplitMix64 output function, counter based)
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

// stride = 2 writes the values as the real parts of a complex array (the
// imaginary parts are set to zero): the sketch is real for complex operators.
template <class TO>
__global__ void sketch_kernel(TO* out, long long nk, uint64_t seed, uint64_t stream_id, int stride) {
  const int b = blockIdx.y;
  const uint64_t base = mix64(mix64(seed) + stream_id + (uint64_t)b);
  TO* o = out + (long long)b * nk * stride;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nk;
       i += (long long)gridDim.x * blockDim.x) {
    const uint64_t h = mix64(base + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull);
    // (h >> 11) < 2^53 converts exactly; the affine map below is exact too.
    const double v = 2.0 * (double)(h >> 11) * 0x1p-53 - 1.0;
    o[i * stride] = (TO)v;
    if (stride == 2) o[i * 2 + 1] = (TO)0;
  }
}

// ---------------------------------------------------------------------------
// Cholesky factor and its inverse for one k x k Gram matrix per workgroup.
// Gaussian elimination of the Hermitian G without pivoting: step j subtracts
// (conj(A[j,i]) / d_j) row j from every row i > j, with d_j = A[j,j].  The
// upper triangle ends as U = D R (R = chol(G), G = R^H R, D = diag(sqrt d))
// and the same row operations applied to the identity give the unit lower
// triangular M with M G = U, i.e. M = D R^-H; M is kept in the strict lower
// triangle of the same array.  Hence R = D^-1 U and R^-1 = M^H D^-1 without
// a separate triangular inversion.  Step j reads row j and writes rows > j
// only: one barrier per step.  The step is latency-bound (k sequential
// steps of a few LDS round trips), so it is kept short: four wavefronts,
// lane = column (and column + 64), rows i > j dealt round-robin to the
// wavefronts, and all the rows of a wavefront loaded in one batch with
// clamped (always in-range) addresses, updated, and stored under a mask.
constexpr int kCholThreads = 512;
constexpr int kCholWaves = kCholThreads / 64;
// LDS of one instance: the k x k array and one spare slot per lane
size_t chol_lds_bytes(int k, bool cplx) { return (size_t)(k * k + 64) * (cplx ? 16 : 8); }

template <bool CPLX, bool TWO>
__global__ __launch_bounds__(kCholThreads) void chol_inv_kernel(const double* Gall, long long n_rows,
                                                                 int k, int pass, double* Rinv_all,
                                                                 double* Racc_all, int* flags, int r_only) {
  using T = typename S<CPLX>::T;
  constexpr int kB = TWO ? 8 : 6;  // rows per wavefront and LDS round trip (k <= 49 or 113: one)
  extern __shared__ double smem[];
  T* A = reinterpret_cast<T*>(smem);
  __shared__ double dg[128], sq[128], rs[128];
  __shared__ double red[kCholWaves];
  const int b = blockIdx.x, tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(wave);  // as a scalar
  const int kk = k * k;
  const T* G = reinterpret_cast<const T*>(Gall) + (long long)b * kk;
  T* Rinv = reinterpret_cast<T*>(Rinv_all) + (long long)b * kk;
  T* Racc = Racc_all ? reinterpret_cast<T*>(Racc_all) + (long long)b * kk : nullptr;
  int f = flags[b];

  auto write_identity = [&]() {
    for (int e = tid; e < kk; e += kCholThreads) {
      const int r = e / k;
      const T v = (e - r * k == r) ? S<CPLX>::one() : S<CPLX>::zero();
      Rinv[e] = v;
      if (r_only && Racc) Racc[e] = v;
    }
  };
  if (pass == 3 && !(f & FLAG_THIRD_PASS)) {
    write_identity();
    return;
  }
  if (pass == 1) f = 0;

  // trace of G for the shift
  double tr = 0.0;
  for (int i = tid; i < k; i += kCholThreads) tr += S<CPLX>::re(G[i * k + i]);
  tr = wave_sum(tr);
  if (lane == 0) red[wave] = tr;
  __syncthreads();
  tr = 0.0;
  for (int w = 0; w < kCholWaves; ++w) tr += red[w];
  // shifted CholeskyQR: s = 11 (n k + k (k + 1)) u ||Y||^2, with ||Y||_2^2 <= trace(G)
  const double shift = 11.0 * ((double)n_rows * k + (double)k * (k + 1)) * 0x1p-53 * tr;

  // the lane's columns (the second one when k > 64: TWO), clamped for reads
  const int c0 = lane, c1 = lane + 64;
  const int c0r = min(c0, k - 1), c1r = min(c1, k - 1);
  bool ok = false;
  for (int attempt = 0; attempt < 2; ++attempt) {
    // upper triangle of G (+ shift), zero strict lower triangle (M = I)
    for (int e = tid; e < kk; e += kCholThreads) {
      const int i = e / k, c = e - i * k;
      T v = c >= i ? G[e] : S<CPLX>::zero();
      if (attempt == 1 && c == i) {
        if constexpr (CPLX) v.re += shift; else v += shift;
      }
      A[e] = v;
    }
    __syncthreads();
    ok = true;
    for (int j = 0; j < k; ++j) {
      const T* Aj = A + j * k;
      // Every load of the step is issued before the first use (one LDS round
      // trip): the pivot, row j at the lane's columns, and the first batch of
      // this wavefront's rows i > j, i % kCholWaves == wave.  A batch has a
      // fixed length: rows past the end are clamped for reads and their
      // results go to the lane's spare slot, so the only branch is the
      // wavefront-uniform one that skips an empty batch.
      const int r0 = j + 1 + ((wv - (j + 1)) & (kCholWaves - 1));
      T aji[kB], a0[kB], a1[kB];
      auto load_batch = [&](int i0) {
#pragma unroll
        for (int q = 0; q < kB; ++q) {
          const int i = min(i0 + kCholWaves * q, k - 1);
          aji[q] = Aj[i];
          a0[q] = A[i * k + c0r];
          if constexpr (TWO) a1[q] = A[i * k + c1r];
        }
      };
      const double d = S<CPLX>::re(Aj[j]);  // same value in every thread
      T ajc0 = Aj[c0r], ajc1 = TWO ? Aj[c1r] : S<CPLX>::zero();
      if (r0 < k) load_batch(r0);
      // row j at the lane's columns; M[j, j] = 1
      if (c0 == j) ajc0 = S<CPLX>::one();
      if (c1 == j) ajc1 = S<CPLX>::one();
      if (!(d > 0.0) || !isfinite(d)) {
        ok = false;
        break;
      }
      if (tid == 0) dg[j] = d;
      const double invd = 1.0 / d;
      // last row that updates column c: every row for an M column (c <= j),
      // rows up to c for a U column (c >= i), none past the end
      const int hi0 = c0 >= k ? -1 : (c0 <= j ? k - 1 : c0);
      const int hi1 = c1 >= k ? -1 : (c1 <= j ? k - 1 : c1);
      for (int i0 = r0; i0 < k;) {
#pragma unroll
        for (int q = 0; q < kB; ++q) {
          const int i = i0 + kCholWaves * q;
          // multiplier of row i: conj(A[j, i]) / d_j
          const T mu = S<CPLX>::scale(S<CPLX>::conj(aji[q]), invd);
          A[i <= hi0 ? i * k + c0 : kk + lane] = S<CPLX>::sub(a0[q], S<CPLX>::mul(mu, ajc0));
          if constexpr (TWO) A[i <= hi1 ? i * k + c1 : kk + lane] = S<CPLX>::sub(a1[q], S<CPLX>::mul(mu, ajc1));
        }
        i0 += kCholWaves * kB;
        if (i0 < k) load_batch(i0);
      }
      __syncthreads();
    }
    if (ok) {
      // conditioning estimate from the diagonal of R
      double mn = 1e300, mx = 0;
      for (int i = 0; i < k; ++i) {
        mn = fmin(mn, dg[i]);
        mx = fmax(mx, dg[i]);
      }
      const bool illcond = sqrt(mn) < 1e-7 * sqrt(mx);
      if (attempt == 0 && illcond && pass == 1) {
        f |= FLAG_THIRD_PASS;
        __syncthreads();
        continue;  // redo with the shift
      }
      // the first pass's output is still this ill-conditioned: the sketch is
      // numerically rank-deficient (condition number beyond about 1e13)
      if (attempt == 0 && illcond && pass == 2) f |= FLAG_RANK_DEFICIENT;
      break;
    }
    f |= FLAG_THIRD_PASS;
    // or the Gram of the first pass's output breaks down
    if (attempt == 0 && pass == 2) f |= FLAG_RANK_DEFICIENT;
    __syncthreads();
  }
  if (!ok) {
    f |= FLAG_NUMERIC;
    write_identity();
    if (tid == 0) flags[b] = f;
    return;
  }
  for (int i = tid; i < k; i += kCholThreads) {
    sq[i] = sqrt(dg[i]);
    rs[i] = 1.0 / sqrt(dg[i]);
  }
  __syncthreads();
  // R[i, l] = U[i, l] / sqrt(d_i) (l >= i), R^-1[a, c] = conj(M[c, a]) / sqrt(d_c) (a <= c)
  auto R_at = [&](int i, int l) -> T {
    if (l < i) return S<CPLX>::zero();
    return l == i ? S<CPLX>::scale(S<CPLX>::one(), sq[i]) : S<CPLX>::scale(A[i * k + l], rs[i]);
  };
  // Racc <- R (pass 1, or r_only) or R * Racc (later passes; staged through Rinv)
  if (Racc) {
    if (pass == 1 || r_only) {
      for (int e = tid; e < kk; e += kCholThreads) {
        const int i = e / k;
        Racc[e] = R_at(i, e - i * k);
      }
    } else {
      for (int e = tid; e < kk; e += kCholThreads) {
        const int i = e / k, l = e - i * k;
        T sacc = S<CPLX>::zero();
        for (int t = i; t <= l; ++t) sacc = S<CPLX>::add(sacc, S<CPLX>::mul(R_at(i, t), Racc[t * k + l]));
        Rinv[e] = sacc;
      }
      __syncthreads();
      for (int e = tid; e < kk; e += kCholThreads) Racc[e] = Rinv[e];
      __syncthreads();
    }
  }
  for (int e = tid; e < kk; e += kCholThreads) {
    const int a = e / k, c = e - a * k;
    T v = S<CPLX>::zero();
    if (c == a) v = S<CPLX>::scale(S<CPLX>::one(), rs[a]);
    else if (c > a) v = S<CPLX>::scale(S<CPLX>::conj(A[c * k + a]), rs[c]);
    Rinv[e] = v;
  }
  if (tid == 0) flags[b] = f;
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD of K = Racc^H, columns rotated in the
// parallel round-robin (circle) order.  A group of 16 lanes owns one column
// pair of a round (lane i holds rows i, i + 16, ... of both columns), so a
// wavefront rotates four pairs with the same instructions and the three inner
// products of a pair are row-local DPP sums; the workgroup has one wavefront
// per four pairs and one barrier per round.  (Every wavefront instruction
// occupies its SIMD for four cycles: the rotation arithmetic, identical in
// all lanes of a group, is shared by four pairs instead of repeated per pair.)
// ROWS = ceil(k / 16) rows per lane (k <= 16 ROWS).
constexpr int kJacMaxThreads = 1024;  // 64 pairs (k <= 128) / 4 per wavefront

template <bool CPLX, int ROWS>
__global__ __launch_bounds__(kJacMaxThreads) void jacobi_kernel(const double* Racc_all, int k, int max_sweeps,
                                                                double* Z_all, double* sigma_all,
                                                                double* inv_sigma_all, double* inv_sigma1,
                                                                double* log_scale, int* stats) {
  using T = typename S<CPLX>::T;
  extern __shared__ double smem[];
  const int n = (k + 1) / 2 * 2;  // even number of columns (one zero column if k is odd)
  T* Kc = reinterpret_cast<T*>(smem);  // column-major: Kc[c * k + r]
  __shared__ int rotated, chk;
  __shared__ int perm[128];
  __shared__ double nrm[128];
  const int b = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int kk = k * k;
  const T* R = reinterpret_cast<const T*>(Racc_all) + (long long)b * kk;
  // column c of K = R^H is the conjugated row c of R
  for (int e = tid; e < n * k; e += nt) {
    const int c = e / k, r = e - c * k;
    Kc[e] = (c < k) ? S<CPLX>::conj(R[c * k + r]) : S<CPLX>::zero();
  }
  __syncthreads();
  const int wave = tid >> 6, lane = tid & 63, nw = nt >> 6;
  const int li = lane & 15;
  const int npairs = n / 2;
  const int pair = tid >> 4;  // lane group = column pair of the round
  const bool active = pair < npairs;
  const double tol = sqrt((double)k) * 0x1p-52;
  const double tol2 = tol * tol;
  int sweep = 0;
  bool converged = false;
  for (sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < n - 1; ++round) {
      // circle method: position 0 fixed, the others rotate ((pos - 1 + round)
      // mod (n - 1) by one conditional subtraction: both terms are < n - 1)
      auto at = [&](int pos) {
        int t = pos - 1 + round;
        t -= t >= n - 1 ? n - 1 : 0;
        return pos == 0 ? 0 : 1 + t;
      };
      const int ca = active ? at(pair) : 0, cb = active ? at(n - 1 - pair) : 0;
      T* xc = Kc + ca * k;
      T* yc = Kc + cb * k;
      T x[ROWS], y[ROWS];
      double a2 = 0, b2 = 0, gr = 0, gi = 0;
#pragma unroll
      for (int h = 0; h < ROWS; ++h) {
        const int r = li + 16 * h;
        const bool in = active && r < k;
        x[h] = in ? xc[r] : S<CPLX>::zero();
        y[h] = in ? yc[r] : S<CPLX>::zero();
        a2 += S<CPLX>::abs2(x[h]);
        b2 += S<CPLX>::abs2(y[h]);
        if constexpr (CPLX) {
          const cd g = cmul(cconj(x[h]), y[h]);
          gr += g.re;
          gi += g.im;
        } else {
          gr += x[h] * y[h];
        }
      }
      a2 = row_sum16(a2);
      b2 = row_sum16(b2);
      gr = row_sum16(gr);
      if constexpr (CPLX) gi = row_sum16(gi);
      const double g2 = gr * gr + gi * gi;
      if (active && a2 > 0 && b2 > 0 && g2 > tol2 * a2 * b2) {
        // The rotation angle (|theta| <= pi/4, tan 2 theta = 2 |gamma| / dl,
        // dl = b2 - a2) by reciprocal square roots, no division: with
        // r = (dl^2 + 4 |gamma|^2)^-1/2, cos 2 theta = |dl| r and
        // u = (2 + 2 cos 2 theta)^-1/2, cos theta = (1 + cos 2 theta) u and
        // sin theta = sign(dl) 2 |gamma| r u.
        const double dl = b2 - a2;
        const double r = rsqrt(dl * dl + 4.0 * g2);
        const double C2 = fabs(dl) * r;
        const double u = rsqrt(2.0 + 2.0 * C2);
        const double c = (1.0 + C2) * u;
        const double inv_ga = CPLX ? rsqrt(g2) : 1.0;
        const double s = (dl >= 0 ? 2.0 : -2.0) * r * u * (CPLX ? g2 * inv_ga : fabs(gr));
        // y~ = conj(e) y with e = gamma / |gamma|, then a real rotation of (x, y~)
        const double er = CPLX ? gr * inv_ga : (gr >= 0 ? 1.0 : -1.0), ei = gi * inv_ga;
#pragma unroll
        for (int h = 0; h < ROWS; ++h) {
          const int r = li + 16 * h;
          if (r < k) {
            const T xv = x[h];
            if constexpr (CPLX) {
              const T yv = y[h];
              const T yt = {er * yv.re + ei * yv.im, er * yv.im - ei * yv.re};
              xc[r] = {c * xv.re - s * yt.re, c * xv.im - s * yt.im};
              yc[r] = {s * xv.re + c * yt.re, s * xv.im + c * yt.im};
            } else {
              const T yt = er * y[h];
              xc[r] = c * xv - s * yt;
              yc[r] = s * xv + c * yt;
            }
          }
        }
        if (li == 0) atomicAdd(&rotated, 1);
      }
      __syncthreads();
    }
    const int nrot = rotated;
    if (nrot == 0) {
      converged = true;
      ++sweep;
      break;
    }
    __syncthreads();
    if (nrot <= k && k <= 64) {
      // Few rotations left: test every pair against the rotation threshold
      // in one pass (counted as the confirming sweep) instead of a sweep of
      // n - 1 rounds that would find none to rotate (no column changes in
      // such a sweep, so it makes exactly these tests).  Above k = 64 the
      // pass (one pair per thread, k rows each) costs more than it saves.
      if (tid == 0) chk = 0;
      __syncthreads();
      for (int pq = tid; pq < k * (k - 1) / 2; pq += nt) {
        int ca = 0, rem = pq;
        while (rem >= k - 1 - ca) {
          rem -= k - 1 - ca;
          ++ca;
        }
        const int cb = ca + 1 + rem;
        const T* xc = Kc + ca * k;
        const T* yc = Kc + cb * k;
        double a2 = 0, b2 = 0, gr = 0, gi = 0;
        for (int r = 0; r < k; ++r) {
          const T x = xc[r], y = yc[r];
          a2 += S<CPLX>::abs2(x);
          b2 += S<CPLX>::abs2(y);
          if constexpr (CPLX) {
            const cd g = cmul(cconj(x), y);
            gr += g.re;
            gi += g.im;
          } else {
            gr += x * y;
          }
        }
        if (a2 > 0 && b2 > 0 && gr * gr + gi * gi > tol2 * a2 * b2) chk = 1;
      }
      __syncthreads();
      if (chk == 0) {
        converged = true;
        sweep += 2;
        break;
      }
    }
  }
  // singular values = column norms; sort descending (stable in column index)
  for (int c = wave; c < k; c += nw) {
    double a2 = 0;
    for (int r = lane; r < k; r += 64) a2 += S<CPLX>::abs2(Kc[c * k + r]);
    a2 = wave_sum(a2);
    if (lane == 0) nrm[c] = sqrt(a2);
  }
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < k; ++i) perm[i] = i;
    for (int i = 1; i < k; ++i) {
      const int v = perm[i];
      int j = i - 1;
      while (j >= 0 && nrm[perm[j]] < nrm[v]) {
        perm[j + 1] = perm[j];
        --j;
      }
      perm[j + 1] = v;
    }
  }
  __syncthreads();
  T* Z = reinterpret_cast<T*>(Z_all) + (long long)b * kk;
  for (int e = tid; e < kk; e += nt) {
    const int r = e / k, i = e - r * k;
    const int c = perm[i];
    const double s = nrm[c];
    Z[e] = s > 0 ? S<CPLX>::scale(Kc[c * k + r], 1.0 / s) : S<CPLX>::zero();
  }
  for (int i = tid; i < k; i += nt) {
    const double s = nrm[perm[i]];
    sigma_all[(long long)b * k + i] = s;
    inv_sigma_all[(long long)b * k + i] = s > 0 ? 1.0 / s : 0.0;
  }
  if (tid == 0) {
    const double s1 = nrm[perm[0]];
    inv_sigma1[b] = s1 > 0 ? 1.0 / s1 : 0.0;
    if (log_scale) log_scale[b] += log(s1);
    stats[b] = converged ? sweep : -sweep;
  }
}

// ---------------------------------------------------------------------------
// Small kernels of the einsumsvd adjoint (one workgroup per instance)

// G1^H for the truncated-SVD backward of M = Z Sigma V^H (k x k per instance):
//   C = (F o (ZZ - ZZ^H)) S + S (F o (VV - VV^H)) + diag(sbar + i Im(ZZ_ii) / s_i)
//   G1 = C - S^-1 VV^H,   F_ij = d / (d^2 + eps s_1^4), d = s_j^2 - s_i^2
// (F_ij = 0 where d = 0, and on the diagonal) with ZZ = Z^H Zbar, VV = V^H Vbar:
// eps is a width relative to the largest singular value (scale invariant).
template <bool CPLX>
__global__ void svd_bwd_core_kernel(const double* ZZall, const double* VVall, const double* sall,
                                    const double* sball, int k, double eps, double* G1Hall) {
  using T = typename S<CPLX>::T;
  const int b = blockIdx.x;
  const long long kk = (long long)k * k;
  const T* ZZ = reinterpret_cast<const T*>(ZZall) + b * kk;
  const T* VV = reinterpret_cast<const T*>(VVall) + b * kk;
  const double* s = sall + (long long)b * k;
  const double* sb = sball + (long long)b * k;
  T* G1H = reinterpret_cast<T*>(G1Hall) + b * kk;
  const double w = eps * (s[0] * s[0]) * (s[0] * s[0]);
  for (long long e = threadIdx.x; e < kk; e += blockDim.x) {
    const int i = (int)(e / k), j = (int)(e % k);
    const double dd = s[j] * s[j] - s[i] * s[i];
    const double F = (i == j || dd == 0.0) ? 0.0 : dd / (dd * dd + w);
    const double inv_si = s[i] > 0 ? 1.0 / s[i] : 0.0;
    T c = S<CPLX>::add(S<CPLX>::scale(S<CPLX>::sub(ZZ[e], S<CPLX>::conj(ZZ[(long long)j * k + i])), F * s[j]),
                       S<CPLX>::scale(S<CPLX>::sub(VV[e], S<CPLX>::conj(VV[(long long)j * k + i])), F * s[i]));
    if (i == j) {
      if constexpr (CPLX) {
        c.re += sb[i];
        c.im += ZZ[e].im * inv_si;
      } else {
        c += sb[i];
      }
    }
    const T g = S<CPLX>::sub(c, S<CPLX>::scale(S<CPLX>::conj(VV[(long long)j * k + i]), inv_si));
    G1H[(long long)j * k + i] = S<CPLX>::conj(g);
  }
}

// M <- tril(-M, -1) + tril(-M, -1)^H - Re diag(M) (in place; the strict upper
// part is overwritten).  The real diagonal is the QR backward's for R with a
// real positive diagonal: Q^H dQ then has an imaginary diagonal that the
// loss only sees through phases, which the R gauge fixes.
template <bool CPLX>
__global__ void copyltu_neg_kernel(double* Mall, int k) {
  using T = typename S<CPLX>::T;
  T* M = reinterpret_cast<T*>(Mall) + (long long)blockIdx.x * k * k;
  for (long long e = threadIdx.x; e < (long long)k * k; e += blockDim.x) {
    const int i = (int)(e / k), j = (int)(e % k);
    if (j > i) continue;
    T v = S<CPLX>::sub(S<CPLX>::zero(), M[e]);
    if constexpr (CPLX) {
      if (i == j) v.im = 0.0;
    }
    M[e] = v;
    if (j < i) M[(long long)j * k + i] = S<CPLX>::conj(v);
  }
}

// y += alpha x over n doubles
__global__ void axpy_kernel(double* y, const double* x, double alpha, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] += alpha * x[i];
}

// Y[r, i] += X[r, i] * d[i] (rows x k per instance, d: k per instance)
template <bool CPLX>
__global__ void axpy_colscale_kernel(double* Yall, const double* Xall, const double* dall, long long rows, int k) {
  using T = typename S<CPLX>::T;
  const int b = blockIdx.y;
  T* Y = reinterpret_cast<T*>(Yall) + b * rows * k;
  const T* X = reinterpret_cast<const T*>(Xall) + b * rows * k;
  const double* d = dall + (long long)b * k;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < rows * k; e += (long long)gridDim.x * blockDim.x)
    Y[e] = S<CPLX>::add(Y[e], S<CPLX>::scale(X[e], d[e % k]));
}

// Vbar[c, i] = conj(dR[i, c]) * (s ? s[i] : 1) * (rs ? rs[b] : 1) for i < mp,
// 0 for mp <= i < k
template <bool CPLX>
__global__ void vbar_kernel(const double* dRall, const double* sall, const double* rs, long long cols, int mp,
                            int k, double* Vall) {
  using T = typename S<CPLX>::T;
  const int b = blockIdx.y;
  const T* dR = reinterpret_cast<const T*>(dRall) + b * (long long)mp * cols;
  T* Vb = reinterpret_cast<T*>(Vall) + b * cols * k;
  const double f = rs ? rs[b] : 1.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < cols * k; e += (long long)gridDim.x * blockDim.x) {
    const long long c = e / k;
    const int i = (int)(e % k);
    T v = S<CPLX>::zero();
    if (i < mp)
      v = S<CPLX>::scale(S<CPLX>::conj(dR[(long long)i * cols + c]), (sall ? sall[(long long)b * k + i] : 1.0) * f);
    Vb[e] = v;
  }
}

// sbar[i] = dsigma[i] (+ rs Re sum_c dR[i, c] V[c, i] when right) for i < mp, 0 beyond
template <bool CPLX>
__global__ void sbar_kernel(const double* dsall, const double* dRall, const double* Vall, const double* rs,
                            long long cols, int mp, int k, int right, double* sball) {
  using T = typename S<CPLX>::T;
  __shared__ double red[4];
  const int b = blockIdx.x, tid = threadIdx.x;
  const T* dR = reinterpret_cast<const T*>(dRall) + b * (long long)mp * cols;
  const T* V = reinterpret_cast<const T*>(Vall) + b * cols * k;
  const double f = rs ? rs[b] : 1.0;
  for (int i = 0; i < k; ++i) {
    double acc = 0.0;
    if (right && i < mp)
      for (long long c = tid; c < cols; c += blockDim.x) acc += S<CPLX>::re(S<CPLX>::mul(dR[(long long)i * cols + c], V[c * k + i]));
    acc = wave_sum(acc);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
      sball[(long long)b * k + i] = i < mp ? (dsall ? dsall[(long long)b * mp + i] : 0.0) + f * t : 0.0;
    }
    __syncthreads();
  }
}

// Derivative of the canonical phase choice (complex only).  For each kept
// pair i the output U[:, i] = U0[:, i] e^{-i th} and R[i, :] = e^{i th} R0[i, :]
// with th = arg(w . U0[:, i]); at the fixed point z = w . U[:, i] is real
// positive.  The loss sees th through
//   thbar = Im <dU_i, U_i> - Im <dR_i, R_i>,   R[i, c] = sc_i conj(V[c, i]),
// and th through z: dU[:, i] += w * (i thbar / z).  sc_i = (s ? s_i : 1) * (rs ? rs : 1).
// dU, U: rows x mp; dR: mp x cols; V: cols x k (row-major per instance).
__global__ __launch_bounds__(256) void gauge_bwd_kernel(double* dUall, const double* Uall, const double* dRall,
                                                        const double* Vall, const double* sall, const double* rs,
                                                        long long rows, long long cols, int mp, int k) {
  using T = S<true>::T;
  const int b = blockIdx.x, tid = threadIdx.x;
  T* dU = reinterpret_cast<T*>(dUall) + (long long)b * rows * mp;
  const T* U = reinterpret_cast<const T*>(Uall) + (long long)b * rows * mp;
  const T* dR = reinterpret_cast<const T*>(dRall) + (long long)b * mp * cols;
  const T* V = reinterpret_cast<const T*>(Vall) + (long long)b * cols * k;
  __shared__ double r0[256], r1[256], r2[256];
  __shared__ double coef;
  const uint64_t base = mix64(mix64(0ull) + 0ull);
  const double f = rs ? rs[b] : 1.0;
  for (int i = 0; i < mp; ++i) {
    double a = 0.0, zr = 0.0, bb = 0.0;
    for (long long r = tid; r < rows; r += blockDim.x) {
      const uint64_t h = mix64(base + (uint64_t)(r + 1) * 0x9E3779B97F4A7C15ull);
      const double w = 2.0 * (double)(h >> 11) * 0x1p-53 - 1.0;
      const T u = U[r * mp + i], du = dU[r * mp + i];
      a += du.re * u.im - du.im * u.re;  // Im(conj(du) u)
      zr += w * u.re;
    }
    for (long long c = tid; c < cols; c += blockDim.x) {
      const T x = S<true>::mul(dR[(long long)i * cols + c], V[c * k + i]);
      bb += x.im;
    }
    r0[tid] = a;
    r1[tid] = zr;
    r2[tid] = bb;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
      if (tid < st) {
        r0[tid] += r0[tid + st];
        r1[tid] += r1[tid + st];
        r2[tid] += r2[tid + st];
      }
      __syncthreads();
    }
    if (tid == 0) {
      const double sc = (sall ? sall[(long long)b * k + i] : 1.0) * f;
      // Im <dR_i, R_i> = Im sum conj(dR) sc conj(V) = -sc Im sum dR V
      const double thbar = r0[0] + sc * r2[0];
      coef = r1[0] > 0.0 ? thbar / r1[0] : 0.0;
    }
    __syncthreads();
    const double cf = coef;
    for (long long r = tid; r < rows; r += blockDim.x) {
      const uint64_t h = mix64(base + (uint64_t)(r + 1) * 0x9E3779B97F4A7C15ull);
      const double w = 2.0 * (double)(h >> 11) * 0x1p-53 - 1.0;
      dU[r * mp + i].im += w * cf;
    }
    __syncthreads();
  }
}

// dst[b][r * ncols + c] = src[b * sSrc + rowmap(r) + colmap(c)] (row-major
// mode nesting in both maps: the last mode varies fastest)
struct Map2D {
  int nr = 0, nc = 0;
  long long rd[kMaxModes], rst[kMaxModes], cd[kMaxModes], cst[kMaxModes];
};

__device__ inline long long map_offset(long long idx, int n, const long long* dims, const long long* str) {
  long long off = 0;
  for (int t = n - 1; t >= 0; --t) {
    const long long q = idx / dims[t];
    off += (idx - q * dims[t]) * str[t];
    idx = q;
  }
  return off;
}

template <bool CPLX>
__global__ void gather2d_kernel(const double* srcall, long long sSrc, Map2D m, long long rows, long long cols,
                                double* dstall) {
  using T = typename S<CPLX>::T;
  const int b = blockIdx.y;
  const T* src = reinterpret_cast<const T*>(srcall) + b * sSrc;
  T* dst = reinterpret_cast<T*>(dstall) + b * rows * cols;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < rows * cols; e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / cols, c = e - r * cols;
    dst[e] = src[map_offset(r, m.nr, m.rd, m.rst) + map_offset(c, m.nc, m.cd, m.cst)];
  }
}

__global__ void sqrt_pair_kernel(const double* s, long long n, double* sq, double* isq) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double r = sqrt(fmax(s[i], 0.0));
    sq[i] = r;
    isq[i] = r > 0 ? 1.0 / r : 0.0;
  }
}

__global__ void f64_to_bf16_kernel(const double* in, __bf16* out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = (__bf16)in[i];
}

__global__ void f64_to_f32_kernel(const double* in, float* out, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

// Frobenius norm per batch instance, safe against underflow and overflow:
// pass 1 finds max|x| (block partials, then a finalize), pass 2 sums
// (x / max)^2; norm = max * sqrt(sum).
__global__ void absmax_partial_kernel(const double* x, long long n, double* part) {
  const int b = blockIdx.y;
  const double* xb = x + (long long)b * n;
  double s = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    s = fmax(s, fabs(xb[i]));
  __shared__ double red[16];
  for (int o = 32; o > 0; o >>= 1) s = fmax(s, __shfl_xor(s, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) t = fmax(t, red[w]);
    part[(long long)b * gridDim.x + blockIdx.x] = t;
  }
}

__global__ void absmax_finalize_kernel(const double* part, int nparts, double* mx) {
  const int b = blockIdx.x;
  if (threadIdx.x == 0) {
    double t = 0;
    for (int i = 0; i < nparts; ++i) t = fmax(t, part[(long long)b * nparts + i]);
    mx[b] = t;
  }
}

__global__ void sumsq_partial_kernel(const double* x, long long n, const double* mx, double* part) {
  const int b = blockIdx.y;
  const double* xb = x + (long long)b * n;
  const double f = mx[b] > 0 ? 1.0 / mx[b] : 1.0;
  double s = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double v = xb[i] * f;
    s += v * v;
  }
  __shared__ double red[16];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) t += red[w];
    part[(long long)b * gridDim.x + blockIdx.x] = t;
  }
}

// inv_norm[b] holds 1/max on entry (scale of the sums); writes 1/norm
__global__ void norm_finalize_kernel(const double* part, int nparts, const double* mx, double* inv_norm,
                                     double* log_scale) {
  const int b = blockIdx.x;
  if (threadIdx.x == 0) {
    double t = 0;
    for (int i = 0; i < nparts; ++i) t += part[(long long)b * nparts + i];
    const double m = mx[b];
    if (m > 0 && t > 0) {
      // 1/norm = (1/m) / sqrt(t), computed without forming m * sqrt(t)
      inv_norm[b] = (1.0 / m) / sqrt(t);
      if (log_scale) log_scale[b] += log(m) + 0.5 * log(t);
    } else {
      inv_norm[b] = 1.0;
    }
  }
}

__global__ void scale_kernel(double* x, long long n, const double* s) {
  const int b = blockIdx.y;
  double* xb = x + (long long)b * n;
  const double f = s[b];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    xb[i] *= f;
}

__global__ void copy_sigma_kernel(const double* sk, int k, int mp, int batch, double* out) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < batch * mp; t += gridDim.x * blockDim.x) {
    const int b = t / mp, i = t % mp;
    out[t] = sk[(long long)b * k + i];
  }
}

// Diagnostics of a batch (third CholeskyQR passes, non-finite factors, the
// largest Jacobi sweep count, capped sweeps, Householder fallbacks): per-thread partials over the
// instances, one block reduction, one update of acc (integers: exact and
// independent of the order).
constexpr int kStatsThreads = 256;
__global__ __launch_bounds__(kStatsThreads) void stats_kernel(const int* flags, const int* sweeps, int batch,
                                                              int* acc) {
  __shared__ int part[5][kStatsThreads];
  const int tid = threadIdx.x;
  int third = 0, numeric = 0, smax = 0, capped = 0, house = 0;
  for (int b = tid; b < batch; b += kStatsThreads) {
    if (flags) {
      const int f = flags[b];
      third += (f & FLAG_THIRD_PASS) != 0;
      numeric += (f & FLAG_NUMERIC) != 0;
      house += (f & FLAG_HOUSEHOLDER) != 0;
    }
    if (sweeps) {
      const int sw = sweeps[b];
      smax = max(smax, sw < 0 ? -sw : sw);
      capped += sw < 0;
    }
  }
  part[0][tid] = third;
  part[1][tid] = numeric;
  part[2][tid] = smax;
  part[3][tid] = capped;
  part[4][tid] = house;
  __syncthreads();
  for (int st = kStatsThreads / 2; st > 0; st >>= 1) {
    if (tid < st) {
      part[0][tid] += part[0][tid + st];
      part[1][tid] += part[1][tid + st];
      part[2][tid] = max(part[2][tid], part[2][tid + st]);
      part[3][tid] += part[3][tid + st];
      part[4][tid] += part[4][tid + st];
    }
    __syncthreads();
  }
  if (tid == 0) {
    acc[0] += part[0][0];
    acc[2] += part[1][0];
    acc[1] = max(acc[1], part[2][0]);
    acc[3] += part[3][0];
    acc[4] += part[4][0];
  }
}

size_t small_lds_bytes(int k, bool cplx) { return (size_t)k * k * (cplx ? 16 : 8); }

__global__ void fill_value_kernel(double* p, long long n, double v, int cplx) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    if (cplx) {
      p[2 * i] = v;
      p[2 * i + 1] = 0.0;
    } else {
      p[i] = v;
    }
  }
}

// Canonical phase of the singular vectors: for each column i < mp of the
// left factor U = P Z (row-major rows x mp), the projection z = w . U[:, i]
// on the fixed vector w (the sketch generator's values for seed 0, stream 0,
// one column) is made real positive by rotating column i of Z by
// conj(z)/|z|.  A projection on a generic vector is immune to the exact
// magnitude ties that the ket/bra symmetry of <psi|psi> networks creates
// between entries.
//
// Pass 1 spreads the rows over the chip: block (c, b) takes rows
// [c kGaugeRows, (c + 1) kGaugeRows) of instance b, forms w for them once in
// LDS, and accumulates w_r U[r, i] with threads on consecutive columns of a
// row (coalesced), two rows at a time; its sums per column go to
// part[b][c][i].  Pass 2 adds the chunks in order (deterministic) and
// applies the phases to Z.
constexpr int kGaugeRows = 256;

template <bool CPLX>
__global__ __launch_bounds__(256) void gauge_partial_kernel(const double* Uall, long long rows, int mp,
                                                            int nchunks, double* part) {
  using T = typename S<CPLX>::T;
  const int c = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
  const T* U = reinterpret_cast<const T*>(Uall) + (long long)b * rows * mp;
  __shared__ double w[kGaugeRows];
  __shared__ double acc[2][128][2];
  const long long r0 = (long long)c * kGaugeRows;
  const uint64_t base = mix64(mix64(0ull) + 0ull);
  {
    const long long r = r0 + tid;
    const uint64_t h = mix64(base + (uint64_t)(r + 1) * 0x9E3779B97F4A7C15ull);
    w[tid] = 2.0 * (double)(h >> 11) * 0x1p-53 - 1.0;
  }
  __syncthreads();
  const int i = tid & 127, half = tid >> 7;
  double zr = 0.0, zi = 0.0;
  if (i < mp) {
    const long long rend = min(rows, r0 + kGaugeRows);
    for (long long r = r0 + half; r < rend; r += 2) {
      const double wr = w[r - r0];
      const T u = U[r * mp + i];
      if constexpr (CPLX) {
        zr += wr * u.re;
        zi += wr * u.im;
      } else {
        zr += wr * u;
      }
    }
  }
  acc[half][i][0] = zr;
  acc[half][i][1] = zi;
  __syncthreads();
  if (tid < mp) {
    double* o = part + (((long long)b * nchunks + c) * mp + tid) * 2;
    o[0] = acc[0][tid][0] + acc[1][tid][0];
    o[1] = acc[0][tid][1] + acc[1][tid][1];
  }
}

template <bool CPLX>
__global__ __launch_bounds__(256) void gauge_apply_kernel(const double* part, int nchunks, int mp, double* Zall,
                                                          int k) {
  using T = typename S<CPLX>::T;
  const int b = blockIdx.x, tid = threadIdx.x;
  T* Z = reinterpret_cast<T*>(Zall) + (long long)b * k * k;
  __shared__ T phase[128];  // mp <= k <= 128
  if (tid < mp) {
    double zr = 0.0, zi = 0.0;
    for (int c = 0; c < nchunks; ++c) {
      const double* o = part + (((long long)b * nchunks + c) * mp + tid) * 2;
      zr += o[0];
      zi += o[1];
    }
    if constexpr (CPLX) {
      const double m = sqrt(zr * zr + zi * zi);
      phase[tid] = m > 0 ? T{zr / m, -zi / m} : T{1.0, 0.0};  // conj(z)/|z|
    } else {
      phase[tid] = zr < 0 ? -1.0 : 1.0;
    }
  }
  __syncthreads();
  for (int e = tid; e < k * mp; e += 256) {
    const int r = e / mp, i = e - r * mp;
    Z[(long long)r * k + i] = S<CPLX>::mul(Z[(long long)r * k + i], phase[i]);
  }
}

__global__ void copy_scalar_kernel(const double* src, int cplx, double* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    dst[0] = src[0];
    dst[1] = cplx ? src[1] : 0.0;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers

void sketch(Ctx& ctx, void* out, bool f32, int64_t n, int64_t k, int batch, uint64_t seed,
            uint64_t stream_id, bool cplx_out) {
  const long long nk = (long long)n * k;
  dim3 grid((unsigned)std::min<long long>(cdiv(nk, 256), 2048), (unsigned)batch);
  HP_REQUIRE(!(f32 && cplx_out), HPEPS_ERR_DTYPE, "complex sketches are FP64");
  if (f32)
    sketch_kernel<float><<<grid, 256, 0, ctx.stream>>>((float*)out, nk, seed, stream_id, 1);
  else
    sketch_kernel<double><<<grid, 256, 0, ctx.stream>>>((double*)out, nk, seed, stream_id, cplx_out ? 2 : 1);
  HP_CHECK_HIP(hipGetLastError());
}

void gram(Ctx& ctx, bool cplx, const void* Y, int64_t n, int64_t k, int batch, double* G,
          const int* active) {
  GemmDesc d;
  d.M = k;
  d.N = k;
  d.K = n;
  d.Am.add(k, 1);   // A = Y^H: row i -> column i of Y
  d.Ak.add(n, k);
  d.Bk.add(n, k);   // B = Y
  d.Bn.add(k, 1);
  d.Cm.add(k, k);
  d.Cn.add(k, 1);
  GemmCall c;
  c.A = Y;
  c.B = Y;
  c.C = G;
  c.sA = c.sB = n * k;
  c.sC = k * k;
  c.batch = batch;
  c.conjA = cplx;
  c.skip_if_zero = active;
  gemm(ctx, cplx ? Prec::C128 : Prec::F64, d, c);
}

void chol_inv(Ctx& ctx, bool cplx, const double* G, int64_t n_rows, int64_t k, int batch, int pass,
              double* Rinv, double* Racc, int* flags, bool r_only) {
  const size_t lds = chol_lds_bytes((int)k, cplx);
  HP_REQUIRE(k <= 128 && lds <= 160 * 1024 - 2048, HPEPS_ERR_UNSUPPORTED,
             "sketch width too large for the small factorizations (k <= 128, complex k <= 88)");
  const int rec = ctx.prof_begin("chol_inv");
  // kernels are launched by name (a launch through a pointer to the kernel
  // has run nothing, without an error, in host code built with
  // instrumentation); the tags carry the template arguments
  auto launch = [&](auto cplx_c, auto big_c) {
    constexpr bool C = decltype(cplx_c)::value, BIG = decltype(big_c)::value;
    HP_CHECK_HIP(hipFuncSetAttribute((const void*)&chol_inv_kernel<C, BIG>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    chol_inv_kernel<C, BIG><<<batch, kCholThreads, lds, ctx.stream>>>(G, n_rows, (int)k, pass, Rinv, Racc, flags,
                                                                      r_only ? 1 : 0);
  };
  using T = std::true_type;
  using F = std::false_type;
  if (cplx)
    k > 64 ? launch(T{}, T{}) : launch(T{}, F{});
  else
    k > 64 ? launch(F{}, T{}) : launch(F{}, F{});
  HP_CHECK_HIP(hipGetLastError());
  ctx.prof_end(rec, (double)batch * k * k * k / 3.0 * (cplx ? 4 : 1), 0.0);
}

void jacobi_svd(Ctx& ctx, bool cplx, const double* Racc, int64_t k, int batch, int max_sweeps,
                double* Z, double* sigma, double* inv_sigma, double* inv_sigma1, double* log_scale,
                int* stats) {
  HP_REQUIRE(k <= 128, HPEPS_ERR_UNSUPPORTED, "small SVD supports k <= 128");
  const int n = (int)((k + 1) / 2 * 2);
  // one wavefront per four column pairs
  const int threads = std::max(64, (n / 2 + 3) / 4 * 64);
  const size_t lds = (size_t)n * k * (cplx ? 16 : 8);
  HP_REQUIRE(lds <= 160 * 1024 - 2048, HPEPS_ERR_UNSUPPORTED, "small SVD too large for LDS");
  const int rec = ctx.prof_begin("jacobi_svd");
  struct EndRec {
    Ctx& c;
    int r;
    ~EndRec() {
      try {
        c.prof_end(r, 0.0, 0.0);
      } catch (...) {
      }
    }
  } end_rec{ctx, rec};
  // launched by name, never through a pointer to the kernel (the tags carry
  // the template arguments)
  auto launch = [&](auto cplx_c, auto rows_c) {
    constexpr bool C = decltype(cplx_c)::value;
    constexpr int RB = decltype(rows_c)::value;
    HP_CHECK_HIP(hipFuncSetAttribute((const void*)&jacobi_kernel<C, RB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds));
    jacobi_kernel<C, RB><<<batch, threads, lds, ctx.stream>>>(Racc, (int)k, max_sweeps, Z, sigma, inv_sigma,
                                                              inv_sigma1, log_scale, stats);
  };
  auto by_rows = [&](auto cplx_c) {
    switch ((k + 15) / 16) {
      case 1: launch(cplx_c, std::integral_constant<int, 1>{}); break;
      case 2: launch(cplx_c, std::integral_constant<int, 2>{}); break;
      case 3: launch(cplx_c, std::integral_constant<int, 3>{}); break;
      case 4: launch(cplx_c, std::integral_constant<int, 4>{}); break;
      case 5: launch(cplx_c, std::integral_constant<int, 5>{}); break;
      case 6: launch(cplx_c, std::integral_constant<int, 6>{}); break;
      case 7: launch(cplx_c, std::integral_constant<int, 7>{}); break;
      default: launch(cplx_c, std::integral_constant<int, 8>{}); break;
    }
  };
  if (cplx)
    by_rows(std::true_type{});
  else
    by_rows(std::false_type{});
  HP_CHECK_HIP(hipGetLastError());
}

void svd_bwd_core(Ctx& ctx, bool cplx, const double* ZZ, const double* VV, const double* s,
                  const double* sbar, int64_t k, int batch, double eps, double* G1H) {
  if (cplx)
    svd_bwd_core_kernel<true><<<batch, 256, 0, ctx.stream>>>(ZZ, VV, s, sbar, (int)k, eps, G1H);
  else
    svd_bwd_core_kernel<false><<<batch, 256, 0, ctx.stream>>>(ZZ, VV, s, sbar, (int)k, eps, G1H);
  HP_CHECK_HIP(hipGetLastError());
}

void copyltu_neg(Ctx& ctx, bool cplx, double* M, int64_t k, int batch) {
  if (cplx)
    copyltu_neg_kernel<true><<<batch, 256, 0, ctx.stream>>>(M, (int)k);
  else
    copyltu_neg_kernel<false><<<batch, 256, 0, ctx.stream>>>(M, (int)k);
  HP_CHECK_HIP(hipGetLastError());
}

void axpy(Ctx& ctx, double* y, const double* x, double alpha, int64_t n) {
  if (n <= 0) return;
  axpy_kernel<<<std::min<unsigned>(cdiv(n, 256), 4096), 256, 0, ctx.stream>>>(y, x, alpha, n);
  HP_CHECK_HIP(hipGetLastError());
}

void axpy_colscale(Ctx& ctx, bool cplx, double* Y, const double* X, const double* d, int64_t rows,
                   int64_t k, int batch) {
  dim3 grid(std::min<unsigned>(cdiv(rows * k, 256), 1024), batch);
  if (cplx)
    axpy_colscale_kernel<true><<<grid, 256, 0, ctx.stream>>>(Y, X, d, rows, (int)k);
  else
    axpy_colscale_kernel<false><<<grid, 256, 0, ctx.stream>>>(Y, X, d, rows, (int)k);
  HP_CHECK_HIP(hipGetLastError());
}

void vbar_from_dr(Ctx& ctx, bool cplx, const double* dR, const double* s, const double* rscale,
                  int64_t cols, int64_t mp, int64_t k, int batch, double* Vbar) {
  dim3 grid(std::min<unsigned>(cdiv(cols * k, 256), 1024), batch);
  if (cplx)
    vbar_kernel<true><<<grid, 256, 0, ctx.stream>>>(dR, s, rscale, cols, (int)mp, (int)k, Vbar);
  else
    vbar_kernel<false><<<grid, 256, 0, ctx.stream>>>(dR, s, rscale, cols, (int)mp, (int)k, Vbar);
  HP_CHECK_HIP(hipGetLastError());
}

void sigma_bar(Ctx& ctx, bool cplx, const double* dsigma, const double* dR, const double* V,
               const double* rscale, int64_t cols, int64_t mp, int64_t k, int batch, bool right,
               double* sbar) {
  if (cplx)
    sbar_kernel<true><<<batch, 256, 0, ctx.stream>>>(dsigma, dR, V, rscale, cols, (int)mp, (int)k, right, sbar);
  else
    sbar_kernel<false><<<batch, 256, 0, ctx.stream>>>(dsigma, dR, V, rscale, cols, (int)mp, (int)k, right, sbar);
  HP_CHECK_HIP(hipGetLastError());
}

void gauge_backward(Ctx& ctx, double* dU, const double* U, const double* dR, const double* V,
                    const double* s, const double* rscale, int64_t rows, int64_t cols, int64_t mp,
                    int64_t k, int batch) {
  gauge_bwd_kernel<<<batch, 256, 0, ctx.stream>>>(dU, U, dR, V, s, rscale, rows, cols, (int)mp, (int)k);
  HP_CHECK_HIP(hipGetLastError());
}

void gather2d(Ctx& ctx, bool cplx, const void* src, int64_t sSrc, const IndexMap& rows,
              const IndexMap& cols, void* dst, int batch) {
  Map2D m;
  m.nr = rows.n;
  m.nc = cols.n;
  for (int t = 0; t < rows.n; ++t) {
    m.rd[t] = rows.dim[t];
    m.rst[t] = rows.stride[t];
  }
  for (int t = 0; t < cols.n; ++t) {
    m.cd[t] = cols.dim[t];
    m.cst[t] = cols.stride[t];
  }
  const int64_t nr = rows.size(), nc = cols.size();
  if (nr * nc == 0) return;
  int64_t maxoff = 0;
  for (int t = 0; t < rows.n; ++t) maxoff += (rows.dim[t] - 1) * rows.stride[t];
  for (int t = 0; t < cols.n; ++t) maxoff += (cols.dim[t] - 1) * cols.stride[t];
  HP_REQUIRE(maxoff < sSrc, HPEPS_ERR_SHAPE, "gather out of bounds");
  dim3 grid(std::min<unsigned>(cdiv(nr * nc, 256), 1024), batch);
  if (cplx)
    gather2d_kernel<true><<<grid, 256, 0, ctx.stream>>>((const double*)src, sSrc, m, nr, nc, (double*)dst);
  else
    gather2d_kernel<false><<<grid, 256, 0, ctx.stream>>>((const double*)src, sSrc, m, nr, nc, (double*)dst);
  HP_CHECK_HIP(hipGetLastError());
}

namespace {
__global__ void identity_kernel(double* p, long long n, long long total, int es) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const long long r = (e / n) % n, c = e % n;
  p[e * es] = r == c ? 1.0 : 0.0;
  if (es == 2) p[e * es + 1] = 0.0;
}
}  // namespace

void fill_identity(Ctx& ctx, double* p, int64_t n, int batch, bool cplx) {
  const long long total = (long long)batch * n * n;
  identity_kernel<<<(unsigned)cdiv(total, 256), 256, 0, ctx.stream>>>(p, n, total, cplx ? 2 : 1);
  HP_CHECK_HIP(hipGetLastError());
}

void sqrt_pair(Ctx& ctx, const double* s, int64_t n, double* sq, double* isq) {
  if (n <= 0) return;
  sqrt_pair_kernel<<<std::min<unsigned>(cdiv(n, 256), 1024), 256, 0, ctx.stream>>>(s, n, sq, isq);
  HP_CHECK_HIP(hipGetLastError());
}

void convert_f64_to_bf16(Ctx& ctx, const double* in, void* out, int64_t n) {
  if (n <= 0) return;
  f64_to_bf16_kernel<<<std::min<unsigned>(cdiv(n, 256), 4096), 256, 0, ctx.stream>>>(
      in, static_cast<__bf16*>(out), n);
  HP_CHECK_HIP(hipGetLastError());
}

void convert_f64_to_f32(Ctx& ctx, const double* in, float* out, int64_t n) {
  if (n <= 0) return;
  f64_to_f32_kernel<<<std::min<unsigned>(cdiv(n, 256), 4096), 256, 0, ctx.stream>>>(in, out, n);
  HP_CHECK_HIP(hipGetLastError());
}

void fill_zero(Ctx& ctx, void* p, int64_t bytes) {
  HP_CHECK_HIP(hipMemsetAsync(p, 0, bytes, ctx.stream));
}

void fill_value(Ctx& ctx, double* p, int64_t n, double v, bool cplx) {
  if (n <= 0) return;
  fill_value_kernel<<<std::max<unsigned>(1, std::min<unsigned>(cdiv(n, 256), 1024)), 256, 0, ctx.stream>>>(
      p, n, v, cplx ? 1 : 0);
  HP_CHECK_HIP(hipGetLastError());
}

void gauge_fix(Ctx& ctx, bool cplx, const double* U, int64_t rows, int64_t mp, double* Z, int64_t k,
               int batch) {
  HP_REQUIRE(mp >= 1 && mp <= k && k <= 128, HPEPS_ERR_SHAPE, "canonical phase: k above 128");
  HP_REQUIRE(rows >= 1, HPEPS_ERR_SHAPE, "canonical phase: no rows");
  const int64_t nchunks = cdiv(rows, (int64_t)kGaugeRows);
  HP_REQUIRE(nchunks < 65536 && batch < 65536, HPEPS_ERR_UNSUPPORTED, "canonical phase: too many rows");
  double* part = ctx.ws<double>(2 * nchunks * mp * batch);
  const dim3 g1((unsigned)nchunks, (unsigned)batch);
  if (cplx) {
    gauge_partial_kernel<true><<<g1, 256, 0, ctx.stream>>>(U, rows, (int)mp, (int)nchunks, part);
    gauge_apply_kernel<true><<<batch, 256, 0, ctx.stream>>>(part, (int)nchunks, (int)mp, Z, (int)k);
  } else {
    gauge_partial_kernel<false><<<g1, 256, 0, ctx.stream>>>(U, rows, (int)mp, (int)nchunks, part);
    gauge_apply_kernel<false><<<batch, 256, 0, ctx.stream>>>(part, (int)nchunks, (int)mp, Z, (int)k);
  }
  HP_CHECK_HIP(hipGetLastError());
}

void copy_scalar(Ctx& ctx, const double* src, bool cplx, double* dst) {
  copy_scalar_kernel<<<1, 64, 0, ctx.stream>>>(src, cplx ? 1 : 0, dst);
  HP_CHECK_HIP(hipGetLastError());
}

void normalize(Ctx& ctx, bool cplx, void* x, int64_t n, int batch, double* log_scale) {
  const int64_t nd = cplx ? 2 * n : n;  // a complex array is 2n doubles; same sum of squares
  const int nparts = (int)std::min<int64_t>(cdiv(nd, 256 * 4), 256);
  double* part = ctx.ws<double>((int64_t)nparts * batch);
  double* mx = ctx.ws<double>(batch);
  double* inv = ctx.ws<double>(batch);
  absmax_partial_kernel<<<dim3(nparts, batch), 256, 0, ctx.stream>>>((const double*)x, nd, part);
  absmax_finalize_kernel<<<batch, 64, 0, ctx.stream>>>(part, nparts, mx);
  sumsq_partial_kernel<<<dim3(nparts, batch), 256, 0, ctx.stream>>>((const double*)x, nd, mx, part);
  norm_finalize_kernel<<<batch, 64, 0, ctx.stream>>>(part, nparts, mx, inv, log_scale);
  scale_kernel<<<dim3(std::min<unsigned>(cdiv(nd, 256), 1024), batch), 256, 0, ctx.stream>>>((double*)x, nd, inv);
  HP_CHECK_HIP(hipGetLastError());
  tape_scale(ctx, cplx, (double*)x, n, inv, batch);
}

void scale_by(Ctx& ctx, double* x, int64_t nd, const double* s, int batch) {
  if (nd <= 0) return;
  scale_kernel<<<dim3(std::min<unsigned>(cdiv(nd, 256), 1024), batch), 256, 0, ctx.stream>>>(x, nd, s);
  HP_CHECK_HIP(hipGetLastError());
}

void copy_sigma(Ctx& ctx, const double* sigma_k, int64_t k, int64_t mp, int batch, double* out) {
  copy_sigma_kernel<<<std::max<unsigned>(1, cdiv(batch * mp, 256)), 256, 0, ctx.stream>>>(sigma_k, (int)k, (int)mp,
                                                                                          batch, out);
  HP_CHECK_HIP(hipGetLastError());
}

void stats_reduce(Ctx& ctx, const int* flags, const int* sweeps, int batch, int* acc) {
  stats_kernel<<<1, kStatsThreads, 0, ctx.stream>>>(flags, sweeps, batch, acc);
  HP_CHECK_HIP(hipGetLastError());
}

}  // namespace hp
