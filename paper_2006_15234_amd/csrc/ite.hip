// Two-site gate application by QR-SVD (Alg. 1, Eq. 4) and batched TEBD
// sweeps for imaginary-time evolution (Sec. II-D).
//
// One workgroup updates one bond entirely on chip:
//   1. both sites are matricized as (other legs) x (shared bond, p) while
//      they are gathered into LDS (thread t owns rows t, t + NT, ... of
//      both; 512 threads for the 512-row sites of bond 8); a site with more
//      rows than columns is QR-factored there by CholeskyQR2 (explicit Q),
//      or, when its Gram is too ill-conditioned for that, by Householder
//      reflections (the two sites side by side, one barrier per column);
//      otherwise Q = I and R is the site itself;
//   2. Theta = G R1 R2 (d^2 x d^2 gate, tiny);
//   3. Theta = Q_T R_T (Householder, Q_T accumulated), then one-sided Jacobi
//      on the columns of R_T^T with Q_T's columns rotated alike (<= 32 x 32,
//      in LDS), truncation to D' = min(Dmax, rows, cols), normalisation of
//      the kept values and the sqrt(s) split;
//   4. T' = Q [R~; 0], one product per row with the explicit Q or the parked
//      reflectors applied in reverse order, scattered straight into the
//      canonical [u,d,l,r,p] layout with the new bond.
// Bond dimensions live in a device table, so a whole sweep (four launches,
// one per layer of non-overlapping bonds) is a static sequence that is
// captured once in a HIP graph and replayed.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "contract.h"
#include "dpp.h"
#include "peps.h"

struct hpeps_ite_plan {
  hp::Ctx* ctx = nullptr;
  int nrow = 0, ncol = 0, d = 0;
  int64_t dmax = 0, cap = 0;
  double* sites = nullptr;
  int* dims = nullptr;
  // layers of a sweep, in order: a two-site layer lists (s1, s2, axis, gate)
  // per bond (s1 left of / above s2), a one-site layer (site, gate, 0, 0)
  std::vector<int*> bonds;
  std::vector<int> nb;
  std::vector<char> onesite;
  double* gates = nullptr;   // two-site gates [d,d,d,d]
  double* gates1 = nullptr;  // one-site gates [d,d]
  double* sigma = nullptr;  // per two-site bond of a sweep (layer order): max_rank kept values
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t gstream = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
};

namespace hp {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kT = 256;     // threads per bond workgroup
constexpr int kMaxTh = 32;  // Theta is at most 32 x 32 (D d^2 <= 32)
constexpr int kMaxC = 16;   // columns of a site matricization (shared bond x p) <= 16
constexpr int kMaxRpt = 3;  // rows of a site matricization <= 3 * kT

struct IteArgs {
  double* sites;
  long long cap;
  int* dims;
  const int* bonds;  // per bond: s1, s2, axis, gate
  const double* gates;
  int dmax;
  double* sigma;     // per bond: dmax values (or null)
  int max_rows;
};

struct SiteGeom {
  int dims[5];
  long long st[5];
  int shared;    // index of the shared leg
  int other[3];  // the other virtual legs, canonical order
  int rows, cols;
};

__device__ void site_geom(const int* dims, int shared, SiteGeom& g) {
  for (int i = 0; i < 5; ++i) g.dims[i] = dims[i];
  g.st[4] = 1;
  for (int i = 3; i >= 0; --i) g.st[i] = g.st[i + 1] * g.dims[i + 1];
  g.shared = shared;
  int q = 0;
  for (int i = 0; i < 4; ++i)
    if (i != shared) g.other[q++] = i;
  g.rows = g.dims[g.other[0]] * g.dims[g.other[1]] * g.dims[g.other[2]];
  g.cols = g.dims[shared] * g.dims[4];
}

// element offset of the matricized row (over the other legs, canonical order)
__device__ __forceinline__ long long row_off(const SiteGeom& g, int row) {
  const int o2 = row % g.dims[g.other[2]];
  const int r1 = row / g.dims[g.other[2]];
  const int o1 = r1 % g.dims[g.other[1]], o0 = r1 / g.dims[g.other[1]];
  return o0 * g.st[g.other[0]] + o1 * g.st[g.other[1]] + o2 * g.st[g.other[2]];
}

// Cross-wavefront sums of the partials of one column step.  Every thread
// adds the four wavefronts' values; buffers alternate between steps so that
// one barrier per step suffices (a wavefront can be at most one step ahead).
template <int NT>
struct StepBuf {
  double part[2][NT / 64][kMaxC];
  double row[2][kMaxC];  // snapshot of the pivot row
};

// Wavefront sums of 16 values per lane by recursive halving, on DPP lane
// moves: each stage pairs a lane with a partner in its 16-lane row that
// differs in one more bit of the lane index (row mirror: bit 3, half-row
// mirror: bit 2, quad permutations: bits 1 and 0); the lane keeps the half of
// its remaining values that this bit selects and adds the partner's copy of
// it, so that after four stages lane i holds the row sum of value i & 15.
// Two shuffles then add the four rows.  The adds are not contracted (the
// partner's values are rounded sums).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long x = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)x, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double wave_reduce_scatter16(const double (&v)[16], int lane) {
#pragma clang fp contract(off)
  double a[8], b[4], c[2];
  bool hi = lane & 8;
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = (hi ? v[i + 8] : v[i]) + dpp_mov<0x140>(hi ? v[i] : v[i + 8]);  // row_mirror
  hi = lane & 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) b[i] = (hi ? a[i + 4] : a[i]) + dpp_mov<0x141>(hi ? a[i] : a[i + 4]);  // half mirror
  hi = lane & 2;
#pragma unroll
  for (int i = 0; i < 2; ++i) c[i] = (hi ? b[i + 2] : b[i]) + dpp_mov<0x4e>(hi ? b[i] : b[i + 2]);  // [2,3,0,1]
  hi = lane & 1;
  double d = (hi ? c[1] : c[0]) + dpp_mov<0xb1>(hi ? c[0] : c[1]);  // quad_perm [1,0,3,2]
  d += __shfl_xor(d, 16);
  d += __shfl_xor(d, 32);
  return d;
}

// w[l] = x of lane l (l < MC), the same in every lane (scalar registers).
template <int MC>
__device__ __forceinline__ void lanes_to_scalars(double x, double (&w)[MC]) {
  const long long b = __builtin_bit_cast(long long, x);
#pragma unroll
  for (int l = 0; l < MC; ++l) {
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    w[l] = __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
  }
}

// Totals of the per-wavefront sums part[w][v] (v < 16) over the NT / 64
// wavefronts, for every v, in every thread: lane L adds the partials of
// value L & 15 of the wavefronts congruent to L >> 4 mod 4, two shuffles add
// the four rows, and the 16 totals (the same in every lane) are read out of
// lanes 0..15 into scalar registers.
template <int NT, int MC>
__device__ __forceinline__ void cross_wave_totals(const double (*part)[kMaxC], int lane, double (&w)[MC]) {
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < (NT / 64 + 3) / 4; ++q) {
    const int wv = (lane >> 4) + 4 * q;
    if (wv < NT / 64) t += part[wv][lane & 15];
  }
  t += __shfl_xor(t, 16);
  t += __shfl_xor(t, 32);
  lanes_to_scalars<MC>(t, w);
}

// Householder QR of the two site matricizations at once (P[s]: rows x
// cols[s], LDS, column-major with leading dimension LD; cols[s] = 0 skips a
// site): thread t owns rows t, t + NT, ... of both and only ever touches
// those rows.  One barrier per column step, shared by the two sites: the
// pivot row's owner publishes it, every thread reduces x^T y_l over its rows
// for all l >= j at once (x = column j, y_l = column l, rows >= j), and the
// reflector v = x - alpha e_j (H = I - tau v v^T) follows in every thread
// from ||x||^2, x_j and those sums (v^T y_l = x^T y_l - alpha y_l[j]).
// Afterwards column j of P[s] holds v below and on the diagonal, tau[s][j]
// and row j of R[s] (ld kMaxC) are in LDS.
template <int NT, int RPT, int MC, int LD>
__device__ __forceinline__ void house_factor2(double* const (&P)[2], const int (&cols)[2], double* const (&R)[2],
                                              double* const (&tau)[2], StepBuf<NT> (&sb)[2], int& step) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nj = max(cols[0], cols[1]);
  for (int j = 0; j < nj; ++j) {
    const int buf = step++ & 1;
    double xr[2][RPT];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (j >= cols[s]) continue;  // same in every thread
      const double* x = P[s] + j * LD;
      // the pivot row j < 16 belongs to lane j of wavefront 0, whose other
      // lanes copy it (in program order after its last update)
      if (tid < MC) sb[s].row[buf][tid] = P[s][tid * LD + j];
      // every load is in range (P has MC columns of LD rows): load all, then
      // mask, so that the loads of a step form one batch without branches
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const double xv = x[tid + q * NT];
        xr[s][q] = tid + q * NT >= j ? xv : 0.0;
      }
      // unmasked: columns past cols[s] are zero, and the sums of columns
      // up to j are never used
      double pv[16];
#pragma unroll
      for (int l = 0; l < 16; ++l) {
        double sacc = 0.0;
        if (l < MC) {
#pragma unroll
          for (int q = 0; q < RPT; ++q) sacc += xr[s][q] * P[s][l * LD + tid + q * NT];
        }
        pv[l] = sacc;
      }
      const double tot = wave_reduce_scatter16(pv, lane);
      if (lane < MC) sb[s].part[buf][wave][lane] = tot;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (j >= cols[s]) continue;
      double w[MC];
      cross_wave_totals<NT, MC>(sb[s].part[buf], lane, w);
      double nrm2 = 0.0;
#pragma unroll
      for (int l = 0; l < MC; ++l)
        if (l == j) nrm2 = w[l];
      const double x0 = sb[s].row[buf][j];
      if (nrm2 == 0.0) {  // zero column: H = I, R[j, :] = 0 (the pivot row is zero too)
        if (tid < cols[s]) R[s][j * kMaxC + tid] = 0.0;
        if (tid == 0) tau[s][j] = 0.0;
        continue;
      }
      const double alpha = -copysign(sqrt(nrm2), x0);
      const double v0 = x0 - alpha;
      const double vn2 = nrm2 - x0 * x0 + v0 * v0;
      const double t = vn2 > 0 ? 2.0 / vn2 : 0.0;
#pragma unroll
      for (int l = 0; l < MC; ++l) {
        const double wl = t * (w[l] - alpha * sb[s].row[buf][l]);  // tau v^T y_l
        w[l] = (l > j && l < cols[s]) ? wl : 0.0;
      }
      // rows below j have v = 0 and columns up to j have w = 0: those stores
      // write back the loaded values, so the update needs no branches
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = tid + q * NT;
        const double v = r == j ? v0 : xr[s][q];
        double y[MC];
#pragma unroll
        for (int l = 0; l < MC; ++l) y[l] = P[s][l * LD + r];
#pragma unroll
        for (int l = 0; l < MC; ++l) P[s][l * LD + r] = l == j && r == j ? v0 : y[l] - w[l] * v;
      }
      // row j of R from the updated pivot row (lane j of wavefront 0 wrote it
      // above, in program order before these reads)
      if (tid < cols[s]) R[s][j * kMaxC + tid] = tid < j ? 0.0 : (tid == j ? alpha : P[s][tid * LD + j]);
      if (tid == 0) tau[s][j] = t;
    }
  }
}

// B[s] := H_0 H_1 ... H_{cols[s]-1} B[s] for the reflectors of house_factor2
// in P[s] (same row ownership), for both sites at once; B[s] (registers, RPT
// rows x MC columns) has ncol columns.  One barrier per reflector index,
// shared by the two sites; an index whose reflectors are both the identity
// (tau = 0, the same value in every thread) is skipped.
template <int NT, int RPT, int MC, int LD>
__device__ __forceinline__ void house_apply2(const double* const (&P)[2], const int (&cols)[2],
                                             const double* const (&tau)[2], double (&B)[2][RPT][MC], int ncol,
                                             StepBuf<NT> (&sb)[2], int& step) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = max(cols[0], cols[1]) - 1; j >= 0; --j) {
    double t[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) t[s] = j < cols[s] ? tau[s][j] : 0.0;
    if (t[0] == 0.0 && t[1] == 0.0) continue;
    const int buf = step++ & 1;
    double v[2][RPT];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (t[s] == 0.0) continue;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const double pvq = P[s][j * LD + tid + q * NT];
        v[s][q] = tid + q * NT >= j ? pvq : 0.0;
      }
      double pv[16];  // columns past ncol are zero
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        double sacc = 0.0;
        if (c < MC) {
#pragma unroll
          for (int q = 0; q < RPT; ++q) sacc += v[s][q] * B[s][q][c < MC ? c : 0];
        }
        pv[c] = sacc;
      }
      const double tot = wave_reduce_scatter16(pv, lane);
      if (lane < MC) sb[s].part[buf][wave][lane] = tot;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (t[s] == 0.0) continue;
      double tot[MC];
      cross_wave_totals<NT, MC>(sb[s].part[buf], lane, tot);
#pragma unroll
      for (int c = 0; c < MC; ++c) {
        const double wc = c < ncol ? t[s] * tot[c] : 0.0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) B[s][q][c] -= wc * v[s][q];
      }
    }
  }
}

// Packed upper triangle of a 16 x 16 symmetric matrix: (a, b), a <= b, at
// a * 16 - a (a - 1) / 2 + b - a (136 entries).
__host__ __device__ constexpr int upk(int a, int b) { return a * 16 - a * (a - 1) / 2 + (b - a); }
// CholeskyQR2 of the site matricizations P[s] (rows[s] x cols[s], LDS,
// column-major, ld LD) that have on[s]: two passes of Gram -> Cholesky ->
// Q := A R^-1, so that P[s] ends as the explicit Q and R[s] (row-major, ld
// kMaxC) as R = R_2 R_1.  Each pass: (A) the two halves of the workgroup form
// the two sites' Grams on the matrix cores (each wavefront a block of rows;
// the upper triangle of each wavefront's 16 x 16 MFMA product goes to LDS);
// (B) one wavefront per site adds the partials and factors the Gram in
// registers (lane l holds column l; row j of R goes back to every lane
// through LDS); (C) every thread solves q R = a for its rows (forward
// substitution with R from LDS).  A site whose Cholesky breaks down, whose
// first-pass pivots span more than 1e12 (condition number beyond about 1e6,
// where CholeskyQR2 loses accuracy) or whose second-pass pivots are not near
// 1 gets fail[s] = 1 and is left to the Householder path (its P[s] must then
// be gathered again: the first pass may have overwritten it).
// scratch: 2 (NT / 128) 136 partials + 2 x 256 pass factors + 2 x 16
// reciprocal diagonals (at most 1632 doubles).
template <int NT, int RPT, int MC, int LD>
__device__ void cholqr2_sites(double* P0, double* P1, bool on0, bool on1, int rows0, int rows1, int cols0,
                              int cols1, double* R0, double* R1, double* scratch, int* fail) {
  constexpr int WPS = NT / 128;  // wavefronts per site in the Gram phase
  constexpr int TPS = NT / 2;    // threads per site
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* part = scratch;                 // [2][WPS][136]
  double* Rp = scratch + 2 * WPS * 136;   // [2][256]: this pass's factor
  double* rdi = Rp + 2 * 256;                  // [2][16]: its reciprocal diagonal
  auto Psel = [&](int s) { return s == 0 ? P0 : P1; };
  auto Rsel = [&](int s) { return s == 0 ? R0 : R1; };
  auto on = [&](int s) { return s == 0 ? on0 : on1; };
  auto nrows = [&](int s) { return s == 0 ? rows0 : rows1; };
  auto ncols = [&](int s) { return s == 0 ? cols0 : cols1; };
  if (tid < 2) fail[tid] = 0;
  for (int pass = 0; pass < 2; ++pass) {
    __syncthreads();  // P final from the previous pass (or the gather); fail reset
    // ---- (A) Gram partial sums on the matrix cores ----
    // G = A^T A over a wavefront's rows: v_mfma_f64_16x16x4 with A^T as the
    // first and A as the second operand, so that lane (li, lk) feeds the same
    // element A[r0 + lk][li] to both; accumulator r holds G[lk + 4 r][li].
    {
      const int s = wave / WPS, wl = wave % WPS;
      if (on(s)) {  // wavefront-uniform
        const int li = lane & 15, lk = lane >> 4;
        const double* Ps = Psel(s) + (li < MC ? li : 0) * LD + wl * (LD / WPS) + lk;
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
        for (int kb = 0; kb < LD / WPS / 4; ++kb) {
          const double x = li < MC ? Ps[4 * kb] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ra = lk + 4 * r;
          if (ra <= li) part[(s * WPS + wl) * 136 + upk(ra, li)] = acc[r];
        }
      }
    }
    __syncthreads();
    // ---- (B) Cholesky of each Gram by one wavefront ----
    {
      const int s = wave / WPS;
      if (wave % WPS == 0 && on(s)) {  // wavefronts 0 and WPS
        const int n = ncols(s), l = lane & 15;
        double g[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int a = i < l ? i : l, b = i < l ? l : i;
          double t = 0.0;
#pragma unroll
          for (int w = 0; w < WPS; ++w) t += part[(s * WPS + w) * 136 + upk(a, b)];
          g[i] = t;
        }
        double dmin = 1e300, dmax = 0.0;
        bool bad = false;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          if (j >= n || bad) continue;  // uniform; no break, so that j stays a constant
          const long long gj = __builtin_bit_cast(long long, g[j]);
          const double d = __builtin_bit_cast(
              double, ((long long)__builtin_amdgcn_readlane((int)(gj >> 32), j) << 32) |
                          (long long)(unsigned)__builtin_amdgcn_readlane((int)gj, j));
          if (!(d > 0.0) || !isfinite(d)) {
            bad = true;
            continue;
          }
          dmin = fmin(dmin, d);
          dmax = fmax(dmax, d);
          const double inv = rsqrt(d), rjj = d * inv;
          const double rjl = l > j ? g[j] * inv : (l == j ? rjj : 0.0);  // R[j][l]
          if (lane < 16) Rp[s * 256 + j * 16 + lane] = rjl;
          if (lane == 0) rdi[s * 16 + j] = inv;
          // row j of R back to every lane through LDS (this wavefront wrote
          // it just above: program order)
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            if (i <= j) continue;
            g[i] -= Rp[s * 256 + j * 16 + i] * rjl;  // G[i][l] -= R[j][i] R[j][l]
          }
        }
        if (pass == 0 && !bad && dmin < 1e-12 * dmax) bad = true;
        if (pass == 1 && !bad && (dmin < 0.5 || dmax > 2.0)) bad = true;
        if (lane == 0 && bad) fail[s] = 1;
      }
    }
    __syncthreads();
    // ---- (C) Q := A R^-1 row by row (thread t owns rows t, t + NT, ...) ----
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (!on(s) || fail[s]) continue;  // uniform
      const double* Rs = Rp + s * 256;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int r = tid + NT * q;
        double x[MC];
#pragma unroll
        for (int c = 0; c < MC; ++c) x[c] = Psel(s)[c * LD + r];
#pragma unroll
        for (int c = 0; c < MC; ++c) {
          double t = x[c];
#pragma unroll
          for (int m = 0; m < MC; ++m)
            if (m < c) t -= x[m] * Rs[m * 16 + c];
          x[c] = c < ncols(s) ? t * rdi[s * 16 + c] : 0.0;
        }
        if (r < nrows(s)) {
#pragma unroll
          for (int c = 0; c < MC; ++c) Psel(s)[c * LD + r] = x[c];
        }
      }
    }
    // ---- R := R_pass R (the Cholesky wavefronts; lane l owns column l) ----
    {
      const int s = wave / WPS;
      if (wave % WPS == 0 && on(s) && !fail[s] && lane < 16) {
        const int l = lane;
        double col[16], out[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) col[m] = pass == 0 ? (m == l ? 1.0 : 0.0) : Rsel(s)[m * kMaxC + l];
        // every read before the first write (the compiler cannot tell the two
        // LDS arrays apart, and would otherwise wait on each read in turn)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          double t = 0.0;
#pragma unroll
          for (int m = 0; m < 16; ++m)
            if (m >= i) t += Rp[s * 256 + i * 16 + m] * col[m];
          out[i] = t;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) Rsel(s)[i * kMaxC + l] = i < ncols(s) && l < ncols(s) ? out[i] : 0.0;
      }
    }
  }
  __syncthreads();
}

// One bond per workgroup (Alg. 1): both site matricizations are gathered
// into LDS and QR-factored together (QR skipped when a site has no more rows
// than columns), Q (explicit, or as reflectors) stays there, Theta = G R1 R2 is
// decomposed by a QR-preconditioned one-sided Jacobi in LDS, and the new
// sites Q [R~; 0] are formed in registers and scattered into the
// [u,d,l,r,p] layout with the new bond.  NT threads, RPT rows and MC columns
// per thread; dynamic LDS: two column-major (RPT NT + 1) x MC panel blocks.
// The panels' LDS leaves room for one workgroup per CU, i.e. NT / 256
// wavefronts per SIMD: the register allocator may use that budget to keep
// more LDS loads in flight.
template <int NT, int RPT, int MC>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT / 256, NT / 256)))
void qrsvd_bond_kernel(IteArgs a) {
  extern __shared__ double park[];                          // [2][MC][RPT NT]
  __shared__ double R1[kMaxC * kMaxC], R2[kMaxC * kMaxC];  // k x cols, ld kMaxC
  // Theta (column-major, col * nr + row) and Q / right vectors (column-major),
  // one array so that the site factorization can use both as scratch first
  __shared__ double ThJ[2 * kMaxTh * kMaxTh];
  double* const Th = ThJ;
  double* const J = ThJ + kMaxTh * kMaxTh;
  __shared__ int cqf[2];  // CholeskyQR2 left a site to the Householder path
  __shared__ double tau1[kMaxC], tau2[kMaxC];
  __shared__ double tauT[kMaxTh], alphaT[kMaxTh];  // Householder QR of Theta
  __shared__ double red[NT / 64];
  __shared__ double sig[kMaxTh], sv[kMaxTh];
  __shared__ long long coff1[kMaxC], coff2[kMaxC];
  __shared__ StepBuf<NT> sb[2];
  __shared__ int perm[kMaxTh];
  __shared__ int rot, chk;
  __shared__ SiteGeom g1, g2, go[2];
  // odd leading dimension: accesses that stride across columns (the 16 lanes
  // of an MFMA operand, the pivot-row copies) fall in distinct LDS banks
  constexpr int LD = RPT * NT + 1;
  const int bi = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = NT / 64;
  const int s1 = a.bonds[4 * bi], s2 = a.bonds[4 * bi + 1], axis = a.bonds[4 * bi + 2];
  if (tid == 0) {
    site_geom(a.dims + 5 * s1, axis == 0 ? 3 : 1, g1);
    site_geom(a.dims + 5 * s2, axis == 0 ? 2 : 0, g2);
  }
  __syncthreads();
  const int d = g1.dims[4];
  if (tid < kMaxC) {
    coff1[tid] = (long long)(tid / d) * g1.st[g1.shared] + (tid % d);
    coff2[tid] = (long long)(tid / d) * g2.st[g2.shared] + (tid % d);
  }
  __syncthreads();
  const double* G = a.gates + (long long)a.bonds[4 * bi + 3] * d * d * d * d;
  const int h = g1.dims[g1.shared];
  double* site1 = a.sites + (long long)s1 * a.cap;
  double* site2 = a.sites + (long long)s2 * a.cap;
  int step = 0;

  // ---- gather and factor both sites (matricizations in LDS) -------------
  const bool qr1 = g1.rows > g1.cols, qr2 = g2.rows > g2.cols;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const SiteGeom& g = s == 0 ? g1 : g2;
    const long long* coff = s == 0 ? coff1 : coff2;
    const double* site = s == 0 ? site1 : site2;
    double* P = park + (long long)s * MC * LD;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + q * NT;
      const bool in = r < g.rows;
      const long long ro = in ? row_off(g, r) : 0;
#pragma unroll
      for (int c = 0; c < MC; ++c) P[c * LD + r] = (in && c < g.cols) ? site[ro + coff[c]] : 0.0;
    }
    if (!(s == 0 ? qr1 : qr2) && tid < g.rows) {
      // no QR: R is the matricization itself (rows <= cols <= 16: thread r owns row r)
      double* R = s == 0 ? R1 : R2;
      for (int c = 0; c < g.cols; ++c) R[tid * kMaxC + c] = P[c * LD + tid];
    }
  }
  double* const Pf[2] = {park, park + (long long)MC * LD};
  cholqr2_sites<NT, RPT, MC, LD>(park, park + (long long)MC * LD, qr1, qr2, g1.rows, g2.rows, g1.cols, g2.cols, R1,
                                 R2, ThJ, cqf);
  // sites that CholeskyQR2 could not take: gathered again and Householder-QR
  // factored (reflectors parked in P)
  const bool hh1 = qr1 && cqf[0] != 0, hh2 = qr2 && cqf[1] != 0;
  const bool ex1 = qr1 && !hh1, ex2 = qr2 && !hh2;  // explicit Q in P
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (!(s == 0 ? hh1 : hh2)) continue;  // uniform
    const SiteGeom& g = s == 0 ? g1 : g2;
    const long long* coff = s == 0 ? coff1 : coff2;
    const double* site = s == 0 ? site1 : site2;
    double* P = park + (long long)s * MC * LD;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + q * NT;
      const bool in = r < g.rows;
      const long long ro = in ? row_off(g, r) : 0;
#pragma unroll
      for (int c = 0; c < MC; ++c) P[c * LD + r] = (in && c < g.cols) ? site[ro + coff[c]] : 0.0;
    }
  }
  const int qcols[2] = {hh1 ? g1.cols : 0, hh2 ? g2.cols : 0};
  {
    double* const Rf[2] = {R1, R2};
    double* const tf[2] = {tau1, tau2};
    house_factor2<NT, RPT, MC, LD>(Pf, qcols, Rf, tf, sb, step);
  }
  __syncthreads();
  const int k1 = qr1 ? g1.cols : g1.rows;
  const int k2 = qr2 ? g2.cols : g2.rows;

  // ---- Theta[(k1,a),(b,l)] = sum_{h,i,j} G[a,b,i,j] R1[k1,(h,i)] R2[l,(h,j)] ----
  const int nr = k1 * d, nc = d * k2;
  for (int e = tid; e < nr * nc; e += NT) {
    const int col = e / nr, row = e - col * nr;
    const int kk1 = row / d, aa = row - kk1 * d, bb = col / k2, ll = col - bb * k2;
    double acc = 0;
    for (int i = 0; i < d; ++i)
      for (int j = 0; j < d; ++j) {
        const double gv = G[((aa * d + bb) * d + i) * d + j];
        if (gv == 0.0) continue;
        double w = 0;
        for (int hh = 0; hh < h; ++hh) w += R1[kk1 * kMaxC + hh * d + i] * R2[ll * kMaxC + hh * d + j];
        acc += gv * w;
      }
    Th[e] = acc;
  }
  __syncthreads();

  // ---- Theta = Q R (Householder), K = R^T, Q explicit --------------------
  // One-sided Jacobi on the columns of K = R^T converges in far fewer sweeps
  // than on Theta itself (the rows of R are graded: 6-8 sweeps instead of
  // 14-18 on the spectra of these updates); the rotations are mirrored on
  // the columns of Q, so that at the end Theta = (Q J) Sigma W^T with
  // W = K J Sigma^-1: the left vectors are Q's rotated columns, the right
  // vectors K's rotated columns normalised.  Q is accumulated in J's
  // storage during the factorization, K then overwrites Theta's.
  double fro2 = 0;
  {
    double f2 = 0;
    for (int e = tid; e < nr * nc; e += NT) f2 += Th[e] * Th[e];
    f2 = wave_sum(f2);
    if (lane == 0) red[wave] = f2;
    __syncthreads();
    for (int w = 0; w < nw; ++w) fro2 += red[w];
  }
  const int nk = min(nr, nc);
  // Q accumulates Q := Q H_j (nr x nr, in J's storage); 16-lane groups own a
  // trailing column of Theta and a row of Q each (lanes: rows / columns gl
  // and gl + 16), with DPP row sums for the dot products
  const int qg = tid >> 4, ql = tid & 15;
  for (int e = tid; e < nr * nr; e += NT) J[e] = (e / nr == e % nr) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = 0; j < nk; ++j) {
    if (qg == 0) {
      const double x0 = ql >= j && ql < nr ? Th[j * nr + ql] : 0.0;
      const double x1 = ql + 16 >= j && ql + 16 < nr ? Th[j * nr + ql + 16] : 0.0;
      const double n2 = row_sum16(x0 * x0 + x1 * x1);
      if (ql == 0) {
        const double xj = Th[j * nr + j];
        const double al = n2 > 0 ? -copysign(sqrt(n2), xj) : 0.0;
        const double v0 = xj - al;
        const double vn2 = n2 - xj * xj + v0 * v0;
        tauT[j] = vn2 > 0 ? 2.0 / vn2 : 0.0;
        alphaT[j] = al;
        Th[j * nr + j] = v0;  // v: rows >= j of column j
      }
    }
    __syncthreads();
    const double t = tauT[j];
    const double v0r = ql >= j && ql < nr ? Th[j * nr + ql] : 0.0;
    const double v1r = ql + 16 >= j && ql + 16 < nr ? Th[j * nr + ql + 16] : 0.0;
    // trailing columns l = j + 1 + qg (+ 16): y -= tau (v^T y) v over rows >= j
    for (int l = j + 1 + qg; l < nc; l += NT / 16) {
      double* y = Th + l * nr;
      const double y0 = ql < nr ? y[ql] : 0.0, y1 = ql + 16 < nr ? y[ql + 16] : 0.0;
      const double w = t * row_sum16(v0r * y0 + v1r * y1);
      if (ql >= j && ql < nr) y[ql] = y0 - w * v0r;
      if (ql + 16 >= j && ql + 16 < nr) y[ql + 16] = y1 - w * v1r;
    }
    // rows i = qg (+ 16) of Q: q -= tau (q . v) v^T over columns >= j
    for (int i = qg; i < nr; i += NT / 16) {
      const double q0 = ql < nr ? J[ql * nr + i] : 0.0, q1 = ql + 16 < nr ? J[(ql + 16) * nr + i] : 0.0;
      const double w = t * row_sum16(q0 * v0r + q1 * v1r);
      if (ql >= j && ql < nr) J[ql * nr + i] = q0 - w * v0r;
      if (ql + 16 >= j && ql + 16 < nr) J[(ql + 16) * nr + i] = q1 - w * v1r;
    }
    __syncthreads();
  }
  // K[c][i] = R[c][i] (row c of R as column c of K, length nc) in Theta's
  // storage, through registers (the two layouts overlap)
  constexpr int KV = kMaxTh * kMaxTh / NT;
  double kv[KV];
#pragma unroll
  for (int q = 0; q < KV; ++q) {
    const int e = tid + q * NT;
    const int c = e / nc, i = e - c * nc;
    kv[q] = (e >= nk * nc || i < c) ? 0.0 : (i == c ? alphaT[c] : Th[i * nr + c]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < KV; ++q) {
    const int e = tid + q * NT;
    if (e < nk * nc) Th[e] = kv[q];
  }
  __syncthreads();
  // the roles of the two buffers below: K in Th (column c at c * nc, length
  // nc), Q in J (column c at c * nr, length nr)

  // ---- one-sided Jacobi on the columns of K (Q's columns rotated alike) --
  // A pair (x, y) with Gram entries a2 = |x|^2, b2 = |y|^2, g = x.y is
  // rotated while |g| exceeds both sqrt(nc) eps |x| |y| (relative
  // convergence) and delta ||Theta||_F max(|x|, |y|), delta = 512 eps.
  // Leaving a pair unrotated moves its singular values by at most
  // |g| / max(|x|, |y|) (the degenerate case) and the two-site product by
  // as much, so the second test bounds every kept value and the product at
  // delta ||Theta||_F, for large and small singular values alike, while it
  // stops the rotations among columns of rounding noise (rank-deficient
  // Theta near product states), whose correlations stay O(1) relative to
  // their norms.
  const double acc2 = 0x1p-86 * fro2;  // (delta ||Theta||_F)^2, delta = 512 eps = 2^-43
  const int n = (nk + 1) / 2 * 2;
  const double tol2 = (double)nc * 0x1p-104;  // (sqrt(nc) eps)^2
  // one 16-lane group per column pair (nk <= 32: at most 16 pairs per round,
  // all in flight at once); a group reduces over the rows with DPP row sums
  const int grp = tid >> 4, gl = tid & 15;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) rot = 0;
    __syncthreads();
    for (int round = 0; round < n - 1; ++round) {
      // circle positions; (pos - 1 + round) mod (n - 1) by one conditional
      // subtraction (both terms are below n - 1)
      int ca = nk, cb = nk;
      if (grp < n / 2) {
        int ta = grp - 1 + round;
        ta -= ta >= n - 1 ? n - 1 : 0;
        ca = grp == 0 ? 0 : 1 + ta;
        int tb = n - 2 - grp + round;
        tb -= tb >= n - 1 ? n - 1 : 0;
        cb = 1 + tb;
      }
      const bool act = ca < nk && cb < nk;
      double* x = Th + (act ? ca : 0) * nc;
      double* y = Th + (act ? cb : 0) * nc;
      // rows gl and gl + 16 of the pair (nc <= 32)
      const bool in0 = act && gl < nc, in1 = act && gl + 16 < nc;
      const double x0 = in0 ? x[gl] : 0.0, y0 = in0 ? y[gl] : 0.0;
      const double x1 = in1 ? x[gl + 16] : 0.0, y1 = in1 ? y[gl + 16] : 0.0;
      // Q's rows of the pair, loaded with the pair (off the critical path)
      double* qx = J + (act ? ca : 0) * nr;
      double* qy = J + (act ? cb : 0) * nr;
      const bool j0 = act && gl < nr, j1 = act && gl + 16 < nr;
      const double qx0 = j0 ? qx[gl] : 0.0, qy0 = j0 ? qy[gl] : 0.0;
      const double qx1 = j1 ? qx[gl + 16] : 0.0, qy1 = j1 ? qy[gl + 16] : 0.0;
      double a2 = x0 * x0 + x1 * x1, b2 = y0 * y0 + y1 * y1, gm = x0 * y0 + x1 * y1;
      a2 = row_sum16(a2);
      b2 = row_sum16(b2);
      gm = row_sum16(gm);
      // |gm| > sqrt(nc) eps sqrt(a2 b2) without square roots.  The rotation
      // (|theta| <= pi/4, tan 2 theta = 2 gm / dl, dl = b2 - a2) by two
      // reciprocal square roots: with r = (dl^2 + 4 gm^2)^-1/2,
      // C = cos 2 theta = |dl| r, S = sin 2 theta = sign(dl) 2 gm r and
      // u = (2 (1 + C))^-1/2: cos theta = (1 + C) u, sin theta = S u.
      if (act && gm * gm > tol2 * a2 * b2 && gm * gm > acc2 * fmax(a2, b2)) {
        const double dl = b2 - a2;
        const double r = rsqrt(dl * dl + 4.0 * gm * gm);
        const double C = fabs(dl) * r, S = (dl >= 0 ? 2.0 : -2.0) * gm * r;
        const double u = rsqrt(2.0 + 2.0 * C);
        const double c = (1.0 + C) * u, sn = S * u;
        if (in0) {
          x[gl] = c * x0 - sn * y0;
          y[gl] = sn * x0 + c * y0;
        }
        if (in1) {
          x[gl + 16] = c * x1 - sn * y1;
          y[gl + 16] = sn * x1 + c * y1;
        }
        if (j0) {
          qx[gl] = c * qx0 - sn * qy0;
          qy[gl] = sn * qx0 + c * qy0;
        }
        if (j1) {
          qx[gl + 16] = c * qx1 - sn * qy1;
          qy[gl + 16] = sn * qx1 + c * qy1;
        }
        if (gl == 0) atomicAdd(&rot, 1);
      }
      __syncthreads();
    }
    const int nrot = rot;
    __syncthreads();
    if (nrot == 0) break;
    if (nrot <= nk) {
      // Few rotations left: test every pair against the rotation thresholds
      // at once (one pair per thread, one barrier) instead of a sweep of
      // n - 1 rounds that would find none to rotate (no column changes in
      // such a sweep, so it makes exactly these tests).
      if (tid == 0) chk = 0;
      __syncthreads();
      for (int pq = tid; pq < nk * (nk - 1) / 2; pq += NT) {
        int ca = 0, rem = pq;
        while (rem >= nk - 1 - ca) {
          rem -= nk - 1 - ca;
          ++ca;
        }
        const int cb = ca + 1 + rem;
        const double* x = Th + ca * nc;
        const double* y = Th + cb * nc;
        double a2 = 0.0, b2 = 0.0, gm = 0.0;
        for (int i = 0; i < nc; ++i) {
          a2 += x[i] * x[i];
          b2 += y[i] * y[i];
          gm += x[i] * y[i];
        }
        if (gm * gm > tol2 * a2 * b2 && gm * gm > acc2 * fmax(a2, b2)) chk = 1;
      }
      __syncthreads();
      const bool conv = chk == 0;
      if (conv) break;
    }
  }
  for (int c = wave; c < nk; c += nw) {
    double a2 = 0;
    for (int r = lane; r < nc; r += 64) a2 += Th[(long long)c * nc + r] * Th[(long long)c * nc + r];
    a2 = wave_sum(a2);
    if (lane == 0) sig[c] = sqrt(a2);
  }
  __syncthreads();
  const int Dn = min(a.dmax, nk);
  // descending order, ties by index: the rank of value i is the number of
  // values that precede it
  if (tid < nk) {
    const double v = sig[tid];
    int rank = 0;
    for (int j = 0; j < nk; ++j) rank += (sig[j] > v) || (sig[j] == v && j < tid);
    perm[rank] = tid;
  }
  __syncthreads();
  if (tid == 0) {
    double nn = 0;
    for (int b = 0; b < Dn; ++b) nn += sig[perm[b]] * sig[perm[b]];
    nn = sqrt(nn);
    for (int b = 0; b < Dn; ++b) sv[b] = nn > 0 ? sig[perm[b]] / nn : 0.0;
    if (a.sigma)
      for (int b = 0; b < a.dmax; ++b) a.sigma[(long long)bi * a.dmax + b] = b < Dn ? sv[b] : 0.0;
  }
  __syncthreads();

  // ---- new sites: T' = Q [R~; 0] with columns (b, p) ---------------------
  const int ncol_out = Dn * d;
  // R~[kk, (b, a)] of a site: X[(row,aa),b] from Q_T's rotated columns (site 1)
  // or Y[(aa,row),b] from K's normalised columns (site 2), times sqrt(s_b)
  auto rtilde = [&](int s, int row, int col) -> double {
    const int b = col / d, aa = col - b * d;
    const int c = perm[b];
    const double sg = sig[c];
    const double rs = sqrt(sv[b]);
    if (s == 0) return J[(long long)c * nr + row * d + aa] * rs;
    return sg > 0 ? Th[(long long)c * nc + aa * k2 + row] / sg * rs : 0.0;
  };
  // explicit-Q sites: R~ into R1 / R2 (free since Theta was formed), then
  // every row is Q[row, :] R~
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (!(s == 0 ? ex1 : ex2)) continue;
    const int kk = s == 0 ? k1 : k2;
    double* Rs = s == 0 ? R1 : R2;
    for (int e = tid; e < kk * ncol_out; e += NT) {
      const int row = e / ncol_out, col = e - row * ncol_out;
      Rs[row * kMaxC + col] = rtilde(s, row, col);
    }
  }
  __syncthreads();
  double B[2][RPT][MC];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int kk = s == 0 ? k1 : k2;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int row = tid + q * NT;
      if (s == 0 ? ex1 : ex2) {
        const double* Ps = park + (long long)s * MC * LD;
        const double* Rs = s == 0 ? R1 : R2;
        double qr[MC];
#pragma unroll
        for (int c = 0; c < MC; ++c) qr[c] = Ps[c * LD + row];
#pragma unroll
        for (int col = 0; col < MC; ++col) {
          double acc = 0.0;
          if (col < ncol_out) {
#pragma unroll
            for (int c = 0; c < MC; ++c)
              if (c < kk) acc += qr[c] * Rs[c * kMaxC + col];
          }
          B[s][q][col] = acc;
        }
      } else {
        // R~ in the rows the thread owns (rows >= kk are zero)
#pragma unroll
        for (int col = 0; col < MC; ++col) B[s][q][col] = row < kk && col < ncol_out ? rtilde(s, row, col) : 0.0;
      }
    }
  }
  {
    const double* const Pc[2] = {Pf[0], Pf[1]};
    const double* const tc[2] = {tau1, tau2};
    house_apply2<NT, RPT, MC, LD>(Pc, qcols, tc, B, ncol_out, sb, step);
  }
  // scatter into the canonical layout with the new shared dimension
  if (tid == 0) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const SiteGeom& g = s == 0 ? g1 : g2;
      go[s] = g;
      go[s].dims[g.shared] = Dn;
      go[s].st[4] = 1;
      for (int i = 3; i >= 0; --i) go[s].st[i] = go[s].st[i + 1] * go[s].dims[i + 1];
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const SiteGeom& g = s == 0 ? g1 : g2;
    double* site = s == 0 ? site1 : site2;
    const long long sst = go[s].st[g.shared];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r = tid + q * NT;
      if (r >= g.rows) continue;
      const long long ro = row_off(go[s], r);
#pragma unroll
      for (int col = 0; col < MC; ++col) {
        if (col < ncol_out) {
          const int b = col / d, aa = col - b * d;
          site[ro + b * sst + aa] = B[s][q][col];
        }
      }
    }
  }
  if (tid == 0) {
    a.dims[5 * s1 + g1.shared] = Dn;
    a.dims[5 * s2 + g2.shared] = Dn;
  }
}

void check_dims(int64_t dmax, int d) {
  HP_REQUIRE(dmax >= 1 && d >= 1, HPEPS_ERR_INVALID_ARG, "bad bond or physical dimension");
  HP_REQUIRE(dmax * d * d <= kMaxTh, HPEPS_ERR_UNSUPPORTED, "QR-SVD kernel supports D d^2 <= 32");
  HP_REQUIRE(dmax * d <= kMaxC && dmax * dmax * dmax <= kMaxRpt * kT, HPEPS_ERR_UNSUPPORTED,
             "QR-SVD kernel supports D d <= 16 and D^3 <= 768");
}

// Variants: threads x rows per thread x register columns.  Up to 512 rows
// each thread owns one row of both sites (512 threads: two wavefronts per
// SIMD hide each other's LDS round trips; the LDS of the two 512 x 16
// panels allows one workgroup per CU).  D^3 > 512 needs D >= 9, hence d = 1
// and at most 9 columns.
template <int NT, int RPT, int MC>
struct BondVariant {
  static constexpr int nt = NT, rpt = RPT, mc = MC;
};

void launch_layer(hipStream_t st, const IteArgs& a, int nb) {
  if (nb == 0) return;
  // the dynamic LDS limit is raised once per variant and process
  static std::once_flag once[3];
  // the kernel is launched by name, never through a pointer to it (such a
  // launch has run nothing, without an error, in host code built with
  // instrumentation); the tag carries the variant's template arguments
  auto go = [&](auto t, int v) {
    using T = decltype(t);
    constexpr int NT = T::nt, RPT = T::rpt, MC = T::mc;
    const size_t lds = (size_t)2 * MC * (RPT * NT + 1) * sizeof(double);
    hipError_t e = hipSuccess;
    std::call_once(once[v], [&] {
      e = hipFuncSetAttribute((const void*)&qrsvd_bond_kernel<NT, RPT, MC>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    });
    HP_CHECK_HIP(e);
    qrsvd_bond_kernel<NT, RPT, MC><<<nb, NT, lds, st>>>(a);
  };
  if (a.max_rows <= kT)
    go(BondVariant<kT, 1, kMaxC>{}, 0);
  else if (a.max_rows <= 2 * kT)
    go(BondVariant<2 * kT, 1, kMaxC>{}, 1);
  else
    go(BondVariant<kT, 3, 9>{}, 2);
}

// One-site gates (Eq. 3) of a layer, in place: workgroup b applies the d x d
// gate bonds[4 b + 1] to site bonds[4 b] fiber by fiber (the physical leg is
// the contiguous one); a site appears at most once per layer.
__global__ __launch_bounds__(kT) void onesite_kernel(IteArgs a, const double* gates1) {
  const int s = a.bonds[4 * blockIdx.x], gi = a.bonds[4 * blockIdx.x + 1];
  const int* dm = a.dims + 5 * s;
  const int d = dm[4];
  const long long fibers = (long long)dm[0] * dm[1] * dm[2] * dm[3];
  const double* O = gates1 + (long long)gi * d * d;
  double* site = a.sites + (long long)s * a.cap;
  constexpr int kMaxD = 8;
  for (long long f = threadIdx.x; f < fibers; f += blockDim.x) {
    double x[kMaxD];
    for (int q = 0; q < d; ++q) x[q] = site[f * d + q];
    for (int P = 0; P < d; ++P) {
      double acc = 0.0;
      for (int q = 0; q < d; ++q) acc += O[P * d + q] * x[q];
      site[f * d + P] = acc;
    }
  }
}

IteArgs plan_args(hpeps_ite_plan* p, int layer) {
  IteArgs a{};
  a.sites = p->sites;
  a.cap = p->cap;
  a.dims = p->dims;
  a.bonds = p->bonds[layer];
  a.gates = p->gates;
  a.dmax = (int)p->dmax;
  int off = 0;
  for (int l = 0; l < layer; ++l) off += p->onesite[l] ? 0 : p->nb[l];
  a.sigma = p->sigma + (int64_t)off * p->dmax;
  a.max_rows = (int)(p->dmax * p->dmax * p->dmax);
  return a;
}

}  // namespace
}  // namespace hp

// ---------------------------------------------------------------------------
// ABI

namespace {
template <class F>
hpeps_status guard_i(hp::Ctx* c, F&& f) {
  try {
    f();
    return HPEPS_OK;
  } catch (const hp::Error& e) {
    if (c) c->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    if (c) c->last_error = "host allocation failed";
    return HPEPS_ERR_ALLOC;
  } catch (...) {
    if (c) c->last_error = "unknown error";
    return HPEPS_ERR_INVALID_ARG;
  }
}

void free_plan(hpeps_ite_plan* p) {
  if (!p) return;
  if (p->gstream) (void)hipStreamSynchronize(p->gstream);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->gstream) (void)hipStreamDestroy(p->gstream);
  for (auto e : p->ev)
    if (e) (void)hipEventDestroy(e);
  (void)hipFree(p->sites);
  (void)hipFree(p->dims);
  for (auto& b : p->bonds) (void)hipFree(b);
  (void)hipFree(p->gates);
  (void)hipFree(p->gates1);
  (void)hipFree(p->sigma);
  delete p;
}

int total_bonds(const hpeps_ite_plan* p) {
  int t = 0;
  for (size_t l = 0; l < p->nb.size(); ++l) t += p->onesite[l] ? 0 : p->nb[l];
  return t;
}

// One layer's launch (every entry its own workgroup).
void launch_any(hpeps_ite_plan* p, hipStream_t st, int l, const hp::IteArgs& a, int n) {
  if (n == 0) return;
  if (p->onesite[l]) {
    hp::onesite_kernel<<<n, hp::kT, 0, st>>>(a, p->gates1);
    HP_CHECK_HIP(hipGetLastError());
  } else {
    hp::launch_layer(st, a, n);
  }
}

// An operation of a compiled sweep: a two-site gate on a bond (s1 left of /
// above s2) or a one-site gate.
struct Op {
  bool one;
  int s1, s2, axis, gate;
};

// Builds the device side of a plan from the initial lattice, the layers of a
// sweep and the gate tables (host, FP64).
hpeps_ite_plan* build_plan(hp::Ctx& c, const hp::Lattice& L, int64_t max_rank, const std::vector<std::vector<Op>>& layers,
                           const std::vector<double>& g2, const std::vector<double>& g1) {
  const int d = (int)L.sites[0].dims[4];
  hpeps_ite_plan* p = new hpeps_ite_plan();
  try {
    p->ctx = &c;
    p->nrow = L.nrow;
    p->ncol = L.ncol;
    p->d = d;
    p->dmax = max_rank;
    p->cap = max_rank * max_rank * max_rank * max_rank * d;
    const int ns = L.nrow * L.ncol;
    HP_CHECK_HIP(hipMalloc(&p->sites, (size_t)ns * p->cap * sizeof(double)));
    std::vector<int> dims(5 * ns);
    for (int s = 0; s < ns; ++s) {
      HP_CHECK_HIP(hipMemcpyAsync(p->sites + (int64_t)s * p->cap, L.sites[s].p, L.sites[s].size() * sizeof(double),
                                  hipMemcpyDeviceToDevice, c.stream));
      for (int e = 0; e < 5; ++e) dims[5 * s + e] = (int)L.sites[s].dims[e];
    }
    HP_CHECK_HIP(hipMalloc(&p->dims, dims.size() * sizeof(int)));
    HP_CHECK_HIP(hipMemcpy(p->dims, dims.data(), dims.size() * sizeof(int), hipMemcpyHostToDevice));
    for (const auto& layer : layers) {
      std::vector<int> tb;
      for (const Op& o : layer)
        if (o.one) tb.insert(tb.end(), {o.s1, o.gate, 0, 0});
        else tb.insert(tb.end(), {o.s1, o.s2, o.axis, o.gate});
      int* dev = nullptr;
      HP_CHECK_HIP(hipMalloc(&dev, std::max<size_t>(tb.size(), 4) * sizeof(int)));
      p->bonds.push_back(dev);
      p->nb.push_back((int)layer.size());
      p->onesite.push_back(!layer.empty() && layer[0].one);
      if (!tb.empty()) HP_CHECK_HIP(hipMemcpy(dev, tb.data(), tb.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    HP_CHECK_HIP(hipMalloc(&p->gates, std::max<size_t>(g2.size(), 1) * sizeof(double)));
    if (!g2.empty()) HP_CHECK_HIP(hipMemcpy(p->gates, g2.data(), g2.size() * sizeof(double), hipMemcpyHostToDevice));
    HP_CHECK_HIP(hipMalloc(&p->gates1, std::max<size_t>(g1.size(), 1) * sizeof(double)));
    if (!g1.empty()) HP_CHECK_HIP(hipMemcpy(p->gates1, g1.data(), g1.size() * sizeof(double), hipMemcpyHostToDevice));
    const int total_nb = total_bonds(p);
    HP_CHECK_HIP(hipMalloc(&p->sigma, (size_t)std::max(total_nb, 1) * max_rank * sizeof(double)));
    HP_CHECK_HIP(hipMemsetAsync(p->sigma, 0, (size_t)std::max(total_nb, 1) * max_rank * sizeof(double), c.stream));
    HP_CHECK_HIP(hipStreamSynchronize(c.stream));
  } catch (...) {
    free_plan(p);
    throw;
  }
  return p;
}

// Compiles a gate list into layers.  A two-site gate on sites a, b that are
// not nearest neighbours becomes a SWAP chain (Sec. II-C): b's state is moved
// by SWAP gates along its row to a's column, then along that column until it
// is a neighbour of a; the gate acts there; the SWAPs are undone in reverse
// order.  A gate whose second site ends up left of or above the first is
// applied transposed (G[Q,P,q,p]).  Each operation is placed in the first
// layer after the last one that touches its sites (one-site and two-site
// operations never share a layer), so every site sees its operations in list
// order and no layer touches a site twice.
std::vector<std::vector<Op>> compile_ops(int nrow, int ncol, int d, int n_ops, const int32_t* ops, int n2, int n1,
                                         std::vector<double>& g2) {
  const int64_t g4 = (int64_t)d * d * d * d;
  // SWAP[P,Q,p,q] = delta(P,q) delta(Q,p), appended to the table
  const int swap_id = n2;
  std::vector<int> transposed(n2 + 1, -1);
  {
    std::vector<double> sw(g4, 0.0);
    for (int P = 0; P < d; ++P)
      for (int Q = 0; Q < d; ++Q) sw[((P * d + Q) * d + Q) * d + P] = 1.0;
    g2.insert(g2.end(), sw.begin(), sw.end());
    transposed[swap_id] = swap_id;
  }
  auto transpose_of = [&](int g) {
    if (transposed[g] < 0) {
      const int64_t base = (int64_t)g * g4;
      std::vector<double> t(g4);
      for (int P = 0; P < d; ++P)
        for (int Q = 0; Q < d; ++Q)
          for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) t[((Q * d + P) * d + b) * d + a] = g2[base + ((P * d + Q) * d + a) * d + b];
      transposed[g] = (int)(g2.size() / g4);
      g2.insert(g2.end(), t.begin(), t.end());
    }
    return transposed[g];
  };
  std::vector<Op> seq;
  auto bond_op = [&](int ia, int ja, int ib, int jb, int g) {
    // a, b nearest neighbours; oriented so that s1 is left of / above s2
    const bool ab = (ia == ib && jb == ja + 1) || (ja == jb && ib == ia + 1);
    const bool ba = (ia == ib && ja == jb + 1) || (ja == jb && ia == ib + 1);
    HP_REQUIRE(ab || ba, HPEPS_ERR_INVALID_ARG, "internal: bond sites not adjacent");
    Op o{false, 0, 0, 0, 0};
    if (ab) {
      o.s1 = ia * ncol + ja; o.s2 = ib * ncol + jb; o.gate = g;
    } else {
      o.s1 = ib * ncol + jb; o.s2 = ia * ncol + ja; o.gate = transpose_of(g);
    }
    o.axis = ia == ib ? 0 : 1;
    seq.push_back(o);
  };
  for (int t = 0; t < n_ops; ++t) {
    const int32_t* e = ops + 6 * t;
    const int kind = e[0], i1 = e[1], j1 = e[2], i2 = e[3], j2 = e[4], g = e[5];
    HP_REQUIRE(kind == 1 || kind == 2, HPEPS_ERR_INVALID_ARG, "operation kind must be 1 or 2");
    HP_REQUIRE(i1 >= 0 && i1 < nrow && j1 >= 0 && j1 < ncol, HPEPS_ERR_INVALID_ARG, "site out of range");
    if (kind == 1) {
      HP_REQUIRE(g >= 0 && g < n1, HPEPS_ERR_INVALID_ARG, "one-site gate index out of range");
      seq.push_back(Op{true, i1 * ncol + j1, -1, 0, g});
      continue;
    }
    HP_REQUIRE(i2 >= 0 && i2 < nrow && j2 >= 0 && j2 < ncol, HPEPS_ERR_INVALID_ARG, "site out of range");
    HP_REQUIRE(!(i1 == i2 && j1 == j2), HPEPS_ERR_INVALID_ARG, "a two-site gate needs two distinct sites");
    HP_REQUIRE(g >= 0 && g < n2, HPEPS_ERR_INVALID_ARG, "two-site gate index out of range");
    // the path of site b toward a
    std::vector<std::array<int, 2>> path{{i2, j2}};
    auto adjacent = [&](int i, int j) { return std::abs(i - i1) + std::abs(j - j1) == 1; };
    int ci = i2, cj = j2;
    while (!adjacent(ci, cj)) {
      if (cj != j1 && !(ci == i1 && std::abs(cj - j1) == 1)) cj += cj < j1 ? 1 : -1;
      else ci += ci < i1 ? 1 : -1;
      path.push_back({ci, cj});
    }
    for (size_t q = 0; q + 1 < path.size(); ++q)
      bond_op(path[q][0], path[q][1], path[q + 1][0], path[q + 1][1], swap_id);
    bond_op(i1, j1, ci, cj, g);
    for (size_t q = path.size() - 1; q >= 1; --q)
      bond_op(path[q - 1][0], path[q - 1][1], path[q][0], path[q][1], swap_id);
  }
  // layering
  std::vector<std::vector<Op>> layers;
  std::vector<int> last(nrow * ncol, -1);
  for (const Op& o : seq) {
    int L = last[o.s1] + 1;
    if (!o.one) L = std::max(L, last[o.s2] + 1);
    while (L < (int)layers.size() && !layers[L].empty() && layers[L][0].one != o.one) ++L;
    if (L >= (int)layers.size()) layers.resize(L + 1);
    layers[L].push_back(o);
    last[o.s1] = L;
    if (!o.one) last[o.s2] = L;
  }
  return layers;
}

// layer lists of a lattice: horizontal bonds at even / odd columns, vertical
// bonds at even / odd rows; entries (s1, s2, axis)
std::vector<std::vector<std::array<int, 3>>> lattice_layers(int nrow, int ncol) {
  std::vector<std::vector<std::array<int, 3>>> L(4);
  for (int par = 0; par < 2; ++par)
    for (int i = 0; i < nrow; ++i)
      for (int j = par; j + 1 < ncol; j += 2) L[par].push_back({i * ncol + j, i * ncol + j + 1, 0});
  for (int par = 0; par < 2; ++par)
    for (int i = par; i + 1 < nrow; i += 2)
      for (int j = 0; j < ncol; ++j) L[2 + par].push_back({i * ncol + j, (i + 1) * ncol + j, 1});
  return L;
}
}  // namespace

namespace {

// Static scratch of the allocation-free two-site gate update: one copy per
// GPU the library runs on, held until the process ends.  Host code never
// names it except to resolve its device address (hipGetSymbolAddress, once
// per device, when a context is created on it).
constexpr size_t kGateScratchBytes = (size_t)1 << 20;
static __device__ __align__(256) unsigned char scratch[kGateScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Bytes of one buffer rounded up to the 256-byte alignment of every piece.
size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// One QR-SVD update of the bond (i, j)-(i2, j2) on the context's stream, with
// the device buffers (staging copies of the two sites, dimension and bond
// tables, gate, singular values) taken from `take`.
template <class Take>
void gate_update(hp::Ctx& c, hpeps_peps* peps, const int64_t* capacity, int32_t i, int32_t j, int32_t axis,
                 const void* G, int64_t max_rank, int64_t* new_bond, double* sigma_out, Take take) {
  HP_REQUIRE(peps && capacity && G && new_bond, HPEPS_ERR_INVALID_ARG, "null argument");
  HP_REQUIRE(axis == 0 || axis == 1, HPEPS_ERR_INVALID_ARG, "axis must be 0 or 1");
  hp::Lattice L = hp::lattice_from_abi(peps);
  HP_REQUIRE(!L.cplx, HPEPS_ERR_DTYPE, "the QR-SVD kernel is FP64 real");
  const int i2 = axis == 0 ? i : i + 1, j2 = axis == 0 ? j + 1 : j;
  HP_REQUIRE(i >= 0 && j >= 0 && i2 < L.nrow && j2 < L.ncol, HPEPS_ERR_INVALID_ARG, "bond outside the lattice");
  const int d = (int)L.sites[0].dims[4];
  hp::check_dims(max_rank, d);
  const int q1 = i * L.ncol + j, q2 = i2 * L.ncol + j2;
  const hp::DevTensor &T1 = L.sites[q1], &T2 = L.sites[q2];
  for (int e = 0; e < 4; ++e)
    HP_REQUIRE(T1.dims[e] <= max_rank && T2.dims[e] <= max_rank, HPEPS_ERR_SHAPE, "bond exceeds max_rank");
  // new bond, from the shapes alone
  const int sh1 = axis == 0 ? 3 : 1, sh2 = axis == 0 ? 2 : 0;
  const int64_t rows1 = T1.size() / (T1.dims[sh1] * d), rows2 = T2.size() / (T2.dims[sh2] * d);
  const int64_t c1 = T1.dims[sh1] * d, c2 = T2.dims[sh2] * d;
  const int64_t k1 = std::min(rows1, c1), k2 = std::min(rows2, c2);
  const int64_t Dn = std::min<int64_t>(max_rank, std::min(k1 * d, d * k2));
  HP_REQUIRE(capacity[q1] >= T1.size() / T1.dims[sh1] * Dn && capacity[q2] >= T2.size() / T2.dims[sh2] * Dn,
             HPEPS_ERR_SHAPE, "site buffers too small for the new bond");
  const int64_t cap = max_rank * max_rank * max_rank * max_rank * d;
  double* arena = (double*)take(2 * cap * sizeof(double));
  int* dims_dev = (int*)take(10 * sizeof(int));
  int* bond_dev = (int*)take(4 * sizeof(int));
  double* gate_dev = (double*)take((size_t)d * d * d * d * sizeof(double));
  double* sig = (double*)take(max_rank * sizeof(double));
  int hd[10], hb[4] = {0, 1, axis, 0};
  for (int e = 0; e < 5; ++e) {
    hd[e] = (int)T1.dims[e];
    hd[5 + e] = (int)T2.dims[e];
  }
  HP_CHECK_HIP(hipMemcpyAsync(arena, T1.p, T1.size() * 8, hipMemcpyDeviceToDevice, c.stream));
  HP_CHECK_HIP(hipMemcpyAsync(arena + cap, T2.p, T2.size() * 8, hipMemcpyDeviceToDevice, c.stream));
  HP_CHECK_HIP(hipMemcpyAsync(dims_dev, hd, sizeof(hd), hipMemcpyHostToDevice, c.stream));
  HP_CHECK_HIP(hipMemcpyAsync(bond_dev, hb, sizeof(hb), hipMemcpyHostToDevice, c.stream));
  HP_CHECK_HIP(hipMemcpyAsync(gate_dev, G, d * d * d * d * 8, hipMemcpyDeviceToDevice, c.stream));
  hp::IteArgs a{};
  a.sites = arena;
  a.cap = cap;
  a.dims = dims_dev;
  a.bonds = bond_dev;
  a.gates = gate_dev;
  a.dmax = (int)max_rank;
  a.sigma = sig;
  a.max_rows = (int)(max_rank * max_rank * max_rank);
  hp::launch_layer(c.stream, a, 1);
  HP_CHECK_HIP(hipGetLastError());
  int64_t* shp = const_cast<int64_t*>(peps->shapes);
  shp[5 * q1 + sh1] = Dn;
  shp[5 * q2 + sh2] = Dn;
  const int64_t n1 = T1.size() / T1.dims[sh1] * Dn, n2 = T2.size() / T2.dims[sh2] * Dn;
  HP_CHECK_HIP(hipMemcpyAsync(T1.p, arena, n1 * 8, hipMemcpyDeviceToDevice, c.stream));
  HP_CHECK_HIP(hipMemcpyAsync(T2.p, arena + cap, n2 * 8, hipMemcpyDeviceToDevice, c.stream));
  if (sigma_out)
    HP_CHECK_HIP(hipMemcpyAsync(sigma_out, sig, Dn * 8, hipMemcpyDeviceToDevice, c.stream));
  HP_CHECK_HIP(hipStreamSynchronize(c.stream));
  *new_bond = Dn;
}

// Device bytes gate_update takes for (max_rank, d), each piece 256-aligned.
size_t gate_scratch_bytes(int64_t max_rank, int d) {
  const size_t cap = (size_t)(max_rank * max_rank * max_rank * max_rank * d);
  return round256(2 * cap * sizeof(double)) + round256(10 * sizeof(int)) + round256(4 * sizeof(int)) +
         round256((size_t)d * d * d * d * sizeof(double)) + round256((size_t)max_rank * sizeof(double));
}

}  // namespace

namespace hp {
// Resolves this device's copy of the static gate scratch (the device must be
// current); idempotent.
void gate_scratch_init(int device) {
  HP_REQUIRE(device >= 0 && device < kMaxDevices, HPEPS_ERR_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  HP_CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  HP_REQUIRE(ptr != nullptr, HPEPS_ERR_HIP, "static gate scratch has no device address");
  g_scratch_ptr[device] = ptr;
}
}  // namespace hp

extern "C" {

hpeps_status hpeps_ite_plan_create(hpeps_ctx* ctx, const hpeps_peps* init, int32_t n_gates,
                                   const void* gates, const int32_t* bond_gate, int64_t max_rank,
                                   hpeps_ite_plan** out) {
  if (!ctx || !out) return HPEPS_ERR_INVALID_ARG;
  hp::Ctx& c = *ctx->impl;
  *out = nullptr;
  return guard_i(&c, [&] {
    HP_REQUIRE(gates && bond_gate && n_gates >= 1, HPEPS_ERR_INVALID_ARG, "null gates");
    hp::Lattice L = hp::lattice_from_abi(init);
    HP_REQUIRE(!L.cplx, HPEPS_ERR_DTYPE, "the batched QR-SVD sweep is FP64 real");
    const int d = (int)L.sites[0].dims[4];
    hp::check_dims(max_rank, d);
    for (auto& t : L.sites)
      for (int e = 0; e < 4; ++e) HP_REQUIRE(t.dims[e] <= max_rank, HPEPS_ERR_SHAPE, "initial bond exceeds max_rank");
    const auto ll = lattice_layers(L.nrow, L.ncol);
    std::vector<std::vector<Op>> layers(4);
    int q = 0;
    for (int l = 0; l < 4; ++l)
      for (auto& bd : ll[l]) {
        const int gi = bond_gate[q++];
        HP_REQUIRE(gi >= 0 && gi < n_gates, HPEPS_ERR_INVALID_ARG, "gate index out of range");
        layers[l].push_back(Op{false, bd[0], bd[1], bd[2], gi});
      }
    std::vector<double> g2((size_t)n_gates * d * d * d * d);
    HP_CHECK_HIP(hipMemcpy(g2.data(), gates, g2.size() * sizeof(double), hipMemcpyDeviceToHost));
    *out = build_plan(c, L, max_rank, layers, g2, {});
  });
}

hpeps_status hpeps_circuit_plan_create(hpeps_ctx* ctx, const hpeps_peps* init, int32_t n_gates2,
                                       const double* gates2, int32_t n_gates1, const double* gates1,
                                       int32_t n_ops, const int32_t* ops, int64_t max_rank,
                                       hpeps_ite_plan** out) {
  if (!ctx || !out) return HPEPS_ERR_INVALID_ARG;
  hp::Ctx& c = *ctx->impl;
  *out = nullptr;
  return guard_i(&c, [&] {
    HP_REQUIRE(n_gates2 >= 0 && n_gates1 >= 0 && n_ops >= 1 && ops, HPEPS_ERR_INVALID_ARG, "null operations");
    HP_REQUIRE((n_gates2 == 0 || gates2) && (n_gates1 == 0 || gates1), HPEPS_ERR_INVALID_ARG, "null gates");
    hp::Lattice L = hp::lattice_from_abi(init);
    HP_REQUIRE(!L.cplx, HPEPS_ERR_DTYPE, "the batched QR-SVD sweep is FP64 real");
    const int d = (int)L.sites[0].dims[4];
    hp::check_dims(max_rank, d);
    HP_REQUIRE(d <= 8, HPEPS_ERR_UNSUPPORTED, "one-site gates support d <= 8");
    for (auto& t : L.sites)
      for (int e = 0; e < 4; ++e) HP_REQUIRE(t.dims[e] <= max_rank, HPEPS_ERR_SHAPE, "initial bond exceeds max_rank");
    std::vector<double> g2(gates2, gates2 + (size_t)n_gates2 * d * d * d * d);
    std::vector<double> g1(gates1, gates1 + (size_t)n_gates1 * d * d);
    const auto layers = compile_ops(L.nrow, L.ncol, d, n_ops, ops, n_gates2, n_gates1, g2);
    *out = build_plan(c, L, max_rank, layers, g2, g1);
  });
}

hpeps_status hpeps_ite_plan_layers(hpeps_ite_plan* p, int32_t* n_layers, int32_t* n_bonds) {
  if (!p) return HPEPS_ERR_INVALID_ARG;
  if (n_layers) *n_layers = (int32_t)p->nb.size();
  if (n_bonds) *n_bonds = total_bonds(p);
  return HPEPS_OK;
}

hpeps_status hpeps_ite_run(hpeps_ite_plan* p, int32_t n_sweeps, int32_t use_graph) {
  if (!p || n_sweeps < 0 || use_graph < 0 || use_graph > 2) return HPEPS_ERR_INVALID_ARG;
  hp::Ctx& c = *p->ctx;
  return guard_i(&c, [&] {
    const int nl = (int)p->nb.size();
    auto sweep = [&](hipStream_t st) {
      for (int l = 0; l < nl; ++l) launch_any(p, st, l, hp::plan_args(p, l), p->nb[l]);
    };
    if (use_graph == 2) {
      // plain form: one launch per bond, no graph (the baseline the batched
      // layer launches and their graph replay are measured against)
      for (int s = 0; s < n_sweeps; ++s)
        for (int l = 0; l < nl; ++l) {
          hp::IteArgs a = hp::plan_args(p, l);
          for (int b = 0; b < p->nb[l]; ++b) {
            hp::IteArgs ab = a;
            ab.bonds = a.bonds + 4 * b;
            ab.sigma = p->onesite[l] ? a.sigma : a.sigma + (int64_t)b * p->dmax;
            launch_any(p, c.stream, l, ab, 1);
          }
        }
      HP_CHECK_HIP(hipGetLastError());
      return;
    }
    if (!use_graph) {
      for (int s = 0; s < n_sweeps; ++s) sweep(c.stream);
      HP_CHECK_HIP(hipGetLastError());
      return;
    }
    // the graph is captured on the plan's own stream (default priority) and
    // ordered after / before the context stream's work through events
    if (!p->exec) {
      HP_CHECK_HIP(hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking));
      HP_CHECK_HIP(hipEventCreateWithFlags(&p->ev[0], hipEventDisableTiming));
      HP_CHECK_HIP(hipEventCreateWithFlags(&p->ev[1], hipEventDisableTiming));
      HP_CHECK_HIP(hipStreamBeginCapture(p->gstream, hipStreamCaptureModeThreadLocal));
      sweep(p->gstream);
      HP_CHECK_HIP(hipStreamEndCapture(p->gstream, &p->graph));
      HP_CHECK_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    }
    HP_CHECK_HIP(hipEventRecord(p->ev[0], c.stream));
    HP_CHECK_HIP(hipStreamWaitEvent(p->gstream, p->ev[0], 0));
    for (int s = 0; s < n_sweeps; ++s) HP_CHECK_HIP(hipGraphLaunch(p->exec, p->gstream));
    HP_CHECK_HIP(hipEventRecord(p->ev[1], p->gstream));
    HP_CHECK_HIP(hipStreamWaitEvent(c.stream, p->ev[1], 0));
  });
}

hpeps_status hpeps_ite_get_state(hpeps_ite_plan* p, int64_t* shapes, void* const* sites) {
  if (!p || !shapes) return HPEPS_ERR_INVALID_ARG;
  hp::Ctx& c = *p->ctx;
  return guard_i(&c, [&] {
    const int ns = p->nrow * p->ncol;
    std::vector<int> dims(5 * ns);
    HP_CHECK_HIP(hipMemcpyAsync(dims.data(), p->dims, dims.size() * sizeof(int), hipMemcpyDeviceToHost, c.stream));
    HP_CHECK_HIP(hipStreamSynchronize(c.stream));
    for (int i = 0; i < 5 * ns; ++i) shapes[i] = dims[i];
    if (sites) {
      for (int s = 0; s < ns; ++s) {
        int64_t sz = 1;
        for (int e = 0; e < 5; ++e) sz *= dims[5 * s + e];
        HP_REQUIRE(sites[s], HPEPS_ERR_INVALID_ARG, "null site buffer");
        HP_CHECK_HIP(hipMemcpyAsync(sites[s], p->sites + (int64_t)s * p->cap, sz * sizeof(double),
                                    hipMemcpyDeviceToDevice, c.stream));
      }
      HP_CHECK_HIP(hipStreamSynchronize(c.stream));
    }
  });
}

hpeps_status hpeps_ite_spectra(hpeps_ite_plan* p, double* out) {
  if (!p || !out) return HPEPS_ERR_INVALID_ARG;
  hp::Ctx& c = *p->ctx;
  return guard_i(&c, [&] {
    const int total = total_bonds(p);
    HP_CHECK_HIP(hipMemcpyAsync(out, p->sigma, (size_t)total * p->dmax * sizeof(double), hipMemcpyDeviceToDevice,
                                c.stream));
  });
}

hpeps_status hpeps_ite_plan_destroy(hpeps_ite_plan* p) {
  if (!p) return HPEPS_ERR_INVALID_ARG;
  (void)hipStreamSynchronize(p->ctx->stream);
  free_plan(p);
  return HPEPS_OK;
}

hpeps_status hpeps_apply_one_site_gate(hpeps_ctx* ctx, hpeps_dtype dtype, const int64_t* dims, const void* site,
                                       const void* G, void* out) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  hp::Ctx& c = *ctx->impl;
  return guard_i(&c, [&] {
    c.ws_reset();
    HP_REQUIRE(dims && site && G && out, HPEPS_ERR_INVALID_ARG, "null argument");
    HP_REQUIRE(dtype == HPEPS_F64 || dtype == HPEPS_C128, HPEPS_ERR_DTYPE, "one-site gates run in FP64 / complex128");
    const bool cplx = dtype == HPEPS_C128;
    std::vector<int64_t> dv(dims, dims + 5);
    int64_t n = 1;
    for (auto x : dv) {
      HP_REQUIRE(x >= 1, HPEPS_ERR_SHAPE, "dimensions must be >= 1");
      n *= x;
    }
    const int64_t d = dv[4];
    // through the workspace, so that out may alias site
    void* tmp = c.ws<double>(n * (cplx ? 2 : 1));
    hp::contract2(c, cplx, hp::tview_rm(site, "udlrp", dv), hp::tview_rm(G, "Pp", {d, d}), "udlrP", tmp, n);
    HP_CHECK_HIP(hipMemcpyAsync(out, tmp, (size_t)n * (cplx ? 16 : 8), hipMemcpyDeviceToDevice, c.stream));
  });
}

hpeps_status hpeps_apply_two_site_gate(hpeps_ctx* ctx, hpeps_peps* peps, const int64_t* capacity, int32_t i,
                                       int32_t j, int32_t axis, const void* G, int64_t max_rank,
                                       int64_t* new_bond, double* sigma_out) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  hp::Ctx& c = *ctx->impl;
  return guard_i(&c, [&] {
    c.ws_reset();
    gate_update(c, peps, capacity, i, j, axis, G, max_rank, new_bond, sigma_out,
                [&](size_t bytes) { return (void*)c.ws<unsigned char>((int64_t)bytes); });
  });
}

hpeps_status hpeps_apply_two_site_gate_noalloc(hpeps_ctx* ctx, hpeps_peps* peps, const int64_t* capacity,
                                               int32_t i, int32_t j, int32_t axis, const void* G,
                                               int64_t max_rank, int64_t* new_bond, double* sigma_out) {
  if (!ctx) return HPEPS_ERR_INVALID_ARG;
  hp::Ctx& c = *ctx->impl;
  return guard_i(&c, [&] {
    HP_REQUIRE(max_rank >= 1 && peps && peps->nrow >= 1 && peps->ncol >= 1 && peps->shapes,
               HPEPS_ERR_INVALID_ARG, "bad lattice or max_rank");
    const int d = (int)peps->shapes[4];
    HP_REQUIRE(d >= 1, HPEPS_ERR_SHAPE, "bad physical dimension");
    hp::check_dims(max_rank, d);
    const size_t need = gate_scratch_bytes(max_rank, d);
    HP_REQUIRE(need <= kGateScratchBytes, HPEPS_ERR_ALLOC,
               "allocation-free gate update needs " + std::to_string(need) + " bytes of scratch, the static "
               "scratch holds " + std::to_string(kGateScratchBytes));
    void* base = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      base = g_scratch_ptr[c.device];
    }
    HP_REQUIRE(base, HPEPS_ERR_HIP, "static gate scratch not resolved for this device");
    size_t off = 0;
    gate_update(c, peps, capacity, i, j, axis, G, max_rank, new_bond, sigma_out, [&](size_t bytes) {
      void* p = (unsigned char*)base + off;
      off += round256(bytes);
      return p;
    });
  });
}

}  // extern "C"
