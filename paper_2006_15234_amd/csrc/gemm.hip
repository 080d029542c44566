// Gathered-operand batched GEMM on CDNA4 matrix cores.
//
// Every contraction of the method (the four stages of an implicit operator
// application A X / A^* Y, Gram matrices, triangular updates, factor
// products) is one call of
//
//   C[b][rC[m] + cC[n]] = s * sum_k A[b][rA[m] + cA[k]] * B[b][rB[k] + cB[n]]
//
// where rA, cA, ... are int32 offset tables, one entry per row / column index
// of the matricized operand.  A tensor contraction with any leg permutation
// is therefore a GEMM whose tile loads gather through the tables: no
// reshape/transpose kernels are ever launched (the GPU counterpart of the
// paper's reshape-avoiding design, Sec. V-C).
//
// Tiling: 256 threads = 4 wavefronts of 64 lanes; the block tile is
// (WM*TM*16) x (WN*TN*16) with K-steps of 16, each wavefront owns TM x TN
// 16x16 MFMA tiles (v_mfma_f64_16x16x4 for FP64 and complex128,
// v_mfma_f32_16x16x4 for FP32).  Operand tiles are staged through LDS with a
// register prefetch of the next K-step; the load mapping follows the
// contiguous direction of each operand so that global loads coalesce.
// Blocks are renumbered so that neighbouring tiles land on the same XCD
// (consecutive hardware block ids are dealt round-robin over the 8 XCDs).
#include <algorithm>
#include <climits>
#include <cmath>

#include "internal.h"

namespace hp {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

struct GemmArgs {
  const void* A;
  const void* B;
  void* C;
  const int* rA;
  const int* cA;
  const int* rB;
  const int* cB;
  const int* rC;
  const int* cC;
  long long sA, sB, sC;
  int M, N, K;
  int mtiles, ntiles, ntotal;
  int ksplit, kchunk;
  int conjA, conjB, conjC;
  int a_kfast, b_kfast;
  int accumulate;
  double alpha;
  const double* scale;
  const double* nscale;
  long long nscale_ld;
  const int* copy_if_zero;
  void* partial;
};

template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  using acc_t = v4d;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<float> {
  using acc_t = v4f;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// storage helpers -----------------------------------------------------------
template <class TC, bool CPLX>
struct Elem {
  TC re, im;
};

template <class TC, bool CPLX, class TIn>
__device__ __forceinline__ Elem<TC, CPLX> load_in(const TIn* p, long long off, bool conj) {
  Elem<TC, CPLX> e;
  if constexpr (CPLX) {
    const double2 v = reinterpret_cast<const double2*>(p)[off];
    e.re = (TC)v.x;
    e.im = conj ? (TC)(-v.y) : (TC)v.y;
  } else {
    e.re = (TC)p[off];
    e.im = (TC)0;
  }
  return e;
}

template <bool CPLX, class TOut>
__device__ __forceinline__ void store_out(TOut* C, long long off, double re, double im, bool acc) {
  if constexpr (CPLX) {
    double2* c = reinterpret_cast<double2*>(C) + off;
    if (acc) {
      double2 o = *c;
      re += o.x;
      im += o.y;
    }
    *c = make_double2(re, im);
  } else {
    if (acc) re += (double)C[off];
    C[off] = (TOut)re;
  }
}

template <class TC, bool CPLX, class TIn, class TOut>
__device__ __forceinline__ void epilogue(const GemmArgs& g, int b, int m, int n, double re,
                                         double im) {
  double s = g.alpha;
  if (g.scale) s *= g.scale[b];
  if (g.nscale) s *= g.nscale[(long long)b * g.nscale_ld + n];
  re *= s;
  im *= s;
  if (g.conjC) im = -im;
  TOut* C = reinterpret_cast<TOut*>(g.C) + (CPLX ? 0 : 0);
  long long off = (long long)b * g.sC + (long long)g.rC[m] + (long long)g.cC[n];
  store_out<CPLX, TOut>(C, off, re, im, g.accumulate != 0);
}

template <class TC, bool CPLX, class TIn, class TOut, int WM, int WN, int TM, int TN>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16, BK = 16;
  constexpr int LDA = BM + 1, LDB = BN + 1;
  constexpr int NA = BM * BK / 256, NB = BN * BK / 256;
  constexpr int NP = CPLX ? 2 : 1;
  using acc_t = typename Mfma<TC>::acc_t;

  __shared__ TC sA[NP][BK * LDA];
  __shared__ TC sB[NP][BK * LDB];

  // XCD-aware renumbering of the tile index (see header comment)
  const int nb = gridDim.x;
  const int bid = blockIdx.x;
  const int per = nb / 8;  // grid.x is padded to a multiple of 8
  const int tile = (bid % 8) * per + bid / 8;
  if (tile >= g.ntotal) return;
  const int mt = tile % g.mtiles, nt = tile / g.mtiles;
  const int bz = blockIdx.y;
  const int b = bz / g.ksplit, ks = bz % g.ksplit;
  const int m0 = mt * BM, n0 = nt * BN;
  const int tid = threadIdx.x;

  const TIn* A = reinterpret_cast<const TIn*>(g.A) + (CPLX ? 0 : 0);
  const TIn* B = reinterpret_cast<const TIn*>(g.B);
  const long long aoff = (long long)b * g.sA, boff = (long long)b * g.sB;

  if (g.copy_if_zero && g.copy_if_zero[b] == 0) {
    // pass-through: C[m, n] := A[m, n] (used when a factorization pass is skipped)
    for (int e = tid; e < BM * BN; e += 256) {
      const int m = m0 + e / BN, n = n0 + e % BN;
      if (m < g.M && n < g.N) {
        Elem<TC, CPLX> v = load_in<TC, CPLX, TIn>(A, aoff + g.rA[m] + g.cA[n], false);
        TOut* C = reinterpret_cast<TOut*>(g.C);
        store_out<CPLX, TOut>(C, (long long)b * g.sC + g.rC[m] + g.cC[n], (double)v.re,
                              (double)v.im, false);
      }
    }
    return;
  }

  const int kbeg = ks * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);

  // per-thread fixed row / column offsets of the elements this thread loads
  int a_mm[NA], a_kk[NA], a_roff[NA];
  int b_nn[NB], b_kk[NB], b_coff[NB];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int e = tid + i * 256;
    if (g.a_kfast) {
      a_kk[i] = e % BK;
      a_mm[i] = e / BK;
    } else {
      a_mm[i] = e % BM;
      a_kk[i] = e / BM;
    }
    const int m = m0 + a_mm[i];
    a_roff[i] = (m < g.M) ? g.rA[m] : -1;
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int e = tid + i * 256;
    if (g.b_kfast) {
      b_kk[i] = e % BK;
      b_nn[i] = e / BK;
    } else {
      b_nn[i] = e % BN;
      b_kk[i] = e / BN;
    }
    const int n = n0 + b_nn[i];
    b_coff[i] = (n < g.N) ? g.cB[n] : -1;
  }

  Elem<TC, CPLX> ra[NA], rb[NB];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int k = k0 + a_kk[i];
      if (a_roff[i] >= 0 && k < kend)
        ra[i] = load_in<TC, CPLX, TIn>(A, aoff + a_roff[i] + g.cA[k], g.conjA != 0);
      else
        ra[i].re = ra[i].im = (TC)0;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int k = k0 + b_kk[i];
      if (b_coff[i] >= 0 && k < kend)
        rb[i] = load_in<TC, CPLX, TIn>(B, boff + g.rB[k] + b_coff[i], g.conjB != 0);
      else
        rb[i].re = rb[i].im = (TC)0;
    }
  };

  acc_t acc[NP * NP][TM][TN];
#pragma unroll
  for (int c = 0; c < NP * NP; ++c)
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) acc[c][i][j] = acc_t{0, 0, 0, 0};

  const int wave = tid >> 6, lane = tid & 63;
  const int wm = wave % WM, wn = wave / WM;
  const int li = lane & 15, lk = lane >> 4;

  if (kbeg < kend) load_tiles(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      sA[0][a_kk[i] * LDA + a_mm[i]] = ra[i].re;
      if constexpr (CPLX) sA[NP - 1][a_kk[i] * LDA + a_mm[i]] = ra[i].im;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      sB[0][b_kk[i] * LDB + b_nn[i]] = rb[i].re;
      if constexpr (CPLX) sB[NP - 1][b_kk[i] * LDB + b_nn[i]] = rb[i].im;
    }
    __syncthreads();
    if (k0 + BK < kend) load_tiles(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      TC ar[TM], br[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) ar[i] = sA[0][(kk + lk) * LDA + wm * TM * 16 + i * 16 + li];
#pragma unroll
      for (int j = 0; j < TN; ++j) br[j] = sB[0][(kk + lk) * LDB + wn * TN * 16 + j * 16 + li];
      if constexpr (!CPLX) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[0][i][j] = Mfma<TC>::op(ar[i], br[j], acc[0][i][j]);
      } else {
        TC ai[TM], bi[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) ai[i] = sA[1][(kk + lk) * LDA + wm * TM * 16 + i * 16 + li];
#pragma unroll
        for (int j = 0; j < TN; ++j) bi[j] = sB[1][(kk + lk) * LDB + wn * TN * 16 + j * 16 + li];
        // acc[0] = Re*Re, acc[1] = Im*Im, acc[2] = Re*Im, acc[3] = Im*Re
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            acc[0][i][j] = Mfma<TC>::op(ar[i], br[j], acc[0][i][j]);
            acc[1][i][j] = Mfma<TC>::op(ai[i], bi[j], acc[1][i][j]);
            acc[2][i][j] = Mfma<TC>::op(ar[i], bi[j], acc[2][i][j]);
            acc[3][i][j] = Mfma<TC>::op(ai[i], br[j], acc[3][i][j]);
          }
      }
    }
  }

  // epilogue: accumulator register r of a lane holds column li of each 16x16
  // tile and row lk + 4 r (f64 MFMA) or 4 lk + r (f32 MFMA) -- measured layouts
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = (sizeof(TC) == 8) ? (lk + 4 * r) : (lk * 4 + r);
        const int m = m0 + wm * TM * 16 + i * 16 + row;
        const int n = n0 + wn * TN * 16 + j * 16 + li;
        if (m >= g.M || n >= g.N) continue;
        double re, im = 0.0;
        if constexpr (CPLX) {
          re = (double)acc[0][i][j][r] - (double)acc[1][i][j][r];
          im = (double)acc[2][i][j][r] + (double)acc[3][i][j][r];
        } else {
          re = (double)acc[0][i][j][r];
        }
        if (g.ksplit > 1) {
          double* P = reinterpret_cast<double*>(g.partial);
          const long long idx = (((long long)b * g.ksplit + ks) * g.M + m) * (long long)g.N + n;
          if constexpr (CPLX) {
            P[2 * idx] = re;
            P[2 * idx + 1] = im;
          } else {
            P[idx] = re;
          }
        } else {
          epilogue<TC, CPLX, TIn, TOut>(g, b, m, n, re, im);
        }
      }
}

// Sum of split-K partials followed by the epilogue (fixed order: deterministic).
template <bool CPLX, class TOut>
__global__ void splitk_reduce_kernel(GemmArgs g, int batch) {
  const long long MN = (long long)g.M * g.N;
  const long long total = MN * batch;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (long long)gridDim.x * blockDim.x) {
    const int b = (int)(t / MN);
    const long long mn = t % MN;
    const int m = (int)(mn / g.N), n = (int)(mn % g.N);
    const double* P = reinterpret_cast<const double*>(g.partial);
    double re = 0, im = 0;
    for (int s = 0; s < g.ksplit; ++s) {
      const long long idx = ((long long)b * g.ksplit + s) * MN + mn;
      if constexpr (CPLX) {
        re += P[2 * idx];
        im += P[2 * idx + 1];
      } else {
        re += P[idx];
      }
    }
    epilogue<double, CPLX, double, TOut>(g, b, m, n, re, im);
  }
}

// ---------------------------------------------------------------------------
// host side

namespace {

struct Cfg {
  int WM, WN, TM, TN;
  int BM() const { return WM * TM * 16; }
  int BN() const { return WN * TN * 16; }
};

// Tile shapes: a square default and skinny variants for the many products
// whose N (sketch width k <= 128) or M is small.
const Cfg kCfgs[] = {
    {2, 2, 2, 2},  // 64 x 64
    {4, 1, 2, 3},  // 128 x 48
    {4, 1, 2, 2},  // 128 x 32
    {1, 4, 3, 2},  // 48 x 128
    {2, 2, 2, 4},  // 64 x 128
};

int pick_cfg(int64_t M, int64_t N, bool cplx) {
  auto waste = [&](const Cfg& c) {
    const double bm = c.BM(), bn = c.BN();
    const double tm = std::ceil(M / bm) * bm, tn = std::ceil(N / bn) * bn;
    return (tm * tn) / double(M * N);
  };
  int best = 0;
  double bw = 1e30;
  for (int i = 0; i < 5; ++i) {
    // complex products keep four accumulator sets: only the 2x2-tile shapes fit
    if (cplx && kCfgs[i].TM * kCfgs[i].TN > 4) continue;
    // prefer larger tiles at equal waste (more reuse)
    const double w = waste(kCfgs[i]) * (1.0 + 0.02 * (4096.0 / (kCfgs[i].BM() * kCfgs[i].BN())));
    if (w < bw) {
      bw = w;
      best = i;
    }
  }
  return best;
}

template <class TC, bool CPLX, class TIn, class TOut>
void launch_cfg(int ci, dim3 grid, hipStream_t st, const GemmArgs& a) {
  switch (ci) {
    case 0: gemm_kernel<TC, CPLX, TIn, TOut, 2, 2, 2, 2><<<grid, 256, 0, st>>>(a); break;
    case 1: gemm_kernel<TC, CPLX, TIn, TOut, 4, 1, 2, 3><<<grid, 256, 0, st>>>(a); break;
    case 2: gemm_kernel<TC, CPLX, TIn, TOut, 4, 1, 2, 2><<<grid, 256, 0, st>>>(a); break;
    case 3: gemm_kernel<TC, CPLX, TIn, TOut, 1, 4, 3, 2><<<grid, 256, 0, st>>>(a); break;
    default: gemm_kernel<TC, CPLX, TIn, TOut, 2, 2, 2, 4><<<grid, 256, 0, st>>>(a); break;
  }
}

bool innermost_is_k(const IndexMap& mm, const IndexMap& kk) {
  // the operand is "k-fast" when its smallest stride belongs to a K mode
  int64_t sm = INT64_MAX, sk = INT64_MAX;
  for (int i = 0; i < mm.n; ++i)
    if (mm.dim[i] > 1) sm = std::min(sm, mm.stride[i]);
  for (int i = 0; i < kk.n; ++i)
    if (kk.dim[i] > 1) sk = std::min(sk, kk.stride[i]);
  return sk < sm;
}

}  // namespace

void gemm(Ctx& ctx, Prec prec, const GemmDesc& d, const GemmCall& c) {
  if (d.M <= 0 || d.N <= 0) return;
  HP_REQUIRE(d.M < (1LL << 31) && d.N < (1LL << 31) && d.K < (1LL << 31), HPEPS_ERR_UNSUPPORTED,
             "gemm dimension exceeds int32");
  // host-side bounds check of every gathered access (index maps vs extents)
  auto maxoff = [](const IndexMap& a, const IndexMap& b) {
    int64_t o = 0;
    for (int i = 0; i < a.n; ++i) o += (a.dim[i] - 1) * a.stride[i];
    for (int i = 0; i < b.n; ++i) o += (b.dim[i] - 1) * b.stride[i];
    return o;
  };
  HP_REQUIRE(d.Am.size() == d.M && d.Cm.size() == d.M && d.Bn.size() == d.N && d.Cn.size() == d.N &&
                 d.Ak.size() == d.K && d.Bk.size() == d.K,
             HPEPS_ERR_SHAPE, "gemm index maps disagree with M/N/K");
  // instances are contiguous blocks: the batch stride is the extent unless given
  const int64_t nA = c.nA ? c.nA : c.sA, nB = c.nB ? c.nB : c.sB, nC = c.nC ? c.nC : c.sC;
  HP_REQUIRE(nA > 0 && maxoff(d.Am, d.Ak) < nA, HPEPS_ERR_SHAPE, "gemm A access out of bounds");
  HP_REQUIRE(nB > 0 && maxoff(d.Bk, d.Bn) < nB, HPEPS_ERR_SHAPE, "gemm B access out of bounds");
  HP_REQUIRE(nC > 0 && maxoff(d.Cm, d.Cn) < nC, HPEPS_ERR_SHAPE, "gemm C access out of bounds");
  if (c.copy_if_zero) HP_REQUIRE(d.K == d.N, HPEPS_ERR_SHAPE, "pass-through gemm needs K == N");
  GemmArgs a{};
  a.A = c.A;
  a.B = c.B;
  a.C = c.C;
  a.rA = ctx.table(d.Am);
  a.cA = ctx.table(d.Ak);
  a.rB = ctx.table(d.Bk);
  a.cB = ctx.table(d.Bn);
  a.rC = ctx.table(d.Cm);
  a.cC = ctx.table(d.Cn);
  a.sA = c.sA;
  a.sB = c.sB;
  a.sC = c.sC;
  a.M = (int)d.M;
  a.N = (int)d.N;
  a.K = (int)d.K;
  a.conjA = c.conjA;
  a.conjB = c.conjB;
  a.conjC = c.conjC;
  a.a_kfast = innermost_is_k(d.Am, d.Ak);
  a.b_kfast = innermost_is_k(d.Bn, d.Bk);
  a.accumulate = c.accumulate;
  a.alpha = c.alpha;
  a.scale = c.scale;
  a.nscale = c.nscale;
  a.nscale_ld = c.nscale_ld;
  a.copy_if_zero = c.copy_if_zero;

  const int ci = pick_cfg(d.M, d.N, prec == Prec::C128);
  const Cfg cf = kCfgs[ci];
  a.mtiles = (int)cdiv(d.M, cf.BM());
  a.ntiles = (int)cdiv(d.N, cf.BN());
  a.ntotal = a.mtiles * a.ntiles;

  // split K when the tile grid alone cannot fill the 256 CUs
  int ksplit = 1;
  const int64_t blocks = (int64_t)a.ntotal * c.batch;
  if (blocks < 512 && d.K > 256 && !c.copy_if_zero) {
    ksplit = (int)std::min<int64_t>((1024 + blocks - 1) / blocks, (d.K + 255) / 256);
    ksplit = std::max(1, std::min(ksplit, 4096 / std::max(1, c.batch)));
  }
  int kchunk = (int)d.K;
  if (ksplit > 1) {
    kchunk = (int)(((d.K + ksplit - 1) / ksplit + 15) / 16 * 16);
    ksplit = (int)((d.K + kchunk - 1) / kchunk);
  }
  a.ksplit = ksplit;
  a.kchunk = std::max(kchunk, 1);
  const bool cplx = prec == Prec::C128;
  if (ksplit > 1) {
    a.partial = ctx.ws_alloc((int64_t)c.batch * ksplit * d.M * d.N * (cplx ? 16 : 8));
  }
  HP_REQUIRE(c.batch * ksplit < 65536, HPEPS_ERR_UNSUPPORTED, "gemm batch too large");
  const unsigned gx = ((unsigned)a.ntotal + 7) / 8 * 8;
  dim3 grid(gx, (unsigned)(c.batch * ksplit));
  hipStream_t st = ctx.stream;
  int rec = -1;
  if (ctx.prof_on) {
    static const char* pn[] = {"f64", "c128", "f32"};
    const std::string name = std::string("gemm_") + pn[(int)prec] +
                             (prec == Prec::F32 && !c.out_f64 ? "o32" : "") + "_" +
                             std::to_string(cf.BM()) + "x" + std::to_string(cf.BN());
    rec = ctx.prof_begin(name);
  }
  switch (prec) {
    case Prec::F64:
      launch_cfg<double, false, double, double>(ci, grid, st, a);
      if (ksplit > 1)
        splitk_reduce_kernel<false, double><<<1024, 256, 0, st>>>(a, c.batch);
      break;
    case Prec::C128:
      launch_cfg<double, true, double, double>(ci, grid, st, a);
      if (ksplit > 1)
        splitk_reduce_kernel<true, double><<<1024, 256, 0, st>>>(a, c.batch);
      break;
    case Prec::F32:
      if (c.out_f64) {
        launch_cfg<float, false, float, double>(ci, grid, st, a);
        if (ksplit > 1) splitk_reduce_kernel<false, double><<<1024, 256, 0, st>>>(a, c.batch);
      } else {
        launch_cfg<float, false, float, float>(ci, grid, st, a);
        if (ksplit > 1) splitk_reduce_kernel<false, float><<<1024, 256, 0, st>>>(a, c.batch);
      }
      break;
  }
  HP_CHECK_HIP(hipGetLastError());
  if (rec >= 0) {
    // algorithmic work of the product: 2 M N K per instance (complex: 4 real
    // products per multiply-add); bytes: each operand element once
    const double mnk = 2.0 * (double)d.M * (double)d.N * (double)d.K * c.batch * (cplx ? 4 : 1);
    const double elt = prec == Prec::F32 ? 4.0 : (cplx ? 16.0 : 8.0);
    const double byt = ((double)d.M * d.K + (double)d.K * d.N + (double)d.M * d.N) * c.batch * elt;
    ctx.prof_end(rec, mnk, byt);
  }
}

}  // namespace hp
