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
// (WM*TM*16) x (WN*TN*16) with K-steps of 16*KS, each wavefront owns TM x TN
// 16x16 MFMA tiles (v_mfma_f64_16x16x4 for FP64 and complex128,
// v_mfma_f32_16x16x4 for FP32).
//  * LDS holds both operand tiles k-contiguous ([row][k], rows padded by 16
//    bytes so that the 16 rows one MFMA reads fall in distinct bank groups).
//    Lane (i, q) of a wavefront feeds the MFMA sub-steps of a K-step with the
//    k values 4 KS q .. 4 KS q + 4 KS - 1 of its row, fetched with 128-bit LDS
//    reads; A and B use the same k assignment, so the product is unchanged.
//  * Two LDS stages: the global loads of K-step t+1 are in flight in
//    registers while step t computes, then land in the other stage; one
//    barrier per K-step.
//  * K offsets: affine K index maps are computed (k * step); general ones
//    are staged from their table into LDS once per block.
//  * Work items (tile, K-split part, instance) are dealt to the 8 XCDs in
//    contiguous ranges (consecutive hardware block ids go round-robin over
//    the XCDs), so the tiles of one instance share an L2, and no XCD is left
//    without work when the tile count is not a multiple of 8.
// The tile shape, K-step and split-K count of each product come from a size
// heuristic or from the autotuner, which times every variant on the first
// product of a new shape/layout key and caches the winner (JSON export and
// import through the C ABI).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <tuple>
#include <type_traits>

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
  int mtiles, ntotal;   // tiles of one instance
  int ksplit, kchunk;
  int nwork, per_xcd;   // ntotal * batch * ksplit work items; ceil(nwork / 8)
  int conjA, conjB, conjC;
  int a_kfast, b_kfast;
  int tabA, tabB;       // K offsets from LDS tables (else k * step)
  int a_kstep, b_kstep;
  int accumulate;
  int rA_step, cB_step, rC_step, cC_step;  // row / column offsets m * step (-1: from the table;
                                           // affine maps skip the dependent table load)
  double alpha;
  const double* scale;
  const double* nscale;
  long long nscale_ld;
  const int* copy_if_zero;
  const int* skip_if_zero;
  void* partial;
  unsigned nA_bytes, nB_bytes;  // per-instance operand extents (buffer ranges)
};

template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  using acc_t = v4d;
  static constexpr int kvals = 1;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // four consecutive values of a 16-byte aligned LDS row
  static __device__ __forceinline__ void quad(const double* p, double* v) {
    const double2 x = reinterpret_cast<const double2*>(p)[0];
    const double2 y = reinterpret_cast<const double2*>(p)[1];
    v[0] = x.x;
    v[1] = x.y;
    v[2] = y.x;
    v[3] = y.y;
  }
};
template <>
struct Mfma<float> {
  using acc_t = v4f;
  static constexpr int kvals = 1;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ void quad(const float* p, float* v) {
    const float4 x = reinterpret_cast<const float4*>(p)[0];
    v[0] = x.x;
    v[1] = x.y;
    v[2] = x.z;
    v[3] = x.w;
  }
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
template <>
struct Mfma<__bf16> {
  using acc_t = v4f;
  // v_mfma_f32_16x16x32_bf16: each lane supplies 8 consecutive k of its row
  static constexpr int kvals = 8;
  static __device__ __forceinline__ acc_t op8(const __bf16* a, const __bf16* b, acc_t c) {
    bf16x8 av, bv;
    __builtin_memcpy(&av, a, 16);
    __builtin_memcpy(&bv, b, 16);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  }
};

// N consecutive values of a 16-byte aligned LDS row, as 128-bit reads
template <class T, int N>
__device__ __forceinline__ void lds_read(const T* p, T* v) {
  static_assert((N * sizeof(T)) % 16 == 0, "whole 16-byte chunks");
#pragma unroll
  for (int c = 0; c < (int)(N * sizeof(T) / 16); ++c) {
    const float4 x = reinterpret_cast<const float4*>(p)[c];
    __builtin_memcpy(v + c * (16 / sizeof(T)), &x, 16);
  }
}

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

typedef double d2v __attribute__((ext_vector_type(2)));

// One element through a buffer resource (byte offset; zero when past the
// extent).  Complex values are (re, im) double pairs.
template <class TC, bool CPLX, class TIn>
__device__ __forceinline__ Elem<TC, CPLX> buf_load(__amdgpu_buffer_rsrc_t r, unsigned off,
                                                   unsigned soff = 0) {
  Elem<TC, CPLX> e;
  if constexpr (CPLX) {
    const d2v v = __builtin_bit_cast(d2v, __builtin_amdgcn_raw_buffer_load_b128(r, off, soff, 0));
    e.re = (TC)v[0];
    e.im = (TC)v[1];
  } else if constexpr (sizeof(TIn) == 8) {
    e.re = (TC)__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
    e.im = (TC)0;
  } else if constexpr (sizeof(TIn) == 2) {
    e.re = (TC)__builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0));
    e.im = (TC)0;
  } else {
    e.re = (TC)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
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
    if constexpr (sizeof(TOut) == 8)
      C[off] = (TOut)re;
    else
      C[off] = (TOut)(float)re;
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
  TOut* C = reinterpret_cast<TOut*>(g.C);
  long long off = (long long)b * g.sC + (long long)g.rC[m] + (long long)g.cC[n];
  store_out<CPLX, TOut>(C, off, re, im, g.accumulate != 0);
}

// Tile position of element e for an operand whose rows (M or N index) are
// contiguous in memory: each group of 16 lanes reads 16 consecutive rows
// (one 128-byte line) at one k, the four groups of a wavefront take four
// consecutive k.  In the k-contiguous LDS tile ([row][k], row pitch an odd
// multiple of 16 bytes) the 64-bit writes of each half-wavefront then hit
// distinct banks.
template <int R>
__device__ __forceinline__ void tile_pos(int e, int& row, int& kk) {
  const int li = e & 15, grp = (e >> 4) & 3, rest = e >> 6;
  row = (rest % (R / 16)) * 16 + li;
  kk = (rest / (R / 16)) * 4 + grp;
}

// One work item w (tile, K-split part, instance) of the product.
template <class TC, bool CPLX, class TIn, class TOut, int WM, int WN, int TM, int TN, int KS>
__device__ __forceinline__ void gemm_item(const GemmArgs& g, int w, unsigned char* smem_raw) {
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16, BK = 16 * KS;
  constexpr int LDK = BK + 16 / (int)sizeof(TC);  // row pitch (elements), odd multiple of 16 B
  constexpr int NA = BM * BK / 256, NB = BN * BK / 256;  // elements each thread loads per K-step
  constexpr int KQ = 4 * KS;                              // k values per lane and row per K-step
  constexpr int NP = CPLX ? 2 : 1;
  constexpr int SA = BM * LDK, SB = BN * LDK;
  constexpr int STAGE = NP * (SA + SB);
  using acc_t = typename Mfma<TC>::acc_t;

  TC* sbuf = reinterpret_cast<TC*>(smem_raw);
  int* sKA = reinterpret_cast<int*>(sbuf + 2 * STAGE);
  int* sKB = sKA + (g.tabA ? g.kchunk : 0);

  const int tile = w % g.ntotal;
  const int rest = w / g.ntotal;
  const int ks = rest % g.ksplit, b = rest / g.ksplit;
  const int mt = tile % g.mtiles, nt = tile / g.mtiles;
  const int m0 = mt * BM, n0 = nt * BN;
  const int tid = threadIdx.x;

  const TIn* A = reinterpret_cast<const TIn*>(g.A);
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
  if (g.skip_if_zero && g.skip_if_zero[b] == 0) return;  // whole block: b is per work item

  const int kbeg = ks * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  // staged K tables, zero-padded to the chunk length so that every table
  // read of the loop below stays in range
  if (g.tabA)
    for (int t = tid; t < g.kchunk; t += 256) sKA[t] = kbeg + t < kend ? g.cA[kbeg + t] : 0;
  if (g.tabB)
    for (int t = tid; t < g.kchunk; t += 256) sKB[t] = kbeg + t < kend ? g.rB[kbeg + t] : 0;

  // Buffer resources over this instance's operands.  A load whose byte
  // offset lies past the extent returns zero: ragged tile edges and the K
  // tail are padded by giving such elements the offset 0xffffffff, without
  // branches.
  constexpr unsigned ELT = CPLX ? 16u : (unsigned)sizeof(TIn);
  constexpr unsigned kOut = 0xffffffffu;
  const auto rsA = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char*>(reinterpret_cast<const char*>(g.A) + aoff * ELT), (short)0, (int)g.nA_bytes,
      0x00020000);
  const auto rsB = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char*>(reinterpret_cast<const char*>(g.B) + boff * ELT), (short)0, (int)g.nB_bytes,
      0x00020000);

  // (row, k) position of element i of this thread in a K-step tile; the
  // mapping follows the contiguous direction of each operand so that global
  // loads coalesce.  Kept per element: the LDS slot row * LDK + kk (row and
  // kk are recovered from it on the slow paths) and the byte offset of
  // (row, kk) at k = 0.
  int a_lds[NA], b_lds[NB];
  unsigned a_base[NA], b_base[NB];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int e = tid + i * 256;
    int row, kk;
    if (g.a_kfast) {
      kk = e % BK;
      row = e / BK;
    } else {
      tile_pos<BM>(e, row, kk);
    }
    a_lds[i] = row * LDK + kk;
    const int m = m0 + row;
    const int roff = (m < g.M) ? (g.rA_step >= 0 ? m * g.rA_step : g.rA[m]) : 0;
    // rows past M read row 0 instead (those accumulator rows are never
    // stored); with K offset tables a_kstep is 0 and this is the row offset
    a_base[i] = (unsigned)(roff + kk * g.a_kstep) * ELT;
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int e = tid + i * 256;
    int col, kk;
    if (g.b_kfast) {
      kk = e % BK;
      col = e / BK;
    } else {
      tile_pos<BN>(e, col, kk);
    }
    b_lds[i] = col * LDK + kk;
    const int n = n0 + col;
    const int coff = (n < g.N) ? (g.cB_step >= 0 ? n * g.cB_step : g.cB[n]) : 0;
    b_base[i] = (unsigned)(coff + kk * g.b_kstep) * ELT;
  }
  // row (or column) of a tile and k within the step, from an LDS slot
  auto slot_rk = [](int slot, int& r, int& kk) {
    r = slot / LDK;
    kk = slot - r * LDK;
  };

  Elem<TC, CPLX> ra[NA], rb[NB];
  // K-step starting at k0.  A full step of an affine operand needs no
  // per-element arithmetic: the k offset goes into the scalar offset of the
  // buffer load.  The partial last step and table-gathered operands check
  // every element (k past the end reads zero).
  auto load_global = [&](int k0, bool full) {
    if (!g.tabA && full) {
      const unsigned so = (unsigned)(k0 * g.a_kstep) * ELT;
#pragma unroll
      for (int i = 0; i < NA; ++i) ra[i] = buf_load<TC, CPLX, TIn>(rsA, a_base[i], so);
    } else if (g.tabA) {
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        int row, kk;
        slot_rk(a_lds[i], row, kk);
        const int k = k0 + kk;
        const int ko = sKA[k - kbeg];
        const bool ok = (m0 + row < g.M) & (k < kend);
        ra[i] = buf_load<TC, CPLX, TIn>(rsA, ok ? a_base[i] + (unsigned)ko * ELT : kOut);
      }
    } else {
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        int row, kk;
        slot_rk(a_lds[i], row, kk);
        const bool ok = (m0 + row < g.M) & (k0 + kk < kend);
        ra[i] = buf_load<TC, CPLX, TIn>(rsA, ok ? a_base[i] + (unsigned)(k0 * g.a_kstep) * ELT : kOut);
      }
    }
    if (!g.tabB && full) {
      const unsigned so = (unsigned)(k0 * g.b_kstep) * ELT;
#pragma unroll
      for (int i = 0; i < NB; ++i) rb[i] = buf_load<TC, CPLX, TIn>(rsB, b_base[i], so);
    } else if (g.tabB) {
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        int col, kk;
        slot_rk(b_lds[i], col, kk);
        const int k = k0 + kk;
        const int ko = sKB[k - kbeg];
        const bool ok = (n0 + col < g.N) & (k < kend);
        rb[i] = buf_load<TC, CPLX, TIn>(rsB, ok ? b_base[i] + (unsigned)ko * ELT : kOut);
      }
    } else {
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        int col, kk;
        slot_rk(b_lds[i], col, kk);
        const bool ok = (n0 + col < g.N) & (k0 + kk < kend);
        rb[i] = buf_load<TC, CPLX, TIn>(rsB, ok ? b_base[i] + (unsigned)(k0 * g.b_kstep) * ELT : kOut);
      }
    }
  };
  auto store_lds = [&](auto stage_c) {
    constexpr int stage = decltype(stage_c)::value;
    TC* sa = sbuf + stage * STAGE;
    TC* sb = sa + NP * SA;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      sa[a_lds[i]] = ra[i].re;
      if constexpr (CPLX) sa[SA + a_lds[i]] = g.conjA ? -ra[i].im : ra[i].im;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      sb[b_lds[i]] = rb[i].re;
      if constexpr (CPLX) sb[SB + b_lds[i]] = g.conjB ? -rb[i].im : rb[i].im;
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

  auto compute = [&](auto stage_c) {
    constexpr int stage = decltype(stage_c)::value;
    constexpr int KV = Mfma<TC>::kvals;  // k values per lane per MFMA
    const TC* sa = sbuf + stage * STAGE + (wm * TM * 16 + li) * LDK + lk * KQ;
    const TC* sb = sbuf + stage * STAGE + NP * SA + (wn * TN * 16 + li) * LDK + lk * KQ;
    TC ar[TM][KQ], br[TN][KQ];
#pragma unroll
    for (int i = 0; i < TM; ++i) lds_read<TC, KQ>(sa + i * 16 * LDK, ar[i]);
#pragma unroll
    for (int j = 0; j < TN; ++j) lds_read<TC, KQ>(sb + j * 16 * LDK, br[j]);
    if constexpr (KV > 1) {
#pragma unroll
      for (int s8 = 0; s8 < KQ; s8 += KV)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[0][i][j] = Mfma<TC>::op8(&ar[i][s8], &br[j][s8], acc[0][i][j]);
    } else if constexpr (!CPLX) {
#pragma unroll
      for (int s = 0; s < KQ; ++s)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[0][i][j] = Mfma<TC>::op(ar[i][s], br[j][s], acc[0][i][j]);
    } else {
      TC ai[TM][KQ], bi[TN][KQ];
#pragma unroll
      for (int i = 0; i < TM; ++i) lds_read<TC, KQ>(sa + SA + i * 16 * LDK, ai[i]);
#pragma unroll
      for (int j = 0; j < TN; ++j) lds_read<TC, KQ>(sb + SB + j * 16 * LDK, bi[j]);
      // acc[0] = Re*Re, acc[1] = Im*Im, acc[2] = Re*Im, acc[3] = Im*Re
#pragma unroll
      for (int s = 0; s < KQ; ++s)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            acc[0][i][j] = Mfma<TC>::op(ar[i][s], br[j][s], acc[0][i][j]);
            acc[1][i][j] = Mfma<TC>::op(ai[i][s], bi[j][s], acc[1][i][j]);
            acc[2][i][j] = Mfma<TC>::op(ar[i][s], bi[j][s], acc[2][i][j]);
            acc[3][i][j] = Mfma<TC>::op(ai[i][s], br[j][s], acc[3][i][j]);
          }
    }
  };

  // K-steps t = 0 .. nsteps-1 alternate between the two LDS stages (t % 2);
  // the loop is unrolled by two so that stage offsets are immediates
  const std::integral_constant<int, 0> st0;
  const std::integral_constant<int, 1> st1;
  const int nsteps = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  const bool last_full = (kend - kbeg) % BK == 0;
  auto full = [&](int t) { return t < nsteps - 1 || last_full; };
  __syncthreads();  // K offset tables staged
  if (nsteps > 0) {
    load_global(kbeg, full(0));
    store_lds(st0);
  }
  __syncthreads();
  int t = 0;
  // The scheduling barriers keep the LDS stores (which wait for the global
  // loads) behind the MFMAs of the step, so that the loads are in flight
  // while the step computes.
  for (; t + 1 < nsteps; t += 2) {
    load_global(kbeg + (t + 1) * BK, full(t + 1));
    compute(st0);
    __builtin_amdgcn_sched_barrier(0);
    store_lds(st1);
    __syncthreads();
    const bool more = t + 2 < nsteps;
    if (more) load_global(kbeg + (t + 2) * BK, full(t + 2));
    compute(st1);
    __builtin_amdgcn_sched_barrier(0);
    if (more) store_lds(st0);
    __syncthreads();
  }
  if (t < nsteps) compute(st0);

  // epilogue: accumulator register r of a lane holds column li of each 16x16
  // tile and row lk + 4 r (f64 MFMA) or 4 lk + r (f32 MFMA) -- measured layouts
  auto acc_val = [&](int i, int j, int r, double& re, double& im) {
    if constexpr (CPLX) {
      re = (double)acc[0][i][j][r] - (double)acc[1][i][j][r];
      im = (double)acc[2][i][j][r] + (double)acc[3][i][j][r];
    } else {
      re = (double)acc[0][i][j][r];
      im = 0.0;
    }
  };
  if (g.ksplit > 1) {
    double* P = reinterpret_cast<double*>(g.partial);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = (sizeof(TC) == 8) ? (lk + 4 * r) : (lk * 4 + r);  // f64 / f32-accumulator layouts
          const int m = m0 + wm * TM * 16 + i * 16 + row;
          const int n = n0 + wn * TN * 16 + j * 16 + li;
          if (m >= g.M || n >= g.N) continue;
          double re, im;
          acc_val(i, j, r, re, im);
          const long long idx = (((long long)b * g.ksplit + ks) * g.M + m) * (long long)g.N + n;
          if constexpr (CPLX) {
            P[2 * idx] = re;
            P[2 * idx + 1] = im;
          } else {
            P[idx] = re;
          }
        }
    return;
  }
  // column offsets and column scales of this lane's outputs, loaded once
  int coff[TN];
  double cs[TN];
  const double sb = g.alpha * (g.scale ? g.scale[b] : 1.0);
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = n0 + wn * TN * 16 + j * 16 + li;
    coff[j] = n < g.N ? (g.cC_step >= 0 ? n * g.cC_step : g.cC[n]) : -1;
    cs[j] = (g.nscale && n < g.N) ? sb * g.nscale[(long long)b * g.nscale_ld + n] : sb;
  }
  TOut* Cb = reinterpret_cast<TOut*>(g.C);
  const long long cbase = (long long)b * g.sC;
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = (sizeof(TC) == 8) ? (lk + 4 * r) : (lk * 4 + r);  // f64 / f32-accumulator layouts
      const int m = m0 + wm * TM * 16 + i * 16 + row;
      const int roff = m < g.M ? (g.rC_step >= 0 ? m * g.rC_step : g.rC[m]) : -1;
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        if (roff < 0 || coff[j] < 0) continue;
        double re, im;
        acc_val(i, j, r, re, im);
        re *= cs[j];
        im *= cs[j];
        if (g.conjC) im = -im;
        store_out<CPLX, TOut>(Cb, cbase + roff + coff[j], re, im, g.accumulate != 0);
      }
    }
}

// Occupancy hint (waves per SIMD) for the register allocator: the real FP64
// shapes below fit that many waves without spilling, which the allocator
// does not find by itself (128 x 48: 3 instead of 2 waves; 64 x 64: 4
// instead of 3).  Everything else keeps the default.
template <class TC, bool CPLX, int WM, int WN, int TM, int TN, int KS>
constexpr int gemm_waves() {
  if (!std::is_same<TC, double>::value || CPLX || KS != 1) return 1;
  if (TM * TN == 6) return 3;
  if (WM == 2 && WN == 2 && TM == 2 && TN == 2) return 4;
  return 1;
}

// Work items are dealt to the XCDs in contiguous ranges: XCD x = blockIdx % 8
// (consecutive hardware block ids go round-robin over the XCDs) owns items
// [x per_xcd, (x + 1) per_xcd), one per block.
template <class TC, bool CPLX, class TIn, class TOut, int WM, int WN, int TM, int TN, int KS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(gemm_waves<TC, CPLX, WM, WN, TM, TN, KS>())))
void gemm_kernel(GemmArgs g) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int w = (int)(blockIdx.x & 7) * g.per_xcd + (int)(blockIdx.x >> 3);
  if (w < g.nwork) gemm_item<TC, CPLX, TIn, TOut, WM, WN, TM, TN, KS>(g, w, smem_raw);
}

// Products with a short reduction (K <= 16; real, N >= 72, C columns in
// contiguous runs of VN) are bound by writing C: a
// K-deep MFMA step would be mostly padding, and the tile epilogue stores
// 8-byte pieces.  Here each thread owns VN consecutive columns (8 or 16
// bytes of C), holds their K values of B in registers, and sweeps up to
// kSkRows rows whose K values of A sit in LDS (B is read once per row group),
// so every row is one vector store per thread.  Work items (row group, column chunk,
// instance) are dealt to the XCDs as in gemm_kernel.
constexpr int kSkRows = 128;  // rows per work item (all rows of most products: B is read once)

// columns per thread: 16 bytes of FP64 or FP32 output, 8 bytes of BF16 output
// (the sketch width k, the fastest output leg, is then a multiple of 4)
template <class T>
struct SkCols;
template <>
struct SkCols<double> {
  static constexpr int n = 2;
};
template <>
struct SkCols<float> {
  static constexpr int n = 4;
};
template <>
struct SkCols<__bf16> {
  static constexpr int n = 4;
};

// Template arguments of a short-reduction / few-rows kernel, so that the
// launchers name the kernel at the launch (never through a pointer to it).
template <class TIn, class TAcc, class TOut, int N>
struct KTag {
  using In = TIn;
  using Acc = TAcc;
  using Out = TOut;
  static constexpr int n = N;
};

template <class TIn, class TC, class TOut, int KMAX>
__global__ __launch_bounds__(256) void smallk_kernel(GemmArgs g, int nchunks, int mgroups, int gpr) {
  constexpr int VN = SkCols<TOut>::n;
  constexpr int VB = VN * (int)sizeof(TOut);  // bytes per store
  __shared__ TC sA[kSkRows * KMAX];
  const int w = (int)(blockIdx.x & 7) * g.per_xcd + (int)(blockIdx.x >> 3);
  if (w >= g.nwork) return;
  const int chunk = w % nchunks, rest = w / nchunks;
  const int mg = rest % mgroups, b = rest / mgroups;
  const int m0 = mg * kSkRows, tid = threadIdx.x;
  const TIn* A = reinterpret_cast<const TIn*>(g.A) + (long long)b * g.sA;
  const TIn* B = reinterpret_cast<const TIn*>(g.B) + (long long)b * g.sB;
  // A[m0 .. m0 + kSkRows) x K (zero past the ends); every load is issued
  // before the first LDS store
  constexpr int IA = kSkRows * KMAX / 256;
  TC av[IA];
#pragma unroll
  for (int it = 0; it < IA; ++it) {
    const int e = tid + 256 * it, r = e / KMAX, k = e - r * KMAX, m = m0 + r;
    TC v = (TC)0;
    if (m < g.M && k < g.K) {
      const int ro = g.rA_step >= 0 ? m * g.rA_step : g.rA[m];
      const int ko = g.tabA ? g.cA[k] : k * g.a_kstep;
      v = (TC)A[ro + ko];
    }
    av[it] = v;
  }
#pragma unroll
  for (int it = 0; it < IA; ++it) sA[tid + 256 * it] = av[it];
  // C row offsets of the work item's rows (a gathered map costs one load each)
  __shared__ int sRC[kSkRows];
  if (tid < kSkRows) {
    const int m = m0 + tid;
    sRC[tid] = m < g.M ? (g.rC_step >= 0 ? m * g.rC_step : g.rC[m]) : 0;
  }
  // the thread's column group (gpr groups of VN columns per pass over the
  // rows; 256 / gpr rows per pass when the rows are narrower than 256 groups)
  const int rpp = 256 / gpr, grp = tid % gpr, rsub = tid / gpr;
  // B at this thread's columns, all k
  const int n0 = (chunk * gpr + grp) * VN;
  TC bv[KMAX][VN];
  double cs[VN];
  const double sb = g.alpha * (g.scale ? g.scale[b] : 1.0);
#pragma unroll
  for (int v = 0; v < VN; ++v) {
    const int n = n0 + v;
    const bool in = n < g.N;
    const int co = in ? (g.cB_step >= 0 ? n * g.cB_step : g.cB[n]) : 0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int ko = k < g.K ? (g.tabB ? g.rB[k] : k * g.b_kstep) : 0;
      bv[k][v] = (in && k < g.K) ? (TC)B[ko + co] : (TC)0;
    }
    cs[v] = (g.nscale && in) ? sb * g.nscale[(long long)b * g.nscale_ld + n] : sb;
  }
  __syncthreads();
  TOut* C = reinterpret_cast<TOut*>(g.C) + (long long)b * g.sC;
  if (n0 >= g.N || rsub >= rpp) return;
  // the VN columns are contiguous in C (checked on the host): one offset
  const bool full = n0 + VN <= g.N;
  const int co = g.cC_step >= 0 ? n0 * g.cC_step : g.cC[n0];
  for (int r = rsub; r < kSkRows; r += rpp) {
    const int m = m0 + r;
    if (m >= g.M) break;
    TC acc[VN];
#pragma unroll
    for (int v = 0; v < VN; ++v) acc[v] = (TC)0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const TC a = sA[r * KMAX + k];
#pragma unroll
      for (int v = 0; v < VN; ++v) acc[v] += a * bv[k][v];
    }
    const long long off = (long long)sRC[r] + co;
    TOut o[VN];
    if (full && (((long long)b * g.sC + off) % VN) == 0) {
      if (g.accumulate) __builtin_memcpy(o, C + off, VB);
#pragma unroll
      for (int v = 0; v < VN; ++v) {
        const double x = (double)acc[v] * cs[v] + (g.accumulate ? (double)o[v] : 0.0);
        o[v] = sizeof(TOut) == 8 ? (TOut)x : (TOut)(float)x;
      }
      __builtin_memcpy(C + off, o, VB);
    } else {
#pragma unroll
      for (int v = 0; v < VN; ++v) {
        if (n0 + v >= g.N) break;
        double x = (double)acc[v] * cs[v];
        if (g.accumulate) x += (double)C[off + v];
        C[off + v] = sizeof(TOut) == 8 ? (TOut)x : (TOut)(float)x;
      }
    }
  }
}

// Products with few rows (M <= 8) and a moderate reduction (K <= 256) over
// wide operands (real, N >= 256) are bound by reading B: a 16-row MFMA tile
// would idle at least half of its rows while the tile loads wait.  Here each thread
// owns VN consecutive columns, streams their K values of B with one vector
// load per k (8 k in flight), and keeps all M rows of the result in
// registers; A (M x K) sits in LDS.  The host checks that every vector load
// and store is aligned (unit-stride fastest leg with a multiple of VN
// values, all other strides multiples of VN).
constexpr int kSmMaxK = 256;

template <class TIn, class TC, class TOut, int MMAX>
__global__ __launch_bounds__(256) void smallm_kernel(GemmArgs g, int nchunks) {
  constexpr int VN = 16 / (int)sizeof(TIn) < 4 ? 16 / (int)sizeof(TIn) : 4;  // 2 doubles, 4 floats or bf16
  __shared__ TC sA[MMAX * kSmMaxK];
  const int w = (int)(blockIdx.x & 7) * g.per_xcd + (int)(blockIdx.x >> 3);
  if (w >= g.nwork) return;
  const int chunk = w % nchunks, b = w / nchunks, tid = threadIdx.x;
  const TIn* A = reinterpret_cast<const TIn*>(g.A) + (long long)b * g.sA;
  const TIn* B = reinterpret_cast<const TIn*>(g.B) + (long long)b * g.sB;
  // A (MMAX x K, zero past M); every load is issued before the first LDS store
  constexpr int IA = MMAX * kSmMaxK / 256;
  TC av[IA];
#pragma unroll
  for (int it = 0; it < IA; ++it) {
    const int e = tid + 256 * it, m = e / g.K, k = e - m * g.K;
    TC v = (TC)0;
    if (e < MMAX * g.K && m < g.M) {
      const int ro = g.rA_step >= 0 ? m * g.rA_step : g.rA[m];
      const int ko = g.tabA ? g.cA[k] : k * g.a_kstep;
      v = (TC)A[ro + ko];
    }
    av[it] = v;
  }
#pragma unroll
  for (int it = 0; it < IA; ++it)
    if (tid + 256 * it < MMAX * g.K) sA[tid + 256 * it] = av[it];
  __syncthreads();
  const int n0 = (chunk * 256 + tid) * VN;
  if (n0 >= g.N) return;
  const int co = g.cB_step >= 0 ? n0 * g.cB_step : g.cB[n0];
  TC acc[MMAX][VN];
#pragma unroll
  for (int m = 0; m < MMAX; ++m)
#pragma unroll
    for (int v = 0; v < VN; ++v) acc[m][v] = (TC)0;
  auto load = [&](int k, TIn* x) {
    const int ko = g.tabB ? g.rB[k] : k * g.b_kstep;
    __builtin_memcpy(x, B + ko + co, VN * sizeof(TIn));
  };
  auto fma_k = [&](int k, const TIn* x) {
#pragma unroll
    for (int m = 0; m < MMAX; ++m) {
      const TC a = sA[m * g.K + k];
#pragma unroll
      for (int v = 0; v < VN; ++v) acc[m][v] += a * (TC)x[v];
    }
  };
  int k = 0;
  for (; k + 8 <= g.K; k += 8) {
    TIn x[8][VN];
#pragma unroll
    for (int u = 0; u < 8; ++u) load(k + u, x[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u) fma_k(k + u, x[u]);
  }
  for (; k < g.K; ++k) {
    TIn x[VN];
    load(k, x);
    fma_k(k, x);
  }
  const double sb = g.alpha * (g.scale ? g.scale[b] : 1.0);
  double cs[VN];
#pragma unroll
  for (int v = 0; v < VN; ++v) cs[v] = g.nscale ? sb * g.nscale[(long long)b * g.nscale_ld + n0 + v] : sb;
  TOut* C = reinterpret_cast<TOut*>(g.C) + (long long)b * g.sC;
  const int cco = g.cC_step >= 0 ? n0 * g.cC_step : g.cC[n0];
#pragma unroll
  for (int m = 0; m < MMAX; ++m) {
    if (m >= g.M) continue;
    TOut* c = C + (g.rC_step >= 0 ? m * g.rC_step : g.rC[m]) + cco;
    TOut o[VN];
    if (g.accumulate) __builtin_memcpy(o, c, VN * sizeof(TOut));
#pragma unroll
    for (int v = 0; v < VN; ++v) {
      const double x = (double)acc[m][v] * cs[v] + (g.accumulate ? (double)o[v] : 0.0);
      o[v] = sizeof(TOut) == 8 ? (TOut)x : (TOut)(float)x;
    }
    __builtin_memcpy(c, o, VN * sizeof(TOut));
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
    if (g.skip_if_zero && g.skip_if_zero[b] == 0) continue;
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

constexpr int kLdsBytes = 160 * 1024;

struct Cfg {
  int WM, WN, TM, TN;
  int BM() const { return WM * TM * 16; }
  int BN() const { return WN * TN * 16; }
};

// Tile shapes: square defaults and skinny variants for the many products
// whose N (sketch width k <= 128) or M (a bond or physical dimension) is small.
const Cfg kCfgs[] = {
    {2, 2, 2, 2},  // 0: 64 x 64
    {4, 1, 2, 3},  // 1: 128 x 48
    {4, 1, 2, 2},  // 2: 128 x 32
    {1, 4, 3, 2},  // 3: 48 x 128
    {2, 2, 2, 4},  // 4: 64 x 128
    {2, 2, 4, 2},  // 5: 128 x 64
    {2, 2, 4, 4},  // 6: 128 x 128
    {1, 4, 1, 4},  // 7: 16 x 256
    {4, 1, 4, 1},  // 8: 256 x 16
    {1, 4, 2, 2},  // 9: 32 x 128
    // shapes that fit the bond-sized dimensions with little padding:
    // M = 100 (112), M = 200 (208), N = 72 (80), N = 100 or 108 (112)
    {1, 4, 7, 1},   // 10: 112 x 64
    {1, 4, 13, 1},  // 11: 208 x 64
    {4, 1, 1, 5},   // 12: 64 x 80
    {4, 1, 2, 5},   // 13: 128 x 80
    {4, 1, 1, 7},   // 14: 64 x 112
};
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);

// complex products keep four accumulator sets: only shapes with at most four
// MFMA tiles per wavefront fit the register file
bool cfg_ok(int ci, bool cplx) { return !cplx || kCfgs[ci].TM * kCfgs[ci].TN <= 4; }
// the 32-deep K-step doubles the staging registers: complex products and the
// shapes of more than 8 MFMA tiles per wavefront would spill
bool ks_ok(int ci, int ks, bool cplx) {
  return ks == 1 || (ks == 2 && !cplx && kCfgs[ci].TM * kCfgs[ci].TN <= 8);
}
// BF16 products need 32-deep K-steps (one v_mfma_f32_16x16x32_bf16 per tile and step)
bool ks_ok(int ci, int ks, Prec prec) {
  if (prec == Prec::BF16) return ks == 2 && kCfgs[ci].TM * kCfgs[ci].TN <= 8;
  return ks_ok(ci, ks, prec == Prec::C128);
}

// Tile shape from a simple cost model: time = max(padded MFMA work at a
// shape-dependent efficiency, HBM traffic with the re-reads the tiling
// implies), divided by the fill of the chip.  An operand is re-read once per
// tile row (B) or column (A) unless one instance of it fits in an L2 share.
double tile_cost(const Cfg& c, int64_t M, int64_t N, int64_t K, int64_t batch, double elt) {
  const double mt = std::ceil(M / double(c.BM())), nt = std::ceil(N / double(c.BN()));
  const double work = 2.0 * mt * c.BM() * nt * c.BN() * std::max<int64_t>(K, 1) * batch;
  // MFMA efficiency grows with the MFMA tiles a wavefront owns (LDS reads
  // per MFMA fall); the 16-tile shape runs at one wavefront per SIMD
  static const double eff_by_tiles[17] = {0, .30, .45, .55, .70, .70, .75, .75, .80,
                                          .80, .80, .80, .80, .80, .80, .80, .70};
  const double eff = eff_by_tiles[std::min(16, c.TM * c.TN)];
  const double l2 = 2.0 * 1024 * 1024;
  const double a = double(M) * K * elt, b = double(K) * N * elt, cc = double(M) * N * elt;
  const double bytes = batch * (a * (a < l2 ? 1 : nt) + b * (b < l2 ? 1 : mt) + cc);
  // compute and memory overlap imperfectly
  const double tc = work / (78.6e12 * eff), tm = bytes / 6.0e12;
  const double t = std::max(tc, tm) + 0.25 * std::min(tc, tm);
  // long-K products are split when the tile grid is small (see make_plan)
  double blocks = mt * nt * batch;
  if (blocks < 1024 && K >= 256) blocks *= std::min(std::ceil(1024.0 / blocks), double(K / 128));
  return t / std::min(1.0, blocks / 512.0);
}

int pick_cfg(int64_t M, int64_t N, int64_t K, int64_t batch, Prec prec, double elt) {
  int best = 0;
  double bc = 1e300;
  for (int i = 0; i < kNumCfgs; ++i) {
    if (!cfg_ok(i, prec == Prec::C128) || !ks_ok(i, prec == Prec::BF16 ? 2 : 1, prec)) continue;
    const double c = tile_cost(kCfgs[i], M, N, K, batch, elt);
    if (c < bc * 0.999) {
      bc = c;
      best = i;
    }
  }
  return best;
}

template <class TC, bool CPLX, class TIn, class TOut, int WM, int WN, int TM, int TN, int KS>
void launch_one(unsigned grid, size_t lds, hipStream_t st, const GemmArgs& a) {
  if constexpr ((CPLX && (TM * TN > 4 || KS > 1)) || (TM * TN > 8 && KS > 1)) {
    throw Error{HPEPS_ERR_UNSUPPORTED, "gemm variant not available"};
  } else {
    // dynamic LDS above the default 64 KB needs the function attribute raised
    static size_t lds_allowed = 64 * 1024;
    if (lds > lds_allowed) {
      HP_CHECK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_kernel<TC, CPLX, TIn, TOut, WM, WN, TM, TN, KS>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      lds_allowed = lds;
    }
    // launched by name: a launch through a pointer to the kernel has run
    // nothing, without an error, in host code built with instrumentation
    gemm_kernel<TC, CPLX, TIn, TOut, WM, WN, TM, TN, KS><<<grid, 256, lds, st>>>(a);
  }
}

template <class TC, bool CPLX, class TIn, class TOut, int KS>
void launch_cfg(int ci, unsigned grid, size_t lds, hipStream_t st, const GemmArgs& a) {
  switch (ci) {
    case 0: launch_one<TC, CPLX, TIn, TOut, 2, 2, 2, 2, KS>(grid, lds, st, a); break;
    case 1: launch_one<TC, CPLX, TIn, TOut, 4, 1, 2, 3, KS>(grid, lds, st, a); break;
    case 2: launch_one<TC, CPLX, TIn, TOut, 4, 1, 2, 2, KS>(grid, lds, st, a); break;
    case 3: launch_one<TC, CPLX, TIn, TOut, 1, 4, 3, 2, KS>(grid, lds, st, a); break;
    case 4: launch_one<TC, CPLX, TIn, TOut, 2, 2, 2, 4, KS>(grid, lds, st, a); break;
    case 5: launch_one<TC, CPLX, TIn, TOut, 2, 2, 4, 2, KS>(grid, lds, st, a); break;
    case 6: launch_one<TC, CPLX, TIn, TOut, 2, 2, 4, 4, KS>(grid, lds, st, a); break;
    case 7: launch_one<TC, CPLX, TIn, TOut, 1, 4, 1, 4, KS>(grid, lds, st, a); break;
    case 8: launch_one<TC, CPLX, TIn, TOut, 4, 1, 4, 1, KS>(grid, lds, st, a); break;
    case 9: launch_one<TC, CPLX, TIn, TOut, 1, 4, 2, 2, KS>(grid, lds, st, a); break;
    case 10: launch_one<TC, CPLX, TIn, TOut, 1, 4, 7, 1, KS>(grid, lds, st, a); break;
    case 11: launch_one<TC, CPLX, TIn, TOut, 1, 4, 13, 1, KS>(grid, lds, st, a); break;
    case 12: launch_one<TC, CPLX, TIn, TOut, 4, 1, 1, 5, KS>(grid, lds, st, a); break;
    case 13: launch_one<TC, CPLX, TIn, TOut, 4, 1, 2, 5, KS>(grid, lds, st, a); break;
    default: launch_one<TC, CPLX, TIn, TOut, 4, 1, 1, 7, KS>(grid, lds, st, a); break;
  }
}

template <class TC, bool CPLX, class TIn, class TOut>
void launch_ks(int ci, int ks, unsigned grid, size_t lds, hipStream_t st, const GemmArgs& a) {
  if (ks == 2)
    launch_cfg<TC, CPLX, TIn, TOut, 2>(ci, grid, lds, st, a);
  else
    launch_cfg<TC, CPLX, TIn, TOut, 1>(ci, grid, lds, st, a);
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

// Step of an index map whose offsets are i * step for every linear index i
// (modes nest without gaps); -1 when the map is not affine.
int64_t affine_step(const IndexMap& m) {
  int64_t step = -1, span = 1;  // span: element count of the faster modes
  for (int i = m.n - 1; i >= 0; --i) {
    if (m.dim[i] == 1) continue;
    if (step < 0)
      step = m.stride[i];
    else if (m.stride[i] != step * span)
      return -1;
    span *= m.dim[i];
  }
  return step < 0 ? 0 : step;
}

// Everything a launch needs besides the shared arguments.
struct Plan {
  int ci = 0, ks = 1;
  int64_t ksplit = 1, kchunk = 1;
  size_t lds = 0;
  unsigned grid = 0;
};

Plan make_plan(Prec prec, const GemmDesc& d, const GemmCall& c, const GemmArgs& a, GemmVariant v) {
  const bool cplx = prec == Prec::C128;
  Plan p;
  p.ci = (v.cfg >= 0 && v.cfg < kNumCfgs && cfg_ok(v.cfg, cplx))
             ? v.cfg
             : pick_cfg(d.M, d.N, d.K, c.batch, prec,
                        prec == Prec::F32 ? 4.0 : prec == Prec::BF16 ? 2.0 : (cplx ? 16.0 : 8.0));
  p.ks = v.ks == 1 || v.ks == 2 ? v.ks : 1;
  if (prec == Prec::BF16) {
    p.ks = 2;
    if (!ks_ok(p.ci, 2, prec)) p.ci = 5;
  }
  if (!ks_ok(p.ci, p.ks, prec)) p.ks = 1;
  const Cfg cf = kCfgs[p.ci];
  const int64_t ntotal = (int64_t)cdiv(d.M, cf.BM()) * cdiv(d.N, cf.BN());
  const int bk = 16 * p.ks;
  // split K when the tile grid alone gives fewer than ~4 blocks per CU
  int64_t ksplit = 1;
  const int64_t blocks = ntotal * c.batch;
  if (v.split > 0)
    ksplit = v.split;
  else if (blocks < 1024 && d.K >= 256)
    ksplit = std::max<int64_t>(1, std::min<int64_t>((1024 + blocks - 1) / blocks, d.K / 128));
  if (c.copy_if_zero) ksplit = 1;
  ksplit = std::min<int64_t>(ksplit, std::max<int64_t>(1, d.K / bk));
  int64_t kchunk = (d.K + ksplit - 1) / ksplit;
  // the staged K tables must fit next to the two operand stages
  const int elt_c = prec == Prec::F32 ? 4 : (prec == Prec::BF16 ? 2 : 8);
  const int ldk = bk + 16 / elt_c;
  const int64_t stage_bytes = 2LL * (cplx ? 2 : 1) * (cf.BM() + cf.BN()) * ldk * elt_c;
  const int ntab = a.tabA + a.tabB;
  if (ntab > 0) {
    const int64_t kmax = (kLdsBytes - stage_bytes) / (4 * ntab) / bk * bk;
    HP_REQUIRE(kmax >= bk, HPEPS_ERR_UNSUPPORTED, "gemm tile does not fit in LDS");
    kchunk = std::min(kchunk, kmax);
  }
  kchunk = std::max<int64_t>(bk, (kchunk + bk - 1) / bk * bk);
  ksplit = std::max<int64_t>(1, (d.K + kchunk - 1) / kchunk);
  if (c.copy_if_zero) HP_REQUIRE(ksplit == 1, HPEPS_ERR_UNSUPPORTED, "pass-through gemm too long");
  const int64_t nwork = ntotal * c.batch * ksplit;
  HP_REQUIRE(nwork < (1LL << 30), HPEPS_ERR_UNSUPPORTED, "gemm launch too large");
  p.ksplit = ksplit;
  p.kchunk = kchunk;
  p.lds = (size_t)(stage_bytes + (int64_t)ntab * kchunk * 4);
  p.grid = (unsigned)((nwork + 7) / 8) * 8u;
  return p;
}

// Enqueues the product with plan p (split-K partials from the workspace).
void run_plan(Ctx& ctx, Prec prec, const GemmDesc& d, const GemmCall& c, GemmArgs a, const Plan& p) {
  const bool cplx = prec == Prec::C128;
  const Cfg cf = kCfgs[p.ci];
  a.mtiles = (int)cdiv(d.M, cf.BM());
  a.ntotal = (int)(a.mtiles * (int64_t)cdiv(d.N, cf.BN()));
  a.ksplit = (int)p.ksplit;
  a.kchunk = (int)p.kchunk;
  a.nwork = (int)((int64_t)a.ntotal * c.batch * p.ksplit);
  a.per_xcd = (int)(p.grid / 8);
  a.partial = nullptr;
  if (p.ksplit > 1)
    a.partial = ctx.ws_alloc((int64_t)c.batch * p.ksplit * d.M * d.N * (cplx ? 16 : 8));
  hipStream_t st = ctx.stream;
  switch (prec) {
    case Prec::F64:
      launch_ks<double, false, double, double>(p.ci, p.ks, p.grid, p.lds, st, a);
      if (p.ksplit > 1) splitk_reduce_kernel<false, double><<<1024, 256, 0, st>>>(a, c.batch);
      break;
    case Prec::C128:
      launch_ks<double, true, double, double>(p.ci, p.ks, p.grid, p.lds, st, a);
      if (p.ksplit > 1) splitk_reduce_kernel<true, double><<<1024, 256, 0, st>>>(a, c.batch);
      break;
    case Prec::F32:
      if (c.out_f64) {
        launch_ks<float, false, float, double>(p.ci, p.ks, p.grid, p.lds, st, a);
        if (p.ksplit > 1) splitk_reduce_kernel<false, double><<<1024, 256, 0, st>>>(a, c.batch);
      } else {
        launch_ks<float, false, float, float>(p.ci, p.ks, p.grid, p.lds, st, a);
        if (p.ksplit > 1) splitk_reduce_kernel<false, float><<<1024, 256, 0, st>>>(a, c.batch);
      }
      break;
    case Prec::BF16:
      if (c.out_f64) {
        launch_cfg<__bf16, false, __bf16, double, 2>(p.ci, p.grid, p.lds, st, a);
        if (p.ksplit > 1) splitk_reduce_kernel<false, double><<<1024, 256, 0, st>>>(a, c.batch);
      } else {
        launch_cfg<__bf16, false, __bf16, __bf16, 2>(p.ci, p.grid, p.lds, st, a);
        if (p.ksplit > 1) splitk_reduce_kernel<false, __bf16><<<1024, 256, 0, st>>>(a, c.batch);
      }
      break;
  }
  HP_CHECK_HIP(hipGetLastError());
}

// True when the column index map of C runs through memory in contiguous
// groups of vn: its fastest mode has unit stride and a multiple of vn values.
bool contiguous_runs(const IndexMap& m, int vn) {
  for (int i = m.n - 1; i >= 0; --i)
    if (m.dim[i] > 1) return m.stride[i] == 1 && m.dim[i] % vn == 0;
  return false;
}

// Enqueues the short-reduction kernel (see smallk_kernel).
void run_smallk(Ctx& ctx, Prec prec, const GemmDesc& d, const GemmCall& c, GemmArgs a) {
  const int vn = prec == Prec::F64 || c.out_f64 ? 2 : 4;
  const int gpr = (int)std::min<int64_t>(cdiv(d.N, vn), 256);
  const int64_t nchunks = cdiv(cdiv(d.N, vn), gpr), mgroups = cdiv(d.M, kSkRows);
  const int64_t nwork = nchunks * mgroups * c.batch;
  HP_REQUIRE(nwork < (1LL << 30), HPEPS_ERR_UNSUPPORTED, "gemm launch too large");
  a.nwork = (int)nwork;
  const unsigned grid = (unsigned)((nwork + 7) / 8) * 8u;
  a.per_xcd = (int)(grid / 8);
  a.ksplit = 1;
  int rec = -1;
  if (ctx.prof_on) {
    static const char* pn[] = {"f64", "c128", "f32", "bf16"};
    std::string name = std::string("gemm_") + pn[(int)prec] + (prec == Prec::F32 && !c.out_f64 ? "o32" : "") +
                       (prec == Prec::BF16 && !c.out_f64 ? "o16" : "") + "_smallk";
    if (ctx.prof_shapes)
      name += "_M" + std::to_string(d.M) + "_N" + std::to_string(d.N) + "_K" + std::to_string(d.K) + "_b" +
              std::to_string(c.batch);
    rec = ctx.prof_begin(name);
  }
  hipStream_t st = ctx.stream;
  const int nc = (int)nchunks, mgr = (int)mgroups;
  auto go = [&](auto t) {
    using T = decltype(t);
    smallk_kernel<typename T::In, typename T::Acc, typename T::Out, T::n><<<grid, 256, 0, st>>>(a, nc, mgr, gpr);
  };
  const bool k8 = d.K <= 8;
  switch (prec) {
    case Prec::F64:
      k8 ? go(KTag<double, double, double, 8>{}) : go(KTag<double, double, double, 16>{});
      break;
    case Prec::F32:
      if (c.out_f64)
        k8 ? go(KTag<float, float, double, 8>{}) : go(KTag<float, float, double, 16>{});
      else
        k8 ? go(KTag<float, float, float, 8>{}) : go(KTag<float, float, float, 16>{});
      break;
    case Prec::BF16:
      if (c.out_f64)
        k8 ? go(KTag<__bf16, float, double, 8>{}) : go(KTag<__bf16, float, double, 16>{});
      else
        k8 ? go(KTag<__bf16, float, __bf16, 8>{}) : go(KTag<__bf16, float, __bf16, 16>{});
      break;
    default:
      throw Error{HPEPS_ERR_UNSUPPORTED, "short-reduction kernel: real products only"};
  }
  HP_CHECK_HIP(hipGetLastError());
  if (rec >= 0) {
    const double elt = prec == Prec::F32 ? 4 : prec == Prec::BF16 ? 2 : 8;
    const double eout = c.out_f64 || prec == Prec::F64 ? 8 : elt;
    ctx.prof_end(rec, 2.0 * (double)d.M * d.N * d.K * c.batch,
                 ((double)d.M * d.K * elt + (double)d.K * d.N * elt + (double)d.M * d.N * eout) * c.batch);
  }
}

// True when every vn-group of consecutive columns of the map is contiguous
// and starts at a multiple of vn elements: the fastest mode has unit stride
// and a multiple of vn values, every other stride of the maps in `others`
// (and of this map) is a multiple of vn.
bool vec_aligned(const IndexMap& cols, std::initializer_list<const IndexMap*> others, int64_t inst_stride,
                 const void* base, int vn, int64_t elt) {
  if (!contiguous_runs(cols, vn) || inst_stride % vn != 0 || reinterpret_cast<uintptr_t>(base) % (vn * elt) != 0)
    return false;
  int last = cols.n - 1;
  while (last >= 0 && cols.dim[last] == 1) --last;
  for (int i = 0; i < last; ++i)
    if (cols.dim[i] > 1 && cols.stride[i] % vn != 0) return false;
  for (const IndexMap* m : others)
    for (int i = 0; i < m->n; ++i)
      if (m->dim[i] > 1 && m->stride[i] % vn != 0) return false;
  return true;
}

// Enqueues the few-rows kernel (see smallm_kernel).
void run_smallm(Ctx& ctx, Prec prec, const GemmDesc& d, const GemmCall& c, GemmArgs a) {
  const int vn = prec == Prec::F64 ? 2 : 4;
  const int64_t nchunks = cdiv(d.N, 256 * vn);
  const int64_t nwork = nchunks * c.batch;
  HP_REQUIRE(nwork < (1LL << 30), HPEPS_ERR_UNSUPPORTED, "gemm launch too large");
  a.nwork = (int)nwork;
  const unsigned grid = (unsigned)((nwork + 7) / 8) * 8u;
  a.per_xcd = (int)(grid / 8);
  a.ksplit = 1;
  int rec = -1;
  if (ctx.prof_on) {
    static const char* pn[] = {"f64", "c128", "f32", "bf16"};
    std::string name = std::string("gemm_") + pn[(int)prec] + (prec == Prec::F32 && !c.out_f64 ? "o32" : "") +
                       (prec == Prec::BF16 && !c.out_f64 ? "o16" : "") + "_smallm";
    if (ctx.prof_shapes)
      name += "_M" + std::to_string(d.M) + "_N" + std::to_string(d.N) + "_K" + std::to_string(d.K) + "_b" +
              std::to_string(c.batch);
    rec = ctx.prof_begin(name);
  }
  hipStream_t st = ctx.stream;
  const int nc = (int)nchunks;
  auto go = [&](auto t) {
    using T = decltype(t);
    smallm_kernel<typename T::In, typename T::Acc, typename T::Out, T::n><<<grid, 256, 0, st>>>(a, nc);
  };
  switch (prec) {
    case Prec::F64:
      go(KTag<double, double, double, 8>{});
      break;
    case Prec::F32:
      c.out_f64 ? go(KTag<float, float, double, 8>{}) : go(KTag<float, float, float, 8>{});
      break;
    case Prec::BF16:
      c.out_f64 ? go(KTag<__bf16, float, double, 8>{}) : go(KTag<__bf16, float, __bf16, 8>{});
      break;
    default:
      throw Error{HPEPS_ERR_UNSUPPORTED, "few-rows kernel: real products only"};
  }
  HP_CHECK_HIP(hipGetLastError());
  if (rec >= 0) {
    const double elt = prec == Prec::F32 ? 4 : prec == Prec::BF16 ? 2 : 8;
    const double eout = c.out_f64 || prec == Prec::F64 ? 8 : elt;
    ctx.prof_end(rec, 2.0 * (double)d.M * d.N * d.K * c.batch,
                 ((double)d.M * d.K * elt + (double)d.K * d.N * elt + (double)d.M * d.N * eout) * c.batch);
  }
}

std::string tune_key(Prec prec, const GemmDesc& d, const GemmCall& c, const GemmArgs& a) {
  char buf[160];
  snprintf(buf, sizeof(buf), "%s_M%lld_N%lld_K%lld_b%d_a%d%d_b%d%d",
           prec == Prec::F64    ? "f64"
           : prec == Prec::C128 ? "c128"
           : prec == Prec::F32  ? (c.out_f64 ? "f32" : "f32o32")
                                : (c.out_f64 ? "bf16" : "bf16o16"),
           (long long)d.M, (long long)d.N, (long long)d.K, c.batch, a.a_kfast, a.tabA, a.b_kfast,
           a.tabB);
  return buf;
}

// A product may be re-run for timing only when it is idempotent: no
// accumulation into C and C disjoint from A and B.
bool tunable(Ctx& ctx, Prec prec, const GemmCall& c, int64_t nA, int64_t nB, int64_t nC) {
  if (c.accumulate) return false;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(ctx.stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
    return false;
  const int64_t ein = prec == Prec::F32 ? 4 : prec == Prec::BF16 ? 2 : (prec == Prec::C128 ? 16 : 8);
  const int64_t eout = c.out_f64 || prec == Prec::F64 || prec == Prec::C128 ? (prec == Prec::C128 ? 16 : 8)
                                                                            : ein;
  auto range = [](const void* p, int64_t s, int64_t n, int batch, int64_t e) {
    const char* b = static_cast<const char*>(p);
    return std::make_pair(b, b + ((int64_t)(batch - 1) * s + n) * e);
  };
  const auto ra = range(c.A, c.sA, nA, c.batch, ein), rb = range(c.B, c.sB, nB, c.batch, ein),
             rc = range(c.C, c.sC, nC, c.batch, eout);
  auto overlap = [](std::pair<const char*, const char*> x, std::pair<const char*, const char*> y) {
    return x.first < y.second && y.first < x.second;
  };
  return !overlap(rc, ra) && !overlap(rc, rb);
}

constexpr int kTuneReps = 8;  // timed launches per variant (after one warm-up launch)

GemmVariant tune(Ctx& ctx, Prec prec, const GemmDesc& d, const GemmCall& c, const GemmArgs& a) {
  const bool cplx = prec == Prec::C128;
  hipEvent_t e0, e1;
  HP_CHECK_HIP(hipEventCreate(&e0));
  HP_CHECK_HIP(hipEventCreate(&e1));
  GemmVariant best;
  float best_ms = 1e30f;
  std::vector<std::tuple<int, int, int64_t>> seen;
  for (int ci = 0; ci < kNumCfgs; ++ci) {
    if (!cfg_ok(ci, cplx)) continue;
    for (int ks = 1; ks <= 2; ++ks) {
      if (!ks_ok(ci, ks, prec)) continue;
      const int64_t h = make_plan(prec, d, c, a, GemmVariant{ci, ks, 0}).ksplit;
      for (int64_t sp : {(int64_t)0, (int64_t)1, 2 * h, 4 * h}) {
        GemmVariant v{ci, ks, (int)sp};
        Plan p;
        try {
          p = make_plan(prec, d, c, a, v);
        } catch (const Error&) {
          continue;
        }
        const auto id = std::make_tuple(p.ci, p.ks, p.ksplit);
        if (std::find(seen.begin(), seen.end(), id) != seen.end()) continue;
        seen.push_back(id);
        const int chunk = ctx.ws_chunk();
        const int64_t off = ctx.ws_offset();
        run_plan(ctx, prec, d, c, a, p);  // warm-up (also first-launch setup)
        HP_CHECK_HIP(hipEventRecord(e0, ctx.stream));
        for (int r = 0; r < kTuneReps; ++r) run_plan(ctx, prec, d, c, a, p);
        HP_CHECK_HIP(hipEventRecord(e1, ctx.stream));
        HP_CHECK_HIP(hipEventSynchronize(e1));
        float ms = 0;
        HP_CHECK_HIP(hipEventElapsedTime(&ms, e0, e1));
        ctx.ws_restore(chunk, off);
        if (ms < best_ms) {
          best_ms = ms;
          best = GemmVariant{p.ci, p.ks, (int)p.ksplit};
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
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
  HP_REQUIRE(c.batch >= 1, HPEPS_ERR_INVALID_ARG, "gemm batch must be >= 1");
  tape_gemm(ctx, prec, d, c);
  const bool cplx = prec == Prec::C128;
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
  a.rA_step = (int)affine_step(d.Am);
  a.cB_step = (int)affine_step(d.Bn);
  a.rC_step = (int)affine_step(d.Cm);
  a.cC_step = (int)affine_step(d.Cn);
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
  a.skip_if_zero = c.skip_if_zero;
  // per-instance extents for the buffer resources (byte offsets are 32-bit)
  const int64_t elt_in = prec == Prec::F32 ? 4 : prec == Prec::BF16 ? 2 : (cplx ? 16 : 8);
  HP_REQUIRE(nA * elt_in < (1LL << 32) - 16 && nB * elt_in < (1LL << 32) - 16, HPEPS_ERR_UNSUPPORTED,
             "gemm operand exceeds 4 GiB per instance");
  a.nA_bytes = (unsigned)(nA * elt_in);
  a.nB_bytes = (unsigned)(nB * elt_in);
  // K offsets: affine maps are computed in the kernel, others staged in LDS
  const int64_t stepA = affine_step(d.Ak), stepB = affine_step(d.Bk);
  const bool affA = stepA >= 0 && stepA * std::max<int64_t>(d.K, 1) < (1LL << 31);
  const bool affB = stepB >= 0 && stepB * std::max<int64_t>(d.K, 1) < (1LL << 31);
  a.tabA = affA ? 0 : 1;
  a.tabB = affB ? 0 : 1;
  a.a_kstep = affA ? (int)stepA : 0;
  a.b_kstep = affB ? (int)stepB : 0;

  // short reductions (output columns in contiguous runs): the store-bound
  // kernel; below ~70 columns the MFMA tiles were measured as fast or faster
  if (!cplx && !c.copy_if_zero && !c.skip_if_zero && ctx.smallk && ctx.gemm_force.cfg < 0 && d.K <= 16 &&
      d.N >= 72 &&
      reinterpret_cast<uintptr_t>(c.C) % 16 == 0 &&
      contiguous_runs(d.Cn, prec == Prec::F64 || c.out_f64 ? 2 : 4)) {
    run_smallk(ctx, prec, d, c, a);
    return;
  }
  // few rows over wide operands: the read-bound kernel
  if (!cplx && !c.copy_if_zero && !c.skip_if_zero && ctx.smallk && ctx.gemm_force.cfg < 0 && d.M <= 8 &&
      d.N >= 256 &&
      d.K <= kSmMaxK) {
    const int vn = prec == Prec::F64 ? 2 : 4;
    const int64_t ein = prec == Prec::F64 ? 8 : prec == Prec::F32 ? 4 : 2;
    const int64_t eout = prec == Prec::F64 || c.out_f64 ? 8 : ein;
    if (vec_aligned(d.Bn, {&d.Bk}, c.sB, c.B, vn, ein) && vec_aligned(d.Cn, {&d.Cm}, c.sC, c.C, vn, eout)) {
      run_smallm(ctx, prec, d, c, a);
      return;
    }
  }

  // launch variant: forced, tuned, tuned now, or the heuristic
  GemmVariant v = ctx.gemm_force;
  if (v.cfg < 0) {
    const std::string key = tune_key(prec, d, c, a);
    auto it = ctx.gemm_tuned.find(key);
    if (it != ctx.gemm_tuned.end()) {
      v = it->second;
    } else if (ctx.autotune && tunable(ctx, prec, c, nA, nB, nC)) {
      v = tune(ctx, prec, d, c, a);
      ctx.gemm_tuned[key] = v;
    }
  }
  const Plan p = make_plan(prec, d, c, a, v);
  const Cfg cf = kCfgs[p.ci];
  int rec = -1;
  if (ctx.prof_on) {
    static const char* pn[] = {"f64", "c128", "f32", "bf16"};
    const std::string name = std::string("gemm_") + pn[(int)prec] +
                             (prec == Prec::F32 && !c.out_f64 ? "o32" : "") +
                             (prec == Prec::BF16 && !c.out_f64 ? "o16" : "") + "_" +
                             std::to_string(cf.BM()) + "x" + std::to_string(cf.BN()) + "k" +
                             std::to_string(16 * p.ks) +
                             (ctx.prof_shapes ? "_M" + std::to_string(d.M) + "_N" + std::to_string(d.N) + "_K" +
                                                    std::to_string(d.K) + "_b" + std::to_string(c.batch)
                                              : std::string());
    rec = ctx.prof_begin(name);
  }
  run_plan(ctx, prec, d, c, a, p);
  if (rec >= 0) {
    // algorithmic work of the product: 2 M N K per instance (complex: 4 real
    // products per multiply-add); bytes: each operand element once
    const double mnk = 2.0 * (double)d.M * (double)d.N * (double)d.K * c.batch * (cplx ? 4 : 1);
    const double elt = prec == Prec::F32 ? 4.0 : prec == Prec::BF16 ? 2.0 : (cplx ? 16.0 : 8.0);
    const double byt = ((double)d.M * d.K + (double)d.K * d.N + (double)d.M * d.N) * c.batch * elt;
    ctx.prof_end(rec, mnk, byt);
  }
}

// ---------------------------------------------------------------------------
// autotune cache as JSON: {"gemm": {"<key>": [cfg, ks, split], ...}}

std::string autotune_export(const Ctx& ctx) {
  std::string s = "{\"gemm\": {";
  bool first = true;
  for (const auto& kv : ctx.gemm_tuned) {
    char buf[64];
    snprintf(buf, sizeof(buf), "[%d, %d, %d]", kv.second.cfg, kv.second.ks, kv.second.split);
    if (!first) s += ", ";
    s += "\"" + kv.first + "\": " + buf;
    first = false;
  }
  s += "}}";
  return s;
}

void autotune_import(Ctx& ctx, const std::string& json) {
  // entries are "key": [int, int, int]; keys hold no quotes or brackets
  size_t pos = json.find("\"gemm\"");
  HP_REQUIRE(pos != std::string::npos, HPEPS_ERR_INVALID_ARG, "autotune JSON has no \"gemm\" object");
  pos = json.find('{', pos);
  HP_REQUIRE(pos != std::string::npos, HPEPS_ERR_INVALID_ARG, "autotune JSON is malformed");
  std::map<std::string, GemmVariant> parsed;
  while (true) {
    const size_t q0 = json.find_first_of("\"}", pos + 1);
    HP_REQUIRE(q0 != std::string::npos, HPEPS_ERR_INVALID_ARG, "autotune JSON is malformed");
    if (json[q0] == '}') break;
    const size_t q1 = json.find('"', q0 + 1);
    const size_t lb = q1 == std::string::npos ? q1 : json.find('[', q1);
    const size_t rb = lb == std::string::npos ? lb : json.find(']', lb);
    HP_REQUIRE(rb != std::string::npos, HPEPS_ERR_INVALID_ARG, "autotune JSON is malformed");
    GemmVariant v;
    HP_REQUIRE(sscanf(json.c_str() + lb, "[%d , %d , %d ]", &v.cfg, &v.ks, &v.split) == 3,
               HPEPS_ERR_INVALID_ARG, "autotune JSON entry is malformed");
    HP_REQUIRE(v.cfg >= 0 && v.cfg < kNumCfgs && (v.ks == 1 || v.ks == 2) && v.split >= 0,
               HPEPS_ERR_INVALID_ARG, "autotune JSON entry out of range");
    parsed[json.substr(q0 + 1, q1 - q0 - 1)] = v;
    pos = rb;
  }
  for (auto& kv : parsed) ctx.gemm_tuned[kv.first] = kv.second;
}

}  // namespace hp
