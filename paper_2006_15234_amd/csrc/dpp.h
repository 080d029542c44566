// Cross-lane sums with DPP lane moves (VALU data paths, no LDS traffic).
// Every lane of the wavefront must be active where these are called.
#pragma once
#include <hip/hip_runtime.h>

namespace hp {

// v + (v moved by the DPP control CTRL within the rows of ROW_MASK).  The add
// is never contracted into an FMA with the product that made v: a lane would
// then add its own unrounded product to its partner's rounded one, and the
// butterfly sums would differ between lanes in the last bit.  Callers rely on
// every lane of a row holding the same sum (rotation parameters computed in
// each lane must agree).
//
// With every row enabled (ROW_MASK 0xf, a move within each row) no lane keeps
// the destination's old value, so the plain DPP move is used and the
// compiler does not zero the destination first; a partial row mask (the row
// broadcasts) leaves the other rows at the old value 0, which adds nothing.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
#pragma clang fp contract(off)
  const long long x = __builtin_bit_cast(long long, v);
  int lo, hi;
  if constexpr (ROW_MASK == 0xf) {
    lo = __builtin_amdgcn_mov_dpp((int)x, CTRL, 0xf, 0xf, false);
    hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, 0xf, 0xf, false);
  } else {
    lo = __builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, ROW_MASK, 0xf, false);
  }
  return v + __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 16 lanes of a DPP row, returned in all of them: quad
// butterflies, then the half-row and row mirrors.
__device__ __forceinline__ double row_sum16(double v) {
  v = dpp_add<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);  // row_mirror
  return v;
}

// Wavefront sum, returned in every lane: row sums, then the two row
// broadcasts leave the total in lane 63, which is read back.
__device__ __forceinline__ double wave_sum(double v) {
  v = row_sum16(v);
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const long long x = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)x, 63);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), 63);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

}  // namespace hp
