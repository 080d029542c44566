// Named-leg two-operand contractions (see contract.hip).
#pragma once
#include <string>
#include <vector>

#include "internal.h"

namespace hp {

struct TView {
  const void* p = nullptr;
  std::string legs;             // one character per leg
  std::vector<int64_t> dims;
  std::vector<int64_t> strides; // element strides
  int64_t extent = 0;           // element count reachable from p
  bool conj = false;            // read complex-conjugated
};

TView tview(const void* p, const std::string& legs, const std::vector<int64_t>& dims,
            const std::vector<int64_t>& strides, int64_t extent, bool conj = false);
TView tview_rm(const void* p, const std::string& legs, const std::vector<int64_t>& dims,
               bool conj = false);
int64_t leg_dim(const TView& t, char c);

// C[out] = sum over shared legs of A * B (C += ... with accumulate); C
// row-major in the order of `out`.  Returns the output dims.  c_capacity:
// element capacity of C.
std::vector<int64_t> contract2(Ctx& ctx, bool cplx, const TView& A, const TView& B,
                               const std::string& out, void* C, int64_t c_capacity,
                               bool accumulate = false);
// The sub-view of `v` with leg `leg` restricted to [start, start + len).
TView restrict_leg(const TView& v, char leg, int64_t start, int64_t len, bool cplx);

}  // namespace hp
