// Two-operand tensor contraction by named legs, lowered to one gathered
// GEMM: legs present in both operands and absent from the output are summed
// (K), legs of only one operand become the rows (M, from A) or columns
// (N, from B) of the product, the output is written in the row-major order
// of its leg string.  A leg present in both operands and in the output (at
// most one) is a batch leg: instance i of the product reads A and B at i
// times their strides of that leg and writes the output at i times its
// stride there; within an instance every access must stay below those
// strides.  Used for the strip contractions of expectation values and the
// batched amplitudes.
#include "contract.h"

namespace hp {

TView tview(const void* p, const std::string& legs, const std::vector<int64_t>& dims,
            const std::vector<int64_t>& strides, int64_t extent, bool conj) {
  HP_REQUIRE(legs.size() == dims.size() && dims.size() == strides.size(), HPEPS_ERR_SHAPE,
             "tensor view: legs/dims/strides lengths differ");
  TView v;
  v.p = p;
  v.legs = legs;
  v.dims = dims;
  v.strides = strides;
  v.extent = extent;
  v.conj = conj;
  return v;
}

TView tview_rm(const void* p, const std::string& legs, const std::vector<int64_t>& dims, bool conj) {
  int64_t n = 1;
  for (auto d : dims) n *= d;
  return tview(p, legs, dims, rm_strides(dims), n, conj);
}

int64_t leg_dim(const TView& t, char c) {
  const auto pos = t.legs.find(c);
  return pos == std::string::npos ? -1 : t.dims[pos];
}

TView restrict_leg(const TView& v, char leg, int64_t start, int64_t len, bool cplx) {
  const auto pos = v.legs.find(leg);
  HP_REQUIRE(pos != std::string::npos && start >= 0 && len >= 1 && start + len <= v.dims[pos], HPEPS_ERR_SHAPE,
             std::string("bad sub-range of leg ") + leg);
  TView r = v;
  const int64_t off = start * v.strides[pos];
  r.p = static_cast<const double*>(v.p) + off * (cplx ? 2 : 1);
  r.dims[pos] = len;
  r.extent = v.extent - off;
  return r;
}

std::vector<int64_t> contract2(Ctx& ctx, bool cplx, const TView& A, const TView& B,
                               const std::string& out, void* C, int64_t c_capacity, bool accumulate) {
  auto dim_of = [&](char c) {
    const int64_t a = leg_dim(A, c), b = leg_dim(B, c);
    HP_REQUIRE(a < 0 || b < 0 || a == b, HPEPS_ERR_SHAPE, std::string("leg dims differ for ") + c);
    return a >= 0 ? a : b;
  };
  std::vector<int64_t> odims;
  char bleg = 0;
  for (char c : out) {
    const int64_t d = dim_of(c);
    HP_REQUIRE(d >= 1, HPEPS_ERR_SHAPE, std::string("output leg not in the operands: ") + c);
    if (leg_dim(A, c) >= 0 && leg_dim(B, c) >= 0) {
      HP_REQUIRE(!bleg, HPEPS_ERR_SHAPE, "at most one batch leg");
      bleg = c;
    }
    odims.push_back(d);
  }
  const auto ost = rm_strides(odims);
  int64_t osize = 1;
  for (auto d : odims) osize *= d;
  HP_REQUIRE(osize <= c_capacity, HPEPS_ERR_SHAPE, "contraction output exceeds its buffer");
  GemmDesc D;
  D.M = D.N = D.K = 1;
  // M: legs of A kept in the output (output order), N: legs of B kept
  for (size_t i = 0; i < out.size(); ++i) {
    const char c = out[i];
    if (c == bleg) continue;
    const auto pa = A.legs.find(c);
    if (pa != std::string::npos) {
      D.Am.add(A.dims[pa], A.strides[pa]);
      D.Cm.add(odims[i], ost[i]);
      D.M *= odims[i];
    } else {
      const auto pb = B.legs.find(c);
      D.Bn.add(B.dims[pb], B.strides[pb]);
      D.Cn.add(odims[i], ost[i]);
      D.N *= odims[i];
    }
  }
  // K: legs shared by A and B and absent from the output
  for (size_t i = 0; i < A.legs.size(); ++i) {
    const char c = A.legs[i];
    if (out.find(c) != std::string::npos) continue;
    const auto pb = B.legs.find(c);
    HP_REQUIRE(pb != std::string::npos, HPEPS_ERR_SHAPE,
               std::string("leg of A neither summed nor kept: ") + c);
    HP_REQUIRE(A.dims[i] == B.dims[pb], HPEPS_ERR_SHAPE, std::string("summed leg dims differ: ") + c);
    D.Ak.add(A.dims[i], A.strides[i]);
    D.Bk.add(B.dims[pb], B.strides[pb]);
    D.K *= A.dims[i];
  }
  for (char c : B.legs)
    HP_REQUIRE(out.find(c) != std::string::npos || A.legs.find(c) != std::string::npos, HPEPS_ERR_SHAPE,
               std::string("leg of B neither summed nor kept: ") + c);
  // index maps need at least one mode
  if (D.Am.n == 0) D.Am.add(1, 0);
  if (D.Cm.n == 0) D.Cm.add(1, 0);
  if (D.Bn.n == 0) D.Bn.add(1, 0);
  if (D.Cn.n == 0) D.Cn.add(1, 0);
  if (D.Ak.n == 0) {
    D.Ak.add(1, 0);
    D.Bk.add(1, 0);
  }
  GemmCall g;
  g.A = A.p;
  g.B = B.p;
  g.C = C;
  g.sA = A.extent;
  g.sB = B.extent;
  g.sC = osize;
  if (bleg) {
    const auto pa = A.legs.find(bleg), pb = B.legs.find(bleg), po = out.find(bleg);
    const int64_t nb = odims[po];
    g.batch = (int)nb;
    g.sA = A.strides[pa];
    g.sB = B.strides[pb];
    g.sC = ost[po];
    HP_REQUIRE(nb < (1LL << 31) && g.sA >= 1 && g.sB >= 1 && nb * g.sA <= A.extent && nb * g.sB <= B.extent,
               HPEPS_ERR_SHAPE, "batch leg strides exceed the operands");
  }
  g.conjA = cplx && A.conj;
  g.conjB = cplx && B.conj;
  g.accumulate = accumulate;
  gemm(ctx, cplx ? Prec::C128 : Prec::F64, D, g);
  return odims;
}

}  // namespace hp
