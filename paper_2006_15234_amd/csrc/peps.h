// Boundary-MPS contraction, norms, energies and two-site updates (internals).
#pragma once
#include <array>

#include "esvd.h"

namespace hp {

// A tensor in device memory with its leg dims (row-major, contiguous).
struct DevTensor {
  void* p = nullptr;
  std::vector<int64_t> dims;
  int64_t size() const {
    int64_t s = 1;
    for (auto d : dims) s *= d;
    return s;
  }
};

enum Side { kTop = 0, kBottom = 1 };
enum Dir { kL2R = 0, kR2L = 1 };

// A site [u,d,l,r,p] seen in an oriented frame: roles (up, down, left, right,
// phys) -> dims and strides of the stored tensor.
struct SiteView {
  const void* p = nullptr;
  int64_t n[5];
  int64_t s[5];
  int64_t extent = 0;
};
SiteView orient_site(const DevTensor& t, Side side, Dir dir);

// A boundary tensor [mL, x, X, mR] seen in an oriented frame: roles (left, x,
// X, right).
struct BndView {
  const void* p = nullptr;
  int64_t n[4];
  int64_t s[4];
  int64_t extent = 0;
};
BndView orient_bnd(const DevTensor& t, Dir dir);

// Exact first-row boundary: out[j] = [l*L, x, X, r*R] (x: down legs for
// side kTop, up legs for kBottom), each normalised; log_dev += logs.
void first_row_boundary(Ctx& ctx, bool cplx, const std::vector<SiteView>& ket,
                        const std::vector<SiteView>& bra, std::vector<DevTensor>& out,
                        double* log_dev);

// Output shapes of a zip-up absorption (host-side shape propagation).
std::vector<std::array<int64_t, 4>> absorb_shapes(const std::vector<BndView>& bnd,
                                                  const std::vector<SiteView>& ket, int64_t m,
                                                  int64_t p);

// One ApproxApply (Alg. 3) in the oriented frame: views are listed in sweep
// order; out[j] receive the canonical [mL,x,X,mR] tensors of the same sweep
// position (their dims are set here); dir tells how to store them.
void absorb_row(Ctx& ctx, bool cplx, const std::vector<BndView>& bnd,
                const std::vector<SiteView>& ket, const std::vector<SiteView>& bra, Dir dir,
                const hpeps_esvd_opts& o, const std::vector<uint64_t>& stream_ids,
                std::vector<DevTensor>& out, double* log_dev);

// Everything a checkpointed zip-up row needs to be rerun in the reverse walk
// (views of its input boundary and sites, its direction, options and sketch
// streams, and its output tensors).
struct RowCheckpoint {
  bool cplx = false;
  std::vector<BndView> bnd;
  std::vector<SiteView> ket, bra;
  Dir dir = kL2R;
  hpeps_esvd_opts o{};
  std::vector<uint64_t> sids;
  std::vector<DevTensor> out;
};

// absorb_row under a recording tape: with Ctx::checkpoint_rows the row runs
// unrecorded and one checkpoint op is recorded in its place; otherwise every
// operation of the row is recorded.  Without a tape it is absorb_row.
void absorb_row_recorded(Ctx& ctx, bool cplx, const std::vector<BndView>& bnd,
                         const std::vector<SiteView>& ket, const std::vector<SiteView>& bra, Dir dir,
                         const hpeps_esvd_opts& o, const std::vector<uint64_t>& stream_ids,
                         std::vector<DevTensor>& out, double* log_dev);

// Exact contraction of a boundary MPS with a last row (its far legs of dim 1)
// in the oriented frame (L2R); writes the (complex) scalar mantissa to
// result_dev (2 doubles) and adds the logs to log_dev.
void contract_last_row(Ctx& ctx, bool cplx, const std::vector<BndView>& bnd,
                       const std::vector<SiteView>& ket, const std::vector<SiteView>& bra,
                       double* result_dev, double* log_dev, double** final_E = nullptr);

// Host view of an ABI PEPS.
struct Lattice {
  int nrow = 0, ncol = 0;
  bool cplx = false;
  std::vector<DevTensor> sites;  // row-major
  const DevTensor& at(int i, int j) const { return sites[(size_t)i * ncol + j]; }
};
Lattice lattice_from_abi(const hpeps_peps* p);

// Copies the accumulated gradient of every site of K (zero where none
// flowed) into the caller's per-site buffers.
void write_site_grads(Ctx& ctx, const Tape& tape, const Lattice& K, void* const* grads);
// Copies every site into the workspace divided by its Frobenius norm; the
// logarithms of the norms are added to log_dev.
Lattice normalized_copy(Ctx& ctx, const Lattice& L, double* log_dev);

// <bra|ket> by the boundary MPS (the lattices must have equal shapes):
// dev[0] = log scale, dev[1..2] = unit-modulus phase (device, 3 doubles).
void norm_lattices(Ctx& c, const Lattice& ket, const Lattice& bra, const hpeps_esvd_opts& o, double* dev);

// Boundary pass from one side storing every intermediate boundary MPS:
// envs[t] = boundary after the first t+1 rows seen from `side`.
void boundary_pass(Ctx& ctx, const Lattice& ket, const Lattice& bra, Side side,
                   const hpeps_esvd_opts& o, int upto, std::vector<std::vector<DevTensor>>& envs,
                   double* log_dev);

}  // namespace hp
