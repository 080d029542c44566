// Reverse-mode tape for the contraction algorithms (einsumsvd adjoints).
//
// While a tape records (Ctx::tape set and not suspended), every gathered
// product, in-place rescaling, exact carry, zip-up einsumsvd and device copy
// that the forward code issues is logged with its operands, and workspace
// scopes keep their memory, so every value the reverse walk reads is still
// in place (single assignment: a recorded op may not overwrite a buffer that
// an earlier op read or wrote, except an in-place rescaling of a fresh value).
// The reverse walk accumulates conjugate-Wirtinger cotangents (dL/dRe +
// i dL/dIm of a real loss) into one adjoint buffer per forward buffer:
//   * product C = op(A) op(B):  the two adjoint products, conjugations
//     propagated, accumulated into the adjoints of A and B;
//   * rescaling x *= s:         the factor is a constant (normalisations only
//     move logarithmic accumulators; ratios and log-derivatives do not see
//     them), so adj(x) *= s;
//   * einsumsvd:                zip_esvd_backward (forward recomputed from its
//     recorded inputs: per-einsumsvd checkpoint and recompute);
//   * exact carry:              carry_backward;
//   * copy dst = src:           adj(src) += adj(dst);
//   * segment (checkpoint):     an energy strip, handled like a row below;
//   * zip-up row (checkpoint):  the row ran unrecorded in the forward pass;
//     the reverse walk reruns it from its recorded input boundary and sites
//     on a tape of its own, seeds that tape with the adjoints of the row's
//     outputs, walks it back and adds the adjoints of the row's inputs
//     (per-row checkpoint and recompute: only the boundary MPS of each row
//     is kept between the passes).
// Only values that depend on an input marked with mark_input get adjoints.
#pragma once
#include <functional>
#include <map>
#include <set>
#include <vector>

#include "esvd.h"

#include <memory>

namespace hp {

struct RowCheckpoint;  // peps.h

// A checkpointed segment of the forward pass (one energy strip): its inputs
// and outputs, and a closure that reruns it writing the outputs to the given
// buffers (in the order of `outputs`).
struct SegmentCheckpoint {
  bool cplx = false;
  std::vector<std::pair<const void*, int64_t>> inputs;   // (pointer, elements)
  std::vector<std::pair<void*, int64_t>> outputs;        // (pointer, elements)
  std::function<void(Ctx&, const std::vector<void*>&)> rerun;
};

struct TapeOp {
  enum Kind { GEMM, SCALE, ZIP, CARRY, COPY, ROW, SEG } kind = GEMM;
  // ROW
  std::shared_ptr<const RowCheckpoint> row;
  // SEG
  std::shared_ptr<const SegmentCheckpoint> seg;
  bool cplx = false;
  // GEMM
  Prec prec = Prec::F64;
  GemmDesc d;
  GemmCall c;
  // SCALE (x[b][0..n) *= s[b], n elements) / COPY (dst[0..n) = src[0..n))
  double* x = nullptr;
  const double* s = nullptr;
  int64_t n = 0;
  int batch = 1;
  void* dst = nullptr;
  const void* src = nullptr;
  // ZIP
  ZipDims z;
  ZipLayout L;
  ZipOperands op;
  hpeps_esvd_opts o{};
  hpeps_absorb absorb = HPEPS_ABSORB_CARRY;
  ZipOut out;
  void* U = nullptr;
  void* R = nullptr;
  // CARRY
  CarryDims cd;
  CarryLayout cl;
  const void* Lm = nullptr;
  const void* T = nullptr;
  const void* Bra = nullptr;
  void* V = nullptr;
};

class Tape {
 public:
  explicit Tape(bool cplx) : cplx_(cplx) {}
  int suspended = 0;
  bool active() const { return suspended == 0; }

  void mark_input(const void* p, int64_t n);   // n elements
  void record(const TapeOp& op);
  bool depends(const void* p) const { return dep_.count(p) != 0; }
  // adjoint buffer of p (allocated and zeroed on first use), marked live
  double* grad(Ctx& ctx, const void* p);
  // adjoint of p if it was ever accumulated into, else nullptr
  double* grad_if_live(const void* p) const;
  // walk the tape backwards (the context's tape must already be detached)
  void backward(Ctx& ctx, double broadening);

 private:
  bool cplx_;
  std::vector<TapeOp> ops_;
  std::map<const void*, int64_t> extent_;      // elements
  std::set<const void*> dep_, read_, written_;
  struct Adj {
    double* g = nullptr;
    bool live = false;
  };
  std::map<const void*, Adj> adj_;
  void touch(const void* p, int64_t n);
  void note_read(const void* p, int64_t n);
  void note_write(const void* p, int64_t n, bool in_place = false);
  void check_overlaps() const;
};

// RAII: suspends recording (the einsumsvd and carry macro-ops record
// themselves once and run their internals unrecorded)
struct TapeSuspend {
  Ctx& c;
  explicit TapeSuspend(Ctx& ctx);
  ~TapeSuspend();
};

bool taping(const Ctx& ctx);
// reverse step of a checkpointed row (peps.hip): recompute, local tape, adjoints
void row_backward(Ctx& ctx, const RowCheckpoint& r, Tape& main, double broadening);
// Runs `run` (writing the listed outputs) unrecorded and records one segment
// op in its place when a tape records with Ctx::checkpoint_rows; otherwise
// runs it recorded (or plainly, without a tape).
void run_segment(Ctx& ctx, bool cplx, const std::vector<std::pair<const void*, int64_t>>& inputs,
                 const std::vector<std::pair<void*, int64_t>>& outputs,
                 std::function<void(Ctx&, const std::vector<void*>&)> run);
void tape_zip(Ctx& ctx, bool cplx, const ZipDims& z, const ZipLayout& L, const ZipOperands& op, int batch,
              const hpeps_esvd_opts& o, hpeps_absorb absorb, const ZipOut& out, void* U, void* R);
void tape_carry(Ctx& ctx, bool cplx, const CarryDims& cd, const CarryLayout& cl, const void* Lm, const void* T,
                const void* Bra, void* V, int batch);

}  // namespace hp
