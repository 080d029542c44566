// Reverse-mode tape (see tape.h).
#include <algorithm>

#include "peps.h"
#include "tape.h"

namespace hp {

namespace {

int64_t span(const IndexMap& a, const IndexMap& b) {
  int64_t off = 0;
  for (int i = 0; i < a.n; ++i) off += (a.dim[i] - 1) * a.stride[i];
  for (int i = 0; i < b.n; ++i) off += (b.dim[i] - 1) * b.stride[i];
  return off + 1;
}

int64_t batched(int64_t one, int64_t stride, int batch) { return one + (int64_t)(batch - 1) * stride; }

}  // namespace

bool taping(const Ctx& ctx) { return ctx.tape && ctx.tape->active(); }

void segment_backward(Ctx& ctx, const SegmentCheckpoint& g, Tape& main, double broadening);
bool tape_keeps_workspace(const Ctx& ctx) { return taping(ctx); }

TapeSuspend::TapeSuspend(Ctx& ctx) : c(ctx) {
  if (c.tape) ++c.tape->suspended;
}
TapeSuspend::~TapeSuspend() {
  if (c.tape) --c.tape->suspended;
}

void Tape::touch(const void* p, int64_t n) {
  HP_REQUIRE(p, HPEPS_ERR_INVALID_ARG, "tape: null operand");
  auto it = extent_.find(p);
  if (it == extent_.end())
    extent_[p] = n;
  else
    it->second = std::max(it->second, n);
}

void Tape::note_read(const void* p, int64_t n) {
  touch(p, n);
  read_.insert(p);
}

void Tape::note_write(const void* p, int64_t n, bool in_place) {
  touch(p, n);
  if (in_place) {
    HP_REQUIRE(!read_.count(p), HPEPS_ERR_UNSUPPORTED, "tape: in-place rescaling of a value already read");
  } else {
    HP_REQUIRE(!read_.count(p) && !written_.count(p), HPEPS_ERR_UNSUPPORTED,
               "tape: a recorded operation overwrites a live buffer");
  }
  written_.insert(p);
}

void Tape::mark_input(const void* p, int64_t n) {
  touch(p, n);
  dep_.insert(p);
}

void Tape::record(const TapeOp& op) {
  TapeOp r = op;
  r.cplx = cplx_;
  bool dep = false;
  auto rd = [&](const void* p, int64_t n) {
    note_read(p, n);
    dep = dep || depends(p);
  };
  switch (r.kind) {
    case TapeOp::GEMM: {
      const GemmCall& c = r.c;
      HP_REQUIRE(r.prec == Prec::F64 || r.prec == Prec::C128, HPEPS_ERR_UNSUPPORTED,
                 "tape: products must be FP64 / complex128");
      HP_REQUIRE(!c.nscale && !c.copy_if_zero && !c.accumulate && !c.conjC, HPEPS_ERR_UNSUPPORTED,
                 "tape: unsupported product form");
      HP_REQUIRE(c.batch == 1 || (c.sA > 0 && c.sB > 0 && c.sC > 0), HPEPS_ERR_UNSUPPORTED,
                 "tape: broadcast operands are not supported");
      rd(c.A, batched(span(r.d.Am, r.d.Ak), c.sA, c.batch));
      rd(c.B, batched(span(r.d.Bk, r.d.Bn), c.sB, c.batch));
      note_write(c.C, batched(span(r.d.Cm, r.d.Cn), c.sC, c.batch));
      if (dep) dep_.insert(c.C);
      break;
    }
    case TapeOp::SCALE:
      note_write(r.x, r.n * r.batch, true);
      break;
    case TapeOp::COPY:
      rd(r.src, r.n);
      note_write(r.dst, r.n);
      if (dep) dep_.insert(r.dst);
      break;
    case TapeOp::ZIP:
      HP_REQUIRE(r.o.sketch_precision == HPEPS_F64, HPEPS_ERR_UNSUPPORTED,
                 "tape: einsumsvds must use the FP64 sketch");
      rd(r.op.V, r.L.nV * r.batch);
      rd(r.op.S, r.L.nS * r.batch);
      rd(r.op.T, r.L.nT * r.batch);
      rd(r.op.Bra, r.L.nB * r.batch);
      note_write(r.U, r.out.nU * r.batch);
      note_write(r.R, r.out.nR * r.batch);
      if (dep) {
        dep_.insert(r.U);
        dep_.insert(r.R);
      }
      break;
    case TapeOp::SEG: {
      for (const auto& e : r.seg->inputs) rd(e.first, e.second);
      for (const auto& e : r.seg->outputs) note_write(e.first, e.second);
      if (dep)
        for (const auto& e : r.seg->outputs) dep_.insert(e.first);
      break;
    }
    case TapeOp::ROW: {
      const RowCheckpoint& w = *r.row;
      for (const auto& b : w.bnd) rd(b.p, b.extent);
      for (const auto& t : w.ket) rd(t.p, t.extent);
      for (const auto& t : w.bra) rd(t.p, t.extent);
      for (const auto& o : w.out) note_write(o.p, o.size());
      if (dep)
        for (const auto& o : w.out) dep_.insert(o.p);
      break;
    }
    case TapeOp::CARRY: {
      rd(r.Lm, r.cl.nL * r.batch);
      rd(r.T, r.cl.nT * r.batch);
      rd(r.Bra, r.cl.nB * r.batch);
      const int64_t nv = r.cd.a * r.cd.x * r.cd.x * r.cd.b * r.cd.h * r.cd.h;
      note_write(r.V, nv * r.batch);
      if (dep) dep_.insert(r.V);
      break;
    }
  }
  ops_.push_back(r);
}

double* Tape::grad(Ctx& ctx, const void* p) {
  Adj& a = adj_[p];
  if (!a.g) {
    auto it = extent_.find(p);
    HP_REQUIRE(it != extent_.end(), HPEPS_ERR_INVALID_ARG, "tape: gradient of an unrecorded buffer");
    const int64_t nd = it->second * (cplx_ ? 2 : 1);
    a.g = ctx.ws<double>(nd);
    fill_zero(ctx, a.g, nd * (int64_t)sizeof(double));
  }
  a.live = true;
  return a.g;
}

double* Tape::grad_if_live(const void* p) const {
  auto it = adj_.find(p);
  return it != adj_.end() && it->second.live ? it->second.g : nullptr;
}

void Tape::check_overlaps() const {
  const int64_t es = cplx_ ? 16 : 8;
  std::vector<std::pair<uintptr_t, uintptr_t>> iv;
  for (auto& e : extent_) iv.push_back({(uintptr_t)e.first, (uintptr_t)e.first + (uintptr_t)(e.second * es)});
  std::sort(iv.begin(), iv.end());
  for (size_t i = 1; i < iv.size(); ++i)
    HP_REQUIRE(iv[i].first >= iv[i - 1].second, HPEPS_ERR_UNSUPPORTED,
               "tape: recorded buffers overlap (views into one allocation)");
}

void Tape::backward(Ctx& ctx, double broadening) {
  HP_REQUIRE(ctx.tape == nullptr, HPEPS_ERR_INVALID_ARG, "tape: detach before the reverse walk");
  check_overlaps();
  const int es = cplx_ ? 2 : 1;
  for (auto it = ops_.rbegin(); it != ops_.rend(); ++it) {
    const TapeOp& r = *it;
    switch (r.kind) {
      case TapeOp::GEMM: {
        const double* Cb = grad_if_live(r.c.C);
        if (!Cb) break;
        const GemmDesc& d = r.d;
        const GemmCall& c = r.c;
        if (depends(c.A)) {
          // Abar[m,k] += sum_n Cbar[m,n] conj(op(B)[k,n])   (conjugated when A was)
          GemmDesc D;
          D.M = d.M; D.N = d.K; D.K = d.N;
          D.Am = d.Cm; D.Ak = d.Cn;
          D.Bk = d.Bn; D.Bn = d.Bk;
          D.Cm = d.Am; D.Cn = d.Ak;
          GemmCall g;
          g.A = Cb; g.B = c.B; g.C = grad(ctx, c.A);
          g.sA = c.sC; g.sB = c.sB; g.sC = c.sA;
          g.nA = c.nC; g.nB = c.nB; g.nC = c.nA;
          g.batch = c.batch;
          g.conjA = r.cplx && c.conjA;
          g.conjB = r.cplx && (c.conjA ? c.conjB : !c.conjB);
          g.alpha = c.alpha;
          g.scale = c.scale;
          g.accumulate = true;
          gemm(ctx, r.prec, D, g);
        }
        if (depends(c.B)) {
          // Bbar[k,n] += sum_m conj(op(A)[m,k]) Cbar[m,n]   (conjugated when B was)
          GemmDesc D;
          D.M = d.K; D.N = d.N; D.K = d.M;
          D.Am = d.Ak; D.Ak = d.Am;
          D.Bk = d.Cm; D.Bn = d.Cn;
          D.Cm = d.Bk; D.Cn = d.Bn;
          GemmCall g;
          g.A = c.A; g.B = Cb; g.C = grad(ctx, c.B);
          g.sA = c.sA; g.sB = c.sC; g.sC = c.sB;
          g.nA = c.nA; g.nB = c.nC; g.nC = c.nB;
          g.batch = c.batch;
          g.conjA = r.cplx && (c.conjB ? c.conjA : !c.conjA);
          g.conjB = r.cplx && c.conjB;
          g.alpha = c.alpha;
          g.scale = c.scale;
          g.accumulate = true;
          gemm(ctx, r.prec, D, g);
        }
        break;
      }
      case TapeOp::SCALE: {
        double* g = grad_if_live(r.x);
        if (g) scale_by(ctx, g, r.n * es, r.s, r.batch);
        break;
      }
      case TapeOp::COPY: {
        const double* g = grad_if_live(r.dst);
        if (g && depends(r.src)) axpy(ctx, grad(ctx, r.src), g, 1.0, r.n * es);
        break;
      }
      case TapeOp::ZIP: {
        if (!grad_if_live(r.U) && !grad_if_live(r.R)) break;
        const double* dU = grad(ctx, r.U);
        const double* dR = grad(ctx, r.R);
        auto gp = [&](const void* p) -> void* { return depends(p) ? grad(ctx, p) : nullptr; };
        void* gV = gp(r.op.V);
        void* gS = gp(r.op.S);
        void* gT = gp(r.op.T);
        void* gB = gp(r.op.Bra);
        if (!gV && !gS && !gT && !gB) break;
        zip_esvd_backward(ctx, r.cplx, r.z, r.L, r.op, r.batch, r.o, r.absorb, broadening, r.out, dU, nullptr, dR,
                          gV, gS, gT, gB);
        break;
      }
      case TapeOp::ROW:
        row_backward(ctx, *r.row, *this, broadening);
        break;
      case TapeOp::SEG:
        segment_backward(ctx, *r.seg, *this, broadening);
        break;
      case TapeOp::CARRY: {
        const double* gVc = grad_if_live(r.V);
        if (!gVc) break;
        auto gp = [&](const void* p) -> void* { return depends(p) ? grad(ctx, p) : nullptr; };
        void* gL = gp(r.Lm);
        void* gT = gp(r.T);
        void* gB = gp(r.Bra);
        if (!gL && !gT && !gB) break;
        carry_backward(ctx, r.cplx, r.cd, r.cl, r.Lm, r.T, r.Bra, gVc, gL, gT, gB, r.batch);
        break;
      }
    }
  }
}

void tape_gemm(Ctx& ctx, Prec prec, const GemmDesc& d, const GemmCall& c) {
  if (!taping(ctx)) return;
  TapeOp op;
  op.kind = TapeOp::GEMM;
  op.prec = prec;
  op.d = d;
  op.c = c;
  ctx.tape->record(op);
}

void tape_scale(Ctx& ctx, bool, double* x, int64_t n, const double* s, int batch) {
  if (!taping(ctx)) return;
  TapeOp op;
  op.kind = TapeOp::SCALE;
  op.x = x;
  op.n = n;
  op.s = s;
  op.batch = batch;
  ctx.tape->record(op);
}

void tape_copy(Ctx& ctx, bool, void* dst, const void* src, int64_t n) {
  if (!taping(ctx)) return;
  TapeOp op;
  op.kind = TapeOp::COPY;
  op.dst = dst;
  op.src = src;
  op.n = n;
  ctx.tape->record(op);
}

void tape_zip(Ctx& ctx, bool, const ZipDims& z, const ZipLayout& L, const ZipOperands& zo, int batch,
              const hpeps_esvd_opts& o, hpeps_absorb absorb, const ZipOut& out, void* U, void* R) {
  if (!taping(ctx)) return;
  TapeOp op;
  op.kind = TapeOp::ZIP;
  op.z = z;
  op.L = L;
  op.op = zo;
  op.batch = batch;
  op.o = o;
  op.absorb = absorb;
  op.out = out;
  op.U = U;
  op.R = R;
  ctx.tape->record(op);
}

void tape_carry(Ctx& ctx, bool, const CarryDims& cd, const CarryLayout& cl, const void* Lm, const void* T,
                const void* Bra, void* V, int batch) {
  if (!taping(ctx)) return;
  TapeOp op;
  op.kind = TapeOp::CARRY;
  op.cd = cd;
  op.cl = cl;
  op.Lm = Lm;
  op.T = T;
  op.Bra = Bra;
  op.V = V;
  op.batch = batch;
  ctx.tape->record(op);
}

void run_segment(Ctx& ctx, bool cplx, const std::vector<std::pair<const void*, int64_t>>& inputs,
                 const std::vector<std::pair<void*, int64_t>>& outputs,
                 std::function<void(Ctx&, const std::vector<void*>&)> run) {
  std::vector<void*> outs;
  for (const auto& e : outputs) outs.push_back(e.first);
  if (!taping(ctx) || !ctx.checkpoint_rows) {
    run(ctx, outs);
    return;
  }
  {
    TapeSuspend unrecorded(ctx);  // the segment's workspace is released at its end
    WsScope scope(ctx);
    run(ctx, outs);
  }
  auto seg = std::make_shared<SegmentCheckpoint>();
  seg->cplx = cplx;
  seg->inputs = inputs;
  seg->outputs = outputs;
  seg->rerun = std::move(run);
  TapeOp op;
  op.kind = TapeOp::SEG;
  op.seg = seg;
  ctx.tape->record(op);
}

// The reverse step of a checkpointed segment: rerun it on a tape of its own
// into fresh outputs, seed that tape with the adjoints of the recorded
// outputs, walk it back and add the adjoints of the inputs.
void segment_backward(Ctx& ctx, const SegmentCheckpoint& g, Tape& main, double broadening) {
  const int es = g.cplx ? 2 : 1;
  bool any = false;
  for (const auto& e : g.outputs) any = any || main.grad_if_live(e.first);
  if (!any) return;
  std::vector<std::pair<const void*, int64_t>> ins;
  for (const auto& e : g.inputs) {
    if (!main.depends(e.first)) continue;
    bool seen = false;
    for (auto& x : ins)
      if (x.first == e.first) {
        x.second = std::max(x.second, e.second);
        seen = true;
      }
    if (!seen) ins.push_back(e);
  }
  std::vector<double*> gmain;
  for (auto& e : ins) gmain.push_back(main.grad(ctx, e.first));
  WsScope scope(ctx);
  std::vector<void*> outs;
  for (const auto& e : g.outputs) outs.push_back(ctx.ws<double>(e.second * es));
  Tape sub(g.cplx);
  for (auto& e : ins) sub.mark_input(e.first, e.second);
  ctx.tape = &sub;
  try {
    g.rerun(ctx, outs);
  } catch (...) {
    ctx.tape = nullptr;
    throw;
  }
  ctx.tape = nullptr;
  for (size_t q = 0; q < g.outputs.size(); ++q) {
    const double* gm = main.grad_if_live(g.outputs[q].first);
    if (gm && sub.depends(outs[q]))
      HP_CHECK_HIP(hipMemcpyAsync(sub.grad(ctx, outs[q]), gm, g.outputs[q].second * es * sizeof(double),
                                  hipMemcpyDeviceToDevice, ctx.stream));
  }
  sub.backward(ctx, broadening);
  for (size_t i = 0; i < ins.size(); ++i) {
    const double* gs = sub.grad_if_live(ins[i].first);
    if (gs) axpy(ctx, gmain[i], gs, 1.0, ins[i].second * es);
  }
}

}  // namespace hp
