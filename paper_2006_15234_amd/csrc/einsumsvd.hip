// einsumsvd of an arbitrary tensor network (Sec. II-C): the network given by
// an einsum-style subscript string is read as a matrix whose rows are the
// open legs left of '|' and whose columns are the open legs right of it,
// and is factorized by the randomized SVD of Alg. 4 without ever being
// formed: A X and A^* Y are evaluated as sequences of pairwise tensor
// contractions of the network with the sketch panel (Sec. IV-A), each one
// gathered GEMM (contract.hip).
#include <algorithm>
#include <string>
#include <vector>

#include "contract.h"
#include "esvd.h"

namespace hp {
namespace {

constexpr char kSketchLeg = '#';  // the panel's k leg (never a subscript letter)
constexpr char kBatchLeg = '$';   // the instance leg of the batched form (likewise)

struct Network {
  std::vector<TView> ops;
  std::string left, right;               // open legs of the rows / columns, in order
  std::vector<int64_t> ldims, rdims;
  int64_t rows = 1, cols = 1;
  // batched form: every operand carries the instance leg kBatchLeg (its
  // leading dimension); 0 for the single network
  int64_t batch = 0;
  std::string bl() const { return batch ? std::string(1, kBatchLeg) : std::string(); }
  std::vector<int64_t> bd() const { return batch ? std::vector<int64_t>{batch} : std::vector<int64_t>{}; }
};

// Legs of the product of the running tensor `cur` with `op` (the legs of
// either that the other lacks; the instance leg first and kept) and the
// number of legs they share besides it.
std::string product_legs(const Network& net, const TView& cur, const TView& op, int* shared) {
  std::string o = net.bl();
  *shared = 0;
  for (char c : cur.legs) {
    if (c == kBatchLeg) continue;
    if (op.legs.find(c) == std::string::npos) o += c; else ++*shared;
  }
  for (char c : op.legs)
    if (c != kBatchLeg && cur.legs.find(c) == std::string::npos) o += c;
  return o;
}

bool leg_char(char c) { return (c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z'); }

// batch 0: the single network; batch >= 1: every operand has one more,
// leading, dimension of extent `batch` (the instance leg), whose stride is
// at least one instance's extent.
Network parse(const char* subscripts, int n_ops, const hpeps_tensor* ops, bool cplx, int64_t batch = 0) {
  HP_REQUIRE(subscripts && ops && n_ops >= 1 && n_ops <= 64, HPEPS_ERR_INVALID_ARG, "bad einsumsvd operands");
  HP_REQUIRE(batch >= 0 && batch < (1LL << 31), HPEPS_ERR_INVALID_ARG, "bad batch count");
  const std::string s(subscripts);
  const auto arrow = s.find("->");
  HP_REQUIRE(arrow != std::string::npos, HPEPS_ERR_INVALID_ARG, "subscripts need '->'");
  const std::string lhs = s.substr(0, arrow), rhs = s.substr(arrow + 2);
  const auto bar = rhs.find('|');
  HP_REQUIRE(bar != std::string::npos && rhs.find('|', bar + 1) == std::string::npos, HPEPS_ERR_INVALID_ARG,
             "the output needs exactly one '|' between row legs and column legs");
  Network net;
  net.batch = batch;
  const int lead = batch ? 1 : 0;
  net.left = rhs.substr(0, bar);
  net.right = rhs.substr(bar + 1);
  HP_REQUIRE(!net.left.empty() && !net.right.empty(), HPEPS_ERR_INVALID_ARG, "empty row or column legs");
  std::vector<std::string> terms;
  size_t start = 0;
  for (;;) {
    const auto comma = lhs.find(',', start);
    terms.push_back(lhs.substr(start, comma == std::string::npos ? std::string::npos : comma - start));
    if (comma == std::string::npos) break;
    start = comma + 1;
  }
  HP_REQUIRE((int)terms.size() == n_ops, HPEPS_ERR_INVALID_ARG, "subscripts and operand count differ");
  // leg counts: every leg must appear twice over operands and output
  int count[128] = {0};
  int64_t dim[128];
  std::fill(dim, dim + 128, -1);
  for (int i = 0; i < n_ops; ++i) {
    const std::string& t = terms[i];
    const hpeps_tensor& o = ops[i];
    HP_REQUIRE(o.data, HPEPS_ERR_INVALID_ARG, "null operand");
    HP_REQUIRE(o.ndim >= 1 + lead && o.ndim <= 8 && (int)t.size() + lead == o.ndim, HPEPS_ERR_SHAPE,
               "operand " + std::to_string(i) + (batch ? ": legs + 1 (the batch dimension) and ndim differ"
                                                       : ": legs and ndim differ"));
    std::vector<int64_t> dims(o.shape + lead, o.shape + o.ndim), strides(o.strides + lead, o.strides + o.ndim);
    int64_t extent = 1;
    for (int q = 0; q < (int)t.size(); ++q) {
      const char c = t[q];
      HP_REQUIRE(leg_char(c), HPEPS_ERR_INVALID_ARG, "legs are letters a-z, A-Z");
      HP_REQUIRE(t.find(c) == (size_t)q, HPEPS_ERR_INVALID_ARG, "a leg repeated within one operand");
      HP_REQUIRE(dims[q] >= 1, HPEPS_ERR_SHAPE, "dimensions must be >= 1");
      HP_REQUIRE(strides[q] >= 1 || dims[q] == 1, HPEPS_ERR_SHAPE, "strides must be >= 1");
      if (dims[q] == 1) strides[q] = std::max<int64_t>(strides[q], 0);
      extent += (dims[q] - 1) * strides[q];
      HP_REQUIRE(dim[(int)c] < 0 || dim[(int)c] == dims[q], HPEPS_ERR_SHAPE, std::string("dims of leg ") + c + " differ");
      dim[(int)c] = dims[q];
      ++count[(int)c];
    }
    if (batch) {
      // instances are disjoint blocks: the batch stride covers one instance
      HP_REQUIRE(o.shape[0] == batch, HPEPS_ERR_SHAPE,
                 "operand " + std::to_string(i) + ": leading dimension differs from the batch count");
      const int64_t bs = batch == 1 ? std::max<int64_t>(o.strides[0], extent) : o.strides[0];
      HP_REQUIRE(bs >= extent, HPEPS_ERR_SHAPE,
                 "operand " + std::to_string(i) + ": batch stride smaller than one instance");
      dims.insert(dims.begin(), batch);
      strides.insert(strides.begin(), bs);
      extent = batch * bs;
      net.ops.push_back(tview(o.data, std::string(1, kBatchLeg) + t, dims, strides, extent, cplx && o.conj != 0));
    } else {
      net.ops.push_back(tview(o.data, t, dims, strides, extent, cplx && o.conj != 0));
    }
  }
  for (char c : net.left + net.right) {
    HP_REQUIRE(leg_char(c), HPEPS_ERR_INVALID_ARG, "legs are letters a-z, A-Z");
    HP_REQUIRE(count[(int)c] == 1, HPEPS_ERR_INVALID_ARG,
               std::string("open leg ") + c + " must appear in exactly one operand and once in the output");
    ++count[(int)c];
  }
  for (int c = 0; c < 128; ++c)
    HP_REQUIRE(count[c] == 0 || count[c] == 2, HPEPS_ERR_INVALID_ARG,
               std::string("leg ") + (char)c + " must join exactly two operands or be open");
  for (char c : net.left) {
    net.ldims.push_back(dim[(int)c]);
    net.rows *= dim[(int)c];
  }
  for (char c : net.right) {
    net.rdims.push_back(dim[(int)c]);
    net.cols *= dim[(int)c];
  }
  return net;
}

int64_t vol(const std::string& legs, const TView& A, const TView& B) {
  int64_t n = 1;
  for (char c : legs) {
    const int64_t a = leg_dim(A, c);
    n *= a >= 0 ? a : leg_dim(B, c);
  }
  return n;
}

// Contracts the panel X (legs `in` + k) with every operand, greedily: next
// the operand sharing the most legs with the running tensor (ties: the
// smaller result); the last product writes Y in the row-major order `out` + k.
void apply_network(Ctx& ctx, bool cplx, const Network& net, bool adjoint, const double* X, double* Y, int64_t k) {
  WsScope scope(ctx);
  const std::string& in = adjoint ? net.left : net.right;
  const std::string& out = adjoint ? net.right : net.left;
  std::vector<int64_t> idims = net.bd();
  for (int64_t d : adjoint ? net.ldims : net.rdims) idims.push_back(d);
  idims.push_back(k);
  TView cur = tview_rm(X, net.bl() + in + kSketchLeg, idims);
  std::vector<TView> rest = net.ops;
  if (adjoint)
    for (auto& v : rest) v.conj = cplx && !v.conj;
  while (!rest.empty()) {
    int best = -1, best_shared = -1;
    int64_t best_size = 0;
    std::string best_out;
    for (int i = 0; i < (int)rest.size(); ++i) {
      int shared = 0;
      const std::string o = product_legs(net, cur, rest[i], &shared);
      const int64_t sz = vol(o, cur, rest[i]);
      if (shared > best_shared || (shared == best_shared && sz < best_size)) {
        best = i;
        best_shared = shared;
        best_size = sz;
        best_out = o;
      }
    }
    const TView op = rest[best];
    rest.erase(rest.begin() + best);
    if (rest.empty()) {
      // the legs left must be the output legs and the panel leg
      std::string want = net.bl() + out + kSketchLeg;
      HP_REQUIRE(best_out.size() == want.size(), HPEPS_ERR_INVALID_ARG, "network legs do not close");
      for (char c : want)
        HP_REQUIRE(best_out.find(c) != std::string::npos, HPEPS_ERR_INVALID_ARG, "network legs do not close");
      int64_t n = 1;
      for (char c : want) n *= std::max(leg_dim(cur, c), leg_dim(op, c));
      contract2(ctx, cplx, cur, op, want, Y, n);
    } else {
      double* buf = ctx.ws<double>(best_size * (cplx ? 2 : 1));
      const auto dims = contract2(ctx, cplx, cur, op, best_out, buf, best_size);
      cur = tview_rm(buf, best_out, dims);
    }
  }
}

// The network contracted into its matrix: A [rows][cols] (legs left + right),
// or A^* [cols][rows] (legs right + left, every operand conjugated) with
// `adjoint`.  Operands are taken greedily as in apply_network, starting from
// the first.
void form_network(Ctx& ctx, bool cplx, const Network& net, bool adjoint, double* M) {
  WsScope scope(ctx);
  std::vector<TView> rest = net.ops;
  if (adjoint)
    for (auto& v : rest) v.conj = cplx && !v.conj;
  const std::string want = net.bl() + (adjoint ? net.right + net.left : net.left + net.right);
  const int64_t total = std::max<int64_t>(net.batch, 1) * net.rows * net.cols;
  if (rest.size() == 1) {
    // one operand: a permuted copy, as a contraction with a one-element tensor
    // over a unit leg
    double* one = ctx.ws<double>(cplx ? 2 : 1);
    fill_value(ctx, one, 1, 1.0, cplx);
    TView op = rest[0];
    op.legs += '@';
    op.dims.push_back(1);
    op.strides.push_back(0);
    contract2(ctx, cplx, op, tview_rm(one, "@", {1}), want, M, total);
    return;
  }
  TView cur = rest[0];
  rest.erase(rest.begin());
  while (!rest.empty()) {
    int best = -1, best_shared = -1;
    int64_t best_size = 0;
    std::string best_out;
    for (int i = 0; i < (int)rest.size(); ++i) {
      int shared = 0;
      const std::string o = product_legs(net, cur, rest[i], &shared);
      const int64_t sz = vol(o, cur, rest[i]);
      if (shared > best_shared || (shared == best_shared && sz < best_size)) {
        best = i;
        best_shared = shared;
        best_size = sz;
        best_out = o;
      }
    }
    const TView op = rest[best];
    rest.erase(rest.begin() + best);
    if (rest.empty()) {
      HP_REQUIRE(best_out.size() == want.size(), HPEPS_ERR_INVALID_ARG, "network legs do not close");
      for (char c : want)
        HP_REQUIRE(best_out.find(c) != std::string::npos, HPEPS_ERR_INVALID_ARG, "network legs do not close");
      contract2(ctx, cplx, cur, op, want, M, total);
    } else {
      double* buf = ctx.ws<double>(best_size * (cplx ? 2 : 1));
      const auto dims = contract2(ctx, cplx, cur, op, best_out, buf, best_size);
      cur = tview_rm(buf, best_out, dims);
    }
  }
}

// Contracts the tensors `ts` greedily (as apply_network, from the first)
// into C, row-major in the order of `want`, adding to what C holds.
void contract_all(Ctx& ctx, bool cplx, const Network& net, std::vector<TView> ts, const std::string& want, void* C,
                  int64_t c_elems) {
  WsScope scope(ctx);
  TView cur = ts[0];
  ts.erase(ts.begin());
  while (!ts.empty()) {
    int best = -1, best_shared = -1;
    int64_t best_size = 0;
    std::string best_out;
    for (int i = 0; i < (int)ts.size(); ++i) {
      int shared = 0;
      const std::string o = product_legs(net, cur, ts[i], &shared);
      const int64_t sz = vol(o, cur, ts[i]);
      if (shared > best_shared || (shared == best_shared && sz < best_size)) {
        best = i;
        best_shared = shared;
        best_size = sz;
        best_out = o;
      }
    }
    const TView op = ts[best];
    ts.erase(ts.begin() + best);
    if (ts.empty()) {
      HP_REQUIRE(best_out.size() == want.size(), HPEPS_ERR_INVALID_ARG, "network legs do not close");
      for (char c : want)
        HP_REQUIRE(best_out.find(c) != std::string::npos, HPEPS_ERR_INVALID_ARG, "network legs do not close");
      contract2(ctx, cplx, cur, op, want, C, c_elems, true);
    } else {
      double* buf = ctx.ws<double>(best_size * (cplx ? 2 : 1));
      const auto dims = contract2(ctx, cplx, cur, op, best_out, buf, best_size);
      cur = tview_rm(buf, best_out, dims);
    }
  }
}

// The einsumsvd of BMPS: the explicit matrix and its dense truncated SVD.
void einsumsvd_explicit(Ctx& ctx, bool cplx, const Network& net, const hpeps_esvd_opts& o, hpeps_absorb absorb,
                        void* U, double* sigma, void* R, double* log_scale) {
  WsScope scope(ctx);
  const int64_t rows = net.rows, cols = net.cols;
  const int64_t k = std::min(rows, cols);
  const int64_t mp = std::min<int64_t>(o.rank, k);
  HP_REQUIRE(k <= (cplx ? 88 : 128), HPEPS_ERR_SHAPE,
             "explicit einsumsvd: min(rows, cols) must be <= 128 (88 complex)");
  ctx.last_rank = mp;
  ctx.last_k = k;
  const int es = cplx ? 2 : 1;
  const int nb = (int)std::max<int64_t>(net.batch, 1);
  double* M = ctx.ws<double>(nb * rows * cols * es);
  ZipOut out;
  out.Urows.add(rows, mp);
  out.Ucol.add(mp, 1);
  out.Rrow.add(mp, cols);
  out.Rcols.add(cols, 1);
  out.nU = rows * mp;
  out.nR = mp * cols;
  const bool wide = rows <= cols;
  form_network(ctx, cplx, net, wide, M);
  std::vector<int64_t> mdims = net.bd(), pdims = net.bd();
  mdims.insert(mdims.end(), net.ldims.begin(), net.ldims.end());
  mdims.insert(mdims.end(), net.rdims.begin(), net.rdims.end());
  pdims.insert(pdims.end(), net.ldims.begin(), net.ldims.end());
  pdims.push_back(k);
  const std::string b = net.bl();
  dense_finish(ctx, cplx, rows, cols, mp, nb, o, absorb, out, U, sigma, R, log_scale, M,
               [&](bool, const double* P, double* Bs) {
                 contract2(ctx, cplx, tview_rm(M, b + net.left + net.right, mdims, cplx),
                           tview_rm(P, b + net.left + kSketchLeg, pdims), b + net.right + kSketchLeg, Bs,
                           nb * cols * k);
               });
}

}  // namespace

void einsumsvd_network(Ctx& ctx, bool cplx, const char* subscripts, int n_ops, const hpeps_tensor* ops,
                       const hpeps_esvd_opts& o, hpeps_absorb absorb, void* U, double* sigma, void* R,
                       double* log_scale, int64_t batch) {
  WsScope scope(ctx);
  HP_REQUIRE(o.sketch_precision == HPEPS_F64, HPEPS_ERR_DTYPE, "network einsumsvd runs in FP64 / complex128");
  const Network net = parse(subscripts, n_ops, ops, cplx, batch);
  HP_REQUIRE(o.method == HPEPS_ESVD_IMPLICIT || o.method == HPEPS_ESVD_EXPLICIT, HPEPS_ERR_INVALID_ARG,
             "unknown einsumsvd method");
  if (o.method == HPEPS_ESVD_EXPLICIT) {
    HP_REQUIRE(net.rows < (1LL << 31) && net.cols < (1LL << 31), HPEPS_ERR_UNSUPPORTED, "matrix dimension too large");
    einsumsvd_explicit(ctx, cplx, net, o, absorb, U, sigma, R, log_scale);
    return;
  }
  const int64_t rows = net.rows, cols = net.cols;
  const int64_t k = sketch_width(o.rank, o.oversample, rows, cols);
  const int64_t mp = std::min<int64_t>(o.rank, k);
  HP_REQUIRE(k >= 1 && k <= (cplx ? 88 : 128), HPEPS_ERR_SHAPE, "sketch width k out of range");
  HP_REQUIRE(rows < (1LL << 31) && cols < (1LL << 31), HPEPS_ERR_UNSUPPORTED, "matrix dimension too large");
  ctx.last_rank = mp;
  ctx.last_k = k;
  const int es = cplx ? 2 : 1;
  // instance b of a batch draws its sketch from stream stream_id + b
  const int nb = (int)std::max<int64_t>(net.batch, 1);
  double* Om = ctx.ws<double>(nb * cols * k * es);
  double* Y0 = ctx.ws<double>(nb * rows * k * es);
  sketch(ctx, Om, false, cols, k, nb, o.seed, o.stream_id, cplx);
  apply_network(ctx, cplx, net, false, Om, Y0, k);
  ZipOut out;
  out.Urows.add(rows, mp);
  out.Ucol.add(mp, 1);
  out.Rrow.add(mp, cols);
  out.Rcols.add(cols, 1);
  out.nU = rows * mp;
  out.nR = mp * cols;
  rsvd_finish(ctx, cplx, rows, cols, k, mp, nb, o, absorb, out, U, sigma, R, log_scale, Y0,
              [&](bool adj, const double* X, double* Y) { apply_network(ctx, cplx, net, adj, X, Y, k); });
}

// Adjoint of the network einsumsvd.  The reverse walk through Alg. 4 gives
// the operator's cotangent as rank-k terms Abar = sum_t L_t R_t^H; the
// gradient of operand i is the network without operand i, closed by L_t on
// the row legs and R_t on the column legs (summed over the k leg and the
// terms).  Gradients follow the conjugate-Wirtinger convention (dL/dRe +
// i dL/dIm): for an operand that enters as itself the contraction takes L_t,
// conj(R_t) and every other operand conjugated once more; for one that
// enters conjugated, conj(L_t), R_t and the others as they enter.
void einsumsvd_network_backward(Ctx& ctx, bool cplx, const char* subscripts, int n_ops, const hpeps_tensor* ops,
                                const hpeps_esvd_opts& o, hpeps_absorb absorb, double broadening, const void* dU,
                                const double* dsigma, const void* dR, void* const* grads, int64_t batch) {
  WsScope scope(ctx);
  HP_REQUIRE(o.method == HPEPS_ESVD_IMPLICIT, HPEPS_ERR_UNSUPPORTED,
             "the adjoint differentiates the randomized (implicit) einsumsvd");
  HP_REQUIRE(grads && dU && dR, HPEPS_ERR_INVALID_ARG, "null argument");
  const Network net = parse(subscripts, n_ops, ops, cplx, batch);
  const int64_t rows = net.rows, cols = net.cols;
  const int64_t k = sketch_width(o.rank, o.oversample, rows, cols);
  const int64_t mp = std::min<int64_t>(o.rank, k);
  HP_REQUIRE(k >= 1 && k <= (cplx ? 88 : 128), HPEPS_ERR_SHAPE, "sketch width k out of range");
  HP_REQUIRE(rows < (1LL << 31) && cols < (1LL << 31), HPEPS_ERR_UNSUPPORTED, "matrix dimension too large");
  const int nb = (int)std::max<int64_t>(net.batch, 1);
  const int es = cplx ? 2 : 1;
  ZipOut out;
  out.Urows.add(rows, mp);
  out.Ucol.add(mp, 1);
  out.Rrow.add(mp, cols);
  out.Rcols.add(cols, 1);
  out.nU = rows * mp;
  out.nR = mp * cols;
  RankTerms terms;
  rsvd_backward_terms(ctx, cplx, rows, cols, nb, o, absorb, broadening, out, dU, dsigma, dR,
                      [&](bool adj, const double* X, double* Y) { apply_network(ctx, cplx, net, adj, X, Y, k); },
                      terms);
  const std::string b = net.bl();
  std::vector<int64_t> ldk = net.bd(), rdk = net.bd();
  ldk.insert(ldk.end(), net.ldims.begin(), net.ldims.end());
  ldk.push_back(k);
  rdk.insert(rdk.end(), net.rdims.begin(), net.rdims.end());
  rdk.push_back(k);
  for (int i = 0; i < n_ops; ++i) {
    if (!grads[i]) continue;
    const TView& oi = net.ops[i];
    int64_t n = 1;
    for (int64_t d : oi.dims) n *= d;
    fill_zero(ctx, grads[i], n * es * 8);
    const bool flip = !oi.conj;
    for (const auto& t : terms) {
      std::vector<TView> ts;
      ts.push_back(tview_rm(t.first, b + net.left + kSketchLeg, ldk, cplx && !flip));
      ts.push_back(tview_rm(t.second, b + net.right + kSketchLeg, rdk, cplx && flip));
      for (int j = 0; j < n_ops; ++j) {
        if (j == i) continue;
        TView v = net.ops[j];
        v.conj = cplx && (v.conj != flip);
        ts.push_back(v);
      }
      contract_all(ctx, cplx, net, ts, oi.legs, grads[i], n);
    }
  }
}

void einsumsvd_query(const char* subscripts, int n_ops, const hpeps_tensor* ops, const hpeps_esvd_opts& o,
                     int64_t* rows, int64_t* cols, int64_t* rank) {
  const Network net = parse(subscripts, n_ops, ops, false);
  const int64_t k = sketch_width(o.rank, o.oversample, net.rows, net.cols);
  if (rows) *rows = net.rows;
  if (cols) *cols = net.cols;
  if (rank) *rank = std::min<int64_t>(o.rank, k);
}

}  // namespace hp
