// Internal declarations of the hpeps library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_complex.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/hpeps.h"

namespace hp {

// ---------------------------------------------------------------------------
// errors
struct Error {
  hpeps_status code;
  std::string msg;
};

#define HP_CHECK_HIP(expr)                                                        \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw ::hp::Error{HPEPS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define HP_REQUIRE(cond, code, msg)                       \
  do {                                                    \
    if (!(cond)) throw ::hp::Error{code, std::string(msg)}; \
  } while (0)

// ---------------------------------------------------------------------------
// index maps: a linear index i over a list of modes (last mode fastest) maps
// to the element offset sum_m idx_m * stride_m.
constexpr int kMaxModes = 12;
struct IndexMap {
  int n = 0;
  int64_t dim[kMaxModes];
  int64_t stride[kMaxModes];
  int64_t size() const {
    int64_t s = 1;
    for (int i = 0; i < n; ++i) s *= dim[i];
    return s;
  }
  IndexMap& add(int64_t d, int64_t s) {
    if (n >= kMaxModes) throw Error{HPEPS_ERR_UNSUPPORTED, "too many index modes in one operand"};
    dim[n] = d;
    stride[n] = s;
    ++n;
    return *this;
  }
  std::string key() const;
};

// Row-major strides of a shape.
std::vector<int64_t> rm_strides(const std::vector<int64_t>& shape);

// ---------------------------------------------------------------------------
// GEMM with gathered operands:
//   C[b][rC[m] + cC[n]] = scale * sum_k A[b][rA[m] + cA[k]] * B[b][rB[k] + cB[n]]
// F32 / BF16: inputs in that type, FP32 accumulation; output FP64 or the input type
enum class Prec { F64, C128, F32, BF16 };

struct GemmDesc {
  IndexMap Am, Ak, Bk, Bn, Cm, Cn;  // M/K/N index maps of each operand
  int64_t M = 0, N = 0, K = 0;
};

struct GemmCall {
  const void* A = nullptr;
  const void* B = nullptr;
  void* C = nullptr;
  int64_t sA = 0, sB = 0, sC = 0;  // batch strides (elements)
  int batch = 1;
  bool conjA = false, conjB = false, conjC = false;
  double alpha = 1.0;
  const double* scale = nullptr;   // per batch multiplier (device) or null
  const double* nscale = nullptr;  // per (batch, n) multiplier (device) or null
  int64_t nscale_ld = 0;
  bool accumulate = false;         // C += result
  const int* copy_if_zero = nullptr; // per batch flag: when 0, C := A (no product)
  const int* skip_if_zero = nullptr; // per batch flag: when 0, the instance is skipped (C untouched)
  // storage types (F32 / BF16 compute only): inputs float / bf16; output that
  // type, or double when out_f64
  bool out_f64 = true;
  // per-instance element counts of A, B, C: every gathered offset is checked
  // against them on the host before the launch (0 = the operand is not checked)
  int64_t nA = 0, nB = 0, nC = 0;
};

// Launch variant of the GEMM kernel: tile shape index, K-step multiple
// (K-step = 16 ks) and split-K count (0 = chosen by the size heuristic).
struct GemmVariant {
  int cfg = -1;
  int ks = 0;
  int split = 0;
};

class Ctx;
class Tape;
void gemm(Ctx& ctx, Prec prec, const GemmDesc& d, const GemmCall& c);
// JSON text of the tuned variants of a context / merge such a text into it
std::string autotune_export(const Ctx& ctx);
void autotune_import(Ctx& ctx, const std::string& json);

// ---------------------------------------------------------------------------
// small dense linear algebra kernels (launchers)
// Gram: G[b] = Y[b]^H Y[b] (Y: n x k row-major, batch stride n*k); G k x k.
// With `active`, instances whose flag is 0 are skipped (G[b] left as it was).
void gram(Ctx& ctx, bool cplx, const void* Y, int64_t n, int64_t k, int batch, double* G,
          const int* active);
// Per-instance flag bits of the orthogonalization (set by the factor step,
// read by the later passes, the Householder fallback and the diagnostics).
constexpr int FLAG_THIRD_PASS = 2;   // ill-conditioned or rank-deficient: third pass / fallback
constexpr int FLAG_NUMERIC = 4;      // non-finite values met
constexpr int FLAG_HOUSEHOLDER = 8;  // the Householder fallback replaced the factor
constexpr int FLAG_RANK_DEFICIENT = 16;  // pass 2's unshifted Cholesky broke down or spans 1e7 (kappa above ~1e13)
// CholeskyQR step on G (k x k, Hermitian): writes Rinv (k x k upper).  pass 1
// may shift; flags[b] bit 1 is set when a third pass is needed, bit 2 on
// non-finite values.  pass 3 is skipped (Rinv = I) unless bit 1 is set.
// Racc (optional): pass 1 writes R, later passes Racc <- R Racc; with r_only
// every pass writes its own R (the identity where pass 3 is skipped).
void chol_inv(Ctx& ctx, bool cplx, const double* G, int64_t n_rows, int64_t k, int batch,
              int pass, double* Rinv, double* Racc, int* flags, bool r_only = false);
// One-sided Jacobi SVD of K = Racc^H (k x k) per batch: writes Z (k x k,
// left singular vectors of K in columns, sorted by descending sigma), sigma
// (k), inv_sigma (k), inv_sigma1 (1); log_scale (optional) += log sigma_1;
// stats[b] = sweeps used (negative if the cap was hit).
void jacobi_svd(Ctx& ctx, bool cplx, const double* Racc, int64_t k, int batch, int max_sweeps,
                double* Z, double* sigma, double* inv_sigma, double* inv_sigma1,
                double* log_scale, int* stats);
// Sketch generator (see hpeps.h); writes n*k values per batch instance,
// instance b uses stream_id + b.  out is double or float (f32).
void sketch(Ctx& ctx, void* out, bool f32, int64_t n, int64_t k, int batch, uint64_t seed,
            uint64_t stream_id, bool cplx_out = false);
// Elementwise conversion and scaling helpers.
void convert_f64_to_f32(Ctx& ctx, const double* in, float* out, int64_t n);
// round to nearest even bfloat16 (out: n 16-bit values)
void convert_f64_to_bf16(Ctx& ctx, const double* in, void* out, int64_t n);
void fill_zero(Ctx& ctx, void* p, int64_t bytes);
// p[0..n) = v (complex: real part v, imaginary part 0), by a kernel (no memset
// nodes, so the call can sit in a captured graph)
void fill_value(Ctx& ctx, double* p, int64_t n, double v, bool cplx);
// p[b] = I (n x n, row-major) for b < batch, by a kernel
void fill_identity(Ctx& ctx, double* p, int64_t n, int batch, bool cplx);
// Canonical phase of singular pairs: U (row-major rows x mp per instance) is
// the left factor P Z; column i of Z (k x k) is rotated so that the
// projection of U[:, i] on a fixed counter-generated vector becomes real
// positive.
void gauge_fix(Ctx& ctx, bool cplx, const double* U, int64_t rows, int64_t mp, double* Z, int64_t k,
               int batch);
// dst[0..1] = src as a complex number (imaginary part 0 for real src)
void copy_scalar(Ctx& ctx, const double* src, bool cplx, double* dst);
// Frobenius norm of x (n doubles, or n complex if cplx) per batch (batch
// stride n elements); x is divided by the norm and log_scale[b] += log(norm).
void normalize(Ctx& ctx, bool cplx, void* x, int64_t n, int batch, double* log_scale);
// x[b][0..nd) *= s[b] (nd doubles per instance)
void scale_by(Ctx& ctx, double* x, int64_t nd, const double* s, int batch);
// sq[i] = sqrt(s[i]), isq[i] = 1 / sq[i] (0 where s[i] = 0)
void sqrt_pair(Ctx& ctx, const double* s, int64_t n, double* sq, double* isq);
// hooks of the reverse-mode tape (no-ops unless a tape records)
void tape_gemm(Ctx& ctx, Prec prec, const GemmDesc& d, const GemmCall& c);
void tape_scale(Ctx& ctx, bool cplx, double* x, int64_t n, const double* s, int batch);
void tape_copy(Ctx& ctx, bool cplx, void* dst, const void* src, int64_t n);
bool tape_keeps_workspace(const Ctx& ctx);
// diag(out)[..] helpers for tests of the gemm itself are not exported.
void copy_sigma(Ctx& ctx, const double* sigma_k, int64_t k, int64_t mp, int batch, double* out);
void stats_reduce(Ctx& ctx, const int* flags, const int* sweeps, int batch, int* acc);
// Householder QR (tall-skinny, one reduction level) of the row-major n x k
// panels Y (batch stride n k, unchanged) of the instances whose flag has a
// bit of `mask` (all instances when flags is null): the orthonormal Q to P
// (row-major n x k) and / or R to R (row-major k x k, zero below the
// diagonal), each when non-null; sets FLAG_HOUSEHOLDER on those instances.
// Other instances' P and R are left untouched.  k <= 128.
void householder_qr(Ctx& ctx, bool cplx, const double* Y, int64_t n, int64_t k, int batch, int* flags, int mask,
                    double* P, double* R);
int householder_blocks(int64_t n, int64_t k);
// Resolves the device address of the allocation-free gate update's static
// scratch on `device` (current), once per device; called at context creation.
void gate_scratch_init(int device);
// einsumsvd adjoint helpers (k x k / panel elementwise work, one workgroup per instance)
void svd_bwd_core(Ctx& ctx, bool cplx, const double* ZZ, const double* VV, const double* s,
                  const double* sbar, int64_t k, int batch, double eps, double* G1H);
void copyltu_neg(Ctx& ctx, bool cplx, double* M, int64_t k, int batch);
void axpy(Ctx& ctx, double* y, const double* x, double alpha, int64_t n);
void axpy_colscale(Ctx& ctx, bool cplx, double* Y, const double* X, const double* d, int64_t rows,
                   int64_t k, int batch);
// Vbar[c, i] = conj(dR[i, c]) s_i rscale (s, rscale nullable = 1), zero for i >= mp
void vbar_from_dr(Ctx& ctx, bool cplx, const double* dR, const double* s, const double* rscale,
                  int64_t cols, int64_t mp, int64_t k, int batch, double* Vbar);
// sbar_i = dsigma_i + (right ? rscale Re sum_c dR[i, c] V[c, i] : 0), zero for i >= mp
void sigma_bar(Ctx& ctx, bool cplx, const double* dsigma, const double* dR, const double* V,
               const double* rscale, int64_t cols, int64_t mp, int64_t k, int batch, bool right,
               double* sbar);
// cotangent of U through the canonical phase choice (complex; see the kernel)
void gauge_backward(Ctx& ctx, double* dU, const double* U, const double* dR, const double* V,
                    const double* s, const double* rscale, int64_t rows, int64_t cols, int64_t mp,
                    int64_t k, int batch);
// dst[b] (row-major rows.size() x cols.size()) = src[b * sSrc + rows(r) + cols(c)]
void gather2d(Ctx& ctx, bool cplx, const void* src, int64_t sSrc, const IndexMap& rows,
              const IndexMap& cols, void* dst, int batch);

// ---------------------------------------------------------------------------
// context: stream, workspace arena, cached index tables, diagnostics
class Ctx {
 public:
  explicit Ctx(int device);
  ~Ctx();
  int device;
  hipStream_t stream = nullptr;
  std::string last_error;
  int64_t ws_limit = 0;
  // byte budget of one intermediate of an energy strip column (larger ones are
  // split along the bottom-environment leg)
  int64_t strip_chunk_bytes = (int64_t)1 << 30;
  // reverse mode: checkpoint each zip-up row of a boundary pass (store its
  // input boundary, recompute the row in the reverse walk) instead of
  // recording every intermediate of the row
  bool checkpoint_rows = true;
  // high-water mark of the workspace arena (bytes in use), since creation or
  // the last hpeps_workspace_peak reset
  int64_t ws_peak = 0;

  // device index table for an IndexMap (int32 offsets), cached
  const int* table(const IndexMap& m);

  // workspace: a bump allocator that is reset at the start of every ABI call
  void ws_reset();
  void* ws_alloc(int64_t bytes);
  template <class T>
  T* ws(int64_t n) { return reinterpret_cast<T*>(ws_alloc(n * (int64_t)sizeof(T))); }
  // reserve at least bytes for the coming call (grows the arena; syncs)
  void ws_reserve(int64_t bytes);
  // scoped reuse: the position can be saved and restored (all work is on one
  // stream, so later kernels run after the earlier users of the memory)
  int ws_chunk() const { return cur_; }
  int64_t ws_offset() const { return ws_off_; }
  void ws_restore(int chunk, int64_t off) {
    cur_ = chunk;
    ws_off_ = off;
  }

  // diagnostics accumulator on the device: [extra passes, max sweeps,
  // numeric errors, not converged]
  int* stats_dev = nullptr;
  int64_t last_rank = 0, last_k = 0;

  // Live kernel timing with HIP events on the context stream.  While
  // profiling is on, launches whose class name contains `prof_filter` (all
  // when empty) are bracketed by two events; prof_read aggregates per class.
  bool prof_on = false;
  bool prof_shapes = false;  // GEMM class names carry the product's M, N, K and batch
  std::string prof_filter;
  int prof_begin(const std::string& cls);            // -1 when not recorded
  void prof_end(int rec, double flops, double bytes);
  struct ProfAgg {
    std::string name;
    int64_t launches = 0;
    double ms = 0, flops = 0, bytes = 0;
  };
  std::vector<ProfAgg> prof_read();                  // synchronises, clears

  // GEMM variant selection: a forced variant (cfg >= 0; kernel tests), the
  // tuned cache keyed by shape / layout / precision, and the autotune switch
  // (when on, the first product of a new key times every variant and keeps
  // the fastest; that call synchronises the stream)
  GemmVariant gemm_force;
  bool smallk = true;  // skinny real products (K <= 16, or M <= 8 with N >= 256) on their own kernels
  bool autotune = false;
  std::map<std::string, GemmVariant> gemm_tuned;

  // reverse-mode recording (set only inside a backward ABI call): while a
  // tape records, products, in-place rescalings, exact carries, einsumsvds
  // and copies are logged, and workspace scopes do not release memory
  Tape* tape = nullptr;
  // contraction order of the zip-up operator's middle stages: 0 chosen by
  // the cost model, 1 classic, 2 boundary first (kernel tests)
  int zip_order_force = 0;

 private:
  struct ProfRec {
    int cls;
    hipEvent_t a, b;
    double flops, bytes;
  };
  std::vector<ProfRec> prof_recs_;
  std::vector<hipEvent_t> ev_pool_;
  size_t ev_used_ = 0;
  std::vector<std::string> prof_names_;
  std::map<std::string, int> prof_ids_;
  hipEvent_t next_event();

 public:

 private:
  std::map<std::string, int*> tables_;
  struct Chunk {
    char* base = nullptr;
    int64_t cap = 0;
  };
  std::vector<Chunk> chunks_;
  int cur_ = 0;
  int64_t ws_off_ = 0;
};

// Launch-size helper
inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace hp

// the opaque handle of the ABI
struct hpeps_ctx {
  hp::Ctx* impl;
};
