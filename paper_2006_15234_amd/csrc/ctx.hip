// Context: stream, workspace arena and the cache of gather tables.
#include <algorithm>
#include <sstream>

#include "internal.h"

namespace hp {

std::string IndexMap::key() const {
  std::ostringstream os;
  for (int i = 0; i < n; ++i) os << dim[i] << ':' << stride[i] << ',';
  return os.str();
}

std::vector<int64_t> rm_strides(const std::vector<int64_t>& shape) {
  std::vector<int64_t> s(shape.size(), 1);
  for (int i = (int)shape.size() - 2; i >= 0; --i) s[i] = s[i + 1] * shape[i + 1];
  return s;
}

namespace {
struct TableArgs {
  int n;
  long long div[kMaxModes];
  long long dim[kMaxModes];
  long long stride[kMaxModes];
};

// out[i] = sum over modes of ((i / div) % dim) * stride
__global__ void fill_table_kernel(int* out, long long total, TableArgs a) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    long long off = 0;
    for (int m = 0; m < a.n; ++m) off += ((i / a.div[m]) % a.dim[m]) * a.stride[m];
    out[i] = (int)off;
  }
}
}  // namespace

Ctx::Ctx(int dev) : device(dev) {
  HP_CHECK_HIP(hipSetDevice(dev));
  gate_scratch_init(dev);
  HP_CHECK_HIP(hipMalloc(&stats_dev, 8 * sizeof(int)));
  HP_CHECK_HIP(hipMemset(stats_dev, 0, 8 * sizeof(int)));
}

hipEvent_t Ctx::next_event() {
  if (ev_used_ == ev_pool_.size()) {
    hipEvent_t e;
    HP_CHECK_HIP(hipEventCreate(&e));
    ev_pool_.push_back(e);
  }
  return ev_pool_[ev_used_++];
}

int Ctx::prof_begin(const std::string& cls) {
  if (!prof_on) return -1;
  if (!prof_filter.empty() && cls.find(prof_filter) == std::string::npos) return -1;
  auto it = prof_ids_.find(cls);
  int id;
  if (it == prof_ids_.end()) {
    id = (int)prof_names_.size();
    prof_names_.push_back(cls);
    prof_ids_[cls] = id;
  } else {
    id = it->second;
  }
  ProfRec r{id, next_event(), next_event(), 0, 0};
  HP_CHECK_HIP(hipEventRecord(r.a, stream));
  prof_recs_.push_back(r);
  return (int)prof_recs_.size() - 1;
}

void Ctx::prof_end(int rec, double flops, double bytes) {
  if (rec < 0) return;
  ProfRec& r = prof_recs_[rec];
  HP_CHECK_HIP(hipEventRecord(r.b, stream));
  r.flops = flops;
  r.bytes = bytes;
}

std::vector<Ctx::ProfAgg> Ctx::prof_read() {
  HP_CHECK_HIP(hipStreamSynchronize(stream));
  std::vector<ProfAgg> agg(prof_names_.size());
  for (size_t i = 0; i < agg.size(); ++i) agg[i].name = prof_names_[i];
  for (auto& r : prof_recs_) {
    float ms = 0;
    HP_CHECK_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    ProfAgg& a = agg[r.cls];
    a.launches += 1;
    a.ms += ms;
    a.flops += r.flops;
    a.bytes += r.bytes;
  }
  prof_recs_.clear();
  ev_used_ = 0;
  return agg;
}

Ctx::~Ctx() {
  for (auto e : ev_pool_) (void)hipEventDestroy(e);
  (void)hipDeviceSynchronize();
  for (auto& kv : tables_) (void)hipFree(kv.second);
  for (auto& c : chunks_) (void)hipFree(c.base);
  if (stats_dev) (void)hipFree(stats_dev);
}

const int* Ctx::table(const IndexMap& m) {
  const std::string key = m.key();
  auto it = tables_.find(key);
  if (it != tables_.end()) return it->second;
  const int64_t total = std::max<int64_t>(m.size(), 1);
  int64_t maxoff = 0;
  for (int i = 0; i < m.n; ++i) maxoff += (m.dim[i] - 1) * m.stride[i];
  HP_REQUIRE(maxoff < (1LL << 31), HPEPS_ERR_UNSUPPORTED, "tensor too large for int32 offsets");
  TableArgs a{};
  a.n = m.n;
  long long div = 1;
  for (int i = m.n - 1; i >= 0; --i) {
    a.div[i] = div;
    a.dim[i] = m.dim[i];
    a.stride[i] = m.stride[i];
    div *= m.dim[i];
  }
  int* d = nullptr;
  HP_CHECK_HIP(hipMalloc(&d, total * sizeof(int)));
  if (m.n == 0) {
    HP_CHECK_HIP(hipMemsetAsync(d, 0, sizeof(int), stream));
  } else {
    const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
    fill_table_kernel<<<blocks, 256, 0, stream>>>(d, total, a);
    HP_CHECK_HIP(hipGetLastError());
  }
  tables_[key] = d;
  return d;
}

// The arena is a list of chunks.  A call that outgrows the current chunks
// gets a new chunk (hipMalloc does not wait for queued work, so buffers that
// earlier kernels of the call still use stay valid); at the next reset the
// chunks are merged into one of the combined size.
void Ctx::ws_reserve(int64_t bytes) {
  bytes = (bytes + 4095) / 4096 * 4096;
  int64_t have = 0;
  for (auto& c : chunks_) have += c.cap;
  if (bytes <= have && chunks_.size() <= 1) return;
  HP_REQUIRE(ws_limit <= 0 || bytes <= ws_limit, HPEPS_ERR_ALLOC,
             "workspace of " + std::to_string(bytes) + " bytes exceeds the limit");
  HP_CHECK_HIP(hipStreamSynchronize(stream));
  for (auto& c : chunks_) HP_CHECK_HIP(hipFree(c.base));
  chunks_.clear();
  Chunk c;
  if (hipMalloc(&c.base, std::max(bytes, have)) != hipSuccess)
    throw Error{HPEPS_ERR_ALLOC, "workspace allocation of " + std::to_string(bytes) + " bytes failed"};
  c.cap = std::max(bytes, have);
  chunks_.push_back(c);
  cur_ = 0;
  ws_off_ = 0;
}

void Ctx::ws_reset() {
  if (chunks_.size() > 1) {
    int64_t total = 0;
    for (auto& c : chunks_) total += c.cap;
    ws_reserve(total);
  }
  cur_ = 0;
  ws_off_ = 0;
}

void* Ctx::ws_alloc(int64_t bytes) {
  bytes = (bytes + 255) / 256 * 256;
  while (cur_ < (int)chunks_.size() && ws_off_ + bytes > chunks_[cur_].cap) {
    ++cur_;
    ws_off_ = 0;
  }
  if (cur_ >= (int)chunks_.size()) {
    int64_t used = 0;
    for (auto& c : chunks_) used += c.cap;
    HP_REQUIRE(ws_limit <= 0 || used + bytes <= ws_limit, HPEPS_ERR_ALLOC,
               "workspace exceeds the limit");
    Chunk c;
    c.cap = std::max<int64_t>(bytes, 64 << 20);
    if (hipMalloc(&c.base, c.cap) != hipSuccess)
      throw Error{HPEPS_ERR_ALLOC, "workspace allocation of " + std::to_string(c.cap) + " bytes failed"};
    chunks_.push_back(c);
    cur_ = (int)chunks_.size() - 1;
    ws_off_ = 0;
  }
  void* p = chunks_[cur_].base + ws_off_;
  ws_off_ += bytes;
  int64_t in_use = ws_off_;
  for (int i = 0; i < cur_; ++i) in_use += chunks_[i].cap;
  ws_peak = std::max(ws_peak, in_use);
  return p;
}

}  // namespace hp
