// Serving runtime: a request loop that colours independent graphs with
// JP-ADG as they arrive (adg_server_* in include/adg.h).
//
// Continuous batching.  Requests wait in arrival order.  Whenever a worker
// is idle it admits the next job that fits into the device arena:
//   - a large request (nnz > small_nnz) alone: its CSR, colours and a
//     color_graph workspace;
//   - otherwise a group of consecutive small requests, packed into one
//     concatenated CSR and coloured by one color_graph_batched launch.
// Each worker owns a HIP stream, so jobs admitted while others run overlap
// on the device; arena space and workers come free as jobs complete.  A
// request that does not fit may be overtaken by later ones at most
// max_bypass times; after that nothing new is admitted until it fits.
// Every request's result equals what a standalone color_graph call returns
// for its graph (the batched path colours every graph exactly as alone).
//
// The arena is one device buffer owned by the caller; the server carves
// per-job regions out of it (first fit, coalescing free list) and never
// allocates device memory itself.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/adg.h"
#include "adg_host.h"

namespace adg {
namespace serve {

constexpr size_t ALIGN = 256;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) with coalescing.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) {
    if (size) free_[0] = size;
  }
  // offset of a block of `bytes`, or SIZE_MAX
  size_t alloc(size_t bytes) {
    bytes = align_up(std::max<size_t>(bytes, 1), ALIGN);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > bytes) free_[off + bytes] = len - bytes;
      used_ += bytes;
      return off;
    }
    return SIZE_MAX;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(std::max<size_t>(bytes, 1), ALIGN);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  bool fits(size_t bytes) const {
    bytes = align_up(std::max<size_t>(bytes, 1), ALIGN);
    for (const auto& kv : free_)
      if (kv.second >= bytes) return true;
    return false;
  }
  size_t size() const { return size_; }

 private:
  size_t size_;
  size_t used_ = 0;
  std::map<size_t, size_t> free_;
};

struct Request {
  uint64_t tag;
  int64_t n, nnz;
  const int64_t* rp;   // host
  const int32_t* col;  // host
  int32_t* color;      // host output
  double t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
  int bypassed = 0;
  int status = ADG_OK;
  int num_colors = 0, num_rounds = 0, group = 1;
};

// Device bytes of one job.  Both layouts place each array at a 256-byte
// aligned offset inside the job's region.
size_t large_bytes(int64_t n, int64_t nnz) {
  size_t b = 0;
  b += align_up(adg_workspace_bytes(n, nnz), ALIGN);
  b += align_up(8 * (size_t)(n + 1), ALIGN);
  b += align_up(4 * (size_t)std::max<int64_t>(nnz, 1), ALIGN);
  b += align_up(4 * (size_t)std::max<int64_t>(n, 1), ALIGN);
  b += ALIGN;  // num_colors, num_rounds
  return b;
}
size_t group_bytes(int64_t G, int64_t tn, int64_t tnnz) {
  size_t b = 0;
  b += align_up(adg_batched_workspace_bytes((int32_t)G, tn, tnnz), ALIGN);
  b += align_up(8 * (size_t)(G + 1), ALIGN);
  b += align_up(8 * (size_t)(tn + 1), ALIGN);
  b += align_up(4 * (size_t)std::max<int64_t>(tnnz, 1), ALIGN);
  b += align_up(4 * (size_t)std::max<int64_t>(tn, 1), ALIGN);
  b += 2 * align_up(4 * (size_t)G, ALIGN);
  return b;
}

struct Job {
  std::vector<Request*> reqs;
  bool grouped = false;
  size_t off = 0, bytes = 0;
  int64_t sum_active = 0, cut_edges = 0;   // ADG counters of the job
};

}  // namespace serve
}  // namespace adg

struct adg_server {
  adg_server_config_t cfg;
  char* arena_base;
  adg::serve::Arena arena;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<adg::serve::Request*> pending;
  std::deque<adg::serve::Request*> done;
  int64_t in_flight = 0;   // submitted and not yet polled out of `done`
  int64_t running = 0;     // admitted jobs not finished
  adg_server_counters_t ctr{};   // totals over finished jobs
  bool stop = false;
  std::vector<std::thread> workers;

  adg_server(const adg_server_config_t& c, void* base, size_t bytes)
      : cfg(c), arena_base((char*)base), arena(bytes) {}
};

namespace adg {
namespace serve {

// Next job to run, or false.  Called with the server's mutex held.
bool form_job(adg_server* S, Job& job) {
  auto& q = S->pending;
  for (size_t i = 0; i < q.size(); ++i) {
    Request* r = q[i];
    const bool small = r->nnz <= S->cfg.small_nnz;
    if (!small) {
      const size_t b = large_bytes(r->n, r->nnz);
      if (!S->arena.fits(b)) {
        if (i == 0 && ++r->bypassed > S->cfg.max_bypass) return false;
        continue;
      }
      job.reqs = {r};
      job.grouped = false;
      job.bytes = b;
      job.off = S->arena.alloc(b);
      q.erase(q.begin() + (long)i);
      return true;
    }
    // a group of small requests, in arrival order, starting here
    std::vector<size_t> idx;
    int64_t tn = 0, tnnz = 0;
    size_t b = 0;
    for (size_t j = i; j < q.size() && (int)idx.size() < S->cfg.max_group; ++j) {
      Request* s = q[j];
      if (s->nnz > S->cfg.small_nnz) continue;
      const size_t nb = group_bytes((int64_t)idx.size() + 1, tn + s->n, tnnz + s->nnz);
      if (!S->arena.fits(nb)) break;
      idx.push_back(j);
      tn += s->n;
      tnnz += s->nnz;
      b = nb;
    }
    if (idx.empty()) {
      if (i == 0 && ++r->bypassed > S->cfg.max_bypass) return false;
      continue;
    }
    job.reqs.clear();
    for (size_t j : idx) job.reqs.push_back(q[j]);
    for (size_t k = idx.size(); k-- > 0;) q.erase(q.begin() + (long)idx[k]);
    job.grouped = true;
    job.bytes = b;
    job.off = S->arena.alloc(b);
    return true;
  }
  return false;
}

int run_large(adg_server* S, Job& job, hipStream_t s) {
  Request* r = job.reqs[0];
  char* base = S->arena_base + job.off;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* p = base + o;
    o += align_up(std::max<size_t>(bytes, 1), ALIGN);
    return p;
  };
  const size_t wsb = adg_workspace_bytes(r->n, r->nnz);
  void* ws = take(wsb);
  int64_t* rp = (int64_t*)take(8 * (size_t)(r->n + 1));
  int32_t* col = (int32_t*)take(4 * (size_t)std::max<int64_t>(r->nnz, 1));
  int32_t* color = (int32_t*)take(4 * (size_t)std::max<int64_t>(r->n, 1));
  int32_t* scal = (int32_t*)take(8);
  HIPCHK(hipMemcpyAsync(rp, r->rp, 8 * (size_t)(r->n + 1), hipMemcpyHostToDevice, s));
  if (r->nnz) HIPCHK(hipMemcpyAsync(col, r->col, 4 * (size_t)r->nnz, hipMemcpyHostToDevice, s));
  adg_csr_t g{r->n, r->nnz, rp, col};
  int rc = color_graph(&g, S->cfg.eps_num, S->cfg.eps_den, S->cfg.seed, color, nullptr, scal, scal + 1, ws, wsb, s);
  if (rc) return rc;
  if (r->n) HIPCHK(hipMemcpyAsync(r->color, color, 4 * (size_t)r->n, hipMemcpyDeviceToHost, s));
  int32_t h[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(h, scal, 8, hipMemcpyDeviceToHost, s));
  adg_stats_t st{};
  rc = adg_get_stats(ws, wsb, &st, s);  // synchronises s
  if (rc) return rc;
  if (st.error) return (int)st.error;
  r->num_colors = h[0];
  r->num_rounds = h[1];
  job.sum_active = st.sum_active;
  job.cut_edges = st.cut_edges;
  return ADG_OK;
}

int run_group(adg_server* S, Job& job, hipStream_t s, std::vector<int64_t>& stage) {
  const int64_t G = (int64_t)job.reqs.size();
  int64_t tn = 0, tnnz = 0;
  for (Request* r : job.reqs) {
    tn += r->n;
    tnnz += r->nnz;
  }
  char* base = S->arena_base + job.off;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* p = base + o;
    o += align_up(std::max<size_t>(bytes, 1), ALIGN);
    return p;
  };
  const size_t wsb = adg_batched_workspace_bytes((int32_t)G, tn, tnnz);
  void* ws = take(wsb);
  int64_t* vo = (int64_t*)take(8 * (size_t)(G + 1));
  int64_t* rp = (int64_t*)take(8 * (size_t)(tn + 1));
  int32_t* col = (int32_t*)take(4 * (size_t)std::max<int64_t>(tnnz, 1));
  int32_t* color = (int32_t*)take(4 * (size_t)std::max<int64_t>(tn, 1));
  int32_t* nc = (int32_t*)take(4 * (size_t)G);
  int32_t* nr = (int32_t*)take(4 * (size_t)G);
  // host staging: [vtx_off | absolute row_ptr]
  stage.resize((size_t)(G + 1) + (size_t)(tn + 1));
  int64_t* hvo = stage.data();
  int64_t* hrp = hvo + (G + 1);
  int64_t v = 0, e = 0;
  for (int64_t g = 0; g < G; ++g) {
    const Request* r = job.reqs[g];
    hvo[g] = v;
    for (int64_t i = 0; i < r->n; ++i) hrp[v + i] = e + r->rp[i];
    if (r->nnz) HIPCHK(hipMemcpyAsync(col + e, r->col, 4 * (size_t)r->nnz, hipMemcpyHostToDevice, s));
    v += r->n;
    e += r->nnz;
  }
  hvo[G] = v;
  hrp[tn] = e;
  HIPCHK(hipMemcpyAsync(vo, hvo, 8 * (size_t)(G + 1), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(rp, hrp, 8 * (size_t)(tn + 1), hipMemcpyHostToDevice, s));
  adg_batch_t b{(int32_t)G, tn, tnnz, vo, rp, col};
  int rc = color_graph_batched(&b, S->cfg.eps_num, S->cfg.eps_den, S->cfg.seed, color, nullptr, nc, nr, nullptr,
                               ws, wsb, s);
  if (rc) return rc;
  v = 0;
  for (Request* r : job.reqs) {
    if (r->n) HIPCHK(hipMemcpyAsync(r->color, color + v, 4 * (size_t)r->n, hipMemcpyDeviceToHost, s));
    v += r->n;
  }
  std::vector<int32_t> h(2 * (size_t)G);
  HIPCHK(hipMemcpyAsync(h.data(), nc, 4 * (size_t)G, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(h.data() + G, nr, 4 * (size_t)G, hipMemcpyDeviceToHost, s));
  adg_stats_t st{};
  rc = adg_batched_get_stats(ws, wsb, &st, s);  // synchronises s
  if (rc) return rc;
  if (st.error) return (int)st.error;
  for (int64_t g = 0; g < G; ++g) {
    job.reqs[g]->num_colors = h[g];
    job.reqs[g]->num_rounds = h[G + g];
    job.reqs[g]->group = (int)G;
  }
  job.sum_active = st.sum_active;
  job.cut_edges = st.cut_edges;
  return ADG_OK;
}

void worker(adg_server* S) {
  (void)hipSetDevice(S->device);
  hipStream_t s = nullptr;
  const bool have_stream = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
  std::vector<int64_t> stage;
  for (;;) {
    Job job;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (;;) {
        if (S->stop && S->pending.empty()) {
          lk.unlock();
          if (have_stream) (void)hipStreamDestroy(s);
          return;
        }
        if (form_job(S, job)) break;
        S->cv.wait(lk);
      }
      ++S->running;
      const double t = now_s();
      for (Request* r : job.reqs) r->t_admit = t;
    }
    const double t0 = now_s();
    for (Request* r : job.reqs) r->t_start = t0;
    int rc = have_stream ? (job.grouped ? run_group(S, job, s, stage) : run_large(S, job, s)) : ADG_ERR_HIP;
    if (rc && have_stream) (void)hipStreamSynchronize(s);   // nothing of the job may still run
    const double t1 = now_s();
    {
      std::lock_guard<std::mutex> g(S->mu);
      S->arena.release(job.off, job.bytes);
      if (!rc) {
        adg_server_counters_t& c = S->ctr;
        if (job.grouped) {
          c.grouped_jobs += 1;
          c.grouped_requests += (int64_t)job.reqs.size();
        } else {
          c.single_jobs += 1;
        }
        for (Request* r : job.reqs) {
          c.vertices += r->n;
          c.entries += r->nnz;
        }
        c.sum_active += job.sum_active;
        c.cut_edges += job.cut_edges;
      }
      for (Request* r : job.reqs) {
        r->t_done = t1;
        r->status = rc;
        S->done.push_back(r);
      }
      --S->running;
    }
    S->cv.notify_all();
  }
}

}  // namespace serve
}  // namespace adg

using namespace adg;
using namespace adg::serve;

extern "C" {

adg_server_config_t adg_server_default_config(void) {
  adg_server_config_t c;
  c.eps_num = 1;
  c.eps_den = 10;
  c.seed = 0;
  c.workers = 4;
  c.small_nnz = 1 << 20;
  c.max_group = 256;
  c.max_bypass = 64;
  return c;
}

size_t adg_server_footprint(const adg_server_config_t* cfg, int64_t n, int64_t nnz) {
  if (!cfg || n < 0 || nnz < 0 || n > 0x7ffffffeLL) return 0;
  return nnz <= cfg->small_nnz ? group_bytes(1, n, nnz) : large_bytes(n, nnz);
}

int adg_server_create(const adg_server_config_t* cfg, void* arena, size_t arena_bytes, adg_server_t** out) {
  if (!cfg || !out || !arena || ((uintptr_t)arena & (ALIGN - 1))) return ADG_ERR_ARG;
  if (cfg->eps_num < 0 || cfg->eps_den < 1 || cfg->workers < 1 || cfg->workers > 16 || cfg->small_nnz < 0 ||
      cfg->max_group < 1 || cfg->max_bypass < 0)
    return ADG_ERR_ARG;
  adg_server* S = new (std::nothrow) adg_server(*cfg, arena, arena_bytes);
  if (!S) return ADG_ERR_ARG;
  if (hipGetDevice(&S->device) != hipSuccess) {
    delete S;
    return ADG_ERR_HIP;
  }
  for (int i = 0; i < cfg->workers; ++i) S->workers.emplace_back(worker, S);
  *out = S;
  return ADG_OK;
}

int adg_server_submit(adg_server_t* S, int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                      int32_t* color_out, uint64_t tag) {
  if (!S || n < 0 || nnz < 0 || n > 0x7ffffffeLL || !row_ptr || (nnz > 0 && !col_idx) || (n > 0 && !color_out))
    return ADG_ERR_ARG;
  if (row_ptr[0] != 0 || row_ptr[n] != nnz) return ADG_ERR_ARG;
  const size_t need = adg_server_footprint(&S->cfg, n, nnz);
  if (need > S->arena.size()) return ADG_ERR_UNSUPPORTED;
  Request* r = new (std::nothrow) Request();
  if (!r) return ADG_ERR_ARG;
  r->tag = tag;
  r->n = n;
  r->nnz = nnz;
  r->rp = row_ptr;
  r->col = col_idx;
  r->color = color_out;
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stop) {
      delete r;
      return ADG_ERR_ARG;
    }
    S->pending.push_back(r);
    ++S->in_flight;
  }
  S->cv.notify_all();
  return ADG_OK;
}

int adg_server_poll(adg_server_t* S, adg_request_result_t* out, int32_t max_results, int32_t wait_ms,
                    int32_t* count_out) {
  if (!S || !count_out || max_results < 0 || (max_results > 0 && !out)) return ADG_ERR_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  if (S->done.empty() && wait_ms > 0)
    S->cv.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !S->done.empty(); });
  int32_t k = 0;
  while (k < max_results && !S->done.empty()) {
    Request* r = S->done.front();
    S->done.pop_front();
    adg_request_result_t& o = out[k++];
    o.tag = r->tag;
    o.status = r->status;
    o.num_colors = r->num_colors;
    o.num_rounds = r->num_rounds;
    o.group_size = r->group;
    o.n = r->n;
    o.nnz = r->nnz;
    o.t_submit = r->t_submit;
    o.t_admit = r->t_admit;
    o.t_start = r->t_start;
    o.t_done = r->t_done;
    --S->in_flight;
    delete r;
  }
  *count_out = k;
  return ADG_OK;
}

int64_t adg_server_in_flight(adg_server_t* S) {
  if (!S) return -1;
  std::lock_guard<std::mutex> g(S->mu);
  return S->in_flight;
}

double adg_server_clock(void) { return now_s(); }

int adg_server_get_counters(adg_server_t* S, adg_server_counters_t* out) {
  if (!S || !out) return ADG_ERR_ARG;
  std::lock_guard<std::mutex> g(S->mu);
  *out = S->ctr;
  return ADG_OK;
}

int adg_server_destroy(adg_server_t* S) {
  if (!S) return ADG_ERR_ARG;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  for (std::thread& t : S->workers) t.join();
  for (Request* r : S->done) delete r;
  delete S;
  return ADG_OK;
}

}  // extern "C"
