// Request-serving engine (rcm_server.h): a device arena with first-fit
// reservations, first-come-first-served admission by memory footprint,
// continuous batching of small requests into rcm_order_batched calls, and
// several executor threads with one HIP stream each.  Host code only: the
// orderings themselves are the library's entry points.

#include "rcm_server.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

constexpr uint64_t kAlign = 256;
constexpr int kMaxExecutors = 8;

inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Device bytes of one request ordered alone: rowptr, colidx, perm, iperm and
// the workspace, each region aligned.
uint64_t alone_bytes(int32_t n, int64_t nnz, const rcm_options* o) {
  if (n <= 0) return 0;
  return align_up(4ull * (static_cast<uint64_t>(n) + 1)) +
         align_up(4ull * static_cast<uint64_t>(nnz)) + 2 * align_up(4ull * n) +
         align_up(rcm_workspace_bytes(n, nnz, o));
}

// Device bytes of a batched call: concatenated rowptr (N + G entries),
// colidx, perm and the batched workspace.
uint64_t batch_bytes(int32_t G, int64_t N, int64_t NNZ, const rcm_options* o) {
  return align_up(4ull * static_cast<uint64_t>(N + G)) + align_up(4ull * static_cast<uint64_t>(NNZ)) +
         align_up(4ull * static_cast<uint64_t>(N)) +
         align_up(rcm_batched_workspace_bytes(G, N, NNZ, o));
}

// First-fit allocator over [0, size) with coalescing frees.
class Arena {
 public:
  explicit Arena(uint64_t size) { free_[0] = size; }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (const auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
  bool reserve(uint64_t bytes, uint64_t* off) {
    bytes = align_up(std::max<uint64_t>(bytes, kAlign));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const uint64_t rest = it->second - bytes;
      const uint64_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      sizes_[*off] = bytes;
      return true;
    }
    return false;
  }
  void release(uint64_t off) {
    auto s = sizes_.find(off);
    if (s == sizes_.end()) return;
    uint64_t bytes = s->second;
    sizes_.erase(s);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t used() const { return used_; }

 private:
  uint64_t used_ = 0;
  std::map<uint64_t, uint64_t> free_;
  std::map<uint64_t, uint64_t> sizes_;
};

struct Request {
  int64_t ticket = 0;
  int32_t n = 0;
  int64_t nnz = 0;
  const int32_t* rowptr = nullptr;
  const int32_t* colidx = nullptr;
  int32_t* perm_out = nullptr;
  uint64_t alone = 0;  // footprint when ordered alone
  bool done = false;
  rcm_request_result res{};
};

}  // namespace

struct rcm_server {
  rcm_server_config cfg{};
  std::string tuning_file;  // the server's own copy of order_options.tuning_file
  int device = 0;
  char* arena_base = nullptr;
  std::unique_ptr<Arena> arena;
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable work_cv;  // executors: queue or memory changed
  std::condition_variable done_cv;  // waiters: a request completed
  std::deque<Request*> queue;
  std::unordered_map<int64_t, std::unique_ptr<Request>> live;
  int64_t next_ticket = 1;
  bool stopping = false;
  rcm_server_counters counters{};
  std::vector<std::thread> executors;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // The requests at the head of the queue that the next call orders, and
  // the bytes it reserves.  Caller holds mu; the head's alone footprint fits.
  std::vector<Request*> take_batch(uint64_t free_bytes, uint64_t* bytes) {
    std::vector<Request*> b{queue.front()};
    uint64_t best = queue.front()->alone;
    int64_t N = queue.front()->n, NNZ = queue.front()->nnz;
    uint64_t max_alone = queue.front()->alone;
    if (queue.front()->nnz <= cfg.batch_nnz_limit) {
      for (size_t i = 1; i < queue.size() && static_cast<int>(b.size()) < cfg.max_batch; ++i) {
        Request* r = queue[i];
        if (r->nnz > cfg.batch_nnz_limit) break;
        const int64_t N2 = N + r->n, NNZ2 = NNZ + r->nnz;
        if (N2 >= (1ll << 31) - 1 - static_cast<int64_t>(b.size()) - 1 ||
            NNZ2 >= (1ll << 31) - 1)
          break;
        const uint64_t need =
            std::max({batch_bytes(static_cast<int32_t>(b.size()) + 1, N2, NNZ2,
                                  &cfg.order_options),
                      max_alone, r->alone});
        if (need > free_bytes) break;
        b.push_back(r);
        N = N2;
        NNZ = NNZ2;
        max_alone = std::max(max_alone, r->alone);
        best = need;
      }
    }
    queue.erase(queue.begin(), queue.begin() + static_cast<long>(b.size()));
    *bytes = best;
    return b;
  }

  void finish(std::vector<Request*>& b, uint64_t off) {
    std::lock_guard<std::mutex> lk(mu);
    arena->release(off);
    counters.bytes_in_flight = arena->used();
    const double t = now();
    for (Request* r : b) {
      r->res.t_done = t;
      r->done = true;
      counters.completed += 1;
      if (r->res.status != RCM_OK) counters.failed += 1;
    }
    work_cv.notify_all();
    done_cv.notify_all();
  }

  // Order one request alone in the device memory at base.
  rcm_status run_alone(Request* r, char* base, hipStream_t s) {
    const int32_t n = r->n;
    const int64_t nnz = r->nnz;
    char* p = base;
    auto take = [&](uint64_t bytes) {
      char* at = p;
      p += align_up(bytes);
      return at;
    };
    int32_t* rp = reinterpret_cast<int32_t*>(take(4ull * (n + 1)));
    int32_t* ci = reinterpret_cast<int32_t*>(take(4ull * nnz));
    int32_t* perm = reinterpret_cast<int32_t*>(take(4ull * n));
    int32_t* iperm = reinterpret_cast<int32_t*>(take(4ull * n));
    const uint64_t wsb = rcm_workspace_bytes(n, nnz, &cfg.order_options);
    void* ws = take(wsb);
    if (hipMemcpyAsync(rp, r->rowptr, 4ull * (n + 1), hipMemcpyHostToDevice, s) != hipSuccess)
      return RCM_ERR_HIP;
    if (nnz > 0 &&
        hipMemcpyAsync(ci, r->colidx, 4ull * nnz, hipMemcpyHostToDevice, s) != hipSuccess)
      return RCM_ERR_HIP;
    rcm_status st = rcm_order_ex(n, rp, ci, perm, iperm, &r->res.stats, &cfg.order_options, ws,
                                 wsb, s);
    if (st != RCM_OK) return st;
    if (hipMemcpyAsync(r->perm_out, perm, 4ull * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return RCM_ERR_HIP;
    return RCM_OK;
  }

  // Order b (more than one request) with one batched call; on failure
  // re-run every request alone so that only the offending ones fail.
  void run_batch(std::vector<Request*>& b, char* base, hipStream_t s) {
    const int32_t G = static_cast<int32_t>(b.size());
    std::vector<int64_t> vo(G + 1, 0), no(G + 1, 0);
    for (int32_t g = 0; g < G; ++g) {
      vo[g + 1] = vo[g] + b[g]->n;
      no[g + 1] = no[g] + b[g]->nnz;
    }
    const int64_t N = vo[G], NNZ = no[G];
    char* p = base;
    auto take = [&](uint64_t bytes) {
      char* at = p;
      p += align_up(bytes);
      return at;
    };
    int32_t* rp = reinterpret_cast<int32_t*>(take(4ull * (N + G)));
    int32_t* ci = reinterpret_cast<int32_t*>(take(4ull * NNZ));
    int32_t* perm = reinterpret_cast<int32_t*>(take(4ull * N));
    const uint64_t wsb = rcm_batched_workspace_bytes(G, N, NNZ, &cfg.order_options);
    void* ws = take(wsb);
    rcm_status st = RCM_OK;
    for (int32_t g = 0; g < G && st == RCM_OK; ++g) {
      if (hipMemcpyAsync(rp + vo[g] + g, b[g]->rowptr, 4ull * (b[g]->n + 1),
                         hipMemcpyHostToDevice, s) != hipSuccess)
        st = RCM_ERR_HIP;
      if (st == RCM_OK && b[g]->nnz > 0 &&
          hipMemcpyAsync(ci + no[g], b[g]->colidx, 4ull * b[g]->nnz, hipMemcpyHostToDevice,
                         s) != hipSuccess)
        st = RCM_ERR_HIP;
    }
    std::vector<rcm_stats> stats(G);
    if (st == RCM_OK)
      st = rcm_order_batched(G, vo.data(), no.data(), rp, ci, perm, stats.data(),
                             &cfg.order_options, ws, wsb, s);
    if (st == RCM_OK) {
      for (int32_t g = 0; g < G && st == RCM_OK; ++g)
        if (b[g]->n > 0 && hipMemcpyAsync(b[g]->perm_out, perm + vo[g], 4ull * b[g]->n,
                                          hipMemcpyDeviceToHost, s) != hipSuccess)
          st = RCM_ERR_HIP;
      if (st == RCM_OK && hipStreamSynchronize(s) != hipSuccess) st = RCM_ERR_HIP;
    }
    if (st == RCM_OK) {
      for (int32_t g = 0; g < G; ++g) {
        b[g]->res.status = RCM_OK;
        b[g]->res.stats = stats[g];
        b[g]->res.batch_size = G;
      }
      return;
    }
    (void)hipStreamSynchronize(s);
    {
      std::lock_guard<std::mutex> lk(mu);
      counters.retried_alone += G;
      counters.batches += G;
    }
    for (Request* r : b) {
      r->res.batch_size = 1;
      r->res.status = run_alone(r, base, s);
    }
  }

  void executor_loop() {
    (void)hipSetDevice(device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    while (true) {
      std::vector<Request*> b;
      uint64_t off = 0, bytes = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        work_cv.wait(lk, [&] {
          return (stopping && queue.empty()) ||
                 (!queue.empty() && queue.front()->alone <= arena->largest_free());
        });
        if (queue.empty()) break;
        b = take_batch(arena->largest_free(), &bytes);
        if (!arena->reserve(bytes, &off)) {
          // cannot happen: bytes <= the largest free block
          for (Request* r : b) r->res.status = RCM_ERR_OUT_OF_MEMORY;
          const double t = now();
          for (Request* r : b) {
            r->res.t_admit = t;
            r->res.t_done = t;
            r->done = true;
            counters.completed += 1;
            counters.failed += 1;
          }
          done_cv.notify_all();
          continue;
        }
        counters.bytes_in_flight = arena->used();
        counters.peak_bytes_in_flight =
            std::max(counters.peak_bytes_in_flight, counters.bytes_in_flight);
        counters.batches += 1;
        counters.max_batch_seen =
            std::max<int64_t>(counters.max_batch_seen, static_cast<int64_t>(b.size()));
        const double t = now();
        for (Request* r : b) r->res.t_admit = t;
        work_cv.notify_all();  // the next head may fit too
      }
      char* base = arena_base + off;
      if (s == nullptr) {
        for (Request* r : b) r->res.status = RCM_ERR_HIP;
      } else if (b.size() == 1) {
        b[0]->res.batch_size = 1;
        b[0]->res.status = run_alone(b[0], base, s);
      } else {
        run_batch(b, base, s);
      }
      finish(b, off);
    }
    if (s) (void)hipStreamDestroy(s);
  }
};

extern "C" {

void rcm_server_default_config(rcm_server_config* cfg) {
  if (cfg) std::memset(cfg, 0, sizeof(*cfg));
}

uint64_t rcm_server_request_bytes(int32_t n, int64_t nnz) {
  return alone_bytes(n, nnz, nullptr);
}

rcm_status rcm_server_create(const rcm_server_config* cfg_in, rcm_server** out) {
  if (!out) return RCM_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  rcm_server_config cfg{};
  if (cfg_in) cfg = *cfg_in;
  if (cfg.max_batch < 0 || cfg.executors < 0 || cfg.executors > kMaxExecutors ||
      cfg.batch_nnz_limit < 0)
    return RCM_ERR_INVALID_ARGUMENT;
  if (cfg.mem_budget_bytes == 0) cfg.mem_budget_bytes = 1ull << 30;
  if (cfg.max_batch == 0) cfg.max_batch = 32;
  if (cfg.executors == 0) cfg.executors = 2;
  if (cfg.batch_nnz_limit == 0) cfg.batch_nnz_limit = (1ll << 31) - 1;
  // reject bad ordering options (and an unreadable tuning table) now rather
  // than per request
  if (rcm_order_ex(0, nullptr, nullptr, nullptr, nullptr, nullptr, &cfg.order_options, nullptr, 0,
                   nullptr) != RCM_OK)
    return RCM_ERR_INVALID_ARGUMENT;
  if (cfg.order_options.tuning_file) {
    rcm_options probe = cfg.order_options;
    if (rcm_tuning_options(cfg.order_options.tuning_file, 1, 1, 1, &probe) != RCM_OK)
      return RCM_ERR_INVALID_ARGUMENT;
  }
  auto srv = std::make_unique<rcm_server>();
  srv->cfg = cfg;
  if (cfg.order_options.tuning_file) {
    srv->tuning_file = cfg.order_options.tuning_file;
    srv->cfg.order_options.tuning_file = srv->tuning_file.c_str();
  }
  if (hipGetDevice(&srv->device) != hipSuccess) return RCM_ERR_HIP;
  void* base = nullptr;
  if (hipMalloc(&base, cfg.mem_budget_bytes) != hipSuccess) return RCM_ERR_OUT_OF_MEMORY;
  srv->arena_base = static_cast<char*>(base);
  srv->arena = std::make_unique<Arena>(cfg.mem_budget_bytes);
  srv->counters.mem_budget_bytes = cfg.mem_budget_bytes;
  srv->t0 = std::chrono::steady_clock::now();
  rcm_server* raw = srv.get();
  for (int i = 0; i < cfg.executors; ++i) raw->executors.emplace_back([raw] { raw->executor_loop(); });
  *out = srv.release();
  return RCM_OK;
}

rcm_status rcm_server_submit(rcm_server* srv, int32_t n, int64_t nnz, const int32_t* rowptr_host,
                             const int32_t* colidx_host, int32_t* perm_out_host,
                             int64_t* ticket_out) {
  if (!srv || !ticket_out || n < 0 || nnz < 0) return RCM_ERR_INVALID_ARGUMENT;
  if (n > 0 && (!rowptr_host || !perm_out_host || (nnz > 0 && !colidx_host)))
    return RCM_ERR_INVALID_ARGUMENT;
  if (nnz >= (1ll << 31) - 1) return RCM_ERR_INVALID_ARGUMENT;
  auto r = std::make_unique<Request>();
  r->n = n;
  r->nnz = nnz;
  r->rowptr = rowptr_host;
  r->colidx = colidx_host;
  r->perm_out = perm_out_host;
  r->alone = alone_bytes(n, nnz, &srv->cfg.order_options);
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stopping) return RCM_ERR_INVALID_ARGUMENT;
  r->ticket = srv->next_ticket++;
  r->res.t_submit = srv->now();
  srv->counters.submitted += 1;
  Request* raw = r.get();
  *ticket_out = r->ticket;
  srv->live.emplace(r->ticket, std::move(r));
  // The device copies hold exactly nnz entries, so the row pointer's ends
  // must agree with nnz before anything reads colidx (the library checks the
  // rest of the pattern on the device).
  const bool bad_ends = n > 0 && (rowptr_host[0] != 0 || rowptr_host[n] != nnz);
  if (n == 0 || bad_ends || raw->alone > srv->cfg.mem_budget_bytes) {
    // nothing to order, malformed, or can never be admitted: complete now
    raw->res.status = n == 0 ? RCM_OK : bad_ends ? RCM_ERR_BAD_CSR : RCM_ERR_OUT_OF_MEMORY;
    raw->res.t_admit = raw->res.t_done = raw->res.t_submit;
    raw->done = true;
    srv->counters.completed += 1;
    if (n != 0) srv->counters.failed += 1;
    srv->done_cv.notify_all();
    return RCM_OK;
  }
  srv->queue.push_back(raw);
  srv->work_cv.notify_one();
  return RCM_OK;
}

rcm_status rcm_server_poll(rcm_server* srv, int64_t ticket, int32_t* done) {
  if (!srv || !done) return RCM_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->live.find(ticket);
  if (it == srv->live.end()) return RCM_ERR_INVALID_ARGUMENT;
  *done = it->second->done ? 1 : 0;
  return RCM_OK;
}

rcm_status rcm_server_wait(rcm_server* srv, int64_t ticket, int64_t timeout_ms,
                           rcm_request_result* result) {
  if (!srv) return RCM_ERR_INVALID_ARGUMENT;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->live.find(ticket);
  if (it == srv->live.end()) return RCM_ERR_INVALID_ARGUMENT;
  Request* r = it->second.get();
  auto ready = [&] { return r->done; };
  if (timeout_ms < 0) {
    srv->done_cv.wait(lk, ready);
  } else if (!srv->done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return RCM_ERR_ABORTED;
  }
  if (result) *result = r->res;
  srv->live.erase(it);
  return RCM_OK;
}

rcm_status rcm_server_counters_get(rcm_server* srv, rcm_server_counters* out) {
  if (!srv || !out) return RCM_ERR_INVALID_ARGUMENT;
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = srv->counters;
  return RCM_OK;
}

void rcm_server_destroy(rcm_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
  }
  srv->work_cv.notify_all();
  for (auto& t : srv->executors) t.join();
  if (srv->arena_base) (void)hipFree(srv->arena_base);
  delete srv;
}

}  // extern "C"
