// Continuous batching of independent solves.  A worker thread admits queued
// requests in arrival order while a slot (HIP stream) is free and the
// request's workspace fits in the caller's device arena, then advances every
// admitted solve whose last device result has arrived; finished solves free
// their slot and arena range at once, so later arrivals join while others
// are still running.  Each request runs the same SolveRun as rte_solve.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <thread>

#include "common.h"

namespace rte {
namespace {

struct Request {
  uint64_t ticket = 0;
  const Operator* op = nullptr;
  const Model* m = nullptr;
  rte_solve_opts o{};
  double* x = nullptr;
  size_t need = 0, off = 0;
  int slot = -1;
  std::unique_ptr<SolveRun> run;
  bool finished = false;
  rte_status status = RTE_EAGAIN;
  rte_solve_stats stats{};
  double t_submit = 0;
};

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct Server {
  char* arena = nullptr;
  size_t bytes = 0;
  int device = 0;
  std::vector<hipStream_t> streams;
  std::vector<bool> busy;
  std::mutex mu;
  std::deque<Request*> queue;
  std::vector<Request*> active;
  std::map<uint64_t, std::unique_ptr<Request>> tickets;
  std::map<size_t, size_t> used;  // offset -> length
  uint64_t next_ticket = 1;
  int64_t submitted = 0, completed = 0;
  size_t in_use = 0, peak = 0;
  std::atomic<bool> stopping{false};
  std::thread worker;

  static size_t align(size_t b) { return (b + 255) & ~size_t(255); }

  // first fit over the gaps between used ranges
  bool alloc(size_t need, size_t* off) {
    size_t cur = 0;
    for (auto& kv : used) {
      if (kv.first >= cur + need) break;
      cur = align(kv.first + kv.second);
    }
    if (cur + need > bytes) return false;
    used[cur] = need;
    *off = cur;
    in_use += need;
    if (in_use > peak) peak = in_use;
    return true;
  }
  void release(size_t off) {
    auto it = used.find(off);
    if (it == used.end()) return;
    in_use -= it->second;
    used.erase(it);
  }

  void retire(Request* r, rte_status st) {
    // nothing of this request may still be writing into its arena range
    if (r->slot >= 0) (void)hipStreamSynchronize(streams[r->slot]);
    r->run.reset();
    std::lock_guard<std::mutex> lk(mu);
    r->status = st;
    r->finished = true;
    r->stats.status = st;
    if (r->slot >= 0) busy[r->slot] = false;
    if (r->slot >= 0) release(r->off);
    ++completed;
  }

  void loop() {
    (void)hipSetDevice(device);
    while (true) {
      std::vector<Request*> admitted;
      {
        std::lock_guard<std::mutex> lk(mu);
        while (!queue.empty()) {
          int slot = -1;
          for (size_t i = 0; i < busy.size(); ++i)
            if (!busy[i]) { slot = int(i); break; }
          if (slot < 0) break;
          Request* r = queue.front();
          size_t off = 0;
          if (!alloc(r->need, &off)) break;  // head of line waits for space
          queue.pop_front();
          r->off = off;
          r->slot = slot;
          busy[slot] = true;
          active.push_back(r);
          admitted.push_back(r);
        }
        if (stopping && queue.empty() && active.empty()) return;
      }
      for (Request* r : admitted) {
        try {
          r->run.reset(new SolveRun(*r->op, r->m, r->o, arena + r->off, r->need, r->x, streams[r->slot]));
          r->run->start();
        } catch (const Error& e) {
          drop(r, e.code);
        } catch (...) {
          drop(r, RTE_EDEVICE);
        }
      }
      bool progress = false;
      for (size_t i = 0; i < active.size();) {
        Request* r = active[i];
        rte_status st = RTE_EAGAIN;
        try {
          if (r->run->ready()) {
            r->run->advance();
            progress = true;
            if (r->run->done()) {
              r->run->fill_stats(&r->stats);
              r->stats.ms_total = now_ms() - r->t_submit;  // arrival to completion
              st = r->run->status();
            }
          }
        } catch (const Error& e) {
          st = e.code;
        } catch (...) {
          st = RTE_EDEVICE;
        }
        if (st != RTE_EAGAIN) {
          {
            std::lock_guard<std::mutex> lk(mu);
            active.erase(active.begin() + i);
          }
          retire(r, st);
        } else {
          ++i;
        }
      }
      if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }

  void drop(Request* r, rte_status st) {
    {
      std::lock_guard<std::mutex> lk(mu);
      for (size_t i = 0; i < active.size(); ++i)
        if (active[i] == r) { active.erase(active.begin() + i); break; }
    }
    retire(r, st);
  }
};

}  // namespace rte

using namespace rte;

struct rte_server {
  std::unique_ptr<Server> s;
};

namespace {
template <class F>
rte_status guarded2(F&& f) {
  try {
    f();
    set_last_error("");
    return RTE_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return RTE_EDEVICE;
  }
}
}  // namespace

extern "C" {

rte_status rte_server_create(void* arena, size_t arena_bytes, int max_slots, rte_server** out) {
  return guarded2([&] {
    RTE_REQUIRE(out && arena, RTE_EINVAL, "rte_server_create: null argument");
    RTE_REQUIRE(max_slots >= 1 && max_slots <= 64, RTE_EINVAL, "max_slots must be in [1, 64]");
    RTE_REQUIRE((reinterpret_cast<uintptr_t>(arena) & 255) == 0, RTE_EINVAL, "arena must be 256-byte aligned");
    std::unique_ptr<Server> s(new Server());
    s->arena = static_cast<char*>(arena);
    s->bytes = arena_bytes;
    RTE_HIP(hipGetDevice(&s->device));
    for (int i = 0; i < max_slots; ++i) {
      hipStream_t st;
      RTE_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      s->streams.push_back(st);
      s->busy.push_back(false);
    }
    Server* raw = s.get();
    s->worker = std::thread([raw] { raw->loop(); });
    auto* h = new rte_server();
    h->s = std::move(s);
    *out = h;
  });
}

rte_status rte_submit(rte_server* h, const rte_operator* op, const mgnet_model* model,
                      const rte_solve_opts* opts, double* psi_out, uint64_t* ticket) {
  return guarded2([&] {
    RTE_REQUIRE(h && op && opts && psi_out && ticket, RTE_EINVAL, "rte_submit: null argument");
    Server& s = *h->s;
    const Model* m = model ? model->m.get() : nullptr;
    validate_opts(*op->op, m, opts);
    RTE_REQUIRE(opts->x0 == nullptr || opts->x0 != psi_out, RTE_EINVAL, "x0 must not alias psi_out");
    std::unique_ptr<Request> r(new Request());
    r->op = op->op.get();
    r->m = m;
    r->o = *opts;
    r->x = psi_out;
    r->need = Server::align(solve_layout(*r->op, m, opts->restart, opts->precond != RTE_PC_NONE).total);
    RTE_REQUIRE(r->need <= s.bytes, RTE_ENOMEM, "request workspace exceeds the arena");
    r->t_submit = now_ms();
    std::lock_guard<std::mutex> lk(s.mu);
    RTE_REQUIRE(!s.stopping, RTE_EINVAL, "server is shutting down");
    RTE_REQUIRE(s.queue.size() < 4096, RTE_EAGAIN, "server queue is full");
    r->ticket = s.next_ticket++;
    *ticket = r->ticket;
    s.queue.push_back(r.get());
    s.tickets[r->ticket] = std::move(r);
    ++s.submitted;
  });
}

rte_status rte_poll(rte_server* h, uint64_t ticket, rte_solve_stats* stats) {
  rte_status result = RTE_OK;
  rte_status st = guarded2([&] {
    RTE_REQUIRE(h != nullptr, RTE_EINVAL, "rte_poll: null server");
    Server& s = *h->s;
    std::lock_guard<std::mutex> lk(s.mu);
    auto it = s.tickets.find(ticket);
    RTE_REQUIRE(it != s.tickets.end(), RTE_ENOTFOUND, "unknown ticket");
    if (!it->second->finished) {
      result = RTE_EAGAIN;
      return;
    }
    if (stats) *stats = it->second->stats;
    result = it->second->status;
    s.tickets.erase(it);
  });
  if (st != RTE_OK) return st;
  if (result == RTE_EAGAIN) set_last_error("not finished");
  return result;
}

rte_status rte_server_query(rte_server* h, rte_server_stats* out) {
  return guarded2([&] {
    RTE_REQUIRE(h && out, RTE_EINVAL, "rte_server_query: null argument");
    Server& s = *h->s;
    std::lock_guard<std::mutex> lk(s.mu);
    out->submitted = s.submitted;
    out->completed = s.completed;
    out->active = int64_t(s.active.size());
    out->queued = int64_t(s.queue.size());
    out->arena_bytes = s.bytes;
    out->arena_in_use = s.in_use;
    out->arena_peak = s.peak;
  });
}

rte_status rte_server_destroy(rte_server* h) {
  return guarded2([&] {
    if (!h) return;
    h->s->stopping = true;
    if (h->s->worker.joinable()) h->s->worker.join();
    for (hipStream_t st : h->s->streams) (void)hipStreamDestroy(st);
    delete h;
  });
}

}  // extern "C"
