// Continuous batching of solves.  A worker thread admits queued requests in
// arrival order while fewer than max_slots solves are active and the
// request's workspace fits in the caller's device arena.  Admitted requests
// of one shape (grid, directions, model, restart length, preconditioner)
// join one Batch: each launch of a batch covers all of its solves, each
// solve runs its own restart cycles, and a request that arrives while
// others run joins at the batch's next tick (Arnoldi step).  Batches of different shapes run on streams of their own and
// overlap on the device.  A finished solve frees its arena range as soon as
// its result has been copied to the caller's buffer.
#include <atomic>
#include <chrono>
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
  bool finished = false;
  rte_status status = RTE_EAGAIN;
  rte_solve_stats stats{};
  double t_submit = 0;
};

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Group {
  std::unique_ptr<Batch> b;
  hipStream_t s = nullptr;
  size_t tab_off = 0;
};

}  // namespace

struct Server {
  char* arena = nullptr;
  size_t bytes = 0;
  int device = 0;
  int max_slots = 1;
  std::mutex mu;
  std::deque<Request*> queue;
  std::map<uint64_t, std::unique_ptr<Request>> tickets;
  std::map<size_t, size_t> used;  // offset -> length
  std::vector<std::unique_ptr<Group>> groups;  // worker thread only
  uint64_t next_ticket = 1;
  int64_t submitted = 0, completed = 0, active = 0;
  size_t in_use = 0, peak = 0;
  std::atomic<bool> stopping{false};
  std::thread worker;

  static size_t align(size_t b) { return (b + 255) & ~size_t(255); }

  // first fit over the gaps between used ranges (caller holds mu)
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

  Group* group_for(const Request* r) {
    for (auto& g : groups)
      if (g->b->compatible(*r->op, r->m, r->o.restart, r->o.precond) && !g->b->full()) return g.get();
    return nullptr;
  }

  // caller holds mu
  Group* make_group(const Request* r) {
    size_t off = 0;
    if (!alloc(align(batch_table_bytes(max_slots)), &off)) return nullptr;
    std::unique_ptr<Group> g(new Group());
    g->tab_off = off;
    try {
      RTE_HIP(hipStreamCreateWithFlags(&g->s, hipStreamNonBlocking));
      g->b.reset(new Batch(*r->op, r->m, r->o.restart, r->o.precond, max_slots, arena + off, g->s));
    } catch (...) {
      if (g->s) (void)hipStreamDestroy(g->s);
      release(off);
      throw;
    }
    groups.push_back(std::move(g));
    return groups.back().get();
  }

  // caller holds mu; frees the tables of batches with nothing to do
  bool reclaim() {
    bool any = false;
    for (size_t i = 0; i < groups.size();) {
      if (groups[i]->b->idle()) {
        groups[i]->b.reset();
        (void)hipStreamDestroy(groups[i]->s);
        release(groups[i]->tab_off);
        groups.erase(groups.begin() + long(i));
        any = true;
      } else {
        ++i;
      }
    }
    return any;
  }

  void retire(const Batch::Finished& f) {
    Request* r = static_cast<Request*>(f.tag);
    std::lock_guard<std::mutex> lk(mu);
    r->status = f.status;
    r->stats = f.stats;
    r->stats.status = f.status;
    r->stats.ms_total = now_ms() - r->t_submit;  // arrival to completion
    r->finished = true;
    release(r->off);
    --active;
    ++completed;
  }

  void fail_request(Request* r, rte_status st) {
    Batch::Finished f{};
    f.tag = r;
    f.status = st;
    retire(f);
  }

  void admit() {
    std::lock_guard<std::mutex> lk(mu);
    while (!queue.empty() && active < max_slots) {
      Request* r = queue.front();
      size_t off = 0;
      bool ws = alloc(r->need, &off);
      if (!ws && reclaim()) ws = alloc(r->need, &off);
      if (!ws) break;  // head of line waits for space
      Group* g = nullptr;
      try {
        g = group_for(r);
        if (!g) g = make_group(r);
        if (!g && reclaim()) g = make_group(r);
      } catch (...) {
        g = nullptr;
      }
      if (!g) {
        release(off);
        break;
      }
      queue.pop_front();
      r->off = off;
      ++active;
      try {
        g->b->add(r, *r->op, r->o, arena + off, r->x, r->t_submit);
      } catch (const Error& e) {
        r->status = e.code;
        r->stats.status = e.code;
        r->finished = true;
        release(off);
        --active;
        ++completed;
      }
    }
  }

  void loop() {
    (void)hipSetDevice(device);
    std::vector<Batch::Finished> done;
    while (true) {
      admit();
      {
        std::lock_guard<std::mutex> lk(mu);
        if (stopping && queue.empty() && active == 0) break;
      }
      bool progress = false;
      for (auto& g : groups) {
        done.clear();
        try {
          if (!g->b->idle() && g->b->ready()) {
            g->b->advance();
            progress = true;
          }
          g->b->collect(done);
        } catch (const Error& e) {
          g->b->abandon(e.code, done);
        } catch (...) {
          g->b->abandon(RTE_EDEVICE, done);
        }
        for (const auto& f : done) retire(f);
      }
      if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    std::lock_guard<std::mutex> lk(mu);
    reclaim();
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
    s->max_slots = max_slots;
    Server* raw = s.get();
    s->worker = std::thread([raw] { raw->loop(); });
    auto* h = new rte_server();
    h->s = std::move(s);
    *out = h;
  });
}

namespace {
// A validated request, not yet queued.
std::unique_ptr<Request> make_request(const Server& s, const rte_operator* op, const mgnet_model* model,
                                      const rte_solve_opts* opts, double* psi_out) {
  RTE_REQUIRE(op && opts && psi_out, RTE_EINVAL, "rte_submit: null argument");
  const Model* m = model ? model->m.get() : nullptr;
  validate_opts(*op->op, m, opts);
  RTE_REQUIRE(opts->x0 == nullptr || opts->x0 != psi_out, RTE_EINVAL, "x0 must not alias psi_out");
  std::unique_ptr<Request> r(new Request());
  r->op = op->op.get();
  r->m = m;
  r->o = *opts;
  r->x = psi_out;
  const bool mg = opts->precond == RTE_PC_MGNET_BF16 || opts->precond == RTE_PC_MGNET_FP32;
  r->need = Server::align(solve_layout(*r->op, m, opts->restart, mg).total);
  RTE_REQUIRE(r->need + Server::align(batch_table_bytes(s.max_slots)) <= s.bytes, RTE_ENOMEM,
              "request workspace exceeds the arena");
  return r;
}

// Queues the requests under one lock, so the worker admits them together.
void enqueue(Server& s, std::vector<std::unique_ptr<Request>>& rs, uint64_t* tickets) {
  const double t = now_ms();
  std::lock_guard<std::mutex> lk(s.mu);
  RTE_REQUIRE(!s.stopping, RTE_EINVAL, "server is shutting down");
  RTE_REQUIRE(s.queue.size() + rs.size() <= 4096, RTE_EAGAIN, "server queue is full");
  for (size_t i = 0; i < rs.size(); ++i) {
    std::unique_ptr<Request>& r = rs[i];
    r->t_submit = t;
    r->ticket = s.next_ticket++;
    tickets[i] = r->ticket;
    s.queue.push_back(r.get());
    s.tickets[r->ticket] = std::move(r);
    ++s.submitted;
  }
}
}  // namespace

rte_status rte_submit(rte_server* h, const rte_operator* op, const mgnet_model* model,
                      const rte_solve_opts* opts, double* psi_out, uint64_t* ticket) {
  return guarded2([&] {
    RTE_REQUIRE(h && ticket, RTE_EINVAL, "rte_submit: null argument");
    std::vector<std::unique_ptr<Request>> rs;
    rs.push_back(make_request(*h->s, op, model, opts, psi_out));
    enqueue(*h->s, rs, ticket);
  });
}

rte_status rte_submit_many(rte_server* h, int count, const rte_operator* const* ops,
                           const mgnet_model* const* models, const rte_solve_opts* opts, double* const* psi_out,
                           uint64_t* tickets) {
  return guarded2([&] {
    RTE_REQUIRE(h && count >= 0 && (count == 0 || (ops && opts && psi_out && tickets)), RTE_EINVAL,
                "rte_submit_many: null argument");
    std::vector<std::unique_ptr<Request>> rs;
    rs.reserve(size_t(count));
    for (int i = 0; i < count; ++i)
      rs.push_back(make_request(*h->s, ops[i], models ? models[i] : nullptr, opts + i, psi_out[i]));
    enqueue(*h->s, rs, tickets);
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
    out->active = s.active;
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
    delete h;
  });
}

}  // extern "C"
