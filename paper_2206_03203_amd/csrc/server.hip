// Serving: a request queue over resident hierarchies with continuous
// admission.  A fixed pool of slots (worker threads, each with its own HIP
// stream) takes requests in arrival order; a request is admitted as soon as a
// slot is free, its system is not already being solved by another slot, and
// the Krylov workspace it needs fits the memory budget (workspaces of idle
// systems are released, least recently used first, to make room).  Work of
// different slots runs concurrently on the device.  With grouping on (off by
// default), the slot that takes a request also takes every other queued
// request of the same system, and their columns run four at a time through
// the system's four-column batch (shared matrix reads), the rest one by one.
// Every kernel's reductions have a fixed order, so a column's result depends
// only on the columns it was grouped with: without grouping it does not
// depend on what else is in flight at all.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <list>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mdp.h"
#include "solver.hpp"

namespace mdp {
void set_last_error(const std::string &msg);
}

using namespace mdp;

namespace {

struct Request {
  uint64_t ticket = 0;
  mdp_handle *h = nullptr;
  const double *b = nullptr;
  double *x = nullptr;
  int32_t nrhs = 0;
  bool done = false;
  int rc = MDP_PENDING;
  std::string msg;  // error text, handed to the polling thread
  std::vector<mdp_stats> stats;
};

constexpr size_t kMaxQueue = 1 << 20;

}  // namespace

struct mdp_server {
  size_t budget = 0;  // bytes of Krylov workspace allowed at once (0 = no bound)
  int slots = 1;
  bool group = false;       // gather queued requests of one system (under mu)
  int64_t columns = 0;      // columns solved (under mu)
  int64_t grouped = 0;      // of which four at a time
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  std::set<mdp_handle *> registered, busy;
  std::list<mdp_handle *> lru;  // idle systems holding a workspace, least recent first
  size_t ws_bytes = 0;          // workspace bytes of registered systems
  uint64_t next_ticket = 1;
  int running = 0;
  bool stop = false;
  std::vector<std::thread> workers;

  size_t ws_of(mdp_handle *h) { return h->s.ws.allocated() ? h->s.ws.device_bytes() : 0; }

  // Under mu: can request r start now?  Releases idle workspaces if needed.
  bool admit(Request *r) {
    mdp_handle *h = r->h;
    if (busy.count(h)) return false;
    if (budget == 0 || h->s.ws.allocated()) return true;
    const size_t need = h->s.workspace_bytes_needed();
    while (ws_bytes + need > budget && !lru.empty()) {
      mdp_handle *v = lru.front();
      lru.pop_front();
      ws_bytes -= ws_of(v);
      v->s.ws.release();
    }
    if (ws_bytes + need <= budget) return true;
    return running == 0;  // nothing else can free memory: let it run alone
  }

  void worker() {
    hipStream_t s = nullptr;  // created on the first request this slot runs
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      Request *r = nullptr;
      cv_work.wait(lk, [&] {
        if (stop && queue.empty()) return true;
        for (Request *q : queue)
          if (admit(q)) return true;
        return false;
      });
      for (auto it = queue.begin(); it != queue.end(); ++it)
        if (admit(*it)) {
          r = *it;
          queue.erase(it);
          break;
        }
      if (!r) {
        if (stop && queue.empty()) break;
        continue;
      }
      mdp_handle *h = r->h;
      // the requests solved together: r, and with grouping every other
      // queued request of the same system, in arrival order
      std::vector<Request *> group_reqs{r};
      if (group)
        for (auto it = queue.begin(); it != queue.end();)
          if ((*it)->h == h) {
            group_reqs.push_back(*it);
            it = queue.erase(it);
          } else {
            ++it;
          }
      const bool grouping = group;
      busy.insert(h);
      lru.remove(h);
      const size_t before = ws_of(h);
      ++running;
      lk.unlock();
      std::vector<PairIO> cols;
      for (Request *q : group_reqs)
        for (int32_t k = 0; k < q->nrhs; ++k)
          cols.push_back(PairIO{q->b + static_cast<int64_t>(k) * h->s.n, q->x + static_cast<int64_t>(k) * h->s.n});
      std::vector<mdp_stats> st(cols.size());
      int64_t n_grouped = 0;
      int fail = MDP_OK;
      std::string msg;
      try {
        if (!s) MDP_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        h->s.ensure_workspace(s);
        solve_columns(h, cols, s, st.data(), grouping, &n_grouped);
      } catch (const Error &e) {
        fail = e.code;
        msg = e.msg;
      } catch (...) {
        fail = MDP_EHIP;
        msg = "unexpected failure in a server slot";
      }
      lk.lock();
      ws_bytes += ws_of(h) - before;
      --running;
      busy.erase(h);
      lru.push_back(h);
      columns += static_cast<int64_t>(cols.size());
      grouped += n_grouped;
      size_t c = 0;
      for (Request *q : group_reqs) {
        int worst = MDP_OK;
        for (int32_t k = 0; k < q->nrhs; ++k, ++c) {
          q->stats[k] = st[c];
          const int rc = fail != MDP_OK ? fail : st[c].status;
          if (rc < 0) {
            if (worst >= 0 || rc < worst) worst = rc;
          } else if (worst >= 0 && rc > worst) {
            worst = rc;
          }
        }
        q->rc = worst;
        if (worst < 0) q->msg = fail != MDP_OK ? msg : "a column of this request failed";
        q->done = true;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    lk.unlock();
    if (s) (void)hipStreamDestroy(s);
  }
};

extern "C" {

int mdp_server_create(size_t mem_budget_bytes, int32_t max_slots, mdp_server **out) {
  if (!out || max_slots < 1 || max_slots > 64) {
    set_last_error("max_slots must be in [1, 64]");
    return MDP_EINVAL;
  }
  auto srv = std::make_unique<mdp_server>();
  srv->budget = mem_budget_bytes;
  srv->slots = max_slots;
  try {
    for (int i = 0; i < max_slots; ++i) srv->workers.emplace_back([p = srv.get()] { p->worker(); });
  } catch (...) {
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->stop = true;
    }
    srv->cv_work.notify_all();
    for (auto &t : srv->workers) t.join();
    set_last_error("could not start server threads");
    return MDP_EINVAL;
  }
  *out = srv.release();
  return MDP_OK;
}

int mdp_server_set_grouping(mdp_server *srv, int32_t on) {
  if (!srv || (on != 0 && on != 1)) {
    set_last_error("NULL server or grouping not 0 / 1");
    return MDP_EINVAL;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->group = on != 0;
  return MDP_OK;
}

int mdp_server_counts(mdp_server *srv, int64_t *columns, int64_t *grouped) {
  if (!srv) {
    set_last_error("NULL server");
    return MDP_EINVAL;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  if (columns) *columns = srv->columns;
  if (grouped) *grouped = srv->grouped;
  return MDP_OK;
}

int mdp_server_register(mdp_server *srv, mdp_handle *h) {
  if (!srv || !h || !h->s.on_device) {
    set_last_error("NULL server or handle, or a host-only handle");
    return MDP_EINVAL;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->registered.insert(h).second) {
    srv->ws_bytes += srv->ws_of(h);
    srv->lru.push_back(h);
  }
  return MDP_OK;
}

int mdp_submit(mdp_server *srv, mdp_handle *h, const double *b, double *x, int32_t nrhs, uint64_t *ticket) {
  if (!srv || !h || !b || !x || nrhs < 1 || !ticket) {
    set_last_error("bad submit arguments");
    return MDP_EINVAL;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  if (!srv->registered.count(h)) {
    set_last_error("handle not registered with this server");
    return MDP_EINVAL;
  }
  if (srv->stop) {
    set_last_error("server is shutting down");
    return MDP_EINVAL;
  }
  if (srv->queue.size() >= kMaxQueue) {
    set_last_error("request queue full");
    return MDP_EBUSY;
  }
  auto r = std::make_unique<Request>();
  r->ticket = srv->next_ticket++;
  r->h = h;
  r->b = b;
  r->x = x;
  r->nrhs = nrhs;
  r->stats.resize(static_cast<size_t>(nrhs));
  *ticket = r->ticket;
  srv->queue.push_back(r.get());
  srv->reqs.emplace(r->ticket, std::move(r));
  srv->cv_work.notify_one();
  return MDP_OK;
}

int mdp_poll(mdp_server *srv, uint64_t ticket, mdp_stats *stats) {
  if (!srv) {
    set_last_error("NULL server");
    return MDP_EINVAL;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) {
    set_last_error("unknown or already collected ticket");
    return MDP_EINVAL;
  }
  Request *r = it->second.get();
  if (!r->done) return MDP_PENDING;
  const int rc = r->rc;
  if (rc < 0) set_last_error(r->msg);
  if (stats)
    for (size_t k = 0; k < r->stats.size(); ++k) stats[k] = r->stats[k];
  srv->reqs.erase(it);
  return rc;
}

int mdp_server_destroy(mdp_server *srv) {
  if (!srv) return MDP_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto &t : srv->workers) t.join();
  delete srv;
  return MDP_OK;
}

}  // extern "C"
