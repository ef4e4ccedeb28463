// Serving engine: a device-resident request loop over the MGR/FGMRES entry points.
//
// Requests (a Jacobian already in HBM, its labels, b, x) arrive at any time through
// mgr_server_submit.  `slots` worker threads, each with its own HIP stream, take admitted
// requests concurrently, so the kernels of several solves overlap on the device
// (continuous batching: a request is admitted as soon as a slot and enough of the HBM
// budget are free).  Admission is FIFO by estimated peak footprint
// (mgr_estimate_footprint for a fresh setup, plus the FGMRES workspace) against the budget;
// idle cached setups are evicted, least recently used first, to make room.  Setups are
// cached by a caller key (e.g. one realization across its Newton steps, whose Jacobians
// share a sparsity pattern): a request whose key has a cached setup with the same pattern
// reuses it, either as is (lagged preconditioner) or after mgr_setup_numeric.  Requests of
// one key run one at a time, in submission order.  Every request records its queueing,
// admission, start and completion times for latency percentiles.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "common.hpp"

using Clock = std::chrono::steady_clock;

struct mgr_server {
  mgr_server_config cfg;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  Clock::time_point t0 = Clock::now();

  struct Req {
    uint64_t ticket;
    mgr_request r;
    mgr_csr A;
    mgr_result res;
    size_t reserve = 0;
    bool done = false;
  };
  struct Entry {
    mgr_handle *h = nullptr;
    size_t bytes = 0;
    int64_t n = 0, nnz = 0;
    uint64_t last_use = 0;
    bool busy = false;
  };
  std::deque<uint64_t> queue;                 // tickets waiting for admission
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  std::map<uint64_t, Entry> cache;            // key -> setup
  std::map<uint64_t, int> key_busy;           // keys with a request in flight
  size_t used = 0;                            // reserved bytes (in flight + cached setups)
  uint64_t next_ticket = 1, use_clock = 0;
  int64_t completed = 0, hits = 0, misses = 0, evictions = 0;
  size_t peak_used = 0;
  std::vector<std::thread> workers;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  }
};

namespace {

size_t fresh_setup_bytes(const mgr_server *S, const mgr_csr &A, int64_t nnz) {
  size_t b = 0;
  mgr_estimate_footprint(mgr::scalar_rows(A), nnz, &S->cfg.opts, &b);
  return b;
}

// evict idle cached setups (LRU) until `need` fits; called with the lock held
bool make_room(mgr_server *S, size_t need) {
  while (S->used + need > S->cfg.budget_bytes) {
    uint64_t victim = 0;
    uint64_t best = UINT64_MAX;
    bool found = false;
    for (auto &kv : S->cache)
      if (!kv.second.busy && kv.second.last_use < best) {
        best = kv.second.last_use;
        victim = kv.first;
        found = true;
      }
    if (!found) return false;
    mgr_destroy(S->cache[victim].h);
    S->used -= S->cache[victim].bytes;
    S->cache.erase(victim);
    ++S->evictions;
  }
  return true;
}

// bytes a batched request adds for its share of the union (matrix copy and vectors)
size_t union_bytes(const mgr_server::Req *q) {
  return (size_t)q->r.nnz * 12 + (size_t)mgr::scalar_rows(q->A) * 40;
}

// With R admitted (no cached setup, small): take further admissible small requests
// without a cached setup, keys not in flight and not behind an earlier request of their
// key, up to batch_max in all.  Called with the lock held; R is batch[0].
void gather_batch(mgr_server *S, mgr_server::Req *R, std::vector<mgr_server::Req *> &batch) {
  batch.assign(1, R);
  const int cap = std::max(1, std::min(S->cfg.batch_max, 65535));
  std::map<uint64_t, bool> blocked;
  for (auto it = S->queue.begin(); it != S->queue.end() && (int)batch.size() < cap;) {
    mgr_server::Req *q = S->reqs[*it].get();
    const uint64_t key = q->r.key;
    bool take = !S->key_busy[key] && !blocked[key] && q->A.block <= 1 &&
                mgr::scalar_rows(q->A) <= S->cfg.batch_rows &&
                S->cache.find(key) == S->cache.end();
    size_t need = 0;
    if (take) {
      need = fgmres_workspace_bytes(mgr::scalar_rows(q->A), S->cfg.fopts.restart) +
             fresh_setup_bytes(S, q->A, q->r.nnz) + union_bytes(q);
      take = S->used + need <= S->cfg.budget_bytes;
    }
    if (!take) {
      blocked[key] = true;
      ++it;
      continue;
    }
    q->reserve = need;
    S->used += need;
    S->key_busy[key] = 1;
    q->res.t_admit_ms = S->now_ms();
    batch.push_back(q);
    it = S->queue.erase(it);
  }
  if (batch.size() > 1) {
    const size_t extra = union_bytes(R);
    R->reserve += extra;
    S->used += extra;
  }
  S->peak_used = std::max(S->peak_used, S->used);
}

// solve a gathered batch with mgr_batch_solve on this slot's stream
void run_batch(mgr_server *S, int slot, hipStream_t st, std::vector<mgr_server::Req *> &batch) {
  const int k = (int)batch.size();
  std::vector<mgr_csr> A(k);
  std::vector<const int8_t *> lab(k);
  std::vector<const double *> b(k);
  std::vector<double *> x(k);
  std::vector<double> rel(k, 0.0);
  std::vector<int32_t> its(k, 0);
  for (int i = 0; i < k; ++i) {
    A[i] = batch[i]->A;
    lab[i] = batch[i]->r.labels;
    b[i] = batch[i]->r.b;
    x[i] = batch[i]->r.x;
  }
  const double t_start = S->now_ms();
  fgmres_result fr{};
  const mgr_status code = mgr_batch_solve(k, A.data(), lab.data(), b.data(), x.data(),
                                          &S->cfg.opts, &S->cfg.fopts, rel.data(), its.data(),
                                          &fr, st);
  (void)hipStreamSynchronize(st);
  const double t_end = S->now_ms();
  std::lock_guard<std::mutex> g(S->mu);
  for (int i = 0; i < k; ++i) {
    mgr_result &res = batch[i]->res;
    res.slot = slot;
    res.t_start_ms = t_start;
    res.t_end_ms = t_end;
    res.setup_ms = 0.0;
    res.solve_ms = t_end - t_start;
    res.iters = its[i];
    res.true_relres = rel[i];
    res.setup_reused = 0;
    res.batch = k;
    res.footprint = 0;
    res.status = code == MGR_OK || code == MGR_ERR_NOT_CONVERGED
                     ? (rel[i] <= S->cfg.fopts.rtol ? MGR_OK : MGR_ERR_NOT_CONVERGED)
                     : code;
    S->used -= batch[i]->reserve;
    S->key_busy[batch[i]->r.key] = 0;
    ++S->misses;
    ++S->completed;
    batch[i]->done = true;
  }
  S->cv_done.notify_all();
  S->cv_work.notify_all();
}

void worker(mgr_server *S, int slot) {
  hipStream_t st = nullptr;
  (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  void *work = nullptr;
  size_t work_bytes = 0;
  std::vector<mgr_server::Req *> batch;
  for (;;) {
    mgr_server::Req *R = nullptr;
    bool hit = false;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      for (;;) {
        if (S->stop && S->queue.empty()) break;
        // first admissible request in FIFO order; requests of a key that is in flight
        // wait (and so do the later requests of that key); a request that can never fit
        // the budget is rejected and the scan restarts
        bool rescan = true;
        while (rescan && !R) {
          rescan = false;
          std::map<uint64_t, bool> blocked;
          for (auto it = S->queue.begin(); it != S->queue.end(); ++it) {
            mgr_server::Req *q = S->reqs[*it].get();
            const uint64_t key = q->r.key;
            if (S->key_busy[key] || blocked[key]) { blocked[key] = true; continue; }
            const int64_t nnz = q->r.nnz;
            auto c = S->cache.find(key);
            if (c != S->cache.end() && !c->second.busy &&
                (c->second.n != mgr::scalar_rows(q->A) || c->second.nnz != nnz)) {
              // the key now names a matrix of another size: drop the stale setup
              mgr_destroy(c->second.h);
              S->used -= c->second.bytes;
              S->cache.erase(c);
              c = S->cache.end();
            }
            const bool cached = c != S->cache.end() && !c->second.busy;
            size_t need = fgmres_workspace_bytes(mgr::scalar_rows(q->A), S->cfg.fopts.restart);
            if (!cached) need += fresh_setup_bytes(S, q->A, nnz);
            if (need > S->cfg.budget_bytes) {
              q->res.status = MGR_ERR_ALLOC;
              q->res.t_admit_ms = q->res.t_start_ms = q->res.t_end_ms = S->now_ms();
              q->done = true;
              S->queue.erase(it);
              S->cv_done.notify_all();
              rescan = true;
              break;
            }
            // a cached setup this request will use is marked busy first, so that making
            // room never evicts it
            if (cached) c->second.busy = true;
            if (S->used + need > S->cfg.budget_bytes && !make_room(S, need)) {
              if (cached) c->second.busy = false;
              break;  // strict FIFO for memory: the head blocks the requests behind it
            }
            R = q;
            hit = cached;
            R->reserve = need;
            S->used += need;
            S->peak_used = std::max(S->peak_used, S->used);
            S->key_busy[key] = 1;
            S->queue.erase(it);
            break;
          }
        }
        if (R) break;
        S->cv_work.wait(lk);
      }
      if (!R) break;
      R->res.t_admit_ms = S->now_ms();
      if (!hit && S->cfg.batch_rows > 0 && R->A.block <= 1 && mgr::scalar_rows(R->A) <= S->cfg.batch_rows)
        gather_batch(S, R, batch);
    }
    if (batch.size() > 1) {
      run_batch(S, slot, st, batch);
      batch.clear();
      continue;
    }
    batch.clear();
    // ---- run the request on this slot's stream (no lock held) ----
    mgr_result &res = R->res;
    res.slot = slot;
    mgr_status st_code = MGR_OK;
    mgr_handle *h = nullptr;
    const uint64_t key = R->r.key;
    const double t_start = S->now_ms();
    res.t_start_ms = t_start;
    if (hit) {
      std::lock_guard<std::mutex> g(S->mu);
      h = S->cache[key].h;
    }
    if (hit && R->r.refresh_setup) {
      st_code = mgr_setup_numeric(h, &R->A, st);
      if (st_code != MGR_OK) {
        // the refresh left no usable setup: drop the cache entry.  A new pattern under the
        // same key goes back to the head of the queue, to be admitted again with the
        // footprint of a fresh setup; any other failure completes the request.
        const bool requeue = st_code == MGR_ERR_PATTERN;
        std::lock_guard<std::mutex> g(S->mu);
        auto c = S->cache.find(key);
        if (c != S->cache.end() && c->second.h == h) {
          S->used -= c->second.bytes;
          S->cache.erase(c);
        }
        mgr_destroy(h);
        h = nullptr;
        S->used -= R->reserve;
        R->reserve = 0;
        S->key_busy[key] = 0;
        if (requeue) {
          S->queue.push_front(R->ticket);
        } else {
          res.status = st_code;
          res.t_end_ms = S->now_ms();
          res.setup_reused = 0;
          res.batch = 1;
          ++S->misses;
          ++S->completed;
          R->done = true;
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
        continue;
      }
    }
    if (!hit) st_code = mgr_setup(&R->A, R->r.labels, &S->cfg.opts, st, &h);
    res.setup_reused = hit ? 1 : 0;
    res.batch = 1;
    const double t_setup = S->now_ms();
    const size_t need_ws = fgmres_workspace_bytes(mgr::scalar_rows(R->A), S->cfg.fopts.restart);
    if (st_code == MGR_OK && need_ws > work_bytes) {
      if (work) mgr::dfree(work, st);
      try {
        work = mgr::dalloc(need_ws, st);
        work_bytes = need_ws;
      } catch (const mgr::Error &) {
        work = nullptr;
        work_bytes = 0;
        st_code = MGR_ERR_ALLOC;
      }
    }
    fgmres_result fr{};
    if (st_code == MGR_OK) {
      st_code = fgmres_solve(&R->A, h, R->r.b, R->r.x, &S->cfg.fopts, work, work_bytes, &fr, st);
      (void)hipStreamSynchronize(st);
    }
    const double t_end = S->now_ms();
    res.status = st_code;
    res.iters = fr.iters;
    res.true_relres = fr.true_relres;
    res.setup_ms = t_setup - t_start;
    res.solve_ms = t_end - t_setup;
    res.t_end_ms = t_end;
    size_t fp = 0;
    if (h) mgr_footprint(h, &fp);
    res.footprint = fp;
    {
      std::lock_guard<std::mutex> g(S->mu);
      S->used -= R->reserve;
      if (h) {
        // a setup is kept when it was built (a solve that failed to converge still leaves
        // a valid setup)
        const bool keep = S->cfg.cache_setups && !R->r.last_use &&
                          (st_code == MGR_OK || st_code == MGR_ERR_NOT_CONVERGED);
        auto c = S->cache.find(key);
        if (keep) {
          if (c == S->cache.end()) {
            mgr_server::Entry e;
            e.h = h;
            e.bytes = fp;
            e.n = mgr::scalar_rows(R->A);
            e.nnz = R->r.nnz;
            S->cache[key] = e;
            S->used += fp;
            S->peak_used = std::max(S->peak_used, S->used);
            c = S->cache.find(key);
          }
          c->second.busy = false;
          c->second.last_use = ++S->use_clock;
        } else {
          if (c != S->cache.end() && c->second.h == h) {
            S->used -= c->second.bytes;
            S->cache.erase(c);
          }
          mgr_destroy(h);
        }
      }
      if (hit) ++S->hits; else ++S->misses;
      S->key_busy[key] = 0;
      R->done = true;
      ++S->completed;
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
  if (work) mgr::dfree(work, st);
  (void)hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

void mgr_server_default_config(mgr_server_config *c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->budget_bytes = (size_t)64 << 30;
  c->slots = 4;
  mgr_default_opts(&c->opts);
  c->fopts.restart = 30;
  c->fopts.maxit = 1000;
  c->fopts.rtol = 1e-6;
  c->cache_setups = 1;
  c->batch_rows = 0;
  c->batch_max = 16;
}

mgr_status mgr_server_create(const mgr_server_config *cfg, mgr_server **out) {
  if (!cfg || !out || cfg->slots < 1 || cfg->slots > 64 || cfg->batch_rows < 0 ||
      (cfg->batch_rows > 0 && (cfg->batch_max < 1 || cfg->batch_max > 65535))) {
    mgr::set_last_error("bad server configuration");
    return MGR_ERR_ARG;
  }
  auto *S = new mgr_server();
  S->cfg = *cfg;
  for (int i = 0; i < cfg->slots; ++i) S->workers.emplace_back(worker, S, i);
  *out = S;
  return MGR_OK;
}

mgr_status mgr_server_submit(mgr_server *S, const mgr_request *r, uint64_t *ticket) {
  if (!S || !r || !r->A || !r->labels || !r->b || !r->x || !ticket) {
    mgr::set_last_error("null argument");
    return MGR_ERR_ARG;
  }
  auto q = std::make_unique<mgr_server::Req>();
  q->r = *r;
  q->A = *r->A;
  q->r.A = &q->A;
  std::memset(&q->res, 0, sizeof(q->res));
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stop) {
      mgr::set_last_error("server is stopping");
      return MGR_ERR_ARG;
    }
    q->ticket = S->next_ticket++;
    q->res.t_submit_ms = S->now_ms();
    *ticket = q->ticket;
    S->queue.push_back(q->ticket);
    S->reqs[q->ticket] = std::move(q);
  }
  S->cv_work.notify_all();
  return MGR_OK;
}

mgr_status mgr_server_wait(mgr_server *S, uint64_t ticket, mgr_result *res) {
  if (!S) return MGR_ERR_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) {
    mgr::set_last_error("unknown ticket");
    return MGR_ERR_ARG;
  }
  S->cv_done.wait(lk, [&] { return it->second->done; });
  if (res) *res = it->second->res;
  const mgr_status st = (mgr_status)it->second->res.status;
  S->reqs.erase(it);
  return st;
}

int32_t mgr_server_poll(mgr_server *S, uint64_t ticket) {
  if (!S) return -1;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return -1;
  return it->second->done ? 1 : 0;
}

mgr_status mgr_server_stats(mgr_server *S, mgr_server_stats_t *out) {
  if (!S || !out) return MGR_ERR_ARG;
  std::lock_guard<std::mutex> g(S->mu);
  out->completed = S->completed;
  out->queued = (int64_t)S->queue.size();
  out->cache_hits = S->hits;
  out->cache_misses = S->misses;
  out->evictions = S->evictions;
  out->cached_setups = (int64_t)S->cache.size();
  out->reserved_bytes = S->used;
  out->peak_reserved_bytes = S->peak_used;
  return MGR_OK;
}

void mgr_server_destroy(mgr_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto &t : S->workers) t.join();
  for (auto &kv : S->cache) mgr_destroy(kv.second.h);
  delete S;
  // The blocks of the server's setups and workspaces went back to the allocator's cache
  // under the streams of its slots, which no longer exist: no later allocation would find
  // them, so they are returned to HIP.
  (void)mgr_release_cache();
}

}  // extern "C"
