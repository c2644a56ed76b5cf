// Continuous-batching server (part of the C ABI in include/osqp_mi.h).
// Included at the end of api.hip: it drives the batch API above.
//
// One scheduler thread owns the device work.  Each pass it (1) retires
// launches whose stream has drained and hands their results to the waiting
// clients, (2) admits queued requests while slots, the HBM budget and the
// launch limit allow: fresh QPs form one new micro-batch, first requests of
// new structure keys one new resident pool, and requests for keys already
// resident one subset re-solve per pool through the vector update and warm
// start of Section 6 -- each launched asynchronously on its batch's stream,
// so work admitted now overlaps work already on the device.  A large fresh
// QP gets a launch of its own, so that small ones admitted with it do not
// wait for it.
#pragma once

#include <atomic>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace {

constexpr int kServerMaxLaunches = 8;   // launches on the device at once
// a fresh QP whose matrices hold at least this many entries (2 nnz(A) +
// nnz(P full) + n + m, the work queue's cost measure) is launched alone: a
// launch's results come back when all of its QPs are done, so small QPs
// admitted in the same round would otherwise wait for it
constexpr int64_t kServerAloneCost = 200000;

struct OwnedQP {
  int n = 0, m = 0;
  std::vector<int> Pp, Pi, Ap, Ai;
  std::vector<double> Px, Ax, q, l, u, xws, yws;
  bool has_x = false, has_y = false;

  void copy_from(const osqp_problem &p, const double *x, const double *y) {
    n = p.n; m = p.m;
    Pp.assign(p.P_upper.indptr, p.P_upper.indptr + n + 1);
    Pi.assign(p.P_upper.indices, p.P_upper.indices + p.P_upper.nnz);
    Px.assign(p.P_upper.data, p.P_upper.data + p.P_upper.nnz);
    Ap.assign(p.A.indptr, p.A.indptr + m + 1);
    Ai.assign(p.A.indices, p.A.indices + p.A.nnz);
    Ax.assign(p.A.data, p.A.data + p.A.nnz);
    q.assign(p.q, p.q + n);
    l.assign(p.l, p.l + m);
    u.assign(p.u, p.u + m);
    has_x = x != nullptr;
    has_y = y != nullptr;
    if (x) xws.assign(x, x + n);
    if (y) yws.assign(y, y + m);
  }
  osqp_problem view() const {
    osqp_problem p;
    p.n = n; p.m = m;
    p.P_upper = {n, n, (int)Px.size(), Pp.data(), Pi.data(), Px.data()};
    p.q = q.data();
    p.A = {m, n, (int)Ax.size(), Ap.data(), Ai.data(), Ax.data()};
    p.l = l.data();
    p.u = u.data();
    return p;
  }
};

struct ServerReq {
  uint64_t ticket = 0, key = 0;
  OwnedQP qp;
  size_t bytes = 0;
  int64_t cost = 0;   // 2 nnz(A) + nnz(P full) + n + m
  double t_submit = 0.0;
};

struct ServerResult {
  bool done = false;
  int rc = OSQP_OK;
  std::vector<double> x, y;
  osqp_info info{};
  double latency = 0.0;
};

// A resident batch holding the structures of several keys: matrices,
// scaling, factors and iterates stay on the device; requests for its keys
// are re-solved as a subset of it (new vectors, warm start from the last
// solution of the same key).
struct Pool {
  osqp_batch *b = nullptr;
  std::vector<uint64_t> keys;   // key of each QP of the batch
  size_t bytes = 0;
  bool busy = false;            // a solve of this batch is on the device
  uint64_t last_use = 0;
};

struct KeySlot {
  int pool = -1, idx = -1;
};

// kind: 0 fresh micro-batch, 1 new pool (first requests of new keys),
// 2 re-solve of a subset of a pool
struct InFlight {
  osqp_batch *b = nullptr;
  int kind = 0, pool = -1;
  size_t bytes = 0;
  std::vector<std::shared_ptr<ServerReq>> reqs;
  std::vector<int> idx;         // batch index of each request
};

// HBM a request needs on the device, an upper bound: the arena, the
// reduced-system path the setup may give it (the largest of those it is
// eligible for: the dense factor, the low-rank blocks, the band factor with
// the largest block) with one workgroup's scratch slot, and the polishing
// workspace of the form it would be polished in.
size_t estimate_bytes(const osqp_problem &p, const osqp_settings &s) {
  const double t = s.precision == OSQP_PRECISION_FP64 ? 8.0 : 4.0;
  const double a = p.A.nnz, pu = p.P_upper.nnz, n = p.n, m = p.m;
  double b = a * (4 + 4 + 8 + 8 + 8 + 8 + 2 * t) + 2.0 * pu * (4 + 8 + 8 + t) +
             n * (12 * 8 + 10 * t) + m * (14 * 8 + 10 * t) +
             1024.0 * 1024;   // descriptors, work lists, grid partials (up to 2048 blocks)
  const int R = count_multi_rows(p);
  const bool lr = lowrank_fits(p, R);
  const double n8 = (p.n + 7) & ~7;
  double path = 0.0;
  if (s.linsys != OSQP_LINSYS_PCG) {
    // dense: factor (n x n8), inverses of its 64 x 64 diagonal blocks, one
    // rank-k scratch slot (n x R)
    const double dense = (n * n8 + (double)((p.n + 63) / 64) * 4096.0 + n * R) * t;
    if (s.linsys == OSQP_LINSYS_DENSE) {
      if (p.n <= kDenseMaxN) path = dense;
    } else {
      if (p.n <= kDenseAutoN) path = dense;
      if (lr) {
        const int ldS = (R + 7) & ~7;
        const double scratch = std::max<double>((double)R * n8,
                                                (double)R * ldS + (double)spd_inverse_extra(R));
        path = std::max(path, 8.0 * ((double)lr_layout(p.n, p.m, R, ldS).total + scratch));
      }
      bool short_rows = p.n <= kBandMaxN;
      for (int i = 0; i < p.m && short_rows; ++i)
        short_rows = p.A.indptr[i + 1] - p.A.indptr[i] <= kBandMaxNB + 1;
      if (short_rows) {
        // tiles 2 ceil(n / nb) nb^2 <= 2 (n nb + nb^2) for nb <= 64, the
        // residual, one formation scratch slot
        const double tiles = 2.0 * (n * kBandMaxNB + (double)kBandMaxNB * kBandMaxNB);
        path = std::max(path, 8.0 * (tiles + n8 + (double)band_scratch(kBandMaxNB)));
      }
    }
  }
  b += path;
  if (s.polish && (lr || p.n <= kPolishMaxN))
    b += 8.0 * ((double)polish_ws_doubles(p.n, p.m, R, lr) + 8.0) + 64.0;
  return (size_t)b;
}

}  // namespace

struct osqp_server {
  osqp_settings set{};
  size_t budget = 0;
  int max_slots = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<ServerReq>> queue;
  std::unordered_map<uint64_t, ServerResult> results;
  std::unordered_map<int, Pool> pools;
  std::unordered_map<uint64_t, KeySlot> keymap;     // resident keys
  std::unordered_map<uint64_t, int> pending_keys;   // keys of a new pool on the device
  int next_pool = 1;
  std::vector<InFlight> inflight;
  size_t used = 0;
  int slots = 0;
  uint64_t next_ticket = 1, tick = 0;
  int64_t completed = 0, batches = 0, peak_inflight = 0, peak_bytes = 0;
  bool stop = false;
  std::thread worker;
};

namespace {

void server_finish(osqp_server *sv, InFlight &f) {
  int rc = osqp_batch_sync(f.b);
  const double now = now_s();
  std::vector<ServerResult> out(f.reqs.size());
  for (size_t k = 0; k < f.reqs.size(); ++k) {
    ServerResult &r = out[k];
    r.done = true;
    r.x.resize(f.reqs[k]->qp.n);
    r.y.resize(f.reqs[k]->qp.m);
    int rk = rc;
    if (rk == OSQP_OK) rk = osqp_batch_get(f.b, f.idx[k], r.x.data(), r.y.data(), &r.info);
    r.rc = rk;
    r.latency = now - f.reqs[k]->t_submit;
  }
  std::lock_guard<std::mutex> g(sv->mu);
  for (size_t k = 0; k < f.reqs.size(); ++k) sv->results[f.reqs[k]->ticket] = std::move(out[k]);
  sv->completed += (int64_t)f.reqs.size();
  sv->slots -= (int)f.reqs.size();
  if (f.kind == 0) {
    osqp_batch_cleanup(f.b);
    sv->used -= f.bytes;
  } else if (f.kind == 1) {
    Pool pl;
    pl.b = f.b;
    pl.bytes = f.bytes;
    pl.last_use = ++sv->tick;
    for (size_t k = 0; k < f.reqs.size(); ++k) {
      pl.keys.push_back(f.reqs[k]->key);
      sv->keymap[f.reqs[k]->key] = KeySlot{f.pool, (int)k};
      sv->pending_keys.erase(f.reqs[k]->key);
    }
    sv->pools[f.pool] = std::move(pl);
  } else {
    Pool &pl = sv->pools[f.pool];
    pl.busy = false;
    pl.last_use = ++sv->tick;
  }
  sv->cv_done.notify_all();
  sv->cv_work.notify_all();
}

void server_fail(osqp_server *sv, const std::vector<std::shared_ptr<ServerReq>> &reqs, int rc,
                 size_t bytes) {
  std::lock_guard<std::mutex> g(sv->mu);
  for (auto &q : reqs) {
    ServerResult r;
    r.done = true;
    r.rc = rc;
    sv->results[q->ticket] = std::move(r);
    sv->pending_keys.erase(q->key);
  }
  sv->slots -= (int)reqs.size();
  sv->used -= bytes;
  sv->completed += (int64_t)reqs.size();
  sv->cv_done.notify_all();
}

// Evict idle pools, least recently used first, until `need` more bytes fit
// (called with the lock held).
bool server_make_room(osqp_server *sv, size_t need) {
  while (sv->used + need > sv->budget) {
    int victim = 0;
    uint64_t best = UINT64_MAX;
    for (auto &kv : sv->pools)
      if (!kv.second.busy && kv.second.last_use < best) { best = kv.second.last_use; victim = kv.first; }
    if (!victim) return false;
    Pool &pl = sv->pools[victim];
    for (uint64_t key : pl.keys) sv->keymap.erase(key);
    osqp_batch_cleanup(pl.b);
    sv->used -= pl.bytes;
    sv->pools.erase(victim);
  }
  return true;
}

// Setup (and warm starts) of a new batch from requests; solve queued.
int server_new_batch(osqp_server *sv, const std::vector<std::shared_ptr<ServerReq>> &reqs,
                     osqp_batch **out) {
  std::vector<osqp_problem> probs;
  for (auto &r : reqs) probs.push_back(r->qp.view());
  osqp_batch *b = nullptr;
  int rc = osqp_batch_setup(&b, (int)probs.size(), probs.data(), &sv->set);
  for (size_t k = 0; rc == OSQP_OK && k < reqs.size(); ++k)
    if (reqs[k]->qp.has_x || reqs[k]->qp.has_y)
      rc = warm_start_impl(b, (int)k, reqs[k]->qp.has_x ? reqs[k]->qp.xws.data() : nullptr,
                           reqs[k]->qp.has_y ? reqs[k]->qp.yws.data() : nullptr, false);
  if (rc == OSQP_OK) rc = osqp_batch_solve_async(b);
  if (rc != OSQP_OK && b) {
    osqp_batch_cleanup(b);
    b = nullptr;
  }
  *out = b;
  return rc;
}

void server_loop(osqp_server *sv) {
  for (;;) {
    // (1) retire drained launches
    std::vector<InFlight> done;
    {
      std::lock_guard<std::mutex> g(sv->mu);
      for (size_t k = 0; k < sv->inflight.size();) {
        if (hipStreamQuery(sv->inflight[k].b->stream) == hipSuccess) {
          done.push_back(std::move(sv->inflight[k]));
          sv->inflight.erase(sv->inflight.begin() + k);
        } else {
          ++k;
        }
      }
    }
    for (auto &f : done) server_finish(sv, f);

    // (2) admission under the lock, launches outside it.  At most
    // kServerMaxLaunches launches are on the device at once; while it is
    // full, requests accumulate and are admitted together when a launch
    // drains (continuous batching: few large launches instead of many small
    // ones queued on the device's few hardware queues).  Each round forms
    // one micro-batch of fresh QPs, one new pool of first requests of new
    // keys, and one subset re-solve per resident pool with requests.
    std::vector<std::shared_ptr<ServerReq>> fresh, firsts, alone;
    std::unordered_map<int, std::vector<std::pair<std::shared_ptr<ServerReq>, int>>> repeats;
    size_t fresh_bytes = 0, first_bytes = 0, alone_bytes = 0;
    int new_pool = 0;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      if (sv->queue.empty() && sv->inflight.empty()) {
        if (sv->stop) return;
        sv->cv_work.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
        if (sv->stop && sv->queue.empty()) return;
      }
      int launches = (int)sv->inflight.size();
      std::unordered_map<uint64_t, int> chosen;
      for (auto it = sv->queue.begin(); it != sv->queue.end();) {
        auto &rq = *it;
        int admitted = (int)(fresh.size() + firsts.size() + alone.size());
        for (auto &kv : repeats) admitted += (int)kv.second.size();
        if (sv->slots + admitted >= sv->max_slots) break;
        const size_t taken = fresh_bytes + first_bytes + alone_bytes;
        if (rq->key == 0 && rq->cost >= kServerAloneCost) {
          // a large fresh QP: a launch of its own (FIFO for fresh QPs)
          if (launches >= kServerMaxLaunches) break;
          if (!server_make_room(sv, taken + rq->bytes)) break;
          ++launches;
          alone_bytes += rq->bytes;
          alone.push_back(rq);
          it = sv->queue.erase(it);
          continue;
        }
        if (rq->key == 0) {
          if (fresh.empty() && launches >= kServerMaxLaunches) break;   // FIFO for fresh QPs
          if (!server_make_room(sv, taken + rq->bytes)) break;
          if (fresh.empty()) ++launches;
          fresh_bytes += rq->bytes;
          fresh.push_back(rq);
          it = sv->queue.erase(it);
          continue;
        }
        if (chosen.count(rq->key) || sv->pending_keys.count(rq->key)) { ++it; continue; }
        auto ks = sv->keymap.find(rq->key);
        if (ks != sv->keymap.end()) {
          Pool &pl = sv->pools[ks->second.pool];
          const bool opens = !repeats.count(ks->second.pool);
          // a pool still re-solving from an earlier round waits; one taken
          // in this round is marked busy at once, so that making room for a
          // later request of this round cannot evict it
          if (opens && (pl.busy || launches >= kServerMaxLaunches)) { ++it; continue; }
          if (opens) {
            ++launches;
            pl.busy = true;
          }
          repeats[ks->second.pool].push_back({rq, ks->second.idx});
          chosen[rq->key] = 1;
          it = sv->queue.erase(it);
          continue;
        }
        // first request of a key: joins this round's new pool
        if (firsts.empty() && launches >= kServerMaxLaunches) { ++it; continue; }
        if (!server_make_room(sv, taken + rq->bytes)) { ++it; continue; }
        if (firsts.empty()) ++launches;
        first_bytes += rq->bytes;
        firsts.push_back(rq);
        chosen[rq->key] = 1;
        it = sv->queue.erase(it);
      }
      if (!firsts.empty()) {
        new_pool = sv->next_pool++;
        for (auto &r : firsts) sv->pending_keys[r->key] = new_pool;
      }
      sv->used += fresh_bytes + first_bytes + alone_bytes;
      int admitted = (int)(fresh.size() + firsts.size() + alone.size());
      for (auto &kv : repeats) admitted += (int)kv.second.size();
      sv->slots += admitted;
      sv->peak_bytes = std::max<int64_t>(sv->peak_bytes, (int64_t)sv->used);
    }
    std::vector<InFlight> launched;
    for (auto &rq : alone) {
      std::vector<std::shared_ptr<ServerReq>> one{rq};
      osqp_batch *b = nullptr;
      const int rc = server_new_batch(sv, one, &b);
      if (rc == OSQP_OK) {
        InFlight f;
        f.b = b; f.kind = 0; f.bytes = rq->bytes; f.reqs = one;
        f.idx.push_back(0);
        launched.push_back(std::move(f));
      } else {
        server_fail(sv, one, rc, rq->bytes);
      }
    }
    if (!fresh.empty()) {
      osqp_batch *b = nullptr;
      const int rc = server_new_batch(sv, fresh, &b);
      if (rc == OSQP_OK) {
        InFlight f;
        f.b = b; f.kind = 0; f.bytes = fresh_bytes; f.reqs = fresh;
        for (size_t k = 0; k < fresh.size(); ++k) f.idx.push_back((int)k);
        launched.push_back(std::move(f));
      } else {
        server_fail(sv, fresh, rc, fresh_bytes);
      }
    }
    if (!firsts.empty()) {
      osqp_batch *b = nullptr;
      const int rc = server_new_batch(sv, firsts, &b);
      if (rc == OSQP_OK) {
        InFlight f;
        f.b = b; f.kind = 1; f.pool = new_pool; f.bytes = first_bytes; f.reqs = firsts;
        for (size_t k = 0; k < firsts.size(); ++k) f.idx.push_back((int)k);
        launched.push_back(std::move(f));
      } else {
        server_fail(sv, firsts, rc, first_bytes);
      }
    }
    for (auto &kv : repeats) {
      osqp_batch *b;
      {
        std::lock_guard<std::mutex> g(sv->mu);
        b = sv->pools[kv.first].b;
      }
      // queued on the pool's stream without waiting: the requests keep their
      // data and the pool stays busy until the solve has drained
      int rc = OSQP_OK;
      std::vector<osqp_int> idx;
      std::vector<std::shared_ptr<ServerReq>> reqs;
      for (auto &pr : kv.second) {
        const auto &rq = pr.first;
        if (rc == OSQP_OK)
          rc = update_vectors_impl(b, pr.second, rq->qp.q.data(), rq->qp.l.data(), rq->qp.u.data(),
                                   false);
        if (rc == OSQP_OK && (rq->qp.has_x || rq->qp.has_y))
          rc = warm_start_impl(b, pr.second, rq->qp.has_x ? rq->qp.xws.data() : nullptr,
                               rq->qp.has_y ? rq->qp.yws.data() : nullptr, false);
        idx.push_back(pr.second);
        reqs.push_back(rq);
      }
      if (rc == OSQP_OK) rc = osqp_batch_solve_subset_async(b, idx.data(), (osqp_int)idx.size());
      if (rc == OSQP_OK) {
        InFlight f;
        f.b = b; f.kind = 2; f.pool = kv.first; f.reqs = reqs;
        for (auto i : idx) f.idx.push_back(i);
        launched.push_back(std::move(f));
      } else {
        {
          std::lock_guard<std::mutex> g(sv->mu);
          sv->pools[kv.first].busy = false;
        }
        server_fail(sv, reqs, rc, 0);
      }
    }
    {
      std::lock_guard<std::mutex> g(sv->mu);
      sv->batches += (int64_t)launched.size();
      for (auto &f : launched) sv->inflight.push_back(std::move(f));
      sv->peak_inflight = std::max<int64_t>(sv->peak_inflight, (int64_t)sv->inflight.size());
    }
    // (3) nothing admitted and work on the device: poll again shortly
    if (launched.empty() && done.empty()) std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

}  // namespace

extern "C" {

osqp_int osqp_server_create(osqp_server **out, size_t hbm_budget_bytes, osqp_int max_slots,
                            const osqp_settings *s) {
  if (!out) return OSQP_ERR_NOT_SETUP;
  *out = nullptr;
  if (max_slots <= 0 || hbm_budget_bytes == 0) return OSQP_ERR_SETTINGS;
  osqp_settings st;
  if (s) st = *s; else osqp_set_default_settings(&st);
  int rc = check_settings(st);
  if (rc) return rc;
  if (st.stream) return OSQP_ERR_SETTINGS;   // every micro-batch owns its stream
  if (osqp_device_count() <= 0) return OSQP_ERR_NO_DEVICE;
  try {
    osqp_server *sv = new osqp_server();
    sv->set = st;
    sv->budget = hbm_budget_bytes;
    sv->max_slots = max_slots;
    sv->worker = std::thread(server_loop, sv);
    *out = sv;
  } catch (...) {
    return OSQP_ERR_ALLOC;
  }
  return OSQP_OK;
}

osqp_int osqp_server_submit(osqp_server *sv, const osqp_problem *p, uint64_t structure_key,
                            const osqp_float *x_ws, const osqp_float *y_ws, uint64_t *ticket) {
  if (!sv || !p || !ticket) return OSQP_ERR_NOT_SETUP;
  int rc = check_problem(*p);
  if (rc) return rc;
  try {
    auto rq = std::make_shared<ServerReq>();
    rq->qp.copy_from(*p, x_ws, y_ws);
    rq->key = structure_key;
    rq->bytes = estimate_bytes(*p, sv->set);
    rq->cost = 2 * (int64_t)p->A.nnz + 2 * (int64_t)p->P_upper.nnz + p->n + p->m;
    if (rq->bytes > sv->budget) return OSQP_ERR_BUDGET;
    rq->t_submit = now_s();
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->stop) return OSQP_ERR_NOT_SETUP;
    rq->ticket = sv->next_ticket++;
    *ticket = rq->ticket;
    sv->results[rq->ticket] = ServerResult();
    sv->queue.push_back(rq);
  } catch (...) {
    return OSQP_ERR_ALLOC;
  }
  sv->cv_work.notify_all();
  return OSQP_OK;
}

osqp_int osqp_server_wait(osqp_server *sv, uint64_t ticket, osqp_float *x, osqp_float *y,
                          osqp_info *info, double *latency_s) {
  if (!sv) return OSQP_ERR_NOT_SETUP;
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->results.find(ticket) == sv->results.end()) return OSQP_ERR_INDEX;
  // a ticket is collected once: a second waiter on it finds it gone
  sv->cv_done.wait(lk, [&] {
    auto f = sv->results.find(ticket);
    return f == sv->results.end() || f->second.done;
  });
  auto it = sv->results.find(ticket);
  if (it == sv->results.end()) return OSQP_ERR_INDEX;
  ServerResult r = std::move(it->second);
  sv->results.erase(it);
  lk.unlock();
  if (r.rc != OSQP_OK) return r.rc;
  if (x) std::memcpy(x, r.x.data(), sizeof(double) * r.x.size());
  if (y && !r.y.empty()) std::memcpy(y, r.y.data(), sizeof(double) * r.y.size());
  if (info) *info = r.info;
  if (latency_s) *latency_s = r.latency;
  return OSQP_OK;
}

osqp_int osqp_server_stats(const osqp_server *sv, int64_t *completed, int64_t *batches,
                           int64_t *peak_inflight, int64_t *peak_bytes) {
  if (!sv) return OSQP_ERR_NOT_SETUP;
  osqp_server *m = const_cast<osqp_server *>(sv);
  std::lock_guard<std::mutex> g(m->mu);
  if (completed) *completed = sv->completed;
  if (batches) *batches = sv->batches;
  if (peak_inflight) *peak_inflight = sv->peak_inflight;
  if (peak_bytes) *peak_bytes = sv->peak_bytes;
  return OSQP_OK;
}

void osqp_server_destroy(osqp_server *sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  for (auto &f : sv->inflight) {
    (void)osqp_batch_sync(f.b);
    if (f.kind != 2) osqp_batch_cleanup(f.b);   // pools are freed below
  }
  for (auto &kv : sv->pools)
    if (kv.second.b) osqp_batch_cleanup(kv.second.b);
  delete sv;
}

}  // extern "C"
