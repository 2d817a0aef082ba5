// Serving loop over the SGF C ABI: continuous batching of factorize / solve
// requests of many operators on one GPU.
//
// * Every operator (a matrix pattern + values + options) keeps its analysis
//   for the server's lifetime; its factor lives on the device while memory
//   allows and is evicted least-recently-used when the HBM budget would be
//   exceeded (the analysis stays, so an evicted operator is refactorized on
//   its next request).
// * `slots` worker threads, each with its own HIP stream (default priority),
//   take requests as soon as a slot and the memory for them are free, so the
//   work of different operators overlaps on the device.
// * Solve requests for the same operator that are waiting together are
//   coalesced into one multi-right-hand-side PCG (the factor is read once
//   per group of columns); each column's arithmetic is independent of the
//   others', so a result does not depend on what it was batched with.
// * Admission: a request is started only when the bytes its operator holds
//   or needs (sgf_estimate_bytes, an upper bound from the plan) fit in the
//   budget beside everything else held or reserved; requests that do not fit
//   wait while later ones that fit go ahead.  (Each slot also keeps the
//   gather / scatter buffers of its largest batch, outside the budget.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <ctime>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "sgf.h"

namespace {

// Seconds on the monotonic clock (the clock of Python's time.monotonic).
double now_s() {
  timespec t;
  clock_gettime(CLOCK_MONOTONIC, &t);
  return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

struct Op {
  int id = 0;                 // index in the server's operator list
  sgf_handle h = nullptr;     // created by the first worker that needs it
  int64_t n = 0, nnz = 0;
  std::vector<double> vals;   // host copy of the values, for (re)factorization
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> col_idx;
  std::vector<double> coords;
  sgf_options opt{};
  sgf_status analysis = SGF_OK;
  bool busy = false;          // a slot is working on it
  bool factored = false;      // factor resident on the device
  int64_t held = 0;           // device bytes it holds (0 when evicted)
  int64_t est1 = 0;           // bound on the bytes to factorize + solve one column
  int64_t per_rhs = 0;        // bytes per additional column
  double last_use = 0;
};

struct Req {
  int64_t ticket = 0;
  int32_t op = 0;
  int32_t refactor = 0;
  int32_t nrhs = 0;
  const double* b = nullptr;
  int64_t ldb = 0;
  double* x = nullptr;
  int64_t ldx = 0;
  double rtol = 0;
  int32_t maxit = 0;
  sgf_request_info info{};
  std::vector<int32_t> iters;
  std::vector<double> relres;
  bool done = false;
};

}  // namespace

struct sgf_server_s {
  sgf_server_options opt{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<std::thread> workers;
  bool stop = false;
  bool trace = std::getenv("SGF_SERVER_TRACE") != nullptr;   // bookkeeping lines on stderr
  std::vector<std::unique_ptr<Op>> ops;
  std::deque<std::shared_ptr<Req>> queue;
  std::map<int64_t, std::shared_ptr<Req>> all;
  int64_t next_ticket = 1;
  int64_t held = 0, reserved = 0, peak = 0;
  int64_t evictions = 0, factorizations = 0, batches = 0;

  // Bytes held plus reserved, after evicting idle factors (LRU) until `need`
  // more fits; false if it cannot fit now.  The operator being admitted
  // (`self`) is never the victim: its need was computed with its factor
  // resident.
  bool admit(int64_t need, const Op* self) {
    while (held + reserved + need > opt.hbm_budget) {
      Op* victim = nullptr;
      for (auto& o : ops)
        if (o.get() != self && !o->busy && o->factored && (!victim || o->last_use < victim->last_use))
          victim = o.get();
      if (!victim) return false;
      sgf_release(victim->h);
      held -= victim->held;
      victim->held = 0;
      victim->factored = false;
      ++evictions;
    }
    return true;
  }

  void run(int slot);
};

void sgf_server_s::run(int slot) {
  hipStream_t st = nullptr;
  (void)hipSetDevice(0);
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
  double* B = nullptr;
  double* X = nullptr;
  size_t cap = 0;
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // pick the first waiting request whose operator is free and whose memory fits
    std::vector<std::shared_ptr<Req>> batch;
    Op* op = nullptr;
    int64_t need = 0;
    bool factor = false;
    for (;;) {
      if (stop && queue.empty()) {
        lk.unlock();
        if (B) (void)hipFree(B);
        if (X) (void)hipFree(X);
        (void)hipStreamDestroy(st);
        return;
      }
      for (auto it = queue.begin(); it != queue.end(); ++it) {
        Op* o = ops[(*it)->op].get();
        if (o->busy) continue;
        const auto& r = *it;
        if (!o->h && o->analysis == SGF_OK) {
          // symbolic analysis (host only) of a new operator, outside the lock
          o->busy = true;
          lk.unlock();
          sgf_handle h = nullptr;
          sgf_status a = sgf_analyze(o->n, o->row_ptr.data(), o->col_idx.data(), o->coords.data(), &o->opt, &h);
          int64_t e1 = 0, e2 = 0;
          if (a == SGF_OK && ((a = sgf_estimate_bytes(h, 1, &e1)) != SGF_OK || (a = sgf_estimate_bytes(h, 2, &e2)) != SGF_OK)) {
            sgf_destroy(h);
            h = nullptr;
          }
          lk.lock();
          o->busy = false;
          o->analysis = a;
          if (a == SGF_OK) {
            o->h = h;
            o->est1 = e1;
            o->per_rhs = std::max<int64_t>(e2 - e1, 0);
            o->row_ptr = {};
            o->col_idx = {};
            o->coords = {};
          }
          cv_work.notify_all();
          goto rescan;
        }
        if (o->analysis != SGF_OK) {
          r->info.status = o->analysis;
          r->info.t_start = r->info.t_end = now_s();
          r->done = true;
          queue.erase(it);
          cv_done.notify_all();
          goto rescan;
        }
        const bool f = r->refactor || !o->factored;
        // the batch: this request and the following solves of the same
        // operator (up to the next refactorization), max_batch_rhs columns
        std::vector<std::shared_ptr<Req>> cand{r};
        int tot = r->nrhs;
        for (auto jt = std::next(it); jt != queue.end(); ++jt) {
          const auto& q = *jt;
          if (q->op != r->op) continue;
          if (q->refactor) break;
          if (q->rtol != r->rtol || q->maxit != r->maxit) continue;
          if (tot + q->nrhs > opt.max_batch_rhs) break;
          cand.push_back(q);
          tot += q->nrhs;
        }
        const int64_t est = o->factored ? o->held + tot * o->per_rhs : o->est1 + (tot - 1) * o->per_rhs;
        const int64_t batch_bytes = (int64_t)2 * o->n * tot * (int64_t)sizeof(double);
        const int64_t grow = std::max<int64_t>(0, est - o->held) + batch_bytes;
        if (est > opt.hbm_budget) {
          // can never fit: fail the request now
          r->info.status = SGF_ENOMEM;
          r->info.t_start = r->info.t_end = now_s();
          r->done = true;
          queue.erase(it);
          cv_done.notify_all();
          goto rescan;
        }
        if (!admit(grow, o)) continue;
        for (const auto& q : cand) queue.erase(std::find(queue.begin(), queue.end(), q));
        batch = std::move(cand);
        op = o;
        need = grow;
        factor = f;
        break;
      }
      if (op) break;
      if (!queue.empty() && reserved == 0 &&
          std::none_of(ops.begin(), ops.end(), [](const std::unique_ptr<Op>& o) { return o->busy; })) {
        // nothing runs and nothing fits even after evicting every idle
        // factor: the head request cannot be served
        auto r = queue.front();
        queue.pop_front();
        r->info.status = SGF_ENOMEM;
        r->info.t_start = r->info.t_end = now_s();
        r->done = true;
        cv_done.notify_all();
        continue;
      }
      cv_work.wait(lk);
    rescan:;
    }
    op->busy = true;
    reserved += need;
    int tot = 0;
    for (auto& r : batch) tot += r->nrhs;
    const double ts = now_s();
    for (auto& r : batch) r->info.t_start = ts;
    lk.unlock();

    // ---- the work, outside the lock -------------------------------------
    sgf_status status = SGF_OK;
    double t_fac = 0;
    std::vector<int32_t> iters(tot, 0);
    std::vector<double> relres(tot, 0.0);
    if (factor) {
      const double a = now_s();
      status = sgf_factorize_numeric(op->h, op->vals.data(), st);
      if (status == SGF_OK && hipStreamSynchronize(st) != hipSuccess) status = SGF_EDEVICE;
      t_fac = now_s() - a;
    }
    if (status == SGF_OK) {
      const size_t want = (size_t)op->n * tot;
      if (want > cap) {
        if (B) (void)hipFree(B);
        if (X) (void)hipFree(X);
        B = X = nullptr;
        cap = 0;
        if (hipMalloc(&B, want * sizeof(double)) != hipSuccess || hipMalloc(&X, want * sizeof(double)) != hipSuccess)
          status = SGF_ENOMEM;
        else
          cap = want;
      }
    }
    if (status == SGF_OK) {
      int64_t col = 0;
      for (auto& r : batch) {
        if (hipMemcpy2DAsync(B + col * op->n, op->n * sizeof(double), r->b, r->ldb * sizeof(double),
                             op->n * sizeof(double), r->nrhs, hipMemcpyDeviceToDevice, st) != hipSuccess)
          status = SGF_EDEVICE;
        col += r->nrhs;
      }
      if (status == SGF_OK)
        status = sgf_pcg_solve(op->h, tot, B, op->n, X, op->n, batch[0]->rtol, batch[0]->maxit, iters.data(),
                               relres.data(), st);
      if (status == SGF_OK || status == SGF_ENOCONV) {
        col = 0;
        for (auto& r : batch) {
          if (hipMemcpy2DAsync(r->x, r->ldx * sizeof(double), X + col * op->n, op->n * sizeof(double),
                               op->n * sizeof(double), r->nrhs, hipMemcpyDeviceToDevice, st) != hipSuccess)
            status = SGF_EDEVICE;
          col += r->nrhs;
        }
      }
      if (hipStreamSynchronize(st) != hipSuccess) status = SGF_EDEVICE;
    }
    sgf_info inf{};
    sgf_get_info(op->h, &inf);

    // ---- bookkeeping -------------------------------------------------------
    lk.lock();
    if (trace)
      std::fprintf(stderr, "[sgf-server] slot %d op %d cols %d factor %d need %lld held %lld -> %lld total %lld reserved %lld\n",
                   slot, op->id, tot, (int)factor, (long long)need, (long long)op->held, (long long)inf.device_bytes,
                   (long long)(held + inf.device_bytes - op->held), (long long)(reserved - need));
    reserved -= need;
    held += inf.device_bytes - op->held;
    op->held = inf.device_bytes;
    peak = std::max(peak, held + reserved);
    if (factor) {
      ++factorizations;
      op->factored = status == SGF_OK || status == SGF_ENOCONV;
    }
    op->busy = false;
    op->last_use = now_s();
    ++batches;
    const double te = now_s();
    int64_t col = 0;
    for (auto& r : batch) {
      r->info.status = status;
      r->info.t_end = te;
      r->info.t_factor = t_fac;
      r->info.factorized = factor ? 1 : 0;
      r->info.batch_rhs = tot;
      r->info.slot = slot;
      r->info.iters_max = 0;
      r->info.relres_max = 0;
      for (int c = 0; c < r->nrhs; ++c) {
        r->iters[c] = iters[col + c];
        r->relres[c] = relres[col + c];
        r->info.iters_max = std::max(r->info.iters_max, iters[col + c]);
        r->info.relres_max = std::max(r->info.relres_max, relres[col + c]);
      }
      col += r->nrhs;
      r->done = true;
    }
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

extern "C" {

void sgf_server_default_options(sgf_server_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->hbm_budget = (int64_t)200 << 30;
  o->slots = 4;
  o->max_batch_rhs = 16;
}

sgf_status sgf_server_create(const sgf_server_options* o, sgf_server* out) {
  if (!o || !out || o->slots < 1 || o->slots > 16 || o->hbm_budget <= 0 || o->max_batch_rhs < 1 ||
      o->max_batch_rhs > 256)
    return SGF_EINVAL;
  auto* s = new (std::nothrow) sgf_server_s();
  if (!s) return SGF_ENOMEM;
  s->opt = *o;
  for (int i = 0; i < o->slots; ++i) s->workers.emplace_back([s, i] { s->run(i); });
  *out = s;
  return SGF_OK;
}

sgf_status sgf_server_add_operator(sgf_server s, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                                   const double* vals, const double* coords, const sgf_options* opt,
                                   int32_t* op_id) {
  if (!s || !vals || !op_id || !row_ptr || !col_idx || !coords || !opt || n < 1 || opt->dofs_per_node < 1)
    return SGF_EINVAL;
  auto op = std::make_unique<Op>();
  op->n = n;
  op->nnz = row_ptr[n];
  op->vals.assign(vals, vals + op->nnz);
  op->row_ptr.assign(row_ptr, row_ptr + n + 1);
  op->col_idx.assign(col_idx, col_idx + op->nnz);
  op->coords.assign(coords, coords + (n / opt->dofs_per_node) * opt->dim);
  op->opt = *opt;
  std::lock_guard<std::mutex> g(s->mu);
  *op_id = (int32_t)s->ops.size();
  op->id = (int)s->ops.size();
  s->ops.push_back(std::move(op));
  return SGF_OK;
}

sgf_status sgf_server_submit(sgf_server s, int32_t op_id, int32_t refactor, int32_t nrhs, const double* b,
                             int64_t ldb, double* x, int64_t ldx, double rtol, int32_t maxit, int64_t* ticket) {
  if (!s || !b || !x || !ticket || nrhs < 1 || maxit < 0) return SGF_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  if (s->stop) return SGF_ESTATE;
  if (op_id < 0 || op_id >= (int32_t)s->ops.size()) return SGF_EINVAL;
  Op* o = s->ops[op_id].get();
  if (ldb < o->n || ldx < o->n || nrhs > s->opt.max_batch_rhs) return SGF_EINVAL;
  auto r = std::make_shared<Req>();
  r->ticket = s->next_ticket++;
  r->op = op_id;
  r->refactor = refactor != 0;
  r->nrhs = nrhs;
  r->b = b;
  r->ldb = ldb;
  r->x = x;
  r->ldx = ldx;
  r->rtol = rtol;
  r->maxit = maxit;
  r->iters.assign(nrhs, 0);
  r->relres.assign(nrhs, 0.0);
  r->info.ticket = r->ticket;
  r->info.op = op_id;
  r->info.nrhs = nrhs;
  r->info.t_submit = now_s();
  s->queue.push_back(r);
  s->all[r->ticket] = r;
  *ticket = r->ticket;
  s->cv_work.notify_all();
  return SGF_OK;
}

sgf_status sgf_server_wait(sgf_server s, int64_t ticket, sgf_request_info* info, int32_t* iters, double* relres) {
  if (!s) return SGF_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return SGF_EINVAL;
  auto r = it->second;
  s->cv_done.wait(lk, [&] { return r->done; });
  if (info) *info = r->info;
  if (iters) std::copy(r->iters.begin(), r->iters.end(), iters);
  if (relres) std::copy(r->relres.begin(), r->relres.end(), relres);
  s->all.erase(it);
  return SGF_OK;
}

double sgf_server_clock(void) { return now_s(); }

sgf_status sgf_server_get_stats(sgf_server s, sgf_server_stats* out) {
  if (!s || !out) return SGF_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  out->held_bytes = s->held;
  out->peak_bytes = s->peak;
  out->evictions = s->evictions;
  out->factorizations = s->factorizations;
  out->batches = s->batches;
  out->queued = (int64_t)s->queue.size();
  int64_t cached = 0;
  for (auto& o : s->ops) cached += o->factored;
  out->cached_operators = cached;
  return SGF_OK;
}

sgf_status sgf_server_destroy(sgf_server s) {
  if (!s) return SGF_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto& o : s->ops)
    if (o->h) sgf_destroy(o->h);
  delete s;
  return SGF_OK;
}

}  // extern "C"
