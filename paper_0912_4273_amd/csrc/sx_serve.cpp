// sx_serve.cpp -- request loop with continuous batching over one context.
//
// Requests (a grid, its physics and a sweep count) arrive at any time from
// any thread.  Worker threads run the host part of the upload
// (sx_grid_prepare) while the GPU sweeps.  One scheduler thread owns the
// context.  It keeps one round in flight: a round is up to round_sweeps
// sweeps over every resident grid as a single batch (each grid runs only the
// sweeps it still needs), enqueued without waiting.  While it runs, the
// scheduler admits prepared requests in arrival order as the HBM budget and
// the active-grid limit allow (sx_grid_commit), and reads back and releases
// the grids the previous round finished; these go on the context's second
// stream, so the GPU keeps sweeping.  When the round ends, the next one is
// enqueued at once over the grids still resident and those just admitted.
// A grid's result does not depend on what it was batched with (each tile's
// arithmetic is independent of the tile list), so it equals the result of
// solving it alone.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "sx.h"
#include "sx_internal.h"

namespace {

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// A deep copy of a grid description.
struct OwnedDesc {
  sx_grid_desc d{};
  std::vector<double> pos, n_H, volume, dL, x_init, bin_dirs, src_rate, src_dir;
  std::vector<int64_t> nbr_ptr;
  std::vector<int32_t> nbr_idx, src_vertex;

  int copy_from(const sx_grid_desc *s) {
    if (!s || s->n_vertices < 1 || !s->pos || !s->nbr_ptr || !s->nbr_idx || !s->n_H ||
        !s->volume || s->n_bins < 1 || !s->bin_dirs || s->n_src < 0 ||
        (s->n_src > 0 && (!s->src_vertex || !s->src_rate)))
      return SX_EINVAL;
    const int64_t n = s->n_vertices;
    const int64_t e = s->nbr_ptr[n];
    if (e < 0) return SX_EINVAL;
    d = *s;
    pos.assign(s->pos, s->pos + 3 * n);
    nbr_ptr.assign(s->nbr_ptr, s->nbr_ptr + n + 1);
    nbr_idx.assign(s->nbr_idx, s->nbr_idx + e);
    n_H.assign(s->n_H, s->n_H + n);
    volume.assign(s->volume, s->volume + n);
    if (s->dL) dL.assign(s->dL, s->dL + n);
    if (s->x_init) x_init.assign(s->x_init, s->x_init + n);
    bin_dirs.assign(s->bin_dirs, s->bin_dirs + 3 * (int64_t)s->n_bins);
    src_vertex.assign(s->src_vertex, s->src_vertex + s->n_src);
    src_rate.assign(s->src_rate, s->src_rate + s->n_src);
    if (s->src_dir) src_dir.assign(s->src_dir, s->src_dir + 3 * (int64_t)s->n_src);
    d.pos = pos.data();
    d.nbr_ptr = nbr_ptr.data();
    d.nbr_idx = nbr_idx.data();
    d.n_H = n_H.data();
    d.volume = volume.data();
    d.dL = s->dL ? dL.data() : nullptr;
    d.x_init = s->x_init ? x_init.data() : nullptr;
    d.bin_dirs = bin_dirs.data();
    d.src_vertex = src_vertex.data();
    d.src_rate = src_rate.data();
    d.src_dir = s->src_dir ? src_dir.data() : nullptr;
    return SX_OK;
  }
};

struct Req {
  int64_t ticket = 0;
  OwnedDesc desc;
  int32_t sweeps = 0;
  int32_t left = 0;
  int status = SX_OK;
  sx_prepared *prep = nullptr;
  sx_grid_id gid = 0;
  double t_submit = 0, t_prepared = 0, t_admit = 0, t_done = 0;
  std::vector<double> x, y;
  sx_tally tally{};
  int64_t n = 0;
  int32_t k = 0;
};

}  // namespace

struct sx_server {
  sx_ctx *ctx = nullptr;
  sx_serve_opts opts{};
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_prep, cv_sched, cv_done;
  std::deque<Req *> submitted, ready, done;
  std::map<int64_t, Req *> taken;   // polled, waiting for sx_serve_take
  int in_prep = 0;
  int64_t next_ticket = 1;
  bool stopping = false;
  std::vector<std::thread> workers;
  std::thread sched;
  // statistics
  int64_t rounds = 0, finished = 0, failed = 0;
  double updates = 0.0, t_first = -1.0, t_last = 0.0, gpu_s = 0.0;
  int32_t peak_active = 0;
  std::vector<double> latency;
  std::string err;
};

namespace {

void finish(sx_server *s, Req *r, int status) {
  // with s->mu held
  r->status = status;
  r->t_done = now_s(s->t0);
  if (r->prep) {
    sx_prepared_free(r->prep);
    r->prep = nullptr;
  }
  if (status == SX_OK) {
    s->finished++;
    s->updates += (double)r->n * r->k * r->sweeps;
    s->latency.push_back(r->t_done - r->t_submit);
  } else {
    s->failed++;
  }
  s->t_last = std::max(s->t_last, r->t_done);
  s->done.push_back(r);
  s->cv_done.notify_all();
}

void worker(sx_server *s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_prep.wait(lk, [&] { return s->stopping || !s->submitted.empty(); });
    if (s->submitted.empty()) return;   // stopping and nothing left
    Req *r = s->submitted.front();
    s->submitted.pop_front();
    s->in_prep++;
    lk.unlock();
    char msg[256] = {0};
    sx_prepared *p = nullptr;
    const int rc = sx_grid_prepare(&r->desc.d, &p, msg, sizeof msg);
    lk.lock();
    s->in_prep--;
    if (rc) {
      finish(s, r, rc);
    } else {
      r->prep = p;
      r->t_prepared = now_s(s->t0);
      s->ready.push_back(r);
    }
    s->cv_sched.notify_all();
  }
}

void scheduler(sx_server *s) {
  // active: resident grids; the running round is over `running`.  Uploads
  // (admission), read-backs and releases go on the context's second stream,
  // so that they overlap the round the GPU is running.
  std::vector<Req *> active, running;
  std::vector<int32_t> run_cnt;
  std::vector<sx_grid_id> ids;
  bool round_on = false;
  auto t_round = std::chrono::steady_clock::now();
  std::unique_lock<std::mutex> lk(s->mu);
  bool dead = false;   // the context failed: finish everything with its error
  sx::set_io_stream(s->ctx, true);
  for (;;) {
    // ---- admission, in arrival order (while a round runs, if one does)
    while (!s->ready.empty() && (int32_t)active.size() < s->opts.max_active) {
      Req *r = s->ready.front();
      if (dead) {
        s->ready.pop_front();
        finish(s, r, SX_EDEVICE);
        continue;
      }
      uint64_t need = 0;
      sx_prepared_bytes(r->prep, &need);
      uint64_t used = 0, budget = 0;
      sx_mem_info(s->ctx, &used, &budget);
      const uint64_t cap = s->opts.hbm_budget ? std::min<uint64_t>(s->opts.hbm_budget, budget)
                                              : budget;
      if (used + need > cap && !active.empty()) break;   // wait for retirements
      lk.unlock();
      sx_grid_id gid = 0;
      const int rc = sx_grid_commit(s->ctx, r->prep, &gid);
      lk.lock();
      uint64_t still = 0;
      if (rc == SX_ENOMEM && !active.empty() && sx_prepared_bytes(r->prep, &still) == SX_OK)
        break;   // not admitted; retried after the next retirements
      s->ready.pop_front();
      if (rc) {
        if (rc == SX_EDEVICE) dead = true;
        finish(s, r, rc);
        continue;
      }
      sx_prepared_free(r->prep);
      r->prep = nullptr;
      r->gid = gid;
      r->left = r->sweeps;
      r->n = r->desc.d.n_vertices;
      r->k = r->desc.d.n_bins;
      r->t_admit = now_s(s->t0);
      if (s->t_first < 0) s->t_first = r->t_admit;
      active.push_back(r);
    }
    s->peak_active = std::max(s->peak_active, (int32_t)active.size());
    if (!round_on && active.empty()) {
      if (s->stopping && s->submitted.empty() && s->ready.empty() && s->in_prep == 0) break;
      s->cv_sched.wait(lk);
      continue;
    }
    // ---- the end of the running round: what is done retires
    std::vector<Req *> retire;
    int rc = SX_OK;
    if (round_on) {
      lk.unlock();
      rc = sx::wait_sweeps(s->ctx);
      const double round_s =
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t_round).count();
      lk.lock();
      round_on = false;
      s->rounds++;
      s->gpu_s += round_s;
      if (rc) dead = true;
      for (size_t i = 0; i < running.size(); ++i) {
        Req *r = running[i];
        if (!rc) r->left -= run_cnt[i];
        if (rc || r->left <= 0) retire.push_back(r);
      }
      running.clear();
      std::vector<Req *> keep;
      for (Req *r : active)
        if (std::find(retire.begin(), retire.end(), r) == retire.end()) keep.push_back(r);
      active.swap(keep);
    }
    if (dead) {
      for (Req *r : active) retire.push_back(r);
      active.clear();
    }
    // ---- the next round over every resident grid, enqueued at once
    if (!active.empty()) {
      ids.clear();
      run_cnt.clear();
      for (Req *r : active) {
        ids.push_back(r->gid);
        run_cnt.push_back(std::min(r->left, s->opts.round_sweeps));
      }
      running = active;
      lk.unlock();
      t_round = std::chrono::steady_clock::now();
      const int lr = sx::solve_launch(s->ctx, ids.data(), (int32_t)ids.size(), run_cnt.data());
      lk.lock();
      if (lr) {
        dead = true;
        rc = lr;
        for (Req *r : active) retire.push_back(r);
        active.clear();
        running.clear();
      } else {
        round_on = true;
      }
    }
    // ---- read back and release the retired grids while that round runs
    std::vector<std::pair<Req *, int>> out;
    lk.unlock();
    for (Req *r : retire) {
      if (dead) {
        (void)sx_grid_free(s->ctx, r->gid);
        out.push_back({r, rc ? rc : SX_EDEVICE});
        continue;
      }
      r->x.resize((size_t)r->n);
      r->y.resize((size_t)r->n);
      sx_state_out so{};
      so.x = r->x.data();
      so.y = r->y.data();
      so.tally = &r->tally;
      int rr = sx_read_state(s->ctx, r->gid, &so);
      const int fr = sx_grid_free(s->ctx, r->gid);
      out.push_back({r, rr ? rr : fr});
    }
    lk.lock();
    for (auto &o : out) finish(s, o.first, o.second);
  }
  sx::set_io_stream(s->ctx, false);
}

}  // namespace

extern "C" {

int sx_serve_start(sx_ctx *ctx, const sx_serve_opts *opts, sx_server **out) {
  if (!ctx || !out) return SX_EINVAL;
  *out = nullptr;
  sx_serve_opts o{};
  if (opts) o = *opts;
  if (o.round_sweeps == 0) o.round_sweeps = 50;
  if (o.max_active == 0) o.max_active = 64;
  if (o.prep_threads == 0) o.prep_threads = 4;
  if (o.round_sweeps < 1 || o.max_active < 1 || o.max_active > 1024 || o.prep_threads < 1 ||
      o.prep_threads > 64)
    return SX_EINVAL;
  sx_server *s = new sx_server();
  s->ctx = ctx;
  s->opts = o;
  s->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < o.prep_threads; ++i) s->workers.emplace_back(worker, s);
  s->sched = std::thread(scheduler, s);
  *out = s;
  return SX_OK;
}

int sx_serve_submit(sx_server *s, const sx_grid_desc *d, int32_t n_sweeps, int64_t *ticket) {
  if (!s || !ticket || n_sweeps < 0) return SX_EINVAL;
  Req *r = new Req();
  if (r->desc.copy_from(d) != SX_OK) {
    delete r;
    return SX_EINVAL;
  }
  r->sweeps = n_sweeps;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) {
    delete r;
    return SX_EINVAL;
  }
  r->ticket = s->next_ticket++;
  r->t_submit = now_s(s->t0);
  *ticket = r->ticket;
  s->submitted.push_back(r);
  s->cv_prep.notify_one();
  return SX_OK;
}

int sx_serve_poll(sx_server *s, double timeout_s, sx_serve_result *res) {
  if (!s || !res) return SX_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  const auto until = std::chrono::steady_clock::now() +
                     std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                         std::chrono::duration<double>(std::max(timeout_s, 0.0)));
  if (!s->cv_done.wait_until(lk, until, [&] { return !s->done.empty(); })) return SX_EAGAIN;
  Req *r = s->done.front();
  s->done.pop_front();
  std::memset(res, 0, sizeof *res);
  res->ticket = r->ticket;
  res->status = r->status;
  res->n_vertices = r->desc.d.n_vertices;
  res->n_bins = r->desc.d.n_bins;
  res->n_sweeps = r->sweeps;
  res->t_submit = r->t_submit;
  res->t_prepared = r->t_prepared;
  res->t_admit = r->t_admit;
  res->t_done = r->t_done;
  res->tally = r->tally;
  s->taken[r->ticket] = r;
  return SX_OK;
}

int sx_serve_take(sx_server *s, int64_t ticket, double *x, double *y) {
  if (!s) return SX_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->taken.find(ticket);
  if (it == s->taken.end()) return SX_ENOTFOUND;
  Req *r = it->second;
  if (r->status == SX_OK) {
    if (x) std::copy(r->x.begin(), r->x.end(), x);
    if (y) std::copy(r->y.begin(), r->y.end(), y);
  }
  s->taken.erase(it);
  delete r;
  return SX_OK;
}

int sx_serve_stop(sx_server *s, sx_serve_stats *st) {
  if (!s) return SX_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv_prep.notify_all();
  s->cv_sched.notify_all();
  for (auto &t : s->workers) t.join();
  {
    // workers are gone: the scheduler drains what is prepared or resident
    std::lock_guard<std::mutex> lk(s->mu);
    s->cv_sched.notify_all();
  }
  s->sched.join();
  if (st) {
    std::memset(st, 0, sizeof *st);
    st->finished = s->finished;
    st->failed = s->failed;
    st->rounds = s->rounds;
    st->peak_active = s->peak_active;
    st->updates = s->updates;
    st->span_s = s->t_first >= 0 ? s->t_last - s->t_first : 0.0;
    st->round_s = s->gpu_s;
    std::vector<double> l = s->latency;
    std::sort(l.begin(), l.end());
    auto q = [&](double f) {
      if (l.empty()) return 0.0;
      const size_t i = (size_t)std::min<double>((double)l.size() - 1.0,
                                                std::ceil(f * (double)l.size()) - 1.0);
      return l[i];
    };
    st->latency_p50_s = q(0.50);
    st->latency_p99_s = q(0.99);
    st->latency_max_s = l.empty() ? 0.0 : l.back();
  }
  for (Req *r : s->done) delete r;
  for (auto &kv : s->taken) delete kv.second;
  delete s;
  return SX_OK;
}

}  // extern "C"
