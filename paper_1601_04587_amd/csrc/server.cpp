// Serving loop: continuous batching of domain-solve requests.
//
// A host thread owns the engine while requests are in flight.  Each round it
// (1) admits queued requests whose device footprint fits the HBM budget and
// whose runner has a free slot (gauge fields and operator blocks stay
// resident and are shared), (2) runs one scheduling round of the batched
// solver (one graph replay per runner, holding the FP64 outer step and K
// inner iterations of every slot; the host reads the slot phases one replay
// behind), and (3) retires the solves the device has finished: their
// solutions are scattered on the stream and the requests complete when an
// event after the scatter has passed, without draining the stream.  A
// request that arrives while others are on the GPU joins the batch at the
// next round, so its work overlaps theirs.  Per-request arithmetic does not
// depend on the batch: the kernels reduce in a fixed order per solve and a
// solve's iterations are independent of its neighbours in the slot table.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <set>

#include "engine.hpp"
#include "server.hpp"

namespace ddml {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

Server::Server(Ctx* c, const ddml_solver_params& p, int mq) : ctx(c), prm(p), max_queue(mq) {
  th = std::thread([this] { loop(); });
}

Server::~Server() {
  {
    std::lock_guard<std::mutex> lk(m);
    stop = true;
  }
  cv.notify_all();
  if (th.joinable()) th.join();
}

int Server::enqueue(std::unique_ptr<Req> q, uint64_t* ticket) {
  std::lock_guard<std::mutex> lk(m);
  if ((int)(incoming.size() + waiting_count) >= max_queue) return DDML_EAGAIN;
  q->ticket = next_ticket++;
  q->res.status = DDML_EAGAIN;
  q->res.arrival_time = q->r.arrival_time;
  q->left = q->levels();
  q->solves.resize(q->levels());
  q->info.assign((size_t)q->levels() * q->r.nrhs, ddml_rhs_info{});
  *ticket = q->ticket;
  incoming.push_back(q.get());
  first_arrival = std::min(first_arrival, q->r.arrival_time);
  reqs[q->ticket] = std::move(q);
  submitted++;
  cv.notify_all();
  return DDML_OK;
}

int Server::submit(const ddml_request& r, uint64_t* ticket) {
  auto q = std::make_unique<Req>();
  q->r = r;
  return enqueue(std::move(q), ticket);
}

int Server::submit_series(const ddml_series_request& r, uint64_t* ticket) {
  auto q = std::make_unique<Req>();
  q->r.gauge_id = r.gauge_id;
  q->r.dom_id = r.dom_ids[0];
  q->r.src = r.src;
  q->r.sol = nullptr;
  q->r.nrhs = r.nrhs;
  q->r.arrival_time = r.arrival_time;
  q->doms.assign(r.dom_ids, r.dom_ids + r.nlevels);
  q->terms = r.terms;
  q->sum = r.sum;
  q->user_info = r.info;
  return enqueue(std::move(q), ticket);
}

int Server::poll(uint64_t t, ddml_result* res) {
  std::lock_guard<std::mutex> lk(m);
  auto it = reqs.find(t);
  if (it == reqs.end()) return DDML_EINVAL;
  if (!it->second->done) return DDML_EAGAIN;
  if (res) *res = it->second->res;
  return DDML_OK;
}

int Server::wait(uint64_t t, ddml_result* res, double timeout) {
  std::unique_lock<std::mutex> lk(m);
  auto it = reqs.find(t);
  if (it == reqs.end()) return DDML_EINVAL;
  Req* q = it->second.get();
  auto pred = [&] { return q->done; };
  if (timeout < 0) cv_done.wait(lk, pred);
  else if (!cv_done.wait_for(lk, std::chrono::duration<double>(timeout), pred)) return DDML_EAGAIN;
  if (res) *res = q->res;
  return DDML_OK;
}

void Server::stats(ddml_server_stats* s) {
  std::lock_guard<std::mutex> lk(m);
  s->submitted = submitted;
  s->completed = completed;
  s->queued = (long)(incoming.size() + waiting_count);
  s->in_flight = in_flight;
  std::vector<double> l = latencies;
  std::sort(l.begin(), l.end());
  auto pct = [&](double q) {
    if (l.empty()) return 0.0;
    size_t k = (size_t)std::ceil(q * l.size()) - 1;
    return l[std::min(k, l.size() - 1)];
  };
  s->p50_latency = pct(0.5);
  s->p99_latency = pct(0.99);
  double sum = 0;
  for (double v : l) sum += v;
  s->mean_latency = l.empty() ? 0 : sum / l.size();
  s->solves_per_s = (completed > 0 && last_finish > first_arrival) ? completed / (last_finish - first_arrival) : 0;
  s->hbm_in_use = ctx->pool->in_use();
  s->hbm_budget = ctx->pool->budget();
}

// Checks a request's buffers (and, for a series, its domains) once the gauge
// field's volume is known; throws Error{EINVAL}.
static void check_request(Ctx* ctx, const Req* q) {
  const size_t bytes = (size_t)q->r.nrhs * gauge_get(ctx, q->r.gauge_id).V * 12 * sizeof(double2);
  bool ok = device_span_ok(q->r.src, bytes, ctx->device);
  if (q->series()) {
    for (int d : q->doms)
      if (d != -1) (void)domain_get(ctx, d);
    ok = ok && device_span_ok(q->terms, bytes * q->doms.size(), ctx->device);
    if (q->sum) ok = ok && device_span_ok(q->sum, bytes, ctx->device);
  } else {
    ok = ok && device_span_ok(q->r.sol, bytes, ctx->device);
  }
  if (!ok) throw Error{DDML_EINVAL, "request buffers do not hold its canonical fields in device memory"};
}

void Server::loop() {
  struct Unit {
    Req* q;
    int lev;
  };
  std::deque<Unit> waiting;
  std::vector<Solve*> live;
  std::map<Solve*, Req*> owner;
  // requests whose last solve (and series difference) is still on the stream
  std::deque<std::pair<hipEvent_t, std::vector<Req*>>> landing;
  std::vector<hipEvent_t> spare;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(m);
      if (live.empty() && waiting.empty() && incoming.empty() && landing.empty()) {
        if (stop) break;
        cv.wait_for(lk, std::chrono::milliseconds(2));
      }
      while (!incoming.empty()) {
        Req* q = incoming.front();
        for (int l = 0; l < q->levels(); ++l) waiting.push_back(Unit{q, l});
        incoming.pop_front();
      }
      waiting_count = waiting.size();
      if (stop && live.empty() && waiting.empty() && landing.empty()) break;
    }
    if (live.empty() && waiting.empty() && landing.empty()) continue;
    std::vector<Req*> finished;   // requests that never reached the GPU
    std::vector<Req*> retired;    // requests whose last solve finished this round
    {
      // API calls of other threads (e.g. the sampler's gauge updates and
      // contractions) go first; the queued replays keep the GPU busy meanwhile
      while (ctx->api_waiting.load() > 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
      std::lock_guard<std::recursive_mutex> g(ctx->mu);
      // a level that will not run: the request fails, and completes once its
      // levels in flight have finished
      auto drop = [&](Req* q, int code) {
        if (q->res.status == DDML_EAGAIN) q->res.status = code;
        if (--q->left == 0) finished.push_back(q);
      };
      // admission by device footprint and free slots
      while (!waiting.empty()) {
        const Unit u = waiting.front();
        Req* q = u.q;
        if (q->res.status != DDML_EAGAIN) {   // an earlier level failed
          waiting.pop_front();
          drop(q, q->res.status);
          continue;
        }
        Solve* s = &q->solves[u.lev];
        s->gauge_id = q->r.gauge_id;
        s->dom_id = q->series() ? q->doms[u.lev] : q->r.dom_id;
        s->nrhs = q->r.nrhs;
        s->prec = prm.prec;
        s->prm = prm;
        s->src = q->r.src;
        s->info = q->info.data() + (size_t)u.lev * q->r.nrhs;
        size_t fp = 0;
        try {
          if (u.lev == 0) check_request(ctx, q);
          const size_t per = (size_t)q->r.nrhs * gauge_get(ctx, q->r.gauge_id).V * 12 * 2;   // doubles
          s->sol = q->series() ? q->terms + per * u.lev : q->r.sol;
          fp = solve_footprint(ctx, s->gauge_id, s->dom_id, s->nrhs, s->prm);
        } catch (const Error& e) {
          waiting.pop_front();
          drop(q, e.code);
          continue;
        }
        if (!live.empty() && !ctx->pool->fits_device(fp)) break;
        if (!solve_slot_free(ctx, s->prec, s->nrhs, s->prm)) break;
        waiting.pop_front();
        try {
          solve_prepare(ctx, s);
          solve_join(ctx, s);
          if (u.lev == 0) q->res.admit_time = now_s();
          live.push_back(s);
          owner[s] = q;
        } catch (const Error& e) {
          solve_release(s);
          if (e.code == DDML_ENOMEM && !live.empty()) {
            // memory frees up as the solves in flight finish: wait for them
            waiting.push_front(u);
            break;
          }
          drop(q, e.code);
        }
      }
      try {
        if (!live.empty()) solve_progress(ctx, live, false);
        for (auto it = live.begin(); it != live.end();) {
          Solve* s = *it;
          if (s->state == 3) {
            Req* q = owner[s];
            solve_finish(ctx, s);
            owner.erase(s);
            it = live.erase(it);
            if (--q->left == 0) {
              if (q->series() && q->res.status == DDML_EAGAIN)
                series_terms(ctx, q->r.gauge_id, q->doms.data(), (int)q->doms.size(), q->terms, q->sum,
                             q->r.nrhs);
              retired.push_back(q);
            }
          } else {
            ++it;
          }
        }
        if (!retired.empty()) {
          hipEvent_t e = nullptr;
          if (!spare.empty()) {
            e = spare.back();
            spare.pop_back();
          } else {
            DDML_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
          }
          DDML_HIP(hipEventRecord(e, ctx->stream));
          landing.emplace_back(e, std::move(retired));
          retired.clear();
        }
        // requests whose results have landed (all of them once nothing is left on the GPU)
        while (!landing.empty()) {
          hipEvent_t e = landing.front().first;
          const hipError_t st = live.empty() ? hipEventSynchronize(e) : hipEventQuery(e);
          if (st == hipErrorNotReady) break;
          DDML_HIP(st);
          for (Req* r : landing.front().second) finished.push_back(r);
          spare.push_back(e);
          landing.pop_front();
        }
      } catch (const Error& e) {
        // a device error ends every request in flight
        std::set<Req*> hit;
        for (Solve* s : live) {
          hit.insert(owner[s]);
          solve_abandon(ctx, s);
        }
        for (Req* r : retired) hit.insert(r);
        for (auto& l : landing) {
          spare.push_back(l.first);
          for (Req* r : l.second) hit.insert(r);
        }
        live.clear();
        owner.clear();
        landing.clear();
        for (Req* r : hit) {
          r->res.status = e.code;
          r->left = 0;
          finished.push_back(r);
        }
        // levels of those requests still waiting are dropped when reached
      }
    }
    const double t = now_s();
    {
      std::lock_guard<std::mutex> lk(m);
      waiting_count = waiting.size();
      in_flight = (long)live.size();
      for (Req* q : finished) {
        ddml_result& r = q->res;
        if (r.status == DDML_EAGAIN) {
          int st = DDML_OK, mo = 0, mi = 0;
          double worst = 0;
          for (const ddml_rhs_info& in : q->info) {
            if (in.status != DDML_OK && st == DDML_OK) st = in.status;
            mo = std::max(mo, in.outer_iters);
            mi = std::max(mi, in.inner_iters);
            worst = std::max(worst, in.true_rel_residual);
          }
          r.status = st;
          r.max_outer = mo;
          r.max_inner_iters = mi;
          r.worst_rel_residual = worst;
        }
        if (q->user_info) std::copy(q->info.begin(), q->info.end(), q->user_info);
        r.finish_time = t;
        q->done = true;
        completed++;
        latencies.push_back(t - q->r.arrival_time);
        last_finish = std::max(last_finish, t);
      }
    }
    if (!finished.empty()) cv_done.notify_all();
  }
  for (hipEvent_t e : spare) (void)hipEventDestroy(e);
}

}  // namespace ddml
