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

int Server::submit(const ddml_request& r, uint64_t* ticket) {
  std::lock_guard<std::mutex> lk(m);
  if ((int)(incoming.size() + waiting_count) >= max_queue) return DDML_EAGAIN;
  auto q = std::make_unique<Req>();
  q->r = r;
  q->ticket = next_ticket++;
  q->res.status = DDML_EAGAIN;
  q->res.arrival_time = r.arrival_time;
  *ticket = q->ticket;
  incoming.push_back(q.get());
  reqs[q->ticket] = std::move(q);
  submitted++;
  first_arrival = std::min(first_arrival, r.arrival_time);
  cv.notify_all();
  return DDML_OK;
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

void Server::loop() {
  std::deque<Req*> waiting;
  std::vector<Solve*> live;
  std::map<Solve*, Req*> owner;
  // retired requests whose solution scatter is still on the stream
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
        waiting.push_back(incoming.front());
        incoming.pop_front();
      }
      waiting_count = waiting.size();
      if (stop && live.empty() && waiting.empty() && landing.empty()) break;
    }
    if (live.empty() && waiting.empty() && landing.empty()) continue;
    std::vector<Req*> finished;
    {
      std::lock_guard<std::recursive_mutex> g(ctx->mu);
      // admission by device footprint
      while (!waiting.empty()) {
        Req* q = waiting.front();
        Solve* s = &q->solve;
        s->gauge_id = q->r.gauge_id;
        s->dom_id = q->r.dom_id;
        s->nrhs = q->r.nrhs;
        s->prec = prm.prec;
        s->prm = prm;
        s->src = q->r.src;
        s->sol = q->r.sol;
        s->info = q->info;
        size_t fp = 0;
        try {
          fp = solve_footprint(ctx, s->gauge_id, s->dom_id, s->nrhs, s->prm);
          const size_t bytes = (size_t)s->nrhs * gauge_get(ctx, s->gauge_id).V * 12 * sizeof(double2);
          if (!device_span_ok(s->src, bytes, ctx->device) || !device_span_ok(s->sol, bytes, ctx->device))
            throw Error{DDML_EINVAL, "request buffers do not hold nrhs canonical fields in device memory"};
        } catch (const Error& e) {
          q->res.status = e.code;
          waiting.pop_front();
          finished.push_back(q);
          continue;
        }
        if (!live.empty() && !ctx->pool->fits_device(fp)) break;
        if (!solve_slot_free(ctx, s->prec, s->nrhs, s->prm)) break;
        waiting.pop_front();
        try {
          solve_prepare(ctx, s);
          solve_join(ctx, s);
          q->res.admit_time = now_s();
          live.push_back(s);
          owner[s] = q;
        } catch (const Error& e) {
          solve_release(s);
          if (e.code == DDML_ENOMEM && !live.empty()) {
            // memory frees up as the solves in flight finish: wait for them
            waiting.push_front(q);
            break;
          }
          q->res.status = e.code;
          finished.push_back(q);
        }
      }
      try {
        if (!live.empty()) solve_progress(ctx, live, false);
        std::vector<Req*> retired;
        for (auto it = live.begin(); it != live.end();) {
          Solve* s = *it;
          if (s->state == 3) {
            solve_finish(ctx, s);
            retired.push_back(owner[s]);
            owner.erase(s);
            it = live.erase(it);
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
        }
        // requests whose scatter has landed (all of them once nothing is left on the GPU)
        while (!landing.empty()) {
          hipEvent_t e = landing.front().first;
          const hipError_t q = live.empty() ? hipEventSynchronize(e) : hipEventQuery(e);
          if (q == hipErrorNotReady) break;
          DDML_HIP(q);
          for (Req* r : landing.front().second) finished.push_back(r);
          spare.push_back(e);
          landing.pop_front();
        }
      } catch (const Error& e) {
        // a device error ends every request in flight
        for (Solve* s : live) {
          Req* q = owner[s];
          q->res.status = e.code;
          finished.push_back(q);
        }
        live.clear();
        owner.clear();
        for (auto& l : landing) {
          spare.push_back(l.first);
          for (Req* r : l.second) {
            r->res.status = e.code;
            finished.push_back(r);
          }
        }
        landing.clear();
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
          for (int col = 0; col < q->r.nrhs; ++col) {
            const ddml_rhs_info& in = q->info[col];
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
