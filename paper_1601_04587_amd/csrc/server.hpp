// Request loop of libddml (continuous batching of domain solves).
#pragma once
#include <condition_variable>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "engine.hpp"

namespace ddml {

double now_s();

// One request: a single domain solve, or a propagator series (one solve per
// nested domain, then the differences of eq. Dseries).
struct Req {
  ddml_request r{};                 // gauge, nrhs, src, arrival; dom_id and sol of a single solve
  uint64_t ticket = 0;
  std::vector<int> doms;            // series: the nested domains (empty for a single solve)
  double* terms = nullptr;          // series: device [levels][nrhs][V][4][3]
  double* sum = nullptr;            // series: device [nrhs][V][4][3] or null
  ddml_rhs_info* user_info = nullptr;  // series: host [levels][nrhs] or null
  std::vector<Solve> solves;        // one per level
  std::vector<ddml_rhs_info> info;  // [levels][nrhs]
  int left = 0;                     // levels not finished yet
  ddml_result res{};
  bool done = false;
  bool series() const { return !doms.empty(); }
  int levels() const { return series() ? (int)doms.size() : 1; }
};

struct Server {
  Ctx* ctx;
  ddml_solver_params prm;
  int max_queue;
  std::mutex m;
  std::condition_variable cv, cv_done;
  std::deque<Req*> incoming;
  int enqueue(std::unique_ptr<Req> q, uint64_t* ticket);
  size_t waiting_count = 0;
  std::map<uint64_t, std::unique_ptr<Req>> reqs;
  uint64_t next_ticket = 1;
  std::vector<double> latencies;
  long submitted = 0, completed = 0, in_flight = 0;
  double first_arrival = std::numeric_limits<double>::infinity(), last_finish = 0;
  bool stop = false;
  std::thread th;

  Server(Ctx* c, const ddml_solver_params& p, int max_queue);
  ~Server();
  int submit(const ddml_request& r, uint64_t* ticket);
  int submit_series(const ddml_series_request& r, uint64_t* ticket);
  int poll(uint64_t ticket, ddml_result* res);
  int wait(uint64_t ticket, ddml_result* res, double timeout_s);
  void stats(ddml_server_stats* s);
  void loop();
};

}  // namespace ddml
