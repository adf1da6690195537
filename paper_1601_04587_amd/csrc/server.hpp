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

struct Req {
  ddml_request r{};
  uint64_t ticket = 0;
  Solve solve;
  ddml_rhs_info info[kMaxRhs]{};
  ddml_result res{};
  bool done = false;
};

struct Server {
  Ctx* ctx;
  ddml_solver_params prm;
  int max_queue;
  std::mutex m;
  std::condition_variable cv, cv_done;
  std::deque<Req*> incoming;
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
  int poll(uint64_t ticket, ddml_result* res);
  int wait(uint64_t ticket, ddml_result* res, double timeout_s);
  void stats(ddml_server_stats* s);
  void loop();
};

}  // namespace ddml
