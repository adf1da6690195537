// Host engine of libddml: device memory, gauge versions, domains, operator
// blocks and the batched mixed-precision solver.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ddml.h"
#include "ddml_common.hpp"
#include "launchers.hpp"

namespace ddml {

struct Error {
  int code;
  std::string msg;
};

#define DDML_HIP(call)                                                                 \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::ddml::Error{DDML_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// ---------------------------------------------------------------- memory
// Caching device allocator with a byte budget.  Blocks are rounded to 2 MiB
// and recycled by exact size, so the repeated same-size allocations of a
// serving loop never reach hipMalloc after warm-up.
class DevPool {
 public:
  explicit DevPool(size_t budget) : budget_(budget) {}
  ~DevPool();
  void* alloc(size_t bytes);   // throws Error{ENOMEM}
  void free(void* p);
  bool fits(size_t bytes) const;
  // fits() and the device's free memory (plus this pool's cache) covers it:
  // memory taken by other allocators (e.g. the caller's tensors) counts too
  bool fits_device(size_t bytes) const;
  size_t in_use() const { return in_use_; }
  size_t budget() const { return budget_; }
  size_t cached() const { return cached_; }
  static size_t round(size_t b) { return ((b + (2u << 20) - 1) >> 21) << 21; }
  void trim();  // release cached blocks

 private:
  std::mutex mu_;
  size_t budget_;
  size_t in_use_ = 0;   // bytes handed out
  size_t cached_ = 0;   // bytes held in free lists
  std::map<size_t, std::vector<void*>> free_;
  std::unordered_map<void*, size_t> sizes_;
};

struct DBuf {
  DevPool* pool = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(DevPool* pl, size_t b) : pool(pl), p(b ? pl->alloc(b) : nullptr), bytes(b) {}
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : pool(o.pool), p(o.p), bytes(o.bytes) { o.p = nullptr; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { reset(); pool = o.pool; p = o.p; bytes = o.bytes; o.p = nullptr; }
    return *this;
  }
  ~DBuf() { reset(); }
  void reset() { if (p && pool) pool->free(p); p = nullptr; bytes = 0; }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// ------------------------------------------------------------ model objects
struct GaugeRec {
  std::shared_ptr<DBuf> base;     // [V][4][9] double2
  std::shared_ptr<DBuf> region;   // [V_region][4][9] or null
  int r_t0 = 0, r_t1 = 0;
  double kappa = 0, csw = 0;
  ddml_lattice lat{};             // the host lattice of this field (the context's by default)
  size_t V = 0;
};

struct DomainRec {
  int lo[4], hi[4];
};

struct OpBlock {
  BlockSpec bs;
  BoxGeom g;
  int ntiles = 0;
  int tps = 0;             // tiles per time slice (0 if a slice is not a whole number of tiles)
  size_t field = 0;        // complex numbers in one [12-column] field: nrhs * 12 * ntiles * 64 / nrhs
  DBuf U64, A64, Ainv64;   // FP64 operator data
  DBuf U32, Ainv32;        // FP32 copies for the inner solve
  DBuf U16, Ainv16, Ainv16n;  // 16-bit copies (built on first use by a DDML_MIXED_FP16 solve)
  DBuf walk[kWalks];       // tile walks of TILE_ORDER_SUB2, SUB4, SUB4T, QUAD
  int xoff[kWalks][kXcd + 1] = {};
  size_t bytes = 0;
  bool su3 = true;         // links are SU(3) to 1e-5 (the FP32 and 16-bit copies keep two rows)
};

struct Ctx;

// One domain solve in flight.
struct Solve {
  int gauge_id = -1, dom_id = -1, nrhs = 0, prec = DDML_MIXED_FP32;
  std::shared_ptr<OpBlock> ob;
  ddml_solver_params prm{};
  // FP64 outer state, each [nrhs][12][Vh]
  DBuf be, bo, xe, xo, re, ro, te, to;
  DBuf partial64;   // [2][nrhs][ntiles]
  DBuf norms;       // double2 [4][nrhs]: |b|^2, |r|^2
  // inner state in the inner precision (16-bit: values then scales; F_X in FP32);
  // BiCGstab uses slots [0, F_NUM), GCR(m) F_R, F_X, F_TMP and the 2m GCR slots
  DBuf f[F_ALL];
  DBuf partial;     // [2][nrhs][ntiles]
  DBuf table1, tstart1, n1;  // one-entry slot table
  int slot = -1;    // position in the batch table
  bool dev = false; // the outer loop runs on the device
  // host bookkeeping
  std::vector<double> bn2, rel;
  std::vector<int> done, inner_iters, status;
  int outer = 0;
  int state = 0;    // 0 new, 1 prepared (host loop: needs a residual), 4 ready to join (host loop),
                    // 2 in a slot, 3 finished
  const double* src = nullptr;   // canonical device pointer
  double* sol = nullptr;         // canonical device pointer
  ddml_rhs_info* info = nullptr; // host
  size_t footprint = 0;
  uint64_t tag = 0;              // serving ticket (0 for direct calls)
};

// Launch choice of the batched stencil: columns per thread R, captured
// iterations K, workgroups, tile order and column splits (workgroups per tile).
struct TuneChoice {
  int R = 1;
  int K = 8;
  int grid = 1024;
  int order = TILE_ORDER_BANDED;
  int splits = 1;
  int stage = 0;
};

// Batched solver for one precision, nrhs and Krylov method: a slot table in
// device memory and a captured graph over it.
//   BiCGstab (device loop): the FP64 outer step of every slot (export of the
//   inner solution, true residual, decision, preparation of the next inner
//   right-hand side and the inner initialisation), then K inner iterations.
//   The host only admits solves into free slots and retires the slots that
//   the device has marked PH_DONE, reading the slot phases asynchronously one
//   replay behind.
//   GCR(m) (host loop): one GCR(m) cycle; the host runs the FP64 outer steps
//   between cycles.
template <typename T2>
struct BatchRunner {
  Ctx* ctx = nullptr;
  int nrhs = 0, R = 3, K = 8, grid = 1024, max_slots = 64, splits = 1, stage = 0;
  int gcr_m = 0;                  // 0: BiCGstab; m > 0: GCR(m)
  bool device = false;            // the outer loop runs on the device (BiCGstab)
  DBuf table, tstart, xstart, nslots, st_all, act_all, gc_all;
  // device loop: per-slot phase, per-column outer state, step flags [3][kMaxRhs]
  // per slot, and the FP64 view tables [4][max_slots] (export, residual even,
  // residual odd, preparation)
  DBuf sst_all, ost_all, oflag_all, views;
  std::vector<SlotDesc<double2>> h_views;
  void* pin_up[2] = {nullptr, nullptr};   // pinned table uploads (two in flight at most)
  void* pin_rb[2] = {nullptr, nullptr};   // pinned phase / outer-state readbacks
  size_t up_bytes = 0, rb_bytes = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool pending[2] = {false, false};
  int rb_used[2] = {0, 0};
  // join number of each slot's occupant (never reused, unlike Solve addresses),
  // now and at the time of each readback
  uint64_t joins = 0;
  std::vector<uint64_t> gen_of, snap[2];
  int ring = 0;
  int order = TILE_ORDER_BANDED;
  std::vector<SlotDesc<T2>> h_table;
  std::vector<int> h_tstart, h_xstart;
  std::vector<Solve*> slot_of;    // slot -> solve (nullptr = free)
  std::vector<BiState> h_st;
  hipGraphExec_t exec = nullptr;
  bool dirty = true;
  int nused = 0;                  // highest used slot + 1
  ~BatchRunner();
  void init(Ctx* c, int nrhs_, const TuneChoice& tn, int max_slots_, int gcr_m_);
  void capture();
  int join(Solve* s);             // returns slot or -1 if full
  void leave(Solve* s);
  void upload();
  void replay();
  int members() const;
  bool has_free() const;
  // device loop: enqueue one replay and its phase readback; then retire the
  // slots the previous readback found finished (their solves get state 3)
  void launch_dev();
  void collect_dev();
};


struct Server;

struct Ctx {
  ddml_lattice lat{};
  int device = 0;
  size_t V = 0;
  hipStream_t stream = nullptr;
  std::unique_ptr<DevPool> pool;
  std::recursive_mutex mu;
  std::atomic<int> api_waiting{0};   // API calls waiting for mu (the request loop yields to them)
  std::string last_error;
  int next_gauge = 1, next_dom = 1;
  std::map<int, GaugeRec> gauges;
  std::map<int, DomainRec> domains;
  std::map<std::pair<int, int>, std::shared_ptr<OpBlock>> blocks;
  std::map<int, std::unique_ptr<BatchRunner<float2>>> run32;   // by nrhs
  std::map<int, std::unique_ptr<BatchRunner<double2>>> run64;
  std::map<int, std::unique_ptr<BatchRunner<h16c>>> run16;
  DBuf flag;        // device int for clover failures
  DomainRec full{};  // the whole lattice (dom_id -1)
  void* pinned = nullptr;   // small pinned host staging area
  size_t pinned_bytes = 0;
  TuneChoice tune64, tune32, tune16;   // launch choices of the FP64, FP32 and 16-bit kernels
  TuneChoice& tune(int prec) {
    return prec == DDML_FP64 ? tune64 : (prec == DDML_MIXED_FP16 ? tune16 : tune32);
  }
  std::unique_ptr<Server> server;
  void* blas = nullptr;   // rocBLAS handle (linalg_blas.cpp), created on first use
  ~Ctx();
};

// engine.cpp
void ctx_init(Ctx* c, const ddml_lattice* lat, int device, size_t budget);
int gauge_new(Ctx* c, const double* U, int on_device, double kappa, double csw);
int gauge_new_lattice(Ctx* c, const ddml_lattice* lat, const double* U, int on_device, double kappa, double csw);
const GaugeRec& gauge_get(Ctx* c, int gauge_id);
int gauge_region(Ctx* c, int base, int t0, int t1, const double* U, int on_device);
// new version whose slices [t0, t1) are the parent's after nsweeps level-1 sweeps
int gauge_level1(Ctx* c, int base, int t0, int t1, double beta, uint64_t seed, uint32_t stream, int nsweeps,
                 int n_or);
void gauge_copy_out(Ctx* c, int id, double* U, int on_device);
void gauge_release(Ctx* c, int id);
int domain_new(Ctx* c, const int lo[4], const int hi[4]);
const DomainRec& domain_get(Ctx* c, int dom_id);  // dom_id -1 = full lattice
std::shared_ptr<OpBlock> opblock(Ctx* c, int gauge_id, int dom_id);
size_t solve_footprint(Ctx* c, int gauge_id, int dom_id, int nrhs, const ddml_solver_params& prm);
// True if [p, p + bytes) lies inside one device allocation on `device`
// (bytes 0: only that p is device memory there).  Host memory gives false.
bool device_span_ok(const void* p, size_t bytes, int device);
// GCR restart length of a parameter set (0 for BiCGstab)
int gcr_len(const ddml_solver_params& prm);
void apply_D(Ctx* c, int gauge_id, int dom_id, const double* in, double* out, int nrhs, hipStream_t st);
void apply_eo(Ctx* c, int gauge_id, int dom_id, const double* in, double* out, int nrhs, int prec, hipStream_t st);
// out = scale * D_{dGamma} in (canonical FP64 fields on the gauge field's lattice)
void apply_boundary(Ctx* c, int gauge_id, int dom_id, const double* in, double* out, int nrhs, double scale,
                    hipStream_t st);
// linalg_blas.cpp (rocBLAS): per-slice Gram matrices G[t] = X_t^dag X_t for t in
// [t0, t1) (zero elsewhere), X = n canonical fields; orthonormalisation of the
// columns of X on rows [row0, row0 + nrows) by Cholesky QR (twice)
void gram_slices(Ctx* c, const double2* X, int n, size_t V, int T, int t0, int t1, double2* G);
void orthonormalize(Ctx* c, double2* X, int n, size_t V, size_t row0, size_t nrows);
// slice sums of the colourless spinors of n fields (xi = 1: of conj(g5 X)), B [T][n^2][4n]
void bary_slices(Ctx* c, const double2* X, int n, size_t V, int T, int t0, int t1, int xi, double2* B);
void blas_release(Ctx* c);
// Runs every solve to completion (continuous batching inside).  Device pointers.
void run_solves(Ctx* c, std::vector<Solve*>& solves);
// Pieces used by the serving loop
void solve_prepare(Ctx* c, Solve* s);                // allocate + set up (state -> 1)
void solve_progress(Ctx* c, std::vector<Solve*>& live, bool block);  // one scheduling round
// Device loop: whether a solve of this kind would find a free slot now, and
// joining a prepared solve to its slot (false: no slot free yet)
bool solve_slot_free(Ctx* c, int prec, int nrhs, const ddml_solver_params& prm);
bool solve_join(Ctx* c, Solve* s);
void solve_finish(Ctx* c, Solve* s);                 // scatter, info, free
void solve_release(Solve* s);                        // free device state (after a failed prepare)
// a solve in flight given up after an error: its slot is freed, its device
// state released, state -> 3 (no results)
void solve_abandon(Ctx* c, Solve* s);
// eq. Dseries in place: terms[0..nlevels) hold S^(0..nlevels-1) (canonical
// device fields, nrhs columns each) and become S^(0), S^(1) - S^(0), ...;
// sum (device, or null) receives S^(nlevels-1).  On the context's stream.
void series_terms(Ctx* c, int gauge_id, const int* dom_ids, int nlevels, double* terms, double* sum, int nrhs);
void check_params(const ddml_solver_params* p);
// Times the two stencil kernels of the inner solver (k_hop_batch, CINV_HOP and
// SCHUR with its fused dot product) on one slot; out = {ms_cinv, ms_schur,
// bytes_cinv, bytes_schur} per launch (algorithmic bytes).  Fields of `want`
// that are <= 0 (order, stage: < 0) take the context's current choice.
void time_stencil(Ctx* c, int gauge_id, int dom_id, int nrhs, int prec, int iters, const TuneChoice& want,
                  double out[4]);
// Picks the fastest stencil launch (R, order, grid, splits, stage) and rebuilds
// the solver graphs.
void autotune(Ctx* c, int gauge_id, int dom_id, int nrhs, int prec, double best[6]);
// Makes `want` the launch choice of precision prec (the solver graphs are rebuilt).
void set_launch(Ctx* c, int prec, const TuneChoice& want);
ddml_solver_params default_params();

}  // namespace ddml
