// C ABI of libddml (declarations and documentation in include/ddml.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "engine.hpp"
#include "server.hpp"

using namespace ddml;

struct ddml_ctx_s {
  Ctx c;
};

namespace {

// Orders the library stream after the caller's stream on entry and the
// caller's stream after the library stream on exit.
struct StreamJoin {
  Ctx* c;
  hipStream_t user;
  StreamJoin(Ctx* ctx, void* s) : c(ctx), user((hipStream_t)s) {
    hipEvent_t e;
    DDML_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    DDML_HIP(hipEventRecord(e, user));
    DDML_HIP(hipStreamWaitEvent(c->stream, e, 0));
    DDML_HIP(hipEventDestroy(e));
  }
  void done() {
    hipEvent_t e;
    DDML_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    DDML_HIP(hipEventRecord(e, c->stream));
    DDML_HIP(hipStreamWaitEvent(user, e, 0));
    DDML_HIP(hipEventDestroy(e));
  }
};

template <typename F>
int guarded(ddml_ctx ctx, F&& f) {
  if (!ctx) return DDML_EINVAL;
  // announce the call, so that the request loop lets it take the context
  // lock between its rounds (std::mutex promises no fairness)
  ctx->c.api_waiting.fetch_add(1);
  std::unique_lock<std::recursive_mutex> lk(ctx->c.mu);
  ctx->c.api_waiting.fetch_sub(1);
  try {
    DDML_HIP(hipSetDevice(ctx->c.device));
    int rc = f(&ctx->c);
    return rc;
  } catch (const Error& e) {
    ctx->c.last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->c.last_error = "host allocation failed";
    return DDML_ENOMEM;
  } catch (const std::exception& e) {
    ctx->c.last_error = e.what();
    return DDML_EINVAL;
  }
}

// Staging of a canonical array: device pointer as is, or a device copy of host data.
struct Staged {
  DBuf buf;
  const double* cptr = nullptr;
  double* ptr = nullptr;
};

Staged stage_in(Ctx* c, const double* p, size_t bytes, int on_device) {
  Staged s;
  if (on_device) {
    s.cptr = p;
    s.ptr = const_cast<double*>(p);
    return s;
  }
  s.buf = DBuf(c->pool.get(), bytes);
  DDML_HIP(hipMemcpyAsync(s.buf.p, p, bytes, hipMemcpyHostToDevice, c->stream));
  s.cptr = s.buf.as<double>();
  s.ptr = s.buf.as<double>();
  return s;
}

Staged stage_out(Ctx* c, double* p, size_t bytes, int on_device) {
  Staged s;
  if (on_device) {
    s.ptr = p;
    s.cptr = p;
    return s;
  }
  s.buf = DBuf(c->pool.get(), bytes);
  s.ptr = s.buf.as<double>();
  s.cptr = s.ptr;
  return s;
}

void copy_back(Ctx* c, double* host, const Staged& s, size_t bytes, int on_device) {
  if (on_device) return;
  DDML_HIP(hipMemcpyAsync(host, s.cptr, bytes, hipMemcpyDeviceToHost, c->stream));
  DDML_HIP(hipStreamSynchronize(c->stream));
}

void need(bool cond, const char* msg) {
  if (!cond) throw Error{DDML_EINVAL, msg};
}

}  // namespace

extern "C" {

double ddml_now(void) { return now_s(); }

int ddml_create(ddml_ctx* out, const ddml_lattice* lat, int device, size_t hbm_budget_bytes) {
  if (!out) return DDML_EINVAL;
  *out = nullptr;
  ddml_ctx ctx = new (std::nothrow) ddml_ctx_s();
  if (!ctx) return DDML_ENOMEM;
  try {
    ctx_init(&ctx->c, lat, device, hbm_budget_bytes);
  } catch (const Error& e) {
    delete ctx;
    return e.code;
  }
  *out = ctx;
  return DDML_OK;
}

int ddml_destroy(ddml_ctx ctx) {
  if (!ctx) return DDML_EINVAL;
  ctx->c.server.reset();
  {
    std::lock_guard<std::recursive_mutex> lk(ctx->c.mu);
    (void)hipSetDevice(ctx->c.device);
    (void)hipStreamSynchronize(ctx->c.stream);
  }
  delete ctx;
  return DDML_OK;
}

const char* ddml_last_error(ddml_ctx ctx) {
  static const char empty[] = "";
  if (!ctx) return empty;
  return ctx->c.last_error.c_str();
}

int ddml_set_gauge(ddml_ctx ctx, const double* U, int on_device, double kappa, double csw, int* gauge_id) {
  return guarded(ctx, [&](Ctx* c) {
    need(gauge_id != nullptr, "gauge_id is NULL");
    *gauge_id = gauge_new(c, U, on_device, kappa, csw);
    return DDML_OK;
  });
}

int ddml_set_gauge_lattice(ddml_ctx ctx, const ddml_lattice* lat, const double* U, int on_device, double kappa,
                           double csw, int* gauge_id) {
  return guarded(ctx, [&](Ctx* c) {
    need(gauge_id != nullptr, "gauge_id is NULL");
    *gauge_id = gauge_new_lattice(c, lat, U, on_device, kappa, csw);
    return DDML_OK;
  });
}

int ddml_set_gauge_region(ddml_ctx ctx, int base_gauge_id, int t0, int t1, const double* U_region, int on_device,
                          int* new_gauge_id) {
  return guarded(ctx, [&](Ctx* c) {
    need(new_gauge_id != nullptr, "new_gauge_id is NULL");
    *new_gauge_id = gauge_region(c, base_gauge_id, t0, t1, U_region, on_device);
    return DDML_OK;
  });
}

int ddml_level1_update(ddml_ctx ctx, int base_gauge_id, int t0, int t1, double beta, uint64_t seed,
                       uint32_t stream, int nsweeps, int n_or, int* new_gauge_id) {
  return guarded(ctx, [&](Ctx* c) {
    need(new_gauge_id != nullptr, "new_gauge_id is NULL");
    *new_gauge_id = gauge_level1(c, base_gauge_id, t0, t1, beta, seed, stream, nsweeps, n_or);
    return DDML_OK;
  });
}

int ddml_get_gauge(ddml_ctx ctx, int gauge_id, double* U, int on_device) {
  return guarded(ctx, [&](Ctx* c) {
    need(U != nullptr, "U is NULL");
    gauge_copy_out(c, gauge_id, U, on_device);
    return DDML_OK;
  });
}

int ddml_release_gauge(ddml_ctx ctx, int gauge_id) {
  return guarded(ctx, [&](Ctx* c) {
    gauge_release(c, gauge_id);
    return DDML_OK;
  });
}

int ddml_set_domain(ddml_ctx ctx, const int lo[4], const int hi[4], int* dom_id) {
  return guarded(ctx, [&](Ctx* c) {
    need(dom_id != nullptr, "dom_id is NULL");
    *dom_id = domain_new(c, lo, hi);
    return DDML_OK;
  });
}

int ddml_apply_Dw(ddml_ctx ctx, int gauge_id, int dom_id, const double* in, double* out, int nrhs, int prec,
                  int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    need(in && out, "NULL buffer");
    need(nrhs >= 1 && nrhs <= kMaxRhs, "nrhs must be in 1..12");
    need(prec == DDML_FP64, "apply_Dw is FP64");
    const size_t bytes = (size_t)nrhs * gauge_get(c, gauge_id).V * 12 * sizeof(double2);
    StreamJoin sj(c, stream);
    Staged si = stage_in(c, in, bytes, on_device);
    Staged so = stage_out(c, out, bytes, on_device);
    apply_D(c, gauge_id, dom_id, si.cptr, so.ptr, nrhs, c->stream);
    copy_back(c, out, so, bytes, on_device);
    sj.done();
    return DDML_OK;
  });
}

int ddml_apply_eo(ddml_ctx ctx, int gauge_id, int dom_id, const double* in, double* out, int nrhs, int prec,
                  int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    need(in && out, "NULL buffer");
    need(nrhs >= 1 && nrhs <= kMaxRhs, "nrhs must be in 1..12");
    need(prec == DDML_FP64 || prec == DDML_MIXED_FP32 || prec == DDML_MIXED_FP16, "unknown precision");
    const size_t bytes = (size_t)nrhs * gauge_get(c, gauge_id).V * 12 * sizeof(double2);
    StreamJoin sj(c, stream);
    Staged si = stage_in(c, in, bytes, on_device);
    Staged so = stage_out(c, out, bytes, on_device);
    apply_eo(c, gauge_id, dom_id, si.cptr, so.ptr, nrhs, prec, c->stream);
    copy_back(c, out, so, bytes, on_device);
    sj.done();
    return DDML_OK;
  });
}

static int solve_many(Ctx* c, int n, const ddml_solve_desc* d, const ddml_solver_params* params, int on_device,
                      void* stream) {
  check_params(params);
  need(n >= 1 && d != nullptr, "no solves");
  std::vector<size_t> bytes(n);  // canonical arrays on each solve's host lattice
  for (int i = 0; i < n; ++i) {
    need(d[i].src && d[i].sol && d[i].info, "NULL buffer in solve desc");
    need(d[i].nrhs >= 1 && d[i].nrhs <= kMaxRhs, "nrhs must be in 1..12");
    need(d[i].nrhs == d[0].nrhs, "all solves of a batch must have the same nrhs");
    bytes[i] = (size_t)d[i].nrhs * gauge_get(c, d[i].gauge_id).V * 12 * sizeof(double2);
    if (d[i].dom_id != -1) (void)domain_get(c, d[i].dom_id);
  }
  StreamJoin sj(c, stream);
  std::vector<Staged> sin, sout;
  std::vector<Solve> solves(n);
  std::vector<Solve*> ptrs;
  for (int i = 0; i < n; ++i) {
    sin.push_back(stage_in(c, d[i].src, bytes[i], on_device));
    sout.push_back(stage_out(c, d[i].sol, bytes[i], on_device));
  }
  for (int i = 0; i < n; ++i) {
    Solve& s = solves[i];
    s.gauge_id = d[i].gauge_id;
    s.dom_id = d[i].dom_id;
    s.nrhs = d[i].nrhs;
    s.prec = params->prec;
    s.prm = *params;
    s.src = sin[i].cptr;
    s.sol = sout[i].ptr;
    s.info = d[i].info;
    ptrs.push_back(&s);
  }
  run_solves(c, ptrs);
  for (int i = 0; i < n; ++i) copy_back(c, d[i].sol, sout[i], bytes[i], on_device);
  sj.done();
  int rc = DDML_OK;
  for (int i = 0; i < n && rc == DDML_OK; ++i)
    for (int col = 0; col < d[i].nrhs; ++col)
      if (d[i].info[col].status != DDML_OK) {
        rc = d[i].info[col].status;
        c->last_error = "a right-hand side did not reach the tolerance";
        break;
      }
  return rc;
}

// ncols canonical device fields solved 12 at a time: the full groups as one
// batch, the remainder as another; info [ncols].  Returns the first failure.
static int solve_columns(Ctx* c, int gauge_id, int dom_id, const double* src, double* sol, int ncols, size_t per,
                         const ddml_solver_params* params, ddml_rhs_info* info) {
  const int nfull = ncols / kMaxRhs, rest = ncols - nfull * kMaxRhs;
  int rc = DDML_OK;
  for (int part = 0; part < 2; ++part) {
    std::vector<ddml_solve_desc> d;
    const int cols = part == 0 ? kMaxRhs : rest;
    const int ng = part == 0 ? nfull : (rest > 0 ? 1 : 0);
    for (int k = 0; k < ng; ++k) {
      const size_t first = (size_t)(part == 0 ? k * kMaxRhs : nfull * kMaxRhs);
      d.push_back(ddml_solve_desc{gauge_id, dom_id, src + 2 * per * first, sol + 2 * per * first, cols, info + first});
    }
    if (!d.empty()) {
      const int r = solve_many(c, (int)d.size(), d.data(), params, 1, c->stream);
      if (rc == DDML_OK) rc = r;
    }
  }
  return rc;
}

int ddml_solve_domain(ddml_ctx ctx, int gauge_id, int dom_id, const double* src, double* sol, int nrhs,
                      const ddml_solver_params* params, ddml_rhs_info* info, int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    ddml_solve_desc d{gauge_id, dom_id, src, sol, nrhs, info};
    return solve_many(c, 1, &d, params, on_device, stream);
  });
}

int ddml_solve_batch(ddml_ctx ctx, int nsolves, const ddml_solve_desc* descs, const ddml_solver_params* params,
                     int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) { return solve_many(c, nsolves, descs, params, on_device, stream); });
}

static int series_many(Ctx* c, int ns, const ddml_series_desc* sd, int nrhs, const ddml_solver_params* params,
                       int on_device, void* stream) {
  need(ns >= 1 && sd != nullptr, "no series");
  need(nrhs >= 1 && nrhs <= kMaxRhs, "nrhs must be in 1..12");
  check_params(params);
  StreamJoin sj(c, stream);
  std::vector<Staged> si, st, ss;
  std::vector<size_t> per(ns);  // complex numbers of one level on the series' host lattice
  std::vector<ddml_solve_desc> d;
  for (int k = 0; k < ns; ++k) {
    need(sd[k].dom_ids && sd[k].nlevels >= 1 && sd[k].src && sd[k].terms && sd[k].info, "bad series desc");
    per[k] = (size_t)nrhs * gauge_get(c, sd[k].gauge_id).V * 12;
    const size_t bytes = per[k] * sizeof(double2);
    si.push_back(stage_in(c, sd[k].src, bytes, on_device));
    st.push_back(stage_out(c, sd[k].terms, bytes * sd[k].nlevels, on_device));
    ss.push_back(sd[k].sum ? stage_out(c, sd[k].sum, bytes, on_device) : Staged{});
  }
  for (int k = 0; k < ns; ++k)
    for (int i = 0; i < sd[k].nlevels; ++i)
      d.push_back(ddml_solve_desc{sd[k].gauge_id, sd[k].dom_ids[i], si[k].cptr, st[k].ptr + 2 * per[k] * i, nrhs,
                                  sd[k].info + (size_t)i * nrhs});
  // the solves read and write device memory already staged
  int rc = solve_many(c, (int)d.size(), d.data(), params, 1, c->stream);
  for (int k = 0; k < ns; ++k) {
    const size_t bytes = per[k] * sizeof(double2);
    series_terms(c, sd[k].gauge_id, sd[k].dom_ids, sd[k].nlevels, st[k].ptr, sd[k].sum ? ss[k].ptr : nullptr, nrhs);
    copy_back(c, sd[k].terms, st[k], bytes * sd[k].nlevels, on_device);
    if (sd[k].sum) copy_back(c, sd[k].sum, ss[k], bytes, on_device);
  }
  DDML_HIP(hipStreamSynchronize(c->stream));
  sj.done();
  return rc;
}

int ddml_propagator_series(ddml_ctx ctx, int gauge_id, const int* dom_ids, int nlevels, const double* src, int nrhs,
                           const ddml_solver_params* params, double* terms, double* sum, ddml_rhs_info* info,
                           int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    ddml_series_desc d{gauge_id, dom_ids, nlevels, src, terms, sum, info};
    return series_many(c, 1, &d, nrhs, params, on_device, stream);
  });
}

int ddml_propagator_series_batch(ddml_ctx ctx, int nseries, const ddml_series_desc* descs, int nrhs,
                                 const ddml_solver_params* params, int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) { return series_many(c, nseries, descs, nrhs, params, on_device, stream); });
}

int ddml_apply_boundary(ddml_ctx ctx, int gauge_id, int dom_id, const double* in, double* out, int nrhs,
                        double scale, int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    need(in && out, "NULL buffer");
    need(nrhs >= 1 && nrhs <= kMaxRhs, "nrhs must be in 1..12");
    const size_t bytes = (size_t)nrhs * gauge_get(c, gauge_id).V * 12 * sizeof(double2);
    const char* a = reinterpret_cast<const char*>(in);
    const char* b = reinterpret_cast<const char*>(out);
    need(a + bytes <= b || b + bytes <= a, "in and out overlap");
    StreamJoin sj(c, stream);
    Staged si = stage_in(c, in, bytes, on_device);
    Staged so = stage_out(c, out, bytes, on_device);
    apply_boundary(c, gauge_id, dom_id, si.cptr, so.ptr, nrhs, scale, c->stream);
    copy_back(c, out, so, bytes, on_device);
    sj.done();
    return DDML_OK;
  });
}

// Two batches: every Gammabar_i solve, then the boundary blocks, then every Gamma* solve.
int ddml_factorized_series(ddml_ctx ctx, int gauge_id, const int* bar_ids, int nlevels, int star_id,
                           const double* src, int nrhs, const ddml_solver_params* params, double* levels_out,
                           double* bar_out, ddml_rhs_info* info, int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    need(bar_ids && src && levels_out && info, "NULL argument");
    need(nlevels >= 1 && nlevels <= 64, "nlevels must be in 1..64");
    need(nrhs >= 1 && nrhs <= kMaxRhs, "nrhs must be in 1..12");
    check_params(params);
    (void)domain_get(c, star_id);
    for (int i = 0; i < nlevels; ++i) (void)domain_get(c, bar_ids[i]);
    const size_t per = (size_t)nrhs * gauge_get(c, gauge_id).V * 12;  // complex numbers of one field
    const size_t bytes = per * sizeof(double2);
    StreamJoin sj(c, stream);
    Staged si = stage_in(c, src, bytes, on_device);
    Staged sl = stage_out(c, levels_out, bytes * nlevels, on_device);
    Staged sb;
    if (bar_out) sb = stage_out(c, bar_out, bytes * nlevels, on_device);
    else sb.buf = DBuf(c->pool.get(), bytes * nlevels), sb.ptr = sb.buf.as<double>();
    DBuf bstar(c->pool.get(), bytes * nlevels);
    std::vector<ddml_solve_desc> d;
    for (int i = 0; i < nlevels; ++i)
      d.push_back(ddml_solve_desc{gauge_id, bar_ids[i], si.cptr, sb.ptr + 2 * per * i, nrhs,
                                  info + (size_t)(2 * i) * nrhs});
    const int rc1 = solve_many(c, nlevels, d.data(), params, 1, c->stream);
    for (int i = 0; i < nlevels; ++i)
      apply_boundary(c, gauge_id, star_id, sb.ptr + 2 * per * i, bstar.as<double>() + 2 * per * i, nrhs, -1.0,
                     c->stream);
    d.clear();
    for (int i = 0; i < nlevels; ++i)
      d.push_back(ddml_solve_desc{gauge_id, star_id, bstar.as<double>() + 2 * per * i, sl.ptr + 2 * per * i, nrhs,
                                  info + (size_t)(2 * i + 1) * nrhs});
    const int rc2 = solve_many(c, nlevels, d.data(), params, 1, c->stream);
    copy_back(c, levels_out, sl, bytes * nlevels, on_device);
    if (bar_out) copy_back(c, bar_out, sb, bytes * nlevels, on_device);
    DDML_HIP(hipStreamSynchronize(c->stream));
    sj.done();
    return rc1 != DDML_OK ? rc1 : rc2;
  });
}

int ddml_factorized_chain(ddml_ctx ctx, int gauge_id, const int* dom_ids, int ndom, const double* src, int nrhs,
                          const ddml_solver_params* params, double* out, double* steps_out, ddml_rhs_info* info,
                          int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    need(dom_ids && src && out && info, "NULL argument");
    need(ndom >= 1 && ndom <= 64, "ndom must be in 1..64");
    need(nrhs >= 1 && nrhs <= kMaxRhs, "nrhs must be in 1..12");
    check_params(params);
    for (int k = 0; k < ndom; ++k) (void)domain_get(c, dom_ids[k]);
    const size_t per = (size_t)nrhs * gauge_get(c, gauge_id).V * 12;  // complex numbers of one field
    const size_t bytes = per * sizeof(double2);
    StreamJoin sj(c, stream);
    Staged si = stage_in(c, src, bytes, on_device);
    Staged so = stage_out(c, out, bytes, on_device);
    Staged ss;
    if (steps_out) ss = stage_out(c, steps_out, bytes * ndom, on_device);
    // psi_k goes to steps_out[k] when given, else it alternates between two
    // buffers (the last step to out)
    DBuf ping, pong;
    if (!steps_out && ndom > 1) {
      ping = DBuf(c->pool.get(), bytes);
      if (ndom > 2) pong = DBuf(c->pool.get(), bytes);
    }
    DBuf rhs(c->pool.get(), ndom > 1 ? bytes : 0);
    auto dest = [&](int k) -> double* {
      if (steps_out) return ss.ptr + 2 * per * k;
      if (k == ndom - 1) return so.ptr;
      return (k % 2 ? pong : ping).as<double>();
    };
    int rc = DDML_OK;
    for (int k = 0; k < ndom; ++k) {
      const double* b = si.cptr;
      if (k > 0) {
        apply_boundary(c, gauge_id, dom_ids[k], dest(k - 1), rhs.as<double>(), nrhs, -1.0, c->stream);
        b = rhs.as<double>();
      }
      ddml_solve_desc d{gauge_id, dom_ids[k], b, dest(k), nrhs, info + (size_t)k * nrhs};
      const int r = solve_many(c, 1, &d, params, 1, c->stream);
      if (rc == DDML_OK) rc = r;
    }
    if (steps_out) {
      DDML_HIP(hipMemcpyAsync(so.ptr, ss.ptr + 2 * per * (ndom - 1), bytes, hipMemcpyDeviceToDevice, c->stream));
      copy_back(c, steps_out, ss, bytes * ndom, on_device);
    }
    copy_back(c, out, so, bytes, on_device);
    DDML_HIP(hipStreamSynchronize(c->stream));
    sj.done();
    return rc;
  });
}

int ddml_contract_pion(ddml_ctx ctx, const double* levels, int nlevels, const double* full, double* levels_out,
                       double* diffs_out, double* rest_out, int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    need(levels && levels_out && nlevels >= 1 && nlevels <= 64, "bad arguments");
    need(full || !rest_out, "rest_out needs the full propagator");
    const int T = c->lat.dims[0];
    const size_t one = (size_t)12 * c->V * 12 * sizeof(double2);
    const int np = nlevels + (full ? 1 : 0);
    StreamJoin sj(c, stream);
    Staged sl = stage_in(c, levels, one * nlevels, on_device);
    Staged sf;
    if (full) sf = stage_in(c, full, one, on_device);
    DBuf W(c->pool.get(), (size_t)np * c->V * sizeof(double2));
    DBuf sums(c->pool.get(), (size_t)np * T * sizeof(double2));
    DBuf o(c->pool.get(), (size_t)(2 * nlevels + 1) * T * sizeof(double));
    DDML_HIP(launch_pion(reinterpret_cast<const double2*>(sl.cptr), c->V, T, nlevels, W.as<double2>(),
                         sums.as<double2>(), c->stream));
    if (full)
      DDML_HIP(launch_pion(reinterpret_cast<const double2*>(sf.cptr), c->V, T, 1,
                           W.as<double2>() + (size_t)nlevels * c->V, sums.as<double2>() + (size_t)nlevels * T,
                           c->stream));
    const double invL3 = 1.0 / ((double)c->lat.dims[1] * c->lat.dims[2] * c->lat.dims[3]);
    DDML_HIP(launch_pion_fin(sums.as<double2>(), nlevels, T, full ? 1 : 0, invL3, o.as<double>(), c->stream));
    const size_t rowb = (size_t)T * sizeof(double);
    DDML_HIP(hipMemcpyAsync(levels_out, o.p, nlevels * rowb, hipMemcpyDeviceToHost, c->stream));
    if (diffs_out)
      DDML_HIP(hipMemcpyAsync(diffs_out, o.as<double>() + (size_t)nlevels * T, nlevels * rowb,
                              hipMemcpyDeviceToHost, c->stream));
    if (rest_out)
      DDML_HIP(hipMemcpyAsync(rest_out, o.as<double>() + (size_t)2 * nlevels * T, rowb, hipMemcpyDeviceToHost,
                              c->stream));
    DDML_HIP(hipStreamSynchronize(c->stream));
    sj.done();
    return DDML_OK;
  });
}

// Stochastic traces with the hopping parameter expansion: solves of gamma5 eta
// (12 sources per solve, batched), p FP64 applications of 1 - 2 kappa D_Gamma,
// and the per-slice contractions with eta before and after them.
int ddml_hpe_trace(ddml_ctx ctx, int gauge_id, int dom_id, const double* eta, int nsrc, int p,
                   const ddml_solver_params* params, double* out, double* psi_out, double* phi_out,
                   ddml_rhs_info* info, int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    need(eta && out && info, "NULL argument");
    need(nsrc >= 1, "nsrc must be >= 1");
    check_params(params);
    const GaugeRec& g = gauge_get(c, gauge_id);
    const int pmax = g.csw != 0.0 ? 2 : 8;
    need(p >= 0 && p <= pmax, "p must be in 0..8 without and 0..2 with the clover term");
    if (dom_id != -1) (void)domain_get(c, dom_id);
    const size_t V = g.V;
    const int T = g.lat.dims[0];
    const double kappa = g.kappa;
    const size_t per = V * 12;  // complex numbers of one source
    const size_t bytes = (size_t)nsrc * per * sizeof(double2);
    StreamJoin sj(c, stream);
    Staged se = stage_in(c, eta, bytes, on_device);
    DBuf g5(c->pool.get(), bytes);
    Staged sp, sf;
    if (psi_out) sp = stage_out(c, psi_out, bytes, on_device);
    else sp.buf = DBuf(c->pool.get(), bytes), sp.ptr = sp.buf.as<double>();
    if (phi_out) sf = stage_out(c, phi_out, bytes, on_device);
    else sf.buf = DBuf(c->pool.get(), bytes), sf.ptr = sf.buf.as<double>();
    DDML_HIP(launch_gamma5(reinterpret_cast<const double2*>(se.cptr), g5.as<double2>(), (size_t)nsrc * V, c->stream));
    const int rc = solve_columns(c, gauge_id, dom_id, g5.as<double>(), sp.ptr, nsrc, per, params, info);
    DBuf W(c->pool.get(), V * sizeof(double2)), sums(c->pool.get(), 2 * (size_t)T * sizeof(double2));
    DDML_HIP(launch_noise_trace(reinterpret_cast<const double2*>(se.cptr), reinterpret_cast<const double2*>(sp.ptr),
                                nsrc, V, T, W.as<double2>(), sums.as<double2>(), c->stream));
    // phi = (1 - 2 kappa D_Gamma)^p psi, 12 sources at a time
    DDML_HIP(hipMemcpyAsync(sf.ptr, sp.ptr, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (p > 0) {
      DBuf tmp(c->pool.get(), (size_t)kMaxRhs * per * sizeof(double2));
      for (int step = 0; step < p; ++step)
        for (int first = 0; first < nsrc; first += kMaxRhs) {
          const int cols = std::min(kMaxRhs, nsrc - first);
          double* ph = sf.ptr + 2 * per * first;
          apply_D(c, gauge_id, dom_id, ph, tmp.as<double>(), cols, c->stream);
          DDML_HIP(launch_axpy_d(reinterpret_cast<double2*>(ph), tmp.as<double2>(), -2.0 * kappa, (size_t)cols * per,
                                 c->stream));
        }
    }
    DDML_HIP(launch_noise_trace(reinterpret_cast<const double2*>(se.cptr), reinterpret_cast<const double2*>(sf.ptr),
                                nsrc, V, T, W.as<double2>(), sums.as<double2>() + T, c->stream));
    std::vector<double2> h(2 * (size_t)T);
    DDML_HIP(hipMemcpyAsync(h.data(), sums.p, h.size() * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
    if (psi_out) copy_back(c, psi_out, sp, bytes, on_device);
    if (phi_out) copy_back(c, phi_out, sf, bytes, on_device);
    DDML_HIP(hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < h.size(); ++k) {
      out[2 * k] = h[k].x / nsrc;
      out[2 * k + 1] = h[k].y / nsrc;
    }
    sj.done();
    return rc;
  });
}

// Time slices [t0, t1) of a domain on the gauge field's lattice.
static void slab_of(Ctx* c, const GaugeRec& g, int dom_id, int& t0, int& t1) {
  if (dom_id == -1) {
    t0 = 0;
    t1 = g.lat.dims[0];
    return;
  }
  const DomainRec& d = domain_get(c, dom_id);
  need(d.hi[0] <= g.lat.dims[0], "domain outside the gauge field's lattice");
  t0 = d.lo[0];
  t1 = d.hi[0];
}

// Subspace (inverse) iteration: v <- orth(D_Gamma^{-1} v), niter times.
int ddml_inverse_iteration(ddml_ctx ctx, int gauge_id, int dom_id, const double* start, int nvec, int niter,
                           const ddml_solver_params* params, double* out, ddml_rhs_info* info, int on_device,
                           void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    need(start && out && info, "NULL argument");
    need(nvec >= 1 && nvec <= 1024, "nvec must be in 1..1024");
    need(niter >= 1, "niter must be >= 1");
    check_params(params);
    const GaugeRec& g = gauge_get(c, gauge_id);
    int t0, t1;
    slab_of(c, g, dom_id, t0, t1);
    const size_t V = g.V, per = V * 12, V3 = V / g.lat.dims[0];
    const size_t bytes = (size_t)nvec * per * sizeof(double2);
    StreamJoin sj(c, stream);
    Staged si = stage_in(c, start, bytes, on_device);
    Staged so = stage_out(c, out, bytes, on_device);
    DBuf tmp(c->pool.get(), bytes);
    // ping-pong so that the last iterate lands in `out`
    double* bufs[2] = {so.ptr, tmp.as<double>()};
    const double* src = si.cptr;
    int rc = DDML_OK;
    for (int it = 0; it < niter; ++it) {
      double* dst = bufs[(niter - 1 - it) % 2];
      const int r = solve_columns(c, gauge_id, dom_id, src, dst, nvec, per, params, info);
      if (rc == DDML_OK) rc = r;
      orthonormalize(c, reinterpret_cast<double2*>(dst), nvec, V, (size_t)t0 * 12 * V3, (size_t)(t1 - t0) * 12 * V3);
      src = dst;
    }
    copy_back(c, out, so, bytes, on_device);
    DDML_HIP(hipStreamSynchronize(c->stream));
    sj.done();
    return rc;
  });
}

// Projector-cut connected pion: chi_j = D_Gammabar^{-1} gamma5 phi_j and
// eta_j = D_Gamma*^{-1} D_dGamma* phi_j, per-slice Gram matrices of both, and
// C(y0, x0) = -(1/L^3) Re Tr(Gt(y0) G(x0)).
int ddml_projected_pion(ddml_ctx ctx, int gauge_id, int bar_id, int star_id, const double* phi, int nvec,
                        const ddml_solver_params* params, double* out, double* gram_bar, double* gram_star,
                        ddml_rhs_info* info, int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    need(phi && out && info, "NULL argument");
    need(nvec >= 1 && nvec <= 1024, "nvec must be in 1..1024");
    check_params(params);
    const GaugeRec& g = gauge_get(c, gauge_id);
    int b0, b1, s0, s1;
    slab_of(c, g, bar_id, b0, b1);
    slab_of(c, g, star_id, s0, s1);
    const int T = g.lat.dims[0];
    const size_t V = g.V, per = V * 12;
    const size_t bytes = (size_t)nvec * per * sizeof(double2);
    const size_t gbytes = (size_t)T * nvec * nvec * sizeof(double2);
    StreamJoin sj(c, stream);
    Staged sp = stage_in(c, phi, bytes, on_device);
    DBuf src(c->pool.get(), bytes), sol(c->pool.get(), bytes);
    DBuf G(c->pool.get(), gbytes), Gt(c->pool.get(), gbytes), o(c->pool.get(), (size_t)T * T * sizeof(double));
    DDML_HIP(launch_gamma5(reinterpret_cast<const double2*>(sp.cptr), src.as<double2>(), (size_t)nvec * V, c->stream));
    int rc = solve_columns(c, gauge_id, bar_id, src.as<double>(), sol.as<double>(), nvec, per, params, info);
    gram_slices(c, sol.as<double2>(), nvec, V, T, b0, b1, G.as<double2>());
    for (int first = 0; first < nvec; first += kMaxRhs) {
      const int cols = std::min(kMaxRhs, nvec - first);
      apply_boundary(c, gauge_id, star_id, sp.cptr + 2 * per * first, src.as<double>() + 2 * per * first, cols, 1.0,
                     c->stream);
    }
    const int r = solve_columns(c, gauge_id, star_id, src.as<double>(), sol.as<double>(), nvec, per, params,
                                info + nvec);
    if (rc == DDML_OK) rc = r;
    gram_slices(c, sol.as<double2>(), nvec, V, T, s0, s1, Gt.as<double2>());
    const double invL3 = 1.0 / ((double)g.lat.dims[1] * g.lat.dims[2] * g.lat.dims[3]);
    DDML_HIP(hipMemsetAsync(o.p, 0, o.bytes, c->stream));
    DDML_HIP(launch_trace_pairs(Gt.as<double2>(), G.as<double2>(), nvec, T, s0, s1, b0, b1, -invL3, o.as<double>(),
                                c->stream));
    DDML_HIP(hipMemcpyAsync(out, o.p, o.bytes, hipMemcpyDeviceToHost, c->stream));
    if (gram_bar) DDML_HIP(hipMemcpyAsync(gram_bar, G.p, gbytes, hipMemcpyDeviceToHost, c->stream));
    if (gram_star) DDML_HIP(hipMemcpyAsync(gram_star, Gt.p, gbytes, hipMemcpyDeviceToHost, c->stream));
    DDML_HIP(hipStreamSynchronize(c->stream));
    sj.done();
    return rc;
  });
}

int ddml_projected_nucleon(ddml_ctx ctx, int gauge_id, int bar_id, int star_id, const double* phi, int nvec,
                           const ddml_solver_params* params, double* out, double* pion_out, ddml_rhs_info* info,
                           int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    need(phi && out && info, "NULL argument");
    need(nvec >= 1 && nvec <= 1024, "nvec must be in 1..1024");
    check_params(params);
    const GaugeRec& g = gauge_get(c, gauge_id);
    int b0, b1, s0, s1;
    slab_of(c, g, bar_id, b0, b1);
    slab_of(c, g, star_id, s0, s1);
    const int T = g.lat.dims[0];
    const size_t V = g.V, per = V * 12;
    const size_t bytes = (size_t)nvec * per * sizeof(double2);
    const size_t bbytes = (size_t)T * nvec * nvec * 4 * nvec * sizeof(double2);
    const double invL3 = 1.0 / ((double)g.lat.dims[1] * g.lat.dims[2] * g.lat.dims[3]);
    StreamJoin sj(c, stream);
    Staged sp = stage_in(c, phi, bytes, on_device);
    DBuf src(c->pool.get(), bytes), sol(c->pool.get(), bytes);
    DBuf Bx(c->pool.get(), bbytes), By(c->pool.get(), bbytes);
    DBuf o(c->pool.get(), (size_t)T * T * sizeof(double2));
    DBuf G, Gt, po;
    if (pion_out) {
      const size_t gbytes = (size_t)T * nvec * nvec * sizeof(double2);
      G = DBuf(c->pool.get(), gbytes);
      Gt = DBuf(c->pool.get(), gbytes);
      po = DBuf(c->pool.get(), (size_t)T * T * sizeof(double));
    }
    // chi = D_Gammabar^{-1} g5 phi; xi = conj(g5 chi)
    DDML_HIP(launch_gamma5(reinterpret_cast<const double2*>(sp.cptr), src.as<double2>(), (size_t)nvec * V, c->stream));
    int rc = solve_columns(c, gauge_id, bar_id, src.as<double>(), sol.as<double>(), nvec, per, params, info);
    bary_slices(c, sol.as<double2>(), nvec, V, T, b0, b1, 1, Bx.as<double2>());
    if (pion_out) gram_slices(c, sol.as<double2>(), nvec, V, T, b0, b1, G.as<double2>());
    // eta = D_Gamma*^{-1} D_dGamma* phi
    for (int first = 0; first < nvec; first += kMaxRhs) {
      const int cols = std::min(kMaxRhs, nvec - first);
      apply_boundary(c, gauge_id, star_id, sp.cptr + 2 * per * first, src.as<double>() + 2 * per * first, cols, 1.0,
                     c->stream);
    }
    const int r = solve_columns(c, gauge_id, star_id, src.as<double>(), sol.as<double>(), nvec, per, params,
                                info + nvec);
    if (rc == DDML_OK) rc = r;
    bary_slices(c, sol.as<double2>(), nvec, V, T, s0, s1, 0, By.as<double2>());
    DDML_HIP(hipMemsetAsync(o.p, 0, o.bytes, c->stream));
    DDML_HIP(launch_bary_pairs(By.as<double2>(), Bx.as<double2>(), nvec, T, s0, s1, b0, b1, invL3, o.as<double2>(),
                               c->stream));
    if (pion_out) {
      gram_slices(c, sol.as<double2>(), nvec, V, T, s0, s1, Gt.as<double2>());
      DDML_HIP(hipMemsetAsync(po.p, 0, po.bytes, c->stream));
      DDML_HIP(launch_trace_pairs(Gt.as<double2>(), G.as<double2>(), nvec, T, s0, s1, b0, b1, -invL3,
                                  po.as<double>(), c->stream));
      DDML_HIP(hipMemcpyAsync(pion_out, po.p, po.bytes, hipMemcpyDeviceToHost, c->stream));
    }
    DDML_HIP(hipMemcpyAsync(out, o.p, o.bytes, hipMemcpyDeviceToHost, c->stream));
    DDML_HIP(hipStreamSynchronize(c->stream));
    sj.done();
    return rc;
  });
}

int ddml_time_stencil(ddml_ctx ctx, int gauge_id, int dom_id, int nrhs, int prec, int iters, int R, int order,
                      int grid, int splits, int stage, double out[4]) {
  return guarded(ctx, [&](Ctx* c) {
    need(out != nullptr, "out is NULL");
    need(prec == DDML_FP64 || prec == DDML_MIXED_FP32 || prec == DDML_MIXED_FP16, "unknown precision");
    TuneChoice w;
    w.R = R;
    w.order = order;
    w.grid = grid;
    w.splits = splits;
    w.stage = stage;
    time_stencil(c, gauge_id, dom_id, nrhs, prec, iters, w, out);
    return DDML_OK;
  });
}

int ddml_set_launch(ddml_ctx ctx, int prec, int R, int order, int grid, int splits, int stage) {
  return guarded(ctx, [&](Ctx* c) {
    need(prec == DDML_FP64 || prec == DDML_MIXED_FP32 || prec == DDML_MIXED_FP16, "unknown precision");
    need(!c->server, "the solver graphs are rebuilt: stop the request loop first");
    TuneChoice w;
    w.R = R;
    w.order = order;
    w.grid = grid;
    w.splits = splits;
    w.stage = stage;
    set_launch(c, prec, w);
    return DDML_OK;
  });
}

int ddml_autotune(ddml_ctx ctx, int gauge_id, int dom_id, int nrhs, int prec, double best[6]) {
  return guarded(ctx, [&](Ctx* c) {
    need(best != nullptr, "best is NULL");
    need(prec == DDML_FP64 || prec == DDML_MIXED_FP32 || prec == DDML_MIXED_FP16, "unknown precision");
    need(!c->server, "the solver graphs are rebuilt: stop the request loop first");
    autotune(c, gauge_id, dom_id, nrhs, prec, best);
    return DDML_OK;
  });
}

int ddml_contract_pp_disconnected(ddml_ctx ctx, const double* terms_x, const double* terms_y, int nlevels,
                                  const int xsrc[4], const int ysrc[4], double* out, int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    need(terms_x && terms_y && xsrc && ysrc && out && nlevels >= 1, "bad arguments");
    const int* L = c->lat.dims;
    for (int m = 0; m < 4; ++m) need(xsrc[m] >= 0 && xsrc[m] < L[m] && ysrc[m] >= 0 && ysrc[m] < L[m], "bad site");
    need(nlevels <= 64, "nlevels <= 64");
    const size_t bytes = (size_t)nlevels * 12 * c->V * 12 * sizeof(double2);
    StreamJoin sj(c, stream);
    Staged sx = stage_in(c, terms_x, bytes, on_device);
    Staged sy = stage_in(c, terms_y, bytes, on_device);
    DBuf o(c->pool.get(), (size_t)nlevels * 4 * sizeof(double2));
    const size_t xs = (((size_t)xsrc[0] * L[1] + xsrc[1]) * L[2] + xsrc[2]) * L[3] + xsrc[3];
    const size_t ys = (((size_t)ysrc[0] * L[1] + ysrc[1]) * L[2] + ysrc[2]) * L[3] + ysrc[3];
    const double invL3 = 1.0 / ((double)L[1] * L[2] * L[3]);
    DDML_HIP(launch_pp(reinterpret_cast<const double2*>(sx.cptr), reinterpret_cast<const double2*>(sy.cptr), c->V,
                       nlevels, xs, ys, invL3, o.as<double2>(), c->stream));
    DDML_HIP(hipMemcpyAsync(out, o.p, (size_t)nlevels * 4 * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
    DDML_HIP(hipStreamSynchronize(c->stream));
    sj.done();
    return DDML_OK;
  });
}

int ddml_trace_g5(ddml_ctx ctx, const double* terms, int nlevels, const int xsrc[4], double* out, int on_device,
                  void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    need(terms && xsrc && out && nlevels >= 1 && nlevels <= 64, "bad arguments");
    const int* L = c->lat.dims;
    for (int m = 0; m < 4; ++m) need(xsrc[m] >= 0 && xsrc[m] < L[m], "bad site");
    const size_t bytes = (size_t)nlevels * 12 * c->V * 12 * sizeof(double2);
    StreamJoin sj(c, stream);
    Staged st = stage_in(c, terms, bytes, on_device);
    DBuf o(c->pool.get(), (size_t)nlevels * sizeof(double2));
    const size_t xs = (((size_t)xsrc[0] * L[1] + xsrc[1]) * L[2] + xsrc[2]) * L[3] + xsrc[3];
    DDML_HIP(launch_g5_traces(reinterpret_cast<const double2*>(st.cptr), c->V, nlevels, xs, o.as<double2>(),
                              c->stream));
    DDML_HIP(hipMemcpyAsync(out, o.p, (size_t)nlevels * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
    DDML_HIP(hipStreamSynchronize(c->stream));
    sj.done();
    return DDML_OK;
  });
}

int ddml_contract_nucleon(ddml_ctx ctx, const double* terms, int nlevels, double* levels_out, double* diffs_out,
                          int on_device, void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    need(terms && levels_out && nlevels >= 1 && nlevels <= 64, "bad arguments");
    const int T = c->lat.dims[0];
    const size_t bytes = (size_t)nlevels * 12 * c->V * 12 * sizeof(double2);
    StreamJoin sj(c, stream);
    Staged st = stage_in(c, terms, bytes, on_device);
    DBuf W(c->pool.get(), (size_t)nlevels * c->V * sizeof(double2));
    DBuf o(c->pool.get(), (size_t)nlevels * T * sizeof(double2));
    DBuf d(c->pool.get(), (size_t)nlevels * T * sizeof(double2));
    DDML_HIP(launch_nucleon(reinterpret_cast<const double2*>(st.cptr), c->V, T, nlevels, W.as<double2>(),
                            o.as<double2>(), c->stream));
    DDML_HIP(hipMemcpyAsync(d.p, o.p, (size_t)nlevels * T * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
    DDML_HIP(launch_series_diff(d.as<double2>(), (size_t)T, nlevels, nullptr, c->stream));
    DDML_HIP(hipMemcpyAsync(levels_out, o.p, (size_t)nlevels * T * sizeof(double2), hipMemcpyDeviceToHost,
                            c->stream));
    if (diffs_out)
      DDML_HIP(hipMemcpyAsync(diffs_out, d.p, (size_t)nlevels * T * sizeof(double2), hipMemcpyDeviceToHost,
                              c->stream));
    DDML_HIP(hipStreamSynchronize(c->stream));
    sj.done();
    return DDML_OK;
  });
}

int ddml_contract_nucleon_noalloc(ddml_ctx ctx, const double* terms, int nlevels, double* levels_out,
                                  double* diffs_out, void* stream) {
  return guarded(ctx, [&](Ctx* c) {
    need(terms && levels_out && nlevels >= 1 && nlevels <= 64, "bad arguments");
    const int T = c->lat.dims[0];
    const size_t need_scratch = (size_t)nlevels * (c->V / 8) * sizeof(double2);
    if (need_scratch > kNucScratchBytes)
      throw Error{DDML_EINVAL, "nlevels x volume too large for the allocation-free nucleon contraction (" +
                                   std::to_string(need_scratch) + " > " + std::to_string(kNucScratchBytes) +
                                   " bytes of scratch)"};
    const size_t bytes = (size_t)nlevels * 12 * c->V * 12 * sizeof(double2);
    const size_t obytes = (size_t)nlevels * T * sizeof(double2);
    need(device_span_ok(terms, bytes, c->device), "terms must be device memory holding nlevels series terms");
    need(device_span_ok(levels_out, obytes, c->device), "levels_out must be device memory of nlevels x T complex");
    need(!diffs_out || device_span_ok(diffs_out, obytes, c->device),
         "diffs_out must be device memory of nlevels x T complex");
    DDML_HIP(launch_nucleon_noalloc(reinterpret_cast<const double2*>(terms), c->V, T, nlevels,
                                    reinterpret_cast<double2*>(levels_out), reinterpret_cast<double2*>(diffs_out),
                                    c->device, static_cast<hipStream_t>(stream)));
    return DDML_OK;
  });
}

int ddml_server_start(ddml_ctx ctx, const ddml_solver_params* params, int max_queue) {
  return guarded(ctx, [&](Ctx* c) {
    check_params(params);
    need(max_queue >= 1, "max_queue >= 1");
    need(!c->server, "server already running");
    c->server.reset(new Server(c, *params, max_queue));
    return DDML_OK;
  });
}

int ddml_submit(ddml_ctx ctx, const ddml_request* req, uint64_t* ticket) {
  if (!ctx || !req || !ticket || !ctx->c.server) return DDML_EINVAL;
  if (req->nrhs < 1 || req->nrhs > kMaxRhs || !req->src || !req->sol) return DDML_EINVAL;
  // the request loop hands these to kernels: refuse host memory here, before
  // anything is queued (their extent is checked at admission, when the
  // field's volume is known)
  if (!device_span_ok(req->src, 0, ctx->c.device) || !device_span_ok(req->sol, 0, ctx->c.device))
    return DDML_EINVAL;
  return ctx->c.server->submit(*req, ticket);
}

int ddml_submit_series(ddml_ctx ctx, const ddml_series_request* req, uint64_t* ticket) {
  if (!ctx || !req || !ticket || !ctx->c.server) return DDML_EINVAL;
  if (req->nrhs < 1 || req->nrhs > kMaxRhs || !req->src || !req->terms || !req->dom_ids) return DDML_EINVAL;
  if (req->nlevels < 1 || req->nlevels > 64) return DDML_EINVAL;
  if (!device_span_ok(req->src, 0, ctx->c.device) || !device_span_ok(req->terms, 0, ctx->c.device) ||
      (req->sum && !device_span_ok(req->sum, 0, ctx->c.device)))
    return DDML_EINVAL;
  return ctx->c.server->submit_series(*req, ticket);
}

int ddml_poll(ddml_ctx ctx, uint64_t ticket, ddml_result* res) {
  if (!ctx || !ctx->c.server) return DDML_EINVAL;
  return ctx->c.server->poll(ticket, res);
}

int ddml_wait(ddml_ctx ctx, uint64_t ticket, ddml_result* res, double timeout_s) {
  if (!ctx || !ctx->c.server) return DDML_EINVAL;
  return ctx->c.server->wait(ticket, res, timeout_s);
}

int ddml_stats(ddml_ctx ctx, ddml_server_stats* stats) {
  if (!ctx || !stats || !ctx->c.server) return DDML_EINVAL;
  ctx->c.server->stats(stats);
  return DDML_OK;
}

int ddml_server_stop(ddml_ctx ctx) {
  if (!ctx || !ctx->c.server) return DDML_EINVAL;
  ctx->c.server.reset();
  return DDML_OK;
}

}  // extern "C"
