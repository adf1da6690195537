// Host engine: gauge versions, domains, operator blocks, the FP64
// defect-correction loop and the batched inner BiCGstab.
//
// Solve of D_Gamma x = b (eq. diric) in hopping units, M = 2 kappa D = A - kappa H:
//   b' = 2 kappa P_Gamma b, x = 0
//   repeat (FP64 outer loop, defect correction):
//     r = b' - M x  (FP64 stencil); stop when |r| <= tol |b'| per column
//     rhat_e = A_ee^{-1} (r_e + kappa H_eo A_oo^{-1} r_o)                (FP64)
//     solve (1 - kappa^2 A_ee^{-1} H_eo A_oo^{-1} H_oe) e_e = rhat_e       (inner, FP32 or FP64)
//     e_o = A_oo^{-1} (r_o + kappa H_oe e_e);  x += e                     (FP64)
// Many solves advance together: the inner iterations of every solve in the
// batch are one replay of a captured HIP graph over a slot table, and solves
// enter and leave the table between replays.
#include "engine.hpp"

#include <type_traits>
#include "server.hpp"
#include "tile_walk.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace ddml {

// ------------------------------------------------------------------ DevPool
DevPool::~DevPool() { trim(); }

void DevPool::trim() {
  std::lock_guard<std::mutex> lk(mu_);
  for (auto& kv : free_)
    for (void* p : kv.second) {
      (void)hipFree(p);
      sizes_.erase(p);
    }
  free_.clear();
  cached_ = 0;
}

void* DevPool::alloc(size_t bytes) {
  const size_t r = round(bytes);
  {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = free_.find(r);
    if (it != free_.end() && !it->second.empty()) {
      void* p = it->second.back();
      it->second.pop_back();
      cached_ -= r;
      in_use_ += r;
      return p;
    }
    if (in_use_ + r > budget_)
      throw Error{DDML_ENOMEM, "device memory budget exceeded (" + std::to_string(in_use_ + r) + " > " +
                                   std::to_string(budget_) + " bytes)"};
  }
  if (in_use_ + cached_ + r > budget_) trim();
  void* p = nullptr;
  if (hipMalloc(&p, r) != hipSuccess) {
    (void)hipGetLastError();
    trim();
    if (hipMalloc(&p, r) != hipSuccess) {
      (void)hipGetLastError();
      throw Error{DDML_ENOMEM, "hipMalloc of " + std::to_string(r) + " bytes failed"};
    }
  }
  std::lock_guard<std::mutex> lk(mu_);
  sizes_[p] = r;
  in_use_ += r;
  return p;
}

void DevPool::free(void* p) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = sizes_.find(p);
  if (it == sizes_.end()) return;
  free_[it->second].push_back(p);
  in_use_ -= it->second;
  cached_ += it->second;
}

bool DevPool::fits(size_t bytes) const { return in_use_ + round(bytes) <= budget_; }

bool DevPool::fits_device(size_t bytes) const {
  if (!fits(bytes)) return false;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    return true;
  }
  return fr + cached_ >= round(bytes) + ((size_t)256 << 20);  // margin for rounding of many buffers
}

// --------------------------------------------------------------- context
Ctx::~Ctx() {
  blas_release(this);
  run32.clear();
  run64.clear();
  run16.clear();
  blocks.clear();
  gauges.clear();
  flag.reset();
  if (pinned) (void)hipHostFree(pinned);
  pool.reset();
  if (stream) (void)hipStreamDestroy(stream);
}

static void* pinned_area(Ctx* c, size_t bytes) {
  if (bytes > c->pinned_bytes) {
    if (c->pinned) DDML_HIP(hipHostFree(c->pinned));
    c->pinned = nullptr;
    size_t nb = std::max<size_t>(bytes, 1 << 16);
    DDML_HIP(hipHostMalloc(&c->pinned, nb, hipHostMallocDefault));
    c->pinned_bytes = nb;
  }
  return c->pinned;
}

void ctx_init(Ctx* c, const ddml_lattice* lat, int device, size_t budget) {
  if (!lat) throw Error{DDML_EINVAL, "lattice is NULL"};
  for (int m = 0; m < 4; ++m)
    if (lat->dims[m] < 2 || lat->dims[m] % 2)
      throw Error{DDML_EINVAL, "lattice extents must be even and >= 2"};
  if (lat->bc_time != DDML_BC_PERIODIC && lat->bc_time != DDML_BC_ANTIPERIODIC && lat->bc_time != DDML_BC_OPEN)
    throw Error{DDML_EINVAL, "bc_time must be DDML_BC_PERIODIC, DDML_BC_ANTIPERIODIC or DDML_BC_OPEN"};
  int ndev = 0;
  DDML_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) throw Error{DDML_EINVAL, "no such device"};
  DDML_HIP(hipSetDevice(device));
  // the allocation-free entry points' scratch: its address on this device
  DDML_HIP(nucleon_scratch_init(device));
  c->lat = *lat;
  c->device = device;
  c->V = (size_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
  if (c->V > (size_t)1 << 30) throw Error{DDML_EINVAL, "lattice too large"};
  DDML_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    DDML_HIP(hipMemGetInfo(&fr, &tot));
    budget = (size_t)(0.9 * (double)fr);
  }
  c->pool.reset(new DevPool(budget));
  c->flag = DBuf(c->pool.get(), sizeof(int));
  c->tune16.stage = 1;  // FP32 and 16-bit fields (two-row links) are always read through the LDS staging
  c->tune32.stage = 1;
  for (int m = 0; m < 4; ++m) {
    c->full.lo[m] = 0;
    c->full.hi[m] = lat->dims[m];
  }
}

// ------------------------------------------------------------------ gauge
static void copy_in(Ctx* c, void* dst, const double* src, size_t bytes, int on_device) {
  DDML_HIP(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
}

static void check_lattice(const ddml_lattice* lat) {
  if (!lat) throw Error{DDML_EINVAL, "lattice is NULL"};
  for (int m = 0; m < 4; ++m)
    if (lat->dims[m] < 2 || lat->dims[m] % 2) throw Error{DDML_EINVAL, "lattice extents must be even and >= 2"};
  if (lat->bc_time != DDML_BC_PERIODIC && lat->bc_time != DDML_BC_ANTIPERIODIC && lat->bc_time != DDML_BC_OPEN)
    throw Error{DDML_EINVAL, "bc_time must be DDML_BC_PERIODIC, DDML_BC_ANTIPERIODIC or DDML_BC_OPEN"};
  const size_t V = (size_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
  if (V > (size_t)1 << 30) throw Error{DDML_EINVAL, "lattice too large"};
}

int gauge_new_lattice(Ctx* c, const ddml_lattice* lat, const double* U, int on_device, double kappa, double csw) {
  check_lattice(lat);
  if (!U) throw Error{DDML_EINVAL, "gauge field pointer is NULL"};
  if (!(kappa > 0) || !std::isfinite(kappa) || !std::isfinite(csw)) throw Error{DDML_EINVAL, "bad kappa or c_sw"};
  GaugeRec g;
  g.lat = *lat;
  g.V = (size_t)lat->dims[0] * lat->dims[1] * lat->dims[2] * lat->dims[3];
  const size_t bytes = g.V * 36 * sizeof(double2);
  g.base = std::make_shared<DBuf>(c->pool.get(), bytes);
  copy_in(c, g.base->p, U, bytes, on_device);
  DDML_HIP(hipStreamSynchronize(c->stream));
  g.kappa = kappa;
  g.csw = csw;
  const int id = c->next_gauge++;
  c->gauges[id] = std::move(g);
  return id;
}

int gauge_new(Ctx* c, const double* U, int on_device, double kappa, double csw) {
  return gauge_new_lattice(c, &c->lat, U, on_device, kappa, csw);
}

const GaugeRec& gauge_get(Ctx* c, int gauge_id) {
  auto it = c->gauges.find(gauge_id);
  if (it == c->gauges.end()) throw Error{DDML_EINVAL, "unknown gauge id"};
  return it->second;
}

// A new version of gauge field `base` that owns the slices [t0, t1), region
// allocated and left for the caller to fill.  It shares the parent's base
// buffer; a parent that is a version itself is materialised into a new base
// first, unless its own slices lie inside [t0, t1) (then the new region
// replaces them and `*overlay` is set to the parent, whose region holds the
// parent's values of those slices).
static GaugeRec version_of(Ctx* c, int base, int t0, int t1, const GaugeRec** overlay) {
  auto it = c->gauges.find(base);
  if (it == c->gauges.end()) throw Error{DDML_EINVAL, "unknown base gauge id"};
  const ddml_lattice& lat = it->second.lat;
  const size_t V = it->second.V;
  if (t0 < 0 || t1 > lat.dims[0] || t0 >= t1) throw Error{DDML_EINVAL, "bad time range"};
  const size_t V3 = V / lat.dims[0];
  const GaugeRec& p = it->second;
  GaugeRec g;
  g.kappa = p.kappa;
  g.csw = p.csw;
  g.lat = lat;
  g.V = V;
  *overlay = nullptr;
  if (p.region && !(p.r_t0 >= t0 && p.r_t1 <= t1)) {
    g.base = std::make_shared<DBuf>(c->pool.get(), V * 36 * sizeof(double2));
    DDML_HIP(hipMemcpyAsync(g.base->p, p.base->p, V * 36 * sizeof(double2), hipMemcpyDeviceToDevice, c->stream));
    DDML_HIP(hipMemcpyAsync(g.base->as<double2>() + (size_t)p.r_t0 * V3 * 36, p.region->p,
                            (size_t)(p.r_t1 - p.r_t0) * V3 * 36 * sizeof(double2), hipMemcpyDeviceToDevice,
                            c->stream));
  } else {
    g.base = p.base;
    if (p.region) *overlay = &p;
  }
  g.region = std::make_shared<DBuf>(c->pool.get(), (size_t)(t1 - t0) * V3 * 36 * sizeof(double2));
  g.r_t0 = t0;
  g.r_t1 = t1;
  return g;
}

int gauge_region(Ctx* c, int base, int t0, int t1, const double* U, int on_device) {
  if (!U) throw Error{DDML_EINVAL, "region pointer is NULL"};
  const GaugeRec* overlay;
  GaugeRec g = version_of(c, base, t0, t1, &overlay);
  copy_in(c, g.region->p, U, g.region->bytes, on_device);
  DDML_HIP(hipStreamSynchronize(c->stream));
  const int id = c->next_gauge++;
  c->gauges[id] = std::move(g);
  return id;
}

int gauge_level1(Ctx* c, int base, int t0, int t1, double beta, uint64_t seed, uint32_t stream, int nsweeps,
                 int n_or) {
  if (!(beta > 0) || nsweeps < 0 || n_or < 0) throw Error{DDML_EINVAL, "need beta > 0, nsweeps >= 0, n_or >= 0"};
  const GaugeRec* overlay;
  GaugeRec g = version_of(c, base, t0, t1, &overlay);
  const size_t V3 = g.V / g.lat.dims[0], link = 36 * sizeof(double2);
  // the region starts from the parent's links on [t0, t1)
  DDML_HIP(hipMemcpyAsync(g.region->p, g.base->as<double2>() + (size_t)t0 * V3 * 36, g.region->bytes,
                          hipMemcpyDeviceToDevice, c->stream));
  if (overlay)
    DDML_HIP(hipMemcpyAsync((char*)g.region->p + (size_t)(overlay->r_t0 - t0) * V3 * link, overlay->region->p,
                            (size_t)(overlay->r_t1 - overlay->r_t0) * V3 * link, hipMemcpyDeviceToDevice, c->stream));
  const GaugeView gv{g.base->as<double2>(), g.region->as<double2>(), t0, t1};
  BlockSpec bs{};
  for (int m = 0; m < 4; ++m) bs.L[m] = g.lat.dims[m];
  DDML_HIP(launch_level1_sweeps(gv, g.region->as<double2>(), bs, beta, seed, stream, nsweeps, n_or, c->stream));
  DDML_HIP(hipStreamSynchronize(c->stream));
  const int id = c->next_gauge++;
  c->gauges[id] = std::move(g);
  return id;
}

void gauge_copy_out(Ctx* c, int id, double* U, int on_device) {
  const GaugeRec& g = gauge_get(c, id);
  const size_t V3 = g.V / g.lat.dims[0], link = 36 * sizeof(double2);
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  DDML_HIP(hipMemcpyAsync(U, g.base->p, g.V * link, kind, c->stream));
  if (g.region)
    DDML_HIP(hipMemcpyAsync((char*)U + (size_t)g.r_t0 * V3 * link, g.region->p,
                            (size_t)(g.r_t1 - g.r_t0) * V3 * link, kind, c->stream));
  DDML_HIP(hipStreamSynchronize(c->stream));
}

void gauge_release(Ctx* c, int id) {
  if (!c->gauges.erase(id)) throw Error{DDML_EINVAL, "unknown gauge id"};
  for (auto it = c->blocks.begin(); it != c->blocks.end();) {
    if (it->first.first == id) it = c->blocks.erase(it);
    else ++it;
  }
}

int domain_new(Ctx* c, const int lo[4], const int hi[4]) {
  if (!lo || !hi) throw Error{DDML_EINVAL, "lo/hi is NULL"};
  DomainRec d;
  for (int m = 0; m < 4; ++m) {
    // checked against the host lattice of each gauge field it is used with
    if (lo[m] < 0 || lo[m] >= hi[m]) throw Error{DDML_EINVAL, "domain outside the lattice or empty"};
    if ((hi[m] - lo[m]) % 2) throw Error{DDML_EINVAL, "domain extents must be even"};
    d.lo[m] = lo[m];
    d.hi[m] = hi[m];
  }
  const int id = c->next_dom++;
  c->domains[id] = d;
  return id;
}

const DomainRec& domain_get(Ctx* c, int dom_id) {
  if (dom_id == -1) return c->full;
  auto it = c->domains.find(dom_id);
  if (it == c->domains.end()) throw Error{DDML_EINVAL, "unknown domain id"};
  return it->second;
}

// The domain on the gauge field's host lattice (dom_id -1: that whole lattice).
static DomainRec domain_on(Ctx* c, const GaugeRec& g, int dom_id) {
  DomainRec d;
  if (dom_id == -1) {
    for (int m = 0; m < 4; ++m) {
      d.lo[m] = 0;
      d.hi[m] = g.lat.dims[m];
    }
    return d;
  }
  d = domain_get(c, dom_id);
  for (int m = 0; m < 4; ++m)
    if (d.hi[m] > g.lat.dims[m]) throw Error{DDML_EINVAL, "domain outside the gauge field's lattice"};
  return d;
}

static void fill_spec(Ctx* c, const GaugeRec& g, const DomainRec& d, BlockSpec& bs, BoxGeom& geo) {
  (void)c;
  for (int m = 0; m < 4; ++m) {
    bs.L[m] = g.lat.dims[m];
    bs.lo[m] = d.lo[m];
    bs.Lb[m] = d.hi[m] - d.lo[m];
    geo.L[m] = bs.Lb[m];
  }
  bs.tbc = g.lat.bc_time;
  bs.kappa = g.kappa;
  bs.csw = g.csw;
  geo.Vh = bs.Lb[0] * bs.Lb[1] * bs.Lb[2] * bs.Lb[3] / 2;
  geo.half3 = bs.Lb[3] / 2;
  geo.ntiles = (geo.Vh + kTile - 1) / kTile;
  geo.twrap = (bs.Lb[0] == bs.L[0] && bs.tbc == DDML_BC_ANTIPERIODIC) ? 1 : 0;
}

static size_t opblock_bytes(size_t nsites) {  // nsites = 2 * ntiles * 64
  return DevPool::round(kLinkSlots * nsites * sizeof(double2)) + DevPool::round(kLinkSlots2 * nsites * sizeof(float2)) +
         2 * DevPool::round(kCloverSlots * nsites * sizeof(double2)) +
         DevPool::round(kCloverSlots * nsites * sizeof(float2)) + 2 * DevPool::round(sizeof(int) * nsites / 128);
}

static void evict_blocks(Ctx* c) {
  for (auto it = c->blocks.begin(); it != c->blocks.end();) {
    if (it->second.use_count() == 1) it = c->blocks.erase(it);
    else ++it;
  }
}

// Tile walk of one box for the sub-banded and quadrant orders (tile_walk.hpp),
// checked to be a permutation of the tiles.
static void build_walk(const BoxGeom& g, int tps, int nrg, int nsub, bool split_x1, int tblock,
                       std::vector<int>& walk, int xoff[kXcd + 1]) {
  if (!tile_walk(g.L, g.ntiles, tps, kTile, kXcd, nrg, nsub, split_x1, tblock, walk, xoff))
    throw Error{DDML_EDEVICE, "internal: tile walk is not a permutation"};
}

// Attaches the walk of `order` (if it uses one) to a kernel argument.
template <typename D>
static void attach_walk(D& d, const OpBlock& ob, int order) {
  if (order >= TILE_ORDER_SUB2) {
    const int w = order - TILE_ORDER_SUB2;
    d.walk = ob.walk[w].as<int>();
    for (int x = 0; x <= kXcd; ++x) d.xoff[x] = ob.xoff[w][x];
  } else {
    d.walk = nullptr;
  }
}

// Tiles XCD x walks in one box under `order` (not used by TILE_ORDER_LINEAR).
template <typename D>
static int xcd_share(const D& d, int order, int x) {
  return order == TILE_ORDER_BANDED ? band_count(d.ntiles, d.tps, x) : d.xoff[x + 1] - d.xoff[x];
}

std::shared_ptr<OpBlock> opblock(Ctx* c, int gauge_id, int dom_id) {
  auto key = std::make_pair(gauge_id, dom_id);
  auto it = c->blocks.find(key);
  if (it != c->blocks.end()) return it->second;
  auto git = c->gauges.find(gauge_id);
  if (git == c->gauges.end()) throw Error{DDML_EINVAL, "unknown gauge id"};
  const DomainRec d = domain_on(c, git->second, dom_id);
  auto ob = std::make_shared<OpBlock>();
  fill_spec(c, git->second, d, ob->bs, ob->g);
  ob->ntiles = ob->g.ntiles;
  const size_t V3h = (size_t)ob->bs.Lb[1] * ob->bs.Lb[2] * ob->bs.Lb[3] / 2;
  ob->tps = (V3h % kTile == 0) ? (int)(V3h / kTile) : 0;
  ob->field = (size_t)12 * ob->ntiles * kTile;
  const size_t ns = (size_t)2 * ob->ntiles * kTile;  // both parities, padded
  ob->bytes = opblock_bytes(ns);
  if (!c->pool->fits(ob->bytes)) evict_blocks(c);
  ob->U64 = DBuf(c->pool.get(), kLinkSlots * ns * sizeof(double2));
  ob->U32 = DBuf(c->pool.get(), kLinkSlots2 * ns * sizeof(float2));
  ob->A64 = DBuf(c->pool.get(), kCloverSlots * ns * sizeof(double2));
  ob->Ainv64 = DBuf(c->pool.get(), kCloverSlots * ns * sizeof(double2));
  ob->Ainv32 = DBuf(c->pool.get(), kCloverSlots * ns * sizeof(float2));
  for (DBuf* b : {&ob->U64, &ob->U32, &ob->A64, &ob->Ainv64, &ob->Ainv32})
    DDML_HIP(hipMemsetAsync(b->p, 0, b->bytes, c->stream));
  std::vector<int> walks[kWalks];
  for (int w = 0; w < kWalks; ++w) {
    // orders 2, 3, 4: x1 ranges split into 2 / 4 / 4 sub-bands along x2 (order 4
    // in blocks of 4 slices); order 5: regions of half the x1 rows and a quarter
    // of the tiles of a plane, 4 sub-bands along x1, blocks of 4 slices
    if (w < 3) build_walk(ob->g, ob->tps, 1, w == 0 ? 2 : 4, false, w == 2 ? 4 : 1, walks[w], ob->xoff[w]);
    else build_walk(ob->g, ob->tps, 4, 4, true, 4, walks[w], ob->xoff[w]);
    ob->walk[w] = DBuf(c->pool.get(), sizeof(int) * walks[w].size());
    DDML_HIP(hipMemcpyAsync(ob->walk[w].p, walks[w].data(), sizeof(int) * walks[w].size(), hipMemcpyHostToDevice,
                            c->stream));
  }
  GaugeView gv;
  gv.base = git->second.base->as<double2>();
  gv.region = git->second.region ? git->second.region->as<double2>() : nullptr;
  gv.r_t0 = git->second.r_t0;
  gv.r_t1 = git->second.r_t1;
  DDML_HIP(hipMemsetAsync(c->flag.p, 0, sizeof(int), c->stream));
  DDML_HIP(launch_build_links(gv, ob->bs, ob->U64.as<double2>(), ob->U32.as<float2>(), c->flag.as<int>(), c->stream));
  DDML_HIP(launch_build_clover(gv, ob->bs, ob->A64.as<double2>(), ob->Ainv64.as<double2>(), ob->Ainv32.as<float2>(),
                               c->flag.as<int>(), c->stream));
  int* hf = (int*)pinned_area(c, sizeof(int));
  DDML_HIP(hipMemcpyAsync(hf, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  DDML_HIP(hipStreamSynchronize(c->stream));
  if (*hf & 1) throw Error{DDML_ENUMERIC, "clover block not positive definite (cannot invert A)"};
  ob->su3 = !(*hf & 2);
  c->blocks[key] = ob;
  return ob;
}

// 16-bit links and A^{-1} of an operator block, built on first use.
static void ensure16(Ctx* c, OpBlock& ob) {
  if (ob.U16.p) return;
  const size_t ns = (size_t)2 * ob.ntiles * kTile;
  ob.U16 = DBuf(c->pool.get(), kLinkSlots2 * ns * sizeof(h16c));
  ob.Ainv16 = DBuf(c->pool.get(), kCloverSlots * ns * sizeof(h16c));
  ob.Ainv16n = DBuf(c->pool.get(), ns * sizeof(float));
  DDML_HIP(launch_quant_links(ob.U32.as<float2>(), ob.U16.as<h16c>(), kLinkSlots2 * ns, c->stream));
  DDML_HIP(launch_quant_clover(ob.Ainv64.as<double2>(), ob.Ainv16.as<h16c>(), ob.Ainv16n.as<float>(), ob.ntiles,
                               c->stream));
  ob.bytes += ob.U16.bytes + ob.Ainv16.bytes + ob.Ainv16n.bytes;
}

// bytes of one inner field of a solve: 16-bit values + scales, or complex FP32/FP64
static size_t inner_field_bytes(int prec, size_t n, int nrhs, size_t ntiles) {
  if (prec == DDML_MIXED_FP16) return n * sizeof(h16c) + (size_t)nrhs * ntiles * kTile * sizeof(float);
  return n * (prec == DDML_FP64 ? sizeof(double2) : sizeof(float2));
}

int gcr_len(const ddml_solver_params& prm) {
  if (prm.solver != 2) return 0;
  return prm.gcr_m > 0 ? prm.gcr_m : kGcrMax;
}

bool device_span_ok(const void* p, size_t bytes, int device) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();   // plain host memory: not an error of the stream
    return false;
  }
  if (a.type != hipMemoryTypeDevice || a.device != device) return false;
  if (bytes == 0) return true;
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  const char* b = static_cast<const char*>(base);
  const char* q = static_cast<const char*>(p);
  return q >= b && (size_t)(q - b) + bytes <= size;
}

size_t solve_footprint(Ctx* c, int gauge_id, int dom_id, int nrhs, const ddml_solver_params& prm) {
  const int prec = prm.prec, m = gcr_len(prm);
  const DomainRec d = domain_on(c, gauge_get(c, gauge_id), dom_id);
  size_t Vb = 1;
  for (int k = 0; k < 4; ++k) Vb *= (size_t)(d.hi[k] - d.lo[k]);
  const size_t Vh = Vb / 2;
  const size_t ntiles = (Vh + kTile - 1) / kTile;
  const size_t n = (size_t)nrhs * 12 * ntiles * kTile;
  const size_t fx = prec == DDML_MIXED_FP16 ? n * sizeof(float2) : inner_field_bytes(prec, n, nrhs, ntiles);
  const size_t nfield = m > 0 ? 2 + 2 * (size_t)m : F_NUM - 2;  // besides F_X (and BiCGstab's unused slot)
  const size_t npart = m > 0 ? std::max(2, m) : kBiPartials;
  return 8 * DevPool::round(n * sizeof(double2)) + nfield * DevPool::round(inner_field_bytes(prec, n, nrhs, ntiles)) +
         DevPool::round(fx) + DevPool::round(npart * nrhs * ntiles * sizeof(double2)) +
         DevPool::round(2 * nrhs * ntiles * sizeof(double2)) + 6 * DevPool::round(64);
}

// ------------------------------------------------------------ operators
static HopItem<double2> item64(const OpBlock& ob, int nrhs, int order) {
  HopItem<double2> it{};
  it.g = ob.g;
  it.U = ob.U64.as<double2>();
  it.nrhs = nrhs;
  it.ntiles = ob.ntiles;
  it.tps = ob.tps;
  attach_walk(it, ob, order);
  return it;
}

void apply_D(Ctx* c, int gauge_id, int dom_id, const double* in, double* out, int nrhs, hipStream_t st) {
  auto ob = opblock(c, gauge_id, dom_id);
  const size_t n = (size_t)nrhs * ob->field;
  DBuf xe(c->pool.get(), n * sizeof(double2)), xo(c->pool.get(), n * sizeof(double2));
  DBuf oe(c->pool.get(), n * sizeof(double2)), oo(c->pool.get(), n * sizeof(double2));
  DDML_HIP(hipMemsetAsync(xe.p, 0, xe.bytes, st));
  DDML_HIP(hipMemsetAsync(xo.p, 0, xo.bytes, st));
  const double2* cin = reinterpret_cast<const double2*>(in);
  double2* cout = reinterpret_cast<double2*>(out);
  DDML_HIP(launch_gather(cin, ob->bs, 0, nrhs, 1.0, xe.as<double2>(), st));
  DDML_HIP(launch_gather(cin, ob->bs, 1, nrhs, 1.0, xo.as<double2>(), st));
  const double kappa = ob->bs.kappa;
  for (int p = 0; p < 2; ++p) {
    HopItem<double2> it = item64(*ob, nrhs, c->tune64.order);
    it.clov = ob->A64.as<double2>();
    it.in = p == 0 ? xo.as<double2>() : xe.as<double2>();
    it.aux = p == 0 ? xe.as<double2>() : xo.as<double2>();
    it.out = p == 0 ? oe.as<double2>() : oo.as<double2>();
    it.par_out = p;
    it.c1 = kappa;
    it.c2 = 1.0 / (2.0 * kappa);
    DDML_HIP(launch_hop_item(it, MODE_M, RED_NONE, 1, c->tune64.order, st));
  }
  DDML_HIP(hipMemsetAsync(out, 0, (size_t)nrhs * gauge_get(c, gauge_id).V * 12 * sizeof(double2), st));
  DDML_HIP(launch_scatter(oe.as<double2>(), ob->bs, 0, nrhs, 1.0, cout, st));
  DDML_HIP(launch_scatter(oo.as<double2>(), ob->bs, 1, nrhs, 1.0, cout, st));
  DDML_HIP(hipStreamSynchronize(st));  // temporaries go back to the pool
}

// Couplings of D from outside a domain into it; no operator block is needed:
// the kernel reads the canonical links of the gauge field directly.
void apply_boundary(Ctx* c, int gauge_id, int dom_id, const double* in, double* out, int nrhs, double scale,
                    hipStream_t st) {
  const GaugeRec& g = gauge_get(c, gauge_id);
  const DomainRec d = domain_on(c, g, dom_id);
  BlockSpec bs{};
  BoxGeom geo{};
  fill_spec(c, g, d, bs, geo);
  GaugeView gv;
  gv.base = g.base->as<double2>();
  gv.region = g.region ? g.region->as<double2>() : nullptr;
  gv.r_t0 = g.r_t0;
  gv.r_t1 = g.r_t1;
  DDML_HIP(launch_boundary(gv, bs, reinterpret_cast<const double2*>(in), reinterpret_cast<double2*>(out), nrhs, scale,
                           st));
}

template <typename T2>
static void schur_apply(Ctx* c, const OpBlock& ob, const T2* U, const T2* Ainv, const T2* xe, T2* tmp, T2* oe,
                        int nrhs, hipStream_t st) {
  const TuneChoice& tn = c->tune(sizeof(T2) == sizeof(double2) ? DDML_FP64 : DDML_MIXED_FP32);
  HopItem<T2> it{};
  it.g = ob.g;
  it.U = U;
  it.clov = Ainv;
  it.nrhs = nrhs;
  it.ntiles = ob.ntiles;
  it.tps = ob.tps;
  attach_walk(it, ob, tn.order);
  it.in = xe;
  it.out = tmp;
  it.par_out = 1;
  DDML_HIP(launch_hop_item(it, MODE_CINV_HOP, RED_NONE, tn.R, tn.order, st));
  it.in = tmp;
  it.aux = xe;
  it.out = oe;
  it.par_out = 0;
  it.c1 = ob.bs.kappa * ob.bs.kappa;
  DDML_HIP(launch_hop_item(it, MODE_SCHUR, RED_NONE, tn.R, tn.order, st));
}

// The Schur operator in FP32 or 16-bit storage (input rounded or quantised,
// both half-stencils through the batched kernels on a one-slot table, output
// read back to FP64).
template <typename T2>
static void schur_apply_staged(Ctx* c, OpBlock& ob, const double2* xe, double2* oe, int nrhs, hipStream_t st) {
  constexpr bool h16 = std::is_same<T2, h16c>::value;
  const int prec = h16 ? DDML_MIXED_FP16 : DDML_MIXED_FP32;
  if (h16) ensure16(c, ob);
  const TuneChoice& tn = c->tune(prec);
  const size_t n = (size_t)nrhs * ob.field, nt = ob.ntiles;
  const size_t fb = inner_field_bytes(prec, n, nrhs, nt);
  DevPool* P = c->pool.get();
  DBuf fx(P, fb), ft(P, fb), fo(P, fb);
  DBuf part(P, 2 * nrhs * nt * sizeof(double2)), act(P, kMaxRhs * sizeof(int));
  DBuf tab(P, sizeof(SlotDesc<T2>)), ts(P, 2 * sizeof(int)), ns(P, sizeof(int)), xs(P, kXcd * 2 * sizeof(int));
  auto scales = [&](DBuf& b) { return reinterpret_cast<float*>(b.as<h16c>() + n); };
  SlotDesc<T2> d{};
  d.g = ob.g;
  d.nrhs = nrhs;
  d.ntiles = ob.ntiles;
  d.tps = ob.tps;
  d.kappa = ob.bs.kappa;
  d.f[F_P] = fx.as<T2>();
  d.f[F_TMP] = ft.as<T2>();
  d.f[F_V] = fo.as<T2>();
  if constexpr (h16) {
    DDML_HIP(launch_quant16(xe, fx.as<h16c>(), scales(fx), nrhs, (int)nt, st));
    d.U = ob.U16.as<h16c>();
    d.Ainv = ob.Ainv16.as<h16c>();
    d.Ainv_nrm = ob.Ainv16n.as<float>();
    d.nrm[F_P] = scales(fx);
    d.nrm[F_TMP] = scales(ft);
    d.nrm[F_V] = scales(fo);
  } else {
    DDML_HIP(launch_cast_to_f(xe, fx.as<float2>(), n, st));
    d.U = ob.U32.as<float2>();
    d.Ainv = ob.Ainv32.as<float2>();
  }
  std::vector<int> ones(kMaxRhs, 1);
  DDML_HIP(hipMemcpyAsync(act.p, ones.data(), kMaxRhs * sizeof(int), hipMemcpyHostToDevice, st));
  d.partial = part.as<double2>();
  d.active = act.as<int>();
  attach_walk(d, ob, tn.order);
  int h_ts[2] = {0, ob.ntiles}, one = 1, h_xs[kXcd * 2];
  for (int x = 0; x < kXcd; ++x) {
    h_xs[2 * x] = 0;
    h_xs[2 * x + 1] = tn.order == TILE_ORDER_LINEAR ? 0 : xcd_share(d, tn.order, x);
  }
  DDML_HIP(hipMemcpyAsync(tab.p, &d, sizeof(d), hipMemcpyHostToDevice, st));
  DDML_HIP(hipMemcpyAsync(ts.p, h_ts, sizeof(h_ts), hipMemcpyHostToDevice, st));
  DDML_HIP(hipMemcpyAsync(ns.p, &one, sizeof(int), hipMemcpyHostToDevice, st));
  DDML_HIP(hipMemcpyAsync(xs.p, h_xs, sizeof(h_xs), hipMemcpyHostToDevice, st));
  const int grid = ((tn.grid + kXcd - 1) / kXcd) * kXcd;
  const int splits = std::min(tn.splits, (nrhs + tn.R - 1) / tn.R);
  auto* tb = tab.as<SlotDesc<T2>>();
  DDML_HIP(launch_hop_batch(tb, ts.as<int>(), xs.as<int>(), 2, ns.as<int>(), nrhs, tn.R, MODE_CINV_HOP, RED_NONE, F_P,
                            -1, F_TMP, -1, 1, grid, tn.order, splits, 1, st));
  // (with the fused shadow dot, the variant every element type has; its partial sums are not used here)
  DDML_HIP(launch_hop_batch(tb, ts.as<int>(), xs.as<int>(), 2, ns.as<int>(), nrhs, tn.R, MODE_SCHUR, RED_DOT, F_TMP,
                            F_P, F_V, -1, 0, grid, tn.order, splits, 1, st));
  if constexpr (h16) DDML_HIP(launch_dequant16(fo.as<h16c>(), scales(fo), oe, nrhs, (int)nt, st));
  else DDML_HIP(launch_cast_to_d(fo.as<float2>(), oe, n, st));
  DDML_HIP(hipStreamSynchronize(st));  // temporaries go back to the pool
}

void apply_eo(Ctx* c, int gauge_id, int dom_id, const double* in, double* out, int nrhs, int prec, hipStream_t st) {
  auto ob = opblock(c, gauge_id, dom_id);
  const size_t n = (size_t)nrhs * ob->field;
  DBuf xe(c->pool.get(), n * sizeof(double2)), oe(c->pool.get(), n * sizeof(double2));
  DDML_HIP(hipMemsetAsync(xe.p, 0, xe.bytes, st));
  DDML_HIP(launch_gather(reinterpret_cast<const double2*>(in), ob->bs, 0, nrhs, 1.0, xe.as<double2>(), st));
  if (prec == DDML_FP64) {
    DBuf tmp(c->pool.get(), n * sizeof(double2));
    schur_apply<double2>(c, *ob, ob->U64.as<double2>(), ob->Ainv64.as<double2>(), xe.as<double2>(),
                         tmp.as<double2>(), oe.as<double2>(), nrhs, st);
    DDML_HIP(hipMemsetAsync(out, 0, (size_t)nrhs * gauge_get(c, gauge_id).V * 12 * sizeof(double2), st));
    DDML_HIP(launch_scatter(oe.as<double2>(), ob->bs, 0, nrhs, 1.0, reinterpret_cast<double2*>(out), st));
    DDML_HIP(hipStreamSynchronize(st));
  } else {
    if (!ob->su3)
      throw Error{DDML_EINVAL, "the FP32 and 16-bit operator copies keep two rows per link and need SU(3) links"};
    if (prec == DDML_MIXED_FP16) schur_apply_staged<h16c>(c, *ob, xe.as<double2>(), oe.as<double2>(), nrhs, st);
    else schur_apply_staged<float2>(c, *ob, xe.as<double2>(), oe.as<double2>(), nrhs, st);
    DDML_HIP(hipMemsetAsync(out, 0, (size_t)nrhs * gauge_get(c, gauge_id).V * 12 * sizeof(double2), st));
    DDML_HIP(launch_scatter(oe.as<double2>(), ob->bs, 0, nrhs, 1.0, reinterpret_cast<double2*>(out), st));
    DDML_HIP(hipStreamSynchronize(st));
  }
}

// ----------------------------------------------------------- batch runner
template <typename T2>
BatchRunner<T2>::~BatchRunner() {
  if (exec) (void)hipGraphExecDestroy(exec);
  for (int k = 0; k < 2; ++k) {
    if (ev[k]) {
      (void)hipEventSynchronize(ev[k]);
      (void)hipEventDestroy(ev[k]);
    }
    if (pin_up[k]) (void)hipHostFree(pin_up[k]);
    if (pin_rb[k]) (void)hipHostFree(pin_rb[k]);
  }
}

// Byte layout of a device-loop table upload: slot table, the four FP64 view
// tables, tile starts, XCD tile starts, slot count.
template <typename T2>
static size_t up_layout(int max_slots, size_t off[5]) {
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  off[0] = 0;
  off[1] = off[0] + al(sizeof(SlotDesc<T2>) * max_slots);
  off[2] = off[1] + al(sizeof(SlotDesc<double2>) * 4 * max_slots);
  off[3] = off[2] + al(sizeof(int) * (max_slots + 1));
  off[4] = off[3] + al(sizeof(int) * kXcd * (max_slots + 1));
  return off[4] + al(sizeof(int));
}

template <typename T2>
void BatchRunner<T2>::init(Ctx* c, int nrhs_, const TuneChoice& tn, int max_slots_, int gcr_m_) {
  ctx = c;
  nrhs = nrhs_;
  gcr_m = gcr_m_;
  R = tn.R;
  K = tn.K;
  grid = ((tn.grid + kXcd - 1) / kXcd) * kXcd;
  max_slots = max_slots_;
  order = tn.order;
  splits = std::min(tn.splits, (nrhs + R - 1) / R);
  stage = tn.stage;
  table = DBuf(c->pool.get(), sizeof(SlotDesc<T2>) * max_slots);
  tstart = DBuf(c->pool.get(), sizeof(int) * (max_slots + 1));
  xstart = DBuf(c->pool.get(), sizeof(int) * kXcd * (max_slots + 1));
  nslots = DBuf(c->pool.get(), sizeof(int));
  st_all = DBuf(c->pool.get(), sizeof(BiState) * max_slots * kMaxRhs);
  act_all = DBuf(c->pool.get(), sizeof(int) * max_slots * kMaxRhs);
  if (gcr_m > 0) gc_all = DBuf(c->pool.get(), sizeof(double2) * max_slots * kMaxRhs * 2 * kGcrMax);
  device = gcr_m == 0;
  if (device) {
    sst_all = DBuf(c->pool.get(), sizeof(SlotState) * max_slots);
    ost_all = DBuf(c->pool.get(), sizeof(OuterState) * max_slots * kMaxRhs);
    oflag_all = DBuf(c->pool.get(), sizeof(int) * max_slots * 3 * kMaxRhs);
    views = DBuf(c->pool.get(), sizeof(SlotDesc<double2>) * 4 * max_slots);
    h_views.assign((size_t)4 * max_slots, SlotDesc<double2>{});
    size_t off[5];
    up_bytes = up_layout<T2>(max_slots, off);
    rb_bytes = sizeof(SlotState) * max_slots + sizeof(OuterState) * max_slots * kMaxRhs;
    for (int k = 0; k < 2; ++k) {
      DDML_HIP(hipHostMalloc(&pin_up[k], up_bytes, hipHostMallocDefault));
      DDML_HIP(hipHostMalloc(&pin_rb[k], rb_bytes, hipHostMallocDefault));
      DDML_HIP(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming));
      snap[k].assign(max_slots, 0);
    }
    DDML_HIP(launch_outer_reset(sst_all.as<SlotState>(), ost_all.as<OuterState>(), act_all.as<int>(),
                                oflag_all.as<int>(), max_slots, PH_IDLE, c->stream));
  }
  SlotDesc<T2> empty{};
  h_table.assign(max_slots, empty);
  h_tstart.assign(max_slots + 1, 0);
  slot_of.assign(max_slots, nullptr);
  gen_of.assign(max_slots, 0);
  h_st.assign((size_t)max_slots * kMaxRhs, BiState{});
  DDML_HIP(hipMemsetAsync(act_all.p, 0, sizeof(int) * max_slots * kMaxRhs, c->stream));
  nused = 0;
  dirty = true;
  upload();
  capture();
}

template <typename T2>
void BatchRunner<T2>::capture() {
  hipStream_t s = ctx->stream;
  const auto* tb = table.as<SlotDesc<T2>>();
  const int* ts = tstart.as<int>();
  const int* xs = xstart.as<int>();
  const int xw = max_slots + 1;
  const int* ns = nslots.as<int>();
  DDML_HIP(hipStreamSynchronize(s));
  hipGraph_t graph = nullptr;
  DDML_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  // a launcher that rejects its arguments returns an error without touching
  // the stream: keep the first one and fail after the capture is closed
  hipError_t first = hipSuccess;
  auto chk = [&](hipError_t r) { if (first == hipSuccess && r != hipSuccess) first = r; };
  if (device) {
    // the FP64 outer step of every slot that needs one (flags set by the gate)
    const auto* vw = views.as<SlotDesc<double2>>();
    const SlotDesc<double2>* vexp = vw;
    const SlotDesc<double2>* vres0 = vw + max_slots;
    const SlotDesc<double2>* vres1 = vw + 2 * max_slots;
    const SlotDesc<double2>* vprep = vw + 3 * max_slots;
    auto outer = [&](int step) { chk(launch_outer(tb, ts, ns, max_slots, nrhs, step, grid, s)); };
    outer(OUTER_GATE);
    // export: t_e = x, t_o = A_oo^{-1}(r_o + kappa H_oe t_e), x += t
    outer(OUTER_CAST);
    chk(launch_hop_batch(vexp, ts, xs, xw, ns, nrhs, 1, MODE_PREP, RED_NONE, O_TE, O_RO, O_TO, -1, 1, grid, order, 1,
                         1, s));
    outer(OUTER_AXPY);
    // r = b' - M x on both parities with |r|^2 partials
    chk(launch_hop_batch(vres0, ts, xs, xw, ns, nrhs, 1, MODE_RES, RED_NORM, O_XO, O_XE, O_RE, O_BE, 0, grid, order,
                         1, 1, s));
    chk(launch_hop_batch(vres1, ts, xs, xw, ns, nrhs, 1, MODE_RES, RED_NORM, O_XE, O_XO, O_RO, O_BO, 1, grid, order,
                         1, 1, s));
    outer(OUTER_DECIDE);
    outer(OUTER_PHASE);
    // rhat_e = A_ee^{-1}(r_e + kappa H_eo A_oo^{-1} r_o), then the inner initialisation
    outer(OUTER_CLOVER);
    chk(launch_hop_batch(vprep, ts, xs, xw, ns, nrhs, 1, MODE_PREP, RED_NONE, O_TO, O_RE, O_TE, -1, 0, grid, order, 1,
                         1, s));
    chk(launch_vec(tb, ts, ns, nrhs, VEC_INIT, grid, s));
    chk(launch_fin(tb, ns, max_slots, FIN_INIT, s));
    chk(launch_vec(tb, ts, ns, nrhs, VEC_RELUP, grid, s));
    chk(launch_fin(tb, ns, max_slots, FIN_RELUP, s));
    chk(launch_vec(tb, ts, ns, nrhs, VEC_PFIX, grid, s));
    outer(OUTER_COMMIT);
  }
  if constexpr (!std::is_same<T2, h16c>::value) {
    // one GCR(m) cycle: step k applies M to p_k, orthogonalises against the
    // cycle's earlier directions and updates x, r and the next direction
    for (int k = 0; k < gcr_m; ++k) {
      chk(launch_hop_batch(tb, ts, xs, xw, ns, nrhs, R, MODE_CINV_HOP, RED_NONE, F_GP0 + k, -1, F_TMP, -1, 1, grid,
                           order, splits, stage, s));
      chk(launch_hop_batch(tb, ts, xs, xw, ns, nrhs, R, MODE_SCHUR, RED_NONE, F_TMP, F_GP0 + k, F_GQ0 + k, -1, 0,
                           grid, order, splits, stage, s));
      if (k > 0) {
        chk(launch_gcr(tb, ts, ns, nrhs, GCR_DOTS, k, gcr_m, grid, s));
        chk(launch_gcr_fin(tb, ns, max_slots, GFIN_BETA, k, s));
      }
      chk(launch_gcr(tb, ts, ns, nrhs, GCR_UPDATE, k, gcr_m, grid, s));
      chk(launch_gcr_fin(tb, ns, max_slots, GFIN_ALPHA, k, s));
      chk(launch_gcr(tb, ts, ns, nrhs, GCR_XR, k, gcr_m, grid, s));
      chk(launch_gcr_fin(tb, ns, max_slots, GFIN_CHECK, k, s));
    }
  }
  // BiCGstab iterations (the direction p of the next iteration is formed by
  // VEC_XRP of this one, and by the (re)initialisation for the first)
  for (int k = 0; k < (gcr_m > 0 ? 0 : K); ++k) {
    chk(launch_hop_batch(tb, ts, xs, xw, ns, nrhs, R, MODE_CINV_HOP, RED_NONE, F_P, -1, F_TMP, -1, 1, grid, order,
                         splits, stage, s));
    chk(launch_hop_batch(tb, ts, xs, xw, ns, nrhs, R, MODE_SCHUR, RED_DOT, F_TMP, F_P, F_V, -1, 0, grid, order,
                         splits, stage, s));
    chk(launch_fin(tb, ns, max_slots, FIN_ALPHA, s));
    chk(launch_vec(tb, ts, ns, nrhs, VEC_S, grid, s));
    chk(launch_hop_batch(tb, ts, xs, xw, ns, nrhs, R, MODE_CINV_HOP, RED_NONE, F_S, -1, F_TMP, -1, 1, grid, order,
                         splits, stage, s));
    chk(launch_hop_batch(tb, ts, xs, xw, ns, nrhs, R, MODE_SCHUR, RED_TS, F_TMP, F_S, F_T, -1, 0, grid, order,
                         splits, stage, s));
    chk(launch_fin(tb, ns, max_slots, FIN_OMEGA, s));
    chk(launch_vec(tb, ts, ns, nrhs, VEC_XRP, grid, s));
    chk(launch_fin(tb, ns, max_slots, FIN_CHECK, s));
  }
  hipError_t e = hipStreamEndCapture(s, &graph);
  if (e != hipSuccess) throw Error{DDML_EDEVICE, std::string("graph capture failed: ") + hipGetErrorString(e)};
  if (first != hipSuccess) {
    (void)hipGraphDestroy(graph);
    throw Error{DDML_EDEVICE, std::string("launch in capture rejected: ") + hipGetErrorString(first)};
  }
  e = hipGetLastError();
  if (e != hipSuccess) throw Error{DDML_EDEVICE, std::string("launch in capture failed: ") + hipGetErrorString(e)};
  if (exec) (void)hipGraphExecDestroy(exec);
  exec = nullptr;
  DDML_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  DDML_HIP(hipGraphDestroy(graph));
}

template <typename T2>
int BatchRunner<T2>::members() const {
  int n = 0;
  for (auto* s : slot_of) n += s != nullptr;
  return n;
}

template <typename T2>
static SlotDesc<T2> make_desc(const Solve* s, BiState* st, int* act, int order);

template <>
SlotDesc<float2> make_desc<float2>(const Solve* s, BiState* st, int* act, int order) {
  SlotDesc<float2> d{};
  d.g = s->ob->g;
  d.nrhs = s->nrhs;
  d.ntiles = s->ob->ntiles;
  d.tps = s->ob->tps;
  d.kappa = s->ob->bs.kappa;
  d.U = s->ob->U32.as<float2>();
  d.Ainv = s->ob->Ainv32.as<float2>();
  for (int k = 0; k < F_ALL; ++k) d.f[k] = s->f[k].as<float2>();
  d.partial = s->partial.as<double2>();
  d.active = act;
  d.st = st;
  d.src64 = s->te.as<double2>();
  attach_walk(d, *s->ob, order);
  return d;
}
template <>
SlotDesc<double2> make_desc<double2>(const Solve* s, BiState* st, int* act, int order) {
  SlotDesc<double2> d{};
  d.g = s->ob->g;
  d.nrhs = s->nrhs;
  d.ntiles = s->ob->ntiles;
  d.tps = s->ob->tps;
  d.kappa = s->ob->bs.kappa;
  d.U = s->ob->U64.as<double2>();
  d.Ainv = s->ob->Ainv64.as<double2>();
  for (int k = 0; k < F_ALL; ++k) d.f[k] = s->f[k].as<double2>();
  d.partial = s->partial.as<double2>();
  d.active = act;
  d.st = st;
  d.src64 = s->te.as<double2>();
  attach_walk(d, *s->ob, order);
  return d;
}

template <>
SlotDesc<h16c> make_desc<h16c>(const Solve* s, BiState* st, int* act, int order) {
  SlotDesc<h16c> d{};
  const OpBlock& ob = *s->ob;
  const size_t n = (size_t)s->nrhs * ob.field;
  d.g = ob.g;
  d.nrhs = s->nrhs;
  d.ntiles = ob.ntiles;
  d.tps = ob.tps;
  d.kappa = ob.bs.kappa;
  d.U = ob.U16.as<h16c>();
  d.Ainv = ob.Ainv16.as<h16c>();
  d.Ainv_nrm = ob.Ainv16n.as<float>();
  for (int k = 0; k < F_NUM; ++k) {
    if (k == F_X || k == F_UNUSED) continue;
    d.f[k] = s->f[k].as<h16c>();
    d.nrm[k] = reinterpret_cast<float*>(d.f[k] + n);
  }
  d.x32 = s->f[F_X].as<float2>();
  d.partial = s->partial.as<double2>();
  d.active = act;
  d.st = st;
  d.src64 = s->te.as<double2>();
  attach_walk(d, ob, order);
  return d;
}

// FP64 view of a solve's outer fields for the batched stencil: f[O_*] are
// b'_e, b'_o, x_e, x_o, r_e, r_o, t_e, t_o; clov is the clover data the
// epilogue applies (A for the residual, A^{-1} otherwise).
static SlotDesc<double2> view64(const Solve* s, int order, int* act, const double2* clov, double2* partial) {
  const OpBlock& ob = *s->ob;
  SlotDesc<double2> d{};
  d.g = ob.g;
  d.nrhs = s->nrhs;
  d.ntiles = ob.ntiles;
  d.tps = ob.tps;
  d.kappa = ob.bs.kappa;
  d.U = ob.U64.as<double2>();
  d.Ainv = clov;
  d.A = clov;
  const DBuf* o[8] = {&s->be, &s->bo, &s->xe, &s->xo, &s->re, &s->ro, &s->te, &s->to};
  for (int k = 0; k < 8; ++k) d.f[k] = o[k]->as<double2>();
  d.partial = partial;
  d.active = act;
  attach_walk(d, ob, order);
  return d;
}

template <typename T2>
bool BatchRunner<T2>::has_free() const {
  for (int i = 0; i < max_slots; ++i)
    if (!slot_of[i]) return true;
  return false;
}

template <typename T2>
int BatchRunner<T2>::join(Solve* s) {
  int slot = -1;
  for (int i = 0; i < max_slots; ++i)
    if (!slot_of[i]) { slot = i; break; }
  if (slot < 0) return -1;
  BiState* st = st_all.as<BiState>() + (size_t)slot * kMaxRhs;
  int* act = act_all.as<int>() + (size_t)slot * kMaxRhs;
  SlotDesc<T2> d = make_desc<T2>(s, st, act, order);
  if (gcr_m > 0) d.gcoef = gc_all.template as<double2>() + (size_t)slot * kMaxRhs * 2 * kGcrMax;
  if (device) {
    const OpBlock& ob = *s->ob;
    SlotState* sst = sst_all.as<SlotState>() + slot;
    OuterState* ost = ost_all.as<OuterState>() + (size_t)slot * kMaxRhs;
    int* ofl = oflag_all.as<int>() + (size_t)slot * 3 * kMaxRhs;
    d.sst = sst;
    d.ost = ost;
    d.oflag = ofl;
    const DBuf* o[8] = {&s->be, &s->bo, &s->xe, &s->xo, &s->re, &s->ro, &s->te, &s->to};
    for (int k = 0; k < 8; ++k) d.o64[k] = o[k]->as<double2>();
    d.Ainv64 = ob.Ainv64.as<double2>();
    d.partial64 = s->partial64.as<double2>();
    d.tol = s->prm.tol;
    d.inner_tol = s->prm.inner_tol;
    d.max_outer = s->prm.max_outer;
    d.max_inner = s->prm.max_inner;
    d.prec = s->prec;
    d.solver = s->prm.solver;
    const size_t half = (size_t)s->nrhs * ob.ntiles;
    double2* p64 = s->partial64.as<double2>();
    h_views[slot] = view64(s, order, ofl + OF_EXPORT * s->nrhs, ob.Ainv64.as<double2>(), nullptr);
    h_views[max_slots + slot] = view64(s, order, ofl + OF_RESID * s->nrhs, ob.A64.as<double2>(), p64);
    h_views[2 * max_slots + slot] = view64(s, order, ofl + OF_RESID * s->nrhs, ob.A64.as<double2>(), p64 + half);
    h_views[3 * max_slots + slot] = view64(s, order, ofl + OF_PREP * s->nrhs, ob.Ainv64.as<double2>(), nullptr);
    // the slot starts at PH_NEW with cleared outer state and flags
    DDML_HIP(launch_outer_reset(sst, ost, act, ofl, 1, PH_NEW, ctx->stream));
    s->dev = true;
  }
  h_table[slot] = d;
  slot_of[slot] = s;
  gen_of[slot] = ++joins;
  s->slot = slot;
  dirty = true;
  return slot;
}

template <typename T2>
void BatchRunner<T2>::leave(Solve* s) {
  if (s->slot < 0) return;
  h_table[s->slot] = SlotDesc<T2>{};
  if (device)
    for (int v = 0; v < 4; ++v) h_views[(size_t)v * max_slots + s->slot] = SlotDesc<double2>{};
  slot_of[s->slot] = nullptr;
  gen_of[s->slot] = 0;
  s->slot = -1;
  dirty = true;
}

template <typename T2>
void BatchRunner<T2>::upload() {
  nused = 0;
  for (int i = 0; i < max_slots; ++i)
    if (slot_of[i]) nused = i + 1;
  h_tstart[0] = 0;
  for (int i = 0; i < max_slots; ++i) h_tstart[i + 1] = h_tstart[i] + (slot_of[i] ? h_table[i].ntiles : 0);
  h_xstart.assign((size_t)kXcd * (max_slots + 1), 0);
  for (int x = 0; x < kXcd; ++x) {
    int* P = h_xstart.data() + (size_t)x * (max_slots + 1);
    for (int i = 0; i < max_slots; ++i)
      P[i + 1] = P[i] + (slot_of[i] && order != TILE_ORDER_LINEAR ? xcd_share(h_table[i], order, x) : 0);
  }
  if (device) {
    // through pinned staging, so that the copies stay asynchronous; the
    // buffer of this ring position was last read by the replay before the
    // previous one, which the host has already waited for
    size_t off[5];
    up_layout<T2>(max_slots, off);
    char* h = static_cast<char*>(pin_up[ring]);
    std::memcpy(h + off[0], h_table.data(), sizeof(SlotDesc<T2>) * max_slots);
    std::memcpy(h + off[1], h_views.data(), sizeof(SlotDesc<double2>) * 4 * max_slots);
    std::memcpy(h + off[2], h_tstart.data(), sizeof(int) * (max_slots + 1));
    std::memcpy(h + off[3], h_xstart.data(), sizeof(int) * h_xstart.size());
    std::memcpy(h + off[4], &nused, sizeof(int));
    hipStream_t st = ctx->stream;
    DDML_HIP(hipMemcpyAsync(table.p, h + off[0], sizeof(SlotDesc<T2>) * max_slots, hipMemcpyHostToDevice, st));
    DDML_HIP(hipMemcpyAsync(views.p, h + off[1], sizeof(SlotDesc<double2>) * 4 * max_slots, hipMemcpyHostToDevice,
                            st));
    DDML_HIP(hipMemcpyAsync(tstart.p, h + off[2], sizeof(int) * (max_slots + 1), hipMemcpyHostToDevice, st));
    DDML_HIP(hipMemcpyAsync(xstart.p, h + off[3], sizeof(int) * h_xstart.size(), hipMemcpyHostToDevice, st));
    DDML_HIP(hipMemcpyAsync(nslots.p, h + off[4], sizeof(int), hipMemcpyHostToDevice, st));
    dirty = false;
    return;
  }
  DDML_HIP(hipMemcpyAsync(table.p, h_table.data(), sizeof(SlotDesc<T2>) * max_slots, hipMemcpyHostToDevice,
                          ctx->stream));
  DDML_HIP(hipMemcpyAsync(tstart.p, h_tstart.data(), sizeof(int) * (max_slots + 1), hipMemcpyHostToDevice,
                          ctx->stream));
  DDML_HIP(hipMemcpyAsync(xstart.p, h_xstart.data(), sizeof(int) * h_xstart.size(), hipMemcpyHostToDevice,
                          ctx->stream));
  DDML_HIP(hipMemcpyAsync(nslots.p, &nused, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
  dirty = false;
}

template <typename T2>
void BatchRunner<T2>::replay() {
  if (dirty) upload();
  DDML_HIP(hipGraphLaunch(exec, ctx->stream));
  const size_t nb = sizeof(BiState) * (size_t)std::max(nused, 1) * kMaxRhs;
  BiState* hs = (BiState*)pinned_area(ctx, nb);
  DDML_HIP(hipMemcpyAsync(hs, st_all.p, nb, hipMemcpyDeviceToHost, ctx->stream));
  DDML_HIP(hipStreamSynchronize(ctx->stream));
  std::memcpy(h_st.data(), hs, nb);
}

template <typename T2>
void BatchRunner<T2>::launch_dev() {
  hipStream_t st = ctx->stream;
  // this ring position's pinned buffers are reused below: its readback must
  // have been taken (two launches in a row, e.g. from two callers)
  if (pending[ring]) collect_dev();   // collects position `ring`
  if (dirty) upload();
  DDML_HIP(hipGraphLaunch(exec, st));
  const int n = std::max(nused, 1);
  char* h = static_cast<char*>(pin_rb[ring]);
  DDML_HIP(hipMemcpyAsync(h, sst_all.p, sizeof(SlotState) * n, hipMemcpyDeviceToHost, st));
  DDML_HIP(hipMemcpyAsync(h + sizeof(SlotState) * max_slots, ost_all.p, sizeof(OuterState) * n * kMaxRhs,
                          hipMemcpyDeviceToHost, st));
  DDML_HIP(hipEventRecord(ev[ring], st));
  snap[ring] = gen_of;
  rb_used[ring] = nused;
  pending[ring] = true;
  ring ^= 1;
}

template <typename T2>
void BatchRunner<T2>::collect_dev() {
  const int k = ring;   // the replay before the latest one
  if (!pending[k]) return;
  DDML_HIP(hipEventSynchronize(ev[k]));
  pending[k] = false;
  const char* h = static_cast<const char*>(pin_rb[k]);
  const SlotState* ss = reinterpret_cast<const SlotState*>(h);
  const OuterState* os = reinterpret_cast<const OuterState*>(h + sizeof(SlotState) * max_slots);
  for (int slot = 0; slot < rb_used[k]; ++slot) {
    // a slot retired since (and maybe taken by another solve) is skipped
    if (snap[k][slot] == 0 || gen_of[slot] != snap[k][slot] || ss[slot].phase != PH_DONE) continue;
    Solve* s = slot_of[slot];
    s->outer = ss[slot].cycles;
    for (int col = 0; col < s->nrhs; ++col) {
      const OuterState& o = os[(size_t)slot * kMaxRhs + col];
      s->inner_iters[col] = o.inner_total;
      s->rel[col] = o.rel;
      s->status[col] = o.status;
      s->done[col] = 1;
    }
    leave(s);
    s->state = 3;
  }
}

template struct BatchRunner<float2>;
template struct BatchRunner<double2>;
template struct BatchRunner<h16c>;

// ------------------------------------------------------------ solve flow
ddml_solver_params default_params() {
  ddml_solver_params p{};
  p.tol = 1e-10;
  p.max_outer = 12;
  p.max_inner = 4000;
  p.inner_tol = 1e-5;
  p.prec = DDML_MIXED_FP32;
  p.solver = 0;
  p.gcr_m = 0;
  return p;
}

void check_params(const ddml_solver_params* p) {
  if (!p) throw Error{DDML_EINVAL, "solver params NULL"};
  if (!(p->tol > 0) || !(p->tol < 1)) throw Error{DDML_EINVAL, "tol must be in (0,1)"};
  if (p->max_outer < 1 || p->max_inner < 1) throw Error{DDML_EINVAL, "max_outer and max_inner must be >= 1"};
  if (!(p->inner_tol > 0) || !(p->inner_tol < 1)) throw Error{DDML_EINVAL, "inner_tol must be in (0,1)"};
  if (p->prec != DDML_FP64 && p->prec != DDML_MIXED_FP32 && p->prec != DDML_MIXED_FP16)
    throw Error{DDML_EINVAL, "unknown precision"};
  if (p->solver < 0 || p->solver > 2)
    throw Error{DDML_EINVAL, "solver must be 0 (BiCGstab restarted), 1 (reliable updates) or 2 (GCR(m))"};
  if (p->solver == 2 && (p->gcr_m < 0 || p->gcr_m > kGcrMax)) throw Error{DDML_EINVAL, "gcr_m must be in 0..8"};
  if (p->solver == 2 && p->prec == DDML_MIXED_FP16)
    throw Error{DDML_EINVAL, "GCR(m) runs with FP32 or FP64 inner vectors"};
}

template <typename T2>
static BatchRunner<T2>& runner(Ctx* c, int nrhs, int m);  // m: GCR restart length, 0 = BiCGstab
template <>
BatchRunner<float2>& runner<float2>(Ctx* c, int nrhs, int m) {
  auto& r = c->run32[nrhs + 64 * m];
  if (!r) {
    r.reset(new BatchRunner<float2>());
    r->init(c, nrhs, c->tune32, 64, m);
  }
  return *r;
}
template <>
BatchRunner<double2>& runner<double2>(Ctx* c, int nrhs, int m) {
  auto& r = c->run64[nrhs + 64 * m];
  if (!r) {
    r.reset(new BatchRunner<double2>());
    r->init(c, nrhs, c->tune64, 64, m);
  }
  return *r;
}
template <>
BatchRunner<h16c>& runner<h16c>(Ctx* c, int nrhs, int m) {
  auto& r = c->run16[nrhs + 64 * m];
  if (!r) {
    r.reset(new BatchRunner<h16c>());
    r->init(c, nrhs, c->tune16, 64, m);
  }
  return *r;
}

void solve_prepare(Ctx* c, Solve* s) {
  if (s->nrhs < 1 || s->nrhs > kMaxRhs) throw Error{DDML_EINVAL, "nrhs must be in 1..12"};
  s->ob = opblock(c, s->gauge_id, s->dom_id);
  if (s->prec != DDML_FP64 && !s->ob->su3)
    throw Error{DDML_EINVAL, "the FP32 and 16-bit operator copies keep two rows per link and need SU(3) links"};
  const size_t Vh = s->ob->g.Vh, n = (size_t)s->nrhs * s->ob->field;
  const size_t nt = s->ob->ntiles;
  DevPool* P = c->pool.get();
  s->be = DBuf(P, n * sizeof(double2));
  s->bo = DBuf(P, n * sizeof(double2));
  s->xe = DBuf(P, n * sizeof(double2));
  s->xo = DBuf(P, n * sizeof(double2));
  s->re = DBuf(P, n * sizeof(double2));
  s->ro = DBuf(P, n * sizeof(double2));
  s->te = DBuf(P, n * sizeof(double2));
  s->to = DBuf(P, n * sizeof(double2));
  s->partial64 = DBuf(P, 2 * s->nrhs * nt * sizeof(double2));
  s->norms = DBuf(P, 3 * s->nrhs * sizeof(double2));
  const int m = gcr_len(s->prm);
  const size_t fb = inner_field_bytes(s->prec, n, s->nrhs, nt);
  for (int k = 0; k < F_ALL; ++k) {
    const bool used = m > 0 ? (k == F_R || k == F_X || k == F_TMP || (k >= F_GP0 && k < F_GP0 + m) ||
                               (k >= F_GQ0 && k < F_GQ0 + m))
                            : (k < F_NUM && k != F_UNUSED);
    if (used) s->f[k] = DBuf(P, (k == F_X && s->prec == DDML_MIXED_FP16) ? n * sizeof(float2) : fb);
  }
  if (s->prec == DDML_MIXED_FP16) ensure16(c, *s->ob);
  s->partial = DBuf(P, (size_t)(m > 0 ? std::max(2, m) : kBiPartials) * s->nrhs * nt * sizeof(double2));
  s->table1 = DBuf(P, std::max({sizeof(SlotDesc<double2>), sizeof(SlotDesc<float2>), sizeof(SlotDesc<h16c>)}));
  s->tstart1 = DBuf(P, 2 * sizeof(int));
  s->n1 = DBuf(P, sizeof(int));
  const double kappa = s->ob->bs.kappa;
  const double2* src = reinterpret_cast<const double2*>(s->src);
  hipStream_t st = c->stream;
  DDML_HIP(hipMemsetAsync(s->be.p, 0, n * sizeof(double2), st));
  DDML_HIP(hipMemsetAsync(s->bo.p, 0, n * sizeof(double2), st));
  DDML_HIP(launch_gather(src, s->ob->bs, 0, s->nrhs, 2.0 * kappa, s->be.as<double2>(), st));
  DDML_HIP(launch_gather(src, s->ob->bs, 1, s->nrhs, 2.0 * kappa, s->bo.as<double2>(), st));
  DDML_HIP(hipMemsetAsync(s->xe.p, 0, n * sizeof(double2), st));
  DDML_HIP(hipMemsetAsync(s->xo.p, 0, n * sizeof(double2), st));
  DDML_HIP(launch_col_norms(s->be.as<double2>(), (int)Vh, s->nrhs, s->partial64.as<double2>(), (int)nt,
                            s->norms.as<double2>(), 0, st));
  DDML_HIP(launch_col_norms(s->bo.as<double2>(), (int)Vh, s->nrhs, s->partial64.as<double2>(), (int)nt,
                            s->norms.as<double2>(), 1, st));
  s->bn2.assign(s->nrhs, 0.0);
  s->rel.assign(s->nrhs, 1.0);
  s->done.assign(s->nrhs, 0);
  s->inner_iters.assign(s->nrhs, 0);
  s->status.assign(s->nrhs, DDML_OK);
  s->outer = 0;
  s->state = 1;
}

// r = b' - M x on both parities with |r|^2 partials
static void launch_residual(Ctx* c, Solve* s) {
  const OpBlock& ob = *s->ob;
  const int nt = ob.ntiles;
  for (int p = 0; p < 2; ++p) {
    HopItem<double2> it = item64(ob, s->nrhs, c->tune64.order);
    it.clov = ob.A64.as<double2>();
    it.in = p == 0 ? s->xo.as<double2>() : s->xe.as<double2>();
    it.aux = p == 0 ? s->xe.as<double2>() : s->xo.as<double2>();
    it.red_a = p == 0 ? s->be.as<double2>() : s->bo.as<double2>();
    it.out = p == 0 ? s->re.as<double2>() : s->ro.as<double2>();
    it.partial = s->partial64.as<double2>() + (size_t)p * s->nrhs * nt;
    it.par_out = p;
    it.c1 = ob.bs.kappa;
    DDML_HIP(launch_hop_item(it, MODE_RES, RED_NORM, 1, c->tune64.order, c->stream));
  }
  DDML_HIP(launch_sum_partials(s->partial64.as<double2>(), 2, s->nrhs, nt, s->norms.as<double2>() + s->nrhs, 0,
                               c->stream));
}

// rhat_e = A_ee^{-1}(r_e + kappa H_eo A_oo^{-1} r_o) into te
static void launch_prepare(Ctx* c, Solve* s) {
  const OpBlock& ob = *s->ob;
  DDML_HIP(launch_clover_apply(ob.g, ob.Ainv64.as<double2>(), 1, s->ro.as<double2>(), s->to.as<double2>(), s->nrhs,
                               c->stream));
  HopItem<double2> it = item64(ob, s->nrhs, c->tune64.order);
  it.clov = ob.Ainv64.as<double2>();
  it.in = s->to.as<double2>();
  it.aux = s->re.as<double2>();
  it.out = s->te.as<double2>();
  it.par_out = 0;
  it.c1 = ob.bs.kappa;
  DDML_HIP(launch_hop_item(it, MODE_PREP, RED_NONE, 1, c->tune64.order, c->stream));
}

// e_e from the inner solution, e_o = A_oo^{-1}(r_o + kappa H_oe e_e), x += e
template <typename T2>
static void launch_export(Ctx* c, Solve* s) {
  const OpBlock& ob = *s->ob;
  const size_t n = (size_t)s->nrhs * ob.field;
  using XT = typename std::conditional<std::is_same<T2, h16c>::value, float2, T2>::type;  // 16-bit: FP32 x
  DDML_HIP(launch_cast_to_d(s->f[F_X].as<XT>(), s->te.as<double2>(), n, c->stream));
  HopItem<double2> it = item64(ob, s->nrhs, c->tune64.order);
  it.clov = ob.Ainv64.as<double2>();
  it.in = s->te.as<double2>();
  it.aux = s->ro.as<double2>();
  it.out = s->to.as<double2>();
  it.par_out = 1;
  it.c1 = ob.bs.kappa;
  DDML_HIP(launch_hop_item(it, MODE_PREP, RED_NONE, 1, c->tune64.order, c->stream));
  DDML_HIP(launch_axpy_d(s->xe.as<double2>(), s->te.as<double2>(), 1.0, n, c->stream));
  DDML_HIP(launch_axpy_d(s->xo.as<double2>(), s->to.as<double2>(), 1.0, n, c->stream));
}


// Host loop (GCR(m)): joins a solve to its runner for one cycle, with the
// per-column request flags and limits of the cycle, and initialises the cycle.
template <typename T2>
static bool try_join(Ctx* c, Solve* s) {
  const int m = gcr_len(s->prm);
  BatchRunner<T2>& run = runner<T2>(c, s->nrhs, m);
  const int slot = run.join(s);
  if (slot < 0) return false;
  std::vector<int> want(kMaxRhs, 0);
  std::vector<BiState> st(kMaxRhs, BiState{});
  const double tol = s->prm.tol;
  for (int col = 0; col < s->nrhs; ++col) {
    want[col] = !s->done[col];
    // reduction needed this cycle: tol |b| / |r|, with a safety factor; never
    // tighter than the requested inner tolerance in mixed precision
    double need = s->rel[col] > 0 ? 0.1 * tol / s->rel[col] : 1e-3;
    double it = s->prec == DDML_FP64 ? std::max(need, 1e-14) : std::max(need, s->prm.inner_tol);
    if (s->prec == DDML_MIXED_FP16) it = std::max(it, kInnerFloor16);
    it = std::min(it, 0.1);
    st[col].tol2 = it * it;
    st[col].max_iters = s->prm.max_inner;
  }
  BiState* dst = run.st_all.template as<BiState>() + (size_t)slot * kMaxRhs;
  int* dact = run.act_all.template as<int>() + (size_t)slot * kMaxRhs;
  DDML_HIP(hipMemcpyAsync(dst, st.data(), sizeof(BiState) * kMaxRhs, hipMemcpyHostToDevice, c->stream));
  DDML_HIP(hipMemcpyAsync(dact, want.data(), sizeof(int) * kMaxRhs, hipMemcpyHostToDevice, c->stream));
  // one-entry table for the (re)initialisation
  SlotDesc<T2> d = run.h_table[slot];
  int ts[2] = {0, d.ntiles};
  int one = 1;
  DDML_HIP(hipMemcpyAsync(s->table1.p, &d, sizeof(d), hipMemcpyHostToDevice, c->stream));
  DDML_HIP(hipMemcpyAsync(s->tstart1.p, ts, sizeof(ts), hipMemcpyHostToDevice, c->stream));
  DDML_HIP(hipMemcpyAsync(s->n1.p, &one, sizeof(int), hipMemcpyHostToDevice, c->stream));
  const int grid = std::min(d.ntiles, 4096);
  if constexpr (!std::is_same<T2, h16c>::value) {   // GCR(m) runs with FP32 or FP64 vectors
    DDML_HIP(launch_gcr(s->table1.as<SlotDesc<T2>>(), s->tstart1.as<int>(), s->n1.as<int>(), s->nrhs, GCR_INIT, 0,
                        m, grid, c->stream));
    DDML_HIP(launch_gcr_fin(s->table1.as<SlotDesc<T2>>(), s->n1.as<int>(), 1, GFIN_INIT, 0, c->stream));
  }
  s->state = 2;
  return true;
}

static void finish_state(Solve* s) { s->state = 3; }

// One scheduling round of the device loop: prepared solves join a free slot
// of their runner, every runner with members replays its graph once (the
// outer step and K inner iterations of every slot), and the slots that the
// previous replay left at PH_DONE retire (state 3).  The host waits only for
// the replay before the latest one, so one replay is always queued.
bool solve_join(Ctx* c, Solve* s) {
  if (gcr_len(s->prm) > 0) return true;   // the host loop joins between cycles
  if (s->slot >= 0) return true;
  int slot = -1;
  if (s->prec == DDML_FP64) slot = runner<double2>(c, s->nrhs, 0).join(s);
  else if (s->prec == DDML_MIXED_FP16) slot = runner<h16c>(c, s->nrhs, 0).join(s);
  else slot = runner<float2>(c, s->nrhs, 0).join(s);
  if (slot < 0) return false;
  s->state = 2;
  return true;
}

static void dev_progress(Ctx* c, std::vector<Solve*>& live) {
  for (Solve* s : live)
    if (s->state == 1 && s->slot < 0) solve_join(c, s);
  auto round = [&](auto& runs) {
    for (auto& kv : runs) {
      auto& run = *kv.second;
      if (!run.device) continue;
      if (run.members() > 0) run.launch_dev();
      run.collect_dev();
    }
  };
  round(c->run32);
  round(c->run64);
  round(c->run16);
}

// True if a prepared solve with these parameters would find a free slot.
bool solve_slot_free(Ctx* c, int prec, int nrhs, const ddml_solver_params& prm) {
  const int m = gcr_len(prm);
  if (m > 0) return true;   // the host loop queues solves for its runner itself
  if (prec == DDML_FP64) return runner<double2>(c, nrhs, 0).has_free();
  if (prec == DDML_MIXED_FP16) return runner<h16c>(c, nrhs, 0).has_free();
  return runner<float2>(c, nrhs, 0).has_free();
}

static void host_progress(Ctx* c, std::vector<Solve*>& live);

// One scheduling round over the live solves: BiCGstab solves run the device
// loop, GCR(m) solves the host loop.
void solve_progress(Ctx* c, std::vector<Solve*>& live, bool block) {
  (void)block;
  std::vector<Solve*> host, dev;
  for (Solve* s : live) (gcr_len(s->prm) > 0 ? host : dev).push_back(s);
  if (!dev.empty()) dev_progress(c, dev);
  if (!host.empty()) host_progress(c, host);
}

// One scheduling round of the host loop (GCR(m) solves).
static void host_progress(Ctx* c, std::vector<Solve*>& live) {
  hipStream_t st = c->stream;
  // 1. residuals of every solve that needs one, one synchronisation
  std::vector<Solve*> need;
  for (Solve* s : live)
    if (s->state == 1) need.push_back(s);
  if (!need.empty()) {
    size_t tot = 0;
    for (Solve* s : need) tot += 3 * s->nrhs;
    double2* h = (double2*)pinned_area(c, tot * sizeof(double2));
    size_t off = 0;
    for (Solve* s : need) {
      launch_residual(c, s);
      DDML_HIP(hipMemcpyAsync(h + off, s->norms.p, 3 * s->nrhs * sizeof(double2), hipMemcpyDeviceToHost, st));
      off += 3 * s->nrhs;
    }
    DDML_HIP(hipStreamSynchronize(st));
    std::vector<double2> hv(h, h + tot);
    off = 0;
    for (Solve* s : need) {
      bool all = true, bad = false;
      for (int col = 0; col < s->nrhs; ++col) {
        const double bn2 = hv[off + col].x;
        const double rn2 = hv[off + s->nrhs + col].x + hv[off + 2 * s->nrhs + col].x;
        s->bn2[col] = bn2;
        double rel = (bn2 > 0 || !std::isfinite(bn2)) ? std::sqrt(rn2 / bn2) : 0.0;
        if (!std::isfinite(rel)) { bad = true; rel = INFINITY; s->status[col] = DDML_ENUMERIC; }
        s->rel[col] = rel;
        s->done[col] = rel <= s->prm.tol || s->status[col] == DDML_ENUMERIC;
        all = all && s->done[col];
      }
      off += 3 * s->nrhs;
      (void)bad;
      if (all || s->outer >= s->prm.max_outer) {
        finish_state(s);
      } else {
        launch_prepare(c, s);
        s->outer += 1;
        s->state = 4;
      }
    }
  }
  // 2. join the batch
  for (Solve* s : live)
    if (s->state == 4) {
      if (s->prec == DDML_FP64) try_join<double2>(c, s);
      else if (s->prec == DDML_MIXED_FP16) try_join<h16c>(c, s);
      else try_join<float2>(c, s);
    }
  // 3. one replay per runner with members; collect finished inner solves
  auto step = [&](auto& runs, auto tag) {
    using T2 = decltype(tag);
    for (auto& kv : runs) {
      auto& run = *kv.second;
      if (run.device || run.members() == 0) continue;
      run.replay();
      for (int slot = 0; slot < run.max_slots; ++slot) {
        Solve* s = run.slot_of[slot];
        if (!s) continue;
        bool any = false;
        for (int col = 0; col < s->nrhs; ++col) any = any || run.h_st[(size_t)slot * kMaxRhs + col].active;
        if (any) continue;
        for (int col = 0; col < s->nrhs; ++col) {
          const BiState& b = run.h_st[(size_t)slot * kMaxRhs + col];
          if (!s->done[col]) s->inner_iters[col] += b.iters;
        }
        run.leave(s);
        launch_export<T2>(c, s);
        s->state = 1;
      }
    }
  };
  step(c->run32, float2{});
  step(c->run64, double2{});
  step(c->run16, h16c{});
}

void series_terms(Ctx* c, int gauge_id, const int* dom_ids, int nlevels, double* terms, double* sum, int nrhs) {
  const GaugeRec& g = gauge_get(c, gauge_id);
  const size_t per = (size_t)nrhs * g.V * 12;   // complex numbers of one level
  // the solutions vanish outside their domains: difference only the time
  // slices the union of the series' domains covers (whole column ranges)
  int t0 = g.lat.dims[0], t1 = 0;
  for (int i = 0; i < nlevels; ++i) {
    const DomainRec& dr = dom_ids[i] == -1 ? DomainRec{{0, 0, 0, 0}, {g.lat.dims[0], 0, 0, 0}}
                                           : domain_get(c, dom_ids[i]);
    t0 = std::min(t0, dr.lo[0]);
    t1 = std::max(t1, std::min(dr.hi[0], g.lat.dims[0]));
  }
  const size_t row = g.V / g.lat.dims[0] * 12;   // complex numbers of one time slice of one column
  double2* s2 = reinterpret_cast<double2*>(sum);
  if (s2 && (t0 > 0 || t1 < g.lat.dims[0])) DDML_HIP(hipMemsetAsync(s2, 0, per * sizeof(double2), c->stream));
  if (t1 > t0)
    DDML_HIP(launch_series_diff(reinterpret_cast<double2*>(terms), per, nlevels, s2, c->stream, nrhs, g.V * 12,
                                (size_t)t0 * row, (size_t)(t1 - t0) * row));
}

void solve_finish(Ctx* c, Solve* s) {
  hipStream_t st = c->stream;
  double2* sol = reinterpret_cast<double2*>(s->sol);
  DDML_HIP(hipMemsetAsync(sol, 0, (size_t)s->nrhs * gauge_get(c, s->gauge_id).V * 12 * sizeof(double2), st));
  DDML_HIP(launch_scatter(s->xe.as<double2>(), s->ob->bs, 0, s->nrhs, 1.0, sol, st));
  DDML_HIP(launch_scatter(s->xo.as<double2>(), s->ob->bs, 1, s->nrhs, 1.0, sol, st));
  if (s->info) {
    for (int col = 0; col < s->nrhs; ++col) {
      ddml_rhs_info& in = s->info[col];
      in.outer_iters = s->outer;
      in.inner_iters = s->inner_iters[col];
      in.true_rel_residual = s->rel[col];
      in.status = s->status[col] == DDML_ENUMERIC ? DDML_ENUMERIC
                  : (s->rel[col] <= s->prm.tol ? DDML_OK : DDML_ENOTCONVERGED);
    }
  }
  // release device state (the scatter is ordered before any reuse of the
  // memory because every later use is on the same stream)
  solve_release(s);
  s->state = 3;
}

// Takes a solve out of its runner's slot table (if it holds a slot) without
// creating a runner; the next replay uploads a table without it.
template <typename T2>
static void leave_slot(std::map<int, std::unique_ptr<BatchRunner<T2>>>& runs, Solve* s) {
  if (s->slot < 0) return;
  auto it = runs.find(s->nrhs + 64 * gcr_len(s->prm));
  if (it != runs.end() && it->second->slot_of[s->slot] == s) it->second->leave(s);
  s->slot = -1;
}

void solve_abandon(Ctx* c, Solve* s) {
  if (s->prec == DDML_FP64) leave_slot(c->run64, s);
  else if (s->prec == DDML_MIXED_FP16) leave_slot(c->run16, s);
  else leave_slot(c->run32, s);
  // buffers go back to the pool, which keeps them allocated: a replay already
  // queued on the stream that still names them touches valid memory
  solve_release(s);
  s->state = 3;
}

void solve_release(Solve* s) {
  s->be.reset(); s->bo.reset(); s->xe.reset(); s->xo.reset();
  s->re.reset(); s->ro.reset(); s->te.reset(); s->to.reset();
  s->partial64.reset(); s->norms.reset(); s->partial.reset();
  for (int k = 0; k < F_ALL; ++k) s->f[k].reset();
  s->table1.reset(); s->tstart1.reset(); s->n1.reset();
  s->ob.reset();
}

template <typename T2>
static void time_stencil_t(Ctx* c, const OpBlock& ob, const T2* U, const T2* Ainv, int nrhs, int iters, int R,
                           int order, int grid, int splits, int stage, double out[4]) {
  hipStream_t st = c->stream;
  const size_t Vh = ob.g.Vh, n = (size_t)nrhs * ob.field;
  constexpr bool h16 = std::is_same<T2, h16c>::value;
  const int prec = h16 ? DDML_MIXED_FP16 : (sizeof(T2) == sizeof(double2) ? DDML_FP64 : DDML_MIXED_FP32);
  const size_t fb = inner_field_bytes(prec, n, nrhs, ob.ntiles), nn = (size_t)nrhs * ob.ntiles * kTile;
  DevPool* P = c->pool.get();
  DBuf fP(P, fb), fT(P, fb), fV(P, fb);
  DBuf part(P, 2 * nrhs * ob.ntiles * sizeof(double2)), act(P, kMaxRhs * sizeof(int));
  DBuf tab(P, sizeof(SlotDesc<T2>)), ts(P, 2 * sizeof(int)), ns(P, sizeof(int)), xs(P, kXcd * 2 * sizeof(int));
  auto scales = [&](DBuf& b) { return reinterpret_cast<float*>(b.as<h16c>() + n); };
  if constexpr (h16) {
    DDML_HIP(launch_fill16(fP.as<h16c>(), n, scales(fP), nn, 1.0, st));
  } else {
    DDML_HIP(launch_fill(fP.as<T2>(), n, 1.0, st));
  }
  std::vector<int> ones(kMaxRhs, 1);
  DDML_HIP(hipMemcpyAsync(act.p, ones.data(), kMaxRhs * sizeof(int), hipMemcpyHostToDevice, st));
  SlotDesc<T2> d{};
  d.g = ob.g;
  d.nrhs = nrhs;
  d.ntiles = ob.ntiles;
  d.tps = ob.tps;
  d.kappa = ob.bs.kappa;
  d.U = U;
  d.Ainv = Ainv;
  d.f[F_P] = fP.as<T2>();
  d.f[F_TMP] = fT.as<T2>();
  d.f[F_V] = fV.as<T2>();
  if constexpr (h16) {
    d.nrm[F_P] = scales(fP);
    d.nrm[F_TMP] = scales(fT);
    d.nrm[F_V] = scales(fV);
    d.Ainv_nrm = ob.Ainv16n.as<float>();
  }
  d.partial = part.as<double2>();
  d.active = act.as<int>();
  attach_walk(d, ob, order);
  int h_ts[2] = {0, ob.ntiles}, one = 1;
  DDML_HIP(hipMemcpyAsync(tab.p, &d, sizeof(d), hipMemcpyHostToDevice, st));
  DDML_HIP(hipMemcpyAsync(ts.p, h_ts, sizeof(h_ts), hipMemcpyHostToDevice, st));
  DDML_HIP(hipMemcpyAsync(ns.p, &one, sizeof(int), hipMemcpyHostToDevice, st));
  int h_xs[kXcd * 2];
  for (int x = 0; x < kXcd; ++x) {
    h_xs[2 * x] = 0;
    h_xs[2 * x + 1] = order == TILE_ORDER_LINEAR ? 0 : xcd_share(d, order, x);
  }
  DDML_HIP(hipMemcpyAsync(xs.p, h_xs, sizeof(h_xs), hipMemcpyHostToDevice, st));
  auto* tb = tab.as<SlotDesc<T2>>();
  auto launch = [&](int which) {
    if (which == 0)
      DDML_HIP(launch_hop_batch(tb, ts.as<int>(), xs.as<int>(), 2, ns.as<int>(), nrhs, R, MODE_CINV_HOP, RED_NONE,
                                F_P, -1, F_TMP, -1, 1, grid, order, splits, stage, st));
    else
      DDML_HIP(launch_hop_batch(tb, ts.as<int>(), xs.as<int>(), 2, ns.as<int>(), nrhs, R, MODE_SCHUR, RED_DOT, F_TMP,
                                F_P, F_V, -1, 0, grid, order, splits, stage, st));
  };
  for (int w = 0; w < 3; ++w) { launch(0); launch(1); }
  std::vector<hipEvent_t> ev(2 * iters + 1);
  for (auto& e : ev) DDML_HIP(hipEventCreate(&e));
  DDML_HIP(hipEventRecord(ev[0], st));
  for (int i = 0; i < iters; ++i) {
    launch(0);
    DDML_HIP(hipEventRecord(ev[2 * i + 1], st));
    launch(1);
    DDML_HIP(hipEventRecord(ev[2 * i + 2], st));
  }
  DDML_HIP(hipEventSynchronize(ev[2 * iters]));
  double t0 = 0, t1 = 0;
  for (int i = 0; i < iters; ++i) {
    float a = 0, b = 0;
    DDML_HIP(hipEventElapsedTime(&a, ev[2 * i], ev[2 * i + 1]));
    DDML_HIP(hipEventElapsedTime(&b, ev[2 * i + 1], ev[2 * i + 2]));
    t0 += a;
    t1 += b;
  }
  for (auto& e : ev) DDML_HIP(hipEventDestroy(e));
  const double s = h16 ? 2.0 : sizeof(T2) / 2;  // bytes per real
  // CINV_HOP: read the input spinor, all links of the box (4 per site), A^{-1} of
  // the output parity; write the output.  SCHUR (+ the hashed-shadow dot): read
  // input and aux, links, A^{-1}; write the output.
  out[0] = t0 / iters;
  out[1] = t1 / iters;
  // 16-bit: plus one 4-byte scale per site and column of every spinor touched
  // and per site of A^{-1}.  Links: 8 per output site, 12 reals each in the
  // two-row FP32 and 16-bit copies, 18 in FP64.
  const double sc = h16 ? 4.0 : 0.0;
  const double lr = std::is_same<T2, double2>::value ? 144.0 : 96.0;
  out[2] = (double)Vh * ((48.0 * nrhs + lr + 72.0) * s + sc * (2 * nrhs + 1));
  out[3] = (double)Vh * ((72.0 * nrhs + lr + 72.0) * s + sc * (3 * nrhs + 1));
}

void time_stencil(Ctx* c, int gauge_id, int dom_id, int nrhs, int prec, int iters, const TuneChoice& want,
                  double out[4]) {
  if (nrhs < 1 || nrhs > kMaxRhs || iters < 1) throw Error{DDML_EINVAL, "bad nrhs or iters"};
  const TuneChoice& tn = c->tune(prec);
  const int R = want.R > 0 ? want.R : tn.R;
  const int order = want.order >= 0 ? want.order : tn.order;
  int grid = want.grid > 0 ? want.grid : tn.grid;
  int splits = want.splits > 0 ? want.splits : tn.splits;
  const int stage = want.stage >= 0 ? want.stage : tn.stage;
  if (R < 1 || R > 3 || order >= TILE_ORDER_NUM || stage > 1)
    throw Error{DDML_EINVAL, "R must be 1..3, order 0..3 and stage 0 or 1"};
  splits = std::min(splits, (nrhs + R - 1) / R);
  grid = ((grid + kXcd - 1) / kXcd) * kXcd;
  auto ob = opblock(c, gauge_id, dom_id);
  if (prec == DDML_FP64) {
    time_stencil_t<double2>(c, *ob, ob->U64.as<double2>(), ob->Ainv64.as<double2>(), nrhs, iters, R, order, grid,
                            splits, stage, out);
  } else if (prec == DDML_MIXED_FP16) {
    if (stage != 1) throw Error{DDML_EINVAL, "16-bit fields need stage 1"};
    ensure16(c, *ob);
    time_stencil_t<h16c>(c, *ob, ob->U16.as<h16c>(), ob->Ainv16.as<h16c>(), nrhs, iters, R, order, grid, splits,
                         stage, out);
  } else {
    if (stage != 1) throw Error{DDML_EINVAL, "FP32 fields need stage 1"};
    time_stencil_t<float2>(c, *ob, ob->U32.as<float2>(), ob->Ainv32.as<float2>(), nrhs, iters, R, order, grid,
                           splits, stage, out);
  }
}

void set_launch(Ctx* c, int prec, const TuneChoice& want) {
  const bool staged = prec != DDML_FP64;   // two-row links are rebuilt in the LDS staging
  if (want.R < 1 || want.R > 3 || want.order < 0 || want.order >= TILE_ORDER_NUM || want.grid < kXcd ||
      want.splits < 1 || want.splits > 12 || want.stage < 0 || want.stage > 1 || (staged && want.stage != 1))
    throw Error{DDML_EINVAL, "invalid launch choice"};
  TuneChoice& t = c->tune(prec);
  const int K = t.K;
  t = want;
  t.K = K;
  c->run32.clear();  // graphs are captured with the launch choice: rebuild on next use
  c->run64.clear();
  c->run16.clear();
}

void autotune(Ctx* c, int gauge_id, int dom_id, int nrhs, int prec, double best[6]) {
  double bt = 1e300;
  TuneChoice b = c->tune(prec);
  for (int stage = prec == DDML_FP64 ? 0 : 1; stage <= 1; ++stage)
    for (int R = 1; R <= 3; ++R)
      for (int splits = 1; splits <= 3; ++splits) {
        if (splits > (nrhs + R - 1) / R) continue;
        for (int order = 0; order < TILE_ORDER_NUM; ++order)
          for (int grid : {512, 1024, 2048}) {
            TuneChoice w = b;
            w.R = R;
            w.order = order;
            w.grid = grid;
            w.splits = splits;
            w.stage = stage;
            double o[4];
            time_stencil(c, gauge_id, dom_id, nrhs, prec, 4, w, o);
            const double t = o[0] + o[1];
            if (t < bt) {
              bt = t;
              b = w;
            }
          }
      }
  c->tune(prec) = b;
  c->run32.clear();  // graphs are captured with the launch choice: rebuild on next use
  c->run64.clear();
  c->run16.clear();
  best[0] = b.R;
  best[1] = b.order;
  best[2] = b.grid;
  best[3] = b.splits;
  best[4] = b.stage;
  best[5] = bt;
}

void run_solves(Ctx* c, std::vector<Solve*>& solves) {
  std::deque<Solve*> queue(solves.begin(), solves.end());
  std::vector<Solve*> live;
  try {
  while (!queue.empty() || !live.empty()) {
    while (!queue.empty()) {
      Solve* s = queue.front();
      if (!solve_slot_free(c, s->prec, s->nrhs, s->prm)) break;   // retry once a slot has retired
      const size_t fp = solve_footprint(c, s->gauge_id, s->dom_id, s->nrhs, s->prm);
      if (!live.empty() && !c->pool->fits_device(fp)) break;
      try {
        solve_prepare(c, s);
      } catch (const Error& e) {
        solve_release(s);
        if (e.code == DDML_ENOMEM && !live.empty()) break;  // retry once solves in flight have finished
        throw;
      }
      solve_join(c, s);
      queue.pop_front();
      live.push_back(s);
    }
    solve_progress(c, live, true);
    for (auto it = live.begin(); it != live.end();) {
      if ((*it)->state == 3) {
        solve_finish(c, *it);
        it = live.erase(it);
      } else {
        ++it;
      }
    }
  }
  } catch (...) {
    // the caller's solves are about to go away: no slot may keep naming them
    for (Solve* s : live) solve_abandon(c, s);
    throw;
  }
  DDML_HIP(hipStreamSynchronize(c->stream));
}

}  // namespace ddml
