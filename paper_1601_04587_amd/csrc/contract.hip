// Propagator series and Wick contractions (FP64).
//
//  * eq. Dseries: terms[0] = S^(0), terms[i] = S^(i) - S^(i-1) (in place, from
//    the last level down) with every S^(i) zero outside its domain.
//  * Section 3 (eqs. W0, rall0, rall): t = tr{g5 S^(i)(x,x)} from the 12
//    point-source columns; pieces f, r1, r2 and the full product.
//  * Section 5.2 (eq. baryfact), C = i g0 g2, P_- = (1 - g0)/2, S_u = S_d = S:
//      W_N1 = eps^{abc} eps^{feg} tr[S^{ag T} C g5 S^{bf} C g5] tr[S^{ce} P_-]
//      W_N2 = eps^{abc} eps^{feg} tr[S^{ag T} C g5 S^{be} P_- S^{cf} C g5]
//    per sink site, then summed over each sink time slice (eq. baryN) in a
//    fixed order.
//  * Connected pseudoscalar (eqs. pipi, W0pc): W(y) = tr{S(y,x) S(y,x)^dag},
//    the sum of |S|^2 over the 144 entries at the sink, summed per time slice
//    and scaled by -1/L^3; series differences (eq. seriespi) and the rest
//    against the full propagator (eq. W0pc2).
//  * Stochastic traces (Section 6, eq. HPEtr and the estimator after it):
//    gamma5 on the sources, and sum_i sum_c conj(eta_i(x)_c) phi_i(x)_c per
//    site (sources, then components, in order) before the slice sums.
// In the chiral basis C = diag(s_2, -s_2), so C g5 = diag(s_2, s_2), and
// P_- = [[1,1],[1,1]]/2 in 2x2 spin blocks; both are applied in closed form below.
#include <mutex>

#include "ddml_common.hpp"
#include "launchers.hpp"

namespace ddml {

// terms[l] <- terms[l] - terms[l-1] (l >= 1) and sum <- terms[last] on the
// elements [lo, lo + len) of each of ncol columns (column stride cstride) of
// fields n apart; the elements outside hold zeros in every level.
__global__ void k_series_diff(double2* __restrict__ terms, size_t n, int nlevels, double2* __restrict__ sum,
                              int ncol, size_t cstride, size_t lo, size_t len) {
  const size_t total = (size_t)ncol * len;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const size_t k = (t / len) * cstride + lo + t % len;
    double2 prev = terms[k];
    for (int l = 1; l < nlevels; ++l) {
      const double2 cur = terms[(size_t)l * n + k];
      terms[(size_t)l * n + k] = make_double2(cur.x - prev.x, cur.y - prev.y);
      prev = cur;
    }
    if (sum) sum[k] = prev;
  }
}

hipError_t launch_series_diff(double2* terms, size_t n, int nlevels, double2* sum, hipStream_t st, int ncol,
                              size_t cstride, size_t lo, size_t len) {
  if (ncol <= 0) {   // the whole field
    ncol = 1;
    cstride = n;
    lo = 0;
    len = n;
  }
  size_t g = ((size_t)ncol * len + 255) / 256;
  if (g > 16384) g = 16384;
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL(k_series_diff, dim3((int)g), dim3(256), 0, st, terms, n, nlevels, sum, ncol, cstride, lo, len);
  return hipGetLastError();
}

// ---------------------------------------------------- disconnected pseudoscalar
// S^(i)(x,x)[alpha a][beta b] = sum_{j<=i} terms[j][3 beta + b][x][alpha][a]
__device__ double2 g5_trace(const double2* __restrict__ terms, size_t V, int level, size_t site) {
  double2 t = make_double2(0, 0);
  for (int j = 0; j <= level; ++j)
    for (int col = 0; col < 12; ++col) {
      const int beta = col / 3, b = col % 3;
      const double2 v = terms[(((size_t)j * 12 + col) * V + site) * 12 + beta * 3 + b];
      const double sg = beta < 2 ? 1.0 : -1.0;   // (g5)_{beta beta}
      t.x += sg * v.x;
      t.y += sg * v.y;
    }
  return t;
}

__global__ void k_pp(const double2* __restrict__ tx_terms, const double2* __restrict__ ty_terms, size_t V,
                     int nlevels, size_t xs, size_t ys, double invL3, double2* __restrict__ out) {
  const int i = threadIdx.x;
  if (i >= nlevels) return;
  const double2 tx = g5_trace(tx_terms, V, i, xs), ty = g5_trace(ty_terms, V, i, ys);
  const double2 fx = g5_trace(tx_terms, V, nlevels - 1, xs), fy = g5_trace(ty_terms, V, nlevels - 1, ys);
  const double2 dx = make_double2(fx.x - tx.x, fx.y - tx.y), dy = make_double2(fy.x - ty.x, fy.y - ty.y);
  auto mul = [](double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); };
  const double2 f = mul(tx, ty);
  const double2 r1a = mul(dx, ty), r1b = mul(tx, dy);
  const double2 r2 = mul(dx, dy);
  const double2 full = mul(fx, fy);
  out[4 * i + 0] = make_double2(f.x * invL3, f.y * invL3);
  out[4 * i + 1] = make_double2((r1a.x + r1b.x) * invL3, (r1a.y + r1b.y) * invL3);
  out[4 * i + 2] = make_double2(r2.x * invL3, r2.y * invL3);
  out[4 * i + 3] = make_double2(full.x * invL3, full.y * invL3);
}

__global__ void k_g5_traces(const double2* __restrict__ terms, size_t V, int nlevels, size_t xs,
                            double2* __restrict__ out) {
  const int i = threadIdx.x;
  if (i < nlevels) out[i] = g5_trace(terms, V, i, xs);
}

hipError_t launch_g5_traces(const double2* terms, size_t V, int nlevels, size_t xs, double2* out, hipStream_t st) {
  hipLaunchKernelGGL(k_g5_traces, dim3(1), dim3(64), 0, st, terms, V, nlevels, xs, out);
  return hipGetLastError();
}

hipError_t launch_pp(const double2* tx, const double2* ty, size_t V, int nlevels, size_t xs, size_t ys, double invL3,
                     double2* out, hipStream_t st) {
  hipLaunchKernelGGL(k_pp, dim3(1), dim3(64), 0, st, tx, ty, V, nlevels, xs, ys, invL3, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ nucleon
__device__ __forceinline__ double2 cm(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

__device__ const int kEps[6][4] = {{0, 1, 2, 1}, {1, 2, 0, 1}, {2, 0, 1, 1}, {0, 2, 1, -1}, {2, 1, 0, -1}, {1, 0, 2, -1}};

// Eight sink sites per workgroup of 64 threads, eight threads per site; thread
// q of a site takes the (abc, feg) pairs q, q + 8, ... of the 36.  The levels
// are walked in order and S^(i) = sum_{j<=i} terms[j] is accumulated in LDS,
// so each term is read once, with loads contiguous over (site, component) for
// each source column.  Sites where S^(i) vanishes (outside the outermost
// domain of the series) skip the spin algebra, which is exact: every product
// there is zero.
//
// The spin algebra uses the rank-2 form of P_-: (M P_-)_{kc} = y_{k, c mod 2}
// with y_{kj} = (M_{kj} + M_{k, j+2}) / 2, so M P_- N = y z with
// z_{jq} = N_{jq} + N_{j+2, q}; W_N2 then needs 40 complex products per pair.
constexpr int kNucSites = 8;
constexpr int kNucThreads = 8;

__device__ __forceinline__ double2 sld(const double2* S, int al, int a, int be, int b) {
  return S[((al * 3 + a) * 4 + be) * 3 + b];
}
// v * (+i) for even k, v * (-i) for odd k: the phase of column k of C g5 = diag(s_2, s_2)
__device__ __forceinline__ double2 mul_ph(double2 v, int k) {
  return (k & 1) ? make_double2(v.y, -v.x) : make_double2(-v.y, v.x);
}

__device__ double2 nucleon_pair(const double2* S, int pair) {
  const int* e1 = kEps[pair / 6];
  const int* e2 = kEps[pair % 6];
  const int a = e1[0], b = e1[1], c = e1[2];
  const int f = e2[0], e = e2[1], g = e2[2];
  const double sgn = (double)(e1[3] * e2[3]);
  // X = (S^{ag})^T C g5:  X_{rk} = ph(k) S^{ag}_{k^1, r}
  double2 X[16];
  for (int r = 0; r < 4; ++r)
    for (int k = 0; k < 4; ++k) X[4 * r + k] = mul_ph(sld(S, k ^ 1, a, r, g), k);
  // W_N1 = tr[X S^{bf} C g5] tr[S^{ce} P_-]
  double2 t1 = make_double2(0, 0);
  for (int r = 0; r < 4; ++r)
    for (int k = 0; k < 4; ++k) t1 = cadd2(t1, cm(X[4 * r + k], mul_ph(sld(S, k, b, r ^ 1, f), r)));
  double2 t2 = make_double2(0, 0);
  for (int r = 0; r < 4; ++r) {
    const double2 u = sld(S, r, c, r & 1, e), v = sld(S, r, c, (r & 1) + 2, e);
    t2 = make_double2(t2.x + 0.5 * (u.x + v.x), t2.y + 0.5 * (u.y + v.y));
  }
  const double2 w1 = cm(t1, t2);
  // W_N2 = tr[X S^{be} P_- S^{cf} C g5] = sum_{r,k,j} X_{rk} y_{kj} z_{jr}
  double2 y[8], z[8];
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 2; ++j) {
      const double2 u = sld(S, k, b, j, e), v = sld(S, k, b, j + 2, e);
      y[2 * k + j] = make_double2(0.5 * (u.x + v.x), 0.5 * (u.y + v.y));
    }
  for (int j = 0; j < 2; ++j)
    for (int q = 0; q < 4; ++q) {
      const double2 u = sld(S, j, c, q ^ 1, f), v = sld(S, j + 2, c, q ^ 1, f);
      z[4 * j + q] = mul_ph(make_double2(u.x + v.x, u.y + v.y), q);
    }
  double2 w2 = make_double2(0, 0);
  for (int r = 0; r < 4; ++r)
    for (int j = 0; j < 2; ++j) {
      double2 v = make_double2(0, 0);
      for (int k = 0; k < 4; ++k) v = cadd2(v, cm(X[4 * r + k], y[2 * k + j]));
      w2 = cadd2(w2, cm(v, z[4 * j + r]));
    }
  return make_double2(sgn * (w1.x - w2.x), sgn * (w1.y - w2.y));
}

// PART = false: W[level][site] per sink site.  PART = true: W[level][block],
// the sum over the workgroup's kNucSites sites in site order (the sites of a
// workgroup lie in one time slice: every extent is even, so L^3 is a multiple
// of 8).
template <bool PART>
__global__ void __launch_bounds__(64) k_nucleon_site(const double2* __restrict__ terms, size_t V, int nlevels,
                                                     double2* __restrict__ W) {
  __shared__ double2 S[kNucSites][144];
  __shared__ double2 part[64];
  __shared__ double2 sites[kNucSites];
  __shared__ int nz[kNucSites];
  const size_t y0 = (size_t)blockIdx.x * kNucSites;
  const int nsite = (int)(V - y0 < (size_t)kNucSites ? V - y0 : kNucSites);
  const int tid = threadIdx.x;
  const int ls = tid / kNucThreads, q = tid % kNucThreads;
  for (int e = tid; e < kNucSites * 144; e += 64) S[e / 144][e % 144] = make_double2(0, 0);
  for (int level = 0; level < nlevels; ++level) {
    if (tid < kNucSites) nz[tid] = 0;
    __syncthreads();
    // term `level`, column col = 3 beta + b holds S[alpha a][beta b] at component 3 alpha + a
    for (int e = tid; e < 12 * kNucSites * 12; e += 64) {
      const int col = e / (kNucSites * 12), r = e % (kNucSites * 12);
      const int site = r / 12, comp = r % 12;
      if (site < nsite) {
        const double2 t = terms[(((size_t)level * 12 + col) * V + y0) * 12 + r];
        const int al = comp / 3, aa = comp % 3, be = col / 3, bb = col % 3;
        double2& d = S[site][((al * 3 + aa) * 4 + be) * 3 + bb];
        d.x += t.x;
        d.y += t.y;
        if (d.x != 0 || d.y != 0) nz[site] = 1;
      }
    }
    __syncthreads();
    double2 acc = make_double2(0, 0);
    if (ls < nsite && nz[ls])
      for (int p = q; p < 36; p += kNucThreads) acc = cadd2(acc, nucleon_pair(S[ls], p));
    part[tid] = acc;
    __syncthreads();
    if (q == 0 && ls < nsite) {
      double2 s = part[tid];                    // fixed order over the site's threads
      for (int k = 1; k < kNucThreads; ++k) s = cadd2(s, part[tid + k]);
      if (PART) sites[ls] = s;
      else W[(size_t)level * V + y0 + ls] = s;
    }
    if (PART) {
      __syncthreads();
      if (tid == 0) {
        double2 s = sites[0];                   // fixed order over the workgroup's sites
        for (int k = 1; k < nsite; ++k) s = cadd2(s, sites[k]);
        W[(size_t)level * (V / kNucSites) + blockIdx.x] = s;
      }
    }
    __syncthreads();
  }
}

// Fixed-order sum over each time slice: one workgroup per (level, t).
__global__ void k_slice_sum(const double2* __restrict__ W, size_t V, int T, double2* __restrict__ out) {
  const int level = blockIdx.y, t = blockIdx.x;
  const size_t V3 = V / T;
  __shared__ double2 part[256];
  double2 s = make_double2(0, 0);
  for (size_t k = threadIdx.x; k < V3; k += blockDim.x) {
    const double2 w = W[(size_t)level * V + (size_t)t * V3 + k];
    s.x += w.x;
    s.y += w.y;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) part[threadIdx.x] = cadd2(part[threadIdx.x], part[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(size_t)level * T + t] = part[0];
}

// ---------------------------------------------------- connected pseudoscalar
// W[prop][site] = sum over the 12 columns and 12 components of |S|^2 (column
// by column, components in order).  Real, kept as double2 (im = 0) for the slice sum.
__global__ void k_pion_site(const double2* __restrict__ props, size_t V, double2* __restrict__ W) {
  const int prop = blockIdx.y;
  for (size_t y = blockIdx.x * (size_t)blockDim.x + threadIdx.x; y < V; y += (size_t)gridDim.x * blockDim.x) {
    double w = 0;
    for (int col = 0; col < 12; ++col) {
      const double2* v = props + (((size_t)prop * 12 + col) * V + y) * 12;
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const double2 e = v[c];
        w += e.x * e.x + e.y * e.y;
      }
    }
    W[(size_t)prop * V + y] = make_double2(w, 0.0);
  }
}

// out rows: [0, n) levels C^(i) = -sums[i]/L^3; [n, 2n) differences; 2n: rest.
__global__ void k_pion_fin(const double2* __restrict__ sums, int nlevels, int T, int has_full, double invL3,
                           double* __restrict__ out) {
  for (int t = threadIdx.x; t < T; t += blockDim.x) {
    double prev = 0;
    for (int i = 0; i < nlevels; ++i) {
      const double c = -sums[(size_t)i * T + t].x * invL3;
      out[(size_t)i * T + t] = c;
      out[(size_t)(nlevels + i) * T + t] = i == 0 ? c : c - prev;
      prev = c;
    }
    out[(size_t)2 * nlevels * T + t] = has_full ? -sums[(size_t)nlevels * T + t].x * invL3 - prev : 0.0;
  }
}

hipError_t launch_pion(const double2* props, size_t V, int T, int nprops, double2* W, double2* sums,
                       hipStream_t st) {
  size_t g = (V + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_pion_site, dim3((unsigned)g, nprops), dim3(256), 0, st, props, V, W);
  hipLaunchKernelGGL(k_slice_sum, dim3(T, nprops), dim3(256), 0, st, W, V, T, sums);
  return hipGetLastError();
}

hipError_t launch_pion_fin(const double2* sums, int nlevels, int T, int has_full, double invL3, double* out,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_pion_fin, dim3(1), dim3(256), 0, st, sums, nlevels, T, has_full, invL3, out);
  return hipGetLastError();
}

// ------------------------------------------------------- stochastic traces
// out = gamma5 in for n sites of canonical spinors (gamma5 = diag(1, 1, -1, -1))
__global__ void k_gamma5(const double2* __restrict__ in, double2* __restrict__ out, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n * 12; k += (size_t)gridDim.x * blockDim.x) {
    const double2 v = in[k];
    const int comp = (int)(k % 12);
    out[k] = comp < 6 ? v : make_double2(-v.x, -v.y);
  }
}

__global__ void k_noise_dot(const double2* __restrict__ eta, const double2* __restrict__ phi, int nsrc, size_t V,
                            double2* __restrict__ W) {
  for (size_t y = blockIdx.x * (size_t)blockDim.x + threadIdx.x; y < V; y += (size_t)gridDim.x * blockDim.x) {
    double2 w = make_double2(0, 0);
    for (int i = 0; i < nsrc; ++i) {
      const double2* e = eta + ((size_t)i * V + y) * 12;
      const double2* f = phi + ((size_t)i * V + y) * 12;
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const double2 a = e[c], b = f[c];
        w.x += a.x * b.x + a.y * b.y;
        w.y += a.x * b.y - a.y * b.x;
      }
    }
    W[y] = w;
  }
}

hipError_t launch_gamma5(const double2* in, double2* out, size_t nsites, hipStream_t st) {
  size_t g = (nsites * 12 + 255) / 256;
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_gamma5, dim3((unsigned)g), dim3(256), 0, st, in, out, nsites);
  return hipGetLastError();
}

hipError_t launch_noise_trace(const double2* eta, const double2* phi, int nsrc, size_t V, int T, double2* W,
                              double2* sums, hipStream_t st) {
  size_t g = (V + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_noise_dot, dim3((unsigned)g), dim3(256), 0, st, eta, phi, nsrc, V, W);
  hipLaunchKernelGGL(k_slice_sum, dim3(T, 1), dim3(256), 0, st, W, V, T, sums);
  return hipGetLastError();
}

hipError_t launch_nucleon(const double2* terms, size_t V, int T, int nlevels, double2* W, double2* out,
                          hipStream_t st) {
  const unsigned blocks = (unsigned)((V + kNucSites - 1) / kNucSites);
  hipLaunchKernelGGL(k_nucleon_site<false>, dim3(blocks), dim3(64), 0, st, terms, V, nlevels, W);
  hipLaunchKernelGGL(k_slice_sum, dim3(T, nlevels), dim3(256), 0, st, W, V, T, out);
  return hipGetLastError();
}

// ------------------------------------------- nucleon without allocations
// Scratch of the allocation-free nucleon contraction: the per-workgroup
// partial sums [nlevels][V / 8] complex.  One copy per device, resolved once
// per device with hipGetSymbolAddress and used through that address only (in
// host code the array's name is not a device address).  Every call on a
// device shares it; calls that overlap on one device race.
static __device__ __align__(256) double2 scratch[kNucScratchBytes / sizeof(double2)];

namespace {
std::mutex g_scratch_mu;
double2* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t nucleon_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<double2*>(p);
  return hipSuccess;
}

// diffs[0] = levels[0], diffs[i] = levels[i] - levels[i-1] (eq. seriesN)
__global__ void k_level_diffs(const double2* __restrict__ levels, int nlevels, int T, double2* __restrict__ diffs) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < T; t += gridDim.x * blockDim.x) {
    double2 prev = make_double2(0, 0);
    for (int i = 0; i < nlevels; ++i) {
      const double2 c = levels[(size_t)i * T + t];
      diffs[(size_t)i * T + t] = make_double2(c.x - prev.x, c.y - prev.y);
      prev = c;
    }
  }
}

hipError_t launch_nucleon_noalloc(const double2* terms, size_t V, int T, int nlevels, double2* levels,
                                  double2* diffs, int device, hipStream_t st) {
  if (device < 0 || device >= kMaxDevices || nlevels < 1 || T < 1 || V % ((size_t)T * kNucSites))
    return hipErrorInvalidValue;
  double2* P;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    P = g_scratch_ptr[device];
  }
  if (!P) return hipErrorNotInitialized;
  if ((size_t)nlevels * (V / kNucSites) * sizeof(double2) > kNucScratchBytes) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)(V / kNucSites);
  hipLaunchKernelGGL(k_nucleon_site<true>, dim3(blocks), dim3(64), 0, st, terms, V, nlevels, P);
  hipLaunchKernelGGL(k_slice_sum, dim3(T, nlevels), dim3(256), 0, st, P, V / kNucSites, T, levels);
  if (diffs) hipLaunchKernelGGL(k_level_diffs, dim3((T + 63) / 64), dim3(64), 0, st, levels, nlevels, T, diffs);
  return hipGetLastError();
}

}  // namespace ddml
