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
// In the chiral basis C = diag(s_2, -s_2), so C g5 = diag(s_2, s_2), and
// P_- = [[1,1],[1,1]]/2 in 2x2 spin blocks; both are applied in closed form below.
#include "ddml_common.hpp"
#include "launchers.hpp"

namespace ddml {

__global__ void k_series_diff(double2* __restrict__ terms, size_t n, int nlevels, double2* __restrict__ sum) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    double2 prev = terms[k];
    for (int l = 1; l < nlevels; ++l) {
      const double2 cur = terms[(size_t)l * n + k];
      terms[(size_t)l * n + k] = make_double2(cur.x - prev.x, cur.y - prev.y);
      prev = cur;
    }
    if (sum) sum[k] = prev;
  }
}

hipError_t launch_series_diff(double2* terms, size_t n, int nlevels, double2* sum, hipStream_t st) {
  size_t g = (n + 255) / 256;
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_series_diff, dim3((int)g), dim3(256), 0, st, terms, n, nlevels, sum);
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

// O = M C g5 with C g5 = diag(s_2, s_2): its only entries are (0,1) = (2,3) = -i and
// (1,0) = (3,2) = +i, so column c of O is column c^1 of M times (+i for even c, -i for odd c).
__device__ __forceinline__ void mul_cg5_right(const double2 M[16], double2 O[16]) {
  for (int r = 0; r < 4; ++r) {
    const double2 m1 = M[4 * r + 1], m0 = M[4 * r + 0], m3v = M[4 * r + 3], m2 = M[4 * r + 2];
    O[4 * r + 0] = make_double2(-m1.y, m1.x);    // +i M_{r1}
    O[4 * r + 1] = make_double2(m0.y, -m0.x);    // -i M_{r0}
    O[4 * r + 2] = make_double2(-m3v.y, m3v.x);  // +i M_{r3}
    O[4 * r + 3] = make_double2(m2.y, -m2.x);    // -i M_{r2}
  }
}
// (M P_-)_{r c} = (M_{r c mod 2} + M_{r, c mod 2 + 2}) / 2 ... P_- = 1/2 [[I, I],[I, I]]
__device__ __forceinline__ void mul_pm_right(const double2 M[16], double2 O[16]) {
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      const int c0 = c & 1;
      O[4 * r + c] = make_double2(0.5 * (M[4 * r + c0].x + M[4 * r + c0 + 2].x),
                                  0.5 * (M[4 * r + c0].y + M[4 * r + c0 + 2].y));
    }
}

// S^{ab} spin matrix at a sink, from LDS holding S[alpha][a][beta][b]
__device__ __forceinline__ void spin_block(const double2* S, int a, int b, double2 M[16]) {
  for (int al = 0; al < 4; ++al)
    for (int be = 0; be < 4; ++be) M[4 * al + be] = S[((al * 3 + a) * 4 + be) * 3 + b];
}

__device__ const int kEps[6][4] = {{0, 1, 2, 1}, {1, 2, 0, 1}, {2, 0, 1, 1}, {0, 2, 1, -1}, {2, 1, 0, -1}, {1, 0, 2, -1}};

// One workgroup of 64 threads per (sink site, level): 36 threads take one
// (abc, feg) pair each.
__global__ void k_nucleon_site(const double2* __restrict__ terms, size_t V, int level_count, int nlevels_total,
                               double2* __restrict__ W) {
  __shared__ double2 S[144];
  __shared__ double2 part[64];
  const size_t y = blockIdx.x;
  const int level = blockIdx.y;
  const int tid = threadIdx.x;
  if (y >= V || level >= level_count) return;
  (void)nlevels_total;
  // S^(level)(y,x)[alpha a][beta b] = sum_{j<=level} terms[j][3 beta + b][y][alpha][a]
  for (int e = tid; e < 144; e += blockDim.x) {
    const int al = e / 36, a = (e / 12) % 3, be = (e / 3) % 4, b = e % 3;
    const int col = 3 * be + b;
    double2 v = make_double2(0, 0);
    for (int j = 0; j <= level; ++j) {
      const double2 t = terms[(((size_t)j * 12 + col) * V + y) * 12 + al * 3 + a];
      v.x += t.x;
      v.y += t.y;
    }
    S[e] = v;
  }
  __syncthreads();
  double2 acc = make_double2(0, 0);
  if (tid < 36) {
    const int* e1 = kEps[tid / 6];
    const int* e2 = kEps[tid % 6];
    const int a = e1[0], b = e1[1], c = e1[2];
    const int f = e2[0], e = e2[1], g = e2[2];
    const double sgn = (double)(e1[3] * e2[3]);
    double2 Sag[16], Sbf[16], Sce[16], Sbe[16], Scf[16], X[16], Y[16], Z[16];
    spin_block(S, a, g, Sag);
    spin_block(S, b, f, Sbf);
    spin_block(S, c, e, Sce);
    spin_block(S, b, e, Sbe);
    spin_block(S, c, f, Scf);
    // X = S^{ag T} Cg5
    double2 SagT[16];
    for (int r = 0; r < 4; ++r)
      for (int q = 0; q < 4; ++q) SagT[4 * r + q] = Sag[4 * q + r];
    mul_cg5_right(SagT, X);
    // W_N1 factor 1: tr[X S^{bf} Cg5]
    mul_cg5_right(Sbf, Y);
    double2 t1 = make_double2(0, 0);
    for (int r = 0; r < 4; ++r)
      for (int k = 0; k < 4; ++k) t1 = cadd2(t1, cm(X[4 * r + k], Y[4 * k + r]));
    // tr[S^{ce} P_-]
    double2 PceM[16];
    mul_pm_right(Sce, PceM);
    double2 t2 = make_double2(0, 0);
    for (int r = 0; r < 4; ++r) t2 = cadd2(t2, PceM[5 * r]);
    const double2 w1 = cm(t1, t2);
    // W_N2: tr[X S^{be} P_- S^{cf} Cg5]
    mul_pm_right(Sbe, Y);          // Y = S^{be} P_-
    mul_cg5_right(Scf, Z);         // Z = S^{cf} Cg5
    double2 YZ[16];
    for (int r = 0; r < 4; ++r)
      for (int q = 0; q < 4; ++q) {
        double2 s = make_double2(0, 0);
        for (int k = 0; k < 4; ++k) s = cadd2(s, cm(Y[4 * r + k], Z[4 * k + q]));
        YZ[4 * r + q] = s;
      }
    double2 w2 = make_double2(0, 0);
    for (int r = 0; r < 4; ++r)
      for (int k = 0; k < 4; ++k) w2 = cadd2(w2, cm(X[4 * r + k], YZ[4 * k + r]));
    acc = make_double2(sgn * (w1.x - w2.x), sgn * (w1.y - w2.y));
  }
  part[tid] = acc;
  __syncthreads();
  if (tid == 0) {
    double2 s = make_double2(0, 0);
    for (int k = 0; k < 36; ++k) s = cadd2(s, part[k]);   // fixed order
    W[(size_t)level * V + y] = s;
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

hipError_t launch_nucleon(const double2* terms, size_t V, int T, int nlevels, double2* W, double2* out,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_nucleon_site, dim3((unsigned)V, nlevels), dim3(64), 0, st, terms, V, nlevels, nlevels, W);
  hipLaunchKernelGGL(k_slice_sum, dim3(T, nlevels), dim3(256), 0, st, W, V, T, out);
  return hipGetLastError();
}

}  // namespace ddml
