// Operator blocks: links, clover term and its inverse for one domain box.
//
// Clover term (the O(a) improvement the paper refers to in the footnotes of
// Sections 4 and 6; it gives no formula): Sheikholeslami-Wohlert form
//   c_sw (i/4) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu}(x),   Fhat = (Q_{mu nu} - Q_{nu mu}) / 8,
// Q_{mu nu}(x) the four plaquettes of the (mu,nu) plane at x.  In hopping units
// (M = 2 kappa D) A = 1 + (i kappa c_sw/2) sum_{mu,nu} sigma Fhat = 1 + i kappa c_sw
// sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}.  In the chiral basis sigma_{0k} = diag(s_k, -s_k)
// and sigma_{jk} = -eps_{jkl} diag(s_l, s_l), so
//   A = diag(1 + sum_l s_l (x) X_l^+,  1 + sum_l s_l (x) X_l^-),
//   X_l^{+-} = i kappa c_sw (+-Fhat_{0l} - B_l),  B_1 = Fhat_23, B_2 = Fhat_31, B_3 = Fhat_12.
// Each 6x6 block is Hermitian; it is inverted in FP64 by a Cholesky
// factorisation (a non-positive pivot is reported).  The clover term of every
// site of the domain is built from the full gauge field, so D_Gamma is exactly
// the diagonal block of D (eq. blkdec).
#include "ddml_common.hpp"
#include "launchers.hpp"

namespace ddml {

__device__ __forceinline__ size_t gidx(const int L[4], const int x[4]) {
  return (((size_t)x[0] * L[1] + x[1]) * L[2] + x[2]) * L[3] + x[3];
}

__device__ __forceinline__ const double2* link_ptr(const GaugeView& gv, const int L[4], const int x[4], int mu) {
  const size_t s = gidx(L, x);
  if (gv.region && x[0] >= gv.r_t0 && x[0] < gv.r_t1) {
    const size_t V3 = (size_t)L[1] * L[2] * L[3];
    return gv.region + ((s - (size_t)gv.r_t0 * V3) * 4 + mu) * 9;
  }
  return gv.base + (s * 4 + mu) * 9;
}

__device__ __forceinline__ void load_link(const GaugeView& gv, const int L[4], const int x[4], int mu, double2 u[9]) {
  const double2* p = link_ptr(gv, L, x, mu);
#pragma unroll
  for (int k = 0; k < 9; ++k) u[k] = p[k];
}

// local lexicographic index -> local coords
__device__ __forceinline__ void lex_coords(const int Lb[4], int s, int y[4]) {
  y[3] = s % Lb[3]; s /= Lb[3];
  y[2] = s % Lb[2]; s /= Lb[2];
  y[1] = s % Lb[1];
  y[0] = s / Lb[1];
}

__device__ __forceinline__ int ntiles_of(const BlockSpec& bs) {
  const int Vh = bs.Lb[0] * bs.Lb[1] * bs.Lb[2] * bs.Lb[3] / 2;
  return (Vh + kTile - 1) / kTile;
}

__global__ void k_build_links(GaugeView gv, BlockSpec bs, double2* __restrict__ U64, float2* __restrict__ U32) {
  const int Vb = bs.Lb[0] * bs.Lb[1] * bs.Lb[2] * bs.Lb[3];
  const int nt = ntiles_of(bs);
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < Vb; s += gridDim.x * blockDim.x) {
    int y[4], x[4];
    lex_coords(bs.Lb, s, y);
    for (int m = 0; m < 4; ++m) x[m] = bs.lo[m] + y[m];
    const int p = (y[0] + y[1] + y[2] + y[3]) & 1;
    const int i = s >> 1;
    for (int mu = 0; mu < 4; ++mu) {
      double2 u[9];
      load_link(gv, bs.L, x, mu, u);
      double f = 1.0;
      if (y[mu] == bs.Lb[mu] - 1) {
        if (bs.Lb[mu] != bs.L[mu]) f = 0.0;                  // Dirichlet face of the domain
        else if (mu == 0 && bs.tbc == 1) f = -1.0;          // antiperiodic wrap in time
        else if (mu == 0 && bs.tbc == 2) f = 0.0;           // open: no hop across the time boundary
      }
#pragma unroll
      for (int k = 0; k < 10; ++k) {  // entry 9 is the zero pad of the last pair
        const double2 v = k < 9 ? make_double2(f * u[k].x, f * u[k].y) : make_double2(0, 0);
        const size_t o = lidx(nt, p, mu, k, i);
        if (U64) U64[o] = v;
        if (U32) U32[o] = make_float2((float)v.x, (float)v.y);
      }
    }
  }
}

// --------------------------------------------------------------- SU(3) FP64
__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 dmulc(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// c = a b, with optional adjoints of a and b
__device__ __forceinline__ void m3(const double2 a[9], bool da, const double2 b[9], bool db, double2 c[9]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = make_double2(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        double2 ak = da ? make_double2(a[3 * k + i].x, -a[3 * k + i].y) : a[3 * i + k];
        double2 bk = db ? make_double2(b[3 * j + k].x, -b[3 * j + k].y) : b[3 * k + j];
        s = make_double2(s.x + ak.x * bk.x - ak.y * bk.y, s.y + ak.x * bk.y + ak.y * bk.x);
      }
      c[3 * i + j] = s;
    }
}

__device__ __forceinline__ void shift(const int L[4], const int x[4], int mu, int dmu, int nu, int dnu, int y[4]) {
  for (int m = 0; m < 4; ++m) y[m] = x[m];
  y[mu] = (y[mu] + dmu + L[mu]) % L[mu];
  y[nu] = (y[nu] + dnu + L[nu]) % L[nu];
}

// Fhat_{mu nu}(x) = (Q - Q^dag)/8 with Q the sum of the four counter-clockwise leaves at x
__device__ void field_strength(const GaugeView& gv, const int L[4], const int x[4], int mu, int nu, double2 F[9]) {
  double2 Q[9], a[9], b[9], c[9], d[9], t1[9], t2[9], t3[9];
  int y[4];
  for (int k = 0; k < 9; ++k) Q[k] = make_double2(0, 0);
  // x -> x+mu -> x+mu+nu -> x+nu -> x
  load_link(gv, L, x, mu, a);
  shift(L, x, mu, 1, nu, 0, y); load_link(gv, L, y, nu, b);
  shift(L, x, mu, 0, nu, 1, y); load_link(gv, L, y, mu, c);
  load_link(gv, L, x, nu, d);
  m3(a, false, b, false, t1); m3(t1, false, c, true, t2); m3(t2, false, d, true, t3);
  for (int k = 0; k < 9; ++k) { Q[k].x += t3[k].x; Q[k].y += t3[k].y; }
  // x -> x+nu -> x+nu-mu -> x-mu -> x
  load_link(gv, L, x, nu, a);
  shift(L, x, mu, -1, nu, 1, y); load_link(gv, L, y, mu, b);
  shift(L, x, mu, -1, nu, 0, y); load_link(gv, L, y, nu, c);
  load_link(gv, L, y, mu, d);
  m3(a, false, b, true, t1); m3(t1, false, c, true, t2); m3(t2, false, d, false, t3);
  for (int k = 0; k < 9; ++k) { Q[k].x += t3[k].x; Q[k].y += t3[k].y; }
  // x -> x-mu -> x-mu-nu -> x-nu -> x
  shift(L, x, mu, -1, nu, 0, y); load_link(gv, L, y, mu, a);
  shift(L, x, mu, -1, nu, -1, y); load_link(gv, L, y, nu, b);
  load_link(gv, L, y, mu, c);
  shift(L, x, mu, 0, nu, -1, y); load_link(gv, L, y, nu, d);
  m3(a, true, b, true, t1); m3(t1, false, c, false, t2); m3(t2, false, d, false, t3);
  for (int k = 0; k < 9; ++k) { Q[k].x += t3[k].x; Q[k].y += t3[k].y; }
  // x -> x-nu -> x-nu+mu -> x+mu -> x
  shift(L, x, mu, 0, nu, -1, y); load_link(gv, L, y, nu, a);
  load_link(gv, L, y, mu, b);
  shift(L, x, mu, 1, nu, -1, y); load_link(gv, L, y, nu, c);
  load_link(gv, L, x, mu, d);
  m3(a, true, b, false, t1); m3(t1, false, c, false, t2); m3(t2, false, d, true, t3);
  for (int k = 0; k < 9; ++k) { Q[k].x += t3[k].x; Q[k].y += t3[k].y; }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      F[3 * i + j] = make_double2((Q[3 * i + j].x - Q[3 * j + i].x) * 0.125, (Q[3 * i + j].y + Q[3 * j + i].y) * 0.125);
}

// In-register inverse of a Hermitian positive definite 6x6 matrix (Cholesky).
// Returns false if a pivot is not positive.
__device__ bool herm6_inverse(const double2 A[36], double2 Ai[36]) {
  double2 Lm[36];
  double dinv[6];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 36; ++k) Lm[k] = make_double2(0, 0);
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double dj = A[6 * j + j].x;
#pragma unroll
    for (int k = 0; k < j; ++k) dj -= Lm[6 * j + k].x * Lm[6 * j + k].x + Lm[6 * j + k].y * Lm[6 * j + k].y;
    if (!(dj > 0)) { ok = false; dj = 1.0; }
    const double ljj = sqrt(dj);
    Lm[6 * j + j] = make_double2(ljj, 0);
    dinv[j] = 1.0 / ljj;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      double2 s = A[6 * i + j];
#pragma unroll
      for (int k = 0; k < j; ++k) {
        const double2 t = dmulc(Lm[6 * j + k], Lm[6 * i + k]);  // L_ik conj(L_jk)
        s.x -= t.x; s.y -= t.y;
      }
      Lm[6 * i + j] = make_double2(s.x * dinv[j], s.y * dinv[j]);
    }
  }
  // W = L^{-1} (lower triangular)
  double2 W[36];
#pragma unroll
  for (int k = 0; k < 36; ++k) W[k] = make_double2(0, 0);
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    W[6 * j + j] = make_double2(dinv[j], 0);
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      double2 s = make_double2(0, 0);
#pragma unroll
      for (int k = j; k < i; ++k) {
        const double2 t = dmul(Lm[6 * i + k], W[6 * k + j]);
        s.x += t.x; s.y += t.y;
      }
      W[6 * i + j] = make_double2(-s.x * dinv[i], -s.y * dinv[i]);
    }
  }
  // A^{-1} = W^dag W
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double2 s = make_double2(0, 0);
#pragma unroll
      for (int k = (i > j ? i : j); k < 6; ++k) {
        const double2 t = dmulc(W[6 * k + i], W[6 * k + j]);
        s.x += t.x; s.y += t.y;
      }
      Ai[6 * i + j] = s;
    }
  return ok;
}

// 18 slots of chiral block blk of site i (parity p): 3 packed diagonal pairs,
// then the 15 upper elements row-major
template <typename T2>
__device__ __forceinline__ void store_herm6(const double2 A[36], T2* arr, int nt, int p, int blk, int i) {
  using T = decltype(T2::x);
  arr[cidx(nt, p, 18 * blk + 0, i)] = mk<T2>((T)A[0].x, (T)A[7].x);
  arr[cidx(nt, p, 18 * blk + 1, i)] = mk<T2>((T)A[14].x, (T)A[21].x);
  arr[cidx(nt, p, 18 * blk + 2, i)] = mk<T2>((T)A[28].x, (T)A[35].x);
  int k = 3;
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = r + 1; c < 6; ++c) {
      arr[cidx(nt, p, 18 * blk + k, i)] = mk<T2>((T)A[6 * r + c].x, (T)A[6 * r + c].y);
      ++k;
    }
}

__global__ void k_build_clover(GaugeView gv, BlockSpec bs, double2* __restrict__ A64, double2* __restrict__ Ainv64,
                               float2* __restrict__ Ainv32, int* __restrict__ bad) {
  const int Vb = bs.Lb[0] * bs.Lb[1] * bs.Lb[2] * bs.Lb[3];
  const int nt = ntiles_of(bs);
  const double c = bs.kappa * bs.csw;  // X = i c (...)
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < Vb; s += gridDim.x * blockDim.x) {
    int y[4], x[4];
    lex_coords(bs.Lb, s, y);
    for (int m = 0; m < 4; ++m) x[m] = bs.lo[m] + y[m];
    const int p = (y[0] + y[1] + y[2] + y[3]) & 1;
    const int i = s >> 1;
    double2 F0[3][9], B[3][9];
    if (c != 0.0) {
      field_strength(gv, bs.L, x, 0, 1, F0[0]);
      field_strength(gv, bs.L, x, 0, 2, F0[1]);
      field_strength(gv, bs.L, x, 0, 3, F0[2]);
      double2 F13[9];
      field_strength(gv, bs.L, x, 2, 3, B[0]);   // B_1 = F_23
      field_strength(gv, bs.L, x, 1, 3, F13);    // B_2 = F_31 = -F_13
      for (int k = 0; k < 9; ++k) B[1][k] = make_double2(-F13[k].x, -F13[k].y);
      field_strength(gv, bs.L, x, 1, 2, B[2]);   // B_3 = F_12
    } else {
      for (int l = 0; l < 3; ++l)
        for (int k = 0; k < 9; ++k) F0[l][k] = B[l][k] = make_double2(0, 0);
    }
    for (int blk = 0; blk < 2; ++blk) {
      const double sg = blk == 0 ? 1.0 : -1.0;
      // X_l = i c (sg F_0l - B_l), Hermitian 3x3
      double2 X[3][9];
      for (int l = 0; l < 3; ++l)
        for (int k = 0; k < 9; ++k) {
          const double re = sg * F0[l][k].x - B[l][k].x, im = sg * F0[l][k].y - B[l][k].y;
          X[l][k] = make_double2(-c * im, c * re);
        }
      // block = 1 + s1 X1 + s2 X2 + s3 X3 on (spin, colour)
      double2 A[36];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          const double id = (a == b) ? 1.0 : 0.0;
          const double2 x1 = X[0][3 * a + b], x2 = X[1][3 * a + b], x3 = X[2][3 * a + b];
          A[6 * a + b] = make_double2(id + x3.x, x3.y);                       // (0,0): 1 + X3
          A[6 * (3 + a) + 3 + b] = make_double2(id - x3.x, -x3.y);            // (1,1): 1 - X3
          A[6 * a + 3 + b] = make_double2(x1.x + x2.y, x1.y - x2.x);          // (0,1): X1 - i X2
          A[6 * (3 + a) + b] = make_double2(x1.x - x2.y, x1.y + x2.x);        // (1,0): X1 + i X2
        }
      double2 Ai[36];
      const bool ok = herm6_inverse(A, Ai);
      if (!ok) atomicOr(bad, 1);
      if (A64) store_herm6<double2>(A, A64, nt, p, blk, i);
      if (Ainv64) store_herm6<double2>(Ai, Ainv64, nt, p, blk, i);
      if (Ainv32) store_herm6<float2>(Ai, Ainv32, nt, p, blk, i);
    }
  }
}

hipError_t launch_build_links(const GaugeView& gv, const BlockSpec& bs, double2* U64, float2* U32, hipStream_t st) {
  const int Vb = bs.Lb[0] * bs.Lb[1] * bs.Lb[2] * bs.Lb[3];
  int grid = (Vb + 255) / 256;
  if (grid > 16384) grid = 16384;
  hipLaunchKernelGGL(k_build_links, dim3(grid), dim3(256), 0, st, gv, bs, U64, U32);
  return hipGetLastError();
}
hipError_t launch_build_clover(const GaugeView& gv, const BlockSpec& bs, double2* A64, double2* Ainv64,
                               float2* Ainv32, int* bad, hipStream_t st) {
  const int Vb = bs.Lb[0] * bs.Lb[1] * bs.Lb[2] * bs.Lb[3];
  int grid = (Vb + 127) / 128;
  if (grid > 16384) grid = 16384;
  hipLaunchKernelGGL(k_build_clover, dim3(grid), dim3(128), 0, st, gv, bs, A64, Ainv64, Ainv32, bad);
  return hipGetLastError();
}

// ------------------------------------------------------------ reordering
__global__ void k_gather(const double2* __restrict__ canon, BlockSpec bs, int p, int nrhs, double scale,
                         double2* __restrict__ eo) {
  const int Vb = bs.Lb[0] * bs.Lb[1] * bs.Lb[2] * bs.Lb[3];
  const int nt = ntiles_of(bs);
  const size_t V = (size_t)bs.L[0] * bs.L[1] * bs.L[2] * bs.L[3];
  const size_t n = (size_t)Vb * nrhs;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    const int s = (int)(t % Vb);
    const int col = (int)(t / Vb);
    int y[4], x[4];
    lex_coords(bs.Lb, s, y);
    if (((y[0] + y[1] + y[2] + y[3]) & 1) != p) continue;
    for (int m = 0; m < 4; ++m) x[m] = bs.lo[m] + y[m];
    const double2* src = canon + ((size_t)col * V + gidx(bs.L, x)) * 12;
    const int i = s >> 1;
#pragma unroll
    for (int c = 0; c < 12; ++c)
      eo[fidx(nt, col, c, i)] = make_double2(scale * src[c].x, scale * src[c].y);
  }
}
__global__ void k_scatter(const double2* __restrict__ eo, BlockSpec bs, int p, int nrhs, double scale,
                          double2* __restrict__ canon) {
  const int Vb = bs.Lb[0] * bs.Lb[1] * bs.Lb[2] * bs.Lb[3];
  const int nt = ntiles_of(bs);
  const size_t V = (size_t)bs.L[0] * bs.L[1] * bs.L[2] * bs.L[3];
  const size_t n = (size_t)Vb * nrhs;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    const int s = (int)(t % Vb);
    const int col = (int)(t / Vb);
    int y[4], x[4];
    lex_coords(bs.Lb, s, y);
    if (((y[0] + y[1] + y[2] + y[3]) & 1) != p) continue;
    for (int m = 0; m < 4; ++m) x[m] = bs.lo[m] + y[m];
    double2* dst = canon + ((size_t)col * V + gidx(bs.L, x)) * 12;
    const int i = s >> 1;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const double2 v = eo[fidx(nt, col, c, i)];
      dst[c] = make_double2(scale * v.x, scale * v.y);
    }
  }
}
// ------------------------------------------------- boundary block D_{dGamma}
// The entries of D that join a site x of the domain Gamma to a neighbour y
// outside it (eq. blkdec; the off-diagonal block of eq. Scmpt2):
//   y = x + mu:  -1/2 (1 - gamma_mu) U_mu(x) psi(y)
//   y = x - mu:  -1/2 (1 + gamma_mu) U_mu(y)^dag psi(y)
// with the time-boundary phase (antiperiodic -1, open: no such hop).  One
// thread per (column, site) of the canonical field; sites outside Gamma and
// inner sites write zero.  Each row of a chiral-basis gamma matrix has a
// single entry: (gamma_mu psi)_a = ph * psi_{col}.
__constant__ int kGamCol[4][4] = {{2, 3, 0, 1}, {3, 2, 1, 0}, {3, 2, 1, 0}, {2, 3, 0, 1}};
__constant__ double kGamRe[4][4] = {{-1, -1, -1, -1}, {0, 0, 0, 0}, {-1, 1, 1, -1}, {0, 0, 0, 0}};
__constant__ double kGamIm[4][4] = {{0, 0, 0, 0}, {-1, -1, 1, 1}, {0, 0, 0, 0}, {-1, 1, 1, -1}};

__device__ __forceinline__ bool in_box(const BlockSpec& bs, const int x[4]) {
  bool in = true;
#pragma unroll
  for (int m = 0; m < 4; ++m) in = in && x[m] >= bs.lo[m] && x[m] < bs.lo[m] + bs.Lb[m];
  return in;
}

__global__ void k_boundary(GaugeView gv, BlockSpec bs, const double2* __restrict__ in, double2* __restrict__ out,
                           int nrhs, double scale) {
  const size_t V = (size_t)bs.L[0] * bs.L[1] * bs.L[2] * bs.L[3];
  const size_t n = V * nrhs;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const size_t site = k % V, col = k / V;
    int x[4];
    size_t r = site;
    x[3] = (int)(r % bs.L[3]); r /= bs.L[3];
    x[2] = (int)(r % bs.L[2]); r /= bs.L[2];
    x[1] = (int)(r % bs.L[1]);
    x[0] = (int)(r / bs.L[1]);
    double2 acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = make_double2(0, 0);
    if (in_box(bs, x)) {
      for (int mu = 0; mu < 4; ++mu)
        for (int d = 1; d >= -1; d -= 2) {
          int y[4] = {x[0], x[1], x[2], x[3]};
          y[mu] += d;
          double ph = -0.5 * scale;
          if (y[mu] < 0 || y[mu] >= bs.L[mu]) {
            y[mu] = (y[mu] + bs.L[mu]) % bs.L[mu];
            if (mu == 0 && bs.tbc == 2) continue;
            if (mu == 0 && bs.tbc == 1) ph = -ph;
          }
          if (in_box(bs, y)) continue;
          double2 u[9];
          load_link(gv, bs.L, d > 0 ? x : y, mu, u);
          const double2* psi = in + (col * V + gidx(bs.L, y)) * 12;
          double2 chi[12];  // U psi or U^dag psi, per spin component
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              double2 t = make_double2(0, 0);
#pragma unroll
              for (int j = 0; j < 3; ++j) {
                const double2 v = psi[3 * a + j];
                const double2 w = d > 0 ? dmul(u[3 * i + j], v) : dmulc(u[3 * j + i], v);
                t.x += w.x;
                t.y += w.y;
              }
              chi[3 * a + i] = t;
            }
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const int b = kGamCol[mu][a];
            const double gr = kGamRe[mu][a], gi = kGamIm[mu][a];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              const double2 v = chi[3 * b + i];
              // (1 - d gamma_mu) chi
              const double2 t = make_double2(chi[3 * a + i].x - d * (gr * v.x - gi * v.y),
                                             chi[3 * a + i].y - d * (gr * v.y + gi * v.x));
              acc[3 * a + i].x += ph * t.x;
              acc[3 * a + i].y += ph * t.y;
            }
          }
        }
    }
    double2* o = out + (col * V + site) * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) o[c] = acc[c];
  }
}

hipError_t launch_boundary(const GaugeView& gv, const BlockSpec& bs, const double2* in, double2* out, int nrhs,
                           double scale, hipStream_t st) {
  const size_t n = (size_t)bs.L[0] * bs.L[1] * bs.L[2] * bs.L[3] * nrhs;
  size_t grid = (n + 255) / 256;
  if (grid > 32768) grid = 32768;
  hipLaunchKernelGGL(k_boundary, dim3((unsigned)grid), dim3(256), 0, st, gv, bs, in, out, nrhs, scale);
  return hipGetLastError();
}

// 16-bit copies for the FP16-storage inner solver: links with scale 1 (their
// entries are bounded by 1 in magnitude), A^{-1} with one scale per site.
__global__ void k_quant_links(const double2* __restrict__ U64, h16c* __restrict__ U16, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const double2 u = U64[k];
    U16[k] = h16c{q16((float)u.x * kQ), q16((float)u.y * kQ)};
  }
}
__global__ void k_quant_clover(const double2* __restrict__ A, h16c* __restrict__ A16, float* __restrict__ nrm,
                               int nt) {
  const size_t nsite = (size_t)2 * nt * kTile;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < nsite; t += (size_t)gridDim.x * blockDim.x) {
    const int p = (int)(t / ((size_t)nt * kTile)), i = (int)(t % ((size_t)nt * kTile));
    double m = 0;
    for (int k = 0; k < kCloverSlots; ++k) {
      const double2 a = A[cidx(nt, p, k, i)];
      m = fmax(m, fmax(fabs(a.x), fabs(a.y)));
    }
    const float mf = (float)m;
    const float inv = mf > 0.f ? kQ / mf : 0.f;
    for (int k = 0; k < kCloverSlots; ++k) {
      const double2 a = A[cidx(nt, p, k, i)];
      A16[cidx(nt, p, k, i)] = h16c{q16((float)a.x * inv), q16((float)a.y * inv)};
    }
    nrm[t] = mf;
  }
}
hipError_t launch_quant_links(const double2* U64, h16c* U16, size_t n, hipStream_t st) {
  size_t g = (n + 255) / 256;
  hipLaunchKernelGGL(k_quant_links, dim3((int)(g > 16384 ? 16384 : (g ? g : 1))), dim3(256), 0, st, U64, U16, n);
  return hipGetLastError();
}
hipError_t launch_quant_clover(const double2* Ainv64, h16c* Ainv16, float* nrm, int ntiles, hipStream_t st) {
  size_t g = ((size_t)2 * ntiles * kTile + 255) / 256;
  hipLaunchKernelGGL(k_quant_clover, dim3((int)(g > 16384 ? 16384 : (g ? g : 1))), dim3(256), 0, st, Ainv64, Ainv16,
                     nrm, ntiles);
  return hipGetLastError();
}

static int grid_of(size_t n) {
  size_t g = (n + 255) / 256;
  return (int)(g > 16384 ? 16384 : (g == 0 ? 1 : g));
}
hipError_t launch_gather(const double2* canon, const BlockSpec& bs, int p, int nrhs, double scale, double2* eo,
                         hipStream_t st) {
  const size_t n = (size_t)bs.Lb[0] * bs.Lb[1] * bs.Lb[2] * bs.Lb[3] * nrhs;
  hipLaunchKernelGGL(k_gather, dim3(grid_of(n)), dim3(256), 0, st, canon, bs, p, nrhs, scale, eo);
  return hipGetLastError();
}
hipError_t launch_scatter(const double2* eo, const BlockSpec& bs, int p, int nrhs, double scale, double2* canon,
                          hipStream_t st) {
  const size_t n = (size_t)bs.Lb[0] * bs.Lb[1] * bs.Lb[2] * bs.Lb[3] * nrhs;
  hipLaunchKernelGGL(k_scatter, dim3(grid_of(n)), dim3(256), 0, st, eo, bs, p, nrhs, scale, canon);
  return hipGetLastError();
}

}  // namespace ddml
