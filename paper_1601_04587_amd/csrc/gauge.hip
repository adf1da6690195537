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

__host__ __device__ __forceinline__ int ntiles_of(const BlockSpec& bs) {
  const int Vh = bs.Lb[0] * bs.Lb[1] * bs.Lb[2] * bs.Lb[3] / 2;
  return (Vh + kTile - 1) / kTile;
}

// FP64 links in the 5-pair layout; the FP32 copy keeps the first two rows
// (two-row layout, lidx2) and the stencil rebuilds the third as the complex
// conjugate of the cross product of the first two, times the face factor
// (+-1; 0 zeroes all rows).  That holds for SU(3) matrices only: a link whose
// third row differs from the rebuilt one by more than 1e-5 sets bit 2 of *bad.
__global__ void k_build_links(GaugeView gv, BlockSpec bs, double2* __restrict__ U64, float2* __restrict__ U32,
                              int* __restrict__ bad) {
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
        if (U64) U64[lidx(nt, p, mu, k, i)] = v;
        if (U32 && k < 6) U32[lidx2(nt, p, mu, k, i)] = make_float2((float)v.x, (float)v.y);
      }
      // third row against conj(row 0 x row 1)
      double dev = 0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int a = (q + 1) % 3, b = (q + 2) % 3;
        const double2 x1 = u[a], y1 = u[3 + b], x2 = u[b], y2 = u[3 + a];
        const double cr = (x1.x * y1.x - x1.y * y1.y) - (x2.x * y2.x - x2.y * y2.y);
        const double ci = (x1.x * y1.y + x1.y * y1.x) - (x2.x * y2.y + x2.y * y2.x);
        dev = fmax(dev, fabs(u[6 + q].x - cr) + fabs(u[6 + q].y + ci));
      }
      if (!(dev <= 1e-5)) atomicOr(bad, 2);
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

// y = x + dmu mu + dnu nu (periodic gauge field), without indexing x by mu
__device__ __forceinline__ void nbr(const int L[4], const int x[4], int mu, int dmu, int nu, int dnu, int y[4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int v = x[m] + (m == mu ? dmu : 0) + (m == nu ? dnu : 0);
    y[m] = v < 0 ? v + L[m] : (v >= L[m] ? v - L[m] : v);
  }
}

// acc <- acc U_dir(x + dmu mu + dnu nu)  (or its adjoint)
__device__ __forceinline__ void leaf_step(const GaugeView& gv, const int L[4], const int x[4], int mu, int dmu,
                                          int nu, int dnu, int dir, bool dag, double2 acc[9]) {
  int y[4];
  nbr(L, x, mu, dmu, nu, dnu, y);
  double2 u[9], t[9];
  load_link(gv, L, y, dir, u);
  m3(acc, false, u, dag, t);
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = t[k];
}

// Fhat_{mu nu}(x) = (Q - Q^dag)/8 with Q the sum of the four counter-clockwise
// leaves at x, each built link by link:
//   U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
//   U_nu(x) U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu)
//   U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu)
//   U_nu(x-nu)^dag U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^dag
__device__ __forceinline__ void field_strength(const GaugeView& gv, const int L[4], const int x[4], int mu, int nu,
                                               double2 F[9]) {
  double2 Q[9], acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Q[k] = make_double2(0, 0);
#pragma unroll 1
  for (int leaf = 0; leaf < 4; ++leaf) {
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = make_double2(k % 4 == 0 ? 1.0 : 0.0, 0.0);
    if (leaf == 0) {
      leaf_step(gv, L, x, mu, 0, nu, 0, mu, false, acc);
      leaf_step(gv, L, x, mu, 1, nu, 0, nu, false, acc);
      leaf_step(gv, L, x, mu, 0, nu, 1, mu, true, acc);
      leaf_step(gv, L, x, mu, 0, nu, 0, nu, true, acc);
    } else if (leaf == 1) {
      leaf_step(gv, L, x, mu, 0, nu, 0, nu, false, acc);
      leaf_step(gv, L, x, mu, -1, nu, 1, mu, true, acc);
      leaf_step(gv, L, x, mu, -1, nu, 0, nu, true, acc);
      leaf_step(gv, L, x, mu, -1, nu, 0, mu, false, acc);
    } else if (leaf == 2) {
      leaf_step(gv, L, x, mu, -1, nu, 0, mu, true, acc);
      leaf_step(gv, L, x, mu, -1, nu, -1, nu, true, acc);
      leaf_step(gv, L, x, mu, -1, nu, -1, mu, false, acc);
      leaf_step(gv, L, x, mu, 0, nu, -1, nu, false, acc);
    } else {
      leaf_step(gv, L, x, mu, 0, nu, -1, nu, true, acc);
      leaf_step(gv, L, x, mu, 0, nu, -1, mu, false, acc);
      leaf_step(gv, L, x, mu, 1, nu, -1, nu, false, acc);
      leaf_step(gv, L, x, mu, 0, nu, 0, mu, true, acc);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      Q[k].x += acc[k].x;
      Q[k].y += acc[k].y;
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      F[3 * i + j] = make_double2((Q[3 * i + j].x - Q[3 * j + i].x) * 0.125, (Q[3 * i + j].y + Q[3 * j + i].y) * 0.125);
}

// A Hermitian 6x6 block is kept packed: the real diagonal d[6] and the 15
// upper elements u[] row-major (row r holds columns r+1..5).
__device__ __forceinline__ constexpr int up_idx(int r, int c) { return r * (11 - r) / 2 + (c - r - 1); }
// strictly lower (i > j) packed row-major
__device__ __forceinline__ constexpr int lo_idx(int i, int j) { return i * (i - 1) / 2 + j; }

// Clover term of every site of the box, as the two chiral 6x6 blocks of
//   A = 1 + sum_l s_l (x) X_l^{+-},  X_l^{+-} = i kappa c_sw (+-Fhat_{0l} - B_l),
// accumulated plane by plane so that only one Fhat and the packed block are
// live: the (0,l) planes enter X_l with +-1, (2,3) enters X_1 with -1, (1,3)
// X_2 with +1 (B_2 = Fhat_31 = -Fhat_13) and (1,2) X_3 with -1.  s_3 puts X_3
// on the diagonal spin blocks with + and -, s_1 and s_2 put X_1 - i X_2 on
// the upper off-diagonal spin block.
__global__ void __launch_bounds__(128) k_build_clover(GaugeView gv, BlockSpec bs, double2* __restrict__ A64) {
  const int Vb = bs.Lb[0] * bs.Lb[1] * bs.Lb[2] * bs.Lb[3];
  const int nt = ntiles_of(bs);
  const double c = bs.kappa * bs.csw;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < Vb; s += gridDim.x * blockDim.x) {
    int y[4], x[4];
    lex_coords(bs.Lb, s, y);
    for (int m = 0; m < 4; ++m) x[m] = bs.lo[m] + y[m];
    const int p = (y[0] + y[1] + y[2] + y[3]) & 1;
    const int i = s >> 1;
#pragma unroll 1
    for (int blk = 0; blk < 2; ++blk) {
      const double sg = blk == 0 ? 1.0 : -1.0;
      double dg[6];
      double2 up[15];
#pragma unroll
      for (int k = 0; k < 6; ++k) dg[k] = 1.0;
#pragma unroll
      for (int k = 0; k < 15; ++k) up[k] = make_double2(0, 0);
      if (c != 0.0) {
#pragma unroll 1
        for (int pl = 0; pl < 6; ++pl) {
          const int mu = pl < 3 ? 0 : (pl == 5 ? 1 : (pl == 3 ? 2 : 1));
          const int nu = pl < 3 ? pl + 1 : (pl == 5 ? 2 : 3);
          const int l = pl < 3 ? pl : pl - 3;                       // X_{l+1}
          const double f = pl < 3 ? sg : (pl == 4 ? 1.0 : -1.0);
          double2 F[9];
          field_strength(gv, bs.L, x, mu, nu, F);
          // contribution i c f Fhat to X_{l+1}
          double2 Z[9];
#pragma unroll
          for (int k = 0; k < 9; ++k) Z[k] = make_double2(-c * f * F[k].y, c * f * F[k].x);
          if (l == 2) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
              dg[a] += Z[4 * a].x;
              dg[3 + a] -= Z[4 * a].x;
#pragma unroll
              for (int b2 = a + 1; b2 < 3; ++b2) {
                const double2 z = Z[3 * a + b2];
                up[up_idx(a, b2)].x += z.x;
                up[up_idx(a, b2)].y += z.y;
                up[up_idx(3 + a, 3 + b2)].x -= z.x;
                up[up_idx(3 + a, 3 + b2)].y -= z.y;
              }
            }
          } else {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
              for (int b2 = 0; b2 < 3; ++b2) {
                const double2 z = Z[3 * a + b2];
                double2& u = up[up_idx(a, 3 + b2)];
                if (l == 0) {            // + X_1
                  u.x += z.x;
                  u.y += z.y;
                } else {                 // - i X_2
                  u.x += z.y;
                  u.y -= z.x;
                }
              }
          }
        }
      }
      A64[cidx(nt, p, 18 * blk + 0, i)] = make_double2(dg[0], dg[1]);
      A64[cidx(nt, p, 18 * blk + 1, i)] = make_double2(dg[2], dg[3]);
      A64[cidx(nt, p, 18 * blk + 2, i)] = make_double2(dg[4], dg[5]);
#pragma unroll
      for (int k = 0; k < 15; ++k) A64[cidx(nt, p, 18 * blk + 3 + k, i)] = up[k];
    }
  }
}

// Inverse of each packed block by Cholesky A = L L^dag in FP64:
//   L_jj = sqrt(A_jj - sum_{k<j} |L_jk|^2),  L_ij = (A_ij - sum_{k<j} L_ik conj(L_jk)) / L_jj,
//   W = L^{-1} (lower),  A^{-1} = W^dag W.
// One thread per (parity, block, site); a non-positive pivot sets *bad.
__global__ void __launch_bounds__(128) k_invert_clover(const double2* __restrict__ A64, int nt, int Vh,
                                                       double2* __restrict__ Ainv64, float2* __restrict__ Ainv32,
                                                       int* __restrict__ bad) {
  const size_t n = (size_t)4 * Vh;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % Vh);
    const int pb = (int)(t / Vh);
    const int p = pb >> 1, blk = pb & 1;
    double ad[6];
    double2 au[15];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double2 v = A64[cidx(nt, p, 18 * blk + k, i)];
      ad[2 * k] = v.x;
      ad[2 * k + 1] = v.y;
    }
#pragma unroll
    for (int k = 0; k < 15; ++k) au[k] = A64[cidx(nt, p, 18 * blk + 3 + k, i)];
    double ld[6], dinv[6];
    double2 lo[15];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double dj = ad[j];
#pragma unroll
      for (int k = 0; k < j; ++k) dj -= lo[lo_idx(j, k)].x * lo[lo_idx(j, k)].x + lo[lo_idx(j, k)].y * lo[lo_idx(j, k)].y;
      if (!(dj > 0)) {
        ok = false;
        dj = 1.0;
      }
      ld[j] = sqrt(dj);
      dinv[j] = 1.0 / ld[j];
#pragma unroll
      for (int r = j + 1; r < 6; ++r) {
        // A_rj = conj(A_jr) for r > j
        double2 s2 = make_double2(au[up_idx(j, r)].x, -au[up_idx(j, r)].y);
#pragma unroll
        for (int k = 0; k < j; ++k) {
          const double2 q = dmulc(lo[lo_idx(j, k)], lo[lo_idx(r, k)]);  // L_rk conj(L_jk)
          s2.x -= q.x;
          s2.y -= q.y;
        }
        lo[lo_idx(r, j)] = make_double2(s2.x * dinv[j], s2.y * dinv[j]);
      }
    }
    if (!ok) atomicOr(bad, 1);
    // W = L^{-1}: diagonal dinv, strictly lower wo
    double2 wo[15];
#pragma unroll
    for (int j = 0; j < 6; ++j)
#pragma unroll
      for (int r = j + 1; r < 6; ++r) {
        double2 s2 = dmul(lo[lo_idx(r, j)], make_double2(dinv[j], 0.0));
#pragma unroll
        for (int k = j + 1; k < r; ++k) {
          const double2 q = dmul(lo[lo_idx(r, k)], wo[lo_idx(k, j)]);
          s2.x += q.x;
          s2.y += q.y;
        }
        wo[lo_idx(r, j)] = make_double2(-s2.x * dinv[r], -s2.y * dinv[r]);
      }
    // (A^{-1})_rc = sum_{k >= max(r,c)} conj(W_kr) W_kc; diagonal real
    auto w = [&](int k, int j) { return k == j ? make_double2(dinv[j], 0.0) : wo[lo_idx(k, j)]; };
    double idg[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      double acc = 0;
#pragma unroll
      for (int k = r; k < 6; ++k) {
        const double2 v = w(k, r);
        acc += v.x * v.x + v.y * v.y;
      }
      idg[r] = acc;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double2 v = make_double2(idg[2 * k], idg[2 * k + 1]);
      if (Ainv64) Ainv64[cidx(nt, p, 18 * blk + k, i)] = v;
      if (Ainv32) Ainv32[cidx(nt, p, 18 * blk + k, i)] = make_float2((float)v.x, (float)v.y);
    }
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int cc = r + 1; cc < 6; ++cc) {
        double2 acc = make_double2(0, 0);
#pragma unroll
        for (int k = cc; k < 6; ++k) {
          const double2 q = dmulc(w(k, r), w(k, cc));
          acc.x += q.x;
          acc.y += q.y;
        }
        if (Ainv64) Ainv64[cidx(nt, p, 18 * blk + 3 + up_idx(r, cc), i)] = acc;
        if (Ainv32) Ainv32[cidx(nt, p, 18 * blk + 3 + up_idx(r, cc), i)] = make_float2((float)acc.x, (float)acc.y);
      }
  }
}

hipError_t launch_build_links(const GaugeView& gv, const BlockSpec& bs, double2* U64, float2* U32, int* bad,
                              hipStream_t st) {
  const int Vb = bs.Lb[0] * bs.Lb[1] * bs.Lb[2] * bs.Lb[3];
  int grid = (Vb + 255) / 256;
  if (grid > 16384) grid = 16384;
  hipLaunchKernelGGL(k_build_links, dim3(grid), dim3(256), 0, st, gv, bs, U64, U32, bad);
  return hipGetLastError();
}
hipError_t launch_build_clover(const GaugeView& gv, const BlockSpec& bs, double2* A64, double2* Ainv64,
                               float2* Ainv32, int* bad, hipStream_t st) {
  const int Vb = bs.Lb[0] * bs.Lb[1] * bs.Lb[2] * bs.Lb[3];
  int grid = (Vb + 127) / 128;
  if (grid > 16384) grid = 16384;
  hipLaunchKernelGGL(k_build_clover, dim3(grid), dim3(128), 0, st, gv, bs, A64);
  const int Vh = Vb / 2;
  int grid2 = (4 * Vh + 127) / 128;
  if (grid2 > 16384) grid2 = 16384;
  hipLaunchKernelGGL(k_invert_clover, dim3(grid2), dim3(128), 0, st, A64, ntiles_of(bs), Vh, Ainv64, Ainv32, bad);
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
// single entry: (gamma_mu psi)_a = ph_mu(a) psi_{col_mu(a)}, with
//   col: a ^ 2 for mu = 0, 3 and 3 - a for mu = 1, 2;
//   ph:  -1 (mu 0); -i, -i, +i, +i (mu 1); -1, +1, +1, -1 (mu 2); -i, +i, +i, -i (mu 3).
__device__ __forceinline__ constexpr int gam_col(int mu, int a) { return (mu == 0 || mu == 3) ? (a ^ 2) : 3 - a; }
__device__ __forceinline__ constexpr double gam_re(int mu, int a) {
  return mu == 0 ? -1.0 : (mu == 2 ? ((a == 0 || a == 3) ? -1.0 : 1.0) : 0.0);
}
__device__ __forceinline__ constexpr double gam_im(int mu, int a) {
  return mu == 1 ? (a < 2 ? -1.0 : 1.0) : (mu == 3 ? ((a == 0 || a == 3) ? -1.0 : 1.0) : 0.0);
}

__device__ __forceinline__ bool in_box(const BlockSpec& bs, const int x[4]) {
  bool in = true;
#pragma unroll
  for (int m = 0; m < 4; ++m) in = in && x[m] >= bs.lo[m] && x[m] < bs.lo[m] + bs.Lb[m];
  return in;
}

__global__ void __launch_bounds__(256) k_boundary(GaugeView gv, BlockSpec bs, const double2* __restrict__ in, double2* __restrict__ out,
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
#pragma unroll
      for (int mu = 0; mu < 4; ++mu)
#pragma unroll
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
            const int b = gam_col(mu, a);
            const double gr = gam_re(mu, a), gi = gam_im(mu, a);
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

// ----------------------------------------------------------- level-1 updates
// Quenched updates of the links of the slab [t0, t1) of a gauge version with
// the spatial links of slice t0 fixed (the level-1 updates of the two-level
// integration): Wilson plaquette action; per link a Cabibbo-Marinari
// heatbath over the SU(2) subgroups (0,1), (0,2), (1,2) with the
// Kennedy-Pendleton sampler, n_or SU(2) over-relaxation passes, projection
// onto SU(3).  One launch updates one (direction, parity) class, whose links
// do not enter each other's staples.  Random numbers: Philox4x32-10 (Salmon
// et al., SC'11), key (seed low word, seed high word ^ stream * 0x85EBCA6B),
// counter (site, mu | sweep << 2, 0x5EED, n), uniform (w + 1) / 2^32.
__device__ __forceinline__ void philox4x32_10(uint32_t x[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, x[0]), lo0 = 0xD2511F53u * x[0];
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, x[2]), lo1 = 0xCD9E8D57u * x[2];
    const uint32_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

struct LinkDraws {
  uint32_t k0, k1, c0, c1, n;
  uint32_t w0, w1, w2, w3;
  int left;
  __device__ double next() {
    if (left == 0) {
      uint32_t x[4] = {c0, c1, 0x5EEDu, n};
      philox4x32_10(x, k0, k1);
      w0 = x[0];
      w1 = x[1];
      w2 = x[2];
      w3 = x[3];
      ++n;
      left = 4;
    }
    const uint32_t w = left == 4 ? w0 : (left == 3 ? w1 : (left == 2 ? w2 : w3));
    --left;
    return ((double)w + 1.0) * (1.0 / 4294967296.0);
  }
};

// A = sum over nu != mu of U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
__device__ void wilson_staples(const GaugeView& gv, const int L[4], const int x[4], int mu, double2 A[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) A[k] = make_double2(0, 0);
#pragma unroll 1
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    double2 a[9], b[9], t[9], w[9];
    int y[4];
    nbr(L, x, mu, 1, nu, 0, y);
    load_link(gv, L, y, nu, a);
    nbr(L, x, mu, 0, nu, 1, y);
    load_link(gv, L, y, mu, b);
    m3(a, false, b, true, t);
    load_link(gv, L, x, nu, a);
    m3(t, false, a, true, w);
#pragma unroll
    for (int k = 0; k < 9; ++k) A[k] = make_double2(A[k].x + w[k].x, A[k].y + w[k].y);
    nbr(L, x, mu, 1, nu, -1, y);
    load_link(gv, L, y, nu, a);
    nbr(L, x, mu, 0, nu, -1, y);
    load_link(gv, L, y, mu, b);
    m3(a, true, b, true, t);
    load_link(gv, L, y, nu, a);
    m3(t, false, a, false, w);
#pragma unroll
    for (int k = 0; k < 9; ++k) A[k] = make_double2(A[k].x + w[k].x, A[k].y + w[k].y);
  }
}

__device__ __forceinline__ void quat_times(const double a[4], const double b[4], double c[4]) {
  c[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  c[1] = a[0] * b[1] + b[0] * a[1] - (a[2] * b[3] - a[3] * b[2]);
  c[2] = a[0] * b[2] + b[0] * a[2] - (a[3] * b[1] - a[1] * b[3]);
  c[3] = a[0] * b[3] + b[0] * a[3] - (a[1] * b[2] - a[2] * b[1]);
}

// Kennedy-Pendleton: x0 with density ~ sqrt(1 - x0^2) exp(alpha x0)
__device__ double kp_sample(double alpha, LinkDraws& d) {
  const double twopi = 2.0 * 3.14159265358979323846;
  for (int tries = 0; tries <= 10000; ++tries) {
    const double r1 = d.next(), r2 = d.next(), r3 = d.next(), r4 = d.next();
    const double c = cos(twopi * r2);
    const double lam2 = -(log(r1) + c * c * log(r3)) / (2.0 * alpha);
    if (r4 * r4 <= 1.0 - lam2) return 1.0 - 2.0 * lam2;
  }
  return 1.0;
}

__device__ void level1_link(double2 U[9], const double2 A[9], double beta, int n_or, LinkDraws& d) {
  const double twopi = 2.0 * 3.14159265358979323846;
  for (int pass = 0; pass <= n_or; ++pass)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int i = k == 2 ? 1 : 0, j = k == 0 ? 1 : 2;
      // the 2x2 block (rows and columns i, j) of W = U A
      double2 wii = make_double2(0, 0), wij = wii, wji = wii, wjj = wii;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double2 ui = U[3 * i + c], uj = U[3 * j + c], ai = A[3 * c + i], aj = A[3 * c + j];
        wii = make_double2(wii.x + ui.x * ai.x - ui.y * ai.y, wii.y + ui.x * ai.y + ui.y * ai.x);
        wij = make_double2(wij.x + ui.x * aj.x - ui.y * aj.y, wij.y + ui.x * aj.y + ui.y * aj.x);
        wji = make_double2(wji.x + uj.x * ai.x - uj.y * ai.y, wji.y + uj.x * ai.y + uj.y * ai.x);
        wjj = make_double2(wjj.x + uj.x * aj.x - uj.y * aj.y, wjj.y + uj.x * aj.y + uj.y * aj.x);
      }
      const double q[4] = {0.5 * (wii.x + wjj.x), 0.5 * (wij.y + wji.y), 0.5 * (wij.x - wji.x),
                           0.5 * (wii.y - wjj.y)};
      const double norm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
      if (norm < 1e-14) continue;
      const double vd[4] = {q[0] / norm, -q[1] / norm, -q[2] / norm, -q[3] / norm};
      double R[4];
      if (pass == 0) {
        const double x0 = kp_sample(2.0 * beta * norm / 3.0, d);
        const double rad = sqrt(fmax(0.0, 1.0 - x0 * x0));
        const double ct = 2.0 * d.next() - 1.0, ph = twopi * d.next();
        const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
        const double X[4] = {x0, rad * st * cos(ph), rad * st * sin(ph), rad * ct};
        quat_times(X, vd, R);
      } else {
        quat_times(vd, vd, R);  // over-relaxation keeps Re tr(R W)
      }
      // rows i, j of U <- [[r0 + i r3, r2 + i r1], [-r2 + i r1, r0 - i r3]] (rows i, j)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double2 ui = U[3 * i + c], uj = U[3 * j + c];
        U[3 * i + c] = make_double2(R[0] * ui.x - R[3] * ui.y + R[2] * uj.x - R[1] * uj.y,
                                    R[0] * ui.y + R[3] * ui.x + R[2] * uj.y + R[1] * uj.x);
        U[3 * j + c] = make_double2(-R[2] * ui.x - R[1] * ui.y + R[0] * uj.x + R[3] * uj.y,
                                    -R[2] * ui.y + R[1] * ui.x + R[0] * uj.y - R[3] * uj.x);
      }
    }
  // back onto SU(3): Gram-Schmidt on rows 0 and 1, row 2 = conj(row 0 x row 1)
  double n = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) n += U[c].x * U[c].x + U[c].y * U[c].y;
  n = 1.0 / sqrt(n);
#pragma unroll
  for (int c = 0; c < 3; ++c) U[c] = make_double2(U[c].x * n, U[c].y * n);
  double2 p = make_double2(0, 0);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double2 t = dmulc(U[c], U[3 + c]);
    p.x += t.x;
    p.y += t.y;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double2 t = dmul(p, U[c]);
    U[3 + c] = make_double2(U[3 + c].x - t.x, U[3 + c].y - t.y);
  }
  n = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) n += U[3 + c].x * U[3 + c].x + U[3 + c].y * U[3 + c].y;
  n = 1.0 / sqrt(n);
#pragma unroll
  for (int c = 0; c < 3; ++c) U[3 + c] = make_double2(U[3 + c].x * n, U[3 + c].y * n);
  auto cross = [&](int a, int b, int e, int f) {  // conj(U[a] U[b] - U[e] U[f])
    const double2 t1 = dmul(U[a], U[b]), t2 = dmul(U[e], U[f]);
    return make_double2(t1.x - t2.x, -(t1.y - t2.y));
  };
  U[6] = cross(1, 5, 2, 4);
  U[7] = cross(2, 3, 0, 5);
  U[8] = cross(0, 4, 1, 3);
}

// One thread per link of the class: sites of parity `par` in slices
// [t0, t1) (spatial directions: [t0 + 1, t1)), enumerated as pairs along x3.
__global__ void __launch_bounds__(128) k_level1_class(GaugeView gv, double2* __restrict__ region, BlockSpec bs,
                                                       int mu, int par, double beta, uint32_t k0, uint32_t k1,
                                                       int sweep, int n_or) {
  const int ta = gv.r_t0 + (mu != 0), t1 = gv.r_t1;  // frozen spatial links of the first slice
  const int h3 = bs.L[3] / 2;
  const size_t rows = (size_t)(t1 - ta) * bs.L[1] * bs.L[2];
  const size_t n = rows * h3;
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    int x[4];
    size_t r = k / h3;
    const int j = (int)(k - r * h3);
    x[2] = (int)(r % bs.L[2]); r /= bs.L[2];
    x[1] = (int)(r % bs.L[1]);
    x[0] = ta + (int)(r / bs.L[1]);
    x[3] = 2 * j + ((par + x[0] + x[1] + x[2]) & 1);
    const size_t s = gidx(bs.L, x);
    double2 A[9], U[9];
    wilson_staples(gv, bs.L, x, mu, A);
    load_link(gv, bs.L, x, mu, U);
    LinkDraws d{k0, k1, (uint32_t)s, (uint32_t)(mu | (sweep << 2)), 0u, 0u, 0u, 0u, 0u, 0};
    level1_link(U, A, beta, n_or, d);
    double2* dst = region + ((s - (size_t)gv.r_t0 * bs.L[1] * bs.L[2] * bs.L[3]) * 4 + mu) * 9;
#pragma unroll
    for (int c = 0; c < 9; ++c) dst[c] = U[c];
  }
}

hipError_t launch_level1_sweeps(const GaugeView& gv, double2* region, const BlockSpec& bs, double beta,
                                uint64_t seed, uint32_t stream, int nsweeps, int n_or, hipStream_t st) {
  const size_t n = (size_t)(gv.r_t1 - gv.r_t0) * bs.L[1] * bs.L[2] * bs.L[3] / 2;
  size_t grid = (n + 127) / 128;
  if (grid > 16384) grid = 16384;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32) ^ (stream * 0x85EBCA6Bu);
  for (int sweep = 0; sweep < nsweeps; ++sweep)
    for (int mu = 0; mu < 4; ++mu)
      for (int par = 0; par < 2; ++par) {
        hipLaunchKernelGGL(k_level1_class, dim3((unsigned)grid), dim3(128), 0, st, gv, region, bs, mu, par, beta, k0,
                           k1, sweep, n_or);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
      }
  return hipSuccess;
}

// 16-bit copies for the FP16-storage inner solver: links with scale 1 (their
// entries are bounded by 1 in magnitude), A^{-1} with one scale per site.
__global__ void k_quant_links(const float2* __restrict__ U32, h16c* __restrict__ U16, size_t n) {
  for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x) {
    const float2 u = U32[k];
    U16[k] = h16c{q16(u.x * kQ), q16(u.y * kQ)};
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
hipError_t launch_quant_links(const float2* U32, h16c* U16, size_t n, hipStream_t st) {
  size_t g = (n + 255) / 256;
  hipLaunchKernelGGL(k_quant_links, dim3((int)(g > 16384 ? 16384 : (g ? g : 1))), dim3(256), 0, st, U32, U16, n);
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
