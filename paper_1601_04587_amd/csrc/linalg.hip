// Small dense linear algebra of the projector-cut factorization (Section 5.2,
// eqs. approxlong2, fullfactpi): the Cholesky factor of an N x N Gram matrix
// (orthonormalisation of the basis vectors by Cholesky QR) and the traces
// Tr(Gt(y0) G(x0)) of products of per-slice Gram matrices.  The GEMMs around
// them are plain library GEMMs (rocBLAS, linalg_blas.cpp).
#include "ddml_common.hpp"
#include "launchers.hpp"

namespace ddml {

// In place: G (column-major N x N, Hermitian positive definite) -> R upper
// triangular with G = R^dag R and positive real diagonal:
//   R_jj = sqrt(G_jj - sum_{k<j} |R_kj|^2),
//   R_ji = (G_ji - sum_{k<j} conj(R_kj) R_ki) / R_jj      (i > j).
// The strictly lower triangle is set to zero.  One workgroup, sums over k in
// order; a non-positive pivot sets *bad.
__global__ void __launch_bounds__(256) k_cholesky_upper(double2* __restrict__ G, int n, int* __restrict__ bad) {
  __shared__ double piv;
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double d = G[j + (size_t)j * n].x;
      for (int k = 0; k < j; ++k) {
        const double2 r = G[k + (size_t)j * n];
        d -= r.x * r.x + r.y * r.y;
      }
      if (!(d > 0)) {
        atomicOr(bad, 1);
        d = 1.0;
      }
      piv = sqrt(d);
      G[j + (size_t)j * n] = make_double2(piv, 0.0);
    }
    __syncthreads();
    const double inv = 1.0 / piv;
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) {
      double2 s = G[j + (size_t)i * n];
      for (int k = 0; k < j; ++k) {
        const double2 a = G[k + (size_t)j * n], b = G[k + (size_t)i * n];  // conj(a) b
        s.x -= a.x * b.x + a.y * b.y;
        s.y -= a.x * b.y - a.y * b.x;
      }
      G[j + (size_t)i * n] = make_double2(s.x * inv, s.y * inv);
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int r = idx % n, cidx_ = idx / n;
    if (r > cidx_) G[idx] = make_double2(0, 0);
  }
}

hipError_t launch_cholesky_upper(double2* G, int n, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(k_cholesky_upper, dim3(1), dim3(256), 0, st, G, n, bad);
  return hipGetLastError();
}

// out[y * T + x] = scale * Re Tr(Gt[y] G[x]) = scale * Re sum_{i,j} Gt[y]_{ij} G[x]_{ji}
// for slices y in [ya, yb), x in [xa, xb) (other entries untouched); one
// workgroup per (y, x), fixed-order sums.  Column-major N x N blocks.
__global__ void __launch_bounds__(256) k_trace_pairs(const double2* __restrict__ Gt, const double2* __restrict__ G,
                                                     int n, int T, int ya, int xa, double scale,
                                                     double* __restrict__ out) {
  const int y = ya + blockIdx.y, x = xa + blockIdx.x;
  const double2* A = Gt + (size_t)y * n * n;
  const double2* B = G + (size_t)x * n * n;
  __shared__ double part[256];
  double s = 0;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx % n, j = idx / n;        // A_ij at i + j n, B_ji at j + i n
    const double2 a = A[i + (size_t)j * n], b = B[j + (size_t)i * n];
    s += a.x * b.x - a.y * b.y;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(size_t)y * T + x] = scale * part[0];
}

hipError_t launch_trace_pairs(const double2* Gt, const double2* G, int n, int T, int ya, int yb, int xa, int xb,
                              double scale, double* out, hipStream_t st) {
  if (yb <= ya || xb <= xa) return hipSuccess;
  hipLaunchKernelGGL(k_trace_pairs, dim3(xb - xa, yb - ya), dim3(256), 0, st, Gt, G, n, T, ya, xa, scale, out);
  return hipGetLastError();
}

// C[s] (m x n, column-major, leading dimension ldc, slices sC apart) = (or +=)
// sum_{q < Q} P[s Q + q] (m x n each, packed): the reduction of a GEMM whose
// long inner dimension was split into Q chunks, in a fixed order.
__global__ void k_sum_chunks(const double2* __restrict__ P, int Q, int m, int n, int nslices,
                             double2* __restrict__ C, int ldc, size_t sC, int accumulate) {
  const size_t mn = (size_t)m * n, total = mn * nslices;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const size_t s = t / mn, e = t % mn;
    const int i = (int)(e % m), j = (int)(e / m);
    double re = 0, im = 0;
    for (int q = 0; q < Q; ++q) {
      const double2 v = P[(s * Q + q) * mn + e];
      re += v.x;
      im += v.y;
    }
    double2* d = C + s * sC + i + (size_t)j * ldc;
    if (accumulate) {
      re += d->x;
      im += d->y;
    }
    *d = make_double2(re, im);
  }
}

hipError_t launch_sum_chunks(const double2* P, int Q, int m, int n, int nslices, double2* C, int ldc, size_t sC,
                             int accumulate, hipStream_t st) {
  size_t g = ((size_t)m * n * nslices + 255) / 256;
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_sum_chunks, dim3((unsigned)(g ? g : 1)), dim3(256), 0, st, P, Q, m, n, nslices, C, ldc, sC,
                     accumulate);
  return hipGetLastError();
}

// ------------------------------------------------- colourless spinors
// Eq. W0tbary: B[s_i, s_j, s_k; x]_alpha = eps^{abc} (s_i^a(x)^T C g5 s_j^b(x)) s_k^c_alpha(x)
// = sum_c e_ij^c(x) s_k^c_alpha(x), with the colour vector of the diquark
// e_ij^c = eps^{abc} d_ij^{ab}, d_ij^{ab} = sum s_i^a_alpha (C g5)_{alpha beta} s_j^b_beta.
// In the chiral basis C g5 = diag(s2, s2): (C g5)_{01} = (C g5)_{23} = -i,
// (C g5)_{10} = (C g5)_{32} = +i.  Summed over a slice, B is one GEMM of the
// matrices these kernels lay out:
//   E[ij][x][c] = e_ij^c(x)                     (column ij of a 3 ns x N^2 matrix)
//   S[k][alpha][x][c] = s_k^c_alpha(x)          (column 4 k + alpha of a 3 ns x 4N matrix)
// for the ns sites [site0, site0 + ns) of vectors X [N][V][4][3].  xi = 1 takes
// s = conj(g5 X) (the xi_i of a gamma5 phi solve), else s = X.
__device__ __forceinline__ double2 bary_load(const double2* X, size_t V, int n, size_t site, int alpha, int c,
                                             int xi) {
  const double2 v = X[((size_t)n * V + site) * 12 + alpha * 3 + c];
  if (!xi) return v;
  const double g = alpha < 2 ? 1.0 : -1.0;
  return make_double2(g * v.x, -g * v.y);
}

__global__ void __launch_bounds__(256) k_bary_diquark(const double2* __restrict__ X, size_t V, int N, size_t site0,
                                                      int ns, int xi, double2* __restrict__ E) {
  const size_t total = (size_t)N * N * ns;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(t % ns);
    const int ij = (int)(t / ns);
    const int i = ij / N, j = ij % N;
    const size_t site = site0 + x;
    double2 si[4][3], sj[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        si[a][c] = bary_load(X, V, i, site, a, c, xi);
        sj[a][c] = bary_load(X, V, j, site, a, c, xi);
      }
    // d^{ab} = i (s_i1^a s_j0^b - s_i0^a s_j1^b + s_i3^a s_j2^b - s_i2^a s_j3^b)
    auto d = [&](int a, int b) {
      double re = 0, im = 0;
      const int p[4][2] = {{1, 0}, {0, 1}, {3, 2}, {2, 3}};
      const double sg[4] = {1, -1, 1, -1};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 u = si[p[q][0]][a], v = sj[p[q][1]][b];
        re += sg[q] * (u.x * v.x - u.y * v.y);
        im += sg[q] * (u.x * v.y + u.y * v.x);
      }
      return make_double2(-im, re);   // times i
    };
    const double2 d12 = d(1, 2), d21 = d(2, 1), d20 = d(2, 0), d02 = d(0, 2), d01 = d(0, 1), d10 = d(1, 0);
    double2* e = E + ((size_t)ij * ns + x) * 3;
    e[0] = make_double2(d12.x - d21.x, d12.y - d21.y);
    e[1] = make_double2(d20.x - d02.x, d20.y - d02.y);
    e[2] = make_double2(d01.x - d10.x, d01.y - d10.y);
  }
}

__global__ void __launch_bounds__(256) k_bary_spinors(const double2* __restrict__ X, size_t V, int N, size_t site0,
                                                      int ns, int xi, double2* __restrict__ S) {
  const size_t total = (size_t)N * 12 * ns;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % 3);
    const size_t r = t / 3;
    const int x = (int)(r % ns);
    const int ka = (int)(r / ns);     // 4 k + alpha
    S[t] = bary_load(X, V, ka / 4, site0 + x, ka % 4, c, xi);
  }
}

static unsigned grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  return (unsigned)(g > 16384 ? 16384 : (g ? g : 1));
}

hipError_t launch_bary_layout(const double2* X, size_t V, int N, size_t site0, int ns, int xi, double2* E,
                              double2* S, hipStream_t st) {
  hipLaunchKernelGGL(k_bary_diquark, dim3(grid_for((size_t)N * N * ns)), dim3(256), 0, st, X, V, N, site0, ns, xi, E);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bary_spinors, dim3(grid_for((size_t)N * 12 * ns)), dim3(256), 0, st, X, V, N, site0, ns, xi,
                     S);
  return hipGetLastError();
}

// out[y * T + x] = scale * sum_{ijk, r} (Bx[x](j,i,k)_r - Bx[x](k,i,j)_r) (P_- By[y](i,j,k))_r for
// y in [ya, yb), x in [xa, xb), with B[t](i,j,k)_r at [t][(i N + j) + N^2 (4 k + r)] (the
// GEMM output) and P_- = (1 - g0)/2 = [[1, 1], [1, 1]] / 2 in 2x2 blocks.  One
// workgroup per (y, x), fixed-order sums.
__global__ void __launch_bounds__(256) k_bary_pairs(const double2* __restrict__ By, const double2* __restrict__ Bx,
                                                    int N, int T, int ya, int xa, double scale,
                                                    double2* __restrict__ out) {
  const int y = ya + blockIdx.y, x = xa + blockIdx.x;
  const size_t NN = (size_t)N * N, blk = NN * 4 * N;
  const double2* A = Bx + (size_t)x * blk;
  const double2* B = By + (size_t)y * blk;
  __shared__ double2 part[256];
  double re = 0, im = 0;
  const int n3 = N * N * N;
  for (int idx = threadIdx.x; idx < n3; idx += blockDim.x) {
    const int k = idx % N, j = (idx / N) % N, i = idx / (N * N);
    const size_t b0 = (size_t)(i * N + j) + NN * (4 * k);
    const size_t a1 = (size_t)(j * N + i) + NN * (4 * k);      // Bx(j,i,k)
    const size_t a2 = (size_t)(k * N + i) + NN * (4 * j);      // Bx(k,i,j)
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const double2 p0 = B[b0 + NN * r], p1 = B[b0 + NN * (r + 2)];
      const double2 pm = make_double2(0.5 * (p0.x + p1.x), 0.5 * (p0.y + p1.y));
      const double2 u0 = A[a1 + NN * r], u1 = A[a1 + NN * (r + 2)];
      const double2 v0 = A[a2 + NN * r], v1 = A[a2 + NN * (r + 2)];
      // (W_N1 term) - (W_N2 term): equal index triples cancel exactly
      const double2 w = make_double2((u0.x + u1.x) - (v0.x + v1.x), (u0.y + u1.y) - (v0.y + v1.y));
      re += w.x * pm.x - w.y * pm.y;
      im += w.x * pm.y + w.y * pm.x;
    }
  }
  part[threadIdx.x] = make_double2(re, im);
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      part[threadIdx.x].x += part[threadIdx.x + off].x;
      part[threadIdx.x].y += part[threadIdx.x + off].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(size_t)y * T + x] = make_double2(scale * part[0].x, scale * part[0].y);
}

hipError_t launch_bary_pairs(const double2* By, const double2* Bx, int N, int T, int ya, int yb, int xa, int xb,
                             double scale, double2* out, hipStream_t st) {
  if (yb <= ya || xb <= xa) return hipSuccess;
  hipLaunchKernelGGL(k_bary_pairs, dim3(xb - xa, yb - ya), dim3(256), 0, st, By, Bx, N, T, ya, xa, scale, out);
  return hipGetLastError();
}

}  // namespace ddml
