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

}  // namespace ddml
