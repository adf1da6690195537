// Library GEMMs of the projector-cut factorization (rocBLAS on the library
// stream): per-slice Gram matrices G(t) = X_t^dag X_t of a set of canonical
// spinor fields (eq. Bpions summed over the slice) and the orthonormalisation
// of a basis by Cholesky QR, applied twice (the second pass restores the
// orthogonality the first loses to rounding: ||Q^dag Q - 1|| ~ eps instead of
// eps cond(X)^2).
#include <rocblas/rocblas.h>

#include <algorithm>

#include "engine.hpp"

namespace ddml {

static rocblas_handle blas(Ctx* c) {
  if (!c->blas) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) throw Error{DDML_EDEVICE, "rocblas_create_handle failed"};
    c->blas = h;
  }
  rocblas_handle h = (rocblas_handle)c->blas;
  if (rocblas_set_stream(h, c->stream) != rocblas_status_success) throw Error{DDML_EDEVICE, "rocblas_set_stream failed"};
  return h;
}

static void chk(rocblas_status s, const char* what) {
  if (s != rocblas_status_success) throw Error{DDML_EDEVICE, std::string("rocBLAS ") + what + " failed"};
}

void blas_release(Ctx* c) {
  if (c->blas) (void)rocblas_destroy_handle((rocblas_handle)c->blas);
  c->blas = nullptr;
}

// X: n canonical fields [n][V][12] (column j at X + j V 12); G: [T][n][n] column-major.
void gram_slices(Ctx* c, const double2* X, int n, size_t V, int T, int t0, int t1, double2* G) {
  DDML_HIP(hipMemsetAsync(G, 0, (size_t)T * n * n * sizeof(double2), c->stream));
  if (t1 <= t0) return;
  const size_t K = 12 * (V / T);
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
  const auto* A = reinterpret_cast<const rocblas_double_complex*>(X) + (size_t)t0 * K;
  auto* C = reinterpret_cast<rocblas_double_complex*>(G) + (size_t)t0 * n * n;
  chk(rocblas_zgemm_strided_batched(blas(c), rocblas_operation_conjugate_transpose, rocblas_operation_none, n, n,
                                    (rocblas_int)K, &one, A, (rocblas_int)(12 * V), (rocblas_stride)K, A,
                                    (rocblas_int)(12 * V), (rocblas_stride)K, &zero, C, n, (rocblas_stride)n * n,
                                    t1 - t0),
      "zgemm_strided_batched");
}

// Columns of X restricted to rows [row0, row0 + nrows) (zero elsewhere) made
// orthonormal: X <- X R^{-1}, G = X^dag X = R^dag R, twice.
void orthonormalize(Ctx* c, double2* X, int n, size_t V, size_t row0, size_t nrows) {
  DBuf G(c->pool.get(), (size_t)n * n * sizeof(double2));
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
  auto* A = reinterpret_cast<rocblas_double_complex*>(X) + row0;
  auto* R = G.as<rocblas_double_complex>();
  const rocblas_int lda = (rocblas_int)(12 * V);
  DDML_HIP(hipMemsetAsync(c->flag.p, 0, sizeof(int), c->stream));
  for (int pass = 0; pass < 2; ++pass) {
    chk(rocblas_zgemm(blas(c), rocblas_operation_conjugate_transpose, rocblas_operation_none, n, n,
                      (rocblas_int)nrows, &one, A, lda, A, lda, &zero, R, n),
        "zgemm");
    DDML_HIP(launch_cholesky_upper(G.as<double2>(), n, c->flag.as<int>(), c->stream));
    chk(rocblas_ztrsm(blas(c), rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                      rocblas_diagonal_non_unit, (rocblas_int)nrows, n, &one, R, n, A, lda),
        "ztrsm");
  }
  int bad = 0;
  DDML_HIP(hipMemcpyAsync(&bad, c->flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  DDML_HIP(hipStreamSynchronize(c->stream));
  if (bad) throw Error{DDML_ENUMERIC, "basis vectors are linearly dependent (Cholesky pivot <= 0)"};
}

// Slice sums of the colourless spinors (eq. W0tbary) of the n fields X for the
// slices [t0, t1): B[t] (column-major n^2 x 4n, entry (i n + j, 4 k + alpha))
// = sum_{x in t} E(x)^T S(x), one ZGEMM per chunk of sites (the chunk keeps the
// diquark matrix E near 1 GiB), accumulated over the chunks of a slice.
void bary_slices(Ctx* c, const double2* X, int n, size_t V, int T, int t0, int t1, int xi, double2* B) {
  const size_t blk = (size_t)n * n * 4 * n;
  DDML_HIP(hipMemsetAsync(B, 0, (size_t)T * blk * sizeof(double2), c->stream));
  if (t1 <= t0) return;
  const size_t V3 = V / T;
  const size_t per_site = (size_t)n * n * 3 * sizeof(double2);
  size_t ns = ((size_t)1 << 30) / per_site;
  ns = std::max<size_t>(1, std::min(ns, V3));
  DBuf E(c->pool.get(), ns * per_site), S(c->pool.get(), (size_t)n * 12 * ns * sizeof(double2));
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
  for (int t = t0; t < t1; ++t)
    for (size_t off = 0; off < V3; off += ns) {
      const int cnt = (int)std::min(ns, V3 - off);
      DDML_HIP(launch_bary_layout(X, V, n, (size_t)t * V3 + off, cnt, xi, E.as<double2>(), S.as<double2>(),
                                  c->stream));
      chk(rocblas_zgemm(blas(c), rocblas_operation_transpose, rocblas_operation_none, n * n, 4 * n, 3 * cnt, &one,
                        E.as<rocblas_double_complex>(), 3 * cnt, S.as<rocblas_double_complex>(), 3 * cnt,
                        off ? &one : &zero, reinterpret_cast<rocblas_double_complex*>(B) + (size_t)t * blk, n * n),
          "zgemm");
    }
}

}  // namespace ddml
