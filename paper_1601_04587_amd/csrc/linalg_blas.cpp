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

// C[s] = op(A_s) B_s for nslices consecutive row blocks of K rows (A_s = A + s K,
// B_s = B + s K; op = transpose or conjugate transpose, so the K rows are the
// inner dimension), accumulate: C[s] += instead of =.  The products here are
// tall and thin (m, n <= a few hundred, K up to millions): one GEMM of the whole
// K keeps only m n / tile^2 workgroups busy, so K is split into Q chunks that
// run as one strided-batched GEMM into partial products, summed in a fixed
// order by k_sum_chunks.
static void ksplit_gemm(Ctx* c, rocblas_operation opA, int m, int n, size_t K, const double2* A, size_t lda,
                        const double2* B, size_t ldb, int nslices, double2* C, int ldc, size_t sC, int accumulate) {
  int Q = 1;
  const size_t part = (size_t)nslices * m * n * sizeof(double2);   // one chunk's partial products
  while (Q < 1024 && K % (2 * (size_t)Q) == 0 && K / (2 * (size_t)Q) >= 2048 && 2 * Q * part <= ((size_t)1 << 29))
    Q *= 2;
  const size_t Kc = K / Q;
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
  DBuf P(c->pool.get(), (size_t)nslices * Q * m * n * sizeof(double2));
  chk(rocblas_zgemm_strided_batched(blas(c), opA, rocblas_operation_none, m, n, (rocblas_int)Kc, &one,
                                    reinterpret_cast<const rocblas_double_complex*>(A), (rocblas_int)lda,
                                    (rocblas_stride)Kc, reinterpret_cast<const rocblas_double_complex*>(B),
                                    (rocblas_int)ldb, (rocblas_stride)Kc, &zero, P.as<rocblas_double_complex>(), m,
                                    (rocblas_stride)m * n, nslices * Q),
      "zgemm_strided_batched");
  DDML_HIP(launch_sum_chunks(P.as<double2>(), Q, m, n, nslices, C, ldc, sC, accumulate, c->stream));
}

// X: n canonical fields [n][V][12] (column j at X + j V 12); G: [T][n][n] column-major.
void gram_slices(Ctx* c, const double2* X, int n, size_t V, int T, int t0, int t1, double2* G) {
  DDML_HIP(hipMemsetAsync(G, 0, (size_t)T * n * n * sizeof(double2), c->stream));
  if (t1 <= t0) return;
  const size_t K = 12 * (V / T);
  const double2* A = X + (size_t)t0 * K;
  ksplit_gemm(c, rocblas_operation_conjugate_transpose, n, n, K, A, 12 * V, A, 12 * V, t1 - t0,
              G + (size_t)t0 * n * n, n, (size_t)n * n, 0);
}

// Columns of X restricted to rows [row0, row0 + nrows) (zero elsewhere) made
// orthonormal: X <- X R^{-1}, G = X^dag X = R^dag R, twice.
void orthonormalize(Ctx* c, double2* X, int n, size_t V, size_t row0, size_t nrows) {
  DBuf G(c->pool.get(), (size_t)n * n * sizeof(double2));
  const rocblas_double_complex one = {1.0, 0.0};
  auto* A = reinterpret_cast<rocblas_double_complex*>(X) + row0;
  auto* R = G.as<rocblas_double_complex>();
  const rocblas_int lda = (rocblas_int)(12 * V);
  DDML_HIP(hipMemsetAsync(c->flag.p, 0, sizeof(int), c->stream));
  for (int pass = 0; pass < 2; ++pass) {
    ksplit_gemm(c, rocblas_operation_conjugate_transpose, n, n, nrows, X + row0, 12 * V, X + row0, 12 * V, 1,
                G.as<double2>(), n, 0, 0);
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
  for (int t = t0; t < t1; ++t)
    for (size_t off = 0; off < V3; off += ns) {
      const int cnt = (int)std::min(ns, V3 - off);
      DDML_HIP(launch_bary_layout(X, V, n, (size_t)t * V3 + off, cnt, xi, E.as<double2>(), S.as<double2>(),
                                  c->stream));
      ksplit_gemm(c, rocblas_operation_transpose, n * n, 4 * n, 3 * (size_t)cnt, E.as<double2>(), 3 * (size_t)cnt,
                  S.as<double2>(), 3 * (size_t)cnt, 1, B + (size_t)t * blk, n * n, 0, off ? 1 : 0);
    }
}

}  // namespace ddml
