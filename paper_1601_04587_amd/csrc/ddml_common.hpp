// Internal definitions shared by the HIP kernels and the host engine of libddml.
//
// Conventions (hopping units).  With m0 = 1/(2 kappa) - 4 the Wilson-Dirac
// operator of Appendix A satisfies 2 kappa D = 1 - kappa D_hop (Section 6); with
// the Sheikholeslami-Wohlert term it becomes M = 2 kappa D = A - kappa H, where
// H = D_hop and A = 1 + i kappa c_sw sum_{mu<nu} sigma_{mu nu} Fhat_{mu nu}.
// A domain solve D_Gamma x = b is carried out as M_Gamma x = 2 kappa b.
//
// Domain-local storage ("operator block").  A domain Gamma = [lo,hi) is stored
// as its own box with even extents Lb[mu], sites split by local parity
// (sum of local coordinates mod 2) and indexed by lex/2 inside each parity.
// Every field is structure-of-arrays with the site index fastest:
//   spinor field of one parity : T2 [nrhs][12][Vh]       (component = spin*3 + colour)
//   links                      : T2 [2][4][9][Vh]        (U_mu(x) for x of each parity)
//   clover A or A^{-1}         : T2 [2][36][Vh]          (two Hermitian 6x6 chiral blocks,
//                                                        18 slots each: 3 packed diagonal pairs,
//                                                        then the 15 upper elements row-major)
// Neighbours are taken with local periodic wrap-around.  Links that would leave
// Gamma through a face that is not a full lattice extent are stored as zero, so
// the Dirichlet restriction of eq. blkdec needs no branch in the stencil; the
// antiperiodic time phase is folded into the time links of the wrap.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddml {

constexpr int kTile = 64;          // sites per tile (one wavefront)
constexpr int kMaxRhs = 12;

// ------------------------------------------------------------------ complex
template <typename T> struct Cpx;
template <> struct Cpx<float> { using T2 = float2; };
template <> struct Cpx<double> { using T2 = double2; };

template <typename T2> __host__ __device__ inline T2 mk(decltype(T2::x) a, decltype(T2::x) b) {
  T2 r; r.x = a; r.y = b; return r;
}
template <typename T2> __device__ __forceinline__ T2 cadd(T2 a, T2 b) { return mk<T2>(a.x + b.x, a.y + b.y); }
template <typename T2> __device__ __forceinline__ T2 csub(T2 a, T2 b) { return mk<T2>(a.x - b.x, a.y - b.y); }
template <typename T2> __device__ __forceinline__ T2 cmul(T2 a, T2 b) {
  return mk<T2>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename T2> __device__ __forceinline__ T2 cmulc(T2 a, T2 b) {
  return mk<T2>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename T2> __device__ __forceinline__ T2 cscale(T2 a, decltype(T2::x) s) { return mk<T2>(a.x * s, a.y * s); }
// i*a and -i*a
template <typename T2> __device__ __forceinline__ T2 ci(T2 a) { return mk<T2>(-a.y, a.x); }
template <typename T2> __device__ __forceinline__ T2 cmi(T2 a) { return mk<T2>(a.y, -a.x); }

// ------------------------------------------------------------------ geometry
struct BoxGeom {
  int L[4];     // box extents (all even)
  int Vh;       // sites per parity
  int half3;    // L[3]/2
};

// local coordinates of EO index i of parity p
__device__ __forceinline__ void eo_coords(const BoxGeom& g, int p, int i, int y[4]) {
  int j = i % g.half3;
  int rest = i / g.half3;
  y[2] = rest % g.L[2]; rest /= g.L[2];
  y[1] = rest % g.L[1];
  y[0] = rest / g.L[1];
  y[3] = 2 * j + ((p + y[0] + y[1] + y[2]) & 1);
}
__device__ __forceinline__ int eo_index(const BoxGeom& g, const int y[4]) {
  return (((y[0] * g.L[1] + y[1]) * g.L[2] + y[2]) * g.L[3] + y[3]) >> 1;
}

// ---------------------------------------------------------- kernel argument
// Work item of the batched launches: one domain solve (or one operator
// application) with its own box, operator data and vectors.
template <typename T2> struct HopItem {
  BoxGeom g;
  const T2* U;        // links [2][4][9][Vh]
  const T2* clov;     // clover data of the output parity [36][Vh] (A or A^{-1}), may be null
  const T2* in;       // input field on the opposite parity [nrhs][12][Vh]
  const T2* aux;      // field on the output parity, may be null
  const T2* red_a;    // first operand of a fused dot product, may be null
  T2* out;            // output field on the output parity
  double2* partial;   // fused reduction partials [nred][nrhs][ntiles], may be null
  const int* active;  // per-rhs flag, may be null (all active)
  int par_out;
  int nrhs;
  int ntiles;
  double c1, c2;
};

// Stencil epilogues (acc = H in on the output parity):
//   MODE_CINV_HOP  out = C acc                       (C = A^{-1}_pp)
//   MODE_SCHUR     out = aux - c1 C acc              (c1 = kappa^2: the Schur operator)
//   MODE_M         out = c2 (C aux - c1 acc)         (C = A_pp, c1 = kappa: M = A - kappa H)
//   MODE_PREP      out = C (aux + c1 acc)            (C = A^{-1}_pp: EO prepare/reconstruct)
//   MODE_RES       out = red_a - (C aux - c1 acc)    (residual b - M x)
enum { MODE_CINV_HOP = 0, MODE_SCHUR = 1, MODE_M = 2, MODE_PREP = 3, MODE_RES = 4 };
// Fused reductions (FP64 partial sums per 64-site tile and column):
//   RED_DOT  (red_a, out);  RED_TS  (out, aux) and |out|^2;  RED_NORM |out|^2
enum { RED_NONE = 0, RED_DOT = 1, RED_TS = 2, RED_NORM = 3 };

// Krylov vector slots of one inner solve (even parity unless noted)
enum { F_R = 0, F_RH = 1, F_P = 2, F_V = 3, F_S = 4, F_T = 5, F_X = 6, F_TMP = 7 /* odd */, F_NUM = 8 };

// Per right-hand-side BiCGstab scalars (device resident).
struct BiState {
  double2 rho, alpha, omega, beta;
  double rr;        // |r|^2 of the inner recursion
  double rr0;       // |r|^2 at the start of the inner solve
  double tol2;      // stop when rr <= tol2 * rr0
  int active;       // 1 while iterating
  int iters;
  int max_iters;
  int status;       // 0 ok/converged, 1 breakdown, 2 max iterations
};

// One inner-solver slot as seen by the batched kernels.
template <typename T2> struct SlotDesc {
  BoxGeom g;
  int nrhs;
  int ntiles;
  double kappa;
  const T2* U;          // links [2][4][9][Vh] in the inner precision
  const T2* Ainv;       // A^{-1} [2][36][Vh] in the inner precision
  T2* f[F_NUM];         // Krylov vectors [nrhs][12][Vh]
  double2* partial;     // [2][nrhs][ntiles]
  int* active;          // [nrhs]
  BiState* st;          // [nrhs]
  const double2* src64; // FP64 even-parity right-hand side [nrhs][12][Vh]
};

}  // namespace ddml
