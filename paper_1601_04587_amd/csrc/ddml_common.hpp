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
// Every field is tile-blocked and pair-packed: sites come in tiles of 64 (one
// wavefront); inside a tile, complex numbers are grouped in pairs and each
// pair is a contiguous run of 64 sites x 2 values.  A lane then reads two
// complex numbers with one 16-byte load (FP32) and a wavefront load is one
// 1 KiB burst; the data of a tile sits in a few KiB instead of planes
// megabytes apart (which alias in the L2 sets).
//   spinor field of one parity : [nrhs][ntiles][6 pairs][64][2]  (component = spin*3 + colour)
//   links, FP64                : [2][ntiles][4 mu][5 pairs][64][2] (9 entries + 1 zero pad)
//   links, FP32 and 16-bit     : [2][ntiles][4 mu][3 pairs][64][2] (the first two rows; the
//                                stencil rebuilds the third, see stage_tile)
//   clover A or A^{-1}         : [2][ntiles][18 pairs][64][2]   (two Hermitian 6x6 chiral blocks,
//                                                              18 slots each: 3 packed diagonal
//                                                              pairs, then the 15 upper elements)
// ntiles = ceil(Vh/64); the padding sites of the last tile hold zeros.
// Neighbours are taken with local periodic wrap-around.  Links that would leave
// Gamma through a face that is not a full lattice extent are stored as zero, so
// the Dirichlet restriction of eq. blkdec needs no branch in the stencil; the
// antiperiodic time phase is folded into the time links of the wrap, and with
// open time boundaries those links are zero as well.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddml {

constexpr int kTile = 64;          // sites per tile (one wavefront)
constexpr int kMaxRhs = 12;

// ------------------------------------------------------- 16-bit storage
// Inner-solver fields of DDML_MIXED_FP16 store a complex number as two int16
// (fixed point): value = q * scale / 32767.  Spinors carry one FP32 scale per
// (site, column), the largest |real component| of its 24 reals; the clover data
// one scale per site; links none (scale 1: every entry of an SU(3) matrix has
// |Re|, |Im| <= 1).  Arithmetic is FP32.
struct h16c {
  short x, y;
};
constexpr float kQ = 32767.0f;
// compute type of an element type
template <typename E> struct CompOf { using type = E; };
template <> struct CompOf<h16c> { using type = float2; };

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
// acc + a b and acc + conj(a) b as four fused multiply-adds
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }
// acc + s a for a real s, as two fused multiply-adds
template <typename T2> __device__ __forceinline__ T2 cmas(T2 acc, T2 a, decltype(T2::x) s) {
  return mk<T2>(fmadd(a.x, s, acc.x), fmadd(a.y, s, acc.y));
}
template <typename T2> __device__ __forceinline__ T2 cmac(T2 acc, T2 a, T2 b) {
  acc.x = fmadd(a.x, b.x, acc.x);
  acc.x = fmadd(-a.y, b.y, acc.x);
  acc.y = fmadd(a.x, b.y, acc.y);
  acc.y = fmadd(a.y, b.x, acc.y);
  return acc;
}
template <typename T2> __device__ __forceinline__ T2 cmacc(T2 acc, T2 a, T2 b) {
  acc.x = fmadd(a.x, b.x, acc.x);
  acc.x = fmadd(a.y, b.y, acc.x);
  acc.y = fmadd(a.x, b.y, acc.y);
  acc.y = fmadd(-a.y, b.x, acc.y);
  return acc;
}
// i*a and -i*a
template <typename T2> __device__ __forceinline__ T2 ci(T2 a) { return mk<T2>(-a.y, a.x); }
template <typename T2> __device__ __forceinline__ T2 cmi(T2 a) { return mk<T2>(a.y, -a.x); }

// ------------------------------------------------------------------ geometry
struct BoxGeom {
  int L[4];     // box extents (all even)
  int Vh;       // sites per parity
  int half3;    // L[3]/2
  int ntiles;   // ceil(Vh / 64)
  int twrap;    // 1 if the time links of the box's last slice carry the antiperiodic sign
                // (the box spans the whole antiperiodic time extent), else 0
};

// tile-blocked, pair-packed offsets (in complex numbers)
constexpr int kSpinorSlots = 12;  // complex per site of a spinor
constexpr int kLinkSlots = 40;    // complex per site of the 4 links (9 + 1 pad each)
constexpr int kCloverSlots = 36;  // complex per site of the clover data
__host__ __device__ __forceinline__ size_t fidx(int ntiles, int col, int c, int i) {
  return ((size_t)(col * ntiles + (i >> 6)) * 6 + (c >> 1)) * 128 + (i & 63) * 2 + (c & 1);
}
__host__ __device__ __forceinline__ size_t lidx(int ntiles, int par, int mu, int k, int i) {
  return ((size_t)(par * ntiles + (i >> 6)) * 20 + mu * 5 + (k >> 1)) * 128 + (i & 63) * 2 + (k & 1);
}
// the two-row link layout of the FP32 and 16-bit copies (entries k = 0..5)
constexpr int kLinkSlots2 = 24;   // complex per site of the 4 links (two rows each)
__host__ __device__ __forceinline__ size_t lidx2(int ntiles, int par, int mu, int k, int i) {
  return ((size_t)(par * ntiles + (i >> 6)) * 12 + mu * 3 + (k >> 1)) * 128 + (i & 63) * 2 + (k & 1);
}
__host__ __device__ __forceinline__ size_t cidx(int ntiles, int par, int k, int i) {
  return ((size_t)(par * ntiles + (i >> 6)) * 18 + (k >> 1)) * 128 + (i & 63) * 2 + (k & 1);
}

// Loads and stores of one pair through the global address space (so that the
// compiler emits global_load/global_store rather than flat accesses).
#define DDML_GLOBAL __attribute__((address_space(1)))
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void ld2(const float2* p, float2& a, float2& b) {
  const f32x4 v = *(const DDML_GLOBAL f32x4*)p;
  a = make_float2(v.x, v.y);
  b = make_float2(v.z, v.w);
}
__device__ __forceinline__ void ld2(const double2* p, double2& a, double2& b) {
  const DDML_GLOBAL f64x2* q = (const DDML_GLOBAL f64x2*)p;
  const f64x2 u = q[0], v = q[1];
  a = make_double2(u.x, u.y);
  b = make_double2(v.x, v.y);
}
__device__ __forceinline__ int ldg(const int* p) { return *(const DDML_GLOBAL int*)p; }
__device__ __forceinline__ float ldgf(const float* p) { return *(const DDML_GLOBAL float*)p; }
__device__ __forceinline__ void stgf(float* p, float v) { *(DDML_GLOBAL float*)p = v; }
__device__ __forceinline__ void stg2(double2* p, double2 v) {
  f64x2 u;
  u.x = v.x; u.y = v.y;
  *(DDML_GLOBAL f64x2*)p = u;
}
// Streaming variants (non-temporal hint): data read or written once per
// kernel, so that it does not push the reused neighbour spinors out of L2.
__device__ __forceinline__ void ld2nt(const float2* p, float2& a, float2& b) {
  const f32x4 v = __builtin_nontemporal_load((const DDML_GLOBAL f32x4*)p);
  a = make_float2(v.x, v.y);
  b = make_float2(v.z, v.w);
}
__device__ __forceinline__ void ld2nt(const double2* p, double2& a, double2& b) {
  const DDML_GLOBAL f64x2* q = (const DDML_GLOBAL f64x2*)p;
  const f64x2 u = __builtin_nontemporal_load(q), v = __builtin_nontemporal_load(q + 1);
  a = make_double2(u.x, u.y);
  b = make_double2(v.x, v.y);
}
__device__ __forceinline__ void st2nt(float2* p, float2 a, float2 b) {
  f32x4 v;
  v.x = a.x; v.y = a.y; v.z = b.x; v.w = b.y;
  __builtin_nontemporal_store(v, (DDML_GLOBAL f32x4*)p);
}
__device__ __forceinline__ void st2nt(double2* p, double2 a, double2 b) {
  DDML_GLOBAL f64x2* q = (DDML_GLOBAL f64x2*)p;
  f64x2 u, v;
  u.x = a.x; u.y = a.y; v.x = b.x; v.y = b.y;
  __builtin_nontemporal_store(u, q);
  __builtin_nontemporal_store(v, q + 1);
}
__device__ __forceinline__ void st2(float2* p, float2 a, float2 b) {
  f32x4 v;
  v.x = a.x; v.y = a.y; v.z = b.x; v.w = b.y;
  *(DDML_GLOBAL f32x4*)p = v;
}
__device__ __forceinline__ void st2(double2* p, double2 a, double2 b) {
  DDML_GLOBAL f64x2* q = (DDML_GLOBAL f64x2*)p;
  f64x2 u, v;
  u.x = a.x; u.y = a.y; v.x = b.x; v.y = b.y;
  q[0] = u;
  q[1] = v;
}

// 16-bit pairs (links and clover data): two complex numbers as 4 x int16 (8
// bytes per lane).  ld2q
// returns the raw integers as floats; the caller applies the scale.
typedef short s16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void ld2q(const h16c* p, float2& a, float2& b) {
  const s16x4 v = *(const DDML_GLOBAL s16x4*)p;
  a = make_float2((float)v.x, (float)v.y);
  b = make_float2((float)v.z, (float)v.w);
}
__device__ __forceinline__ void ld2q_nt(const h16c* p, float2& a, float2& b) {
  const s16x4 v = __builtin_nontemporal_load((const DDML_GLOBAL s16x4*)p);
  a = make_float2((float)v.x, (float)v.y);
  b = make_float2((float)v.z, (float)v.w);
}
__device__ __forceinline__ short q16(float v) { return (short)__float2int_rn(fminf(fmaxf(v, -kQ), kQ)); }
// 16-bit spinor fields are quad-packed: per (column, tile) three blocks of
// 256 complex numbers, block k holding components 4k .. 4k+3 of the tile's 64
// sites, 16 bytes per lane (half the load instructions of the pair layout).
__host__ __device__ __forceinline__ size_t qidx(int ntiles, int col, int i) {
  return (size_t)(col * ntiles + (i >> 6)) * 768 + (i & 63) * 4;
}
typedef short s16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ void ld4q(const h16c* p, float2 r[4], bool nt) {
  const s16x8 w = nt ? __builtin_nontemporal_load((const DDML_GLOBAL s16x8*)p) : *(const DDML_GLOBAL s16x8*)p;
#pragma unroll
  for (int j = 0; j < 4; ++j) r[j] = make_float2((float)w[2 * j], (float)w[2 * j + 1]);
}
// One site-column (12 complex, quad k at base + 256 k, base = field + qidx)
// in 16-bit storage.
// a product that is rounded on its own (never fused into a following add), so
// that a dequantised value is the same number wherever it is used
__device__ __forceinline__ float mul_rounded(float a, float b) {
#pragma clang fp contract(off)
  return a * b;
}
__device__ __forceinline__ void spinor_load_q(const h16c* base, float nrm, float2 v[12], bool nt) {
  const float sc = nrm / kQ;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float2 r[4];
    ld4q(base + 256 * k, r, nt);
#pragma unroll
    for (int j = 0; j < 4; ++j) v[4 * k + j] = make_float2(mul_rounded(r[j].x, sc), mul_rounded(r[j].y, sc));
  }
}
// Stores v with scale max|v| (NaN if any component is not finite) and returns
// in dq the values a later spinor_load_q reads back.
__device__ __forceinline__ void spinor_store_q(h16c* base, float* nrm, const float2 v[12], float2 dq[12], bool nt) {
  float m = 0.f, s = 0.f;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    m = fmaxf(m, fmaxf(fabsf(v[c].x), fabsf(v[c].y)));
    s += fabsf(v[c].x) + fabsf(v[c].y);
  }
  if (!isfinite(s)) m = __builtin_nanf("");
  const float inv = (m > 0.f && isfinite(m)) ? kQ / m : 0.f;
  const float sc = m / kQ;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s16x8 w;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float2 a = make_float2(v[4 * k + j].x * inv, v[4 * k + j].y * inv);
      w[2 * j] = q16(a.x);
      w[2 * j + 1] = q16(a.y);
      dq[4 * k + j] = make_float2((float)w[2 * j] * sc, (float)w[2 * j + 1] * sc);
    }
    if (nt) __builtin_nontemporal_store(w, (DDML_GLOBAL s16x8*)(base + 256 * k));
    else *(DDML_GLOBAL s16x8*)(base + 256 * k) = w;
  }
  stgf(nrm, m);
}

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

// Number of XCDs of the device and the tile orders of the stencil.  With
// every order but TILE_ORDER_LINEAR, workgroup b runs on XCD b % 8 and each XCD
// walks its own part of the box:
//   TILE_ORDER_BANDED  the XCD owns a band of every time slice and walks the
//                      slices in order;
//   TILE_ORDER_SUB2/4  the XCD owns an x1 range of the box, split by the x2
//                      position of the tiles into 2 or 4 sub-bands, and walks
//                      each sub-band slice by slice (walk table of the box);
//   TILE_ORDER_SUB4T   the sub-bands of SUB4 walked in blocks of 4 slices,
//                      the slices of a block innermost, so a tile's time
//                      neighbours are its neighbours in the walk;
//   TILE_ORDER_QUAD    the XCD owns half of the x1 rows and a quarter of the
//                      tiles of each (x2, x3) plane (fewer tiles on the
//                      region's border than an x1 range of every plane),
//                      cut along x1 into 4 sub-bands walked as in SUB4T.
// Either way the neighbours of a tile (same slice, adjacent slices) are read
// through the same L2 shortly after they were first fetched; the sub-bands
// shorten the distance to the next time slice so it stays in the L2.
constexpr int kXcd = 8;
enum { TILE_ORDER_LINEAR = 0, TILE_ORDER_BANDED = 1, TILE_ORDER_SUB2 = 2, TILE_ORDER_SUB4 = 3, TILE_ORDER_SUB4T = 4,
       TILE_ORDER_QUAD = 5, TILE_ORDER_NUM = 6 };
constexpr int kWalks = TILE_ORDER_NUM - TILE_ORDER_SUB2;   // orders with a walk table

// ---------------------------------------------------------- kernel argument
// Work item of the batched launches: one domain solve (or one operator
// application) with its own box, operator data and vectors.
template <typename T2> struct HopItem {
  BoxGeom g;
  const T2* U;        // links [2][ntiles][4][9][64]
  const T2* clov;     // clover data [2][ntiles][36][64] (A or A^{-1})
  const T2* in;       // input field on the opposite parity [nrhs][ntiles][12][64]
  const T2* aux;      // field on the output parity, may be null
  const T2* red_a;    // first operand of a fused dot product, may be null
  T2* out;            // output field on the output parity
  double2* partial;   // fused reduction partials [nred][nrhs][ntiles], may be null
  const int* active;  // per-rhs flag, may be null (all active)
  int par_out;
  int nrhs;
  int ntiles;
  double c1, c2;
  int tps;            // tiles per time slice (banded tile order), 0 = linear order
  const int* walk;    // tile walk of the sub-banded orders (all tiles, XCD-major), may be null
  int xoff[kXcd + 1]; // XCD x walks walk[xoff[x] .. xoff[x+1])
};

// Stencil epilogues (acc = H in on the output parity):
//   MODE_CINV_HOP  out = C acc                       (C = A^{-1}_pp)
//   MODE_SCHUR     out = aux - c1 C acc              (c1 = kappa^2: the Schur operator)
//   MODE_M         out = c2 (C aux - c1 acc)         (C = A_pp, c1 = kappa: M = A - kappa H)
//   MODE_PREP      out = C (aux + c1 acc)            (C = A^{-1}_pp: EO prepare/reconstruct)
//   MODE_RES       out = red_a - (C aux - c1 acc)    (residual b - M x)
enum { MODE_CINV_HOP = 0, MODE_SCHUR = 1, MODE_M = 2, MODE_PREP = 3, MODE_RES = 4 };
// Fused reductions (FP64 partial sums per 64-site tile and column, written to
// partial slot k at [k][nrhs][ntiles]):
//   RED_DOT  slot 0: (h, out), h the shadow vector below
//   RED_TS   slot 0: (out, aux), slot 1: |out|^2, slot 2: (h, out)
//   RED_NORM slot 0: |out|^2
enum { RED_NONE = 0, RED_DOT = 1, RED_TS = 2, RED_NORM = 3 };

// Shadow residual h of the inner BiCGstab: a fixed vector whose entries are
// (+-1 +- i), the signs taken from an integer hash of (column, site) (the
// "lowbias32" finaliser of C. Wellons' hash-prospector), so it is computed
// where a dot product needs it and never stored or read.  BiCGstab admits any
// fixed shadow vector not orthogonal to the residual; a dense random one also
// avoids the poor choice h = r0 for a point source (a vector with a single
// non-zero site).  Bits 2c and 2c + 1 are the signs of Re and Im of component c.
__host__ __device__ __forceinline__ unsigned shadow_bits(int col, int site) {
  unsigned x = (unsigned)site * 0x9E3779B1u ^ ((unsigned)col * 0x85EBCA77u + 0x27D4EB2Fu);
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
// acc += conj(h_c) v_c for the components c0 .. c0 + N - 1 of one site, v
// holding those N components (exact sign flips)
template <typename T2, int N>
__device__ __forceinline__ void shadow_dot_part(unsigned bits, int c0, const T2 v[N], double2& acc) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int c = c0 + k;
    const double vr = v[k].x, vi = v[k].y;
    const double sr = ((bits >> (2 * c)) & 1u) ? -1.0 : 1.0, si = ((bits >> (2 * c + 1)) & 1u) ? -1.0 : 1.0;
    acc.x += sr * vr + si * vi;
    acc.y += sr * vi - si * vr;
  }
}
template <typename T2>
__device__ __forceinline__ void shadow_dot(unsigned bits, const T2 v[12], double2& acc) {
  shadow_dot_part<T2, 12>(bits, 0, v, acc);
}

// Krylov vector slots of one inner solve (even parity unless noted); slot 1
// is unused by BiCGstab (its shadow vector is hashed, see shadow_bits)
enum { F_R = 0, F_UNUSED = 1, F_P = 2, F_V = 3, F_S = 4, F_T = 5, F_X = 6, F_TMP = 7 /* odd */, F_NUM = 8 };
// Partial-sum slots of BiCGstab ([kBiPartials][nrhs][ntiles] per solve)
constexpr int kBiPartials = 4;
// Smallest relative reduction asked of a 16-bit inner solve: below it the
// recursive residual drifts away from the true one by the storage rounding
// (at 3e-4 three FP64 corrections reach 1e-10; at 1e-3 four were needed, at
// 1e-4 the inner solves take more iterations than they save).
constexpr double kInnerFloor16 = 3e-4;
// GCR(m) (solver 2) keeps m search directions p_j and their images q_j = M p_j
// in the field slots after the BiCGstab ones (F_R, F_X and F_TMP are shared).
constexpr int kGcrMax = 8;
constexpr int F_GP0 = F_NUM, F_GQ0 = F_NUM + kGcrMax, F_ALL = F_NUM + 2 * kGcrMax;

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

// Device-side outer loop of a batched solve (defect correction in FP64 run
// by kernels captured with the inner iterations).  A slot goes
//   PH_NEW (x = 0) -> residual -> decide -> PH_PREP -> inner init -> PH_INNER
//   -> (every column's inner solve stopped) PH_EXPORT -> x += e -> residual
//   -> decide -> PH_PREP again, or PH_DONE when every column has converged,
//   failed or used its corrections.
enum { PH_IDLE = 0, PH_NEW = 1, PH_INNER = 2, PH_EXPORT = 3, PH_PREP = 4, PH_DONE = 5 };
// per slot: phase, number of inner cycles started
struct SlotState {
  int phase;
  int cycles;
};
// per column of a slot
struct OuterState {
  double bn2;       // |b'|^2
  double rel;       // last true relative residual |b' - M x| / |b'|
  int inner_total;  // inner iterations over all cycles
  int done;         // 1: converged, failed or out of corrections
  int status;       // 0, or DDML_ENUMERIC
  int pad;
};
// Outer-step column flags ([3][nrhs] per slot): export, residual, prepare.
enum { OF_EXPORT = 0, OF_RESID = 1, OF_PREP = 2 };

// One inner-solver slot as seen by the batched kernels.
template <typename T2> struct SlotDesc {
  BoxGeom g;
  int nrhs;
  int ntiles;
  int tps;              // tiles per time slice if a slice is a whole number of tiles, else 0
  double kappa;
  const T2* U;          // links in the inner precision
  const T2* Ainv;       // A^{-1} in the inner precision
  T2* f[F_ALL];         // Krylov vectors [nrhs][ntiles][12][64] (GCR slots null for BiCGstab)
  double2* partial;     // [2][nrhs][ntiles] (GCR: [max(2, m)][nrhs][ntiles])
  int* active;          // [nrhs]
  BiState* st;          // [nrhs]
  const double2* src64; // FP64 even-parity right-hand side [nrhs][ntiles][12][64]
  double2* gcoef;       // GCR: [nrhs][2 * kGcrMax]: beta_j, then |q_j|^2 (x)
  const int* walk;      // tile walk of the sub-banded orders, as in HopItem
  int xoff[kXcd + 1];
  // 16-bit storage only (T2 = h16c): scales of f[k] ([nrhs][ntiles * 64]),
  // of the clover data ([2][ntiles * 64]), and the FP32 solution vector
  float* nrm[F_ALL];
  const float* Ainv_nrm;
  float2* x32;
  // device-side outer loop (null phase: the host drives it)
  const T2* A;             // clover A, for the FP64 residual views (MODE_RES)
  SlotState* sst;
  OuterState* ost;         // [nrhs]
  int* oflag;              // [3][nrhs]
  double2* o64[8];         // FP64 outer fields: b'_e, b'_o, x_e, x_o, r_e, r_o, t_e, t_o
  const double2* Ainv64;   // FP64 A^{-1} (A_oo^{-1} r_o of the preparation)
  double2* partial64;      // [2][nrhs][ntiles]: |r_e|^2, |r_o|^2 partial sums
  double tol, inner_tol;
  int max_outer, max_inner, prec, solver;
};
enum { O_BE = 0, O_BO = 1, O_XE = 2, O_XO = 3, O_RE = 4, O_RO = 5, O_TE = 6, O_TO = 7 };

// Whether the inner (re)initialisation of kind `kind` (0: fresh start, 1:
// reliable update keeping the Krylov space) runs on slot d.  A host-driven
// slot runs the one the host launched; a device-driven slot runs only in
// PH_PREP, with the reliable update from its second cycle on when asked for.
template <typename T2>
__device__ __forceinline__ bool init_here(const SlotDesc<T2>& d, int kind) {
  if (!d.sst) return true;
  const SlotState st = *d.sst;
  if (st.phase != PH_PREP) return false;
  const int relup = d.solver == 1 && st.cycles > 1;
  return relup == kind;
}

}  // namespace ddml
