// Even-odd Wilson-clover stencil kernels on domain-local boxes (gfx950).
//
// The hopping term H = D_hop of Section 6 (from the covariant differences of
// Appendix A):
//   (H psi)(x) = sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ].
// In the chiral basis g_mu = [[0, e_mu], [e_mu^dag, 0]] (e_0 = -1, e_k = -i s_k),
// so (1 -+ g_mu) psi = [h ; -+ e_mu^dag h] with the half spinor h = psi_u -+ e_mu psi_l.
// Only h (2 spins x 3 colours) is multiplied by the link, then the lower two
// spins are rebuilt; that halves the SU(3) work.
//
// One thread owns one site of the output parity and R right-hand sides; a
// workgroup is one 64-site tile (one wavefront per group of R columns), so the
// waves of one workgroup read the same links and clover data and hit in L1/L2
// instead of HBM.  Domain restriction comes from zeroed face links, so the
// inner loop has no masking branch.  Tiles are visited either linearly or in
// XCD bands (see ddml_common.hpp) so that neighbour tiles share an L2.
#include <type_traits>

// No implicit contraction of a multiply and an add into one FMA in this file:
// every FMA of the stencil is written out (cmac, cmas, fmadd), so each site is
// computed by the same operations whatever launch variant or tile order the
// compiler sees around it, and all variants agree bit for bit by construction.
#pragma clang fp contract(off)

#include "ddml_common.hpp"
#include "launchers.hpp"

namespace ddml {

// ---------------------------------------------------------------- spin maths
template <typename T2>
__device__ __forceinline__ void project(int mu, bool fwd, const T2 psi[12], T2 h[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T2 p0 = psi[c], p1 = psi[3 + c], p2 = psi[6 + c], p3 = psi[9 + c];
    T2 h0, h1;
    switch (mu) {
      case 0:
        h0 = fwd ? cadd(p0, p2) : csub(p0, p2);
        h1 = fwd ? cadd(p1, p3) : csub(p1, p3);
        break;
      case 1:
        h0 = fwd ? cadd(p0, ci(p3)) : csub(p0, ci(p3));
        h1 = fwd ? cadd(p1, ci(p2)) : csub(p1, ci(p2));
        break;
      case 2:
        h0 = fwd ? cadd(p0, p3) : csub(p0, p3);
        h1 = fwd ? csub(p1, p2) : cadd(p1, p2);
        break;
      default:
        h0 = fwd ? cadd(p0, ci(p2)) : csub(p0, ci(p2));
        h1 = fwd ? csub(p1, ci(p3)) : cadd(p1, ci(p3));
        break;
    }
    h[c] = h0;
    h[3 + c] = h1;
  }
}

template <typename T2>
__device__ __forceinline__ void reconstruct(int mu, bool fwd, const T2 g[6], T2 acc[12]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T2 g0 = g[c], g1 = g[3 + c];
    acc[c] = cadd(acc[c], g0);
    acc[3 + c] = cadd(acc[3 + c], g1);
    switch (mu) {
      case 0:
        acc[6 + c] = fwd ? cadd(acc[6 + c], g0) : csub(acc[6 + c], g0);
        acc[9 + c] = fwd ? cadd(acc[9 + c], g1) : csub(acc[9 + c], g1);
        break;
      case 1:
        acc[6 + c] = fwd ? cadd(acc[6 + c], cmi(g1)) : cadd(acc[6 + c], ci(g1));
        acc[9 + c] = fwd ? cadd(acc[9 + c], cmi(g0)) : cadd(acc[9 + c], ci(g0));
        break;
      case 2:
        acc[6 + c] = fwd ? csub(acc[6 + c], g1) : cadd(acc[6 + c], g1);
        acc[9 + c] = fwd ? cadd(acc[9 + c], g0) : csub(acc[9 + c], g0);
        break;
      default:
        acc[6 + c] = fwd ? cadd(acc[6 + c], cmi(g0)) : cadd(acc[6 + c], ci(g0));
        acc[9 + c] = fwd ? cadd(acc[9 + c], ci(g1)) : cadd(acc[9 + c], cmi(g1));
        break;
    }
  }
}

// reconstruct with a scale s folded in (acc += s times the rebuilt spinor):
// every add is a fused multiply-add by s, so a 16-bit input spinor's per-site
// scale is applied here once instead of to each of its loaded components
template <typename T2>
__device__ __forceinline__ void reconstruct_s(int mu, bool fwd, const T2 g[6], decltype(T2::x) s, T2 acc[12]) {
  const decltype(T2::x) m = -s;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T2 g0 = g[c], g1 = g[3 + c];
    acc[c] = cmas(acc[c], g0, s);
    acc[3 + c] = cmas(acc[3 + c], g1, s);
    switch (mu) {
      case 0:
        acc[6 + c] = cmas(acc[6 + c], g0, fwd ? s : m);
        acc[9 + c] = cmas(acc[9 + c], g1, fwd ? s : m);
        break;
      case 1:
        acc[6 + c] = cmas(acc[6 + c], fwd ? cmi(g1) : ci(g1), s);
        acc[9 + c] = cmas(acc[9 + c], fwd ? cmi(g0) : ci(g0), s);
        break;
      case 2:
        acc[6 + c] = cmas(acc[6 + c], g1, fwd ? m : s);
        acc[9 + c] = cmas(acc[9 + c], g0, fwd ? s : m);
        break;
      default:
        acc[6 + c] = cmas(acc[6 + c], fwd ? cmi(g0) : ci(g0), s);
        acc[9 + c] = cmas(acc[9 + c], fwd ? ci(g1) : cmi(g1), s);
        break;
    }
  }
}

// g = U h (dag=false) or U^dag h (dag=true), per spin of the half spinor;
// every complex multiply-add is four fused multiply-adds
template <typename T2>
__device__ __forceinline__ void su3_mul(const T2 u[9], bool dag, const T2 h[6], T2 g[6]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T2 acc = mk<T2>(0, 0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        if (!dag) acc = cmac(acc, u[3 * a + b], h[3 * s + b]);
        else acc = cmacc(acc, u[3 * b + a], h[3 * s + b]);
      }
      g[3 * s + a] = acc;
    }
}

// g = W h per spin of the half spinor, W a link staged in LDS as 5 pairs of
// its 9 row-major entries (pair k at ul + 128 k): each row is read when it is
// needed, so at most a row and a half of W is live.  Every g is the same
// sequence of fused multiply-adds as su3_mul (with W = U^dag for a backward
// hop, conj(u) * h in cmacc is the product w * h in cmac).
template <typename T2>
__device__ __forceinline__ void su3_rows(const T2* ul, const T2 h[6], T2 g[6]);

// Loads of one pair from the LDS staging area of a tile (same pair stride as
// the global layout: pair k of lane l at base + 128 k, base = area + 2 l).
__device__ __forceinline__ void lds2(const float2* p, float2& a, float2& b) {
  const f32x4 v = *(const __attribute__((address_space(3))) f32x4*)p;
  a = make_float2(v.x, v.y);
  b = make_float2(v.z, v.w);
}
__device__ __forceinline__ void lds2(const double2* p, double2& a, double2& b) {
  const __attribute__((address_space(3))) f64x2* q = (const __attribute__((address_space(3))) f64x2*)p;
  const f64x2 u = q[0], v = q[1];
  a = make_double2(u.x, u.y);
  b = make_double2(v.x, v.y);
}
__device__ __forceinline__ void sts2(float2* p, float2 a, float2 b) {
  f32x4 v;
  v.x = a.x; v.y = a.y; v.z = b.x; v.w = b.y;
  *(__attribute__((address_space(3))) f32x4*)p = v;
}
__device__ __forceinline__ void sts2(double2* p, double2 a, double2 b) {
  __attribute__((address_space(3))) f64x2* q = (__attribute__((address_space(3))) f64x2*)p;
  f64x2 u, v;
  u.x = a.x; u.y = a.y; v.x = b.x; v.y = b.y;
  q[0] = u;
  q[1] = v;
}

template <typename T2>
__device__ __forceinline__ void su3_row(const T2 w0, const T2 w1, const T2 w2, const T2 h[6], int a, T2 g[6]) {
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    T2 acc = mk<T2>(0, 0);
    acc = cmac(acc, w0, h[3 * s]);
    acc = cmac(acc, w1, h[3 * s + 1]);
    acc = cmac(acc, w2, h[3 * s + 2]);
    g[3 * s + a] = acc;
  }
}
template <typename T2>
__device__ __forceinline__ void su3_rows(const T2* ul, const T2 h[6], T2 g[6]) {
  T2 w0, w1, w2, w3, w4, w5, w6, w7, w8, wp;
  lds2(ul, w0, w1);
  lds2(ul + 128, w2, w3);
  su3_row(w0, w1, w2, h, 0, g);
  lds2(ul + 256, w4, w5);
  su3_row(w3, w4, w5, h, 1, g);
  lds2(ul + 384, w6, w7);
  lds2(ul + 512, w8, wp);
  su3_row(w6, w7, w8, h, 2, g);
}

// 18 slots of one Hermitian 6x6 block (9 pairs, pair k at base + 128 k)
template <typename T2>
__device__ __forceinline__ void herm6_load(const T2* __restrict__ base, T2 m[18]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) ld2nt(base + 128 * k, m[2 * k], m[2 * k + 1]);
}
template <typename T2>
__device__ __forceinline__ void herm6_load_lds(const T2* base, T2 m[18]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) lds2(base + 128 * k, m[2 * k], m[2 * k + 1]);
}
// the 12 components of a spinor (6 pairs) starting at base
template <typename T2>
__device__ __forceinline__ void spinor_load(const T2* __restrict__ base, T2 v[12]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) ld2(base + 128 * k, v[2 * k], v[2 * k + 1]);
}
template <typename T2>
__device__ __forceinline__ void spinor_store(T2* __restrict__ base, const T2 v[12]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) st2(base + 128 * k, v[2 * k], v[2 * k + 1]);
}
// streaming spinor access: fields read or written once per stencil launch
template <typename T2>
__device__ __forceinline__ void spinor_load_nt(const T2* __restrict__ base, T2 v[12]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) ld2nt(base + 128 * k, v[2 * k], v[2 * k + 1]);
}
template <typename T2>
__device__ __forceinline__ void spinor_store_nt(T2* __restrict__ base, const T2 v[12]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) st2nt(base + 128 * k, v[2 * k], v[2 * k + 1]);
}
template <typename T2>
__device__ __forceinline__ void herm6_apply(const T2 m[18], const T2 x[6], T2 y[6]) {
  using T = decltype(T2::x);
  T d[6] = {m[0].x, m[0].y, m[1].x, m[1].y, m[2].x, m[2].y};
#pragma unroll
  for (int i = 0; i < 6; ++i) y[i] = cscale(x[i], d[i]);
  int k = 3;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i + 1; j < 6; ++j) {
      const T2 h = m[k++];
      y[i] = cmac(y[i], h, x[j]);
      y[j] = cmacc(y[j], h, x[i]);
    }
}

// y = M x for one Hermitian 6x6 block staged in LDS (18 slots in 9 pairs:
// the diagonal packed in slots 0..2, then the 15 upper entries, row by row),
// reading each pair when it is needed: the same operations in the same order
// as herm6_apply on the whole block.
template <typename T2>
__device__ __forceinline__ void herm6_apply_lds(const T2* base, const T2 x[6], T2 y[6]) {
  T2 m0, m1;
  lds2(base, m0, m1);
  y[0] = cscale(x[0], m0.x);
  y[1] = cscale(x[1], m0.y);
  y[2] = cscale(x[2], m1.x);
  y[3] = cscale(x[3], m1.y);
  lds2(base + 128, m0, m1);
  y[4] = cscale(x[4], m0.x);
  y[5] = cscale(x[5], m0.y);
  // slot k (k >= 3) holds entry (i, j) of the upper triangle, row by row
  T2 h = m1;   // slot 3
  int k = 3;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i + 1; j < 6; ++j) {
      if (k > 3) {
        if (k & 1) {
          h = m1;
        } else {
          lds2(base + 128 * (k >> 1), m0, m1);
          h = m0;
        }
      }
      y[i] = cmac(y[i], h, x[j]);
      y[j] = cmacc(y[j], h, x[i]);
      ++k;
    }
}

// ------------------------------------------------------------ the stencil core
// LDS staging of the operator data of one tile (ST = true): the links of the
// 8 hops of every site ([hop = 2 mu + backward][5 pairs]) and the 18 clover
// pairs, as [58 pairs][64 lanes][2] complex (the pair stride of the global
// layout).  The workgroup reads them from HBM/L2 once instead of once per
// wavefront (12 wavefronts share a tile at R = 1).  FP64 links are read whole;
// the FP32 and 16-bit copies hold the first two rows of each link (3 pairs)
// and the third is rebuilt here, as conj(row 0 x row 1) for an SU(3) matrix,
// times -1 for the time links of the last slice of a box that spans the
// whole antiperiodic time extent (the sign folded into the stored rows
// cancels in the cross product); a zeroed face link rebuilds to zero.  One
// wavefront stages all of a link, so one barrier closes the staging.  A
// backward hop's link is staged as U^dag (conjugated transpose), so every hop
// multiplies by the rows of its staged matrix (su3_rows).
constexpr int kStageLinkPairs = 8 * 5;
constexpr int kStagePairs = kStageLinkPairs + 18;

template <typename E>
constexpr bool kIs16 = std::is_same<E, h16c>::value;
template <typename E>
constexpr bool kTwoRow = !std::is_same<E, double2>::value;

// one pair of a staged field (16-bit: dequantised with scale sc)
template <typename E, typename C>
__device__ __forceinline__ void stage_load(const E* src, float sc, C& a, C& b) {
  if constexpr (kIs16<E>) {
    ld2q_nt(src, a, b);
    a = make_float2(a.x * sc, a.y * sc);
    b = make_float2(b.x * sc, b.y * sc);
  } else {
    ld2nt(src, a, b);
  }
}

// E: element type of the fields (float2, double2 or 16-bit h16c); C: compute type.
template <typename E, typename C = typename CompOf<E>::type>
__device__ __forceinline__ void stage_tile(const BoxGeom& g, const E* __restrict__ U, const E* __restrict__ clov,
                                           const float* __restrict__ clov_n, int p, int tile, C* sm) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6, W = blockDim.x >> 6;
  const int i = tile * kTile + lane;
  const bool valid = i < g.Vh;
  const int nt = g.ntiles;
  const int q = 1 - p;
  int y[4] = {0, 0, 0, 0};
  if (valid) eo_coords(g, p, i, y);
  const C z = mk<C>(0, 0);
  // links: hop h = 2 mu + backward, forward from this site, backward from y - mu
  for (int h = w; h < 8; h += W) {
    const int mu = h >> 1;
    const bool bwd = h & 1;
    int par = p, site = i;
    if (valid && bwd) {
      int zz[4] = {y[0], y[1], y[2], y[3]};
      zz[mu] = (y[mu] == 0) ? g.L[mu] - 1 : y[mu] - 1;
      par = q;
      site = eo_index(g, zz);
    }
    C e[10];
    if constexpr (kTwoRow<E>) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        e[2 * k] = z;
        e[2 * k + 1] = z;
        if (valid) stage_load<E, C>(U + lidx2(nt, par, mu, 2 * k, site), 1.0f / kQ, e[2 * k], e[2 * k + 1]);
      }
      // the time link of the box's last slice, if it carries the antiperiodic sign
      const bool flip = g.twrap && mu == 0 && valid && (bwd ? y[0] == 0 : y[0] == g.L[0] - 1);
#pragma unroll
      for (int c3 = 0; c3 < 3; ++c3) {
        const int a = (c3 + 1) % 3, b = (c3 + 2) % 3;
        C v = csub(cmul(e[a], e[3 + b]), cmul(e[b], e[3 + a]));
        e[6 + c3] = flip ? mk<C>(-v.x, v.y) : mk<C>(v.x, -v.y);
      }
      e[9] = z;
    } else {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        e[2 * k] = z;
        e[2 * k + 1] = z;
        if (valid) ld2nt(U + lidx(nt, par, mu, 2 * k, site), e[2 * k], e[2 * k + 1]);
      }
    }
    if (bwd) {   // the hop multiplies by U^dag: stage it as such (rows of U^dag = conj columns of U)
      C t[9];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) t[3 * a + b] = mk<C>(e[3 * b + a].x, -e[3 * b + a].y);
#pragma unroll
      for (int k = 0; k < 9; ++k) e[k] = t[k];
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) sts2(sm + (h * 5 + k) * 128 + lane * 2, e[2 * k], e[2 * k + 1]);
  }
  // clover data of the output parity (padding sites hold zeros)
  for (int j = w; j < 18; j += W) {
    C a = z, b = z;
    float sc = 1.0f / kQ;
    if constexpr (kIs16<E>) sc = ldgf(clov_n + (size_t)p * nt * kTile + i) / kQ;
    stage_load<E, C>(clov + cidx(nt, p, 2 * j, i), sc, a, b);
    sts2(sm + (kStageLinkPairs + j) * 128 + lane * 2, a, b);
  }
  __syncthreads();
}

// on: bit r set if column r0 + r is active (read once per tile by the caller,
// so the direction loop has no load-dependent branch and its loads can overlap)
template <typename E, int R, bool ST, typename C = typename CompOf<E>::type>
__device__ __forceinline__ void hop_sum(const BoxGeom& g, int p, int i, const E* __restrict__ U, const C* sm,
                                        const E* __restrict__ in, const float* __restrict__ in_n, int r0, int nr,
                                        unsigned on, C acc[R][12]) {
  int y[4];
  eo_coords(g, p, i, y);
  const int q = 1 - p;
  const int nt = g.ntiles;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[r][c] = mk<C>(0, 0);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      const bool fwd = dir == 0;
      int z[4] = {y[0], y[1], y[2], y[3]};
      if (fwd) z[mu] = (y[mu] + 1 == g.L[mu]) ? 0 : y[mu] + 1;
      else z[mu] = (y[mu] == 0) ? g.L[mu] - 1 : y[mu] - 1;
      const int n = eo_index(g, z);
      C u[10];
      const C* ul = nullptr;
      if constexpr (ST) {
        ul = sm + (2 * mu + dir) * 5 * 128 + (i & 63) * 2;
      } else {
        static_assert(!kTwoRow<E>, "two-row links (FP32, 16-bit) are read through the LDS staging only");
        const E* __restrict__ ug = fwd ? U + lidx(nt, p, mu, 0, i) : U + lidx(nt, q, mu, 0, n);
#pragma unroll
        for (int k = 0; k < 5; ++k) ld2nt(ug + 128 * k, u[2 * k], u[2 * k + 1]);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r < nr && ((on >> r) & 1u)) {
          C psi[12], h[6], gg[6];
          if constexpr (kIs16<E>) {
            // the stored integers are projected and multiplied as they are
            // (the projection is exact on them) and the spinor's scale enters
            // once, in the fused rebuild
            const h16c* b = in + qidx(nt, r0 + r, n);
            const float sc = ldgf(in_n + (size_t)(r0 + r) * nt * kTile + n) * (1.0f / kQ);
            s16x8 w[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) w[k] = *(const DDML_GLOBAL s16x8*)(b + 256 * k);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
              for (int j = 0; j < 4; ++j) psi[4 * k + j] = make_float2((float)w[k][2 * j], (float)w[k][2 * j + 1]);
            project(mu, fwd, psi, h);
            su3_rows(ul, h, gg);
            reconstruct_s(mu, fwd, gg, sc, acc[r]);
          } else {
            spinor_load(in + fidx(nt, r0 + r, 0, n), psi);
            project(mu, fwd, psi, h);
            if constexpr (ST) su3_rows(ul, h, gg);
            else su3_mul(u, !fwd, h, gg);
            reconstruct(mu, fwd, gg, acc[r]);
          }
        }
      }
    }
  }
}

__device__ __forceinline__ double2 wave_sum(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

// Epilogue on one column.  acc = (H in)(x); cl points at slot 0 of this site.
template <typename T2, int MODE, bool ST>
__device__ __forceinline__ void epilogue_block(const T2* cl, int b, const T2 acc[6], const T2 aux[6], const T2 ra[6],
                                               double c1, double c2, T2 out[6]) {
  using T = decltype(T2::x);
  const T k1 = (T)c1, k2 = (T)c2;
  T2 m[18];
  const T2* cb = cl + 128 * 9 * b;
  if (!ST) herm6_load(cb, m);
  auto apply = [&](const T2 x[6], T2 y[6]) {
    if (ST) herm6_apply_lds(cb, x, y);
    else herm6_apply(m, x, y);
  };
  if (MODE == MODE_CINV_HOP) {
    apply(acc, out);
  } else if (MODE == MODE_SCHUR) {
    T2 y[6];
    apply(acc, y);
#pragma unroll
    for (int c = 0; c < 6; ++c) out[c] = cmas(aux[c], y[c], -k1);
  } else if (MODE == MODE_M || MODE == MODE_RES) {
    T2 y[6];
    apply(aux, y);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      T2 v = cmas(y[c], acc[c], -k1);
      out[c] = (MODE == MODE_M) ? cscale(v, k2) : csub(ra[c], v);
    }
  } else {  // MODE_PREP: out = C (aux + c1 acc)
    T2 v[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = cmas(aux[c], acc[c], k1);
    apply(v, out);
  }
}

// The epilogue on the two chiral blocks of one column (acc = (H in)(x); cl
// points at slot 0 of this site's clover data).
template <typename T2, int MODE, bool ST>
__device__ __forceinline__ void epilogue(const T2* cl, const T2 acc[12], const T2 aux[12],
                                         const T2 ra[12], double c1, double c2, T2 out[12]) {
#pragma unroll
  for (int b = 0; b < 2; ++b)
    epilogue_block<T2, MODE, ST>(cl, b, acc + 6 * b, aux + 6 * b, ra + 6 * b, c1, c2, out + 6 * b);
}

// The fused reductions of one output column over its components [c0, c0 + N)
// (o the output, av the aux field), each accumulated in component order.
template <int RED, int N, typename C>
__device__ __forceinline__ void fused_reductions(unsigned hb, int c0, const C o[N], const C av[N], double2& s0,
                                                 double2& s1, double2& s2) {
  if (RED == RED_DOT) {
    shadow_dot_part<C, N>(hb, c0, o, s0);
  } else if (RED == RED_TS) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const double ox = o[c].x, oy = o[c].y, ax = av[c].x, ay = av[c].y;
      s0.x = fmadd(ox, ax, fmadd(oy, ay, s0.x));
      s0.y = fmadd(ox, ay, fmadd(-oy, ax, s0.y));
      s1.x = fmadd(ox, ox, fmadd(oy, oy, s1.x));
    }
    shadow_dot_part<C, N>(hb, c0, o, s2);
  } else if (RED == RED_NORM) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const double ox = o[c].x, oy = o[c].y;
      s0.x = fmadd(ox, ox, fmadd(oy, oy, s0.x));
    }
  }
}

// Field arguments of one tile launch: element pointers and, for 16-bit
// fields, their per-(site, column) scales.
template <typename E> struct TileArgs {
  const E* U;
  const E* clov;
  const float* clov_n;
  const E* in;
  const float* in_n;
  const E* aux;
  const float* aux_n;
  const E* red_a;
  const float* red_n;
  E* out;
  float* out_n;
};

// One tile on the output parity p.  ST: the tile's links and clover data are
// staged in LDS at sm (stage_tile) and taken from there.  16-bit outputs are
// quantised before the fused reductions, so the dot products are those of the
// stored vectors.
template <typename E, int R, int MODE, int RED, bool ST = false, typename C = typename CompOf<E>::type>
__device__ __forceinline__ void hop_tile(const BoxGeom g, const TileArgs<E>& a, double2* __restrict__ partial,
                                         const int* __restrict__ act, int p, int nrhs, double c1, double c2, int tile,
                                         int wave0 = 0, const C* sm = nullptr) {
  const int lane = threadIdx.x & 63;
  const int grp = wave0 + (threadIdx.x >> 6);
  const int r0 = grp * R;
  if (r0 >= nrhs) return;  // whole wave idle (uniform)
  const int nr = min(R, nrhs - r0);
  const int i = tile * kTile + lane;
  const bool valid = i < g.Vh;
  const int nt = g.ntiles;
  unsigned on = 0;  // active columns of this wavefront
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (r < nr && (act == nullptr || ldg(act + r0 + r))) on |= 1u << r;
  if (on == 0) return;  // uniform across the wave
  C acc[R][12];
  if (valid) hop_sum<E, R, ST>(g, p, i, a.U, sm, a.in, a.in_n, r0, nr, on, acc);
  // keep the epilogue's loads after the hop sum: hoisted above it they would
  // stay live through the hop loop and cost occupancy
  __builtin_amdgcn_sched_barrier(0);
  const C* cl;
  if constexpr (ST) cl = sm + kStageLinkPairs * 128 + lane * 2;
  else cl = a.clov + cidx(nt, p, 0, i);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r >= nr) break;
    const int col = r0 + r;
    if (!((on >> r) & 1u)) continue;  // uniform across the wave
    double2 s0 = make_double2(0, 0), s1 = make_double2(0, 0), s2 = make_double2(0, 0);
    const size_t base = fidx(nt, col, 0, i);
    const size_t ns = (size_t)col * nt * kTile + i;  // scale index of 16-bit fields
    if (valid) {
      const unsigned hb = shadow_bits(col, i);
      if constexpr (kIs16<E>) {
        // one scale over the 12 output components, so the epilogue runs on all
        // of them before the store.  To stay within the register budget it
        // works in place: the aux components become the output, the store
        // returns the stored values in the same registers, and the (t, s)
        // sums read aux again (the first load leaves it in cache for that)
        C w[12], ra[12];
        const size_t qb = qidx(nt, col, i);
        if (MODE != MODE_CINV_HOP) spinor_load_q(a.aux + qb, ldgf(a.aux_n + ns), w, RED != RED_TS);
        if (MODE == MODE_RES) spinor_load_q(a.red_a + qb, ldgf(a.red_n + ns), ra, true);
        epilogue<C, MODE, ST>(cl, acc[r], w, ra, c1, c2, w);
        spinor_store_q(a.out + qb, a.out_n + ns, w, w, true);
        if constexpr (RED == RED_TS) {
          C av[12];
          spinor_load_q(a.aux + qb, ldgf(a.aux_n + ns), av, true);
          fused_reductions<RED, 12>(hb, 0, w, av, s0, s1, s2);
        } else {
          fused_reductions<RED, 12>(hb, 0, w, w, s0, s1, s2);
        }
      } else {
        // chiral block by block: aux in, 6x6 clover block, out, reductions
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          C av[6], ra[6], o[6];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            if (MODE != MODE_CINV_HOP) ld2nt(a.aux + base + 128 * (3 * b + k), av[2 * k], av[2 * k + 1]);
            if (MODE == MODE_RES) ld2nt(a.red_a + base + 128 * (3 * b + k), ra[2 * k], ra[2 * k + 1]);
          }
          epilogue_block<C, MODE, ST>(cl, b, acc[r] + 6 * b, av, ra, c1, c2, o);
#pragma unroll
          for (int k = 0; k < 3; ++k) st2nt(a.out + base + 128 * (3 * b + k), o[2 * k], o[2 * k + 1]);
          fused_reductions<RED, 6>(hb, 6 * b, o, av, s0, s1, s2);
        }
      }
    } else {
      // padding sites of the last tile stay zero
      C z[12], zq[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) z[c] = mk<C>(0, 0);
      if constexpr (kIs16<E>) spinor_store_q(a.out + qidx(nt, col, i), a.out_n + ns, z, zq, false);
      else spinor_store(a.out + base, z);
    }
    if (RED != RED_NONE) {
      s0 = wave_sum(s0);
      if (RED == RED_TS) {
        s1 = wave_sum(s1);
        s2 = wave_sum(s2);
      }
      if (lane == 0) {
        stg2(partial + (size_t)col * nt + tile, s0);
        if (RED == RED_TS) {
          stg2(partial + ((size_t)nrhs + col) * nt + tile, s1);
          stg2(partial + ((size_t)2 * nrhs + col) * nt + tile, s2);
        }
      }
    }
  }
}

// Banded tile order of one box for XCD x: the box is nslice slices of S
// tiles (S = tps, or the whole box if a slice is not a whole number of tiles);
// XCD x owns tiles [x S / 8, (x+1) S / 8) of every slice, slice after slice.
__device__ __forceinline__ void band_of(int ntiles, int tps, int x, int& S, int& lo, int& bs) {
  S = tps > 0 ? tps : ntiles;
  lo = (int)((long)x * S / kXcd);
  bs = (int)((long)(x + 1) * S / kXcd) - lo;
}
__device__ __forceinline__ int band_tile(int S, int lo, int bs, int local) {
  return (local / bs) * S + lo + local % bs;
}

// Single-item launch (operator application, outer FP64 steps).
template <typename T2, int R, int MODE, int RED>
__global__ void __launch_bounds__(64 * ((kMaxRhs + R - 1) / R)) k_hop_item(HopItem<T2> it, int order) {
  const TileArgs<T2> ta{it.U, it.clov, nullptr, it.in, nullptr, it.aux, nullptr, it.red_a, nullptr, it.out, nullptr};
  if (order != TILE_ORDER_LINEAR) {
    const int x = blockIdx.x % kXcd, j = blockIdx.x / kXcd, nb = gridDim.x / kXcd;
    int S = 0, lo = 0, bs = 1, total;
    if (order == TILE_ORDER_BANDED) {
      band_of(it.ntiles, it.tps, x, S, lo, bs);
      total = bs * (it.ntiles / S);
    } else {
      total = it.xoff[x + 1] - it.xoff[x];
    }
    for (int v = j; v < total; v += nb) {
      const int tile = order == TILE_ORDER_BANDED ? band_tile(S, lo, bs, v) : ldg(it.walk + it.xoff[x] + v);
      hop_tile<T2, R, MODE, RED>(it.g, ta, it.partial, it.active, it.par_out, it.nrhs, it.c1, it.c2, tile);
    }
  } else {
    for (int tile = blockIdx.x; tile < it.ntiles; tile += gridDim.x)
      hop_tile<T2, R, MODE, RED>(it.g, ta, it.partial, it.active, it.par_out, it.nrhs, it.c1, it.c2, tile);
  }
}

// Batched launch over solver slots.  Linear order: virtual tile vt of the
// batch maps to (slot, tile) through tile_start[nslots+1].  Other orders:
// XCD x walks xstart[x][*], the prefix over slots of its share of the tiles.
__device__ __forceinline__ int find_slot(const int* __restrict__ start, int n, int vt) {
  int lo = 0, hi = n;  // start[lo] <= vt < start[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (start[mid] <= vt) lo = mid; else hi = mid;
  }
  return lo;
}

// The columns of a tile are split into ng groups of W = blockDim.x / 64
// waves (W * R columns each); virtual item v is (tile v / ng, group v % ng),
// so the groups of one tile run back to back on the same XCD.  ST: the
// workgroup stages each tile's links and clover data in LDS first (the trip
// count of the tile loop is uniform over the workgroup, so every wavefront
// reaches both barriers).
// The FP32 and 16-bit stencil at R = 1 is held to 6 waves per SIMD (80
// VGPRs), so that two 12-wave workgroups (one tile each) share a CU: the odd
// half fits without spills, the even half spills 3-5 registers and still
// runs 4-6% faster than at one workgroup per CU.
template <typename T2, int R, int MODE>
constexpr int kHopWaves = (!std::is_same<T2, double2>::value && R == 1) ? 6 : 1;

template <typename T2, int R, int MODE, int RED, bool ST>
__global__ void __launch_bounds__(64 * ((kMaxRhs + R - 1) / R))
    __attribute__((amdgpu_waves_per_eu(kHopWaves<T2, R, MODE>))) k_hop_batch(const SlotDesc<T2>* __restrict__ slots, const int* __restrict__ tile_start,
                const int* __restrict__ xstart, int xstride, const int* __restrict__ nslots_p, int fin, int faux,
                int fout, int fred, int par_out, int order, int ng) {
  using C = typename CompOf<T2>::type;
  __shared__ C sm[ST ? kStagePairs * 128 : 1];
  const int ns = *nslots_p;
  const int W = blockDim.x >> 6;
  const bool banded = order != TILE_ORDER_LINEAR;
  const int x = blockIdx.x % kXcd;
  const int* P = banded ? xstart + (size_t)x * xstride : tile_start;
  const int first = banded ? blockIdx.x / kXcd : blockIdx.x;
  const int step = banded ? gridDim.x / kXcd : gridDim.x;
  const int total = P[ns] * ng;
  for (int v = first; v < total; v += step) {
    const int tv = v / ng, grp = v - tv * ng;
    const int s = find_slot(P, ns, tv);
    const SlotDesc<T2>& d = slots[s];
    int tile = tv - P[s];
    if (order == TILE_ORDER_BANDED) {
      int S, lo, bs;
      band_of(d.ntiles, d.tps, x, S, lo, bs);
      tile = band_tile(S, lo, bs, tile);
    } else if (order != TILE_ORDER_LINEAR) {
      tile = ldg(d.walk + d.xoff[x] + tile);
    }
    // a workgroup whose columns are all inactive skips the tile (uniform: every
    // thread reads the same flags), before the staging
    {
      const int c0 = grp * W * R, c1 = min(d.nrhs, c0 + W * R);
      bool any = false;
      for (int c = c0; c < c1; ++c) any = any || ldg(d.active + c);
      if (!any) continue;
    }
    const bool h16 = kIs16<T2>;
    const T2* clov = MODE == MODE_RES ? d.A : d.Ainv;   // M = A - kappa H needs A itself
    const TileArgs<T2> ta{d.U, clov, h16 ? d.Ainv_nrm : nullptr,
                          d.f[fin], h16 ? d.nrm[fin] : nullptr,
                          faux >= 0 ? d.f[faux] : nullptr, h16 && faux >= 0 ? d.nrm[faux] : nullptr,
                          fred >= 0 ? d.f[fred] : nullptr, h16 && fred >= 0 ? d.nrm[fred] : nullptr,
                          d.f[fout], h16 ? d.nrm[fout] : nullptr};
    if constexpr (ST) stage_tile<T2>(d.g, d.U, clov, ta.clov_n, par_out, tile, sm);
    // c1: kappa^2 in the Schur operator, kappa in the FP64 residual and preparation
    const double c1 = (MODE == MODE_PREP || MODE == MODE_RES) ? d.kappa : d.kappa * d.kappa;
    hop_tile<T2, R, MODE, RED, ST>(d.g, ta, d.partial, d.active, par_out, d.nrhs, c1, 0.0, tile, grp * W, sm);
    if constexpr (ST) __syncthreads();
  }
}

// Site-local clover application out = C in on parity p.
template <typename T2>
__global__ void k_clover_apply(BoxGeom g, const T2* __restrict__ clov, int p, const T2* __restrict__ in,
                               T2* __restrict__ out, int nrhs) {
  const size_t per = (size_t)g.ntiles * 64;
  const size_t n = per * nrhs;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % per);  // a thread per (site, column)
    const int col = (int)(t / per);
    const size_t base = fidx(g.ntiles, col, 0, i);
    const T2* cl = clov + cidx(g.ntiles, p, 0, i);
    T2 x[12], y[12];
    spinor_load(in + base, x);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      T2 m[18];
      herm6_load(cl + 128 * 9 * b, m);
      herm6_apply(m, x + 6 * b, y + 6 * b);
    }
    if (i >= g.Vh)
#pragma unroll
      for (int c = 0; c < 12; ++c) y[c] = mk<T2>(0, 0);
    spinor_store(out + base, y);
  }
}

// --------------------------------------------------------------- launchers
#define DDML_HOP_DISPATCH(T2, Rv, MODEv, REDv)                                                        \
  if (R == Rv && mode == MODEv && red == REDv) {                                                      \
    hipLaunchKernelGGL((k_hop_item<T2, Rv, MODEv, REDv>), dim3(grid), dim3(block), 0, st, it, order); \
    return hipGetLastError();                                                                         \
  }

template <typename T2>
static hipError_t hop_item_impl(const HopItem<T2>& it, int mode, int red, int R, int order, hipStream_t st) {
  const int block = 64 * ((it.nrhs + R - 1) / R);
  int grid = it.ntiles < 65535 ? it.ntiles : 65535;
  if (order < 0 || order >= TILE_ORDER_NUM || (order >= TILE_ORDER_SUB2 && it.walk == nullptr))
    return hipErrorInvalidValue;
  if (order != TILE_ORDER_LINEAR) grid = ((grid + kXcd - 1) / kXcd) * kXcd;
  DDML_HOP_DISPATCH(T2, 1, MODE_CINV_HOP, RED_NONE)
  DDML_HOP_DISPATCH(T2, 1, MODE_SCHUR, RED_NONE)
  DDML_HOP_DISPATCH(T2, 1, MODE_M, RED_NONE)
  DDML_HOP_DISPATCH(T2, 1, MODE_PREP, RED_NONE)
  DDML_HOP_DISPATCH(T2, 1, MODE_RES, RED_NORM)
  DDML_HOP_DISPATCH(T2, 2, MODE_CINV_HOP, RED_NONE)
  DDML_HOP_DISPATCH(T2, 2, MODE_SCHUR, RED_NONE)
  DDML_HOP_DISPATCH(T2, 3, MODE_CINV_HOP, RED_NONE)
  DDML_HOP_DISPATCH(T2, 3, MODE_SCHUR, RED_NONE)
  (void)block;
  return hipErrorInvalidValue;
}

hipError_t launch_hop_item(const HopItem<double2>& it, int mode, int red, int R, int order, hipStream_t st) {
  return hop_item_impl(it, mode, red, R, order, st);
}

#define DDML_HOPB_DISPATCH1(T2, Rv, MODEv, REDv, STv)                                                    \
  if (R == Rv && mode == MODEv && red == REDv) {                                                         \
    hipLaunchKernelGGL((k_hop_batch<T2, Rv, MODEv, REDv, STv>), dim3(grid), dim3(block), 0, st, slots,   \
                       tile_start, xstart, xstride, nslots_p, fin, faux, fout, fred, par_out, order, ng); \
    return hipGetLastError();                                                                            \
  }
#define DDML_HOPB_DISPATCH_R(T2, Rv, STv)                        \
  DDML_HOPB_DISPATCH1(T2, Rv, MODE_CINV_HOP, RED_NONE, STv)      \
  DDML_HOPB_DISPATCH1(T2, Rv, MODE_SCHUR, RED_DOT, STv)          \
  DDML_HOPB_DISPATCH1(T2, Rv, MODE_SCHUR, RED_TS, STv)           \
  if constexpr (!kIs16<T2>) {                                    \
    DDML_HOPB_DISPATCH1(T2, Rv, MODE_SCHUR, RED_NONE, STv)       \
  }                                                              \
  if constexpr (std::is_same<T2, double2>::value && Rv == 1) {   \
    DDML_HOPB_DISPATCH1(T2, Rv, MODE_PREP, RED_NONE, STv)        \
    DDML_HOPB_DISPATCH1(T2, Rv, MODE_RES, RED_NORM, STv)         \
  }
#define DDML_HOPB_DISPATCH_ST(T2, STv) \
  DDML_HOPB_DISPATCH_R(T2, 1, STv)     \
  DDML_HOPB_DISPATCH_R(T2, 2, STv)     \
  DDML_HOPB_DISPATCH_R(T2, 3, STv)

template <typename T2>
static hipError_t hop_batch_impl(const SlotDesc<T2>* slots, const int* tile_start, const int* xstart, int xstride,
                                 const int* nslots_p, int nrhs, int R, int mode, int red, int fin, int faux, int fout,
                                 int fred, int par_out, int grid, int order, int splits, int stage,
                                 hipStream_t st) {
  // nw waves cover the columns of a tile; they are split into ng blocks of W waves
  const int nw = (nrhs + R - 1) / R;
  if (splits < 1 || splits > nw) return hipErrorInvalidValue;
  const int W = (nw + splits - 1) / splits, ng = (nw + W - 1) / W;
  const int block = 64 * W;
  if (order < 0 || order >= TILE_ORDER_NUM || (order != TILE_ORDER_LINEAR && grid % kXcd)) return hipErrorInvalidValue;
  if (stage) {
    DDML_HOPB_DISPATCH_ST(T2, true)
  } else {
    if constexpr (!kTwoRow<T2>) {
      DDML_HOPB_DISPATCH_ST(T2, false)
    }
  }
  return hipErrorInvalidValue;  // unknown variant; FP32 and 16-bit fields need stage = 1
}

hipError_t launch_hop_batch(const SlotDesc<float2>* slots, const int* tile_start, const int* xstart, int xstride,
                            const int* nslots_p, int nrhs, int R, int mode, int red, int fin, int faux, int fout,
                            int fred, int par_out, int grid, int order, int splits, int stage, hipStream_t st) {
  return hop_batch_impl(slots, tile_start, xstart, xstride, nslots_p, nrhs, R, mode, red, fin, faux, fout, fred,
                        par_out, grid, order, splits, stage, st);
}
hipError_t launch_hop_batch(const SlotDesc<double2>* slots, const int* tile_start, const int* xstart, int xstride,
                            const int* nslots_p, int nrhs, int R, int mode, int red, int fin, int faux, int fout,
                            int fred, int par_out, int grid, int order, int splits, int stage, hipStream_t st) {
  return hop_batch_impl(slots, tile_start, xstart, xstride, nslots_p, nrhs, R, mode, red, fin, faux, fout, fred,
                        par_out, grid, order, splits, stage, st);
}
hipError_t launch_hop_batch(const SlotDesc<h16c>* slots, const int* tile_start, const int* xstart, int xstride,
                            const int* nslots_p, int nrhs, int R, int mode, int red, int fin, int faux, int fout,
                            int fred, int par_out, int grid, int order, int splits, int stage, hipStream_t st) {
  return hop_batch_impl(slots, tile_start, xstart, xstride, nslots_p, nrhs, R, mode, red, fin, faux, fout, fred,
                        par_out, grid, order, splits, stage, st);
}

template <typename T2>
static hipError_t clover_apply_impl(const BoxGeom& g, const T2* clov, int p, const T2* in, T2* out, int nrhs,
                                    hipStream_t st) {
  size_t n = (size_t)g.ntiles * 64 * nrhs;
  int grid = (int)((n + 255) / 256);
  if (grid > 65535) grid = 65535;
  hipLaunchKernelGGL((k_clover_apply<T2>), dim3(grid), dim3(256), 0, st, g, clov, p, in, out, nrhs);
  return hipGetLastError();
}
hipError_t launch_clover_apply(const BoxGeom& g, const double2* clov, int p, const double2* in, double2* out,
                               int nrhs, hipStream_t st) {
  return clover_apply_impl(g, clov, p, in, out, nrhs, st);
}

}  // namespace ddml
