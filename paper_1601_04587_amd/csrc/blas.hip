// Krylov vector kernels and FP64 reductions for the batched BiCGstab.
//
// BiCGstab (van der Vorst 1992) on the even-odd Schur operator, one
// independent recursion per right-hand side, with a hashed shadow vector h
// (shadow_bits) in place of the stored r0.  One iteration:
//   v = M p, alpha = rho / (h, v);  s = r - alpha v;  t = M s,
//   omega = (t, s) / (t, t);  x += alpha p + omega s;  r = s - omega t;
//   p = r + beta (p - omega v),  beta = (rho'/rho)(alpha/omega),
// where rho' = (h, r) of the new residual equals (h, s) - omega (h, t): both
// dot products come from the kernels that write s and t, so beta is known
// before r is formed and the direction update shares the x/r pass (VEC_XRP).
// Reliable updates: when the FP64 defect-correction loop replaces the
// recursive residual by the true one r', the Krylov space is kept and only p
// and rho are rescaled, p = r' + (rho'/rho)(p - r_old) (VEC_RELUP, FIN_RELUP,
// VEC_PFIX); a column whose recursion broke down starts afresh instead.
// Every kernel walks a slot table
// (one entry per domain solve in flight) with a grid-stride loop over virtual
// 64-site tiles; a workgroup is 64 sites x nrhs columns, one wavefront per
// column, so every reduction is a wavefront reduction written to a fixed
// partial slot and the final sums are taken in a fixed order: results do not
// depend on how many solves share the launch.
#include "ddml_common.hpp"
#include "launchers.hpp"

namespace ddml {

__device__ __forceinline__ double2 wsum(double2 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off, 64);
    v.y += __shfl_xor(v.y, off, 64);
  }
  return v;
}

__device__ __forceinline__ int find_slot_v(const int* __restrict__ start, int n, int vt) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (start[mid] <= vt) lo = mid; else hi = mid;
  }
  return lo;
}

// Partial-sum slot k of column col, tile `tile`
__device__ __forceinline__ double2* part_at(double2* partial, int nrhs, int ntiles, int k, int col, int tile) {
  return partial + ((size_t)k * nrhs + col) * ntiles + tile;
}

template <typename T2, int OP>
__global__ void __launch_bounds__(768) k_vec(const SlotDesc<T2>* __restrict__ slots, const int* __restrict__ tile_start,
                                             const int* __restrict__ nslots_p) {
  using T = decltype(T2::x);
  const int ns = *nslots_p;
  const int total = tile_start[ns];
  const int lane = threadIdx.x & 63;
  const int col = threadIdx.x >> 6;
  for (int vt = blockIdx.x; vt < total; vt += gridDim.x) {
    const int s = find_slot_v(tile_start, ns, vt);
    const SlotDesc<T2>& d = slots[s];
    if (col >= d.nrhs) continue;
    if (OP != VEC_INIT && OP != VEC_RELUP && !d.active[col]) continue;  // uniform per wave
    if ((OP == VEC_INIT || OP == VEC_RELUP || OP == VEC_PFIX) && !init_here(d, OP == VEC_INIT ? 0 : 1)) continue;
    const int tile = vt - tile_start[s];
    const int i = tile * kTile + lane;
    const bool valid = i < d.g.Vh;
    const size_t base = fidx(d.ntiles, col, 0, i);
    const BiState& st = d.st[col];
    const unsigned hb = shadow_bits(col, i);
    double2 s0 = make_double2(0, 0), s1 = make_double2(0, 0);
    if (OP == VEC_S) {
      const T2 al = mk<T2>((T)st.alpha.x, (T)st.alpha.y);
      T2 o[12];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const size_t q = base + 128 * k;
        T2 r0 = mk<T2>(0, 0), r1 = r0, v0 = r0, v1 = r0;
        if (valid) {
          ld2(d.f[F_R] + q, r0, r1);
          ld2(d.f[F_V] + q, v0, v1);
        }
        o[2 * k] = csub(r0, cmul(al, v0));
        o[2 * k + 1] = csub(r1, cmul(al, v1));
        st2(d.f[F_S] + q, o[2 * k], o[2 * k + 1]);
      }
      shadow_dot(hb, o, s0);
    } else if (OP == VEC_XRP) {
      if (valid) {
        const T2 al = mk<T2>((T)st.alpha.x, (T)st.alpha.y), om = mk<T2>((T)st.omega.x, (T)st.omega.y);
        const T2 be = mk<T2>((T)st.beta.x, (T)st.beta.y);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const size_t q = base + 128 * k;
          T2 x0, x1, p0, p1, sv0, sv1, t0, t1, v0, v1;
          ld2(d.f[F_X] + q, x0, x1);
          ld2(d.f[F_P] + q, p0, p1);
          ld2(d.f[F_S] + q, sv0, sv1);
          ld2(d.f[F_T] + q, t0, t1);
          ld2(d.f[F_V] + q, v0, v1);
          st2(d.f[F_X] + q, cadd(x0, cadd(cmul(al, p0), cmul(om, sv0))), cadd(x1, cadd(cmul(al, p1), cmul(om, sv1))));
          const T2 n0 = csub(sv0, cmul(om, t0)), n1 = csub(sv1, cmul(om, t1));
          st2(d.f[F_R] + q, n0, n1);
          st2(d.f[F_P] + q, cadd(n0, cmul(be, csub(p0, cmul(om, v0)))), cadd(n1, cmul(be, csub(p1, cmul(om, v1)))));
          s1.x += (double)n0.x * n0.x + (double)n0.y * n0.y + (double)n1.x * n1.x + (double)n1.y * n1.y;
        }
      }
    } else if (OP == VEC_PFIX) {
      if (valid) {
        const T2 be = mk<T2>((T)st.beta.x, (T)st.beta.y);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const size_t q = base + 128 * k;
          T2 p0, p1, r0, r1;
          ld2(d.f[F_P] + q, p0, p1);
          ld2(d.f[F_R] + q, r0, r1);
          st2(d.f[F_P] + q, cadd(r0, cmul(be, p0)), cadd(r1, cmul(be, p1)));
        }
      }
    } else {  // VEC_INIT / VEC_RELUP: r = (T) src64, x = 0 (padding sites: all zero)
      // a fresh column gets p = r; a column that keeps its Krylov space gets
      // p - r_old, which VEC_PFIX turns into r + (rho'/rho)(p - r_old)
      const bool fresh = OP == VEC_INIT || st.status != 0;
      const T2 z = mk<T2>(0, 0);
      T2 o[12];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const size_t q = base + 128 * k;
        double2 b0 = make_double2(0, 0), b1 = b0;
        if (valid) ld2(d.src64 + q, b0, b1);
        const T2 t0 = mk<T2>((T)b0.x, (T)b0.y), t1 = mk<T2>((T)b1.x, (T)b1.y);
        if (fresh) {
          st2(d.f[F_P] + q, t0, t1);
        } else if (valid) {
          T2 p0, p1, r0, r1;
          ld2(d.f[F_P] + q, p0, p1);
          ld2(d.f[F_R] + q, r0, r1);
          st2(d.f[F_P] + q, csub(p0, r0), csub(p1, r1));
        }
        st2(d.f[F_R] + q, t0, t1);
        st2(d.f[F_X] + q, z, z);
        o[2 * k] = t0;
        o[2 * k + 1] = t1;
        s1.x += (double)t0.x * t0.x + (double)t0.y * t0.y + (double)t1.x * t1.x + (double)t1.y * t1.y;
      }
      shadow_dot(hb, o, s0);
    }
    if (OP != VEC_PFIX) {
      if (OP != VEC_XRP) s0 = wsum(s0);
      if (OP != VEC_S) s1 = wsum(s1);
      if (lane == 0) {
        if (OP == VEC_S) *part_at(d.partial, d.nrhs, d.ntiles, 3, col, tile) = s0;
        if (OP == VEC_INIT || OP == VEC_RELUP) *part_at(d.partial, d.nrhs, d.ntiles, 0, col, tile) = s0;
        if (OP != VEC_S) *part_at(d.partial, d.nrhs, d.ntiles, 1, col, tile) = s1;
      }
    }
  }
}

// The same steps on 16-bit fields (DDML_MIXED_FP16): every vector but the
// solution is stored as 16-bit fixed point with one scale per (site, column);
// the solution accumulates in FP32 (x32).  Each output is quantised before the
// fused reductions use it.
__device__ __forceinline__ float2 cm32(float2 a, float2 b) { return cmul(a, b); }

template <int OP>
__global__ void __launch_bounds__(768) k_vec16(const SlotDesc<h16c>* __restrict__ slots,
                                               const int* __restrict__ tile_start, const int* __restrict__ nslots_p) {
  const int ns = *nslots_p;
  const int total = tile_start[ns];
  const int lane = threadIdx.x & 63;
  const int col = threadIdx.x >> 6;
  for (int vt = blockIdx.x; vt < total; vt += gridDim.x) {
    const int s = find_slot_v(tile_start, ns, vt);
    const SlotDesc<h16c>& d = slots[s];
    if (col >= d.nrhs) continue;
    if (OP != VEC_INIT && OP != VEC_RELUP && !d.active[col]) continue;  // uniform per wave
    if ((OP == VEC_INIT || OP == VEC_RELUP || OP == VEC_PFIX) && !init_here(d, OP == VEC_INIT ? 0 : 1)) continue;
    const int tile = vt - tile_start[s];
    const int nt = d.ntiles;
    const int i = tile * kTile + lane;
    const bool valid = i < d.g.Vh;
    const size_t base = fidx(nt, col, 0, i);
    const size_t sx = (size_t)col * nt * kTile + i;
    const BiState& st = d.st[col];
    const unsigned hb = shadow_bits(col, i);
    const size_t qb = qidx(nt, col, i);   // 16-bit fields (quad-packed)
    auto ld = [&](int f, float2 v[12]) { spinor_load_q(d.f[f] + qb, d.nrm[f][sx], v, true); };
    auto stq = [&](int f, const float2 v[12], float2 dq[12]) {
      spinor_store_q(d.f[f] + qb, d.nrm[f] + sx, v, dq, true);
    };
    double2 s0 = make_double2(0, 0), s1 = make_double2(0, 0);
    float2 z[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) z[c] = make_float2(0, 0);
    if (OP == VEC_S) {
      const float2 al = make_float2((float)st.alpha.x, (float)st.alpha.y);
      float2 r[12], v[12], o[12], dq[12];
      if (valid) {
        ld(F_R, r);
        ld(F_V, v);
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = csub(r[c], cm32(al, v[c]));
      } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = z[c];
      }
      stq(F_S, o, dq);
      shadow_dot(hb, dq, s0);
    } else if (OP == VEC_XRP) {
      if (valid) {
        const float2 al = make_float2((float)st.alpha.x, (float)st.alpha.y);
        const float2 om = make_float2((float)st.omega.x, (float)st.omega.y);
        const float2 be = make_float2((float)st.beta.x, (float)st.beta.y);
        float2 p[12], sv[12], t[12], v[12], o[12], dq[12], np[12], dp[12];
        ld(F_P, p);
        ld(F_S, sv);
        ld(F_T, t);
        ld(F_V, v);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          float2 x0, x1;
          ld2(d.x32 + base + 128 * k, x0, x1);
          x0 = cadd(x0, cadd(cm32(al, p[2 * k]), cm32(om, sv[2 * k])));
          x1 = cadd(x1, cadd(cm32(al, p[2 * k + 1]), cm32(om, sv[2 * k + 1])));
          st2(d.x32 + base + 128 * k, x0, x1);
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = csub(sv[c], cm32(om, t[c]));
        stq(F_R, o, dq);
        // the new direction from the stored (quantised) residual
#pragma unroll
        for (int c = 0; c < 12; ++c) np[c] = cadd(dq[c], cm32(be, csub(p[c], cm32(om, v[c]))));
        stq(F_P, np, dp);
#pragma unroll
        for (int c = 0; c < 12; ++c) s1.x += (double)dq[c].x * dq[c].x + (double)dq[c].y * dq[c].y;
      }
    } else if (OP == VEC_PFIX) {
      if (valid) {
        const float2 be = make_float2((float)st.beta.x, (float)st.beta.y);
        float2 p[12], r[12], o[12], dq[12];
        ld(F_P, p);
        ld(F_R, r);
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = cadd(r[c], cm32(be, p[c]));
        stq(F_P, o, dq);
      }
    } else {  // VEC_INIT / VEC_RELUP: r = (16-bit) src64, x = 0; p as in k_vec
      const bool fresh = OP == VEC_INIT || st.status != 0;
      float2 b[12], dq[12];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        double2 b0 = make_double2(0, 0), b1 = b0;
        if (valid) ld2(d.src64 + base + 128 * k, b0, b1);
        b[2 * k] = make_float2((float)b0.x, (float)b0.y);
        b[2 * k + 1] = make_float2((float)b1.x, (float)b1.y);
        st2(d.x32 + base + 128 * k, z[2 * k], z[2 * k + 1]);
      }
      if (!fresh && valid) {
        float2 p[12], r[12], o[12], dp[12];
        ld(F_P, p);
        ld(F_R, r);
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = csub(p[c], r[c]);
        stq(F_P, o, dp);
      }
      stq(F_R, b, dq);
      if (fresh) {
        float2 dp[12];
        stq(F_P, dq, dp);
      }
      shadow_dot(hb, dq, s0);
#pragma unroll
      for (int c = 0; c < 12; ++c) s1.x += (double)dq[c].x * dq[c].x + (double)dq[c].y * dq[c].y;
    }
    if (OP != VEC_PFIX) {
      if (OP != VEC_XRP) s0 = wsum(s0);
      if (OP != VEC_S) s1 = wsum(s1);
      if (lane == 0) {
        if (OP == VEC_S) *part_at(d.partial, d.nrhs, nt, 3, col, tile) = s0;
        if (OP == VEC_INIT || OP == VEC_RELUP) *part_at(d.partial, d.nrhs, nt, 0, col, tile) = s0;
        if (OP != VEC_S) *part_at(d.partial, d.nrhs, nt, 1, col, tile) = s1;
      }
    }
  }
}

__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  const double den = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}
__device__ __forceinline__ double2 cmuld(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ bool finite2(double2 a) { return isfinite(a.x) && isfinite(a.y); }
__device__ __forceinline__ bool zero2(double2 a) { return a.x == 0 && a.y == 0; }

// Sum of partial slot k of a column over its tiles in a fixed order: thread
// t of the workgroup adds tiles t, t + 256, ... in turn, then a fixed tree in
// LDS (the same for every batch the solve is in).  Every thread calls it.
constexpr int kFinThreads = 256;
__device__ __forceinline__ double2 slot_sum(const double2* partial, int nrhs, int ntiles, int k, int col,
                                            double2* red) {
  const int tid = threadIdx.x;
  double2 a = make_double2(0, 0);
  const double2* p = partial + ((size_t)k * nrhs + col) * ntiles;
  for (int t = tid; t < ntiles; t += kFinThreads) {
    const double2 u = p[t];
    a.x += u.x;
    a.y += u.y;
  }
  red[tid] = a;
  __syncthreads();
  for (int off = kFinThreads / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] = make_double2(red[tid].x + red[tid + off].x, red[tid].y + red[tid + off].y);
    __syncthreads();
  }
  const double2 r = red[0];
  __syncthreads();
  return r;
}

// One workgroup per (slot, column): sum the tile partials in a fixed order,
// then update that column's BiCGstab scalars.
template <typename T2, int OP>
__global__ void __launch_bounds__(kFinThreads) k_fin(const SlotDesc<T2>* __restrict__ slots,
                                                     const int* __restrict__ nslots_p) {
  __shared__ double2 red[kFinThreads];
  const int s = blockIdx.x, col = blockIdx.y;
  if (s >= *nslots_p) return;
  const SlotDesc<T2>& d = slots[s];
  if (col >= d.nrhs) return;
  BiState& st = d.st[col];
  if (OP != FIN_INIT && OP != FIN_RELUP && !d.active[col]) return;   // uniform over the workgroup
  if ((OP == FIN_INIT || OP == FIN_RELUP) && !init_here(d, OP == FIN_INIT ? 0 : 1)) return;
  const int nr = d.nrhs, nt = d.ntiles;
  const double2 z = make_double2(0, 0);
  const double2 a = (OP == FIN_CHECK) ? z : slot_sum(d.partial, nr, nt, 0, col, red);
  const double2 b = (OP == FIN_ALPHA) ? z : slot_sum(d.partial, nr, nt, 1, col, red);
  const double2 c2 = (OP == FIN_OMEGA) ? slot_sum(d.partial, nr, nt, 2, col, red) : z;
  const double2 c3 = (OP == FIN_OMEGA) ? slot_sum(d.partial, nr, nt, 3, col, red) : z;
  if (threadIdx.x != 0) return;
  if (OP == FIN_RELUP && st.status == 0) {
    // a = (h, r'), b = |r'|^2 for the replaced residual r'; the Krylov space is
    // kept: VEC_PFIX makes p = r' + (rho'/rho) (p - r_old)
    const int want = d.active[col];
    if (finite2(a) && isfinite(b.x) && !zero2(st.rho)) {
      st.beta = cdiv(a, st.rho);
      st.rho = a;
    } else {
      st.beta = z;   // p = r' + 0: a fresh direction
      st.rho = a;
    }
    st.rr = b.x;
    st.rr0 = b.x;
    st.iters = 0;
    const int on = want && b.x > 0 && isfinite(b.x) && !zero2(a);
    if (want && !isfinite(b.x)) st.status = 3;
    d.active[col] = on;
    st.active = on;
  } else if (OP == FIN_INIT || OP == FIN_RELUP) {
    // a = (h, r), b = |r|^2 ; d.active holds the request flag; p = r already
    const int want = d.active[col];
    st.rr = b.x;
    st.rr0 = b.x;
    st.rho = a;
    st.alpha = make_double2(1, 0);
    st.omega = make_double2(1, 0);
    st.beta = z;
    st.iters = 0;
    st.status = 0;
    const int on = want && b.x > 0 && isfinite(b.x) && finite2(a) && !zero2(a);
    if (want && !isfinite(b.x)) st.status = 3;
    d.active[col] = on;
    st.active = on;
  } else if (OP == FIN_ALPHA) {
    // a = (h, v)
    if (!finite2(a) || zero2(a)) {
      st.status = 1;
      st.active = 0;
      d.active[col] = 0;
      st.alpha = z;
      return;
    }
    st.alpha = cdiv(st.rho, a);
  } else if (OP == FIN_OMEGA) {
    // a = (t, s), b.x = |t|^2, c2 = (h, t), c3 = (h, s); the residual after
    // this iteration is r' = s - omega t, so rho' = (h, r') = c3 - omega c2
    // and the next direction's beta is known before r' is formed
    if (b.x > 0 && isfinite(b.x) && finite2(a)) st.omega = make_double2(a.x / b.x, a.y / b.x);
    else st.omega = z;
    const double2 rho1 = make_double2(c3.x - (st.omega.x * c2.x - st.omega.y * c2.y),
                                      c3.y - (st.omega.x * c2.y + st.omega.y * c2.x));
    if (zero2(st.omega) || !finite2(rho1) || zero2(rho1) || zero2(st.rho)) {
      st.beta = z;     // x and r are still updated; FIN_CHECK ends the column
      st.status = 1;
    } else {
      st.beta = cmuld(cdiv(rho1, st.rho), cdiv(st.alpha, st.omega));
    }
    st.rho = rho1;
  } else {  // FIN_CHECK: b = |r|^2
    st.iters += 1;
    st.rr = b.x;
    const bool conv = b.x <= st.tol2 * st.rr0;
    int on = 1;
    if (!isfinite(b.x)) { st.status = 3; on = 0; }
    else if (conv) { st.status = 0; on = 0; }
    else if (st.status == 1) { on = 0; }
    else if (st.iters >= st.max_iters) { st.status = 2; on = 0; }
    st.active = on;
    d.active[col] = on;
  }
}

// ------------------------------------------------------------------ GCR(m)
// Generalised conjugate residual on the Schur operator (Eisenstat, Elman and
// Schultz 1983), restarted every m steps, one recursion per column.  Step k
// of a cycle, with p_k the current residual (written by the previous step):
//   q_k = M p_k (stencil);  beta_j = (q_j, q_k) / |q_j|^2 for j < k (classical
//   Gram-Schmidt, one pass for all j);  q_k -= sum beta_j q_j, p_k -= sum
//   beta_j p_j;  alpha = (q_k, r) / |q_k|^2;  x += alpha p_k;  r -= alpha q_k;
//   p_{k+1 mod m} = r.
// The residual norm decreases monotonically.  Reductions as in BiCGstab:
// per-tile FP64 partials, fixed-order finalisation.
template <typename T2, int OP>
__global__ void __launch_bounds__(768) k_gcr(const SlotDesc<T2>* __restrict__ slots, const int* __restrict__ tile_start,
                                             const int* __restrict__ nslots_p, int k, int m) {
  using T = decltype(T2::x);
  const int ns = *nslots_p;
  const int total = tile_start[ns];
  const int lane = threadIdx.x & 63;
  const int col = threadIdx.x >> 6;
  for (int vt = blockIdx.x; vt < total; vt += gridDim.x) {
    const int s = find_slot_v(tile_start, ns, vt);
    const SlotDesc<T2>& d = slots[s];
    if (col >= d.nrhs) continue;
    if (OP != GCR_INIT && !d.active[col]) continue;  // uniform per wave
    const int tile = vt - tile_start[s];
    const int nt = d.ntiles;
    const int i = tile * kTile + lane;
    const bool valid = i < d.g.Vh;
    const size_t base = fidx(nt, col, 0, i);
    const double2* gc = d.gcoef + (size_t)col * 2 * kGcrMax;
    double2 red[kGcrMax];
#pragma unroll
    for (int j = 0; j < kGcrMax; ++j) red[j] = make_double2(0, 0);
    if (OP == GCR_INIT) {  // r = (T) src64, x = 0, p_0 = r; red[0] = |r|^2
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const size_t o = base + 128 * q;
        double2 b0 = make_double2(0, 0), b1 = b0;
        if (valid) ld2(d.src64 + o, b0, b1);
        const T2 t0 = mk<T2>((T)b0.x, (T)b0.y), t1 = mk<T2>((T)b1.x, (T)b1.y), z = mk<T2>(0, 0);
        st2(d.f[F_R] + o, t0, t1);
        st2(d.f[F_GP0] + o, t0, t1);
        st2(d.f[F_X] + o, z, z);
        red[0].x += (double)t0.x * t0.x + (double)t0.y * t0.y + (double)t1.x * t1.x + (double)t1.y * t1.y;
      }
    } else if (OP == GCR_DOTS) {  // red[j] = (q_j, q_k), j < k
      if (valid) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const size_t o = base + 128 * q;
          T2 a0, a1;
          ld2(d.f[F_GQ0 + k] + o, a0, a1);
#pragma unroll
          for (int j = 0; j < kGcrMax; ++j) {
            if (j >= k) break;
            T2 b0, b1;
            ld2(d.f[F_GQ0 + j] + o, b0, b1);
            red[j].x += (double)b0.x * a0.x + (double)b0.y * a0.y + (double)b1.x * a1.x + (double)b1.y * a1.y;
            red[j].y += (double)b0.x * a0.y - (double)b0.y * a0.x + (double)b1.x * a1.y - (double)b1.y * a1.x;
          }
        }
      }
    } else if (OP == GCR_UPDATE) {  // orthogonalise q_k, p_k; red[0] = (q_k, r), red[1] = |q_k|^2
      if (valid) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const size_t o = base + 128 * q;
          T2 qa, qb, pa, pb, ra, rb;
          ld2(d.f[F_GQ0 + k] + o, qa, qb);
          ld2(d.f[F_GP0 + k] + o, pa, pb);
#pragma unroll
          for (int j = 0; j < kGcrMax; ++j) {
            if (j >= k) break;
            const T2 be = mk<T2>((T)gc[j].x, (T)gc[j].y);
            T2 u0, u1;
            ld2(d.f[F_GQ0 + j] + o, u0, u1);
            qa = csub(qa, cmul(be, u0));
            qb = csub(qb, cmul(be, u1));
            ld2(d.f[F_GP0 + j] + o, u0, u1);
            pa = csub(pa, cmul(be, u0));
            pb = csub(pb, cmul(be, u1));
          }
          if (k > 0) {
            st2(d.f[F_GQ0 + k] + o, qa, qb);
            st2(d.f[F_GP0 + k] + o, pa, pb);
          }
          ld2(d.f[F_R] + o, ra, rb);
          red[0].x += (double)qa.x * ra.x + (double)qa.y * ra.y + (double)qb.x * rb.x + (double)qb.y * rb.y;
          red[0].y += (double)qa.x * ra.y - (double)qa.y * ra.x + (double)qb.x * rb.y - (double)qb.y * rb.x;
          red[1].x += (double)qa.x * qa.x + (double)qa.y * qa.y + (double)qb.x * qb.x + (double)qb.y * qb.y;
        }
      }
    } else {  // GCR_XR: x += alpha p_k, r -= alpha q_k, p_{k+1 mod m} = r; red[0] = |r|^2
      if (valid) {
        const BiState& st = d.st[col];
        const T2 al = mk<T2>((T)st.alpha.x, (T)st.alpha.y);
        const int nx = (k + 1 == m) ? 0 : k + 1;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
          const size_t o = base + 128 * q;
          T2 x0, x1, p0, p1, q0, q1, r0, r1;
          ld2(d.f[F_X] + o, x0, x1);
          ld2(d.f[F_GP0 + k] + o, p0, p1);
          ld2(d.f[F_GQ0 + k] + o, q0, q1);
          ld2(d.f[F_R] + o, r0, r1);
          st2(d.f[F_X] + o, cadd(x0, cmul(al, p0)), cadd(x1, cmul(al, p1)));
          r0 = csub(r0, cmul(al, q0));
          r1 = csub(r1, cmul(al, q1));
          st2(d.f[F_R] + o, r0, r1);
          st2(d.f[F_GP0 + nx] + o, r0, r1);
          red[0].x += (double)r0.x * r0.x + (double)r0.y * r0.y + (double)r1.x * r1.x + (double)r1.y * r1.y;
        }
      }
    }
    const int nred = OP == GCR_DOTS ? k : (OP == GCR_UPDATE ? 2 : 1);
#pragma unroll
    for (int j = 0; j < kGcrMax; ++j) {
      if (j >= nred) break;
      const double2 v = wsum(red[j]);
      if (lane == 0) d.partial[((size_t)j * d.nrhs + col) * d.ntiles + tile] = v;
    }
  }
}

// One workgroup per slot, one wavefront per column (fixed-order sums).
template <typename T2, int OP>
__global__ void __launch_bounds__(768) k_gcr_fin(const SlotDesc<T2>* __restrict__ slots, const int* __restrict__ nslots_p,
                                                 int k) {
  const int s = blockIdx.x;
  if (s >= *nslots_p) return;
  const SlotDesc<T2>& d = slots[s];
  const int lane = threadIdx.x & 63;
  const int col = threadIdx.x >> 6;
  if (col >= d.nrhs) return;
  BiState& st = d.st[col];
  if (OP != GFIN_INIT && !d.active[col]) return;
  const int nred = OP == GFIN_BETA ? k : (OP == GFIN_ALPHA ? 2 : 1);
  double2 sum[kGcrMax];
#pragma unroll
  for (int j = 0; j < kGcrMax; ++j) {
    sum[j] = make_double2(0, 0);
    if (j >= nred) continue;
    const double2* p = d.partial + ((size_t)j * d.nrhs + col) * d.ntiles;
    for (int t = lane; t < d.ntiles; t += 64) {
      sum[j].x += p[t].x;
      sum[j].y += p[t].y;
    }
    sum[j] = wsum(sum[j]);
  }
  if (lane != 0) return;
  double2* gc = d.gcoef + (size_t)col * 2 * kGcrMax;
  if (OP == GFIN_INIT) {  // st.active holds the request flag
    const int want = d.active[col];
    st.rr = sum[0].x;
    st.rr0 = sum[0].x;
    st.iters = 0;
    st.status = 0;
    const int on = want && sum[0].x > 0 && isfinite(sum[0].x);
    if (want && !isfinite(sum[0].x)) st.status = 3;
    d.active[col] = on;
    st.active = on;
  } else if (OP == GFIN_BETA) {
    for (int j = 0; j < k; ++j) {
      const double qq = gc[kGcrMax + j].x;
      gc[j] = qq > 0 ? make_double2(sum[j].x / qq, sum[j].y / qq) : make_double2(0, 0);
    }
  } else if (OP == GFIN_ALPHA) {  // sum[0] = (q_k, r), sum[1] = |q_k|^2
    const double qq = sum[1].x;
    gc[kGcrMax + k] = make_double2(qq, 0);
    if (!(qq > 0) || !isfinite(qq) || !finite2(sum[0])) {
      st.status = isfinite(qq) ? 1 : 3;
      st.active = 0;
      d.active[col] = 0;
      st.alpha = make_double2(0, 0);
      return;
    }
    st.alpha = make_double2(sum[0].x / qq, sum[0].y / qq);
  } else {  // GFIN_CHECK: sum[0] = |r|^2
    st.iters += 1;
    st.rr = sum[0].x;
    int on = 1;
    if (!isfinite(sum[0].x)) { st.status = 3; on = 0; }
    else if (sum[0].x <= st.tol2 * st.rr0) { st.status = 0; on = 0; }
    else if (st.iters >= st.max_iters) { st.status = 2; on = 0; }
    st.active = on;
    d.active[col] = on;
  }
}

template <typename T2>
static hipError_t gcr_impl(const SlotDesc<T2>* slots, const int* tile_start, const int* nslots_p, int nrhs, int op,
                           int k, int m, int grid, hipStream_t st) {
  if (k < 0 || k >= m || m < 1 || m > kGcrMax) return hipErrorInvalidValue;
  dim3 b(64 * nrhs);
  switch (op) {
    case GCR_INIT: hipLaunchKernelGGL((k_gcr<T2, GCR_INIT>), dim3(grid), b, 0, st, slots, tile_start, nslots_p, k, m); break;
    case GCR_DOTS: hipLaunchKernelGGL((k_gcr<T2, GCR_DOTS>), dim3(grid), b, 0, st, slots, tile_start, nslots_p, k, m); break;
    case GCR_UPDATE: hipLaunchKernelGGL((k_gcr<T2, GCR_UPDATE>), dim3(grid), b, 0, st, slots, tile_start, nslots_p, k, m); break;
    case GCR_XR: hipLaunchKernelGGL((k_gcr<T2, GCR_XR>), dim3(grid), b, 0, st, slots, tile_start, nslots_p, k, m); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template <typename T2>
static hipError_t gcr_fin_impl(const SlotDesc<T2>* slots, const int* nslots_p, int max_slots, int op, int k,
                               hipStream_t st) {
  if (k < 0 || k >= kGcrMax) return hipErrorInvalidValue;
  dim3 b(64 * kMaxRhs);
  switch (op) {
    case GFIN_INIT: hipLaunchKernelGGL((k_gcr_fin<T2, GFIN_INIT>), dim3(max_slots), b, 0, st, slots, nslots_p, k); break;
    case GFIN_BETA: hipLaunchKernelGGL((k_gcr_fin<T2, GFIN_BETA>), dim3(max_slots), b, 0, st, slots, nslots_p, k); break;
    case GFIN_ALPHA: hipLaunchKernelGGL((k_gcr_fin<T2, GFIN_ALPHA>), dim3(max_slots), b, 0, st, slots, nslots_p, k); break;
    case GFIN_CHECK: hipLaunchKernelGGL((k_gcr_fin<T2, GFIN_CHECK>), dim3(max_slots), b, 0, st, slots, nslots_p, k); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_gcr(const SlotDesc<float2>* slots, const int* tile_start, const int* nslots_p, int nrhs, int op,
                      int k, int m, int grid, hipStream_t st) {
  return gcr_impl(slots, tile_start, nslots_p, nrhs, op, k, m, grid, st);
}
hipError_t launch_gcr(const SlotDesc<double2>* slots, const int* tile_start, const int* nslots_p, int nrhs, int op,
                      int k, int m, int grid, hipStream_t st) {
  return gcr_impl(slots, tile_start, nslots_p, nrhs, op, k, m, grid, st);
}
hipError_t launch_gcr_fin(const SlotDesc<float2>* slots, const int* nslots_p, int max_slots, int op, int k,
                          hipStream_t st) {
  return gcr_fin_impl(slots, nslots_p, max_slots, op, k, st);
}
hipError_t launch_gcr_fin(const SlotDesc<double2>* slots, const int* nslots_p, int max_slots, int op, int k,
                          hipStream_t st) {
  return gcr_fin_impl(slots, nslots_p, max_slots, op, k, st);
}

template <typename T2>
static hipError_t vec_impl(const SlotDesc<T2>* slots, const int* tile_start, const int* nslots_p, int nrhs, int op,
                           int grid, hipStream_t st) {
  dim3 b(64 * nrhs);
  switch (op) {
    case VEC_S: hipLaunchKernelGGL((k_vec<T2, VEC_S>), dim3(grid), b, 0, st, slots, tile_start, nslots_p); break;
    case VEC_XRP: hipLaunchKernelGGL((k_vec<T2, VEC_XRP>), dim3(grid), b, 0, st, slots, tile_start, nslots_p); break;
    case VEC_PFIX: hipLaunchKernelGGL((k_vec<T2, VEC_PFIX>), dim3(grid), b, 0, st, slots, tile_start, nslots_p); break;
    case VEC_INIT: hipLaunchKernelGGL((k_vec<T2, VEC_INIT>), dim3(grid), b, 0, st, slots, tile_start, nslots_p); break;
    case VEC_RELUP: hipLaunchKernelGGL((k_vec<T2, VEC_RELUP>), dim3(grid), b, 0, st, slots, tile_start, nslots_p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_vec(const SlotDesc<float2>* slots, const int* tile_start, const int* nslots_p, int nrhs, int op,
                      int grid, hipStream_t st) {
  return vec_impl(slots, tile_start, nslots_p, nrhs, op, grid, st);
}
hipError_t launch_vec(const SlotDesc<double2>* slots, const int* tile_start, const int* nslots_p, int nrhs, int op,
                      int grid, hipStream_t st) {
  return vec_impl(slots, tile_start, nslots_p, nrhs, op, grid, st);
}
hipError_t launch_vec(const SlotDesc<h16c>* slots, const int* tile_start, const int* nslots_p, int nrhs, int op,
                      int grid, hipStream_t st) {
  dim3 b(64 * nrhs);
  switch (op) {
    case VEC_S: hipLaunchKernelGGL(k_vec16<VEC_S>, dim3(grid), b, 0, st, slots, tile_start, nslots_p); break;
    case VEC_XRP: hipLaunchKernelGGL(k_vec16<VEC_XRP>, dim3(grid), b, 0, st, slots, tile_start, nslots_p); break;
    case VEC_PFIX: hipLaunchKernelGGL(k_vec16<VEC_PFIX>, dim3(grid), b, 0, st, slots, tile_start, nslots_p); break;
    case VEC_INIT: hipLaunchKernelGGL(k_vec16<VEC_INIT>, dim3(grid), b, 0, st, slots, tile_start, nslots_p); break;
    case VEC_RELUP: hipLaunchKernelGGL(k_vec16<VEC_RELUP>, dim3(grid), b, 0, st, slots, tile_start, nslots_p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T2>
static hipError_t fin_impl(const SlotDesc<T2>* slots, const int* nslots_p, int max_slots, int op, hipStream_t st) {
  const dim3 b(kFinThreads), grid(max_slots, kMaxRhs);
  switch (op) {
    case FIN_INIT: hipLaunchKernelGGL((k_fin<T2, FIN_INIT>), grid, b, 0, st, slots, nslots_p); break;
    case FIN_ALPHA: hipLaunchKernelGGL((k_fin<T2, FIN_ALPHA>), grid, b, 0, st, slots, nslots_p); break;
    case FIN_OMEGA: hipLaunchKernelGGL((k_fin<T2, FIN_OMEGA>), grid, b, 0, st, slots, nslots_p); break;
    case FIN_CHECK: hipLaunchKernelGGL((k_fin<T2, FIN_CHECK>), grid, b, 0, st, slots, nslots_p); break;
    case FIN_RELUP: hipLaunchKernelGGL((k_fin<T2, FIN_RELUP>), grid, b, 0, st, slots, nslots_p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
hipError_t launch_fin(const SlotDesc<float2>* slots, const int* nslots_p, int max_slots, int op, hipStream_t st) {
  return fin_impl(slots, nslots_p, max_slots, op, st);
}
hipError_t launch_fin(const SlotDesc<double2>* slots, const int* nslots_p, int max_slots, int op, hipStream_t st) {
  return fin_impl(slots, nslots_p, max_slots, op, st);
}
hipError_t launch_fin(const SlotDesc<h16c>* slots, const int* nslots_p, int max_slots, int op, hipStream_t st) {
  return fin_impl(slots, nslots_p, max_slots, op, st);
}

// ------------------------------------------------------- raw elementwise
template <typename Tin>
__global__ void k_cast_d(const Tin* __restrict__ in, double2* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = make_double2((double)in[i].x, (double)in[i].y);
}
__global__ void k_axpy_d(double2* __restrict__ y, const double2* __restrict__ x, double a, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    y[i].x += a * x[i].x;
    y[i].y += a * x[i].y;
  }
}
static int grid_n(size_t n) {
  size_t g = (n + 255) / 256;
  return (int)(g > 16384 ? 16384 : (g == 0 ? 1 : g));
}
hipError_t launch_cast_to_d(const float2* in, double2* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_cast_d<float2>), dim3(grid_n(n)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}
hipError_t launch_cast_to_d(const double2* in, double2* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_cast_d<double2>), dim3(grid_n(n)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}
__global__ void k_cast_f(const double2* __restrict__ in, float2* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = make_float2((float)in[i].x, (float)in[i].y);
}
hipError_t launch_cast_to_f(const double2* in, float2* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_cast_f, dim3(grid_n(n)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}
template <typename T2>
__global__ void k_fill(T2* __restrict__ v, size_t n, double a) {
  using T = decltype(T2::x);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    v[i] = mk<T2>((T)(a * (1.0 + 1e-3 * (double)(i % 97))), (T)(0.5 * a));
}
hipError_t launch_fill(float2* v, size_t n, double a, hipStream_t st) {
  hipLaunchKernelGGL((k_fill<float2>), dim3(grid_n(n)), dim3(256), 0, st, v, n, a);
  return hipGetLastError();
}
hipError_t launch_fill(double2* v, size_t n, double a, hipStream_t st) {
  hipLaunchKernelGGL((k_fill<double2>), dim3(grid_n(n)), dim3(256), 0, st, v, n, a);
  return hipGetLastError();
}
// 16-bit field with values {q, q/2} (q varying per element) and every scale a
__global__ void k_fill16(h16c* __restrict__ v, size_t n, float* __restrict__ nrm, size_t nn, float a) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const short q = (short)(16384 + 100 * (int)(i % 97));
    v[i] = h16c{q, (short)(q / 2)};
  }
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nn; i += (size_t)gridDim.x * blockDim.x)
    nrm[i] = a;
}
hipError_t launch_fill16(h16c* v, size_t n, float* nrm, size_t nn, double a, hipStream_t st) {
  hipLaunchKernelGGL(k_fill16, dim3(grid_n(n)), dim3(256), 0, st, v, n, nrm, nn, (float)a);
  return hipGetLastError();
}
// FP64 field <-> 16-bit field, one thread per (site, column) of [nrhs][ntiles * 64]
__global__ void k_quant16(const double2* __restrict__ in, h16c* __restrict__ out, float* __restrict__ nrm, int nrhs,
                          int ntiles) {
  const size_t per = (size_t)ntiles * kTile;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < per * nrhs; t += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(t / per), i = (int)(t % per);
    const size_t base = fidx(ntiles, col, 0, i);
    float2 v[12], dq[12];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double2 a, b;
      ld2(in + base + 128 * k, a, b);
      v[2 * k] = make_float2((float)a.x, (float)a.y);
      v[2 * k + 1] = make_float2((float)b.x, (float)b.y);
    }
    spinor_store_q(out + qidx(ntiles, col, i), nrm + t, v, dq, false);
  }
}
__global__ void k_dequant16(const h16c* __restrict__ in, const float* __restrict__ nrm, double2* __restrict__ out,
                            int nrhs, int ntiles) {
  const size_t per = (size_t)ntiles * kTile;
  for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < per * nrhs; t += (size_t)gridDim.x * blockDim.x) {
    const int col = (int)(t / per), i = (int)(t % per);
    const size_t base = fidx(ntiles, col, 0, i);
    float2 v[12];
    spinor_load_q(in + qidx(ntiles, col, i), nrm[t], v, false);
#pragma unroll
    for (int k = 0; k < 6; ++k)
      st2(out + base + 128 * k, make_double2(v[2 * k].x, v[2 * k].y), make_double2(v[2 * k + 1].x, v[2 * k + 1].y));
  }
}
hipError_t launch_quant16(const double2* in, h16c* out, float* nrm, int nrhs, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_quant16, dim3(grid_n((size_t)nrhs * ntiles * kTile)), dim3(256), 0, st, in, out, nrm, nrhs,
                     ntiles);
  return hipGetLastError();
}
hipError_t launch_dequant16(const h16c* in, const float* nrm, double2* out, int nrhs, int ntiles, hipStream_t st) {
  hipLaunchKernelGGL(k_dequant16, dim3(grid_n((size_t)nrhs * ntiles * kTile)), dim3(256), 0, st, in, nrm, out, nrhs,
                     ntiles);
  return hipGetLastError();
}

hipError_t launch_axpy_d(double2* y, const double2* x, double a, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_d, dim3(grid_n(n)), dim3(256), 0, st, y, x, a, n);
  return hipGetLastError();
}

// |v_col|^2 per 64-site tile into partial[col][tile]
__global__ void k_col_norms(const double2* __restrict__ v, int Vh, int nrhs, double2* __restrict__ partial, int ntiles) {
  const int lane = threadIdx.x & 63;
  const int col = threadIdx.x >> 6;
  if (col >= nrhs) return;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int i = tile * kTile + lane;
    double2 s = make_double2(0, 0);
    if (i < Vh) {
      for (int c = 0; c < 12; ++c) {
        const double2 a = v[fidx(ntiles, col, c, i)];
        s.x += a.x * a.x + a.y * a.y;
      }
    }
    s = wsum(s);
    if (lane == 0) partial[(size_t)col * ntiles + tile] = s;
  }
}
__global__ void k_sum_partials(const double2* __restrict__ partial, int nred, int nrhs, int ntiles,
                               double2* __restrict__ out, int accumulate) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x;  // (red, col)
  if (k >= nred * nrhs) return;
  const double2* p = partial + (size_t)k * ntiles;
  double2 a = make_double2(0, 0);
  for (int t = lane; t < ntiles; t += 64) {
    a.x += p[t].x;
    a.y += p[t].y;
  }
  a = wsum(a);
  if (lane == 0) {
    if (accumulate) { out[k].x += a.x; out[k].y += a.y; }
    else out[k] = a;
  }
}
hipError_t launch_col_norms(const double2* v, int Vh, int nrhs, double2* partial, int ntiles, double2* out,
                            int accumulate, hipStream_t st) {
  int grid = ntiles < 16384 ? ntiles : 16384;
  hipLaunchKernelGGL(k_col_norms, dim3(grid), dim3(64 * nrhs), 0, st, v, Vh, nrhs, partial, ntiles);
  hipLaunchKernelGGL(k_sum_partials, dim3(nrhs), dim3(64), 0, st, partial, 1, nrhs, ntiles,
                     out, accumulate);
  return hipGetLastError();
}
hipError_t launch_sum_partials(const double2* partial, int nred, int nrhs, int ntiles, double2* out, int accumulate,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_sum_partials, dim3(nred * nrhs), dim3(64), 0, st, partial, nred, nrhs, ntiles, out,
                     accumulate);
  return hipGetLastError();
}

}  // namespace ddml
