// Device-side outer loop of the batched domain solves.
//
// The FP64 defect correction of a mixed-precision solve (solve D_Gamma x = b
// as M x = b', b' = 2 kappa b, with the inner Krylov solver on the even-odd
// Schur operator) runs here as kernels over the whole slot table, captured in
// the solver graph before the inner iterations, so that a batch advances from
// one inner cycle to the next without the host:
//   gate     a slot whose inner solve has stopped on every column moves to
//            PH_EXPORT; the column flags of the outer step are set;
//   export   e_e = (inner x), e_o = A_oo^{-1}(r_o + kappa H_oe e_e), x += e;
//   residual r = b' - M x in FP64 (stencil MODE_RES, both parities) and |r|^2;
//   decide   per column: converged (|r| <= tol |b'|), failed (not finite) or
//            out of corrections, else the next inner tolerance;
//   prepare  r^_e = A_ee^{-1}(r_e + kappa H_eo A_oo^{-1} r_o) (the inner
//            right-hand side) and the inner initialisation;
//   commit   PH_PREP -> PH_INNER.
// The stencil steps are the FP64 batched stencil on views of the slot table
// whose column flags are the outer-step flags; everything here is
// elementwise or per column.  Sums run in a fixed order per slot, so a solve
// does the same arithmetic whichever batch it is in.
#include "../../include/ddml.h"
#include "ddml_common.hpp"
#include "launchers.hpp"

namespace ddml {

__device__ __forceinline__ int outer_find_slot(const int* __restrict__ start, int n, int vt) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= vt) lo = mid; else hi = mid;
  }
  return lo;
}

// One workgroup (64 threads) per slot; thread c is column c.
template <typename T2>
__global__ void __launch_bounds__(64) k_outer_gate(const SlotDesc<T2>* __restrict__ slots,
                                                   const int* __restrict__ nslots_p) {
  const int s = blockIdx.x;
  if (s >= *nslots_p) return;
  const SlotDesc<T2>& d = slots[s];
  if (!d.sst) return;
  const int col = threadIdx.x;
  const int ph = d.sst->phase;
  const bool mine = col < d.nrhs;
  const int act = (mine && ph == PH_INNER) ? d.active[col] : 0;
  const bool stopped = ph == PH_INNER && __syncthreads_or(act) == 0;
  const int nph = stopped ? PH_EXPORT : ph;
  if (mine) {
    OuterState& o = d.ost[col];
    if (stopped && !o.done) o.inner_total += d.st[col].iters;
    const int live = !o.done;
    d.oflag[OF_EXPORT * d.nrhs + col] = (nph == PH_EXPORT) && live;
    d.oflag[OF_RESID * d.nrhs + col] = (nph == PH_EXPORT || nph == PH_NEW) && live;
    d.oflag[OF_PREP * d.nrhs + col] = 0;
  }
  if (col == 0 && stopped) d.sst->phase = PH_EXPORT;
}

// y = M x for one Hermitian 6x6 block of FP64 clover data (18 slots: the
// diagonal packed in slots 0..2, then the upper triangle row by row)
__device__ __forceinline__ void outer_herm6(const double2* __restrict__ cl, int b, int nt, int p, int i,
                                            const double2 x[6], double2 y[6]) {
  double2 m[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) m[k] = cl[cidx(nt, p, 18 * b + k, i)];
  const double dg[6] = {m[0].x, m[0].y, m[1].x, m[1].y, m[2].x, m[2].y};
#pragma unroll
  for (int q = 0; q < 6; ++q) y[q] = make_double2(x[q].x * dg[q], x[q].y * dg[q]);
  int k = 3;
#pragma unroll
  for (int q = 0; q < 6; ++q)
#pragma unroll
    for (int j = q + 1; j < 6; ++j) {
      const double2 h = m[k++];
      y[q] = cmac(y[q], h, x[j]);
      y[j] = cmacc(y[j], h, x[q]);
    }
}

// Elementwise steps of the outer loop over (slot, tile), one wavefront per
// column (workgroup of 64 x nrhs threads), gated by the column flags.
//   OSTEP_CAST    t_e = (double) inner x              (export flag)
//   OSTEP_AXPY    x_e += t_e, x_o += t_o             (export flag)
//   OSTEP_CLOVER  t_o = A_oo^{-1} r_o                (prepare flag)
enum { OSTEP_CAST = 0, OSTEP_AXPY = 1, OSTEP_CLOVER = 2 };

template <typename T2> __device__ __forceinline__ const void* inner_x(const SlotDesc<T2>& d) { return d.f[F_X]; }
template <> __device__ __forceinline__ const void* inner_x<h16c>(const SlotDesc<h16c>& d) { return d.x32; }

template <typename T2, int OP>
__global__ void __launch_bounds__(768) k_outer_vec(const SlotDesc<T2>* __restrict__ slots,
                                                   const int* __restrict__ tile_start,
                                                   const int* __restrict__ nslots_p) {
  const int ns = *nslots_p;
  const int total = tile_start[ns];
  const int lane = threadIdx.x & 63;
  const int col = threadIdx.x >> 6;
  for (int vt = blockIdx.x; vt < total; vt += gridDim.x) {
    const int s = outer_find_slot(tile_start, ns, vt);
    const SlotDesc<T2>& d = slots[s];
    if (!d.sst || col >= d.nrhs) continue;
    const int fl = OP == OSTEP_CLOVER ? OF_PREP : OF_EXPORT;
    if (!d.oflag[fl * d.nrhs + col]) continue;   // uniform per wave
    const int tile = vt - tile_start[s];
    const int nt = d.ntiles;
    const int i = tile * kTile + lane;
    const bool valid = i < d.g.Vh;
    const size_t base = fidx(nt, col, 0, i);
    if (OP == OSTEP_CAST) {
      // the inner solution (FP32, or FP64 when the inner solve is FP64) in FP64
      using XT = typename std::conditional<std::is_same<T2, double2>::value, double2, float2>::type;
      const XT* x = static_cast<const XT*>(inner_x(d));
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const size_t o = base + 128 * (c >> 1) + (c & 1);
        const XT v = valid ? x[o] : mk<XT>(0, 0);
        d.o64[O_TE][o] = make_double2((double)v.x, (double)v.y);
      }
    } else if (OP == OSTEP_AXPY) {
      if (valid) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const size_t o = base + 128 * (c >> 1) + (c & 1);
          const double2 te = d.o64[O_TE][o], to = d.o64[O_TO][o];
          double2 xe = d.o64[O_XE][o], xo = d.o64[O_XO][o];
          xe.x += te.x;
          xe.y += te.y;
          xo.x += to.x;
          xo.y += to.y;
          d.o64[O_XE][o] = xe;
          d.o64[O_XO][o] = xo;
        }
      }
    } else {  // OSTEP_CLOVER
      double2 x[12], y[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) x[c] = valid ? d.o64[O_RO][base + 128 * (c >> 1) + (c & 1)] : make_double2(0, 0);
#pragma unroll
      for (int b = 0; b < 2; ++b) outer_herm6(d.Ainv64, b, nt, 1, i, x + 6 * b, y + 6 * b);
#pragma unroll
      for (int c = 0; c < 12; ++c)
        d.o64[O_TO][base + 128 * (c >> 1) + (c & 1)] = valid ? y[c] : make_double2(0, 0);
    }
  }
}

// Fixed-order sum of region k of the FP64 partials of one column.
constexpr int kOuterThreads = 256;
__device__ __forceinline__ double outer_sum(const double2* partial, int nrhs, int ntiles, int k, int col,
                                           double* red) {
  const int tid = threadIdx.x;
  double a = 0;
  const double2* p = partial + ((size_t)k * nrhs + col) * ntiles;
  for (int t = tid; t < ntiles; t += kOuterThreads) a += p[t].x;
  red[tid] = a;
  __syncthreads();
  for (int off = kOuterThreads / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// One workgroup per (slot, column) with the residual flag: |r|^2 from the two
// parities, the relative residual, and what the column does next.
template <typename T2>
__global__ void __launch_bounds__(kOuterThreads) k_outer_decide(const SlotDesc<T2>* __restrict__ slots,
                                                               const int* __restrict__ nslots_p) {
  __shared__ double red[kOuterThreads];
  const int s = blockIdx.x, col = blockIdx.y;
  if (s >= *nslots_p) return;
  const SlotDesc<T2>& d = slots[s];
  if (!d.sst || col >= d.nrhs || !d.oflag[OF_RESID * d.nrhs + col]) return;   // uniform
  const double rn2 = outer_sum(d.partial64, d.nrhs, d.ntiles, 0, col, red) +
                     outer_sum(d.partial64, d.nrhs, d.ntiles, 1, col, red);
  if (threadIdx.x != 0) return;
  OuterState& o = d.ost[col];
  if (d.sst->phase == PH_NEW) o.bn2 = rn2;   // x = 0: r = b'
  const double rel = (o.bn2 > 0 || !isfinite(o.bn2)) ? sqrt(rn2 / o.bn2) : 0.0;
  o.rel = rel;
  int go = 0;
  if (!isfinite(rel)) {
    o.status = DDML_ENUMERIC;
    o.rel = INFINITY;
    o.done = 1;
  } else if (rel <= d.tol) {
    o.done = 1;
  } else if (d.sst->cycles >= d.max_outer) {
    o.done = 1;   // out of corrections (the caller sees rel > tol)
  } else {
    go = 1;
    // the reduction this cycle must reach: tol |b'| / |r| with a safety
    // factor, never tighter than the inner tolerance in mixed precision
    double it = 0.1 * d.tol / rel;
    it = d.prec == DDML_FP64 ? fmax(it, 1e-14) : fmax(it, d.inner_tol);
    if (d.prec == DDML_MIXED_FP16) it = fmax(it, kInnerFloor16);
    it = fmin(it, 0.1);
    d.st[col].tol2 = it * it;
    d.st[col].max_iters = d.max_inner;
  }
  d.oflag[OF_PREP * d.nrhs + col] = go;
  d.active[col] = go;   // the request flag of the inner initialisation
}

// One thread per slot.  STEP 0 (after decide): PH_NEW / PH_EXPORT -> PH_PREP
// if any column goes on (one more inner cycle), else PH_DONE.  STEP 1 (after
// the inner initialisation): PH_PREP -> PH_INNER.
template <typename T2, int STEP>
__global__ void k_outer_phase(const SlotDesc<T2>* __restrict__ slots, const int* __restrict__ nslots_p) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= *nslots_p) return;
  const SlotDesc<T2>& d = slots[s];
  if (!d.sst) return;
  SlotState& st = *d.sst;
  if (STEP == 0) {
    if (st.phase != PH_NEW && st.phase != PH_EXPORT) return;
    int go = 0;
    for (int c = 0; c < d.nrhs; ++c) go |= d.oflag[OF_PREP * d.nrhs + c];
    if (go) {
      st.phase = PH_PREP;
      st.cycles += 1;
    } else {
      st.phase = PH_DONE;
    }
  } else {
    if (st.phase == PH_PREP) st.phase = PH_INNER;
  }
}

__global__ void __launch_bounds__(64) k_outer_reset(SlotState* sst, OuterState* ost, int* act, int* oflag,
                                                    int phase) {
  const int s = blockIdx.x, c = threadIdx.x;
  if (c < kMaxRhs) {
    OuterState z{};
    ost[(size_t)s * kMaxRhs + c] = z;
    act[(size_t)s * kMaxRhs + c] = 0;
  }
  if (c < 3 * kMaxRhs) oflag[(size_t)s * 3 * kMaxRhs + c] = 0;
  if (c == 0) {
    sst[s].phase = phase;
    sst[s].cycles = 0;
  }
}

hipError_t launch_outer_reset(SlotState* sst, OuterState* ost, int* act, int* oflag, int n, int phase,
                              hipStream_t st) {
  if (n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_outer_reset, dim3(n), dim3(64), 0, st, sst, ost, act, oflag, phase);
  return hipGetLastError();
}

template <typename T2>
static hipError_t outer_impl(const SlotDesc<T2>* slots, const int* tile_start, const int* nslots_p, int max_slots,
                             int nrhs, int step, int grid, hipStream_t st) {
  switch (step) {
    case OUTER_GATE:
      hipLaunchKernelGGL((k_outer_gate<T2>), dim3(max_slots), dim3(64), 0, st, slots, nslots_p);
      break;
    case OUTER_CAST:
      hipLaunchKernelGGL((k_outer_vec<T2, OSTEP_CAST>), dim3(grid), dim3(64 * nrhs), 0, st, slots, tile_start,
                         nslots_p);
      break;
    case OUTER_AXPY:
      hipLaunchKernelGGL((k_outer_vec<T2, OSTEP_AXPY>), dim3(grid), dim3(64 * nrhs), 0, st, slots, tile_start,
                         nslots_p);
      break;
    case OUTER_CLOVER:
      hipLaunchKernelGGL((k_outer_vec<T2, OSTEP_CLOVER>), dim3(grid), dim3(64 * nrhs), 0, st, slots, tile_start,
                         nslots_p);
      break;
    case OUTER_DECIDE:
      hipLaunchKernelGGL((k_outer_decide<T2>), dim3(max_slots, kMaxRhs), dim3(kOuterThreads), 0, st, slots,
                         nslots_p);
      break;
    case OUTER_PHASE:
      hipLaunchKernelGGL((k_outer_phase<T2, 0>), dim3((max_slots + 63) / 64), dim3(64), 0, st, slots, nslots_p);
      break;
    case OUTER_COMMIT:
      hipLaunchKernelGGL((k_outer_phase<T2, 1>), dim3((max_slots + 63) / 64), dim3(64), 0, st, slots, nslots_p);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_outer(const SlotDesc<float2>* slots, const int* tile_start, const int* nslots_p, int max_slots,
                        int nrhs, int step, int grid, hipStream_t st) {
  return outer_impl(slots, tile_start, nslots_p, max_slots, nrhs, step, grid, st);
}
hipError_t launch_outer(const SlotDesc<double2>* slots, const int* tile_start, const int* nslots_p, int max_slots,
                        int nrhs, int step, int grid, hipStream_t st) {
  return outer_impl(slots, tile_start, nslots_p, max_slots, nrhs, step, grid, st);
}
hipError_t launch_outer(const SlotDesc<h16c>* slots, const int* tile_start, const int* nslots_p, int max_slots,
                        int nrhs, int step, int grid, hipStream_t st) {
  return outer_impl(slots, tile_start, nslots_p, max_slots, nrhs, step, grid, st);
}

}  // namespace ddml
