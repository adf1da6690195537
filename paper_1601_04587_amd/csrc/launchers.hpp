// Host-callable launchers for the device kernels of libddml.
#pragma once
#include "ddml_common.hpp"

namespace ddml {

// dirac.hip
hipError_t launch_hop_item(const HopItem<double2>& it, int mode, int red, int R, int order, hipStream_t st);
// xstart: [kXcd][xstride] per-XCD prefix of tile counts (all orders but linear);
// splits: the waves covering the columns of a tile are spread over this many
// workgroups (1 = one workgroup per tile); stage: 1 = stage each tile's links
// and clover data in LDS once per workgroup
hipError_t launch_hop_batch(const SlotDesc<float2>* slots, const int* tile_start, const int* xstart, int xstride,
                            const int* nslots_p, int nrhs, int R, int mode, int red, int fin, int faux, int fout,
                            int fred, int par_out, int grid, int order, int splits, int stage, hipStream_t st);
hipError_t launch_hop_batch(const SlotDesc<double2>* slots, const int* tile_start, const int* xstart, int xstride,
                            const int* nslots_p, int nrhs, int R, int mode, int red, int fin, int faux, int fout,
                            int fred, int par_out, int grid, int order, int splits, int stage, hipStream_t st);
hipError_t launch_hop_batch(const SlotDesc<h16c>* slots, const int* tile_start, const int* xstart, int xstride,
                            const int* nslots_p, int nrhs, int R, int mode, int red, int fin, int faux, int fout,
                            int fred, int par_out, int grid, int order, int splits, int stage, hipStream_t st);
// host mirror of the banded order: tiles of a box (ntiles, tps) owned by XCD x
inline int band_count(int ntiles, int tps, int x) {
  const int S = tps > 0 ? tps : ntiles;
  const int lo = (int)((long)x * S / kXcd), hi = (int)((long)(x + 1) * S / kXcd);
  return (hi - lo) * (ntiles / S);
}
hipError_t launch_clover_apply(const BoxGeom& g, const double2* clov, int p, const double2* in, double2* out,
                               int nrhs, hipStream_t st);

// blas.hip: inner BiCGstab steps over a slot table
// BiCGstab vector steps (k_vec) and scalar steps (k_fin), h the hashed shadow vector:
//   VEC_S     s = r - alpha v;                                     slot 3: (h, s)
//   VEC_XRP   x += alpha p + omega s; r = s - omega t;
//             p = r + beta (p - omega v);                          slot 1: |r|^2
//   VEC_INIT  r = p = b, x = 0;                                    slot 0: (h, r), slot 1: |r|^2
//   VEC_RELUP r = b, x = 0; p = r (fresh column) or p - r_old;     slot 0: (h, r), slot 1: |r|^2
//   VEC_PFIX  p = r + beta p
//   FIN_ALPHA alpha = rho / (h, v)
//   FIN_OMEGA omega = (t, s) / |t|^2; rho' = (h, s) - omega (h, t); beta = (rho'/rho)(alpha/omega)
//   FIN_CHECK stopping test on |r|^2
enum { VEC_S = 1, VEC_XRP = 2, VEC_INIT = 3, VEC_RELUP = 4, VEC_PFIX = 5 };
enum { FIN_INIT = 0, FIN_ALPHA = 1, FIN_OMEGA = 2, FIN_CHECK = 3, FIN_RELUP = 4 };
hipError_t launch_vec(const SlotDesc<float2>* slots, const int* tile_start, const int* nslots_p, int nrhs, int op,
                      int grid, hipStream_t st);
hipError_t launch_vec(const SlotDesc<double2>* slots, const int* tile_start, const int* nslots_p, int nrhs, int op,
                      int grid, hipStream_t st);
hipError_t launch_fin(const SlotDesc<float2>* slots, const int* nslots_p, int max_slots, int op, hipStream_t st);
hipError_t launch_fin(const SlotDesc<double2>* slots, const int* nslots_p, int max_slots, int op, hipStream_t st);
hipError_t launch_vec(const SlotDesc<h16c>* slots, const int* tile_start, const int* nslots_p, int nrhs, int op,
                      int grid, hipStream_t st);
// GCR(m) steps (k = step inside the cycle)
enum { GCR_INIT = 0, GCR_DOTS = 1, GCR_UPDATE = 2, GCR_XR = 3 };
enum { GFIN_INIT = 0, GFIN_BETA = 1, GFIN_ALPHA = 2, GFIN_CHECK = 3 };
hipError_t launch_gcr(const SlotDesc<float2>* slots, const int* tile_start, const int* nslots_p, int nrhs, int op,
                      int k, int m, int grid, hipStream_t st);
hipError_t launch_gcr(const SlotDesc<double2>* slots, const int* tile_start, const int* nslots_p, int nrhs, int op,
                      int k, int m, int grid, hipStream_t st);
hipError_t launch_gcr_fin(const SlotDesc<float2>* slots, const int* nslots_p, int max_slots, int op, int k,
                          hipStream_t st);
hipError_t launch_gcr_fin(const SlotDesc<double2>* slots, const int* nslots_p, int max_slots, int op, int k,
                          hipStream_t st);
hipError_t launch_fin(const SlotDesc<h16c>* slots, const int* nslots_p, int max_slots, int op, hipStream_t st);
// Steps of the device-side outer loop (outer.hip), over the whole slot table.
enum { OUTER_GATE = 0, OUTER_CAST = 1, OUTER_AXPY = 2, OUTER_CLOVER = 3, OUTER_DECIDE = 4, OUTER_PHASE = 5,
       OUTER_COMMIT = 6 };
hipError_t launch_outer(const SlotDesc<float2>* slots, const int* tile_start, const int* nslots_p, int max_slots,
                        int nrhs, int step, int grid, hipStream_t st);
hipError_t launch_outer(const SlotDesc<double2>* slots, const int* tile_start, const int* nslots_p, int max_slots,
                        int nrhs, int step, int grid, hipStream_t st);
// Clears n consecutive slots of the device loop (phase, outer state, column
// and step flags; each slot holds kMaxRhs columns and 3 kMaxRhs flags).
hipError_t launch_outer_reset(SlotState* sst, OuterState* ost, int* act, int* oflag, int n, int phase,
                              hipStream_t st);
hipError_t launch_outer(const SlotDesc<h16c>* slots, const int* tile_start, const int* nslots_p, int max_slots,
                        int nrhs, int step, int grid, hipStream_t st);

// elementwise helpers on raw FP64 / mixed arrays (n complex numbers)
hipError_t launch_cast_to_d(const float2* in, double2* out, size_t n, hipStream_t st);
hipError_t launch_cast_to_d(const double2* in, double2* out, size_t n, hipStream_t st);
hipError_t launch_cast_to_f(const double2* in, float2* out, size_t n, hipStream_t st);
hipError_t launch_fill(float2* v, size_t n, double a, hipStream_t st);
hipError_t launch_fill(double2* v, size_t n, double a, hipStream_t st);
hipError_t launch_axpy_d(double2* y, const double2* x, double a, size_t n, hipStream_t st);
// 16-bit fields: values [nrhs][ntiles][12][64] with scales [nrhs][ntiles * 64]
hipError_t launch_fill16(h16c* v, size_t n, float* nrm, size_t nn, double a, hipStream_t st);
hipError_t launch_quant16(const double2* in, h16c* out, float* nrm, int nrhs, int ntiles, hipStream_t st);
hipError_t launch_dequant16(const h16c* in, const float* nrm, double2* out, int nrhs, int ntiles, hipStream_t st);
// column norms |v_col|^2 of a [nrhs][ntiles][12][64] field into out[nrhs].x (accumulate=1 adds)
hipError_t launch_col_norms(const double2* v, int Vh, int nrhs, double2* partial, int ntiles, double2* out,
                            int accumulate, hipStream_t st);
// sum partial[k][col][tile] over tiles into out[k*nrhs + col] (accumulate=1 adds)
hipError_t launch_sum_partials(const double2* partial, int nred, int nrhs, int ntiles, double2* out,
                               int accumulate, hipStream_t st);

// gauge.hip: operator blocks
struct GaugeView {
  const double2* base;    // [V][4][9] canonical FP64 links of the whole lattice
  const double2* region;  // [V_region][4][9] override for time slices [r_t0, r_t1), may be null
  int r_t0, r_t1;
};
struct BlockSpec {
  int L[4];       // lattice
  int lo[4];      // domain origin
  int Lb[4];      // domain extents (even)
  int tbc;        // time boundary of the lattice: 0 periodic, 1 antiperiodic, 2 open
  double kappa, csw;
};
// FP64 links (5-pair layout) and the two-row FP32 copy; bit 2 of *bad if a link is not SU(3)
hipError_t launch_build_links(const GaugeView& gv, const BlockSpec& bs, double2* U64, float2* U32, int* bad,
                              hipStream_t st);
hipError_t launch_build_clover(const GaugeView& gv, const BlockSpec& bs, double2* A64, double2* Ainv64,
                               float2* Ainv32, int* bad, hipStream_t st);
// 16-bit copies of an operator block's links (from the two-row FP32 copy, n complex
// numbers) and A^{-1} (2 * ntiles * 64 sites)
hipError_t launch_quant_links(const float2* U32, h16c* U16, size_t n, hipStream_t st);
hipError_t launch_quant_clover(const double2* Ainv64, h16c* Ainv16, float* nrm, int ntiles, hipStream_t st);
// canonical [nrhs][V][12] complex128 <-> domain EO field [nrhs][ntiles][12][64] of parity p, scaled
hipError_t launch_gather(const double2* canon, const BlockSpec& bs, int p, int nrhs, double scale, double2* eo,
                         hipStream_t st);
hipError_t launch_scatter(const double2* eo, const BlockSpec& bs, int p, int nrhs, double scale, double2* canon,
                          hipStream_t st);
// level-1 updates of the region [gv.r_t0, gv.r_t1) of a gauge version (bs.L the lattice)
hipError_t launch_level1_sweeps(const GaugeView& gv, double2* region, const BlockSpec& bs, double beta,
                                uint64_t seed, uint32_t stream, int nsweeps, int n_or, hipStream_t st);
// out = scale * D_{dGamma} in on canonical [nrhs][V][12] fields, Gamma = [bs.lo, bs.lo + bs.Lb)
hipError_t launch_boundary(const GaugeView& gv, const BlockSpec& bs, const double2* in, double2* out, int nrhs,
                           double scale, hipStream_t st);

// contract.hip
hipError_t launch_series_diff(double2* terms, size_t n, int nlevels, double2* sum, hipStream_t st, int ncol = 0,
                              size_t cstride = 0, size_t lo = 0, size_t len = 0);
// out[i] = tr{g5 S^(i)(x,x)}, S^(i) the partial sums of a 12-column series (nlevels <= 64)
hipError_t launch_g5_traces(const double2* terms, size_t V, int nlevels, size_t xs, double2* out, hipStream_t st);
hipError_t launch_pp(const double2* tx, const double2* ty, size_t V, int nlevels, size_t xs, size_t ys, double invL3,
                     double2* out, hipStream_t st);
// connected pion: W scratch [nprops][V]; sums [nprops][T] of tr{S S^dag} per time slice
hipError_t launch_pion(const double2* props, size_t V, int T, int nprops, double2* W, double2* sums, hipStream_t st);
// C^(i) = -sums[i] / L^3, the series differences and (has_full: sums[nlevels] is the full
// propagator's) the rest; out: [2 * nlevels + 1][T] = levels, diffs, rest
hipError_t launch_pion_fin(const double2* sums, int nlevels, int T, int has_full, double invL3, double* out,
                           hipStream_t st);
// gamma5 on nsites canonical spinors; noise trace: W scratch [V], sums [T] of
// sum_i eta_i^dag(x) phi_i(x) over the sites of each time slice
hipError_t launch_gamma5(const double2* in, double2* out, size_t nsites, hipStream_t st);
hipError_t launch_noise_trace(const double2* eta, const double2* phi, int nsrc, size_t V, int T, double2* W,
                              double2* sums, hipStream_t st);
// linalg.hip: G (column-major n x n) -> upper Cholesky factor R, G = R^dag R
hipError_t launch_cholesky_upper(double2* G, int n, int* bad, hipStream_t st);
// out[y * T + x] = scale * Re Tr(Gt[y] G[x]) for y in [ya, yb), x in [xa, xb)
// C[s] = (accumulate ? C[s] : 0) + sum_q P[s Q + q]: reduction of a GEMM split along its inner dimension
hipError_t launch_sum_chunks(const double2* P, int Q, int m, int n, int nslices, double2* C, int ldc, size_t sC,
                             int accumulate, hipStream_t st);
// colourless spinors (eq. W0tbary): diquark colour vectors E [N^2][ns][3] and spinors S [N][4][ns][3]
// of the sites [site0, site0 + ns) of X [N][V][4][3] (xi = 1: of conj(g5 X)); then
// out[y T + x] = scale * sum (Bx(j,i,k) - Bx(k,i,j))^T P_- By(i,j,k) for slice pairs
hipError_t launch_bary_layout(const double2* X, size_t V, int N, size_t site0, int ns, int xi, double2* E,
                              double2* S, hipStream_t st);
hipError_t launch_bary_pairs(const double2* By, const double2* Bx, int N, int T, int ya, int yb, int xa, int xb,
                             double scale, double2* out, hipStream_t st);
hipError_t launch_trace_pairs(const double2* Gt, const double2* G, int n, int T, int ya, int yb, int xa, int xb,
                              double scale, double* out, hipStream_t st);
// W: scratch [nlevels][V]; out: [nlevels][T]
hipError_t launch_nucleon(const double2* terms, size_t V, int T, int nlevels, double2* W, double2* out,
                          hipStream_t st);
// Allocation-free nucleon contraction (the scratch is a static device array
// of kNucScratchBytes per device): levels [nlevels][T] and, if not null,
// diffs [nlevels][T], device pointers, stream-ordered on st.
// nucleon_scratch_init resolves the array's address on `device`, which must
// be current; once per device, before the first launch there.
constexpr size_t kNucScratchBytes = (size_t)16 << 20;
constexpr int kMaxDevices = 64;
hipError_t nucleon_scratch_init(int device);
hipError_t launch_nucleon_noalloc(const double2* terms, size_t V, int T, int nlevels, double2* levels,
                                  double2* diffs, int device, hipStream_t st);

}  // namespace ddml
