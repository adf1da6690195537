/*
 * libddml: domain-decomposed Wilson-clover quark propagators on one MI355X.
 *
 * The method (Ce, Giusti, Schaefer, "Domain decomposition, multi-level
 * integration and exponential noise reduction in lattice QCD"):
 *   - D is the Wilson-Dirac operator of Appendix A (eq. wdo) with bare mass
 *     m0 = 1/(2 kappa) - 4, i.e. 2 kappa D = 1 - kappa D_hop (Section 6), plus,
 *     when c_sw != 0, the Sheikholeslami-Wohlert term
 *     c_sw (i/4) sum_{mu,nu} sigma_{mu nu} Fhat_{mu nu} (the O(a) improvement
 *     named in the footnotes of Sections 4 and 6; the paper gives no formula).
 *   - D_Gamma is D restricted to a hyper-cubic domain Gamma with every term
 *     that touches the exterior boundary set to zero (Section 2, eq. blkdec);
 *     S^(i) = D_Gamma_i^{-1} (eq. diric), zero outside Gamma_i.
 *   - The propagator series S = S^(0) + [S^(1) - S^(0)] + ... (eq. Dseries).
 *   - The disconnected pseudoscalar contraction split into W^(f), W^(r1),
 *     W^(r2) (Section 3, eqs. W0, rall0, rall) and the nucleon contraction
 *     W_N1 - W_N2 (Section 5.2, eq. baryfact) summed over sink time slices
 *     (eq. baryN).
 *   - Stochastic disconnected traces with the hopping parameter expansion
 *     (Section 6, eq. HPEtr).
 *   - The two-domain factorized propagator S^(f) = -D_{Gamma*}^{-1}
 *     D_{dGamma*} D_{Gammabar}^{-1} (Section 5.2, eq. approxlong) and the
 *     connected pion correlator built from it (eqs. pipi, W0pc, decpi,
 *     seriespi), and its projector-cut form with inverse-iteration basis
 *     vectors (eqs. approxlong2, fullfactpi, Bpions).
 *
 * Canonical layouts at this boundary (all complex numbers are interleaved
 * (re, im) doubles):
 *   lattice   dims[4] = {T, L1, L2, L3}; site = ((t*L1 + x1)*L2 + x2)*L3 + x3
 *   links     U[site][mu][3][3], row-major colour, U_mu(x) joins x and x+mu
 *   spinors   psi[rhs][site][spin 4][colour 3]
 *   gamma matrices: chiral basis, gamma_0 = [[0,-1],[-1,0]],
 *             gamma_k = [[0,-i s_k],[i s_k,0]], gamma_5 = diag(1,1,-1,-1)
 *   a point-source propagator holds S(y,x)[alpha a][beta b] in column
 *   rhs = 3*beta + b, i.e. psi[3*beta+b][y][alpha][a].
 * Fermion boundary conditions: periodic in space; periodic, antiperiodic or
 * open in time.  The gauge field is periodic (the clover term of every site is
 * built from all four leaves, also next to an open time boundary).
 *
 * Ownership: the caller owns every buffer it passes.  A buffer flagged
 * on_device=1 is device memory on the context's GPU (e.g. a torch tensor's
 * data_ptr()); on_device=0 means host memory.  The library copies what it
 * keeps (gauge fields) and owns all internal device state.  `stream` is a
 * hipStream_t (may be NULL for the default stream); work is ordered after
 * what is already queued on it.  Calls that return solver information
 * (solve_domain, propagator_series, solve_batch) block until the result is
 * ready; apply_Dw and apply_eo with on_device=1 only enqueue.
 *
 * Errors: every call returns a ddml_status; no exception crosses this
 * boundary.  The message of the most recent failure on a context is returned
 * by ddml_last_error.  Calls on one context are serialised internally.
 */
#ifndef DDML_H
#define DDML_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ddml_ctx_s* ddml_ctx;

typedef enum {
  DDML_OK = 0,
  DDML_EINVAL = -1,          /* invalid argument */
  DDML_ENOMEM = -2,          /* allocation failed or HBM budget exceeded */
  DDML_EAGAIN = -3,          /* result not ready / queue full */
  DDML_ENOTCONVERGED = -4,   /* a right-hand side missed the tolerance; info filled */
  DDML_ENUMERIC = -5,        /* NaN/Inf or a non-invertible clover block */
  DDML_EDEVICE = -6          /* HIP runtime error */
} ddml_status;

typedef enum {
  DDML_BC_PERIODIC = 0,
  DDML_BC_ANTIPERIODIC = 1,  /* a hop across the time boundary picks up -1 */
  DDML_BC_OPEN = 2           /* no hops across the time boundary: the quark field
                                vanishes before t = 0 and after t = T-1, the set-up
                                Sections 2 and 5.2 assume */
} ddml_bc;

typedef enum {
  DDML_FP64 = 0,        /* FP64 throughout (the plain FP64 GPU solver) */
  DDML_MIXED_FP32 = 1,  /* FP32 inner Krylov solve, FP64 defect correction */
  DDML_MIXED_FP16 = 2   /* inner Krylov vectors, links and A^{-1} stored as 16-bit
                           fixed point (one FP32 scale per site and column for
                           spinors, per site for A^{-1}), FP32 arithmetic and FP32
                           solution vector, FP64 defect correction.  Inner solves
                           stop at no less than 3e-4 relative reduction. */
} ddml_prec;

typedef struct {
  int dims[4];   /* T, L1, L2, L3; all even */
  int bc_time;   /* ddml_bc */
} ddml_lattice;

typedef struct {
  double tol;        /* target ||b - D_Gamma x|| / ||b|| per rhs (FP64 true residual) */
  int max_outer;     /* defect-correction cycles */
  int max_inner;     /* inner Krylov iterations per cycle */
  double inner_tol;  /* relative reduction of the inner residual per cycle */
  int prec;          /* ddml_prec */
  int solver;        /* 0 = BiCGstab (van der Vorst 1992) restarted (r0 = r, p = v = 0) at every
                        FP64 correction;
                        1 = BiCGstab with reliable updates: the Krylov state is kept and only
                        the residual is replaced by the FP64 one;
                        2 = GCR(m) (Eisenstat, Elman, Schultz 1983), restarted every gcr_m
                        steps: minimal residual over the cycle's directions, orthogonalised
                        by classical Gram-Schmidt; FP32 or FP64 inner vectors only */
  int gcr_m;         /* GCR restart length, 1..8 (0 = 8); ignored by BiCGstab */
} ddml_solver_params;

typedef struct {
  int status;              /* ddml_status of this rhs */
  int outer_iters;         /* defect-correction cycles used */
  int inner_iters;         /* total BiCGstab iterations */
  double true_rel_residual;/* final ||b - D_Gamma x|| / ||b|| in FP64 */
} ddml_rhs_info;

/* Context on GPU `device`.  hbm_budget_bytes bounds the library's own device
 * allocations (0 = 90% of free memory at creation).  Lattice extents must be
 * even.  Errors: EINVAL (bad lattice), EDEVICE. */
int ddml_create(ddml_ctx* out, const ddml_lattice* lat, int device, size_t hbm_budget_bytes);
int ddml_destroy(ddml_ctx ctx);
/* Message of the last failure on ctx (static empty string if none). */
const char* ddml_last_error(ddml_ctx ctx);

/* Gauge field (Appendix A links; the whole lattice, canonical layout, copied)
 * with the operator parameters kappa and c_sw used with it.  Returns a new
 * gauge id.  Errors: EINVAL, ENOMEM. */
int ddml_set_gauge(ddml_ctx ctx, const double* U, int on_device, double kappa, double csw, int* gauge_id);
/* The same for a field on its own host lattice `lat` (extents even, any size):
 * one context can then serve domains of fields of several sizes.  Sources and
 * solutions of solves with this gauge id are [nrhs][V_lat][4][3]; domain ids
 * are interpreted on this lattice (dom_id -1 = the whole of it).  The
 * contraction entry points work on the context's lattice.  Errors: EINVAL,
 * ENOMEM. */
int ddml_set_gauge_lattice(ddml_ctx ctx, const ddml_lattice* lat, const double* U, int on_device, double kappa,
                           double csw, int* gauge_id);
/* Level-1 update of the two-level integration (Section 3.1): a new gauge id
 * equal to base_gauge_id except on time slices [t0, t1), whose links are
 * U_region[(t - t0)*L1*L2*L3 + ...][mu][3][3].  The base is shared, not
 * copied (a base that is itself such a version with slices outside [t0, t1)
 * is copied once into a whole field).  Errors: EINVAL (bad range or id),
 * ENOMEM. */
int ddml_set_gauge_region(ddml_ctx ctx, int base_gauge_id, int t0, int t1, const double* U_region,
                          int on_device, int* new_gauge_id);
/* Level-1 updates generated on the device (Section 3.1): a new gauge id equal
 * to base_gauge_id except on the slab [t0, t1), whose links are the base's
 * after nsweeps quenched sweeps with the Wilson plaquette action at coupling
 * beta, the spatial links of slice t0 held fixed (they are the frozen
 * boundary shared by neighbouring level-0 regions).  One sweep visits, for
 * mu = 0..3 and parity (x0+x1+x2+x3) mod 2 = 0, 1, every link of that class
 * in the slab once: a Cabibbo-Marinari heatbath over the SU(2) subgroups
 * (0,1), (0,2), (1,2) with the Kennedy-Pendleton sampler, then n_or
 * over-relaxation passes over the same subgroups, then projection onto SU(3)
 * (Gram-Schmidt of rows 0 and 1, row 2 their conjugate cross product).  Links
 * outside the slab enter the staples unchanged; the time direction of the
 * gauge field is periodic.  Random numbers: Philox4x32-10 with key
 * (seed mod 2^32, (seed >> 32) ^ (stream * 0x85EBCA6B mod 2^32)) and counter
 * (lexicographic site, mu | sweep << 2, 0x5EED, n) for the n-th block of four
 * words of that link, each word w giving the uniform (w + 1) / 2^32; a link's
 * draws are taken in the order the update consumes them (the sampler four
 * per try, at most 10001 tries, then two for the direction).  Deterministic
 * for given arguments.  Lattice extents must be even.  Errors: EINVAL (bad
 * range, id or parameters), ENOMEM, EDEVICE. */
int ddml_level1_update(ddml_ctx ctx, int base_gauge_id, int t0, int t1, double beta, uint64_t seed,
                       uint32_t stream, int nsweeps, int n_or, int* new_gauge_id);
/* Copy of the links of gauge id (the whole field of its lattice, region
 * included) into U [V][4][3][3] complex (host or device memory, caller
 * owned).  Synchronous.  Errors: EINVAL, EDEVICE. */
int ddml_get_gauge(ddml_ctx ctx, int gauge_id, double* U, int on_device);
/* Drop a gauge id and the operator data built from it. */
int ddml_release_gauge(ddml_ctx ctx, int gauge_id);

/* Hyper-cubic domain Gamma = [lo, hi) (Section 2), half-open per direction,
 * extents even; it must lie inside the lattice of every gauge field it is
 * used with (checked at use).  A direction with hi-lo equal to the lattice
 * extent keeps its (anti)periodic wrap; otherwise hops across the faces are
 * dropped (Dirichlet, eq. blkdec).  Errors: EINVAL. */
int ddml_set_domain(ddml_ctx ctx, const int lo[4], const int hi[4], int* dom_id);

/* out = D_Gamma in (dom_id = -1: the full lattice), canonical layout,
 * nrhs columns; out is zero outside Gamma (eq. blkdec, Appendix A).
 * prec = DDML_FP64 only.  Errors: EINVAL, ENOMEM, EDEVICE. */
int ddml_apply_Dw(ddml_ctx ctx, int gauge_id, int dom_id, const double* in, double* out, int nrhs,
                  int prec, int on_device, void* stream);

/* The even-odd Schur operator used inside the solver:
 *   out_e = in_e - kappa^2 A_ee^{-1} H_eo A_oo^{-1} H_oe in_e
 * with M = 2 kappa D = A - kappa H, on the sites of Gamma whose local parity
 * (sum_mu (x_mu - lo_mu) mod 2) is even; out is zero on all other sites.
 * prec selects FP64, FP32 or 16-bit storage (inputs rounded to the inner
 * format, output widened; DDML_MIXED_FP16 also stores the intermediate odd
 * field and reads 16-bit links and A^{-1}).  Errors: EINVAL, ENOMEM, EDEVICE. */
int ddml_apply_eo(ddml_ctx ctx, int gauge_id, int dom_id, const double* in, double* out, int nrhs, int prec,
                  int on_device, void* stream);

/* sol = D_Gamma^{-1} src for nrhs columns (eq. diric), zero outside Gamma.
 * Sources are restricted to Gamma first.  info[nrhs] receives per-column
 * status, iteration counts and the FP64 true residual.  Returns
 * ENOTCONVERGED if a column missed params->tol.  Errors: EINVAL, ENOMEM,
 * ENUMERIC, EDEVICE. */
int ddml_solve_domain(ddml_ctx ctx, int gauge_id, int dom_id, const double* src, double* sol, int nrhs,
                      const ddml_solver_params* params, ddml_rhs_info* info, int on_device, void* stream);

/* One solve of a batch. */
typedef struct {
  int gauge_id;
  int dom_id;
  const double* src;   /* [nrhs][V][4][3] */
  double* sol;         /* [nrhs][V][4][3] */
  int nrhs;
  ddml_rhs_info* info; /* [nrhs] */
} ddml_solve_desc;

/* Many independent domain solves of uneven size advanced together: every
 * inner iteration is one set of batched launches over all solves in flight,
 * replayed from a captured HIP graph, and solves join and leave the batch as
 * they converge (admission bounded by the HBM budget).  Same semantics per
 * solve as ddml_solve_domain.  All descs must use the same nrhs. */
int ddml_solve_batch(ddml_ctx ctx, int nsolves, const ddml_solve_desc* descs, const ddml_solver_params* params,
                     int on_device, void* stream);

/* eq. Dseries: solves S^(i) on the nested domains dom_ids[0..nlevels) and
 * writes terms[0] = S^(0), terms[i] = S^(i) - S^(i-1) (each [nrhs][V][4][3],
 * contiguous over i) and sum = S^(nlevels-1).  info is [nlevels][nrhs].
 * Errors as ddml_solve_domain. */
int ddml_propagator_series(ddml_ctx ctx, int gauge_id, const int* dom_ids, int nlevels, const double* src,
                           int nrhs, const ddml_solver_params* params, double* terms, double* sum,
                           ddml_rhs_info* info, int on_device, void* stream);

/* One propagator series of a batch (see ddml_propagator_series). */
typedef struct {
  int gauge_id;
  const int* dom_ids;   /* [nlevels], nested Gamma_0 c Gamma_1 c ... */
  int nlevels;
  const double* src;    /* [nrhs][V][4][3] */
  double* terms;        /* [nlevels][nrhs][V][4][3] */
  double* sum;          /* [nrhs][V][4][3] or NULL */
  ddml_rhs_info* info;  /* [nlevels][nrhs] */
} ddml_series_desc;

/* Several series (e.g. one per level-1 slab update) with all their domain
 * solves advanced in one batch (as ddml_solve_batch).  Same nrhs for all. */
int ddml_propagator_series_batch(ddml_ctx ctx, int nseries, const ddml_series_desc* descs, int nrhs,
                                 const ddml_solver_params* params, int on_device, void* stream);

/* Disconnected pseudoscalar pieces (Section 3, eqs. deco1, W0, rall0, rall)
 * from point-source series around x (terms_x) and y (terms_y), 12 columns
 * each, nlevels levels with the last one the full-lattice propagator.
 * For level i, t_x = tr{g5 S^(i)(x,x)} with S^(i) the partial sum of terms up
 * to i, dt_x = t_x(full) - t_x; by eq. bella the r-kernels are [S - S^(i)](x,x).
 * out[level][4] complex = (f, r1, r2, full) / L^3 with
 * f = t_x t_y, r1 = dt_x t_y + t_x dt_y, r2 = dt_x dt_y, full = f + r1 + r2.
 * Errors: EINVAL, EDEVICE. */
int ddml_contract_pp_disconnected(ddml_ctx ctx, const double* terms_x, const double* terms_y, int nlevels,
                                  const int xsrc[4], const int ysrc[4], double* out, int on_device, void* stream);

/* Nucleon with the projector-cut propagator (Section 5.2, eqs. approxlong2,
 * W0tbary): for orthonormal phi_1..phi_n,
 *   xi_i^T = phi_i^dag D_Gammabar^{-1}, computed as xi_i = conj(g5 D_Gammabar^{-1} g5 phi_i)
 *            (gamma5-hermiticity, eq. g5h),
 *   eta_i  = D_Gamma*^{-1} D_dGamma* phi_i,
 * the colourless spinors B[s_i, s_j, s_k; x]_alpha = eps^{abc} (s_i^a(x)^T C g5
 * s_j^b(x)) s_k^c_alpha(x) (C = i g0 g2) summed over each time slice (one
 * library ZGEMM per slice: diquark colour vectors times spinors), and
 *   out[y0][x0] = (1/L^3) sum_{ijk} (Bx(j,i,k) - Bx(k,i,j))^T P_- By(i,j,k),
 * Bx from xi on slice x0 of Gammabar, By from eta on slice y0 of Gamma*: the
 * nucleon correlator (W_N1 - W_N2 of eq. baryfact, summed over x and y) with
 * every propagator replaced by -sum_i eta_i(y) xi_i(x)^T.  Written out, that
 * substitution gives +P_- between the spinors where eq. W0tbary prints
 * -g5 P_-; the form here is the one equal to eq. baryfact.  With phi spanning
 * the sites D_dGamma* reads it equals the point-source factorized nucleon
 * summed over all sources of each slice.
 *   phi       [nvec][V][4][3]
 *   out       [T][T] complex, host (zero outside the two time ranges)
 *   pion_out  [T][T] real, host, or NULL: the projected pion of
 *             ddml_projected_pion from the same solves
 *   info      [2][nvec]: the Gammabar solves, then the Gamma* solves
 * Memory: two [T][nvec^2][4 nvec] complex blocks.  Errors: EINVAL, ENOMEM,
 * ENOTCONVERGED, EDEVICE. */
int ddml_projected_nucleon(ddml_ctx ctx, int gauge_id, int bar_id, int star_id, const double* phi, int nvec,
                           const ddml_solver_params* params, double* out, double* pion_out, ddml_rhs_info* info,
                           int on_device, void* stream);

/* t[i] = tr{g5 S^(i)(x,x)} (eq. W0, without the 1/L^3) for each level of a
 * 12-column point-source series around x, S^(i) the partial sum of terms up
 * to i: the factors whose level-1 means the two-level estimator multiplies.
 * terms [nlevels][12][V][4][3] complex (as for ddml_contract_pp_disconnected),
 * out[nlevels] complex on the host.  Errors: EINVAL, EDEVICE. */
int ddml_trace_g5(ddml_ctx ctx, const double* terms, int nlevels, const int xsrc[4], double* out, int on_device,
                  void* stream);

/* Two-level estimator (Section 3.1; the bins follow the averaging of the
 * numerical part of Section 6).  n0 level-0 fields; for each, n1 level-1
 * updates of region A and, independently, n1 of region B.  a[n0][n1][nc][ma]
 * are measurements of a factor that depends on A's links only (e.g. the
 * per-slice traces tr{g5 D_Gamma0^{-1}} of eq. W0), b[n0][n1][nc][mb] of B's
 * factor.  For each level-0 field i the level-1 means [a]_i, [b]_i are taken
 * separately and multiplied, contracting c:
 *   P_i[x][y] = sum_c [a]_i[c][x] [b]_i[c][y],
 * est_f[ma][mb] = mean over i of P_i, err_f its standard error over the n0
 * values (0 when n0 = 1).  rest[n0][n1][k] (k >= 0; may be NULL when k = 0):
 * the other pieces (e.g. the r1, r2 parts), averaged in bins of n1 per
 * level-0 field; est_r[k], err_r[k] = mean and standard error of the n0 bin
 * means.  Host memory, caller owned, real values (complex data: real and
 * imaginary parts as separate c or k entries).  No context needed.
 * Errors: EINVAL (sizes < 1, NULL pointers). */
int ddml_two_level_average(int n0, int n1, int nc, int ma, int mb, const double* a, const double* b, int k,
                           const double* rest, double* est_f, double* err_f, double* est_r, double* err_r);

/* Nucleon two-point function (eq. baryfact, eq. baryN) for each level of a
 * 12-column point-source series: levels_out[i][y0] = sum_{y in slice y0}
 * (W_N1 - W_N2)(y, x) with S = S^(i) (partial sums of terms), and
 * diffs_out[i][y0] = levels[i] - levels[i-1] (eq. seriesN), diffs[0] = levels[0].
 * Both are [nlevels][T] complex on the host.  Errors: EINVAL, EDEVICE. */
int ddml_contract_nucleon(ddml_ctx ctx, const double* terms, int nlevels, double* levels_out, double* diffs_out,
                          int on_device, void* stream);

/* Allocation-free variant of ddml_contract_nucleon, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It computes the same two arrays (the sum
 * over each sink slice is taken per workgroup of 8 sites first, so results
 * agree with ddml_contract_nucleon to rounding, not bit for bit) and calls no
 * hipMalloc, hipFree or allocating library routine: its scratch, the
 * per-workgroup partial sums of nlevels x V/8 complex numbers, lives in a
 * static device array of 16 MiB per device, held until the process ends.
 * terms [nlevels][12][V][4][3] complex, levels_out and diffs_out (diffs_out
 * may be NULL) [nlevels][T] complex: all device memory on the context's
 * device, owned by the caller.  Work is queued on `stream` (NULL: the null
 * stream) and not waited for.  Every call on one device shares the scratch
 * array and overwrites it, so calls that overlap on one device (several
 * streams, several contexts or threads) race; order them on one stream.
 * Errors: EINVAL (host pointers, buffers too small, nlevels outside 1..64,
 * nlevels x V / 8 x 16 bytes beyond 16 MiB), EDEVICE. */
int ddml_contract_nucleon_noalloc(ddml_ctx ctx, const double* terms, int nlevels, double* levels_out,
                                  double* diffs_out, void* stream);

/* Boundary block of D (Section 2, eq. blkdec; the off-diagonal block of eq.
 * Scmpt2): out = scale * D_{dGamma} in, where D_{dGamma} holds the entries of
 * D that couple a site y outside the domain Gamma to a site x inside it,
 *   forward  y = x + mu:  -1/2 (1 - gamma_mu) U_mu(x)       in(y)
 *   backward y = x - mu:  -1/2 (1 + gamma_mu) U_mu(x - mu)^dag in(y)
 * with the time-boundary phase of the gauge field's lattice (open: no hop).
 * For a time slab these are -P_- U_0 and -P_+ U_0^dag (eq. fact3 up to the
 * sign and 1/2 of eq. wdo).  out is zero outside Gamma; in is read only
 * outside Gamma.  in/out: [nrhs][V][4][3] complex128 on the gauge field's
 * lattice, nrhs 1..12, not overlapping.  FP64.  Errors: EINVAL (ids, sizes),
 * EDEVICE. */
int ddml_apply_boundary(ddml_ctx ctx, int gauge_id, int dom_id, const double* in, double* out, int nrhs,
                        double scale, int on_device, void* stream);

/* Two-domain factorized propagators (Section 5.2, eq. approxlong) for a
 * sequence of growing overlaps Delta (eq. seriespi):
 *   psi_i = D_{Gammabar_i}^{-1} src,
 *   S^(f)_i src = -D_{Gamma*}^{-1} D_{dGamma*} psi_i,     i = 0 .. nlevels-1,
 * Gammabar_i = bar_ids[i] holds the source, Gamma* = star_id the sinks; with
 * time slabs Gammabar_i = [0, x0cut + Delta_i) and Gamma* = [x0cut, T) the
 * overlap thickness is Delta_i.  When Gammabar is the whole lattice S^(f)(y,x)
 * is the exact propagator for x outside Gamma* and y in Gamma* (eq. Scmpt2).
 * All Gammabar solves run as one batch, then all Gamma* solves as another
 * (as ddml_solve_batch, same params).
 *   src        [nrhs][V][4][3]
 *   levels_out [nlevels][nrhs][V][4][3]: S^(f)_i src, zero outside Gamma*
 *   bar_out    [nlevels][nrhs][V][4][3] or NULL: psi_i, zero outside Gammabar_i
 *   info       [nlevels][2][nrhs]: the Gammabar solve, then the Gamma* solve
 * Errors: EINVAL, ENOMEM, ENOTCONVERGED (info filled), EDEVICE. */
int ddml_factorized_series(ddml_ctx ctx, int gauge_id, const int* bar_ids, int nlevels, int star_id,
                           const double* src, int nrhs, const ddml_solver_params* params, double* levels_out,
                           double* bar_out, ddml_rhs_info* info, int on_device, void* stream);

/* Multi-slab factorized propagator (Section 4, steps 1-3, eqs. stp2, dec1,
 * fctpr): with the lattice cut in thick time slices Lambda_i, a source in
 * Lambda_m and sinks in Lambda_l (l > m),
 *   psi_0 = D_{Omega_{m+2}}^{-1} src,          Omega_{m+2} = Lambda_{m-1..m+1},
 *   psi_k = -D_{Omega*_i}^{-1} D_{Lambda_{i,i-1}} psi_{k-1},
 *           Omega*_i = Lambda_i u Lambda_{i+1}, i = m+k, k = 1 .. l-m,
 * and psi_{l-m} = S^(f) src on Omega*_l, a product in which each factor
 * depends on the links of two or three thick slices only.  dom_ids[0..ndom)
 * name Omega_{m+2}, Omega*_{m+1}, ..., Omega*_l (any domains: each step
 * applies the boundary block of dom_ids[k], the entries of D from outside the
 * domain into it, to psi_{k-1}, as ddml_apply_boundary with scale -1).  The
 * solves run one after the other (each needs the previous one), each over the
 * nrhs columns at once (as ddml_solve_domain, same params).
 *   src       [nrhs][V][4][3]
 *   out       [nrhs][V][4][3]: psi_{ndom-1}, zero outside dom_ids[ndom-1]
 *   steps_out [ndom][nrhs][V][4][3] or NULL: every psi_k
 *   info      [ndom][nrhs]
 * Errors: EINVAL, ENOMEM, ENOTCONVERGED (info filled; later steps still run),
 * EDEVICE. */
int ddml_factorized_chain(ddml_ctx ctx, int gauge_id, const int* dom_ids, int ndom, const double* src, int nrhs,
                          const ddml_solver_params* params, double* out, double* steps_out, ddml_rhs_info* info,
                          int on_device, void* stream);

/* Connected pseudoscalar correlator (eqs. pipi, W0pc):
 *   C(y0) = -(1/L^3) sum_{y in slice y0} tr{S(y,x) S(y,x)^dag}
 * for 12-column point-source propagators (the sum over the source position
 * reduces to the one source point), on the context's lattice.
 *   levels     [nlevels][12][V][4][3]: e.g. S^(f) for growing Delta
 *   full       [12][V][4][3] or NULL: the propagator on the whole lattice
 *   levels_out [nlevels][T] (host, real): C^(i)
 *   diffs_out  [nlevels][T] (host) or NULL: C^(0), C^(i) - C^(i-1) (eq. seriespi)
 *   rest_out   [T] (host) or NULL: C[full] - C^(nlevels-1) (eq. W0pc2); needs full
 * Sums run in a fixed order.  Errors: EINVAL, EDEVICE. */
int ddml_contract_pion(ddml_ctx ctx, const double* levels, int nlevels, const double* full, double* levels_out,
                       double* diffs_out, double* rest_out, int on_device, void* stream);

/* Stochastic estimate of the disconnected trace with the hopping parameter
 * expansion (Section 6, eq. HPEtr and the estimator that follows it), per
 * time slice t of the gauge field's lattice:
 *   out[0][t] = (1/nsrc) sum_i sum_{x in slice t} eta_i^dag(x) [D_Gamma^{-1} gamma5 eta_i](x)
 *   out[1][t] = (1/nsrc) sum_i sum_{x in slice t} eta_i^dag(x) [(kappa D_hop)^p D_Gamma^{-1} gamma5 eta_i](x)
 * with kappa D_hop = 1 - 2 kappa D_Gamma (the clover term sits in its site
 * diagonal).  Both estimate sum_x tr{gamma5 D_Gamma^{-1}(x,x)}; the second has
 * the smaller variance.  p: 0..8 without the clover term, 0..2 with it (the
 * range in which the expansion's lower orders have zero trace); else EINVAL.
 *   eta      [nsrc][V][4][3] sources (e.g. Gaussian noise; unit vectors give
 *            the exact trace); only their part on Gamma enters the solves
 *   out      [2][T] complex, host
 *   psi_out  [nsrc][V][4][3] or NULL: D_Gamma^{-1} gamma5 eta
 *   phi_out  [nsrc][V][4][3] or NULL: (kappa D_hop)^p D_Gamma^{-1} gamma5 eta
 *   info     [nsrc]: the solve of each source (12 sources per solve, the
 *            solves batched as ddml_solve_batch)
 * Errors: EINVAL, ENOMEM, ENOTCONVERGED (out still written), EDEVICE. */
int ddml_hpe_trace(ddml_ctx ctx, int gauge_id, int dom_id, const double* eta, int nsrc, int p,
                   const ddml_solver_params* params, double* out, double* psi_out, double* phi_out,
                   ddml_rhs_info* info, int on_device, void* stream);

/* Basis vectors of the projector-cut factorization (Section 5.2, after eq.
 * approxlong2): nvec vectors on the domain Omega (dom_id) from niter inverse
 * iterations of D_Omega, each followed by orthonormalisation:
 *   v <- Q,  D_Omega^{-1} v = Q R  (Q^dag Q = 1, R upper triangular with
 *                                   positive real diagonal: Cholesky QR, twice)
 * starting from `start`.  The orthonormalisation runs over the time slices of
 * Omega (a time slab in the paper's use).  The solves take 12 vectors at a
 * time, batched.
 *   start, out [nvec][V][4][3] (not overlapping); out holds the last Q
 *   info [nvec]: the solves of the last iteration
 * nvec 1..1024, niter >= 1.  Errors: EINVAL, ENOMEM, ENOTCONVERGED,
 * ENUMERIC (dependent vectors), EDEVICE. */
int ddml_inverse_iteration(ddml_ctx ctx, int gauge_id, int dom_id, const double* start, int nvec, int niter,
                           const ddml_solver_params* params, double* out, ddml_rhs_info* info, int on_device,
                           void* stream);

/* Connected pion with the projector-cut propagator (Section 5.2, eqs.
 * approxlong2, fullfactpi, Bpions): for orthonormal phi_1..phi_n,
 *   chi_j = D_Gammabar^{-1} gamma5 phi_j,   eta_j = D_Gamma*^{-1} D_dGamma* phi_j,
 *   G(x0)_ij  = sum_{x in slice x0} chi_i(x)^dag chi_j(x)     (= B_ij summed over the slice),
 *   Gt(y0)_ij = sum_{y in slice y0} eta_i(y)^dag eta_j(y)    (= Btilde_ij; by gamma5-hermiticity
 *               phi_i^dag gamma5 D_d D^{-1} gamma5 is eta_i^dag),
 *   out[y0][x0] = -(1/L^3) Re Tr(Gt(y0) G(x0))   (sums over both x and y of eq. pipi)
 * for y0 in the time range of Gamma* and x0 in that of Gammabar, zero
 * elsewhere.  With phi spanning the sites D_dGamma* reads, the projector is
 * exact there and out equals the factorized correlator summed over all
 * sources.  The Gram matrices are library GEMMs (rocBLAS).
 *   phi        [nvec][V][4][3]
 *   out        [T][T] real, host
 *   gram_bar, gram_star  [T][nvec][nvec] complex column-major, host, or NULL
 *   info       [2][nvec]: the Gammabar solves, then the Gamma* solves
 * Errors: EINVAL, ENOMEM, ENOTCONVERGED, EDEVICE. */
int ddml_projected_pion(ddml_ctx ctx, int gauge_id, int bar_id, int star_id, const double* phi, int nvec,
                        const ddml_solver_params* params, double* out, double* gram_bar, double* gram_star,
                        ddml_rhs_info* info, int on_device, void* stream);

/* Measurement hook for the dominant kernels: times `iters` back-to-back
 * applications of the two half-stencils of the even-odd Schur operator, as
 * launched by the batched solver (links + A^{-1} + fused dot product), on the
 * library stream with HIP events, after 3 untimed warm-up pairs.  out[0],
 * out[1]: average milliseconds per launch of the odd half (out_o = A_oo^{-1}
 * H_oe in_e) and of the even half (out_e = in_e - kappa^2 A_ee^{-1} H_eo t_o
 * with the dot product (h, out_e), h the solver's hashed shadow vector);
 * out[2], out[3]: algorithmic bytes of one
 * launch of each (every array the kernel must touch, counted once).
 * prec: DDML_FP64, DDML_MIXED_FP32 or DDML_MIXED_FP16 (16-bit storage, stage 1
 * only; bytes then count 2 per real plus the scales).  R (columns per thread,
 * 1..3), order, grid (workgroups), splits and stage select the launch; values
 * <= 0 (order, stage: < 0) take the context's current choice.  Tile orders: 0 linear;
 * 1 each of the 8 XCDs owns a band of every time slice and walks the slices in
 * turn; 2 and 3: each XCD owns an x1 range of the domain, split by x2 into 2
 * (order 2) or 4 (order 3) sub-bands, each walked slice by slice; 4: the
 * sub-bands of order 3 walked in blocks of 4 slices, the slices of a block
 * innermost; 5: each XCD owns half of the x1 rows and a quarter of the tiles
 * of each (x2, x3) plane, cut along x1 into 4 sub-bands walked as in order 4
 * (orders 2..5 fall back to order 1 on boxes that do not split so).  splits: the
 * ceil(nrhs / R) wavefronts that cover the columns of a 64-site tile are spread
 * over this many workgroups (1 = one workgroup per tile; clamped to the number
 * of wavefronts).  stage: 1 = each workgroup first copies the links and
 * clover data of its tile to LDS, so they are read once per tile instead of
 * once per wavefront; 0 = every wavefront reads them itself (FP64 only: the
 * FP32 and 16-bit copies keep two rows per link, rebuilt in the staging).
 * Errors: EINVAL, ENOMEM. */
int ddml_time_stencil(ddml_ctx ctx, int gauge_id, int dom_id, int nrhs, int prec, int iters, int R, int order,
                      int grid, int splits, int stage, double out[4]);

/* Autotuner: times the stencil launch variants (stage 0/1 in FP64, 1 otherwise;
 * R in 1..3, splits in 1..3, tile orders 0..5, grid in {512, 1024, 2048}) on (gauge_id, dom_id,
 * nrhs, prec) and makes the fastest the context's choice for every later solve
 * (the captured solver graphs are rebuilt).  best[0..5] = R, order, grid,
 * splits, stage, ms per odd+even pair.
 * Errors: EINVAL (also while the request loop runs), ENOMEM, EDEVICE. */
int ddml_autotune(ddml_ctx ctx, int gauge_id, int dom_id, int nrhs, int prec, double best[6]);

/* Sets the stencil launch of precision prec by hand (same meaning as the
 * arguments of ddml_time_stencil; grid >= 8; 16-bit storage needs stage 1).
 * Every launch choice computes the same bits.
 * Errors: EINVAL (also while the request loop runs). */
int ddml_set_launch(ddml_ctx ctx, int prec, int R, int order, int grid, int splits, int stage);

/* ------------------------------------------------------------- serving */
typedef struct {
  int gauge_id;
  int dom_id;
  const double* src;    /* device pointer [nrhs][V][4][3], must stay valid until completion */
  double* sol;          /* device pointer, written on completion */
  int nrhs;
  double arrival_time;  /* caller's clock (seconds), used for latency */
} ddml_request;

typedef struct {
  int status;             /* ddml_status of the request */
  int max_outer, max_inner_iters;
  double worst_rel_residual;
  double arrival_time, admit_time, finish_time;  /* same clock as arrival_time */
} ddml_result;

typedef struct {
  long submitted, completed, queued, in_flight;
  double p50_latency, p99_latency, mean_latency;  /* seconds, over completed requests */
  double solves_per_s;                            /* completed / (last finish - first arrival) */
  size_t hbm_in_use, hbm_budget;
} ddml_server_stats;

/* Start the request loop on its own host thread.  Requests are admitted as
 * their HBM footprint fits the budget and join the running batch (continuous
 * batching); params applies to every request.  max_queue bounds pending
 * requests (submit returns EAGAIN beyond it). */
int ddml_server_start(ddml_ctx ctx, const ddml_solver_params* params, int max_queue);
/* Queue one request.  src and sol must be device memory on the context's
 * device: host pointers return EINVAL here, before anything is queued; a
 * request whose buffers do not hold nrhs canonical fields of its gauge field's
 * lattice inside one device allocation finishes with status EINVAL at
 * admission, before any kernel touches them. */
int ddml_submit(ddml_ctx ctx, const ddml_request* req, uint64_t* ticket);
/* A propagator series as one request (eq. Dseries, as ddml_propagator_series):
 * one domain solve per nested domain, admitted level by level as they fit;
 * when the last one has finished, terms[0] = S^(0), terms[i] = S^(i) -
 * S^(i-1) and sum = S^(nlevels-1).  The result aggregates every level and
 * column; info, if not NULL, receives the per-level, per-column details
 * before the request completes. */
typedef struct {
  int gauge_id;
  const int* dom_ids;   /* [nlevels], nested; copied at submit */
  int nlevels;          /* 1..64 */
  const double* src;    /* device [nrhs][V][4][3], valid until completion */
  double* terms;        /* device [nlevels][nrhs][V][4][3], written on completion */
  double* sum;          /* device [nrhs][V][4][3] or NULL */
  int nrhs;
  double arrival_time;  /* caller's clock (seconds), used for latency */
  ddml_rhs_info* info;  /* host [nlevels][nrhs] or NULL */
} ddml_series_request;

/* Queue one series request.  Pointers as ddml_submit (host memory: EINVAL
 * here; extents and domains are checked at admission, where a failure ends
 * the request with EINVAL before any kernel touches its buffers). */
int ddml_submit_series(ddml_ctx ctx, const ddml_series_request* req, uint64_t* ticket);
/* EAGAIN while pending; DDML_OK and *res once finished (the result is kept). */
int ddml_poll(ddml_ctx ctx, uint64_t ticket, ddml_result* res);
int ddml_wait(ddml_ctx ctx, uint64_t ticket, ddml_result* res, double timeout_s);
int ddml_stats(ddml_ctx ctx, ddml_server_stats* stats);
int ddml_server_stop(ddml_ctx ctx);

/* Seconds on the library's monotonic clock (the serving loop's clock). */
double ddml_now(void);

#ifdef __cplusplus
}
#endif
#endif
