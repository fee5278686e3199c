/*
 * dwf.h -- C ABI of libdwf: the red-black (Schur) preconditioned Shamir
 * domain-wall operator and the solver / filter built on it, for AMD gfx950.
 *
 * The operators are those of the paper's "Chiral Fermion Actions" section:
 *   D_hop   = sum_mu (1 - g_mu) U_mu(x) d_{x+mu,y} + (1 + g_mu) U_mu(x-mu)^dag d_{x-mu,y}
 *   D_DW    = the Ls x Ls block matrix with D_par = 5 - M5 - D_hop/2 on the
 *             diagonal, -P_- above, -P_+ below, m P_+ / m P_- in the corners
 *   M5D     = D_DW with D_hop removed (= M_ee = M_oo, local in the 4D site)
 *   M_pc    = M_ee - M_eo M_oo^{-1} M_oe = M5D - D_hop^{eo} M5D^{-1} D_hop^{oe} / 4
 *             (first Schur form; the red-black CGNR of the Results section)
 * and the setup filter of the "Deflation basis setup" section.
 *
 * Conventions.  Chiral gamma basis, gamma5 = diag(1,1,-1,-1), P_+- = (1 +- gamma5)/2.
 * Lattice extents dims = {X, Y, Z, T}, all even; periodic 4D boundaries;
 * parity = (x+y+z+t) mod 2, even = 0.  V4 = X*Y*Z*T, V4h = V4/2.
 *
 * Layouts (all device memory, owned by the caller):
 *  - natural gauge field  U[T][Z][Y][X][mu][a][b], complex128 (re, im interleaved);
 *  - natural 5D fermion   psi[rhs][Ls][T][Z][Y][X][spin][colour], complex128;
 *  - packed half field (one parity) per right-hand side, site index
 *    h = (x + X*(y + Y*(z + Z*t))) / 2, spin-colour index c = 3*spin + colour,
 *    slice s; right-hand sides are consecutive blocks:
 *      DWF_F64 : [V4h][12][Ls] complex128, 192 * Ls * V4h bytes per rhs
 *      DWF_F32 : [V4h][6][Ls][2] complex64 (c = 2j + k), 96 * Ls * V4h bytes per rhs
 *      DWF_F16S: [V4h][12][Ls] pairs of IEEE halves (value times the FP32
 *                reciprocal of the scale, round to nearest even) followed by [V4h][Ls] float scales
 *                = max |v| over the 24 reals of the spinor; 52 * Ls * V4h bytes per rhs
 *  - packed "both parities" field: the even half field of all rhs, then the odd.
 *
 * Every call that takes device pointers is asynchronous on the handle's stream
 * unless marked synchronous.  Calls return DWF_OK or a negative status; the
 * message of the last failure on the calling thread is dwf_last_error().
 * No exception crosses the ABI.  A handle must not be used from two host
 * threads at once.
 */
#ifndef DWF_H
#define DWF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dwf_context* dwf_handle;

enum dwf_status {
  DWF_OK = 0,
  DWF_EINVAL = -1,      /* bad argument: odd extent, Ls < 1, null pointer, nrhs out of range */
  DWF_ENOMEM = -2,      /* workspace smaller than dwf_workspace_bytes() */
  DWF_EHIP = -3,        /* a HIP runtime call failed (message holds its text) */
  DWF_ENOCONV = -4,     /* maxiter reached; x holds the last iterate */
  DWF_EBREAKDOWN = -5,  /* non-finite or non-positive curvature in CG (e.g. NaN source) */
  DWF_WLAMBDA = 1       /* warning: filter upper bound below the measured lambda_max */
};

enum dwf_precision { DWF_F64 = 0, DWF_F32 = 1, DWF_F16S = 2 };
enum dwf_parity { DWF_EVEN = 0, DWF_ODD = 1, DWF_BOTH = 2 };

/* ---- set-up -------------------------------------------------------------- */

/* Library plumbing (no passage of the paper defines this call).
 * Bytes of device workspace a handle needs (host only, no GPU call).  prec is
 * the storage precision of the handle's fields; max_nrhs is the number of
 * right-hand sides the operator temporaries hold at once (operator and filter
 * calls with more are processed in chunks of max_nrhs); max_cg_rhs bounds the
 * nrhs of dwf_cg and enables dwf_solve_rb / dwf_force (0 = no solver
 * workspace).  Returns 0 on invalid arguments. */
size_t dwf_workspace_bytes(const int dims[4], int Ls, int prec, int max_nrhs, int max_cg_rhs);

/* Library plumbing (no passage of the paper defines this call).
 * Bytes of one packed half field of nrhs right-hand sides at precision prec
 * (host only). */
size_t dwf_field_bytes(const int dims[4], int Ls, int prec, int nrhs);

/* Create a handle for the operators of the Chiral Fermion Actions section
 * (M5 and mf as in the D_DW matrix there): validates the arguments, carves
 * the caller's workspace (device memory of at least dwf_workspace_bytes bytes, kept alive by the
 * caller until dwf_destroy, 256-byte aligned), packs the links U (natural
 * layout, device) into it and builds the neighbour tables, on `stream` (a
 * hipStream_t; NULL is the null stream).  M5 is the domain-wall height
 * (M5 != 5), mf the quark mass of the corner terms.  Extents must be even and
 * >= 2, 1 <= Ls <= 128. */
int dwf_create(dwf_handle* h, const void* U, const int dims[4], int Ls, double M5, double mf,
               int prec, int max_nrhs, int max_cg_rhs, void* workspace, size_t ws_bytes,
               void* stream);

/* Re-pack new links (same lattice), e.g. after an HMC update of the
 * Conclusions section's sampling. */
int dwf_update_links(dwf_handle h, const void* U);

/* Library plumbing (no passage of the paper defines this call).
 * Change the stream later calls are queued on. */
int dwf_set_stream(dwf_handle h, void* stream);

/* Library plumbing (no passage of the paper defines this call).
 * Free the host-side handle; does not free the caller's workspace. */
int dwf_destroy(dwf_handle h);

/* Library plumbing (no passage of the paper defines this call).
 * Thread-local text of the last failure (never NULL). */
const char* dwf_last_error(void);

/* Natural complex128 <-> packed (handle precision).  parity selects which
 * sites are moved (the even / odd checkerboard of the red-black
 * preconditioning, Conventional Krylov Solvers section); unpack writes only
 * the sites of that parity. */
int dwf_pack(dwf_handle h, const void* natural, void* packed, int nrhs, int parity);
int dwf_unpack(dwf_handle h, const void* packed, void* natural, int nrhs, int parity);

/* ---- operators (handle precision, packed layout) -------------------------- */

/* out = D_hop in (dagger = 0) or D_hop^dag in (dagger = 1) on every slice s,
 * from the other parity into out_parity (Chiral Fermion Actions section, the
 * D_hop equation). */
int dwf_dhop(dwf_handle h, const void* in, void* out, int out_parity, int nrhs, int dagger);

/* out = M5D in or M5D^dag in, and the exact inverses (site-local, one
 * parity): the D_DW matrix of the Chiral Fermion Actions section without its
 * D_hop part, i.e. the diagonal Schur blocks M_ee = M_oo. */
int dwf_m5d(dwf_handle h, const void* in, void* out, int nrhs, int dagger);
int dwf_m5d_inv(dwf_handle h, const void* in, void* out, int nrhs, int dagger);

/* Full D_DW (or D_DW^dag) on both parities (packed "both" layout), the
 * matrix of the Chiral Fermion Actions section. */
int dwf_ddw(dwf_handle h, const void* in, void* out, int nrhs, int dagger);

/* out_e = M_pc in_e (dagger = 0) or M_pc^dag in_e (dagger = 1), the Schur
 * form of the Algorithms section (Algorithm G's table) used by the red-black
 * CGNR of the Conventional Krylov Solvers section: two passes,
 * t_o = M5D^{-1} D_hop^{oe} in_e then out_e = M5D in_e - D_hop^{eo} t_o / 4. */
int dwf_mpc(dwf_handle h, const void* in_e, void* out_e, int nrhs, int dagger);

/* out_e = M_pc^dag M_pc in_e, the normal operator of the CGNR of the
 * Spectrum of domain wall fermions section: four passes. */
int dwf_mpcdagmpc(dwf_handle h, const void* in_e, void* out_e, int nrhs);

/* ---- solver, filter, orthonormalisation ----------------------------------- */

/* SYNCHRONOUS.  Solve M_pc^dag M_pc x = b for nrhs right-hand sides by CG
 * (Hestenes-Stiefel): the CGNR on the normal operator of the Spectrum of
 * domain wall fermions section, the red-black CGNR of the Conventional
 * Krylov Solvers section; the low-precision handles give the mixed-precision
 * variant that the Results section mentions without specifying it.  b and x are FP64 packed even fields whatever the
 * handle precision; x holds the initial guess on entry.  With a DWF_F64
 * handle every step is FP64; with DWF_F32 / DWF_F16S the iteration runs on
 * low-precision fields with FP64 dot products and FP64 reliable updates
 * r = b - A x whenever |r| falls below a tenth of its largest value since
 * the last update, after which p is re-orthogonalised against the new r.
 * Stops when every ||r|| / ||b|| < tol; iters[nrhs] and true_rel_resid[nrhs]
 * are host arrays (either may be NULL) receiving iterations and
 * ||b - A x|| / ||b|| in FP64.  Returns DWF_ENOCONV after maxiter, or early
 * when a low-precision solve stagnates (the true ||r|| has not halved over
 * 12 consecutive reliable updates for every active rhs: the low-precision
 * operator is too coarse for the conditioning), DWF_EBREAKDOWN on NaN. */
int dwf_cg(dwf_handle h, const void* b, void* x, int nrhs, double tol, int maxiter, int* iters,
           double* true_rel_resid);

/* Library plumbing (no passage of the paper defines this call).
 * Progress of the synchronous solvers (dwf_cg, dwf_solve_rb): fn is called on
 * the calling thread after iteration `iteration` with the recursive
 * ||r|| / ||b|| of each of the nrhs right-hand sides (a host array valid for
 * the call only), at least `every` iterations apart (rounded up to the
 * solver's host read-back period: 8 iterations in FP64, 1 in mixed
 * precision).  A nonzero return stops the solve: x keeps the current
 * iterate, iters and the true residuals are filled in, and the solver
 * returns DWF_ENOCONV.  fn = NULL turns reporting off; `user` is passed
 * through untouched.  This is a reporting hook, not part of the method. */
typedef int (*dwf_progress_fn)(void* user, int iteration, int nrhs, const double* rel_resid);
int dwf_set_progress(dwf_handle h, dwf_progress_fn fn, void* user, int every);

/* SYNCHRONOUS.  Red-black solve of D_DW psi = eta (FP64, packed "both"
 * layout, nrhs = 1), the prec-CGNR of the Conventional Krylov Solvers section
 * with the Schur complement of the Two level preconditioner section: eta' = eta_e - M_eo M5D^{-1} eta_o, CG on
 * M_pc^dag M_pc psi_e = M_pc^dag eta', psi_o = M5D^{-1}(eta_o - M_oe psi_e).
 * psi's even half is the initial guess. */
int dwf_solve_rb(dwf_handle h, const void* eta, void* psi, double tol, int maxiter, int* iters,
                 double* true_rel_resid);

/* Red-black operator used by dwf_mpc, dwf_mpcdagmpc, dwf_cg, dwf_solve_rb and
 * dwf_power (Conventional Krylov Solvers section, the Krylov table: the two Schur
 * forms of the preconditioned operator): form 1 (default) M_pc = M_ee - M_eo M_oo^{-1} M_oe; form 2
 * M_pc = 1 - M_ee^{-1} M_eo M_oo^{-1} M_oe, whose red-black solve takes the
 * right-hand side M_ee^{-1} eta'.  The filters, the smoother and the force
 * are defined on form 1 and return DWF_EINVAL under form 2.  The adjoint
 * of form 2 (dwf_mpc with dagger) needs out distinct from in. */
int dwf_set_schur_form(dwf_handle h, int form);

/* SYNCHRONOUS.  Unpreconditioned solve of D_DW psi = eta by CG on
 * D_DW^dag D_DW psi = D_DW^dag eta over both parities (Conventional Krylov
 * Solvers section, the Krylov table's CGNR row), FP64 packed "both" fields, psi holding the initial guess.
 * Needs a DWF_F64 handle with max_cg_rhs >= 2.  iters and true_rel_resid
 * (host, may be NULL) receive the iterations and ||b - A psi|| / ||b|| of the
 * normal equations.  Returns DWF_ENOCONV after maxiter or when stopped by the
 * progress callback. */
int dwf_solve_unprec(dwf_handle h, const void* eta, void* psi, double tol, int maxiter, int* iters,
                     double* true_rel_resid);

/* SYNCHRONOUS.  Power method for lambda_max of M_pc^dag M_pc (Deflation
 * basis setup section: the upper end of the filter interval comes from the
 * power method) from the start vector v (handle precision, one rhs, overwritten with the last iterate).
 * The handle keeps the estimate (a Rayleigh quotient, so never above the true
 * lambda_max) until its links or Schur form change; the three calls below
 * then return the warning DWF_WLAMBDA, with their results computed, when
 * their upper bound lies below it. */
int dwf_power(dwf_handle h, void* v, int iters, double rtol, double* lambda_max, int* iters_done);

/* In place: vecs <- T_order(x(A)) vecs, x(A) = 2 (A - lo) / (hi - lo) - 1,
 * A = M_pc^dag M_pc, for nvecs right-hand sides at once (handle precision),
 * no normalisation (Chebyshev smoothers / Deflation basis setup sections).
 * DWF_WLAMBDA if hi is below dwf_power's lambda_max (see there). */
int dwf_chebyshev_filter(dwf_handle h, int order, double lo, double hi, void* vecs, int nvecs);

/* The recursive series of the setup (Deflation basis setup section): v0 = T_m(x_[lam_lo, lam_max](A)) eta,
 * then out_series[k] = T_{k delta}(2 A / lam_max - 1) v0 for k = 0..nvec-1
 * (one rhs; out_series holds nvec packed fields).  eta is not modified.
 * DWF_WLAMBDA if lam_max is below dwf_power's lambda_max. */
int dwf_chebyshev_series(dwf_handle h, int m, double lam_lo, double lam_max, int delta, int nvec,
                         const void* eta, void* out_series);

/* The Chebyshev smoother of the normal residual system (Chebyshev smoothers
 * section): out = [c_0/2 + sum_{j=1}^{order} c_j T_j(x(A))] M_pc^dag in,
 * A = M_pc^dag M_pc, x(A) = 2 (A - lo) / (hi - lo) - 1, with c_j the Chebyshev
 * interpolation coefficients of 1/y on [lo, hi] at the nodes
 * theta_k = pi (k + 1/2) / order.  A polynomial approximation of
 * (M_pc^dag M_pc)^{-1} M_pc^dag = M_pc^{-1} on [lo, hi]; order applications
 * of A plus one of M_pc^dag.  in, out: nrhs packed even fields (handle
 * precision), distinct.  Requires order >= 1 and 0 < lo < hi.  DWF_WLAMBDA if
 * hi is below dwf_power's lambda_max. */
int dwf_chebyshev_smoother(dwf_handle h, int order, double lo, double hi, const void* in_e, void* out_e,
                           int nrhs);

/* SYNCHRONOUS.  In place Q R = V for nvecs packed even fields (handle
 * precision), the orthonormal basis that the projector P_S of the Two level
 * preconditioner section assumes, with FP64 inner products.  Sets of
 * nvecs <= 64 take Cholesky QR twice (one Gram matrix of all the vectors per
 * round, V <- V R^{-1} in place); a set whose Gram matrix is too close to
 * singular for it (condition number beyond about 1e7), or too large for the
 * handle's scratch, and larger sets take classical Gram-Schmidt applied twice.
 * Both give the unique Q R with a positive real diagonal, up to rounding.
 * R (nvecs x nvecs complex128, row-major, upper triangular, positive real
 * diagonal) is written to host memory R_host if non-NULL.  DWF_EBREAKDOWN if
 * the vectors are numerically dependent. */
int dwf_gram_schmidt(dwf_handle h, void* vecs, int nvecs, double* R_host);

/* <a_r, b_r> = sum over the 5D sites, spins and colours of conj(a_r) b_r for
 * nrhs packed one-parity fields of precision prec (either parity; each
 * operand is nrhs consecutive fields): the inner products of the CG of the
 * Spectrum of domain wall fermions section, and the pseudofermion action
 * S = phi^dag X of the Conclusions section's HMC.  Accumulated in FP64 and
 * reduced in a fixed order, so repeated calls are bitwise identical.
 * result: device array of 2 nrhs doubles (re, im per rhs), written
 * asynchronously on the handle's stream.  The reduction goes through the
 * handle's workspace, so calls on one handle must stay ordered on its
 * stream. */
int dwf_dot(dwf_handle h, int prec, const void* a, const void* b, int nrhs, double* result);

#define DWF_DOT_NOALLOC_MAX_RHS 64
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the inner
 * products of dwf_dot with no handle, no workspace and no allocation.  dims,
 * Ls and prec describe the packed fields as for dwf_field_bytes; a and b are
 * nrhs consecutive one-parity fields each; result is a device array of
 * 2 nrhs doubles (re, im per rhs), written asynchronously on `stream`
 * (a hipStream_t; NULL = the default stream).  The values are bitwise those
 * of dwf_dot.  The partial sums go to a fixed device array of
 * DWF_DOT_NOALLOC_MAX_RHS * 2048 doubles (1 MiB) that each GPU holds from the
 * first call on it until the process ends; nrhs above DWF_DOT_NOALLOC_MAX_RHS
 * is rejected with DWF_EINVAL.  All calls on one GPU share that array, so
 * calls that overlap in time on one GPU (different streams, or threads)
 * race; calls ordered on one stream do not.  Returns DWF_OK, DWF_EINVAL or
 * DWF_EHIP. */
int dwf_dot_noalloc(const int dims[4], int Ls, int prec, const void* a, const void* b, int nrhs, double* result,
                    void* stream);

/* ---- coarse-space transfer ------------------------------------------------ */

/* Blocks of the two-level method (Two level preconditioner section: the
 * blocked basis phi_k^b is phi_k restricted to block b): 4D boxes of
 * block[0..3] = bx, by, bz, bt sites tiling the lattice, each with all Ls
 * slices (the Algorithm A / B table uses 4x2x4x2 and 2^4 at Ls = 16).  Every
 * extent must divide the lattice extent, the block must hold equally many
 * even and odd sites, and (even sites per block) x Ls <= 1024.  Blocks are
 * numbered lexicographically, bx-block index fastest; *nblocks (host, may be
 * NULL) receives their count.  Builds a table in the handle's workspace;
 * SYNCHRONOUS.  The calls below work on even-parity packed fields of the
 * handle's precision and need dwf_set_blocks first. */
int dwf_set_blocks(dwf_handle h, const int block[4], int* nblocks);

/* Blocks of the Two level preconditioner section as dwf_set_blocks, with
 * parity = DWF_EVEN (the same) or DWF_BOTH: then the
 * coarse-space calls below take fields of both parities in the packed
 * "both" layout (for n fields: the n even halves, then the n odd halves),
 * a block holds all bx*by*bz*bt of its sites (sites per block x Ls <= 1024),
 * and dwf_chiral_split writes its 2 nvec outputs in the same layout.  The
 * two-level solver (below) coarsens the full-lattice H_DW this way. */
int dwf_set_blocks_ex(dwf_handle h, const int block[4], int parity, int* nblocks);

/* Chirality split of nvec fields (Deflation basis setup section: the
 * filtered vectors are projected with 1 +- Gamma_5 before coarsening the
 * five-dimensional operator): out[2k] = (1 + Gamma_5) in[k] / 2 and
 * out[2k+1] = (1 - Gamma_5) in[k] / 2, (Gamma_5 v)_s = gamma_5 v_{Ls-1-s}.
 * in: nvec fields, out: 2 nvec fields; they must not overlap. */
int dwf_chiral_split(dwf_handle h, const void* in, void* out, int nvec);

/* Device scratch (bytes) that dwf_block_orthonormalize (Two level
 * preconditioner section) needs for nvec vectors with the current blocks; 0 if blocks are not set or nvec is
 * outside [1, 64]. */
size_t dwf_block_scratch_bytes(dwf_handle h, int nvec);

/* SYNCHRONOUS.  In place: inside every block, orthonormalise
 * phi_0^b .. phi_{nvec-1}^b in index order (the orthonormal blocked basis of
 * the Two level preconditioner section) (Q^b R^b = Phi^b, R^b upper
 * triangular with a positive real diagonal), by two rounds of Cholesky QR
 * with FP64 Gram matrices.  scratch: caller-owned device memory of at least
 * dwf_block_scratch_bytes(h, nvec) bytes.  1 <= nvec <= 64.  Returns
 * DWF_EBREAKDOWN if some block's vectors are linearly dependent. */
int dwf_block_orthonormalize(dwf_handle h, void* basis, int nvec, void* scratch, size_t scratch_bytes);

/* Restriction (the restrictor <phi_k^b| of the Two level preconditioner
 * section): coarse[r][b][k] = <phi_k^b, v_r> = sum over the block's 5D sites,
 * spins and colours of conj(phi_k) v_r, for nrhs fields v (complex128
 * output, [nrhs][nblocks][nvec], device).  Sums are reduced in a fixed
 * order in FP64. */
int dwf_restrict(dwf_handle h, const void* basis, int nvec, const void* v, int nrhs, void* coarse);

/* Prolongation (the prolongator |phi_k^b> of the Two level preconditioner
 * section): v_r = sum_{b,k} coarse[r][b][k]
 * phi_k^b for nrhs coarse vectors laid out as dwf_restrict writes them; FP64
 * accumulation, stored in the handle's precision.  v must not alias the
 * basis. */
int dwf_prolong(dwf_handle h, const void* basis, int nvec, const void* coarse, int nrhs, void* v);

/* ---- two-level HDCR solver (FP64, fields of both parities) ---------------- */

/* out = H_DW in = Gamma_5 D_DW in, (Gamma_5 v)_s = gamma_5 v_{Ls-1-s} (Spectrum
 * of domain wall fermions section), for nrhs packed "both" fields.  Needs a
 * DWF_F64 handle with max_cg_rhs >= 1: D_DW in goes through the handle's FP64
 * CG work fields, so it must not overlap a dwf_cg / dwf_solve_* call on the
 * same handle (both are ordered on the handle's stream). */
int dwf_hdw(dwf_handle h, const void* in, void* out, int nrhs);

/* Parameters of Algorithms A / B (their table): the smoother
 * S_cheb([smoother_lo, smoother_hi], smoother_order) of the Chebyshev
 * smoothers section with M = H_DW; the coarse solve, CG on the normal
 * equations of the little Dirac operator stopped at relative residual
 * coarse_tol of those equations or after coarse_maxiter iterations; the
 * outer GCR restarted every nkrylov directions; and the storage of the
 * little Dirac operator, coarse_prec = DWF_F64 (0, the default of a zeroed
 * struct) or DWF_F32 (complex64 entries, half the bytes of each coarse
 * matvec; coarse vectors and all sums stay FP64). */
typedef struct {
  int smoother_order;
  double smoother_lo, smoother_hi;
  double coarse_tol;
  int coarse_maxiter;
  int nkrylov;
  int coarse_prec;
} dwf_hdcr_params;

typedef struct dwf_hdcr_s* dwf_hdcr;

/* Device workspace (bytes) of an HDCR solver (Algorithms section, Algorithms
 * A / B) with nvec basis vectors and nkrylov outer directions under the handle's current DWF_BOTH blocks: the
 * stencil of the little Dirac operator (nblocks x 9 x nvec^2 complex128),
 * coarse vectors, and 11 + 2 nkrylov FP64 fields of both parities.  0 if
 * blocks are not set with DWF_BOTH or an argument is out of range. */
size_t dwf_hdcr_workspace_bytes(dwf_handle h, int nvec, int nkrylov);

/* Create (and destroy) an HDCR solver of the Algorithms section
 * (Algorithms A / B) on a DWF_F64 handle whose blocks were set with
 * dwf_set_blocks_ex(..., DWF_BOTH, ...); 1 <= nvec <= 64, 1 <= nkrylov <= 64,
 * smoother_order >= 1, 0 < smoother_lo < smoother_hi, coarse_tol > 0.  The
 * caller owns ws (>= dwf_hdcr_workspace_bytes) and keeps it, and the handle,
 * alive until dwf_hdcr_destroy.  Calls on the solver fail with DWF_EINVAL
 * if the handle's blocks are changed afterwards. */
int dwf_hdcr_create(dwf_handle h, int nvec, const dwf_hdcr_params* params, void* ws, size_t ws_bytes,
                    dwf_hdcr* out);
int dwf_hdcr_destroy(dwf_hdcr hd);

/* In place: vecs <- T_order(x(D_DW^dag D_DW)) vecs, x(A) = 2 (A - lo)/(hi - lo) - 1,
 * for nvecs fields of both parities (packed "both" layout), the setup filter
 * of the Deflation basis setup section on the five-dimensional squared
 * operator that Algorithms A / B coarsen.  No normalisation. */
int dwf_hdcr_filter(dwf_hdcr hd, int order, double lo, double hi, void* vecs, int nvecs);

/* The recursive series of the setup on the same operator A = D_DW^dag D_DW:
 * out_series[0] = T_m(x_[lam_lo, lam_max](A)) eta, then out_series[k] =
 * T_{k delta}(2 A / lam_max - 1) out_series[0] for k = 1..nvec-1 (Deflation
 * basis setup section; m + (nvec - 1) delta applications of A).  eta: one
 * field of both parities, unchanged; out_series: nvec fields in the packed
 * "both" layout, distinct from eta. */
int dwf_hdcr_series(dwf_hdcr hd, int m, double lam_lo, double lam_max, int delta, int nvec, const void* eta,
                    void* out_series);

/* SYNCHRONOUS.  Use basis (nvec packed "both" fields, normally chirally split
 * and block-orthonormalised with the DWF_BOTH blocks) as the blocked basis
 * phi_k^b and build the little Dirac operator A^{ab}_{jk} = <phi_j^a | H_DW |
 * phi_k^b> (Two level preconditioner section).  The basis stays owned by
 * the caller and must stay unchanged while the solver uses it. */
int dwf_hdcr_set_basis(dwf_hdcr hd, const void* basis);

/* Device pointer to the little Dirac operator (Two level preconditioner
 * section), a 9-point stencil over the
 * block grid: complex128 (complex64 with coarse_prec = DWF_F32) [nblocks][9][nvec][nvec], entry (j, k) of stencil
 * point d at (d * nvec + k) * nvec + j.  Point d < 8 couples block b to the
 * block that hop direction d leads to (d = 2 mu + 0 forward / 1 backward,
 * mu = x, y, z, t), point 8 to b itself.  NULL for a null solver. */
const void* dwf_hdcr_coarse_data(dwf_hdcr hd);

/* y = A x for one coarse vector (complex128 [nblocks][nvec], device), A the
 * little Dirac operator of the Two level preconditioner section. */
int dwf_hdcr_coarse_apply(dwf_hdcr hd, const void* x, void* y);

/* SYNCHRONOUS.  c = A^{-1} d (the coarse solve inside Q of the Two level
 * preconditioner section) by CG on A^dag A c = A^dag d from c = 0 (A is
 * Hermitian), stopped when the normal equations' relative residual is
 * <= tol or after maxiter iterations; *iters (host, may be NULL) receives
 * the count.  d and c are coarse vectors (device); the solver's coarse
 * work vectors are overwritten. */
int dwf_hdcr_coarse_solve(dwf_hdcr hd, const void* d, void* c, double tol, int maxiter, int* iters);

/* out = S_cheb([lo, hi], N) r with M = H_DW: [c_0/2 + sum_{j=1}^N c_j
 * T_j(x(H_DW^2))] H_DW r (Chebyshev smoothers section), one field of both
 * parities; r and out distinct. */
int dwf_hdcr_smoother(dwf_hdcr hd, const void* r, void* out);

/* SYNCHRONOUS.  x = one V(1,1) cycle applied to r (Composite V(1,1) section):
 * x1 = S r, x2 = x1 + Q (r - H_DW x1), x = x2 + S (r - H_DW x2) with
 * Q = P A^{-1} P^dag from the coarse solve; *coarse_iters (may be NULL)
 * receives the coarse CG iterations.  r and x distinct. */
int dwf_hdcr_vcycle(dwf_hdcr hd, const void* r, void* x, int* coarse_iters);

/* SYNCHRONOUS.  Solve D_DW psi = eta (one field of both parities; psi holds
 * the initial guess) as H_DW psi = Gamma_5 eta by flexible GCR with the
 * V(1,1) cycle as right preconditioner (pGCR(H_DW) of Algorithms A / B):
 * each direction z = V(1,1) r, w = H_DW z, w made orthonormal to the
 * earlier w by modified Gram-Schmidt (the same combination applied to z),
 * psi += <w, r> z, r -= <w, r> w; restarted from the true residual every
 * nkrylov directions.  Stops when ||r|| <= tol ||Gamma_5 eta||.  iters,
 * true_rel_resid (||Gamma_5 eta - H_DW psi|| / ||eta||) and coarse_iters (the
 * coarse CG iterations of all cycles) are host outputs, each may be NULL.
 * Reports progress through dwf_set_progress.  Returns DWF_ENOCONV after
 * maxiter directions or when stopped by the progress callback. */
int dwf_hdcr_solve(dwf_hdcr hd, const void* eta, void* psi, double tol, int maxiter, int* iters,
                   double* true_rel_resid, int* coarse_iters);

/* ---- HMC force ------------------------------------------------------------ */

/* Link gradient of S = phi^dag (M_pc^dag M_pc)^{-1} phi, the pseudofermion
 * estimate of the two-flavour determinant det(M^dag M) whose HMC evolution
 * the Conclusions section motivates, given X = A^{-1} phi and Y = M_pc X
 * (FP64 packed even fields, one rhs):
 *   G_mu(x) = -sum_s sum_spin [ a(x,s) ((1-g_mu) b(x+mu,s))^dag + ((1+g_mu) b(x,s)) a(x+mu,s)^dag ],
 * a = (Y even, M5D^{-dag} M_eo^dag Y odd), b = (X even, M5D^{-1} M_oe X odd),
 * written as grad_U in the natural link layout (complex128), with the
 * convention G = dS/dRe U + i dS/dIm U.  Needs a DWF_F64 handle. */
int dwf_force(dwf_handle h, const void* X_e, const void* Y_e, void* grad_U);

/* The same force in the Lie algebra, the form an HMC momentum update takes
 * (Conclusions: HMC): for every link, F^a_mu(x) = dS/d omega at omega = 0 along
 * U_mu(x) -> exp(i omega T^a) U_mu(x), which in the gradient convention of
 * dwf_force is F^a = -Im tr(T^a U_mu(x) G_mu(x)^dag), with T^a = lambda^a / 2
 * and lambda^1 .. lambda^8 the Gell-Mann matrices in their usual order.
 * U and grad_U: device arrays in the natural link layout
 * [T][Z][Y][X][4][3][3] complex128 (the links the handle was given and the
 * output of dwf_force); F: device array [T][Z][Y][X][4][8] double, written.
 * Caller-owned; ordered on the handle's stream.  Any handle of the lattice;
 * DWF_EINVAL on a null pointer. */
int dwf_lie_force(dwf_handle h, const void* U, const void* grad_U, void* F);

/* ---- introspection -------------------------------------------------------- */

/* Library plumbing (no passage of the paper defines this call).
 * Launch shape of the hopping kernels: 4D sites per workgroup (0 = default,
 * sites_per_block * Ls <= 256), the depth (1..3; 0 keeps the current one)
 * of the neighbour-load pipeline, i.e. how many directions' spinor loads a
 * wave keeps in flight, and the right-hand sides one workgroup loops over
 * with its links staged once in LDS (1..64; 0 keeps the current one). */
int dwf_set_tile(dwf_handle h, int sites_per_block, int pipeline_depth, int rhs_per_block);

/* Library plumbing (no passage of the paper defines this call).
 * SYNCHRONOUS.  Traversal order of the half-lattice sites in the hop kernels
 * (and the force kernel): 0 = lexicographic (x fastest, t slowest); 1 = the
 * (x,y,z) box split into 2x2x2 sub-boxes, one per XCD, each streamed with t
 * slowest (needs X, Y, Z divisible by 4); 2 = eight slabs of consecutive t,
 * one per XCD, each streamed with t fastest, then x, z, y (needs T divisible
 * by 8).  DWF_EINVAL for another mode or one the lattice does not admit.
 * Results do not depend on the order.  An order set here (or by
 * dwf_set_order_box) is kept by dwf_autotune; otherwise the autotuner picks
 * one. */
int dwf_set_order(dwf_handle h, int mode);

/* Library plumbing (no passage of the paper defines this call).
 * SYNCHRONOUS.  Traversal order 3: the (x,y,z) volume cut into nx x ny x nz
 * equal boxes (X/nx even), numbered x fastest and dealt to the XCDs in
 * contiguous groups; inside a box the sites run with t slowest, then z, y, x.
 * nx = 1 keeps whole x rows together.  DWF_EINVAL when the cut does not
 * divide the lattice so.  dwf_get_order reports the order in use (mode 0-3
 * and, for 3, the cut; box may be NULL). */
int dwf_set_order_box(dwf_handle h, int nx, int ny, int nz);
int dwf_get_order(dwf_handle h, int* mode, int box[3]);

/* Library plumbing (no passage of the paper defines this call).
 * Cap the resident hop workgroups per compute unit (0 = no cap) by reserving
 * LDS: fewer sites in flight per XCD keep the stencil's neighbour reuse
 * window inside that XCD's L2.  Results do not depend on it. */
int dwf_set_occupancy(dwf_handle h, int workgroups_per_cu);

/* Library plumbing (no passage of the paper defines this call).
 * SYNCHRONOUS.  Times M_pc^dag M_pc on nrhs right-hand sides (<= max_nrhs),
 * `reps` applications per candidate.  Unless the caller set a traversal
 * order, it first picks one (modes 0-2 and a fixed list of box cuts the
 * lattice admits, in a middle-sized launch shape); then the launch shape --
 * workgroups of 256, 128 and 64 lanes, load-pipeline depth 1..3, 1/2/4/8 rhs
 * per workgroup (<= nrhs).  Keeps the fastest in the handle and reports the
 * shape (any output pointer may be NULL; dwf_get_order reports the order).
 * The result is cached per (GPU architecture, lattice, Ls, nrhs, precision,
 * the caller's traversal order or none, occupancy cap, Schur form) for the
 * life of the process, and in the text file named by the environment variable
 * DWF_TUNE_CACHE when it is set (read on first use, appended to); a cached
 * choice is applied without timing, and best_ms then reports the time
 * measured when it was tuned. */
int dwf_autotune(dwf_handle h, int nrhs, int reps, int* best_spb, int* best_depth, int* best_rpb,
                 double* best_ms);

/* Library plumbing (no passage of the paper defines this call).
 * Empties the process's cache of tuned launch shapes (dwf_autotune); the
 * DWF_TUNE_CACHE file is not changed and is read again on the next tuning.
 * Always DWF_OK. */
int dwf_tune_cache_clear(void);

/* Library plumbing (no passage of the paper defines this call).
 * Timing of the hopping-term kernels by HIP events on the handle's stream.
 * dwf_enable_timing: enable = 0 stops it; 1 times every hop launch; n > 1
 * times every n-th hop launch (a stride coprime with the launches of one
 * solver iteration -- four per CG iteration -- samples every kind evenly and
 * puts fewer event records between the kernels); every call resets the sums.
 * DWF_EINVAL for enable < 0.  dwf_kernel_time reports the summed duration
 * (ms) and the number of timed launches since the last reset (it synchronises
 * the stream). */
int dwf_enable_timing(dwf_handle h, int enable);
int dwf_kernel_time(dwf_handle h, double* ms_total, long long* launches);

#ifdef __cplusplus
}
#endif

#endif /* DWF_H */
