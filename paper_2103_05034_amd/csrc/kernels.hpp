// Launchers exported between the libdwf translation units (internal).
#pragma once

#include "dwf_internal.hpp"
#include "plan.hpp"

namespace dwf {

// bytes of one right-hand side of a packed half field at `prec`
inline size_t field_bytes_rhs(const dwf_context* ctx, int prec) {
  return spinor_bytes(prec) * (size_t)ctx->g.Ls * (size_t)ctx->g.V4h;
}

// Host-side error reporting shared by the entry points: records the message
// returned by dwf_last_error and returns code.
int fail(int code, const char* fmt, ...);
int check_h(dwf_handle h);             // DWF_EINVAL for a null handle
int sync(dwf_context* c);              // synchronise the handle's stream
#define HIP_TRY(expr)                                                                              \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return ::dwf::fail(DWF_EHIP, "%s: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

void timing_begin(dwf_context* ctx);
void timing_end(dwf_context* ctx);

// hop.hip
void fill_shape(const dwf_context* ctx, HopArgs& a);
hipError_t launch_hop(dwf_context* ctx, int prec, HopArgs a, int out_parity, int dag, int epi, int nrhs);
// the same with the neighbour input stored at pin and the operand x at px (output at prec); the
// mixed forms offered are FP16S in -> FP32 out (EPI_M5INV, no x) and FP32 in + FP16S x -> FP32
// out (EPI_M5)
hipError_t launch_hop_ex(dwf_context* ctx, int prec, int pin, int px, HopArgs a, int out_parity, int dag, int epi,
                         int nrhs);
hipError_t launch_site5(dwf_context* ctx, int prec, const char* in, char* out, int dag, int inv, int nrhs);

// setup.hip
hipError_t launch_pack_links(dwf_context* ctx, const void* U);
hipError_t launch_neighbours(dwf_context* ctx);
hipError_t launch_pack(dwf_context* ctx, int prec, const void* natural, char* packed, int nrhs, int parity,
                       bool unpack);

// blas.hip -- per-rhs reductions land in ctx->scalars[rhs * NSCAL + slot] (NSCAL and
// RED_BLOCKS, the partial sums per rhs, come with the workspace plan)
enum Slot {
  S_RR = 0,      // |r|^2 (recursive)
  S_RR_OLD = 1,
  S_PAP = 2,
  S_ALPHA = 3,
  S_BETA = 4,
  S_BB = 5,
  S_ACTIVE = 6,  // 1 while the rhs iterates, 0 once converged
  S_RRMAX = 7,   // largest |r|^2 since the last reliable update (low-precision CG)
  S_TMP = 8,     // scratch dot result (re)
  S_TMPI = 9,    // scratch dot result (im)
  S_TRUE = 10,   // true |r|^2
  S_FLAG = 11,   // breakdown flag
  S_ITERS = 12,  // iterations done while active
  S_ALPHA_K = 13,  // 13..15: alphas of the directions not yet added to x (FP64 CG)
};
static_assert(S_ALPHA_K + 3 <= NSCAL, "the deferred alphas fit the per-rhs scalar slots");

// scal[rhs * NSCAL + slot] = sum_k partials[rhs * count + k] over per-site values (a
// fixed order set by count), then on one thread mode 0: nothing more; mode 1: alpha (slot
// S_PAP); mode 2: beta and the convergence step with tol2 (slot S_RR) -- scal_alpha /
// scal_beta + scal_converge fused; mode 3: beta, the iteration count and S_RRMAX =
// max(S_RRMAX, |r|^2), without retiring a rhs (the low-precision CG retires one only on its
// FP64 true residual).  Uses ctx->partials and ctx->counters as scratch.
hipError_t reduce_sites(dwf_context* ctx, const double* partials, int count, int nrhs, int slot, int mode,
                        double tol2);
// result[rhs] = <a, b> (complex, FP64 accumulation) into scalars[rhs*NSCAL + slot (+1 imag)]
hipError_t blas_dot(dwf_context* ctx, int pa, const char* a, int pb, const char* b, int nrhs, int slot,
                    bool imag);
// result[2 r], result[2 r + 1] = <a_r, b_r> (re, im) for nrhs fields of one precision, reduced
// through `partials` (RED_BLOCKS * 2 doubles per rhs) in the fixed order of blas_dot
hipError_t blas_dot_to(dwf_context* ctx, int prec, const char* a, const char* b, int nrhs, double* partials,
                       double* result);
// y <- alpha x + beta y with per-rhs or constant coefficients; any storage mix
//  coef_mode 0: constants; 1: alpha = scalars[slot_a], beta = cb (device coefficients)
hipError_t blas_axpby(dwf_context* ctx, int px, const char* x, int py, char* y, int nrhs, double ca,
                      double cb, int slot_a, int slot_b, int sign_a);
// out <- in (conversion between precisions)
hipError_t blas_copy(dwf_context* ctx, int pin, const char* in, int pout, char* out, int nrhs);
hipError_t blas_zero(dwf_context* ctx, int prec, char* out, int nrhs);
// CG step: x += alpha p; r -= alpha q; |r|^2 -> slot S_RR (new), per rhs
hipError_t cg_update_xr(dwf_context* ctx, int px, char* x, int pr, char* r, int pp, const char* p, int pq,
                        const char* q, int nrhs);
// p = r + beta p
hipError_t cg_update_p(dwf_context* ctx, int pr, const char* r, int pp, char* p, int nrhs,
                       bool orth = false);  // orth: remove p's component along r first
// r -= alpha q with |r|^2 -> S_RR ; then x += alpha p and p = r + beta p in one pass (old p)
hipError_t cg_update_r(dwf_context* ctx, int pr, char* r, int pq, const char* q, int nrhs);
hipError_t cg_update_xp(dwf_context* ctx, int px, char* x, int pr, const char* r, int pp, char* p, int nrhs);
// CG with the x update deferred: pn = r + beta p (p kept), and alpha copied to slot keep
// (r at pr, p and pn at pp: F64/F64, F32/F32 or F32/F16S)
hipError_t cg_next_dir(dwf_context* ctx, int pr, const char* r, int pp, const char* p, char* pn, int keep, int nrhs);
// x += alpha_0 p_0 + ... + alpha_{n-1} p_{n-1} (x FP64; alpha_k from slot[k]; terms in this
// order, each skipped when its alpha is 0), then, when pn is given, pn = r + beta p_{n-1}
// (pn may be p_0).  1 <= n <= 4; precisions as cg_next_dir.
hipError_t cg_flush_x(dwf_context* ctx, char* x, int pr, const char* r, int pp, char* const p[], const int slot[],
                      int n, char* pn, int nrhs);
// reliable update of the low-precision CG: p += r_true - r_iter, then r_iter = r_true (r_true FP64,
// r_iter FP32, p at pp)
hipError_t cg_reliable_p(dwf_context* ctx, const char* r_true, char* r_iter, int pp, char* p, int nrhs);
// p -= (r^dag p / |r|^2 - 1) r per active rhs (r FP32; the dot in scalars S_TMP, S_TMPI)
hipError_t cg_orth_p(dwf_context* ctx, const char* r, int pp, char* p, int nrhs);
// scalar bookkeeping kernels
hipError_t scal_alpha(dwf_context* ctx, int nrhs);  // alpha = rr / pAp  (0 if inactive)
hipError_t scal_beta(dwf_context* ctx, int nrhs);   // beta = rr_new / rr_old
hipError_t scal_set(dwf_context* ctx, int nrhs, int slot, double v);
hipError_t scal_copy(dwf_context* ctx, int nrhs, int dst, int src);
// per active rhs: count the iteration, flag non-finite residuals, and retire
// the rhs once |r|^2 <= tol2 |b|^2 (only if allow_stop)
hipError_t scal_converge(dwf_context* ctx, int nrhs, double tol2, bool count_iter, int allow_stop = 1);
// GS helpers: dots of v against Q_k (k < j) into coef[k]; v -= sum_k coef[k] Q_k
hipError_t gs_multidot(dwf_context* ctx, int prec, const char* Q, const char* v, int j, double* coef);
hipError_t gs_multiaxpy(dwf_context* ctx, int prec, const char* Q, char* v, int j, const double* coef);
// Cholesky-QR pieces for up to TS_NMAX fields at any storage precision (fields
// consecutive at field_bytes_rhs apart).  ts_gram: G[k][j] =
// <v_j, v_k> for j <= k (complex FP64, n x n) from nwg per-workgroup partial sums in
// `partial` (nwg * n * n complex), added in workgroup order.  ts_combine: in place
// v_k <- sum_{j <= k} W[j][k] v_j (W upper triangular, complex FP64, W[j][k] at j * n + k).
constexpr int TS_NMAX = 64;
hipError_t ts_gram(dwf_context* ctx, int prec, const char* V, int n, double* partial, int nwg, double* G);
hipError_t ts_combine(dwf_context* ctx, int prec, char* V, int n, const double* W);
hipError_t gs_scale(dwf_context* ctx, int prec, char* v, const double* inv_norm);

// coarse.hip (block tables in ctx->bsite; coefficients complex FP64)
hipError_t launch_chiral_split(dwf_context* c, int prec, const char* in, char* out, int nvec);
// coef[r][b][k] = <phi_k^b, v_r> ([b][r][k] with per_block)
hipError_t launch_block_dot(dwf_context* c, int prec, const char* basis, int nvec, const char* v, int nrhs,
                            double* coef, bool per_block);
// out_r = sum_k coef[r][b][k] phi_k^b
hipError_t launch_block_prolong(dwf_context* c, int prec, const char* basis, int nvec, const double* coef, int nrhs,
                                char* out);
// phi_k <- sum_{j<=k} W[b][j][k] phi_j^b in place
hipError_t launch_block_apply(dwf_context* c, int prec, char* basis, int nvec, const double* wmat);
// per block: Gram matrix [b][k][j] = <phi_j, phi_k> (j <= k) with each vector read once
hipError_t launch_block_gram(dwf_context* c, int prec, const char* basis, int nvec, double* gram);
// per block: Cholesky of the Gram matrix ([b][k][j] = <phi_j, phi_k>) and W = R^{-1}
hipError_t launch_block_cholesky(dwf_context* c, const double* gram, double* w, int nvec, int* flag);

// force.hip
hipError_t launch_force(dwf_context* ctx, const char* a_even, const char* a_odd, const char* b_even,
                        const char* b_odd, double* grad_U);
// F[link][a] = -Im tr(T^a U G^dag) for every link (natural layouts; F real, 8 per link)
hipError_t launch_lie_force(dwf_context* ctx, const void* U, const void* G, double* F);

}  // namespace dwf
