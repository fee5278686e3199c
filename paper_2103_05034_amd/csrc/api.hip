// extern "C" entry points of libdwf: argument checks, workspace carving and the
// host-side drivers of the red-black operator, CG, the Chebyshev filter, the
// power method, Gram-Schmidt and the force.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <utility>

#include "dwf_internal.hpp"
#include "kernels.hpp"

using namespace dwf;

namespace {
thread_local std::string g_err = "no error";
}  // namespace

namespace dwf {
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int check_h(dwf_handle h) {
  if (!h) return fail(DWF_EINVAL, "null handle");
  return DWF_OK;
}

int sync(dwf_context* c) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(DWF_EHIP, "stream synchronize: %s", hipGetErrorString(e));
  return DWF_OK;
}
}  // namespace dwf

namespace {

static_assert(SPINOR_BYTES[DWF_F64] == Store<DWF_F64>::bytes_per_spinor &&
                  SPINOR_BYTES[DWF_F32] == Store<DWF_F32>::bytes_per_spinor &&
                  SPINOR_BYTES[DWF_F16S] == Store<DWF_F16S>::bytes_per_spinor,
              "the workspace plan and the kernels agree on the packed spinor sizes");

size_t up(size_t n) { return (n + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }

using plan::valid_dims;

// Points the handle's buffers into its workspace by the host-side plan.
void carve(dwf_context* d, const plan::Workspace& w, char* base) {
  auto at = [&](plan::Buffer b) -> char* { return w.offset[b] == plan::ABSENT ? nullptr : base + w.offset[b]; };
  d->links64 = at(plan::B_LINKS64);
  d->links32 = at(plan::B_LINKS32);
  d->nbr = reinterpret_cast<int*>(at(plan::B_NBR));
  d->t_buf = at(plan::B_T);
  d->u_buf = at(plan::B_U);
  d->cheb_a = at(plan::B_CHEB);
  d->r64 = at(plan::B_R64);
  d->p64 = at(plan::B_P64);
  d->q64 = at(plan::B_Q64);
  d->b64 = at(plan::B_B64);
  d->dir64 = at(plan::B_DIR64);
  d->lo_r = at(plan::B_LO_R);
  d->lo_x = at(plan::B_LO_X);
  d->lo_p = at(plan::B_LO_P);
  d->lo_q = at(plan::B_LO_Q);
  if (d->prec == DWF_F64) {  // FP64 handles run their CG in the handle-precision temporaries
    d->t64 = d->t_buf;
    d->u64 = d->u_buf;
  } else {
    d->t64 = at(plan::B_T64);
    d->u64 = at(plan::B_U64);
  }
  d->order = reinterpret_cast<int*>(at(plan::B_ORDER));
  d->bsite = reinterpret_cast<int*>(at(plan::B_BSITE));
  d->bnbr = reinterpret_cast<int*>(at(plan::B_BNBR));
  d->hop_partials = reinterpret_cast<double*>(at(plan::B_HOP_PARTIALS));
  d->partial_count = (size_t)w.chunk;
  d->partials = reinterpret_cast<double*>(at(plan::B_PARTIALS));
  d->scalars = reinterpret_cast<double*>(at(plan::B_SCALARS));
  d->counters = reinterpret_cast<unsigned*>(at(plan::B_COUNTERS));
  d->coef = reinterpret_cast<double*>(at(plan::B_COEF));
}

size_t fbytes(const dwf_context* c, int prec) { return field_bytes_rhs(c, prec); }

// ---------------------------------------------------------------------------
// Operator compositions (one chunk of at most the temporaries' capacity).
// ---------------------------------------------------------------------------
// Second Schur form (Results, Krylov table): out = in - M5D^{-1} D^{eo} M5D^{-1} D^{oe} in / 4.
// Adjoint: out = in - D^{oe dag} M5D^{-dag} D^{eo dag} M5D^{-dag} in / 4, with out holding
// M5D^{-dag} in until the last pass (out must not alias in).
static hipError_t mpc2_chunk(dwf_context* c, int prec, const char* in, char* out, char* t, int n, int dag,
                             double* partial) {
  hipError_t e;
  const char* src = in;
  if (dag) {
    e = launch_site5(c, prec, in, out, 1, 1, n);
    if (e != hipSuccess) return e;
    src = out;
  }
  HopArgs a{};
  a.in = src;
  a.out = t;
  a.alpha = 1.0;
  e = launch_hop(c, prec, a, DWF_ODD, dag, EPI_M5INV, n);
  if (e != hipSuccess) return e;
  HopArgs b{};
  b.in = t;
  b.x = in;
  b.out = out;
  b.alpha = -0.25;
  b.beta = 1.0;
  b.partial = partial;
  b.x_after = 1;
  return launch_hop(c, prec, b, DWF_EVEN, dag, dag ? EPI_LIN : EPI_M5INV, n);
}

// t_o = M5D^{-1} D_hop^{oe} in ; out = M5D in - D_hop^{eo} t / 4  (optionally |out|^2 partials)
hipError_t mpc_chunk(dwf_context* c, int prec, const char* in, char* out, char* t, int n, int dag,
                     double* partial = nullptr) {
  if (c->schur_form == 2) return mpc2_chunk(c, prec, in, out, t, n, dag, partial);
  HopArgs a{};
  a.in = in;
  a.out = t;
  a.alpha = 1.0;
  hipError_t e = launch_hop(c, prec, a, DWF_ODD, dag, EPI_M5INV, n);
  if (e != hipSuccess) return e;
  HopArgs b{};
  b.in = t;
  b.x = in;
  b.out = out;
  b.alpha = -0.25;
  b.partial = partial;
  return launch_hop(c, prec, b, DWF_EVEN, dag, EPI_M5, n);
}

// q = M_pc^dag M_pc p with p.q = |M_pc p|^2 reduced into slot S_PAP
hipError_t mdagm_pap(dwf_context* c, int prec, const char* p, char* q, char* t, char* u, int n) {
  hipError_t e = mpc_chunk(c, prec, p, u, t, n, 0, c->hop_partials);
  if (e != hipSuccess) return e;
  e = reduce_sites(c, c->hop_partials, (int)c->g.V4h, n, S_PAP, 0, 0.0);
  if (e != hipSuccess) return e;
  return mpc_chunk(c, prec, u, q, t, n, 1);
}

// One FP64 CG operator step without writing A p: u = M_pc p with p.Ap = |u|^2
// into S_PAP, alpha from it, then the last pass of M_pc^dag u updates
// r -= alpha A p in place and leaves |r|^2 in S_RR.
hipError_t cg_step_f64(dwf_context* c, const char* p, char* r, char* t, char* u, int n, double tol2) {
  hipError_t e = mpc_chunk(c, DWF_F64, p, u, t, n, 0, c->hop_partials);
  if (e != hipSuccess) return e;
  e = reduce_sites(c, c->hop_partials, (int)c->g.V4h, n, S_PAP, 1, tol2);  // p.Ap, alpha
  if (e != hipSuccess) return e;
  HopArgs a{};
  a.in = u;
  a.out = t;
  a.alpha = 1.0;
  e = launch_hop(c, DWF_F64, a, DWF_ODD, 1, EPI_M5INV, n);
  if (e != hipSuccess) return e;
  HopArgs b{};
  b.in = t;
  b.x = u;
  b.out = r;
  b.alpha = -0.25;
  b.partial = c->hop_partials;
  b.scal = c->scalars;
  e = launch_hop(c, DWF_F64, b, DWF_EVEN, 1, EPI_CGR, n);
  if (e != hipSuccess) return e;
  return reduce_sites(c, c->hop_partials, (int)c->g.V4h, n, S_RR, 2, tol2);  // |r|^2, beta, convergence
}

hipError_t mdagm_chunk(dwf_context* c, int prec, const char* in, char* out, char* t, char* u, int n) {
  hipError_t e = mpc_chunk(c, prec, in, u, t, n, 0);
  if (e != hipSuccess) return e;
  return mpc_chunk(c, prec, u, out, t, n, 1);
}

// out = ca * A in + cb * y + cc * z + cw * w   (A = M_pc^dag M_pc; out may alias z or w)
hipError_t cheb_step(dwf_context* c, int prec, const char* in, char* out, const char* y, const char* z, double ca,
                     double cb, double cc, char* t, char* u, int n, const char* w = nullptr, double cw = 0.0) {
  hipError_t e = mpc_chunk(c, prec, in, u, t, n, 0);
  if (e != hipSuccess) return e;
  HopArgs a{};
  a.in = u;
  a.out = t;
  a.alpha = 1.0;
  e = launch_hop(c, prec, a, DWF_ODD, 1, EPI_M5INV, n);
  if (e != hipSuccess) return e;
  HopArgs b{};
  b.in = t;
  b.x = u;
  b.y = y;
  b.z = z;
  b.out = out;
  b.alpha = -0.25;
  b.ca = ca;
  b.cb = cb;
  b.cc = cc;
  b.w = w;
  b.cw = cw;
  return launch_hop(c, prec, b, DWF_EVEN, 1, EPI_CHEB, n);
}

int read_scalars(dwf_context* c, int nrhs, std::vector<double>& out) {
  out.resize((size_t)nrhs * NSCAL);
  hipError_t e = hipMemcpyAsync(out.data(), c->scalars, out.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return fail(DWF_EHIP, "scalar readback: %s", hipGetErrorString(e));
  return sync(c);
}

}  // namespace

// kernel timing (used by launch_hop)
namespace dwf {
void timing_begin(dwf_context* ctx) {
  ctx->ev_open = false;
  if (!ctx->timing) return;
  if (ctx->ev_seq++ % ctx->ev_stride != 0) return;  // a launch between the sampled ones
  ctx->ev_open = true;
  if (ctx->ev_used == ctx->ev_pool.size()) {
    // drain
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& p : ctx->ev_pool) {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, p.a, p.b);
      ctx->ev_ms += ms;
    }
    ctx->ev_launches += (long long)ctx->ev_pool.size();
    ctx->ev_used = 0;
  }
  (void)hipEventRecord(ctx->ev_pool[ctx->ev_used].a, ctx->stream);
}
void timing_end(dwf_context* ctx) {
  if (!ctx->timing || !ctx->ev_open) return;
  ctx->ev_open = false;
  (void)hipEventRecord(ctx->ev_pool[ctx->ev_used].b, ctx->stream);
  ctx->ev_used++;
}
}  // namespace dwf

extern "C" {

const char* dwf_last_error(void) { return g_err.c_str(); }

size_t dwf_field_bytes(const int dims[4], int Ls, int prec, int nrhs) {
  std::string why;
  if (!valid_dims(dims, Ls, prec, 1, 0, &why) || nrhs < 0) {
    fail(DWF_EINVAL, "%s", why.c_str());
    return 0;
  }
  const long long V4h = (long long)dims[0] * dims[1] * dims[2] * dims[3] / 2;
  return spinor_bytes(prec) * (size_t)Ls * (size_t)V4h * (size_t)nrhs;
}

size_t dwf_workspace_bytes(const int dims[4], int Ls, int prec, int max_nrhs, int max_cg_rhs) {
  std::string why;
  if (!valid_dims(dims, Ls, prec, max_nrhs, max_cg_rhs, &why)) {
    fail(DWF_EINVAL, "%s", why.c_str());
    return 0;
  }
  return plan::plan_workspace(dims, Ls, prec, max_nrhs, max_cg_rhs).total;
}

int dwf_create(dwf_handle* out, const void* U, const int dims[4], int Ls, double M5, double mf, int prec,
               int max_nrhs, int max_cg_rhs, void* workspace, size_t ws_bytes, void* stream) {
  if (!out) return fail(DWF_EINVAL, "handle pointer is NULL");
  *out = nullptr;
  std::string why;
  if (!valid_dims(dims, Ls, prec, max_nrhs, max_cg_rhs, &why)) return fail(DWF_EINVAL, "%s", why.c_str());
  if (!U || !workspace) return fail(DWF_EINVAL, "U and workspace must be device pointers");
  if (!std::isfinite(M5) || !std::isfinite(mf) || M5 == 5.0) return fail(DWF_EINVAL, "M5 must be finite and != 5");
  const plan::Workspace layout = plan::plan_workspace(dims, Ls, prec, max_nrhs, max_cg_rhs);
  const size_t need = layout.total;
  if (ws_bytes < need) return fail(DWF_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(workspace) % WS_ALIGN) return fail(DWF_EINVAL, "workspace must be 256-byte aligned");
  dwf_context* c = new (std::nothrow) dwf_context();
  if (!c) return fail(DWF_ENOMEM, "host allocation failed");
  c->g = {dims[0], dims[1], dims[2], dims[3], Ls, (long long)dims[0] * dims[1] * dims[2] * dims[3], 0};
  c->g.V4h = c->g.V4 / 2;
  c->M5 = M5;
  c->mf = mf;
  c->prec = prec;
  c->max_nrhs = max_nrhs;
  c->max_cg_rhs = max_cg_rhs;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->ws = reinterpret_cast<char*>(workspace);
  c->ws_bytes = ws_bytes;
  carve(c, layout, c->ws);
  c->spb = 0;
  c->depth[0] = c->depth[1] = c->depth[2] = 2;
  c->rpb = 1;
  c->order_mode = 0;
  c->order_box[0] = c->order_box[1] = c->order_box[2] = 0;
  c->order_explicit = 0;
  c->lds_floor = 0;
  c->schur_form = 1;
  c->timing = false;
  c->ev_used = 0;
  c->ev_ms = 0;
  c->ev_launches = 0;
  c->ev_stride = 1;
  c->ev_seq = 0;
  c->ev_open = false;
  hipError_t e = launch_pack_links(c, U);
  if (e == hipSuccess) e = launch_neighbours(c);
  if (e == hipSuccess) e = hipMemsetAsync(c->scalars, 0, (size_t)(c->partial_count * NSCAL) * sizeof(double), c->stream);
  // the per-site reductions' completion counts start at zero and are reset by the kernel itself
  if (e == hipSuccess) e = hipMemsetAsync(c->counters, 0, c->partial_count * sizeof(unsigned), c->stream);
  if (e == hipSuccess && max_cg_rhs > 0 && prec != DWF_F64) {
    e = hipHostMalloc(reinterpret_cast<void**>(&c->pin_scal), (size_t)2 * max_cg_rhs * NSCAL * sizeof(double),
                      hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->pin_ev[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->pin_ev[1], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    dwf_destroy(c);
    return fail(DWF_EHIP, "set-up launch failed: %s", hipGetErrorString(e));
  }
  *out = c;
  return DWF_OK;
}

int dwf_update_links(dwf_handle h, const void* U) {
  if (int r = check_h(h)) return r;
  if (!U) return fail(DWF_EINVAL, "U is NULL");
  HIP_TRY(launch_pack_links(h, U));
  h->lam_max = 0;  // the operator changed
  return DWF_OK;
}

int dwf_set_stream(dwf_handle h, void* stream) {
  if (int r = check_h(h)) return r;
  h->stream = reinterpret_cast<hipStream_t>(stream);
  return DWF_OK;
}

int dwf_destroy(dwf_handle h) {
  if (!h) return DWF_OK;
  if (h->pin_scal) {
    (void)hipHostFree(h->pin_scal);
    (void)hipEventDestroy(h->pin_ev[0]);
    (void)hipEventDestroy(h->pin_ev[1]);
  }
  for (auto& p : h->ev_pool) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  delete h;
  return DWF_OK;
}

int dwf_pack(dwf_handle h, const void* natural, void* packed, int nrhs, int parity) {
  if (int r = check_h(h)) return r;
  if (!natural || !packed || nrhs < 1 || nrhs > 65535 || parity < 0 || parity > 2)
    return fail(DWF_EINVAL, "dwf_pack: bad argument");
  HIP_TRY(launch_pack(h, h->prec, natural, reinterpret_cast<char*>(packed), nrhs, parity, false));
  return DWF_OK;
}

int dwf_unpack(dwf_handle h, const void* packed, void* natural, int nrhs, int parity) {
  if (int r = check_h(h)) return r;
  if (!natural || !packed || nrhs < 1 || nrhs > 65535 || parity < 0 || parity > 2)
    return fail(DWF_EINVAL, "dwf_unpack: bad argument");
  HIP_TRY(launch_pack(h, h->prec, natural, const_cast<char*>(reinterpret_cast<const char*>(packed)), nrhs, parity,
                      true));
  return DWF_OK;
}

static int check_io(const void* in, const void* out, int nrhs) {
  if (!in || !out) return fail(DWF_EINVAL, "null field pointer");
  if (in == out) return fail(DWF_EINVAL, "in and out must not alias");
  if (nrhs < 1 || nrhs > 65535) return fail(DWF_EINVAL, "nrhs %d out of range", nrhs);
  return DWF_OK;
}

int dwf_dhop(dwf_handle h, const void* in, void* out, int out_parity, int nrhs, int dagger) {
  if (int r = check_h(h)) return r;
  if (int r = check_io(in, out, nrhs)) return r;
  if (out_parity != DWF_EVEN && out_parity != DWF_ODD) return fail(DWF_EINVAL, "out_parity must be 0 or 1");
  HopArgs a{};
  a.in = reinterpret_cast<const char*>(in);
  a.out = reinterpret_cast<char*>(out);
  a.alpha = 1.0;
  HIP_TRY(launch_hop(h, h->prec, a, out_parity, dagger ? 1 : 0, EPI_LIN, nrhs));
  return DWF_OK;
}

int dwf_m5d(dwf_handle h, const void* in, void* out, int nrhs, int dagger) {
  if (int r = check_h(h)) return r;
  if (int r = check_io(in, out, nrhs)) return r;
  HIP_TRY(launch_site5(h, h->prec, reinterpret_cast<const char*>(in), reinterpret_cast<char*>(out), dagger ? 1 : 0, 0,
                       nrhs));
  return DWF_OK;
}

int dwf_m5d_inv(dwf_handle h, const void* in, void* out, int nrhs, int dagger) {
  if (int r = check_h(h)) return r;
  if (!in || !out || nrhs < 1 || nrhs > 65535) return fail(DWF_EINVAL, "dwf_m5d_inv: bad argument");
  HIP_TRY(launch_site5(h, h->prec, reinterpret_cast<const char*>(in), reinterpret_cast<char*>(out), dagger ? 1 : 0, 1,
                       nrhs));
  return DWF_OK;
}

int dwf_ddw(dwf_handle h, const void* in, void* out, int nrhs, int dagger) {
  if (int r = check_h(h)) return r;
  if (int r = check_io(in, out, nrhs)) return r;
  const size_t half = fbytes(h, h->prec) * nrhs;
  const char* in_c = reinterpret_cast<const char*>(in);
  char* out_c = reinterpret_cast<char*>(out);
  for (int p = 0; p < 2; ++p) {
    HopArgs a{};
    a.in = in_c + (1 - p) * half;
    a.x = in_c + p * half;
    a.out = out_c + p * half;
    a.alpha = -0.5;
    HIP_TRY(launch_hop(h, h->prec, a, p, dagger ? 1 : 0, EPI_M5, nrhs));
  }
  return DWF_OK;
}

int dwf_mpc(dwf_handle h, const void* in_e, void* out_e, int nrhs, int dagger) {
  if (int r = check_h(h)) return r;
  if (int r = check_io(in_e, out_e, nrhs)) return r;
  const size_t fb = fbytes(h, h->prec);
  for (int r0 = 0; r0 < nrhs; r0 += h->max_nrhs) {
    const int n = nrhs - r0 < h->max_nrhs ? nrhs - r0 : h->max_nrhs;
    HIP_TRY(mpc_chunk(h, h->prec, reinterpret_cast<const char*>(in_e) + r0 * fb, reinterpret_cast<char*>(out_e) + r0 * fb,
                      h->t_buf, n, dagger ? 1 : 0));
  }
  return DWF_OK;
}

int dwf_mpcdagmpc(dwf_handle h, const void* in_e, void* out_e, int nrhs) {
  if (int r = check_h(h)) return r;
  if (int r = check_io(in_e, out_e, nrhs)) return r;
  const size_t fb = fbytes(h, h->prec);
  for (int r0 = 0; r0 < nrhs; r0 += h->max_nrhs) {
    const int n = nrhs - r0 < h->max_nrhs ? nrhs - r0 : h->max_nrhs;
    HIP_TRY(mdagm_chunk(h, h->prec, reinterpret_cast<const char*>(in_e) + r0 * fb,
                        reinterpret_cast<char*>(out_e) + r0 * fb, h->t_buf, h->u_buf, n));
  }
  return DWF_OK;
}

// ---------------------------------------------------------------------------
// CG
// ---------------------------------------------------------------------------
static int finish_cg(dwf_handle h, int nrhs, int maxiter, int* iters, double* resid, const std::vector<double>& sc,
                     const std::vector<double>& tr, bool stopped = false) {
  bool nconv = false, brk = false;
  for (int r = 0; r < nrhs; ++r) {
    const double* s = &sc[(size_t)r * NSCAL];
    if (iters) iters[r] = (int)s[S_ITERS];
    const double bb = s[S_BB];
    const double rel = bb > 0 ? std::sqrt(tr[r] / bb) : 0.0;
    if (resid) resid[r] = rel;
    if (s[S_FLAG] != 0.0 || !std::isfinite(rel)) brk = true;
    if (s[S_ACTIVE] != 0.0) nconv = true;
  }
  if (brk) return fail(DWF_EBREAKDOWN, "CG breakdown (non-finite or non-positive curvature)");
  if (nconv && stopped) return fail(DWF_ENOCONV, "CG stopped by the progress callback");
  if (nconv) return fail(DWF_ENOCONV, "CG did not converge in %d iterations", maxiter);
  return DWF_OK;
}

// Report progress to the caller's hook (if any) after iteration `it`, at most
// once per progress_every iterations; returns true when the hook asks to stop.
static bool report_progress(dwf_handle h, int it, int nrhs, const std::vector<double>& sc, int& last) {
  if (!h->progress_fn || it - last < h->progress_every) return false;
  last = it;
  std::vector<double> rel(nrhs);
  for (int rr = 0; rr < nrhs; ++rr) {
    const double* s = &sc[(size_t)rr * NSCAL];
    rel[rr] = s[S_BB] > 0 ? std::sqrt(s[S_RR] / s[S_BB]) : 0.0;
  }
  return h->progress_fn(h->progress_user, it, nrhs, rel.data()) != 0;
}

// r = b - A x in FP64 and |r|^2 -> slot, using FP64 temporaries
static hipError_t true_residual(dwf_handle h, const char* b, const char* x, char* r, int nrhs, int slot) {
  hipError_t e = mdagm_chunk(h, DWF_F64, x, r, h->t64, h->u64, nrhs);  // r = A x
  if (e != hipSuccess) return e;
  e = blas_axpby(h, DWF_F64, b, DWF_F64, r, nrhs, 1.0, -1.0, -1, -1, 1);  // r = b - A x
  if (e != hipSuccess) return e;
  return blas_dot(h, DWF_F64, r, DWF_F64, r, nrhs, slot, false);
}

// Search directions of a CG whose x += alpha p waits: the current direction is
// dir[n], and dir[0 .. n-1] hold the earlier ones whose alpha p is not yet in x
// (their alphas in slots S_ALPHA_K + k).  The K-th direction's update adds all K
// to x in the pass that forms the next direction, with the same roundings as one
// update per iteration; x is then streamed once per K iterations.
struct DeferredX {
  static constexpr int K = 4;
  char* dir[K];
  int pr, pp;  // precisions of the residual and the directions
  int n = 0;
  char* current() const { return dir[n]; }
  // after an iteration on dir[n] (alpha, beta and r updated): the next direction
  hipError_t advance(dwf_context* h, char* x, const char* r, int nrhs) {
    if (n < K - 1) {
      const hipError_t e = cg_next_dir(h, pr, r, pp, dir[n], dir[n + 1], S_ALPHA_K + n, nrhs);
      if (e == hipSuccess) ++n;
      return e;
    }
    const int slot[K] = {S_ALPHA_K, S_ALPHA_K + 1, S_ALPHA_K + 2, S_ALPHA};
    const hipError_t e = cg_flush_x(h, x, pr, r, pp, dir, slot, K, dir[0], nrhs);
    if (e == hipSuccess) n = 0;
    return e;
  }
  // adds the waiting directions to x; the current one becomes dir[0]
  hipError_t flush(dwf_context* h, char* x, int nrhs) {
    if (n == 0) return hipSuccess;
    const int slot[K - 1] = {S_ALPHA_K, S_ALPHA_K + 1, S_ALPHA_K + 2};
    const hipError_t e = cg_flush_x(h, x, pr, nullptr, pp, dir, slot, n, nullptr, nrhs);
    if (e != hipSuccess) return e;
    std::swap(dir[0], dir[n]);
    n = 0;
    return hipSuccess;
  }
};
static_assert(DeferredX::K - 1 + S_ALPHA_K <= NSCAL, "slots for the waiting alphas");

// FP64 CG on M_pc^dag M_pc.  On the first Schur form an iteration is the fused
// operator step (alpha, r -= alpha A p with |r|^2, beta and the convergence step)
// and the new direction p' = r + beta p written beside p, with x += alpha p
// deferred (DeferredX).
static int cg_f64(dwf_handle h, const char* b, char* x, int nrhs, double tol, int maxiter, int* iters, double* resid) {
  const double tol2 = tol * tol;
  char *r = h->r64, *p = h->p64, *q = h->q64;
  const size_t fb64 = fbytes(h, DWF_F64) * (size_t)h->max_cg_rhs;
  // the directions of one deferral cycle, on the first Schur form (q is free there)
  DeferredX dx{{p, q, h->dir64, h->dir64 ? h->dir64 + fb64 : nullptr}, DWF_F64, DWF_F64};
  const bool defer = h->schur_form == 1 && h->dir64 != nullptr;
  HIP_TRY(true_residual(h, b, x, r, nrhs, S_RR));
  HIP_TRY(blas_dot(h, DWF_F64, b, DWF_F64, b, nrhs, S_BB, false));
  HIP_TRY(blas_copy(h, DWF_F64, r, DWF_F64, p, nrhs));
  HIP_TRY(scal_set(h, nrhs, S_ACTIVE, 1.0));
  HIP_TRY(scal_set(h, nrhs, S_FLAG, 0.0));
  HIP_TRY(scal_set(h, nrhs, S_ITERS, 0.0));
  HIP_TRY(scal_converge(h, nrhs, tol2, false));
  std::vector<double> sc;
  // The host looks at the scalars every `check` iterations, and sooner when the
  // residual's fall since its last look predicts convergence before the next one:
  // iterations queued after convergence still run (as no-ops) at full cost.
  const int check = 8;
  bool stopped = false;
  int last = 0, next_look = 0, last_look = 0;
  std::vector<double> rr_seen(nrhs, -1.0);
  for (int it = 0; it < maxiter; ++it) {
    if (it == next_look) {
      if (int rc = read_scalars(h, nrhs, sc)) return rc;
      bool any = false;
      for (int rr = 0; rr < nrhs; ++rr) any |= sc[(size_t)rr * NSCAL + S_ACTIVE] != 0.0;
      if (!any) break;
      if (it > 0 && report_progress(h, it, nrhs, sc, last)) {
        stopped = true;
        break;
      }
      int step = check;
      if (it > last_look) {
        int need = 0;  // iterations the slowest active rhs is predicted to need
        for (int rr = 0; rr < nrhs; ++rr) {
          const double* sr = &sc[(size_t)rr * NSCAL];
          if (sr[S_ACTIVE] == 0.0) continue;
          const double now = sr[S_RR], prev = rr_seen[rr], goal = tol2 * sr[S_BB];
          double n = check;
          if (prev > 0.0 && now > 0.0 && now < prev && goal > 0.0) {
            const double fall = std::log(now / prev) / (it - last_look);  // per iteration, < 0
            n = std::log(goal / now) / fall;
          }
          need = std::max(need, n >= check ? check : (int)std::ceil(n));
        }
        step = std::max(1, std::min(check, need));
      }
      for (int rr = 0; rr < nrhs; ++rr) rr_seen[rr] = sc[(size_t)rr * NSCAL + S_RR];
      last_look = it;
      next_look = it + step;
    }
    if (defer) {
      HIP_TRY(cg_step_f64(h, dx.current(), r, h->t64, h->u64, nrhs, tol2));
      HIP_TRY(dx.advance(h, x, r, nrhs));
    } else if (h->schur_form == 1) {
      // alpha, r -= alpha A p, |r|^2, beta and the convergence step; then x += alpha p,
      // p = r + beta p (the convergence step changes neither alpha nor beta)
      HIP_TRY(cg_step_f64(h, p, r, h->t64, h->u64, nrhs, tol2));
      HIP_TRY(cg_update_xp(h, DWF_F64, x, DWF_F64, r, DWF_F64, p, nrhs));
    } else {
      HIP_TRY(mdagm_pap(h, DWF_F64, p, q, h->t64, h->u64, nrhs));
      HIP_TRY(scal_alpha(h, nrhs));
      HIP_TRY(cg_update_r(h, DWF_F64, r, DWF_F64, q, nrhs));
      HIP_TRY(scal_beta(h, nrhs));
      HIP_TRY(cg_update_xp(h, DWF_F64, x, DWF_F64, r, DWF_F64, p, nrhs));
      HIP_TRY(scal_converge(h, nrhs, tol2, true));
    }
  }
  HIP_TRY(dx.flush(h, x, nrhs));
  // true residual at exit
  HIP_TRY(true_residual(h, b, x, q, nrhs, S_TRUE));
  if (int rc = read_scalars(h, nrhs, sc)) return rc;
  std::vector<double> tr(nrhs);
  for (int rr = 0; rr < nrhs; ++rr) tr[rr] = sc[(size_t)rr * NSCAL + S_TRUE];
  return finish_cg(h, nrhs, maxiter, iters, resid, sc, tr, stopped);
}

// Low-precision CG with FP64 reliable updates on the first Schur form.  The
// search direction p is stored at the handle's precision (FP32, or FP16 +
// scale); the operator's intermediate fields t (odd) and u = M_pc p (even) and
// the iterated residual are FP32, so the operator is applied in FP32 to
// exactly the stored p; the solution accumulates in FP64 (an FP32 running sum
// of alpha p loses the low modes' small corrections and costs iterations at
// light mass).  One iteration is four hop launches: t = M5D^{-1} D_hop p;
// u = M5D p - D_hop t / 4 with p.Ap = |u|^2 reduced into alpha;
// t = M5D^{-dag} D_hop^dag u; r -= alpha (M5D^dag u - D_hop^dag t / 4) with
// |r|^2 reduced into beta; then p' = r + beta p beside p, with x += alpha p
// deferred (DeferredX: x is streamed once per four iterations).
// After each iteration the scalars are copied to pinned host memory, and the
// host reads them one iteration later, while the next iteration runs.  A rhs
// whose iterated |r| fell tenfold below its largest value since the last
// reliable update, or below the tolerance, triggers a reliable update of all
// rhs: r = b - A x in FP64, p += r - r_lo (which makes p the direction
// r + beta p_old that the new residual implies), r_lo = r, and p loses p_old's
// component along the new r (r^dag p = |r|^2, as CG's recursion assumes).  A
// rhs retires only on its FP64 true residual.
static int cg_mixed_fused(dwf_handle h, const char* b, char* x, int nrhs, double tol, int maxiter, int* iters,
                          double* resid) {
  const int P = h->prec;
  const double tol2 = tol * tol;
  const double delta2 = 0.01;
  char* r64 = h->r64;
  char* t32 = h->t64;  // FP32 views of the FP64 temporaries, which are free between reliable updates
  char* u32 = h->u64;
  if (!h->pin_scal) return fail(DWF_EINVAL, "dwf_cg: handle has no pinned scalar buffer");
  HIP_TRY(true_residual(h, b, x, r64, nrhs, S_RR));
  HIP_TRY(blas_dot(h, DWF_F64, b, DWF_F64, b, nrhs, S_BB, false));
  HIP_TRY(scal_copy(h, nrhs, S_TRUE, S_RR));
  HIP_TRY(scal_copy(h, nrhs, S_RRMAX, S_RR));
  HIP_TRY(blas_copy(h, DWF_F64, r64, DWF_F32, h->lo_r, nrhs));
  HIP_TRY(blas_copy(h, DWF_F32, h->lo_r, P, h->lo_p, nrhs));
  // directions at the handle's precision; the FP64 p and q are free in this solver
  DeferredX dx{{h->lo_p, h->lo_q, h->p64, h->q64}, DWF_F32, P};
  HIP_TRY(scal_set(h, nrhs, S_ACTIVE, 1.0));
  HIP_TRY(scal_set(h, nrhs, S_FLAG, 0.0));
  HIP_TRY(scal_set(h, nrhs, S_ITERS, 0.0));
  HIP_TRY(scal_converge(h, nrhs, tol2, false));
  std::vector<double> sc;
  if (int rc = read_scalars(h, nrhs, sc)) return rc;
  // Stagnation: a rhs whose true |r| has not halved over `patience`
  // consecutive update cycles (updates asked for by a tenfold fall of the
  // iterated |r|) is stagnant; the solve stops once every active rhs is.
  const int patience = 12;
  std::vector<double> best(nrhs);
  for (int rr = 0; rr < nrhs; ++rr) best[rr] = sc[(size_t)rr * NSCAL + S_RR];
  std::vector<int> idle(nrhs, 0);
  std::vector<char> cycle(nrhs, 0);
  const int nb = (int)h->g.V4h;  // per-site partial sums of the fused passes
  const size_t slot_doubles = (size_t)nrhs * NSCAL;
  bool stagnant = false, stopped = false;
  int it = 0, last = 0;
  auto any_active = [&](const double* snap) {
    for (int rr = 0; rr < nrhs; ++rr)
      if (snap[(size_t)rr * NSCAL + S_ACTIVE] != 0.0) return true;
    return false;
  };
  // pinned slot holding the scalars after the latest queued iteration that the
  // host has not read yet (-1: none)
  int prev_slot = -1;
  while (any_active(sc.data())) {
    int new_slot = -1;
    if (it < maxiter) {  // queue one iteration and the copy of its scalars
      HopArgs a{};
      a.in = dx.current();
      a.out = t32;
      a.alpha = 1.0;
      HIP_TRY(launch_hop_ex(h, DWF_F32, P, DWF_F32, a, DWF_ODD, 0, EPI_M5INV, nrhs));
      HopArgs m{};
      m.in = t32;
      m.x = dx.current();
      m.out = u32;
      m.alpha = -0.25;
      m.partial = h->hop_partials;
      HIP_TRY(launch_hop_ex(h, DWF_F32, DWF_F32, P, m, DWF_EVEN, 0, EPI_M5, nrhs));
      HIP_TRY(reduce_sites(h, h->hop_partials, nb, nrhs, S_PAP, 1, tol2));  // p.Ap, alpha
      HopArgs c{};
      c.in = u32;
      c.out = t32;
      c.alpha = 1.0;
      HIP_TRY(launch_hop(h, DWF_F32, c, DWF_ODD, 1, EPI_M5INV, nrhs));
      HopArgs d{};
      d.in = t32;
      d.x = u32;
      d.out = h->lo_r;
      d.alpha = -0.25;
      d.partial = h->hop_partials;
      d.scal = h->scalars;
      HIP_TRY(launch_hop(h, DWF_F32, d, DWF_EVEN, 1, EPI_CGR, nrhs));
      HIP_TRY(reduce_sites(h, h->hop_partials, nb, nrhs, S_RR, 3, tol2));  // |r|^2, beta, max |r|^2
      HIP_TRY(dx.advance(h, x, h->lo_r, nrhs));
      new_slot = prev_slot == 0 ? 1 : 0;
      HIP_TRY(hipMemcpyAsync(h->pin_scal + new_slot * slot_doubles, h->scalars, slot_doubles * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(hipEventRecord(h->pin_ev[new_slot], h->stream));
      ++it;
    }
    if (prev_slot < 0) {  // nothing to read yet (first iteration, or right after an update)
      if (new_slot < 0) break;
      prev_slot = new_slot;
      continue;
    }
    // the scalars after the iteration before the one just queued (after the last one
    // when nothing was queued), read while the queued iteration runs
    HIP_TRY(hipEventSynchronize(h->pin_ev[prev_slot]));
    const double* snap = h->pin_scal + prev_slot * slot_doubles;
    if (!any_active(snap)) break;  // every rhs stopped on a breakdown
    bool update = new_slot < 0;    // out of iterations: finish with an update
    for (int rr = 0; rr < nrhs; ++rr) {
      const double* s = snap + (size_t)rr * NSCAL;
      cycle[rr] = 0;
      if (s[S_ACTIVE] == 0.0) continue;
      cycle[rr] = s[S_RR] < delta2 * s[S_RRMAX];
      if (cycle[rr] || s[S_RR] < tol2 * s[S_BB] || !std::isfinite(s[S_RR])) update = true;
    }
    if (update) {
      // after the iteration(s) already queued: the FP64 residual of the FP64 solution
      HIP_TRY(dx.flush(h, x, nrhs));
      HIP_TRY(true_residual(h, b, x, r64, nrhs, S_RR));
      HIP_TRY(scal_copy(h, nrhs, S_TRUE, S_RR));
      HIP_TRY(scal_copy(h, nrhs, S_RRMAX, S_RR));
      HIP_TRY(cg_reliable_p(h, r64, h->lo_r, P, dx.current(), nrhs));
      HIP_TRY(blas_dot(h, DWF_F32, h->lo_r, P, dx.current(), nrhs, S_TMP, true));
      HIP_TRY(cg_orth_p(h, h->lo_r, P, dx.current(), nrhs));
      HIP_TRY(scal_converge(h, nrhs, tol2, false, 1));  // retire on the true residual
      if (int rc = read_scalars(h, nrhs, sc)) return rc;
      prev_slot = -1;  // a snapshot queued before the update is stale
      if (new_slot < 0) break;
      bool all_stuck = true;
      for (int rr = 0; rr < nrhs; ++rr) {
        const double* s = &sc[(size_t)rr * NSCAL];
        if (s[S_ACTIVE] == 0.0) continue;
        if (s[S_RR] < 0.25 * best[rr]) {
          best[rr] = s[S_RR];
          idle[rr] = 0;
        } else if (cycle[rr]) {
          ++idle[rr];
        }
        if (idle[rr] < patience) all_stuck = false;
      }
      if (any_active(sc.data()) && all_stuck) {
        stagnant = true;
        break;
      }
      continue;
    }
    if (report_progress(h, it - 1, nrhs, std::vector<double>(snap, snap + slot_doubles), last)) {
      stopped = true;
      break;
    }
    prev_slot = new_slot;
  }
  HIP_TRY(dx.flush(h, x, nrhs));
  HIP_TRY(true_residual(h, b, x, r64, nrhs, S_TRUE));
  if (int rc = read_scalars(h, nrhs, sc)) return rc;
  std::vector<double> tr(nrhs);
  for (int rr = 0; rr < nrhs; ++rr) tr[rr] = sc[(size_t)rr * NSCAL + S_TRUE];
  const int rc = finish_cg(h, nrhs, maxiter, iters, resid, sc, tr, stopped);
  if (rc == DWF_ENOCONV && stagnant)
    return fail(DWF_ENOCONV,
                "mixed-precision CG stagnated: the true residual stopped falling (the low-precision operator is "
                "too coarse for this conditioning; use a higher handle precision)");
  return rc;
}

// Low-precision CG with FP64 reliable updates on the second Schur form
// (operator applied at the handle's precision throughout).
static int cg_mixed(dwf_handle h, const char* b, char* x, int nrhs, double tol, int maxiter, int* iters,
                    double* resid) {
  const int P = h->prec;
  const double tol2 = tol * tol;
  const double delta2 = 0.01;  // reliable update when |r| falls 10x below its largest value since the last one
  char* r64 = h->r64;
  HIP_TRY(true_residual(h, b, x, r64, nrhs, S_RR));
  HIP_TRY(blas_dot(h, DWF_F64, b, DWF_F64, b, nrhs, S_BB, false));
  HIP_TRY(scal_copy(h, nrhs, S_TRUE, S_RR));
  HIP_TRY(blas_copy(h, DWF_F64, r64, DWF_F32, h->lo_r, nrhs));
  HIP_TRY(blas_copy(h, DWF_F32, h->lo_r, P, h->lo_p, nrhs));
  HIP_TRY(blas_zero(h, DWF_F32, h->lo_x, nrhs));
  HIP_TRY(scal_set(h, nrhs, S_ACTIVE, 1.0));
  HIP_TRY(scal_set(h, nrhs, S_FLAG, 0.0));
  HIP_TRY(scal_set(h, nrhs, S_ITERS, 0.0));
  HIP_TRY(scal_converge(h, nrhs, tol2, false));
  std::vector<double> sc;
  if (int rc = read_scalars(h, nrhs, sc)) return rc;
  std::vector<double> rrmax(nrhs);  // largest iterated |r|^2 since the last reliable update
  for (int rr = 0; rr < nrhs; ++rr) rrmax[rr] = sc[(size_t)rr * NSCAL + S_RR];
  // Stagnation: when the low-precision operator's error on the lowest modes
  // exceeds the reduction an update cycle asks for, the true residual stops
  // falling while the iterated one keeps going.  A rhs whose true |r| has
  // not halved over `patience` consecutive update cycles (updates asked for
  // by a tenfold fall of the iterated |r|, not the final tolerance checks)
  // is stagnant; the solve stops once every active rhs is.
  const int patience = 12;
  std::vector<double> best(rrmax);
  std::vector<int> idle(nrhs, 0);
  std::vector<char> cycle(nrhs, 0);
  bool stagnant = false;
  bool pending = false;  // lo_x holds an update not yet folded into x
  bool stopped = false;
  int last = 0;
  for (int it = 0; it < maxiter; ++it) {
    bool any = false;
    for (int rr = 0; rr < nrhs; ++rr) any |= sc[(size_t)rr * NSCAL + S_ACTIVE] != 0.0;
    if (!any) break;
    if (it > 0 && report_progress(h, it, nrhs, sc, last)) {
      stopped = true;
      break;
    }
    HIP_TRY(mdagm_pap(h, P, h->lo_p, h->lo_q, h->t_buf, h->u_buf, nrhs));
    HIP_TRY(scal_alpha(h, nrhs));
    HIP_TRY(cg_update_xr(h, DWF_F32, h->lo_x, DWF_F32, h->lo_r, P, h->lo_p, P, h->lo_q, nrhs));
    pending = true;
    if (int rc = read_scalars(h, nrhs, sc)) return rc;
    bool update = false;
    for (int rr = 0; rr < nrhs; ++rr) {
      const double* s = &sc[(size_t)rr * NSCAL];
      cycle[rr] = 0;
      if (s[S_ACTIVE] == 0.0) continue;
      rrmax[rr] = std::max(rrmax[rr], s[S_RR]);
      cycle[rr] = s[S_RR] < delta2 * rrmax[rr];
      if (cycle[rr] || s[S_RR] < tol2 * s[S_BB] || !std::isfinite(s[S_RR])) update = true;
    }
    if (update) {
      HIP_TRY(blas_axpby(h, DWF_F32, h->lo_x, DWF_F64, x, nrhs, 1.0, 1.0, -1, -1, 1));
      HIP_TRY(blas_zero(h, DWF_F32, h->lo_x, nrhs));
      pending = false;
      HIP_TRY(true_residual(h, b, x, r64, nrhs, S_RR));
      HIP_TRY(scal_copy(h, nrhs, S_TRUE, S_RR));
      HIP_TRY(blas_copy(h, DWF_F64, r64, DWF_F32, h->lo_r, nrhs));
      // r^dag p against the new residual, removed from p in the update below
      HIP_TRY(blas_dot(h, DWF_F32, h->lo_r, P, h->lo_p, nrhs, S_TMP, true));
    }
    HIP_TRY(scal_beta(h, nrhs));
    HIP_TRY(cg_update_p(h, DWF_F32, h->lo_r, P, h->lo_p, nrhs, update));
    HIP_TRY(scal_converge(h, nrhs, tol2, true, update ? 1 : 0));
    if (update) {
      if (int rc = read_scalars(h, nrhs, sc)) return rc;
      bool all_stuck = true, any_active = false;
      for (int rr = 0; rr < nrhs; ++rr) {
        const double* s = &sc[(size_t)rr * NSCAL];
        rrmax[rr] = s[S_RR];
        if (s[S_ACTIVE] == 0.0) continue;
        any_active = true;
        if (s[S_RR] < 0.25 * best[rr]) {
          best[rr] = s[S_RR];
          idle[rr] = 0;
        } else if (cycle[rr]) {
          ++idle[rr];
        }
        if (idle[rr] < patience) all_stuck = false;
      }
      if (any_active && all_stuck) {
        stagnant = true;
        break;
      }
    }
  }
  if (pending) {
    HIP_TRY(blas_axpby(h, DWF_F32, h->lo_x, DWF_F64, x, nrhs, 1.0, 1.0, -1, -1, 1));
  }
  HIP_TRY(true_residual(h, b, x, r64, nrhs, S_TRUE));
  if (int rc = read_scalars(h, nrhs, sc)) return rc;
  std::vector<double> tr(nrhs);
  for (int rr = 0; rr < nrhs; ++rr) tr[rr] = sc[(size_t)rr * NSCAL + S_TRUE];
  const int rc = finish_cg(h, nrhs, maxiter, iters, resid, sc, tr, stopped);
  if (rc == DWF_ENOCONV && stagnant)
    return fail(DWF_ENOCONV,
                "mixed-precision CG stagnated: the true residual stopped falling (the low-precision operator is "
                "too coarse for this conditioning; use a higher handle precision)");
  return rc;
}

int dwf_cg(dwf_handle h, const void* b, void* x, int nrhs, double tol, int maxiter, int* iters,
           double* true_rel_resid) {
  if (int r = check_h(h)) return r;
  if (!b || !x || b == x) return fail(DWF_EINVAL, "dwf_cg: b and x must be distinct device pointers");
  if (nrhs < 1 || nrhs > h->max_cg_rhs) return fail(DWF_EINVAL, "dwf_cg: nrhs %d outside [1, %d]", nrhs, h->max_cg_rhs);
  if (!(tol > 0) || maxiter < 0) return fail(DWF_EINVAL, "dwf_cg: tol must be > 0 and maxiter >= 0");
  if (h->prec == DWF_F64)
    return cg_f64(h, reinterpret_cast<const char*>(b), reinterpret_cast<char*>(x), nrhs, tol, maxiter, iters,
                  true_rel_resid);
  if (h->schur_form == 1)
    return cg_mixed_fused(h, reinterpret_cast<const char*>(b), reinterpret_cast<char*>(x), nrhs, tol, maxiter, iters,
                          true_rel_resid);
  return cg_mixed(h, reinterpret_cast<const char*>(b), reinterpret_cast<char*>(x), nrhs, tol, maxiter, iters,
                  true_rel_resid);
}

int dwf_solve_rb(dwf_handle h, const void* eta, void* psi, double tol, int maxiter, int* iters, double* resid) {
  if (int r = check_h(h)) return r;
  if (!eta || !psi || eta == psi) return fail(DWF_EINVAL, "dwf_solve_rb: eta and psi must be distinct");
  if (h->max_cg_rhs < 1) return fail(DWF_EINVAL, "dwf_solve_rb: handle was created without solver workspace");
  const size_t fb = fbytes(h, DWF_F64);
  const char* eta_e = reinterpret_cast<const char*>(eta);
  const char* eta_o = eta_e + fb;
  char* psi_e = reinterpret_cast<char*>(psi);
  char* psi_o = psi_e + fb;
  // t = M5D^{-1} eta_o ; eta' = eta_e + D_hop^{eo} t / 2 (into psi_o as scratch)
  HIP_TRY(launch_site5(h, DWF_F64, eta_o, h->t64, 0, 1, 1));
  HopArgs a{};
  a.in = h->t64;
  a.x = eta_e;
  a.out = psi_o;
  a.alpha = 0.5;
  a.beta = 1.0;
  HIP_TRY(launch_hop(h, DWF_F64, a, DWF_EVEN, 0, EPI_LIN, 1));
  // b = M_pc^dag eta' (first form); b = M_pc2^dag M5D^{-1} eta' (second form)
  if (h->schur_form == 2) {
    HIP_TRY(launch_site5(h, DWF_F64, psi_o, h->u64, 0, 1, 1));
    HIP_TRY(mpc_chunk(h, DWF_F64, h->u64, h->b64, h->t64, 1, 1));
  } else {
    HIP_TRY(mpc_chunk(h, DWF_F64, psi_o, h->b64, h->t64, 1, 1));
  }
  int rc = dwf_cg(h, h->b64, psi_e, 1, tol, maxiter, iters, resid);
  if (rc != DWF_OK && rc != DWF_ENOCONV) return rc;
  // psi_o = M5D^{-1} (eta_o + D_hop^{oe} psi_e / 2)
  HopArgs c{};
  c.in = psi_e;
  c.x = eta_o;
  c.out = psi_o;
  c.alpha = 0.5;
  c.beta = 1.0;
  HIP_TRY(launch_hop(h, DWF_F64, c, DWF_ODD, 0, EPI_M5INV, 1));
  if (int r2 = sync(h)) return r2;
  return rc;
}

// ---------------------------------------------------------------------------
// Power method, Chebyshev filter and series, Gram-Schmidt
// ---------------------------------------------------------------------------
int dwf_power(dwf_handle h, void* v, int iters, double rtol, double* lambda_max, int* iters_done) {
  if (int r = check_h(h)) return r;
  if (!v || iters < 1) return fail(DWF_EINVAL, "dwf_power: bad argument");
  const int P = h->prec;
  char* vv = reinterpret_cast<char*>(v);
  char* w = h->cheb_a;
  std::vector<double> sc;
  HIP_TRY(blas_dot(h, P, vv, P, vv, 1, S_TMP, false));
  if (int rc = read_scalars(h, 1, sc)) return rc;
  double nv = std::sqrt(sc[S_TMP]);
  if (!(nv > 0)) return fail(DWF_EINVAL, "dwf_power: zero start vector");
  HIP_TRY(blas_axpby(h, P, nullptr, P, vv, 1, 0.0, 1.0 / nv, -1, -1, 1));
  double lam = 0;
  int k = 0;
  for (k = 0; k < iters; ++k) {
    HIP_TRY(mdagm_chunk(h, P, vv, w, h->t_buf, h->u_buf, 1));
    HIP_TRY(blas_dot(h, P, vv, P, w, 1, S_TMP, false));
    HIP_TRY(blas_dot(h, P, w, P, w, 1, S_TRUE, false));
    if (int rc = read_scalars(h, 1, sc)) return rc;
    const double lam_new = sc[S_TMP];
    const double nw = std::sqrt(sc[S_TRUE]);
    if (!(nw > 0) || !std::isfinite(nw)) return fail(DWF_EBREAKDOWN, "dwf_power: non-finite iterate");
    HIP_TRY(blas_axpby(h, P, w, P, vv, 1, 1.0 / nw, 0.0, -1, -1, 1));
    if (k > 0 && std::fabs(lam_new - lam) < rtol * std::fabs(lam_new)) {
      lam = lam_new;
      ++k;
      break;
    }
    lam = lam_new;
  }
  if (int rc = sync(h)) return rc;
  if (lambda_max) *lambda_max = lam;
  if (iters_done) *iters_done = k;
  h->lam_max = lam;
  return DWF_OK;
}

// DWF_WLAMBDA (a warning; the result is computed) when a filter's upper bound lies
// below the lambda_max that dwf_power measured on this operator: the polynomial then
// grows without bound on the modes above it instead of staying within [-1, 1].
static int warn_lambda(dwf_handle h, double hi, const char* who) {
  if (h->lam_max > 0 && hi < h->lam_max)
    return fail(DWF_WLAMBDA, "%s: upper bound %g is below the measured lambda_max %g", who, hi, h->lam_max);
  return DWF_OK;
}

// In place T_order(x(A)) on one chunk V of n rhs; partner buffer W.
static int cheb_chunk(dwf_handle h, int order, double lo, double hi, char* V, char* W, int n) {
  if (order == 0) return DWF_OK;
  const int P = h->prec;
  const double w = hi - lo;
  // T1 = x(A) V = (2/w) A V - ((hi+lo)/w) V
  HIP_TRY(cheb_step(h, P, V, W, V, V, 2.0 / w, -(hi + lo) / w, 0.0, h->t_buf, h->u_buf, n));
  char* prev = V;
  char* cur = W;
  for (int k = 1; k < order; ++k) {
    // T_{k+1} = (4/w) A T_k - (2(hi+lo)/w) T_k - T_{k-1}, written over T_{k-1}
    HIP_TRY(cheb_step(h, P, cur, prev, cur, prev, 4.0 / w, -2.0 * (hi + lo) / w, -1.0, h->t_buf, h->u_buf, n));
    char* t = prev;
    prev = cur;
    cur = t;
  }
  if (cur != V) HIP_TRY(blas_copy(h, P, cur, P, V, n));
  return DWF_OK;
}

int dwf_chebyshev_filter(dwf_handle h, int order, double lo, double hi, void* vecs, int nvecs) {
  if (int r = check_h(h)) return r;
  if (!vecs || nvecs < 1 || order < 0 || !(hi > lo)) return fail(DWF_EINVAL, "dwf_chebyshev_filter: bad argument");
  if (h->schur_form != 1) return fail(DWF_EINVAL, "dwf_chebyshev_filter: needs the first Schur form");
  const size_t fb = fbytes(h, h->prec);
  for (int r0 = 0; r0 < nvecs; r0 += h->max_nrhs) {
    const int n = nvecs - r0 < h->max_nrhs ? nvecs - r0 : h->max_nrhs;
    if (int rc = cheb_chunk(h, order, lo, hi, reinterpret_cast<char*>(vecs) + r0 * fb, h->cheb_a, n)) return rc;
  }
  return warn_lambda(h, hi, "dwf_chebyshev_filter");
}

int dwf_chebyshev_series(dwf_handle h, int m, double lam_lo, double lam_max, int delta, int nvec, const void* eta,
                         void* out_series) {
  if (int r = check_h(h)) return r;
  if (h->schur_form != 1) return fail(DWF_EINVAL, "dwf_chebyshev_series: needs the first Schur form");
  if (!eta || !out_series || m < 0 || delta < 1 || nvec < 1 || !(lam_max > lam_lo) || !(lam_max > 0))
    return fail(DWF_EINVAL, "dwf_chebyshev_series: bad argument");
  const int P = h->prec;
  const size_t fb = fbytes(h, P);
  char* S = reinterpret_cast<char*>(out_series);
  HIP_TRY(blas_copy(h, P, reinterpret_cast<const char*>(eta), P, S, 1));
  if (int rc = cheb_chunk(h, m, lam_lo, lam_max, S, h->cheb_a, 1)) return rc;
  if (nvec == 1) return warn_lambda(h, lam_max, "dwf_chebyshev_series");
  // second recurrence over [0, lam_max]: x(A) = 2A/lam_max - 1
  char* prev = h->cheb_a;
  char* cur = h->cheb_a + fb;
  HIP_TRY(blas_copy(h, P, S, P, prev, 1));
  HIP_TRY(cheb_step(h, P, S, cur, S, S, 2.0 / lam_max, -1.0, 0.0, h->t_buf, h->u_buf, 1));
  int recorded = 1;
  for (int n = 1; recorded < nvec; ++n) {
    if (n % delta == 0) {
      HIP_TRY(blas_copy(h, P, cur, P, S + (size_t)recorded * fb, 1));
      ++recorded;
      if (recorded == nvec) break;
    }
    HIP_TRY(cheb_step(h, P, cur, prev, cur, prev, 4.0 / lam_max, -2.0, -1.0, h->t_buf, h->u_buf, 1));
    char* t = prev;
    prev = cur;
    cur = t;
  }
  return warn_lambda(h, lam_max, "dwf_chebyshev_series");
}

// Chebyshev smoother of the normal system: out = [c_0/2 + sum_{j=1}^N c_j T_j(x(A))] M_pc^dag in,
// x(A) = (2A - (lo+hi)) / (hi - lo), c_j the Chebyshev interpolation coefficients of 1/y on
// [lo, hi] at theta_k = pi (k + 1/2) / N.  Evaluated by Clenshaw's recurrence
// b_k = 2 x(A) b_{k+1} - b_{k+2} + c_k w, result = x(A) b_1 - b_2 + c_0 w / 2, w = M_pc^dag in,
// with the recurrence and the c_k w term fused into the last hop pass.
static void smoother_coeffs(double lo, double hi, int N, std::vector<double>& c) {
  c.assign((size_t)N + 1, 0.0);
  for (int j = 0; j <= N; ++j) {
    double sum = 0.0;
    for (int k = 0; k < N; ++k) {
      const double th = M_PI * (k + 0.5) / N;
      const double y = lo + (hi - lo) * (std::cos(th) + 1.0) / 2.0;
      sum += std::cos(j * th) / y;
    }
    c[j] = 2.0 / N * sum;
  }
}

int dwf_chebyshev_smoother(dwf_handle h, int order, double lo, double hi, const void* in_e, void* out_e, int nrhs) {
  if (int r = check_h(h)) return r;
  if (int r = check_io(in_e, out_e, nrhs)) return r;
  if (order < 1 || !(lo > 0) || !(hi > lo)) return fail(DWF_EINVAL, "dwf_chebyshev_smoother: order >= 1 and 0 < lo < hi");
  if (h->schur_form != 1) return fail(DWF_EINVAL, "dwf_chebyshev_smoother: needs the first Schur form");
  const int P = h->prec;
  const size_t fb = fbytes(h, P);
  std::vector<double> c;
  smoother_coeffs(lo, hi, order, c);
  const double wdt = hi - lo;
  const int cap = std::max(1, (h->max_nrhs > 2 ? h->max_nrhs : 2) / 2);  // two Clenshaw buffers per rhs
  for (int r0 = 0; r0 < nrhs; r0 += cap) {
    const int n = std::min(cap, nrhs - r0);
    const char* in = reinterpret_cast<const char*>(in_e) + r0 * fb;
    char* W = reinterpret_cast<char*>(out_e) + r0 * fb;  // w = M_pc^dag in, kept until the last step
    char* B1 = h->cheb_a;
    char* B2 = h->cheb_a + (size_t)n * fb;
    HIP_TRY(mpc_chunk(h, P, in, W, h->t_buf, n, 1));
    HIP_TRY(blas_axpby(h, P, W, P, B1, n, c[order], 0.0, -1, -1, 1));  // b_N = c_N w
    HIP_TRY(blas_zero(h, P, B2, n));                                   // b_{N+1} = 0
    for (int k = order - 1; k >= 1; --k) {
      // b_k = (4/w) A b_{k+1} - (2(lo+hi)/w) b_{k+1} - b_{k+2} + c_k w, over b_{k+2}
      HIP_TRY(cheb_step(h, P, B1, B2, B1, B2, 4.0 / wdt, -2.0 * (hi + lo) / wdt, -1.0, h->t_buf, h->u_buf, n, W, c[k]));
      std::swap(B1, B2);
    }
    // out = x(A) b_1 - b_2 + c_0 w / 2 (written over w)
    HIP_TRY(cheb_step(h, P, B1, W, B1, B2, 2.0 / wdt, -(hi + lo) / wdt, -1.0, h->t_buf, h->u_buf, n, W, 0.5 * c[0]));
  }
  return warn_lambda(h, hi, "dwf_chebyshev_smoother");
}

int dwf_dot(dwf_handle h, int prec, const void* a, const void* b, int nrhs, double* result) {
  if (int r = check_h(h)) return r;
  if (!a || !b || !result) return fail(DWF_EINVAL, "dwf_dot: null pointer");
  if (prec != DWF_F64 && prec != DWF_F32 && prec != DWF_F16S) return fail(DWF_EINVAL, "dwf_dot: unknown precision");
  if (nrhs < 1 || nrhs > 65535) return fail(DWF_EINVAL, "dwf_dot: nrhs %d out of range", nrhs);
  const size_t fb = fbytes(h, prec);
  const int chunk = (int)h->partial_count;  // rhs whose partial sums the handle's scratch holds at once
  for (int r0 = 0; r0 < nrhs; r0 += chunk) {
    const int n = std::min(chunk, nrhs - r0);
    HIP_TRY(blas_dot_to(h, prec, reinterpret_cast<const char*>(a) + r0 * fb, reinterpret_cast<const char*>(b) + r0 * fb,
                        n, h->partials, result + 2 * (size_t)r0));
  }
  return DWF_OK;
}

// Cholesky QR, twice (Two level preconditioner section: an orthonormal blocked
// basis; this is the whole-lattice case).  One round: G = V^dag V in FP64 from a
// tall-skinny Gram kernel, G = R^dag R on the host, V <- V R^{-1} in place.  The
// second round repairs the orthogonality the first loses to the conditioning,
// and R = R2 R1.  Q and R are CGS2's (the QR factorisation with a real positive
// diagonal is unique) up to rounding.  Returns GS_USE_CGS2, with the vectors
// untouched, when the first round's Gram matrix is too close to singular for
// this form or the scratch is too small; the caller then runs CGS2.
constexpr int GS_USE_CGS2 = 1;

static int gs_cholqr2(dwf_handle h, char* Q, int n, std::vector<double>& Rout) {
  const int P = h->prec;
  const size_t nn = (size_t)n * n;
  // scratch: per-workgroup partial Gram matrices, then G, in t_buf; W in u_buf
  const size_t cap = fbytes(h, P) * (size_t)h->partial_count;
  const size_t per = nn * 2 * sizeof(double);
  if (cap < 2 * per) return GS_USE_CGS2;
  const long long m = h->g.V4h * h->g.Ls * 12;
  long long nwg = (long long)(cap / per) - 1;
  nwg = std::min<long long>({nwg, 2048, (m + 255) / 256});
  if (nwg < 1) return GS_USE_CGS2;
  double* partial = reinterpret_cast<double*>(h->t_buf);
  double* Gd = partial + 2 * nn * (size_t)nwg;
  double* Wd = reinterpret_cast<double*>(h->u_buf);
  std::vector<double> G(2 * nn), R1, R2, W;
  for (int round = 0; round < 2; ++round) {
    HIP_TRY(ts_gram(h, P, Q, n, partial, (int)nwg, Gd));
    HIP_TRY(hipMemcpyAsync(G.data(), Gd, 2 * nn * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    if (int rc = sync(h)) return rc;
    // first round: a pivot below 1e-14 of its diagonal entry (a condition number
    // beyond about 1e7) leaves the set to CGS2
    std::vector<double>& R = round == 0 ? R1 : R2;
    if (!plan::cholesky_upper(G, n, R, round == 0 ? 1e-14 : 0.0)) {
      if (round == 0) return GS_USE_CGS2;
      return fail(DWF_EBREAKDOWN, "dwf_gram_schmidt: the vectors are numerically dependent");
    }
    plan::invert_upper(R, n, W);
    HIP_TRY(hipMemcpyAsync(Wd, W.data(), 2 * nn * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(ts_combine(h, P, Q, n, Wd));
    if (int rc = sync(h)) return rc;  // W's host copy is reused next round
  }
  plan::multiply_upper(R2, R1, n, Rout);  // R = R2 R1
  return DWF_OK;
}

int dwf_gram_schmidt(dwf_handle h, void* vecs, int nvecs, double* R_host) {
  if (int r = check_h(h)) return r;
  if (!vecs || nvecs < 1 || nvecs > GS_MAX) return fail(DWF_EINVAL, "dwf_gram_schmidt: nvecs must be in [1, %d]", GS_MAX);
  const int P = h->prec;
  const size_t fb = fbytes(h, P);
  char* Q = reinterpret_cast<char*>(vecs);
  if (nvecs <= TS_NMAX) {
    std::vector<double> Rq;
    const int rc = gs_cholqr2(h, Q, nvecs, Rq);
    if (rc == DWF_OK) {
      if (R_host) std::memcpy(R_host, Rq.data(), Rq.size() * sizeof(double));
      return DWF_OK;
    }
    if (rc != GS_USE_CGS2) return rc;
  }
  std::vector<double> R((size_t)nvecs * nvecs * 2, 0.0), cf(2 * (size_t)nvecs);
  std::vector<double> sc;
  const int chunk = (int)h->partial_count;
  for (int j = 0; j < nvecs; ++j) {
    char* v = Q + (size_t)j * fb;
    for (int pass = 0; pass < 2 && j > 0; ++pass) {
      for (int k0 = 0; k0 < j; k0 += chunk) {
        const int nk = j - k0 < chunk ? j - k0 : chunk;
        HIP_TRY(gs_multidot(h, P, Q + (size_t)k0 * fb, v, nk, h->coef + 2 * k0));
      }
      HIP_TRY(gs_multiaxpy(h, P, Q, v, j, h->coef));
      HIP_TRY(hipMemcpyAsync(cf.data(), h->coef, 2 * (size_t)j * sizeof(double), hipMemcpyDeviceToHost, h->stream));
      if (int rc = sync(h)) return rc;
      for (int k = 0; k < j; ++k) {
        R[((size_t)k * nvecs + j) * 2] += cf[2 * k];
        R[((size_t)k * nvecs + j) * 2 + 1] += cf[2 * k + 1];
      }
    }
    HIP_TRY(blas_dot(h, P, v, P, v, 1, S_TMP, false));
    if (int rc = read_scalars(h, 1, sc)) return rc;
    const double nrm = std::sqrt(sc[S_TMP]);
    if (!(nrm > 0) || !std::isfinite(nrm)) return fail(DWF_EBREAKDOWN, "dwf_gram_schmidt: vector %d is dependent", j);
    R[((size_t)j * nvecs + j) * 2] = nrm;
    HIP_TRY(blas_axpby(h, P, nullptr, P, v, 1, 0.0, 1.0 / nrm, -1, -1, 1));
  }
  if (int rc = sync(h)) return rc;
  if (R_host) std::memcpy(R_host, R.data(), R.size() * sizeof(double));
  return DWF_OK;
}

// ---------------------------------------------------------------------------
// Force
// ---------------------------------------------------------------------------
int dwf_force(dwf_handle h, const void* X_e, const void* Y_e, void* grad_U) {
  if (int r = check_h(h)) return r;
  if (!X_e || !Y_e || !grad_U) return fail(DWF_EINVAL, "dwf_force: null pointer");
  if (h->max_cg_rhs < 1) return fail(DWF_EINVAL, "dwf_force: handle was created without solver workspace");
  if (h->schur_form != 1) return fail(DWF_EINVAL, "dwf_force: needs the first Schur form");
  const char* X = reinterpret_cast<const char*>(X_e);
  const char* Y = reinterpret_cast<const char*>(Y_e);
  char* Z = h->t64;  // M5D^{-1} M_oe X      (odd)
  char* W = h->r64;  // M5D^{-dag} M_eo^dag Y (odd)
  HopArgs a{};
  a.in = X;
  a.out = Z;
  a.alpha = -0.5;
  HIP_TRY(launch_hop(h, DWF_F64, a, DWF_ODD, 0, EPI_M5INV, 1));
  HopArgs b{};
  b.in = Y;
  b.out = W;
  b.alpha = -0.5;
  HIP_TRY(launch_hop(h, DWF_F64, b, DWF_ODD, 1, EPI_M5INV, 1));
  HIP_TRY(launch_force(h, Y, W, X, Z, reinterpret_cast<double*>(grad_U)));
  return DWF_OK;
}

int dwf_lie_force(dwf_handle h, const void* U, const void* grad_U, void* F) {
  if (int r = check_h(h)) return r;
  if (!U || !grad_U || !F) return fail(DWF_EINVAL, "dwf_lie_force: null pointer");
  HIP_TRY(launch_lie_force(h, U, grad_U, reinterpret_cast<double*>(F)));
  return DWF_OK;
}

// ---------------------------------------------------------------------------
// Introspection
// ---------------------------------------------------------------------------
int dwf_set_tile(dwf_handle h, int sites_per_block, int pipeline_depth, int rhs_per_block) {
  if (int r = check_h(h)) return r;
  if (rhs_per_block < 0 || rhs_per_block > 64) return fail(DWF_EINVAL, "rhs_per_block must be in [0, 64]");
  if (rhs_per_block > 0) h->rpb = rhs_per_block;
  if (sites_per_block < 0 || sites_per_block * h->g.Ls > 256) return fail(DWF_EINVAL, "sites_per_block * Ls must be <= 256");
  if (pipeline_depth < 0 || pipeline_depth > 3) return fail(DWF_EINVAL, "pipeline_depth must be 0 (keep), 1, 2 or 3");
  h->spb = sites_per_block;
  if (pipeline_depth > 0) h->depth[h->prec] = h->depth[DWF_F64] = pipeline_depth;
  return DWF_OK;
}

// ---------------------------------------------------------------------------
// Coarse-space transfer (blocks, chirality split, block orthonormalisation,
// restriction, prolongation)
// ---------------------------------------------------------------------------
int dwf_set_blocks_ex(dwf_handle h, const int block[4], int parity, int* nblocks) {
  if (int r = check_h(h)) return r;
  if (!block) return fail(DWF_EINVAL, "dwf_set_blocks: block is NULL");
  if (parity != DWF_EVEN && parity != DWF_BOTH) return fail(DWF_EINVAL, "dwf_set_blocks: parity must be DWF_EVEN or DWF_BOTH");
  const bool both = parity == DWF_BOTH;
  const Geom& g = h->g;
  std::vector<int> tab, nbt;
  int nb = 0, nsb = 0;
  std::string why;
  if (!plan::build_blocks(g.X, g.Y, g.Z, g.T, g.Ls, block, both, tab, nbt, &nb, &nsb, &why))
    return fail(DWF_EINVAL, "dwf_set_blocks: %s", why.c_str());
  HIP_TRY(hipMemcpyAsync(h->bsite, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipMemcpyAsync(h->bnbr, nbt.data(), nbt.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  for (int i = 0; i < 4; ++i) h->blk[i] = block[i];
  h->nb = (int)nb;
  h->nsb = nsb;
  h->coarse_both = both ? 1 : 0;
  if (nblocks) *nblocks = (int)nb;
  return DWF_OK;
}

int dwf_set_blocks(dwf_handle h, const int block[4], int* nblocks) {
  return dwf_set_blocks_ex(h, block, DWF_EVEN, nblocks);
}

static int check_blocks(dwf_handle h, int nvec, const char* who) {
  if (int r = check_h(h)) return r;
  if (h->nb <= 0) return fail(DWF_EINVAL, "%s: call dwf_set_blocks first", who);
  if (nvec < 1 || nvec > 64) return fail(DWF_EINVAL, "%s: nvec must be in [1, 64]", who);
  return DWF_OK;
}

int dwf_chiral_split(dwf_handle h, const void* in, void* out, int nvec) {
  if (int r = check_h(h)) return r;
  if (!in || !out || in == out) return fail(DWF_EINVAL, "dwf_chiral_split: in and out must be distinct device pointers");
  if (nvec < 1) return fail(DWF_EINVAL, "dwf_chiral_split: nvec must be >= 1");
  HIP_TRY(launch_chiral_split(h, h->prec, reinterpret_cast<const char*>(in), reinterpret_cast<char*>(out), nvec));
  return DWF_OK;
}

size_t dwf_block_scratch_bytes(dwf_handle h, int nvec) {
  if (!h || h->nb <= 0 || nvec < 1 || nvec > 64) return 0;
  return 2 * up((size_t)h->nb * nvec * nvec * 16) + WS_ALIGN;
}

int dwf_block_orthonormalize(dwf_handle h, void* basis, int nvec, void* scratch, size_t scratch_bytes) {
  if (int r = check_blocks(h, nvec, "dwf_block_orthonormalize")) return r;
  if (!basis || !scratch) return fail(DWF_EINVAL, "dwf_block_orthonormalize: NULL pointer");
  if (scratch_bytes < dwf_block_scratch_bytes(h, nvec))
    return fail(DWF_ENOMEM, "dwf_block_orthonormalize: scratch of %zu bytes, %zu needed", scratch_bytes,
                dwf_block_scratch_bytes(h, nvec));
  char* base = reinterpret_cast<char*>(scratch);
  double* gram = reinterpret_cast<double*>(base);
  double* w = reinterpret_cast<double*>(base + up((size_t)h->nb * nvec * nvec * 16));
  int* flag = reinterpret_cast<int*>(base + 2 * up((size_t)h->nb * nvec * nvec * 16));
  char* q = reinterpret_cast<char*>(basis);
  HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), h->stream));
  for (int pass = 0; pass < 2; ++pass) {  // Cholesky QR, twice
    HIP_TRY(launch_block_gram(h, h->prec, q, nvec, gram));
    HIP_TRY(launch_block_cholesky(h, gram, w, nvec, flag));
    HIP_TRY(launch_block_apply(h, h->prec, q, nvec, w));
  }
  int hf = 0;
  HIP_TRY(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (hf) return fail(DWF_EBREAKDOWN, "dwf_block_orthonormalize: a block's vectors are linearly dependent");
  return DWF_OK;
}

int dwf_restrict(dwf_handle h, const void* basis, int nvec, const void* v, int nrhs, void* coarse) {
  if (int r = check_blocks(h, nvec, "dwf_restrict")) return r;
  if (!basis || !v || !coarse || nrhs < 1) return fail(DWF_EINVAL, "dwf_restrict: NULL pointer or nrhs < 1");
  HIP_TRY(launch_block_dot(h, h->prec, reinterpret_cast<const char*>(basis), nvec, reinterpret_cast<const char*>(v),
                           nrhs, reinterpret_cast<double*>(coarse), false));
  return DWF_OK;
}

int dwf_prolong(dwf_handle h, const void* basis, int nvec, const void* coarse, int nrhs, void* v) {
  if (int r = check_blocks(h, nvec, "dwf_prolong")) return r;
  if (!basis || !v || !coarse || nrhs < 1) return fail(DWF_EINVAL, "dwf_prolong: NULL pointer or nrhs < 1");
  if (v == basis) return fail(DWF_EINVAL, "dwf_prolong: v must not alias the basis");
  HIP_TRY(launch_block_prolong(h, h->prec, reinterpret_cast<const char*>(basis), nvec,
                               reinterpret_cast<const double*>(coarse), nrhs, reinterpret_cast<char*>(v)));
  return DWF_OK;
}

int dwf_set_schur_form(dwf_handle h, int form) {
  if (int r = check_h(h)) return r;
  if (form != 1 && form != 2) return fail(DWF_EINVAL, "dwf_set_schur_form: form must be 1 or 2");
  if (form != h->schur_form) h->lam_max = 0;  // another operator
  h->schur_form = form;
  return DWF_OK;
}

// CGNR on D_DW^dag D_DW over both parities (the Krylov table's unpreconditioned
// row), driven from the host: every both-parity vector is two half fields, so
// the BLAS calls run on nrhs = 2 and the two halves' dots are added here.
int dwf_solve_unprec(dwf_handle h, const void* eta, void* psi, double tol, int maxiter, int* iters, double* resid) {
  if (int r = check_h(h)) return r;
  if (!eta || !psi || eta == psi) return fail(DWF_EINVAL, "dwf_solve_unprec: eta and psi must be distinct");
  if (h->prec != DWF_F64) return fail(DWF_EINVAL, "dwf_solve_unprec: needs a DWF_F64 handle");
  if (h->max_cg_rhs < 2) return fail(DWF_EINVAL, "dwf_solve_unprec: needs max_cg_rhs >= 2 (two half fields per vector)");
  if (!(tol > 0) || maxiter < 0) return fail(DWF_EINVAL, "dwf_solve_unprec: tol must be > 0 and maxiter >= 0");
  char* x = reinterpret_cast<char*>(psi);
  char *b = h->b64, *r = h->r64, *p = h->p64, *q = h->q64, *w = h->t64;
  std::vector<double> sc;
  auto dot2 = [&](const char* u, const char* v, double& out) -> int {
    HIP_TRY(blas_dot(h, DWF_F64, u, DWF_F64, v, 2, S_TMP, false));
    if (int rc = read_scalars(h, 2, sc)) return rc;
    out = sc[S_TMP] + sc[NSCAL + S_TMP];
    return DWF_OK;
  };
  auto normal = [&](const char* v, char* out) -> int {  // out = D^dag D v, w = D v
    if (int rc = dwf_ddw(h, v, w, 1, 0)) return rc;
    return dwf_ddw(h, w, out, 1, 1);
  };
  if (int rc = dwf_ddw(h, eta, b, 1, 1)) return rc;  // b = D^dag eta
  double bb = 0, rr = 0, pap = 0;
  if (int rc = dot2(b, b, bb)) return rc;
  if (int rc = normal(x, q)) return rc;
  HIP_TRY(blas_copy(h, DWF_F64, b, DWF_F64, r, 2));
  HIP_TRY(blas_axpby(h, DWF_F64, q, DWF_F64, r, 2, -1.0, 1.0, -1, -1, 1));  // r = b - A x
  HIP_TRY(blas_copy(h, DWF_F64, r, DWF_F64, p, 2));
  if (int rc = dot2(r, r, rr)) return rc;
  const double tol2 = tol * tol;
  int it = 0, last = 0;
  bool stopped = false;
  while (bb > 0 && rr > tol2 * bb && it < maxiter) {
    if (int rc = normal(p, q)) return rc;
    if (int rc = dot2(w, w, pap)) return rc;  // p.A p = |D p|^2
    const double alpha = rr / pap;
    if (!(pap > 0) || !std::isfinite(alpha)) return fail(DWF_EBREAKDOWN, "dwf_solve_unprec: breakdown");
    HIP_TRY(blas_axpby(h, DWF_F64, p, DWF_F64, x, 2, alpha, 1.0, -1, -1, 1));
    HIP_TRY(blas_axpby(h, DWF_F64, q, DWF_F64, r, 2, -alpha, 1.0, -1, -1, 1));
    double rr_new = 0;
    if (int rc = dot2(r, r, rr_new)) return rc;
    ++it;
    if (h->progress_fn && it - last >= h->progress_every) {
      last = it;
      const double rel = std::sqrt(rr_new / bb);
      if (h->progress_fn(h->progress_user, it, 1, &rel)) {
        stopped = true;
        break;
      }
    }
    const double beta = rr_new / rr;
    rr = rr_new;
    HIP_TRY(blas_axpby(h, DWF_F64, r, DWF_F64, p, 2, 1.0, beta, -1, -1, 1));
  }
  // true residual of the normal equations
  if (int rc = normal(x, q)) return rc;
  HIP_TRY(blas_copy(h, DWF_F64, b, DWF_F64, r, 2));
  HIP_TRY(blas_axpby(h, DWF_F64, q, DWF_F64, r, 2, -1.0, 1.0, -1, -1, 1));
  double tr = 0;
  if (int rc = dot2(r, r, tr)) return rc;
  if (iters) *iters = it;
  const double rel = bb > 0 ? std::sqrt(tr / bb) : 0.0;
  if (resid) *resid = rel;
  if (!std::isfinite(rel)) return fail(DWF_EBREAKDOWN, "dwf_solve_unprec: non-finite residual");
  if (stopped) return fail(DWF_ENOCONV, "CG stopped by the progress callback");
  if (bb > 0 && rr > tol2 * bb) return fail(DWF_ENOCONV, "dwf_solve_unprec: no convergence in %d iterations", maxiter);
  return DWF_OK;
}

// Builds and uploads a traversal order (mode 0-2, or 3 with a box cut); false
// when the lattice does not admit it (nothing changes then).
static int apply_order(dwf_handle h, int mode, const int box[3], bool* ok) {
  *ok = true;
  if (mode == 0) {
    h->order_mode = 0;
    h->order_box[0] = h->order_box[1] = h->order_box[2] = 0;
    return DWF_OK;
  }
  std::vector<int> ord;
  const Geom& g = h->g;
  const bool built = mode == 3 ? plan::build_box_order(g.X, g.Y, g.Z, g.T, box[0], box[1], box[2], ord)
                               : plan::build_order(g.X, g.Y, g.Z, g.T, mode, ord);
  if (!built) {
    *ok = false;
    return DWF_OK;
  }
  HIP_TRY(hipMemcpyAsync(h->order, ord.data(), ord.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->order_mode = mode;
  for (int i = 0; i < 3; ++i) h->order_box[i] = mode == 3 ? box[i] : 0;
  return DWF_OK;
}

int dwf_set_order(dwf_handle h, int mode) {
  if (int r = check_h(h)) return r;
  if (mode < 0 || mode > 2) return fail(DWF_EINVAL, "traversal order %d unknown (0, 1, 2; boxes: dwf_set_order_box)", mode);
  const int none[3] = {0, 0, 0};
  bool ok = true;
  if (int rc = apply_order(h, mode, none, &ok)) return rc;
  if (!ok) return fail(DWF_EINVAL, "traversal order %d not available for this lattice", mode);
  h->order_explicit = 1;
  return DWF_OK;
}

int dwf_set_order_box(dwf_handle h, int nx, int ny, int nz) {
  if (int r = check_h(h)) return r;
  const int box[3] = {nx, ny, nz};
  bool ok = true;
  if (int rc = apply_order(h, 3, box, &ok)) return rc;
  if (!ok)
    return fail(DWF_EINVAL, "box cut %d x %d x %d does not divide the %d x %d x %d volume into boxes of even x extent",
                nx, ny, nz, h->g.X, h->g.Y, h->g.Z);
  h->order_explicit = 1;
  return DWF_OK;
}

int dwf_get_order(dwf_handle h, int* mode, int box[3]) {
  if (int r = check_h(h)) return r;
  if (mode) *mode = h->order_mode;
  if (box)
    for (int i = 0; i < 3; ++i) box[i] = h->order_box[i];
  return DWF_OK;
}

int dwf_set_progress(dwf_handle h, dwf_progress_fn fn, void* user, int every) {
  if (int r = check_h(h)) return r;
  if (fn && every < 1) return fail(DWF_EINVAL, "dwf_set_progress: every must be >= 1");
  h->progress_fn = fn;
  h->progress_user = user;
  h->progress_every = fn ? every : 0;
  return DWF_OK;
}

int dwf_set_occupancy(dwf_handle h, int workgroups_per_cu) {
  if (int r = check_h(h)) return r;
  if (workgroups_per_cu < 0 || workgroups_per_cu > 64) return fail(DWF_EINVAL, "workgroups_per_cu must be in [0, 64]");
  // 160 KiB of LDS per CU on gfx950; a launch asking for more than a 1/n share keeps at most n resident
  h->lds_floor = workgroups_per_cu ? (160 * 1024) / workgroups_per_cu - 1024 : 0;
  if (h->lds_floor > 64 * 1024) h->lds_floor = 64 * 1024;
  return DWF_OK;
}

// the tuning-cache key of a handle's current configuration
static int tune_key(dwf_handle h, int nrhs, plan::TuneKey* k) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  k->arch = prop.gcnArchName;
  for (char& ch : k->arch)
    if (ch == ' ' || ch == '\t') ch = '_';
  if (k->arch.empty()) k->arch = "unknown";
  k->dims[0] = h->g.X;
  k->dims[1] = h->g.Y;
  k->dims[2] = h->g.Z;
  k->dims[3] = h->g.T;
  k->Ls = h->g.Ls;
  k->nrhs = nrhs;
  k->prec = h->prec;
  // an order the caller set is part of the key; otherwise the tuner picks it (-1)
  k->order = h->order_explicit
                 ? h->order_mode + 4 * (h->order_box[0] + 64 * (h->order_box[1] + 64 * h->order_box[2]))
                 : -1;
  k->lds_floor = h->lds_floor;
  k->schur_form = h->schur_form;
  return DWF_OK;
}

static void apply_tile(dwf_handle h, int spb, int depth, int rpb) {
  h->spb = spb;
  h->depth[h->prec] = depth;
  h->rpb = rpb;
  if (h->prec != DWF_F64) h->depth[DWF_F64] = depth;
}

int dwf_tune_cache_clear(void) {
  plan::tune_clear();
  return DWF_OK;
}

// ms per M_pc^dag M_pc on nrhs zero fields in the handle's current launch shape and order
static int time_mdagm(dwf_handle h, char* v, int nrhs, int reps, hipEvent_t e0, hipEvent_t e1, double* per) {
  const int P = h->prec;
  for (int w = 0; w < 2; ++w) HIP_TRY(mdagm_chunk(h, P, v, v, h->t_buf, h->u_buf, nrhs));
  HIP_TRY(hipEventRecord(e0, h->stream));
  for (int k = 0; k < reps; ++k) HIP_TRY(mdagm_chunk(h, P, v, v, h->t_buf, h->u_buf, nrhs));
  HIP_TRY(hipEventRecord(e1, h->stream));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  *per = ms / reps;
  return DWF_OK;
}

// The traversal order (unless the caller set one), then the launch shape.
static int autotune_search(dwf_handle h, int nrhs, int reps, hipEvent_t e0, hipEvent_t e1, plan::TuneEntry* best) {
  const int P = h->prec;
  const int Ls = h->g.Ls;
  char* v = h->cheb_a;  // zero field; M_pc^dag M_pc maps it onto itself
  HIP_TRY(blas_zero(h, P, v, nrhs));
  best->order = h->order_mode;
  for (int i = 0; i < 3; ++i) best->box[i] = h->order_box[i];
  if (!h->order_explicit) {
    // stage 1: orders in a middle-sized shape
    apply_tile(h, std::max(1, 128 / Ls), 3, 1);
    double bms = 1e30;
    const int none[3] = {0, 0, 0};
    for (int c = -3; c < plan::NUM_BOX_CANDIDATES; ++c) {
      const int mode = c < 0 ? c + 3 : 3;
      if (mode == 3 && plan::BOX_CANDIDATES[c][0] == 2 && plan::BOX_CANDIDATES[c][1] == 2 &&
          plan::BOX_CANDIDATES[c][2] == 2)
        continue;  // the octants of mode 1
      const int* box = mode == 3 ? plan::BOX_CANDIDATES[c] : none;
      bool ok = true;
      if (int rc = apply_order(h, mode, box, &ok)) return rc;
      if (!ok) continue;
      double per = 0;
      if (int rc = time_mdagm(h, v, nrhs, reps, e0, e1, &per)) return rc;
      if (per < bms) {
        bms = per;
        best->order = mode;
        for (int i = 0; i < 3; ++i) best->box[i] = box[i];
      }
    }
    bool ok = true;
    if (int rc = apply_order(h, best->order, best->box, &ok)) return rc;
  }
  // stage 2: sites per workgroup, pipeline depth, rhs per workgroup
  best->spb = 0;
  best->ms = 1e30;
  for (int threads = 256; threads >= 64; threads /= 2) {
    const int spb = threads / Ls;
    if (spb < 1) continue;
    for (int cand = 0; cand < 12; ++cand) {
      const int depth = 1 + cand % 3;
      const int rpb = 1 << (cand / 3);
      if (rpb > nrhs) continue;
      apply_tile(h, spb, depth, rpb);
      double per = 0;
      if (int rc = time_mdagm(h, v, nrhs, reps, e0, e1, &per)) return rc;
      if (per < best->ms) {
        best->ms = per;
        best->spb = spb;
        best->depth = depth;
        best->rpb = rpb;
      }
    }
  }
  return DWF_OK;
}

int dwf_autotune(dwf_handle h, int nrhs, int reps, int* best_spb, int* best_depth, int* best_rpb, double* best_ms) {
  if (int r = check_h(h)) return r;
  if (nrhs < 1 || nrhs > h->max_nrhs || reps < 1) return fail(DWF_EINVAL, "dwf_autotune: nrhs in [1, max_nrhs], reps >= 1");
  const int P = h->prec;
  plan::TuneKey key;
  if (int rc = tune_key(h, nrhs, &key)) return rc;
  const char* cache_file = std::getenv("DWF_TUNE_CACHE");
  plan::TuneEntry best{};
  if (!plan::tune_lookup(key, &best, cache_file)) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const bool was_timing = h->timing;
    h->timing = false;
    const int old_spb = h->spb, old_depth = h->depth[P], old_rpb = h->rpb;
    const int rc = autotune_search(h, nrhs, reps, e0, e1, &best);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->timing = was_timing;
    if (rc) return rc;
    if (best.spb == 0) {
      apply_tile(h, old_spb, old_depth, old_rpb);
      return fail(DWF_EINVAL, "dwf_autotune: no candidate shape for Ls = %d", h->g.Ls);
    }
    plan::tune_store(key, best, cache_file);
  } else if (!h->order_explicit) {
    bool ok = true;
    if (int rc = apply_order(h, best.order, best.box, &ok)) return rc;
    if (!ok) return fail(DWF_EINVAL, "dwf_autotune: cached traversal order does not fit this lattice");
  }
  apply_tile(h, best.spb, best.depth, best.rpb);
  if (best_spb) *best_spb = best.spb;
  if (best_depth) *best_depth = best.depth;
  if (best_rpb) *best_rpb = best.rpb;
  if (best_ms) *best_ms = best.ms;
  return DWF_OK;
}

int dwf_enable_timing(dwf_handle h, int enable) {
  if (int r = check_h(h)) return r;
  if (enable < 0) return fail(DWF_EINVAL, "dwf_enable_timing: enable must be >= 0");
  if (enable && h->ev_pool.empty()) {
    h->ev_pool.resize(4096);
    for (auto& p : h->ev_pool) {
      HIP_TRY(hipEventCreate(&p.a));
      HIP_TRY(hipEventCreate(&p.b));
    }
  }
  h->timing = enable != 0;
  h->ev_stride = enable > 1 ? enable : 1;
  h->ev_seq = 0;
  h->ev_open = false;
  h->ev_used = 0;
  h->ev_ms = 0;
  h->ev_launches = 0;
  return DWF_OK;
}

int dwf_kernel_time(dwf_handle h, double* ms_total, long long* launches) {
  if (int r = check_h(h)) return r;
  if (h->timing && h->ev_used > 0) {
    if (int rc = sync(h)) return rc;
    for (size_t i = 0; i < h->ev_used; ++i) {
      float ms = 0;
      HIP_TRY(hipEventElapsedTime(&ms, h->ev_pool[i].a, h->ev_pool[i].b));
      h->ev_ms += ms;
    }
    h->ev_launches += (long long)h->ev_used;
    h->ev_used = 0;
  }
  if (ms_total) *ms_total = h->ev_ms;
  if (launches) *launches = h->ev_launches;
  return DWF_OK;
}

}  // extern "C"
