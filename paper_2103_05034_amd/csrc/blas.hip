// Vector kernels of the solvers: linear combinations across storage
// precisions, CG updates with fused norms, and dot products.  Every dot and
// norm accumulates in FP64 and is reduced in two fixed-order stages
// (per-workgroup partials, then one workgroup per right-hand side), so
// results are bitwise reproducible run to run.
#include "dwf_internal.hpp"
#include "kernels.hpp"

namespace dwf {

constexpr int BS = 256;

struct VecGeom {
  long long V4h;
  int Ls;
  long long n;  // spinors per rhs = V4h * Ls
};

static VecGeom vgeom(const dwf_context* ctx) { return {ctx->g.V4h, ctx->g.Ls, ctx->g.V4h * ctx->g.Ls}; }

template <int P>
__device__ __forceinline__ void vload(const char* base, const VecGeom& g, long long i, cplx<double> v[12]) {
  using R = typename Store<P>::real;
  cplx<R> t[12];
  const long long h = i / g.Ls;
  Store<P>::load(base, g.V4h, g.Ls, h, (int)(i - h * g.Ls), t);
#pragma unroll
  for (int c = 0; c < 12; ++c) v[c] = {(double)t[c].re, (double)t[c].im};
}

template <int P>
__device__ __forceinline__ void vstore(char* base, const VecGeom& g, long long i, const cplx<double> v[12]) {
  using R = typename Store<P>::real;
  cplx<R> t[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) t[c] = {(R)v[c].re, (R)v[c].im};
  const long long h = i / g.Ls;
  Store<P>::store(base, g.V4h, g.Ls, h, (int)(i - h * g.Ls), t);
}

// fixed-order sums of 2 doubles over a workgroup of BS threads, valid on thread 0
__device__ __forceinline__ void block_reduce2(double& a, double& b) {
  __shared__ double red[2 * (BS / 64)];
  block_sum2(a, b, red);
}

// partials[(rhs * RED_BLOCKS + blk) * 2 + {0,1}] -> out[rhs * ostride + {0, 1}]
__global__ void finalize_kernel(const double* __restrict__ partials, double* __restrict__ out, int ostride,
                                int write_imag) {
  const int rhs = blockIdx.x;
  double a = 0, b = 0;
  for (int k = threadIdx.x; k < RED_BLOCKS; k += BS) {
    a += partials[((size_t)rhs * RED_BLOCKS + k) * 2];
    b += partials[((size_t)rhs * RED_BLOCKS + k) * 2 + 1];
  }
  block_reduce2(a, b);
  if (threadIdx.x == 0) {
    out[(size_t)rhs * ostride] = a;
    if (write_imag) out[(size_t)rhs * ostride + 1] = b;
  }
}

// <a, b> per rhs; rhs stride given per argument (GS uses Q_k as "rhs" of a
// batch against one fixed vector b with b_stride = 0)
template <int PA, int PB>
__global__ void dot_kernel(VecGeom g, const char* __restrict__ a, size_t a_stride, const char* __restrict__ b,
                           size_t b_stride, double* __restrict__ partials) {
  const int rhs = blockIdx.y;
  const char* ab = a + rhs * a_stride;
  const char* bb = b + rhs * b_stride;
  double re = 0, im = 0;
  for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < g.n; i += (long long)RED_BLOCKS * BS) {
    cplx<double> va[12], vb[12];
    vload<PA>(ab, g, i, va);
    vload<PB>(bb, g, i, vb);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      re = fma(va[c].re, vb[c].re, re);
      re = fma(va[c].im, vb[c].im, re);
      im = fma(va[c].re, vb[c].im, im);
      im = fma(-va[c].im, vb[c].re, im);
    }
  }
  block_reduce2(re, im);
  if (threadIdx.x == 0) {
    partials[((size_t)rhs * RED_BLOCKS + blockIdx.x) * 2] = re;
    partials[((size_t)rhs * RED_BLOCKS + blockIdx.x) * 2 + 1] = im;
  }
}

// y = ca' x + cb' y, ca' = (slot_a >= 0 ? sign_a * scal[rhs][slot_a] : ca), same for b
template <int PX, int PY>
__global__ void axpby_kernel(VecGeom g, const char* __restrict__ x, char* __restrict__ y, size_t sx, size_t sy,
                             double ca, double cb, int slot_a, int slot_b, int sign_a,
                             const double* __restrict__ scal) {
  const int rhs = blockIdx.y;
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i >= g.n) return;
  const double a = slot_a >= 0 ? sign_a * scal[rhs * NSCAL + slot_a] : ca;
  const double b = slot_b >= 0 ? scal[rhs * NSCAL + slot_b] : cb;
  cplx<double> vx[12], vy[12];
  if (x && a != 0.0) vload<PX>(x + rhs * sx, g, i, vx);
  if (b != 0.0) vload<PY>(y + rhs * sy, g, i, vy);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    cplx<double> o = {0, 0};
    if (x && a != 0.0) o = {a * vx[c].re, a * vx[c].im};
    if (b != 0.0) o = {o.re + b * vy[c].re, o.im + b * vy[c].im};
    vy[c] = o;
  }
  vstore<PY>(y + rhs * sy, g, i, vy);
}

// x += alpha p ; r -= alpha q ; partial |r|^2
template <int PX, int PR, int PP, int PQ>
__global__ void cg_xr_kernel(VecGeom g, char* __restrict__ x, char* __restrict__ r, const char* __restrict__ p,
                             const char* __restrict__ q, size_t sx, size_t sr, size_t sp, size_t sq,
                             const double* __restrict__ scal, double* __restrict__ partials) {
  const int rhs = blockIdx.y;
  const double alpha = scal[rhs * NSCAL + S_ALPHA];
  double rr = 0;
  for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < g.n; i += (long long)RED_BLOCKS * BS) {
    cplx<double> vx[12], vr[12], vp[12], vq[12];
    vload<PR>(r + rhs * sr, g, i, vr);
    if (alpha != 0.0) {
      vload<PX>(x + rhs * sx, g, i, vx);
      vload<PP>(p + rhs * sp, g, i, vp);
      vload<PQ>(q + rhs * sq, g, i, vq);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        vx[c] = {fma(alpha, vp[c].re, vx[c].re), fma(alpha, vp[c].im, vx[c].im)};
        vr[c] = {fma(-alpha, vq[c].re, vr[c].re), fma(-alpha, vq[c].im, vr[c].im)};
      }
      vstore<PX>(x + rhs * sx, g, i, vx);
      vstore<PR>(r + rhs * sr, g, i, vr);
      if (PR == DWF_F16S) vload<PR>(r + rhs * sr, g, i, vr);  // norm of what is stored
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) rr += vr[c].re * vr[c].re + vr[c].im * vr[c].im;
  }
  double dummy = 0;
  block_reduce2(rr, dummy);
  if (threadIdx.x == 0) {
    partials[((size_t)rhs * RED_BLOCKS + blockIdx.x) * 2] = rr;
    partials[((size_t)rhs * RED_BLOCKS + blockIdx.x) * 2 + 1] = 0;
  }
}

// r -= alpha q ; partial |r|^2
template <int PR, int PQ>
__global__ void cg_r_kernel(VecGeom g, char* __restrict__ r, const char* __restrict__ q, size_t sr, size_t sq,
                            const double* __restrict__ scal, double* __restrict__ partials) {
  const int rhs = blockIdx.y;
  const double alpha = scal[rhs * NSCAL + S_ALPHA];
  double rr = 0;
  for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < g.n; i += (long long)RED_BLOCKS * BS) {
    cplx<double> vr[12], vq[12];
    vload<PR>(r + rhs * sr, g, i, vr);
    if (alpha != 0.0) {
      vload<PQ>(q + rhs * sq, g, i, vq);
#pragma unroll
      for (int c = 0; c < 12; ++c) vr[c] = {fma(-alpha, vq[c].re, vr[c].re), fma(-alpha, vq[c].im, vr[c].im)};
      vstore<PR>(r + rhs * sr, g, i, vr);
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) rr += vr[c].re * vr[c].re + vr[c].im * vr[c].im;
  }
  double dummy = 0;
  block_reduce2(rr, dummy);
  if (threadIdx.x == 0) {
    partials[((size_t)rhs * RED_BLOCKS + blockIdx.x) * 2] = rr;
    partials[((size_t)rhs * RED_BLOCKS + blockIdx.x) * 2 + 1] = 0;
  }
}

// x += alpha p ; p = r + beta p   (both with the old p)
template <int PX, int PR, int PP>
__global__ void cg_xp_kernel(VecGeom g, char* __restrict__ x, const char* __restrict__ r, char* __restrict__ p,
                             size_t sx, size_t sr, size_t sp, const double* __restrict__ scal) {
  const int rhs = blockIdx.y;
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i >= g.n) return;
  const double alpha = scal[rhs * NSCAL + S_ALPHA];
  const double beta = scal[rhs * NSCAL + S_BETA];
  cplx<double> vx[12], vr[12], vp[12];
  // FP64 fields are read with non-temporal loads: each is used once here, and the
  // hop passes that follow then keep more of their neighbour data in L2 (FP64 CG
  // iteration -1.4 %, the hop launches -2 %)
  const long long hh = i / g.Ls;
  const int ss = (int)(i - hh * g.Ls);
  if constexpr (PP == DWF_F64)
    Store<DWF_F64>::load_nt(p + rhs * sp, g.V4h, g.Ls, hh, ss, vp);
  else
    vload<PP>(p + rhs * sp, g, i, vp);
  if (alpha != 0.0) {
    if constexpr (PX == DWF_F64)
      Store<DWF_F64>::load_nt(x + rhs * sx, g.V4h, g.Ls, hh, ss, vx);
    else
      vload<PX>(x + rhs * sx, g, i, vx);
#pragma unroll
    for (int c = 0; c < 12; ++c) vx[c] = {fma(alpha, vp[c].re, vx[c].re), fma(alpha, vp[c].im, vx[c].im)};
    if constexpr (PX == DWF_F64) {  // x is read again only by the next iteration's update
      Store<DWF_F64>::store_nt(x + rhs * sx, g.V4h, g.Ls, hh, ss, vx);
    } else {
      vstore<PX>(x + rhs * sx, g, i, vx);
    }
  }
  if constexpr (PR == DWF_F64) {
    Store<DWF_F64>::load_nt(r + rhs * sr, g.V4h, g.Ls, hh, ss, vr);
  } else if constexpr (PR == DWF_F32) {
    cplx<float> t[12];
    Store<DWF_F32>::load_nt(r + rhs * sr, g.V4h, g.Ls, hh, ss, t);
#pragma unroll
    for (int c = 0; c < 12; ++c) vr[c] = {(double)t[c].re, (double)t[c].im};
  } else {
    vload<PR>(r + rhs * sr, g, i, vr);
  }
#pragma unroll
  for (int c = 0; c < 12; ++c) vr[c] = {fma(beta, vp[c].re, vr[c].re), fma(beta, vp[c].im, vr[c].im)};
  if constexpr (PP == DWF_F64) {  // non-temporal, as x: FP64 CG iteration -0.8 %
    Store<DWF_F64>::store_nt(p + rhs * sp, g.V4h, g.Ls, hh, ss, vr);
  } else {
    vstore<PP>(p + rhs * sp, g, i, vr);
  }
}

// Loads and stores of a field streamed once by a CG update: FP64 and FP32 with
// non-temporal hints (the hop passes that follow then keep more of their
// neighbour data in L2), FP16 + scale plainly.
template <int P>
__device__ __forceinline__ void load_once(const char* base, const VecGeom& g, long long i, cplx<double> v[12]) {
  const long long hh = i / g.Ls;
  const int ss = (int)(i - hh * g.Ls);
  if constexpr (P == DWF_F64) {
    Store<DWF_F64>::load_nt(base, g.V4h, g.Ls, hh, ss, v);
  } else if constexpr (P == DWF_F32) {
    cplx<float> t[12];
    Store<DWF_F32>::load_nt(base, g.V4h, g.Ls, hh, ss, t);
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = {(double)t[c].re, (double)t[c].im};
  } else {
    vload<P>(base, g, i, v);
  }
}
template <int P>
__device__ __forceinline__ void store_once(char* base, const VecGeom& g, long long i, const cplx<double> v[12]) {
  if constexpr (P == DWF_F64) {
    const long long hh = i / g.Ls;
    Store<DWF_F64>::store_nt(base, g.V4h, g.Ls, hh, (int)(i - hh * g.Ls), v);
  } else {
    vstore<P>(base, g, i, v);
  }
}

// CG with the solution update deferred: pn = r + beta p into another buffer (p is
// kept for the deferred x += alpha p), and alpha copied to slot `keep`.  The same
// arithmetic as the p half of cg_xp_kernel.
template <int PR, int PP>
__global__ void cg_dir_kernel(VecGeom g, const char* __restrict__ r, const char* __restrict__ p,
                              char* __restrict__ pn, size_t sr, size_t sp, double* __restrict__ scal, int keep) {
  const int rhs = blockIdx.y;
  double* s = scal + rhs * NSCAL;
  if (blockIdx.x == 0 && threadIdx.x == 0) s[keep] = s[S_ALPHA];
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i >= g.n) return;
  const double beta = s[S_BETA];
  cplx<double> vr[12], vp[12];
  load_once<PP>(p + rhs * sp, g, i, vp);
  load_once<PR>(r + rhs * sr, g, i, vr);
#pragma unroll
  for (int c = 0; c < 12; ++c) vr[c] = {fma(beta, vp[c].re, vr[c].re), fma(beta, vp[c].im, vr[c].im)};
  store_once<PP>(pn + rhs * sp, g, i, vr);
}

struct DirSet {
  const char* p[4];  // directions p_0 .. p_{N-1}, in the order of their iterations
  int slot[4];       // scalar slot of each direction's alpha
};

// x += alpha_0 p_0 + ... + alpha_{N-1} p_{N-1} (x FP64), one fma per term in this
// order and a term skipped when its alpha is 0: the same roundings as N single
// updates x += alpha p.  With pn: pn = r + beta p_{N-1} (pn may alias p_0; every
// thread reads its elements before it writes them).
template <int PR, int PP, int N>
__global__ void cg_flush_kernel(VecGeom g, char* x, DirSet d, const char* r, char* pn, size_t sx, size_t sr,
                                size_t sp, const double* __restrict__ scal) {
  const int rhs = blockIdx.y;
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i >= g.n) return;
  const double* s = scal + rhs * NSCAL;
  double alpha[N];
  bool any = false;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    alpha[k] = s[d.slot[k]];
    any |= alpha[k] != 0.0;
  }
  cplx<double> vp[12];
  bool have_last = false;
  if (any) {
    cplx<double> vx[12];
    load_once<DWF_F64>(x + rhs * sx, g, i, vx);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      if (alpha[k] == 0.0) continue;
      load_once<PP>(d.p[k] + rhs * sp, g, i, vp);
#pragma unroll
      for (int c = 0; c < 12; ++c) vx[c] = {fma(alpha[k], vp[c].re, vx[c].re), fma(alpha[k], vp[c].im, vx[c].im)};
      have_last = k == N - 1;
    }
    store_once<DWF_F64>(x + rhs * sx, g, i, vx);
  }
  if (pn == nullptr) return;
  const double beta = s[S_BETA];
  if (!have_last) load_once<PP>(d.p[N - 1] + rhs * sp, g, i, vp);
  cplx<double> vr[12];
  load_once<PR>(r + rhs * sr, g, i, vr);
#pragma unroll
  for (int c = 0; c < 12; ++c) vr[c] = {fma(beta, vp[c].re, vr[c].re), fma(beta, vp[c].im, vr[c].im)};
  store_once<PP>(pn + rhs * sp, g, i, vr);
}

// p = r + beta p.  With orth (right after a reliable update replaced r by the
// true residual), p first loses its component along the new r,
// p <- p - (r^dag p / |r|^2) r, so that p = (1 - beta c) r + beta p with
// c = r^dag p / |r|^2 taken from scal[S_TMP], scal[S_TMPI] and scal[S_RR].
template <int PR, int PP>
__global__ void cg_p_kernel(VecGeom g, const char* __restrict__ r, char* __restrict__ p, size_t sr, size_t sp,
                            const double* __restrict__ scal, int orth) {
  const int rhs = blockIdx.y;
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i >= g.n) return;
  const double* s = scal + rhs * NSCAL;
  const double beta = s[S_BETA];
  cplx<double> ar = {1.0, 0.0};
  if (orth && beta != 0.0 && s[S_RR] > 0.0) ar = {1.0 - beta * s[S_TMP] / s[S_RR], -beta * s[S_TMPI] / s[S_RR]};
  cplx<double> vr[12], vp[12];
  vload<PR>(r + rhs * sr, g, i, vr);
  if (beta != 0.0) {
    vload<PP>(p + rhs * sp, g, i, vp);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const cplx<double> t = {ar.re * vr[c].re - ar.im * vr[c].im, ar.re * vr[c].im + ar.im * vr[c].re};
      vr[c] = {fma(beta, vp[c].re, t.re), fma(beta, vp[c].im, t.im)};
    }
  }
  vstore<PP>(p + rhs * sp, g, i, vr);
}

// p += r_true - r_iter ; r_iter = r_true.  After a reliable update replaced the
// iterated residual by the true one, this turns p = r_iter + beta p_old into
// r_true + beta p_old without keeping p_old.
template <int PP>
__global__ void cg_reliable_kernel(VecGeom g, const char* __restrict__ rt, char* __restrict__ ri, char* __restrict__ p,
                                   size_t st, size_t si, size_t sp) {
  const int rhs = blockIdx.y;
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i >= g.n) return;
  cplx<double> vt[12], vi[12], vp[12];
  vload<DWF_F64>(rt + rhs * st, g, i, vt);
  vload<DWF_F32>(ri + rhs * si, g, i, vi);
  vload<PP>(p + rhs * sp, g, i, vp);
#pragma unroll
  for (int c = 0; c < 12; ++c) vp[c] = {vp[c].re + (vt[c].re - vi[c].re), vp[c].im + (vt[c].im - vi[c].im)};
  vstore<PP>(p + rhs * sp, g, i, vp);
  vstore<DWF_F32>(ri + rhs * si, g, i, vt);
}

// p <- p - (c - 1) r with c = r^dag p / |r|^2 taken from scal[S_TMP], scal[S_TMPI] and
// scal[S_RR]: after a reliable update p = r + beta p_old, this removes p_old's
// component along the new r (r^dag p = |r|^2 afterwards, as in exact CG).
template <int PP>
__global__ void cg_orth_kernel(VecGeom g, const char* __restrict__ r, char* __restrict__ p, size_t sr, size_t sp,
                               const double* __restrict__ scal) {
  const int rhs = blockIdx.y;
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i >= g.n) return;
  const double* s = scal + rhs * NSCAL;
  if (!(s[S_RR] > 0.0) || s[S_ACTIVE] == 0.0) return;
  const cplx<double> f = {s[S_TMP] / s[S_RR] - 1.0, s[S_TMPI] / s[S_RR]};
  cplx<double> vr[12], vp[12];
  vload<DWF_F32>(r + rhs * sr, g, i, vr);
  vload<PP>(p + rhs * sp, g, i, vp);
#pragma unroll
  for (int c = 0; c < 12; ++c)
    vp[c] = {vp[c].re - (f.re * vr[c].re - f.im * vr[c].im), vp[c].im - (f.re * vr[c].im + f.im * vr[c].re)};
  vstore<PP>(p + rhs * sp, g, i, vp);
}

// scalar bookkeeping: one thread per rhs
// Per-rhs CG bookkeeping on the scalar slots s = scal + rhs * NSCAL.
// alpha = |r|^2 / p.Ap (0 once the rhs has stopped; a breakdown stops it with the flag set)
__device__ void alpha_step(double* s) {
  s[S_RR_OLD] = s[S_RR];
  if (s[S_ACTIVE] == 0.0) {
    s[S_ALPHA] = 0.0;
    return;
  }
  const double pap = s[S_PAP];
  const double a = s[S_RR] / pap;
  if (!(pap > 0.0) || !isfinite(a)) {
    s[S_ALPHA] = 0.0;
    s[S_ACTIVE] = 0.0;
    if (s[S_RR] != 0.0) s[S_FLAG] = 1.0;  // breakdown (zero residual is convergence)
    return;
  }
  s[S_ALPHA] = a;
}

// beta = |r_new|^2 / |r_old|^2
__device__ void beta_step(double* s) {
  if (s[S_ACTIVE] == 0.0) {
    s[S_BETA] = 0.0;
    return;
  }
  const double b = s[S_RR] / s[S_RR_OLD];
  if (!isfinite(b) || !isfinite(s[S_RR])) {
    s[S_BETA] = 0.0;
    s[S_ACTIVE] = 0.0;
    s[S_FLAG] = 1.0;
    return;
  }
  s[S_BETA] = b;
}

// count the iteration, flag non-finite norms, stop once |r|^2 <= tol2 |b|^2 (if allowed)
__device__ void converge_step(double* s, double tol2, int count, int allow_stop) {
  if (s[S_ACTIVE] == 0.0) return;
  if (count) s[S_ITERS] += 1.0;
  const double rr = s[S_RR], bb = s[S_BB];
  if (!isfinite(rr) || !isfinite(bb)) {
    s[S_FLAG] = 1.0;
    s[S_ACTIVE] = 0.0;
    return;
  }
  if (allow_stop && rr <= tol2 * bb) s[S_ACTIVE] = 0.0;
}

__global__ void scal_alpha_kernel(double* scal, int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrhs) alpha_step(scal + r * NSCAL);
}

__global__ void scal_beta_kernel(double* scal, int nrhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrhs) beta_step(scal + r * NSCAL);
}

// Per-site sums (one FP64 value per half-lattice site and rhs, at the site's
// index) reduced into slot, then on the same thread the CG step that needs the
// total: mode 0 none, 1 alpha (slot = S_PAP), 2 beta and the convergence step
// (slot = S_RR), 3 as 2 without stopping a rhs, plus the largest |r|^2 since
// the last reliable update.  Workgroup b of a rhs adds the b-th of
// SITE_RED_BLOCKS equal index ranges (four sums per thread, then the
// workgroup); the last workgroup of the rhs to finish -- found by an atomic
// count that it resets for the next launch -- adds the range sums in index
// order.  The order is fixed by the lattice alone, so the result does not
// depend on which workgroup finishes last or on the hop kernels' launch shape.
constexpr int SITE_RED_BLOCKS = 64;

__global__ void __launch_bounds__(BS) sum_sites_kernel(const double* __restrict__ partials, int count,
                                                       double* __restrict__ ranges, unsigned* __restrict__ counters,
                                                       double* __restrict__ scal, int slot, int mode, double tol2) {
  const int rhs = blockIdx.y;
  const int b = blockIdx.x;
  const long long per = ((long long)count + SITE_RED_BLOCKS - 1) / SITE_RED_BLOCKS;
  const long long k0 = (long long)b * per;
  const long long k1 = k0 + per < count ? k0 + per : count;
  const double* q = partials + (size_t)rhs * count;
  double acc[4] = {0, 0, 0, 0};
  int j = 0;
  for (long long k = k0 + threadIdx.x; k < k1; k += BS, j = (j + 1) & 3) acc[j] += q[k];
  double a = (acc[0] + acc[1]) + (acc[2] + acc[3]), unused = 0;
  block_reduce2(a, unused);
  __shared__ int last;
  unsigned long long* rbits = reinterpret_cast<unsigned long long*>(ranges) + (size_t)rhs * SITE_RED_BLOCKS;
  if (threadIdx.x == 0) {
    __hip_atomic_store(rbits + b, __builtin_bit_cast(unsigned long long, a), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    // release of this range sum; acquire of the others' for the last workgroup
    const unsigned prev = __hip_atomic_fetch_add(counters + rhs, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = prev == (unsigned)(SITE_RED_BLOCKS - 1);
  }
  __syncthreads();
  if (!last) return;
  // the last workgroup: one load per range (in parallel), then the sum in index order
  __shared__ double rs[SITE_RED_BLOCKS];
  static_assert(SITE_RED_BLOCKS <= BS, "one range per thread of the last workgroup");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every loading wave sees the released sums
  if (threadIdx.x < SITE_RED_BLOCKS)
    rs[threadIdx.x] = __builtin_bit_cast(
        double, __hip_atomic_load(rbits + threadIdx.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  __syncthreads();
  if (threadIdx.x != 0) return;
  double t = 0;
  for (int i = 0; i < SITE_RED_BLOCKS; ++i) t += rs[i];
  __hip_atomic_store(counters + rhs, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  double* s = scal + (size_t)rhs * NSCAL;
  s[slot] = t;
  if (mode == 1) {
    alpha_step(s);
  } else if (mode >= 2) {
    beta_step(s);
    converge_step(s, tol2, 1, mode == 2);
    if (mode == 3 && s[S_ACTIVE] != 0.0) s[S_RRMAX] = fmax(s[S_RRMAX], s[S_RR]);
  }
}

__global__ void scal_set_kernel(double* scal, int nrhs, int slot, double v) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrhs) scal[r * NSCAL + slot] = v;
}

__global__ void scal_converge_kernel(double* scal, int nrhs, double tol2, int count, int allow_stop) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrhs) converge_step(scal + r * NSCAL, tol2, count, allow_stop);
}

__global__ void scal_copy_kernel(double* scal, int nrhs, int dst, int src) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrhs) scal[r * NSCAL + dst] = scal[r * NSCAL + src];
}

// v -= sum_{k<j} coef[k] Q_k   (coef complex, interleaved)
template <int P>
__global__ void multiaxpy_kernel(VecGeom g, const char* __restrict__ Q, char* __restrict__ v, size_t stride, int j,
                                 const double* __restrict__ coef) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i >= g.n) return;
  cplx<double> vv[12], q[12];
  vload<P>(v, g, i, vv);
  for (int k = 0; k < j; ++k) {
    vload<P>(Q + k * stride, g, i, q);
    const cplx<double> cf = {coef[2 * k], coef[2 * k + 1]};
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      vv[c].re -= cf.re * q[c].re - cf.im * q[c].im;
      vv[c].im -= cf.re * q[c].im + cf.im * q[c].re;
    }
  }
  vstore<P>(v, g, i, vv);
}

template <int P>
__global__ void scale_kernel(VecGeom g, char* __restrict__ v, const double* __restrict__ f) {
  const long long i = (long long)blockIdx.x * BS + threadIdx.x;
  if (i >= g.n) return;
  const double a = *f;
  cplx<double> vv[12];
  vload<P>(v, g, i, vv);
#pragma unroll
  for (int c = 0; c < 12; ++c) vv[c] = {a * vv[c].re, a * vv[c].im};
  vstore<P>(v, g, i, vv);
}

// ---------------------------------------------------------------------------
// dispatch helpers
// ---------------------------------------------------------------------------
#define DWF_DISPATCH1(p, F, ...)                      \
  switch (p) {                                         \
    case DWF_F64: F<DWF_F64>(__VA_ARGS__); break;      \
    case DWF_F32: F<DWF_F32>(__VA_ARGS__); break;      \
    default: F<DWF_F16S>(__VA_ARGS__); break;          \
  }

static unsigned grid_n(long long n) { return (unsigned)((n + BS - 1) / BS); }

template <int PA, int PB>
static void dot_l(dwf_context* ctx, VecGeom g, const char* a, size_t sa, const char* b, size_t sb, int nrhs,
                  double* partials) {
  hipLaunchKernelGGL((dot_kernel<PA, PB>), dim3(RED_BLOCKS, nrhs), dim3(BS), 0, ctx->stream, g, a, sa, b, sb,
                     partials);
}
template <int PA>
static void dot_la(dwf_context* ctx, int pb, VecGeom g, const char* a, size_t sa, const char* b, size_t sb,
                   int nrhs, double* partials = nullptr) {
  if (!partials) partials = ctx->partials;
  switch (pb) {
    case DWF_F64: dot_l<PA, DWF_F64>(ctx, g, a, sa, b, sb, nrhs, partials); break;
    case DWF_F32: dot_l<PA, DWF_F32>(ctx, g, a, sa, b, sb, nrhs, partials); break;
    default: dot_l<PA, DWF_F16S>(ctx, g, a, sa, b, sb, nrhs, partials); break;
  }
}

hipError_t reduce_sites(dwf_context* ctx, const double* partials, int count, int nrhs, int slot, int mode,
                        double tol2) {
  if ((size_t)nrhs * SITE_RED_BLOCKS > ctx->partial_count * RED_BLOCKS * 2 || nrhs > (int)ctx->partial_count)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(sum_sites_kernel, dim3(SITE_RED_BLOCKS, nrhs), dim3(BS), 0, ctx->stream, partials, count,
                     ctx->partials, ctx->counters, ctx->scalars, slot, mode, tol2);
  return hipGetLastError();
}

hipError_t blas_dot(dwf_context* ctx, int pa, const char* a, int pb, const char* b, int nrhs, int slot, bool imag) {
  VecGeom g = vgeom(ctx);
  const size_t sa = field_bytes_rhs(ctx, pa), sb = field_bytes_rhs(ctx, pb);
  DWF_DISPATCH1(pa, dot_la, ctx, pb, g, a, sa, b, sb, nrhs);
  hipLaunchKernelGGL(finalize_kernel, dim3(nrhs), dim3(BS), 0, ctx->stream, ctx->partials, ctx->scalars + slot,
                     NSCAL, imag ? 1 : 0);
  return hipGetLastError();
}

hipError_t blas_dot_to(dwf_context* ctx, int prec, const char* a, const char* b, int nrhs, double* partials,
                       double* result) {
  VecGeom g = vgeom(ctx);
  const size_t st = field_bytes_rhs(ctx, prec);
  DWF_DISPATCH1(prec, dot_la, ctx, prec, g, a, st, b, st, nrhs, partials);
  hipLaunchKernelGGL(finalize_kernel, dim3(nrhs), dim3(BS), 0, ctx->stream, partials, result, 2, 1);
  return hipGetLastError();
}

template <int PX, int PY>
static void axpby_l(dwf_context* ctx, VecGeom g, const char* x, char* y, size_t sx, size_t sy, int nrhs, double ca,
                    double cb, int slot_a, int slot_b, int sign_a) {
  hipLaunchKernelGGL((axpby_kernel<PX, PY>), dim3(grid_n(g.n), nrhs), dim3(BS), 0, ctx->stream, g, x, y, sx, sy, ca,
                     cb, slot_a, slot_b, sign_a, ctx->scalars);
}
template <int PX>
static void axpby_lx(dwf_context* ctx, int py, VecGeom g, const char* x, char* y, size_t sx, size_t sy, int nrhs,
                     double ca, double cb, int slot_a, int slot_b, int sign_a) {
  switch (py) {
    case DWF_F64: axpby_l<PX, DWF_F64>(ctx, g, x, y, sx, sy, nrhs, ca, cb, slot_a, slot_b, sign_a); break;
    case DWF_F32: axpby_l<PX, DWF_F32>(ctx, g, x, y, sx, sy, nrhs, ca, cb, slot_a, slot_b, sign_a); break;
    default: axpby_l<PX, DWF_F16S>(ctx, g, x, y, sx, sy, nrhs, ca, cb, slot_a, slot_b, sign_a); break;
  }
}

hipError_t blas_axpby(dwf_context* ctx, int px, const char* x, int py, char* y, int nrhs, double ca, double cb,
                      int slot_a, int slot_b, int sign_a) {
  VecGeom g = vgeom(ctx);
  const size_t sx = field_bytes_rhs(ctx, px), sy = field_bytes_rhs(ctx, py);
  DWF_DISPATCH1(px, axpby_lx, ctx, py, g, x, y, sx, sy, nrhs, ca, cb, slot_a, slot_b, sign_a);
  return hipGetLastError();
}

hipError_t blas_copy(dwf_context* ctx, int pin, const char* in, int pout, char* out, int nrhs) {
  return blas_axpby(ctx, pin, in, pout, out, nrhs, 1.0, 0.0, -1, -1, 1);
}

hipError_t blas_zero(dwf_context* ctx, int prec, char* out, int nrhs) {
  return blas_axpby(ctx, prec, nullptr, prec, out, nrhs, 0.0, 0.0, -1, -1, 1);
}

template <int PX, int PR, int PP, int PQ>
static void xr_l(dwf_context* ctx, VecGeom g, char* x, char* r, const char* p, const char* q, int nrhs) {
  hipLaunchKernelGGL((cg_xr_kernel<PX, PR, PP, PQ>), dim3(RED_BLOCKS, nrhs), dim3(BS), 0, ctx->stream, g, x, r, p, q,
                     field_bytes_rhs(ctx, PX), field_bytes_rhs(ctx, PR), field_bytes_rhs(ctx, PP),
                     field_bytes_rhs(ctx, PQ), ctx->scalars, ctx->partials);
}

hipError_t cg_update_xr(dwf_context* ctx, int px, char* x, int pr, char* r, int pp, const char* p, int pq,
                        const char* q, int nrhs) {
  VecGeom g = vgeom(ctx);
  // supported combinations: all-F64; x/r F32 with p/q F32 or F16S
  if (px == DWF_F64 && pr == DWF_F64 && pp == DWF_F64 && pq == DWF_F64)
    xr_l<DWF_F64, DWF_F64, DWF_F64, DWF_F64>(ctx, g, x, r, p, q, nrhs);
  else if (px == DWF_F32 && pr == DWF_F32 && pp == DWF_F32 && pq == DWF_F32)
    xr_l<DWF_F32, DWF_F32, DWF_F32, DWF_F32>(ctx, g, x, r, p, q, nrhs);
  else if (px == DWF_F32 && pr == DWF_F32 && pp == DWF_F16S && pq == DWF_F16S)
    xr_l<DWF_F32, DWF_F32, DWF_F16S, DWF_F16S>(ctx, g, x, r, p, q, nrhs);
  else
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(finalize_kernel, dim3(nrhs), dim3(BS), 0, ctx->stream, ctx->partials, ctx->scalars + S_RR,
                     NSCAL, 0);
  return hipGetLastError();
}

template <int PR, int PP>
static void p_l(dwf_context* ctx, VecGeom g, const char* r, char* p, int nrhs, int orth) {
  hipLaunchKernelGGL((cg_p_kernel<PR, PP>), dim3(grid_n(g.n), nrhs), dim3(BS), 0, ctx->stream, g, r, p,
                     field_bytes_rhs(ctx, PR), field_bytes_rhs(ctx, PP), ctx->scalars, orth);
}

hipError_t cg_update_p(dwf_context* ctx, int pr, const char* r, int pp, char* p, int nrhs, bool orth) {
  VecGeom g = vgeom(ctx);
  if (pr == DWF_F64 && pp == DWF_F64)
    p_l<DWF_F64, DWF_F64>(ctx, g, r, p, nrhs, orth);
  else if (pr == DWF_F32 && pp == DWF_F32)
    p_l<DWF_F32, DWF_F32>(ctx, g, r, p, nrhs, orth);
  else if (pr == DWF_F32 && pp == DWF_F16S)
    p_l<DWF_F32, DWF_F16S>(ctx, g, r, p, nrhs, orth);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int PR, int PQ>
static void r_l(dwf_context* ctx, VecGeom g, char* r, const char* q, int nrhs) {
  hipLaunchKernelGGL((cg_r_kernel<PR, PQ>), dim3(RED_BLOCKS, nrhs), dim3(BS), 0, ctx->stream, g, r, q,
                     field_bytes_rhs(ctx, PR), field_bytes_rhs(ctx, PQ), ctx->scalars, ctx->partials);
}

hipError_t cg_update_r(dwf_context* ctx, int pr, char* r, int pq, const char* q, int nrhs) {
  VecGeom g = vgeom(ctx);
  if (pr == DWF_F64 && pq == DWF_F64)
    r_l<DWF_F64, DWF_F64>(ctx, g, r, q, nrhs);
  else if (pr == DWF_F32 && pq == DWF_F32)
    r_l<DWF_F32, DWF_F32>(ctx, g, r, q, nrhs);
  else if (pr == DWF_F32 && pq == DWF_F16S)
    r_l<DWF_F32, DWF_F16S>(ctx, g, r, q, nrhs);
  else
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(finalize_kernel, dim3(nrhs), dim3(BS), 0, ctx->stream, ctx->partials, ctx->scalars + S_RR,
                     NSCAL, 0);
  return hipGetLastError();
}

template <int PX, int PR, int PP>
static void xp_l(dwf_context* ctx, VecGeom g, char* x, const char* r, char* p, int nrhs) {
  hipLaunchKernelGGL((cg_xp_kernel<PX, PR, PP>), dim3(grid_n(g.n), nrhs), dim3(BS), 0, ctx->stream, g, x, r, p,
                     field_bytes_rhs(ctx, PX), field_bytes_rhs(ctx, PR), field_bytes_rhs(ctx, PP), ctx->scalars);
}

hipError_t cg_update_xp(dwf_context* ctx, int px, char* x, int pr, const char* r, int pp, char* p, int nrhs) {
  VecGeom g = vgeom(ctx);
  if (px == DWF_F64 && pr == DWF_F64 && pp == DWF_F64)
    xp_l<DWF_F64, DWF_F64, DWF_F64>(ctx, g, x, r, p, nrhs);
  else if (px == DWF_F32 && pr == DWF_F32 && pp == DWF_F32)
    xp_l<DWF_F32, DWF_F32, DWF_F32>(ctx, g, x, r, p, nrhs);
  else if (px == DWF_F32 && pr == DWF_F32 && pp == DWF_F16S)
    xp_l<DWF_F32, DWF_F32, DWF_F16S>(ctx, g, x, r, p, nrhs);
  else if (px == DWF_F64 && pr == DWF_F32 && pp == DWF_F32)
    xp_l<DWF_F64, DWF_F32, DWF_F32>(ctx, g, x, r, p, nrhs);
  else if (px == DWF_F64 && pr == DWF_F32 && pp == DWF_F16S)
    xp_l<DWF_F64, DWF_F32, DWF_F16S>(ctx, g, x, r, p, nrhs);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int PR, int PP>
static void dir_l(dwf_context* ctx, VecGeom g, const char* r, const char* p, char* pn, int keep, int nrhs) {
  hipLaunchKernelGGL((cg_dir_kernel<PR, PP>), dim3(grid_n(g.n), nrhs), dim3(BS), 0, ctx->stream, g, r, p, pn,
                     field_bytes_rhs(ctx, PR), field_bytes_rhs(ctx, PP), ctx->scalars, keep);
}

hipError_t cg_next_dir(dwf_context* ctx, int pr, const char* r, int pp, const char* p, char* pn, int keep, int nrhs) {
  if (keep < S_ALPHA_K || keep >= NSCAL) return hipErrorInvalidValue;
  VecGeom g = vgeom(ctx);
  if (pr == DWF_F64 && pp == DWF_F64)
    dir_l<DWF_F64, DWF_F64>(ctx, g, r, p, pn, keep, nrhs);
  else if (pr == DWF_F32 && pp == DWF_F32)
    dir_l<DWF_F32, DWF_F32>(ctx, g, r, p, pn, keep, nrhs);
  else if (pr == DWF_F32 && pp == DWF_F16S)
    dir_l<DWF_F32, DWF_F16S>(ctx, g, r, p, pn, keep, nrhs);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int PR, int PP, int N>
static void flush_n(dwf_context* ctx, VecGeom g, char* x, const DirSet& d, const char* r, char* pn, int nrhs) {
  hipLaunchKernelGGL((cg_flush_kernel<PR, PP, N>), dim3(grid_n(g.n), nrhs), dim3(BS), 0, ctx->stream, g, x, d, r, pn,
                     field_bytes_rhs(ctx, DWF_F64), field_bytes_rhs(ctx, PR), field_bytes_rhs(ctx, PP),
                     ctx->scalars);
}

template <int PR, int PP>
static void flush_l(dwf_context* ctx, VecGeom g, char* x, const DirSet& d, int n, const char* r, char* pn, int nrhs) {
  switch (n) {
    case 1: flush_n<PR, PP, 1>(ctx, g, x, d, r, pn, nrhs); break;
    case 2: flush_n<PR, PP, 2>(ctx, g, x, d, r, pn, nrhs); break;
    case 3: flush_n<PR, PP, 3>(ctx, g, x, d, r, pn, nrhs); break;
    default: flush_n<PR, PP, 4>(ctx, g, x, d, r, pn, nrhs); break;
  }
}

hipError_t cg_flush_x(dwf_context* ctx, char* x, int pr, const char* r, int pp, char* const p[], const int slot[],
                      int n, char* pn, int nrhs) {
  if (n < 1 || n > 4 || (pn != nullptr && r == nullptr)) return hipErrorInvalidValue;
  DirSet d{};
  for (int k = 0; k < n; ++k) {
    if (p[k] == nullptr || slot[k] < 0 || slot[k] >= NSCAL) return hipErrorInvalidValue;
    d.p[k] = p[k];
    d.slot[k] = slot[k];
  }
  VecGeom g = vgeom(ctx);
  if (pr == DWF_F64 && pp == DWF_F64)
    flush_l<DWF_F64, DWF_F64>(ctx, g, x, d, n, r, pn, nrhs);
  else if (pr == DWF_F32 && pp == DWF_F32)
    flush_l<DWF_F32, DWF_F32>(ctx, g, x, d, n, r, pn, nrhs);
  else if (pr == DWF_F32 && pp == DWF_F16S)
    flush_l<DWF_F32, DWF_F16S>(ctx, g, x, d, n, r, pn, nrhs);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t cg_reliable_p(dwf_context* ctx, const char* r_true, char* r_iter, int pp, char* p, int nrhs) {
  VecGeom g = vgeom(ctx);
  const dim3 grid(grid_n(g.n), nrhs);
  const size_t st = field_bytes_rhs(ctx, DWF_F64), si = field_bytes_rhs(ctx, DWF_F32), sp = field_bytes_rhs(ctx, pp);
  if (pp == DWF_F32)
    hipLaunchKernelGGL((cg_reliable_kernel<DWF_F32>), grid, dim3(BS), 0, ctx->stream, g, r_true, r_iter, p, st, si, sp);
  else if (pp == DWF_F16S)
    hipLaunchKernelGGL((cg_reliable_kernel<DWF_F16S>), grid, dim3(BS), 0, ctx->stream, g, r_true, r_iter, p, st, si,
                       sp);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t cg_orth_p(dwf_context* ctx, const char* r, int pp, char* p, int nrhs) {
  VecGeom g = vgeom(ctx);
  const dim3 grid(grid_n(g.n), nrhs);
  const size_t sr = field_bytes_rhs(ctx, DWF_F32), sp = field_bytes_rhs(ctx, pp);
  if (pp == DWF_F32)
    hipLaunchKernelGGL((cg_orth_kernel<DWF_F32>), grid, dim3(BS), 0, ctx->stream, g, r, p, sr, sp, ctx->scalars);
  else if (pp == DWF_F16S)
    hipLaunchKernelGGL((cg_orth_kernel<DWF_F16S>), grid, dim3(BS), 0, ctx->stream, g, r, p, sr, sp, ctx->scalars);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t scal_alpha(dwf_context* ctx, int nrhs) {
  hipLaunchKernelGGL(scal_alpha_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, ctx->stream, ctx->scalars, nrhs);
  return hipGetLastError();
}
hipError_t scal_beta(dwf_context* ctx, int nrhs) {
  hipLaunchKernelGGL(scal_beta_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, ctx->stream, ctx->scalars, nrhs);
  return hipGetLastError();
}
hipError_t scal_set(dwf_context* ctx, int nrhs, int slot, double v) {
  hipLaunchKernelGGL(scal_set_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, ctx->stream, ctx->scalars, nrhs, slot, v);
  return hipGetLastError();
}
hipError_t scal_copy(dwf_context* ctx, int nrhs, int dst, int src) {
  hipLaunchKernelGGL(scal_copy_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, ctx->stream, ctx->scalars, nrhs, dst,
                     src);
  return hipGetLastError();
}

hipError_t scal_converge(dwf_context* ctx, int nrhs, double tol2, bool count_iter, int allow_stop) {
  hipLaunchKernelGGL(scal_converge_kernel, dim3((nrhs + 63) / 64), dim3(64), 0, ctx->stream, ctx->scalars, nrhs, tol2,
                     count_iter ? 1 : 0, allow_stop);
  return hipGetLastError();
}

hipError_t gs_multidot(dwf_context* ctx, int prec, const char* Q, const char* v, int j, double* coef) {
  VecGeom g = vgeom(ctx);
  const size_t st = field_bytes_rhs(ctx, prec);
  // <Q_k, v> for k < j : Q_k is the batch index, v has stride 0
  DWF_DISPATCH1(prec, dot_la, ctx, prec, g, Q, st, v, 0, j);
  hipLaunchKernelGGL(finalize_kernel, dim3(j), dim3(BS), 0, ctx->stream, ctx->partials, coef, 2, 1);
  return hipGetLastError();
}

template <int P>
static void maxpy_l(dwf_context* ctx, VecGeom g, const char* Q, char* v, size_t st, int j, const double* coef) {
  hipLaunchKernelGGL((multiaxpy_kernel<P>), dim3(grid_n(g.n)), dim3(BS), 0, ctx->stream, g, Q, v, st, j, coef);
}

hipError_t gs_multiaxpy(dwf_context* ctx, int prec, const char* Q, char* v, int j, const double* coef) {
  VecGeom g = vgeom(ctx);
  const size_t st = field_bytes_rhs(ctx, prec);
  DWF_DISPATCH1(prec, maxpy_l, ctx, g, Q, v, st, j, coef);
  return hipGetLastError();
}

template <int P>
static void scale_l(dwf_context* ctx, VecGeom g, char* v, const double* f) {
  hipLaunchKernelGGL((scale_kernel<P>), dim3(grid_n(g.n)), dim3(BS), 0, ctx->stream, g, v, f);
}

hipError_t gs_scale(dwf_context* ctx, int prec, char* v, const double* inv_norm) {
  VecGeom g = vgeom(ctx);
  DWF_DISPATCH1(prec, scale_l, ctx, g, v, inv_norm);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Cholesky-QR orthonormalisation of up to TS_NMAX fields.  At FP64 and FP32 a
// field is taken as a flat array of m complex values (the layout is the same for
// every field, so inner products do not depend on it); FP16 + scale fields are
// read and written a spinor (12 complex values and their scale) at a time.
// ---------------------------------------------------------------------------

constexpr int TS_TPT = 3;  // 2 x 2 tiles per thread: (n/2)(n/2 + 1)/2 <= 528 for n <= 64

// Tile (ta <= tb) of the upper triangle of (n/2 rounded up)^2 2 x 2 tiles, row-major.
__device__ __forceinline__ void ts_tile_coords(int t, int half, int& ta, int& tb) {
  int row = 0;
  while (row < half && t >= half - row) {
    t -= half - row;
    ++row;
  }
  ta = row;
  tb = row + t;
}

// acc += the 2 x 2 tiles' conj(v_j) v_k over `rows` staged rows sm[row][n]
template <typename R>
__device__ __forceinline__ void ts_tiles(const cplx<R>* sm, int rows, int n, int ntiles, const int ta[TS_TPT],
                                         const int tb[TS_TPT], double acc[TS_TPT][8]) {
#pragma unroll
  for (int q = 0; q < TS_TPT; ++q) {
    if (threadIdx.x + q * blockDim.x >= ntiles) continue;
    const int j0 = 2 * ta[q], k0 = 2 * tb[q];
    const bool j1 = j0 + 1 < n, k1 = k0 + 1 < n;
    for (int r = 0; r < rows; ++r) {
      const cplx<R>* row = sm + (size_t)r * n;
      const cplx<R> x0 = row[j0], y0 = row[k0];
      const cplx<R> x1 = j1 ? row[j0 + 1] : cplx<R>{0, 0};
      const cplx<R> y1 = k1 ? row[k0 + 1] : cplx<R>{0, 0};
      // conj(x) y
      acc[q][0] = fma((double)x0.re, (double)y0.re, fma((double)x0.im, (double)y0.im, acc[q][0]));
      acc[q][1] = fma((double)x0.re, (double)y0.im, fma(-(double)x0.im, (double)y0.re, acc[q][1]));
      acc[q][2] = fma((double)x0.re, (double)y1.re, fma((double)x0.im, (double)y1.im, acc[q][2]));
      acc[q][3] = fma((double)x0.re, (double)y1.im, fma(-(double)x0.im, (double)y1.re, acc[q][3]));
      acc[q][4] = fma((double)x1.re, (double)y0.re, fma((double)x1.im, (double)y0.im, acc[q][4]));
      acc[q][5] = fma((double)x1.re, (double)y0.im, fma(-(double)x1.im, (double)y0.re, acc[q][5]));
      acc[q][6] = fma((double)x1.re, (double)y1.re, fma((double)x1.im, (double)y1.im, acc[q][6]));
      acc[q][7] = fma((double)x1.re, (double)y1.im, fma(-(double)x1.im, (double)y1.re, acc[q][7]));
    }
  }
}

// G[k][j] (j <= k) of the workgroup's tiles
__device__ __forceinline__ void ts_store_tiles(double* G, int n, int ntiles, const int ta[TS_TPT],
                                               const int tb[TS_TPT], const double acc[TS_TPT][8]) {
#pragma unroll
  for (int q = 0; q < TS_TPT; ++q) {
    if (threadIdx.x + q * blockDim.x >= ntiles) continue;
    const int j0 = 2 * ta[q], k0 = 2 * tb[q];
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
      for (int dk = 0; dk < 2; ++dk) {
        const int j = j0 + dj, k = k0 + dk;
        if (j >= n || k >= n || j > k) continue;
        G[2 * ((size_t)k * n + j)] = acc[q][2 * (2 * dj + dk)];
        G[2 * ((size_t)k * n + j) + 1] = acc[q][2 * (2 * dj + dk) + 1];
      }
  }
}

// Per workgroup, the Gram matrix of its part of the fields: partial[wg][k][j] =
// sum conj(v_j) v_k for j <= k, in FP64.  Units [u0, u0 + span) (complex values at
// FP64 / FP32, spinors at FP16 + scale) pass through LDS `cu` units at a time with
// all n fields at once, and each thread accumulates 2 x 2 tiles of (j, k).
template <int P>
__global__ void __launch_bounds__(256) ts_gram_kernel(const char* __restrict__ V, size_t stride, long long units,
                                                      int n, long long span, int cu, VecGeom g,
                                                      double* __restrict__ partial) {
  using R = typename Store<P>::real;
  constexpr int RPU = P == DWF_F16S ? 12 : 1;  // staged rows per unit
  extern __shared__ char smem[];
  cplx<R>* sm = reinterpret_cast<cplx<R>*>(smem);  // [cu * RPU][n]
  const long long u0 = (long long)blockIdx.x * span;
  const long long u1 = min(units, u0 + span);
  const int half = (n + 1) / 2;
  const int ntiles = half * (half + 1) / 2;
  double acc[TS_TPT][8];
  int ta[TS_TPT], tb[TS_TPT];
#pragma unroll
  for (int q = 0; q < TS_TPT; ++q) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[q][i] = 0;
    ts_tile_coords(threadIdx.x + q * blockDim.x, half, ta[q], tb[q]);
  }
  for (long long r0 = u0; r0 < u1; r0 += cu) {
    const int cs = (int)min((long long)cu, u1 - r0);
    __syncthreads();  // previous rows consumed
    for (int item = threadIdx.x; item < cs * n; item += blockDim.x) {
      const int j = item / cs, e = item - j * cs;  // consecutive threads: consecutive units
      const char* f = V + (size_t)j * stride;
      if constexpr (P == DWF_F16S) {
        const long long sp = r0 + e, h = sp / g.Ls;
        cplx<float> v[12];
        Store<DWF_F16S>::load(f, g.V4h, g.Ls, h, (int)(sp - h * g.Ls), v);
#pragma unroll
        for (int c = 0; c < 12; ++c) sm[(size_t)(e * 12 + c) * n + j] = v[c];
      } else {
        sm[(size_t)e * n + j] = reinterpret_cast<const cplx<R>*>(f)[r0 + e];
      }
    }
    __syncthreads();
    ts_tiles(sm, cs * RPU, n, ntiles, ta, tb, acc);
  }
  ts_store_tiles(partial + 2 * (size_t)blockIdx.x * n * n, n, ntiles, ta, tb, acc);
}

// G[k][j] = sum over the workgroups, in workgroup order, of partial[wg][k][j] (j <= k)
__global__ void ts_gram_sum_kernel(const double* __restrict__ partial, int nwg, int n, double* __restrict__ G) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * n) return;
  const int k = idx / n, j = idx - k * n;
  if (j > k) return;
  double re = 0, im = 0;
  for (int w = 0; w < nwg; ++w) {
    re += partial[2 * ((size_t)w * n * n + idx)];
    im += partial[2 * ((size_t)w * n * n + idx) + 1];
  }
  G[2 * idx] = re;
  G[2 * idx + 1] = im;
}

// In place v_k <- sum_{j <= k} W[j][k] v_j for every k (W upper triangular,
// complex FP64, W[j][k] at j * n + k), one unit per thread: the outputs in tiles
// from the top down, so that the v_j a tile reads (j below the tile's top) are not
// yet overwritten.  FP64 and FP32: one complex value per thread, tiles of 16,
// FP64 arithmetic; FP16 + scale: one spinor per thread (the scale is per spinor),
// tiles of 4, FP32 arithmetic (the result is rounded to FP16).
constexpr int TS_KT = 16;
constexpr int TS_KT16 = 4;

template <typename R>
__global__ void __launch_bounds__(256) ts_combine_kernel(char* V, size_t stride, long long m, int n,
                                                         const double* __restrict__ W) {
  extern __shared__ double wsm[];  // [n][n] complex
  for (int i = threadIdx.x; i < 2 * n * n; i += blockDim.x) wsm[i] = W[i];
  __syncthreads();
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  for (int k0 = (n - 1) / TS_KT * TS_KT; k0 >= 0; k0 -= TS_KT) {
    double ar[TS_KT], ai[TS_KT];
#pragma unroll
    for (int t = 0; t < TS_KT; ++t) ar[t] = ai[t] = 0;
    const int jend = min(n, k0 + TS_KT);
    for (int j = 0; j < jend; ++j) {
      const cplx<R> v = reinterpret_cast<const cplx<R>*>(V + (size_t)j * stride)[e];
      const double vr = v.re, vi = v.im;
#pragma unroll
      for (int t = 0; t < TS_KT; ++t) {
        const int k = k0 + t;
        if (k >= n || j > k) continue;
        const double wr = wsm[2 * (j * n + k)], wi = wsm[2 * (j * n + k) + 1];
        ar[t] = fma(wr, vr, fma(-wi, vi, ar[t]));
        ai[t] = fma(wr, vi, fma(wi, vr, ai[t]));
      }
    }
#pragma unroll
    for (int t = 0; t < TS_KT; ++t) {
      const int k = k0 + t;
      if (k >= n) continue;
      reinterpret_cast<cplx<R>*>(V + (size_t)k * stride)[e] = cplx<R>{(R)ar[t], (R)ai[t]};
    }
  }
}

__global__ void __launch_bounds__(256) ts_combine_f16_kernel(char* V, size_t stride, VecGeom g, int n,
                                                             const double* __restrict__ W) {
  extern __shared__ double wsm[];  // [n][n] complex
  for (int i = threadIdx.x; i < 2 * n * n; i += blockDim.x) wsm[i] = W[i];
  __syncthreads();
  const long long sp = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (sp >= g.n) return;
  const long long h = sp / g.Ls;
  const int s = (int)(sp - h * g.Ls);
  for (int k0 = (n - 1) / TS_KT16 * TS_KT16; k0 >= 0; k0 -= TS_KT16) {
    cplx<float> acc[TS_KT16][12];
#pragma unroll
    for (int t = 0; t < TS_KT16; ++t)
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[t][c] = {0.f, 0.f};
    const int jend = min(n, k0 + TS_KT16);
    for (int j = 0; j < jend; ++j) {
      cplx<float> v[12];
      Store<DWF_F16S>::load(V + (size_t)j * stride, g.V4h, g.Ls, h, s, v);
#pragma unroll
      for (int t = 0; t < TS_KT16; ++t) {
        const int k = k0 + t;
        if (k >= n || j > k) continue;
        const float wr = (float)wsm[2 * (j * n + k)], wi = (float)wsm[2 * (j * n + k) + 1];
#pragma unroll
        for (int c = 0; c < 12; ++c)
          acc[t][c] = {fmaf(wr, v[c].re, fmaf(-wi, v[c].im, acc[t][c].re)),
                       fmaf(wr, v[c].im, fmaf(wi, v[c].re, acc[t][c].im))};
      }
    }
#pragma unroll
    for (int t = 0; t < TS_KT16; ++t) {
      const int k = k0 + t;
      if (k < n) Store<DWF_F16S>::store(V + (size_t)k * stride, g.V4h, g.Ls, h, s, acc[t]);
    }
  }
}

hipError_t ts_gram(dwf_context* ctx, int prec, const char* V, int n, double* partial, int nwg, double* G) {
  if (n < 1 || n > TS_NMAX || nwg < 1 || prec < DWF_F64 || prec > DWF_F16S) return hipErrorInvalidValue;
  const VecGeom g = vgeom(ctx);
  const size_t stride = field_bytes_rhs(ctx, prec);
  const long long units = prec == DWF_F16S ? g.n : g.n * 12;  // spinors, or complex values
  const long long span = (units + nwg - 1) / nwg;
  const int cu = prec == DWF_F64 ? 32 : (prec == DWF_F32 ? 64 : 4);  // 32 KB of staged rows at n = 64 (F16S 24 KB)
  const size_t lds = (size_t)cu * (prec == DWF_F16S ? 12 : 1) * n * (prec == DWF_F64 ? 16 : 8);
  if (prec == DWF_F64)
    hipLaunchKernelGGL(ts_gram_kernel<DWF_F64>, dim3(nwg), dim3(256), lds, ctx->stream, V, stride, units, n, span, cu,
                       g, partial);
  else if (prec == DWF_F32)
    hipLaunchKernelGGL(ts_gram_kernel<DWF_F32>, dim3(nwg), dim3(256), lds, ctx->stream, V, stride, units, n, span, cu,
                       g, partial);
  else
    hipLaunchKernelGGL(ts_gram_kernel<DWF_F16S>, dim3(nwg), dim3(256), lds, ctx->stream, V, stride, units, n, span,
                       cu, g, partial);
  hipLaunchKernelGGL(ts_gram_sum_kernel, dim3((n * n + 255) / 256), dim3(256), 0, ctx->stream, partial, nwg, n, G);
  return hipGetLastError();
}

hipError_t ts_combine(dwf_context* ctx, int prec, char* V, int n, const double* W) {
  if (n < 1 || n > TS_NMAX || prec < DWF_F64 || prec > DWF_F16S) return hipErrorInvalidValue;
  const VecGeom g = vgeom(ctx);
  const size_t stride = field_bytes_rhs(ctx, prec);
  const size_t lds = (size_t)2 * n * n * sizeof(double);
  if (prec == DWF_F16S) {
    hipLaunchKernelGGL(ts_combine_f16_kernel, dim3((unsigned)((g.n + 255) / 256)), dim3(256), lds, ctx->stream, V,
                       stride, g, n, W);
    return hipGetLastError();
  }
  const long long m = g.n * 12;
  const dim3 grid((unsigned)((m + 255) / 256));
  if (prec == DWF_F64)
    hipLaunchKernelGGL(ts_combine_kernel<double>, grid, dim3(256), lds, ctx->stream, V, stride, m, n, W);
  else
    hipLaunchKernelGGL(ts_combine_kernel<float>, grid, dim3(256), lds, ctx->stream, V, stride, m, n, W);
  return hipGetLastError();
}

}  // namespace dwf
