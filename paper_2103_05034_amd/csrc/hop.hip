// Half-lattice Wilson hopping term on every fifth-dimension slice, with the
// fifth-dimension terms of the Schur blocks fused into its epilogue.
//
// D_hop psi(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)
// (Chiral Fermion Actions section, the D_hop equation); the adjoint swaps the
// projector signs.  Links are packed per output parity with the backward link
// already conjugate-transposed, so all eight directions are "project, rotate
// by a 3x3 matrix, reconstruct".
//
// Thread mapping: a workgroup owns `spb` consecutive half-lattice sites and
// all Ls slices of each; lane = site_local * Ls + s.  Loads of a spinor
// component are contiguous along s, the Ls lanes of a site read the same link
// entries, and the M5D / M5D^{-1} epilogues see whole s-columns of a site.
// Workgroups are remapped so that each XCD (workgroups are dealt round-robin
// over the 8 XCDs) sweeps one contiguous range of sites, which keeps the
// stencil's neighbour reuse inside one L2.
#include <cmath>

#include "dwf_internal.hpp"
#include "kernels.hpp"

namespace dwf {

template <class R>
struct LinkT;
template <>
struct LinkT<double> {
  using vec = double2;
};
template <>
struct LinkT<float> {
  using vec = float2;
};

template <int PREC, bool DAG, int MU, int BACK>
__device__ __forceinline__ void hop_dir(const HopArgs& a, const char* in, long long h, int s,
                                        cplx<typename Store<PREC>::real> acc[12]) {
  using R = typename Store<PREC>::real;
  using V = typename LinkT<R>::vec;
  constexpr int DIR = 2 * MU + BACK;
  constexpr int SIGMA = DAG ? (BACK ? -1 : +1) : (BACK ? +1 : -1);
  const long long V4h = a.V4h;
  const long long nh = a.nbr[DIR * V4h + h];
  cplx<R> psi[12];
  Store<PREC>::load(in, V4h, a.Ls, nh, s, psi);
  cplx<R> hs[6];
  project<MU, SIGMA>(psi, hs);
  const V* lp = reinterpret_cast<const V*>(a.links) + (size_t)DIR * 9 * V4h + h;
  cplx<R> u[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    V t = lp[(size_t)k * V4h];
    u[k] = {t.x, t.y};
  }
  cplx<R> chi[6];
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cplx<R> v = cmul(u[3 * i + 0], hs[3 * sp + 0]);
      v = cfma(u[3 * i + 1], hs[3 * sp + 1], v);
      v = cfma(u[3 * i + 2], hs[3 * sp + 2], v);
      chi[3 * sp + i] = v;
    }
  }
  reconstruct<MU, SIGMA>(chi, acc);
}

// (M5D x)_s or (M5D^dag x)_s for one lane, from x at s, s-1 and s+1 (cyclic).
template <class R, bool DAG>
__device__ __forceinline__ void m5d_lane(const cplx<R> xs[12], const cplx<R> xlo[12], const cplx<R> xhi[12],
                                         int s, int Ls, R d, R mf, cplx<R> out[12]) {
  const R c_lo = (s == 0) ? mf : (R)-1;       // coefficient of x_{s-1} (wraps with +m)
  const R c_hi = (s == Ls - 1) ? mf : (R)-1;  // coefficient of x_{s+1}
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const bool upper = c < 6;  // P_+ spins
    const bool use_lo = DAG ? !upper : upper;
    const cplx<R> nb = use_lo ? xlo[c] : xhi[c];
    const R cf = use_lo ? c_lo : c_hi;
    out[c] = {d * xs[c].re + cf * nb.re, d * xs[c].im + cf * nb.im};
  }
}

// In-LDS inverse of M5D (or M5D^dag) on the columns of a workgroup.  buf is
// [spb][12][LP] with LP = Ls + 1.  Per chirality the matrix is d - S with S a
// cyclic shift whose wrap carries -m (lower shift for P_+, upper for P_-;
// transposed for the adjoint), so the solve is the recursion
// y_j = (v_j + y_{j-1}) / d along the shift direction, started from
// y_{-1} = -m y_{Ls-1}; a first pass with zero start gives y_{Ls-1}'s
// dependence and fixes y_{-1} = corner * z_{Ls-1}, corner = -m / (1 + m d^-Ls).
template <class R, bool DAG>
__device__ __forceinline__ void m5inv_columns(cplx<R>* buf, int spb, int Ls, long long h0, long long V4h,
                                              R inv_d, R corner) {
  const int LP = Ls + 1;
  for (int idx = threadIdx.x; idx < spb * 12; idx += blockDim.x) {
    const int sl = idx / 12;
    const int c = idx - 12 * sl;
    if (h0 + sl >= V4h) continue;
    const bool upper = c < 6;
    const bool fwd = DAG ? !upper : upper;
    cplx<R>* col = buf + (size_t)(sl * 12 + c) * LP;
    cplx<R> z = {0, 0};
    for (int j = 0; j < Ls; ++j) {
      const int sj = fwd ? j : Ls - 1 - j;
      z = {(col[sj].re + z.re) * inv_d, (col[sj].im + z.im) * inv_d};
    }
    cplx<R> y = {corner * z.re, corner * z.im};
    for (int j = 0; j < Ls; ++j) {
      const int sj = fwd ? j : Ls - 1 - j;
      y = {(col[sj].re + y.re) * inv_d, (col[sj].im + y.im) * inv_d};
      col[sj] = y;
    }
  }
}

template <int PREC, bool DAG, int EPI>
__global__ void __launch_bounds__(256) hop_kernel(HopArgs a) {
  using R = typename Store<PREC>::real;
  extern __shared__ char smem_raw[];
  const int Ls = a.Ls;
  const int b = blockIdx.x;
  const int logical = (b & 7) * a.nb8 + (b >> 3);
  if (logical >= a.nblocks) return;  // whole workgroup leaves together
  const int tid = threadIdx.x;
  const int sl = tid / Ls;
  const int s = tid - sl * Ls;
  const long long h0 = (long long)logical * a.spb;
  const long long h = h0 + sl;
  const bool valid = (sl < a.spb) && (h < a.V4h);
  const size_t off = (size_t)blockIdx.y * a.stride;
  const char* in = a.in + off;

  cplx<R> acc[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
  if (valid) {
    hop_dir<PREC, DAG, 0, 0>(a, in, h, s, acc);
    hop_dir<PREC, DAG, 0, 1>(a, in, h, s, acc);
    hop_dir<PREC, DAG, 1, 0>(a, in, h, s, acc);
    hop_dir<PREC, DAG, 1, 1>(a, in, h, s, acc);
    hop_dir<PREC, DAG, 2, 0>(a, in, h, s, acc);
    hop_dir<PREC, DAG, 2, 1>(a, in, h, s, acc);
    hop_dir<PREC, DAG, 3, 0>(a, in, h, s, acc);
    hop_dir<PREC, DAG, 3, 1>(a, in, h, s, acc);
  }
  const R alpha = (R)a.alpha;
  char* out = a.out + off;

  if (EPI == EPI_LIN || EPI == EPI_M5INV) {
    cplx<R> v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = cscale(alpha, acc[c]);
    if (a.x != nullptr && valid) {
      cplx<R> xv[12];
      Store<PREC>::load(a.x + off, a.V4h, Ls, h, s, xv);
      const R beta = (R)a.beta;
#pragma unroll
      for (int c = 0; c < 12; ++c) v[c] = {v[c].re + beta * xv[c].re, v[c].im + beta * xv[c].im};
    }
    if (EPI == EPI_LIN) {
      if (valid) Store<PREC>::store(out, a.V4h, Ls, h, s, v);
      return;
    }
    cplx<R>* buf = reinterpret_cast<cplx<R>*>(smem_raw);
    const int LP = Ls + 1;
    if (valid) {
#pragma unroll
      for (int c = 0; c < 12; ++c) buf[(size_t)(sl * 12 + c) * LP + s] = v[c];
    }
    __syncthreads();
    m5inv_columns<R, DAG>(buf, a.spb, Ls, h0, a.V4h, (R)a.inv_d, (R)a.corner);
    __syncthreads();
    if (valid) {
#pragma unroll
      for (int c = 0; c < 12; ++c) v[c] = buf[(size_t)(sl * 12 + c) * LP + s];
      Store<PREC>::store(out, a.V4h, Ls, h, s, v);
    }
    return;
  } else {  // EPI_M5, EPI_CHEB
    if (!valid) return;
    const char* x = a.x + off;
    const int s_lo = (s == 0) ? Ls - 1 : s - 1;
    const int s_hi = (s == Ls - 1) ? 0 : s + 1;
    cplx<R> xs[12], xlo[12], xhi[12], v[12];
    Store<PREC>::load(x, a.V4h, Ls, h, s, xs);
    Store<PREC>::load(x, a.V4h, Ls, h, s_lo, xlo);
    Store<PREC>::load(x, a.V4h, Ls, h, s_hi, xhi);
    m5d_lane<R, DAG>(xs, xlo, xhi, s, Ls, (R)a.d, (R)a.mf, v);
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = {v[c].re + alpha * acc[c].re, v[c].im + alpha * acc[c].im};
    if (EPI == EPI_CHEB) {
      cplx<R> yv[12], zv[12];
      Store<PREC>::load(a.y + off, a.V4h, Ls, h, s, yv);
      Store<PREC>::load(a.z + off, a.V4h, Ls, h, s, zv);
      const R ca = (R)a.ca, cb = (R)a.cb, cc = (R)a.cc;
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        v[c].re = ca * v[c].re + cb * yv[c].re + cc * zv[c].re;
        v[c].im = ca * v[c].im + cb * yv[c].im + cc * zv[c].im;
      }
    }
    Store<PREC>::store(out, a.V4h, Ls, h, s, v);
  }
}

// Site-local fifth-dimension operator without the hop: out = M5D in, M5D^dag in,
// or their inverses.
template <int PREC, bool DAG, bool INV>
__global__ void __launch_bounds__(256) site5_kernel(HopArgs a) {
  using R = typename Store<PREC>::real;
  extern __shared__ char smem_raw[];
  const int Ls = a.Ls;
  const int b = blockIdx.x;
  const int logical = (b & 7) * a.nb8 + (b >> 3);
  if (logical >= a.nblocks) return;
  const int tid = threadIdx.x;
  const int sl = tid / Ls;
  const int s = tid - sl * Ls;
  const long long h0 = (long long)logical * a.spb;
  const long long h = h0 + sl;
  const bool valid = (sl < a.spb) && (h < a.V4h);
  const size_t off = (size_t)blockIdx.y * a.stride;
  const char* in = a.in + off;
  char* out = a.out + off;
  if (!INV) {
    if (!valid) return;
    const int s_lo = (s == 0) ? Ls - 1 : s - 1;
    const int s_hi = (s == Ls - 1) ? 0 : s + 1;
    cplx<R> xs[12], xlo[12], xhi[12], v[12];
    Store<PREC>::load(in, a.V4h, Ls, h, s, xs);
    Store<PREC>::load(in, a.V4h, Ls, h, s_lo, xlo);
    Store<PREC>::load(in, a.V4h, Ls, h, s_hi, xhi);
    m5d_lane<R, DAG>(xs, xlo, xhi, s, Ls, (R)a.d, (R)a.mf, v);
    Store<PREC>::store(out, a.V4h, Ls, h, s, v);
    return;
  }
  cplx<R>* buf = reinterpret_cast<cplx<R>*>(smem_raw);
  const int LP = Ls + 1;
  cplx<R> v[12];
  if (valid) {
    Store<PREC>::load(in, a.V4h, Ls, h, s, v);
#pragma unroll
    for (int c = 0; c < 12; ++c) buf[(size_t)(sl * 12 + c) * LP + s] = v[c];
  }
  __syncthreads();
  m5inv_columns<R, DAG>(buf, a.spb, Ls, h0, a.V4h, (R)a.inv_d, (R)a.corner);
  __syncthreads();
  if (valid) {
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = buf[(size_t)(sl * 12 + c) * LP + s];
    Store<PREC>::store(out, a.V4h, Ls, h, s, v);
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void fill_shape(const dwf_context* ctx, HopArgs& a) {
  const int Ls = ctx->g.Ls;
  int spb = ctx->spb;
  if (spb <= 0) {
    spb = 256 / Ls;
    if (spb > 64) spb = 64;
  }
  if (spb * Ls > 256) spb = 256 / Ls;
  if (spb < 1) spb = 1;
  // the M5D^{-1} epilogue stages spb * 12 * (Ls + 1) FP64 complex values in LDS: keep it <= 64 KiB
  while (spb > 1 && (size_t)spb * 12 * (Ls + 1) * 16 > 65536) --spb;
  a.spb = spb;
  a.Ls = Ls;
  a.V4h = ctx->g.V4h;
  a.nblocks = (int)((ctx->g.V4h + spb - 1) / spb);
  a.nb8 = (a.nblocks + 7) / 8;
  const double d = 5.0 - ctx->M5;
  a.d = d;
  a.inv_d = 1.0 / d;
  a.mf = ctx->mf;
  a.corner = -ctx->mf / (1.0 + ctx->mf * std::pow(d, -(double)Ls));
}

template <int PREC, bool DAG, int EPI>
static hipError_t launch_hop_t(const HopArgs& a, int nrhs, hipStream_t st) {
  using R = typename Store<PREC>::real;
  dim3 grid(a.nb8 * 8, nrhs);
  dim3 block(a.spb * a.Ls);
  size_t lds = (EPI == EPI_M5INV) ? (size_t)a.spb * 12 * (a.Ls + 1) * sizeof(cplx<R>) : 0;
  hipLaunchKernelGGL((hop_kernel<PREC, DAG, EPI>), grid, block, lds, st, a);
  return hipGetLastError();
}

template <int PREC>
static hipError_t launch_hop_p(const HopArgs& a, int dag, int epi, int nrhs, hipStream_t st) {
  switch (epi * 2 + (dag ? 1 : 0)) {
    case EPI_LIN * 2 + 0: return launch_hop_t<PREC, false, EPI_LIN>(a, nrhs, st);
    case EPI_LIN * 2 + 1: return launch_hop_t<PREC, true, EPI_LIN>(a, nrhs, st);
    case EPI_M5INV * 2 + 0: return launch_hop_t<PREC, false, EPI_M5INV>(a, nrhs, st);
    case EPI_M5INV * 2 + 1: return launch_hop_t<PREC, true, EPI_M5INV>(a, nrhs, st);
    case EPI_M5 * 2 + 0: return launch_hop_t<PREC, false, EPI_M5>(a, nrhs, st);
    case EPI_M5 * 2 + 1: return launch_hop_t<PREC, true, EPI_M5>(a, nrhs, st);
    case EPI_CHEB * 2 + 0: return launch_hop_t<PREC, false, EPI_CHEB>(a, nrhs, st);
    case EPI_CHEB * 2 + 1: return launch_hop_t<PREC, true, EPI_CHEB>(a, nrhs, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_hop(dwf_context* ctx, int prec, HopArgs a, int out_parity, int dag, int epi, int nrhs) {
  fill_shape(ctx, a);
  const long long V4h = ctx->g.V4h;
  a.nbr = ctx->nbr + (size_t)out_parity * 8 * V4h;
  const size_t link_elems = (size_t)out_parity * 8 * 9 * V4h;
  if (prec == DWF_F64)
    a.links = reinterpret_cast<const double2*>(ctx->links64) + link_elems;
  else
    a.links = reinterpret_cast<const float2*>(ctx->links32) + link_elems;
  a.stride = field_bytes_rhs(ctx, prec);
  timing_begin(ctx);
  hipError_t e;
  switch (prec) {
    case DWF_F64: e = launch_hop_p<DWF_F64>(a, dag, epi, nrhs, ctx->stream); break;
    case DWF_F32: e = launch_hop_p<DWF_F32>(a, dag, epi, nrhs, ctx->stream); break;
    default: e = launch_hop_p<DWF_F16S>(a, dag, epi, nrhs, ctx->stream); break;
  }
  timing_end(ctx);
  return e;
}

template <int PREC, bool DAG, bool INV>
static hipError_t launch_site5_t(const HopArgs& a, int nrhs, hipStream_t st) {
  using R = typename Store<PREC>::real;
  dim3 grid(a.nb8 * 8, nrhs);
  dim3 block(a.spb * a.Ls);
  size_t lds = INV ? (size_t)a.spb * 12 * (a.Ls + 1) * sizeof(cplx<R>) : 0;
  hipLaunchKernelGGL((site5_kernel<PREC, DAG, INV>), grid, block, lds, st, a);
  return hipGetLastError();
}

template <int PREC>
static hipError_t launch_site5_p(const HopArgs& a, int dag, int inv, int nrhs, hipStream_t st) {
  switch ((inv ? 2 : 0) + (dag ? 1 : 0)) {
    case 0: return launch_site5_t<PREC, false, false>(a, nrhs, st);
    case 1: return launch_site5_t<PREC, true, false>(a, nrhs, st);
    case 2: return launch_site5_t<PREC, false, true>(a, nrhs, st);
    default: return launch_site5_t<PREC, true, true>(a, nrhs, st);
  }
}

hipError_t launch_site5(dwf_context* ctx, int prec, const char* in, char* out, int dag, int inv, int nrhs) {
  HopArgs a{};
  fill_shape(ctx, a);
  a.in = in;
  a.out = out;
  a.stride = field_bytes_rhs(ctx, prec);
  switch (prec) {
    case DWF_F64: return launch_site5_p<DWF_F64>(a, dag, inv, nrhs, ctx->stream);
    case DWF_F32: return launch_site5_p<DWF_F32>(a, dag, inv, nrhs, ctx->stream);
    default: return launch_site5_p<DWF_F16S>(a, dag, inv, nrhs, ctx->stream);
  }
}

}  // namespace dwf
