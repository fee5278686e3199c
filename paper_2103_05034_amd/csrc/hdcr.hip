// Two-level HDCR solver on the full lattice (Algorithms A / B: pGCR(H_DW) with
// the composite V(1,1) preconditioner, a Chebyshev smoother and a CGNR coarse
// solve), FP64.
//
// * H_DW = Gamma_5 D_DW, (Gamma_5 v)_s = gamma_5 v_{Ls-1-s} (Spectrum of domain
//   wall fermions section).  D_DW is the two-launch hop pass of dwf_ddw; the
//   Gamma_5 is folded into a combine kernel.
// * Little Dirac operator A^{ab}_{jk} = <phi_j^a | H_DW | phi_k^b> (Two level
//   preconditioner section).  It couples a block to itself and to its eight
//   neighbours only, and is stored as that 9-point stencil, [nb][9][n][n]
//   complex with entry (j, k) at k * n + j: stencil point d < 8 is the block
//   that the hop direction d (2 mu + 0 forward, + 1 backward) leads to, point 8
//   the block itself.  It is built one basis vector k at a time: one kernel
//   writes the nine fields F_d = Gamma_5 (-1/2) D_hop^{(d), across a block face}
//   phi_k and F_8 = Gamma_5 (M5D - 1/2 D_hop^{(inside the block)}) phi_k, whose
//   restrictions onto the basis are column k of every stencil matrix.
// * Smoother S_cheb([a,b],N) (Chebyshev smoothers section) with M = H_DW:
//   [c_0/2 + sum c_j T_j(x(D^dag D))] H_DW r by Clenshaw's recurrence, each
//   step D_DW then D_DW^dag with the recurrence fused into the last hop pass.
// * Coarse solve: CG on A^dag A = A^2 (A is Hermitian because H_DW is).
// * V(1,1) (Composite V(1,1) section) and flexible GCR, host-driven.
#include <algorithm>
#include <cmath>
#include <new>
#include <type_traits>
#include <vector>

#include "dwf_internal.hpp"
#include "kernels.hpp"

using namespace dwf;

namespace dwf {
namespace {

constexpr int CB = 256;       // threads per block of the vector kernels
constexpr int CRED = 1024;    // partial sums of a reduction

// out = a + cb * Gamma_5 b on fields of both parities, one rhs ([2 V4h][12][Ls]
// complex); a may be null or alias out, b must not alias out (it is read at the
// mirrored slice).
__global__ void __launch_bounds__(CB) g5_combine_kernel(long long nsite, int Ls, const double2* __restrict__ a,
                                                         const double2* __restrict__ b, double cb,
                                                         double2* __restrict__ out) {
  const long long i = (long long)blockIdx.x * CB + threadIdx.x;
  const long long n = nsite * 12 * Ls;
  if (i >= n) return;
  const int s = (int)(i % Ls);
  const long long sc = i / Ls;  // site * 12 + component
  const int c = (int)(sc % 12);
  const double sg = c < 6 ? cb : -cb;  // gamma_5 = +1 on spins 0, 1
  const double2 v = b[sc * Ls + (Ls - 1 - s)];
  double2 o = make_double2(sg * v.x, sg * v.y);
  if (a) {
    const double2 w = a[i];
    o.x += w.x;
    o.y += w.y;
  }
  out[i] = o;
}

// One hop direction D at a site of the out parity: acc = (1 -+ g_mu) U psi
// (non-adjoint D_hop), the link read from the packed [D][9][V4h] table.
template <int D>
__device__ __forceinline__ void dir_term(const double2* __restrict__ lk, long long V4h, const cplx<double> psi[12],
                                         cplx<double> acc[12]) {
  constexpr int MU = D / 2;
  constexpr int SIGMA = (D % 2) ? +1 : -1;
  cplx<double> hs[6], chi[6];
  project<MU, SIGMA>(psi, hs);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double2 u0 = lk[(size_t)(3 * i + 0) * V4h], u1 = lk[(size_t)(3 * i + 1) * V4h],
                  u2 = lk[(size_t)(3 * i + 2) * V4h];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      cplx<double> v = cmul(cplx<double>{u0.x, u0.y}, hs[3 * sp + 0]);
      v = cfma(cplx<double>{u1.x, u1.y}, hs[3 * sp + 1], v);
      v = cfma(cplx<double>{u2.x, u2.y}, hs[3 * sp + 2], v);
      chi[3 * sp + i] = v;
    }
  }
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
  reconstruct<MU, SIGMA>(chi, acc);
}

struct CoarsenArgs {
  Geom g;
  int blk[4];
  double d, mf;                // 5 - M5, mass
  const double2* links;        // [2][8][9][V4h]
  const int* nbr;              // [2][8][V4h]
  const char* phi_e;           // basis vector, even half
  const char* phi_o;           // odd half
  char* out;                   // 9 fields, both layout: even halves of F_0..F_8, then the odd halves
  size_t fb;                   // bytes of a half field
};

template <int D>
__device__ __forceinline__ void coarsen_dir(const CoarsenArgs& a, int p, long long h, int s_src, const int c[4],
                                            const int ext[4], cplx<double> inside[12], cplx<double> face[12],
                                            bool& is_face) {
  constexpr int MU = D / 2;
  const long long V4h = a.g.V4h;
  const int nh = a.nbr[((size_t)p * 8 + D) * V4h + h];
  const char* src = p ? a.phi_e : a.phi_o;  // neighbours live on the other parity
  cplx<double> psi[12], t[12];
  Store<DWF_F64>::load(src, V4h, a.g.Ls, nh, s_src, psi);
  dir_term<D>(reinterpret_cast<const double2*>(a.links) + ((size_t)(p * 8 + D) * 9) * V4h + h, V4h, psi, t);
  const int cn = (D % 2) ? (c[MU] + ext[MU] - 1) % ext[MU] : (c[MU] + 1) % ext[MU];
  is_face = cn / a.blk[MU] != c[MU] / a.blk[MU];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    face[k] = is_face ? t[k] : cplx<double>{0, 0};
    if (!is_face) inside[k] = cadd(inside[k], t[k]);
  }
}

// Thread per (parity, half-lattice site, s).  F_r at slice s takes the terms at
// the mirrored slice Ls-1-s (the reflection in Gamma_5), times gamma_5.
__global__ void __launch_bounds__(CB) coarsen_kernel(CoarsenArgs a) {
  const long long V4h = a.g.V4h;
  const int Ls = a.g.Ls;
  const long long i = (long long)blockIdx.x * CB + threadIdx.x;
  if (i >= 2 * V4h * Ls) return;
  const int p = (int)(i / (V4h * Ls));
  const long long rem = i - (long long)p * V4h * Ls;
  const long long h = rem / Ls;
  const int s = (int)(rem - h * Ls);
  const int sr = Ls - 1 - s;
  int c[4];
  site_coords(a.g, p, h, c[0], c[1], c[2], c[3]);
  const int ext[4] = {a.g.X, a.g.Y, a.g.Z, a.g.T};
  cplx<double> inside[12], face[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) inside[k] = {0, 0};
  bool f;
  auto emit = [&](int r) {
    cplx<double> o[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double sg = k < 6 ? -0.5 : 0.5;  // Gamma_5 (-1/2)
      o[k] = {sg * face[k].re, sg * face[k].im};
    }
    Store<DWF_F64>::store(a.out + ((size_t)p * 9 + r) * a.fb, V4h, Ls, h, s, o);
  };
  coarsen_dir<0>(a, p, h, sr, c, ext, inside, face, f);
  emit(0);
  coarsen_dir<1>(a, p, h, sr, c, ext, inside, face, f);
  emit(1);
  coarsen_dir<2>(a, p, h, sr, c, ext, inside, face, f);
  emit(2);
  coarsen_dir<3>(a, p, h, sr, c, ext, inside, face, f);
  emit(3);
  coarsen_dir<4>(a, p, h, sr, c, ext, inside, face, f);
  emit(4);
  coarsen_dir<5>(a, p, h, sr, c, ext, inside, face, f);
  emit(5);
  coarsen_dir<6>(a, p, h, sr, c, ext, inside, face, f);
  emit(6);
  coarsen_dir<7>(a, p, h, sr, c, ext, inside, face, f);
  emit(7);
  // M5D at the mirrored slice: (5 - M5) v_s - P_- v_{s+1} - P_+ v_{s-1}, the
  // ends wrapping round with +mf instead of -1
  const char* self = p ? a.phi_o : a.phi_e;
  cplx<double> v0[12], vu[12], vd[12];
  Store<DWF_F64>::load(self, V4h, Ls, h, sr, v0);
  const int su = sr + 1 < Ls ? sr + 1 : 0, sd = sr > 0 ? sr - 1 : Ls - 1;
  const double cu = sr + 1 < Ls ? -1.0 : a.mf, cd = sr > 0 ? -1.0 : a.mf;
  Store<DWF_F64>::load(self, V4h, Ls, h, su, vu);
  Store<DWF_F64>::load(self, V4h, Ls, h, sd, vd);
  cplx<double> o[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    cplx<double> m = {a.d * v0[k].re, a.d * v0[k].im};
    if (k < 6) {  // P_+ (upper spins) from below
      m.re += cd * vd[k].re;
      m.im += cd * vd[k].im;
    } else {  // P_- (lower spins) from above
      m.re += cu * vu[k].re;
      m.im += cu * vu[k].im;
    }
    m.re -= 0.5 * inside[k].re;
    m.im -= 0.5 * inside[k].im;
    const double sg = k < 6 ? 1.0 : -1.0;
    o[k] = {sg * m.re, sg * m.im};
  }
  Store<DWF_F64>::store(a.out + ((size_t)p * 9 + 8) * a.fb, V4h, Ls, h, s, o);
}

// Stencil storage: complex128, or complex64 (the coarse solve's tolerance of a
// few per cent does not need FP64 matrix entries; vectors and sums stay FP64).
__device__ __forceinline__ void put(double2* p, double2 v) { *p = v; }
__device__ __forceinline__ void put(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }

// A[b][r][k][j] = coef[r][b][j] for basis vector k.
template <class T>
__global__ void __launch_bounds__(CB) coarse_scatter_kernel(const double2* __restrict__ coef, T* __restrict__ A,
                                                            int nb, int n, int k) {
  const long long i = (long long)blockIdx.x * CB + threadIdx.x;
  if (i >= (long long)9 * nb * n) return;
  const int j = (int)(i % n);
  const long long rb = i / n;
  const int b = (int)(rb % nb);
  const int r = (int)(rb / nb);
  put(&A[(((size_t)b * 9 + r) * n + k) * n + j], coef[i]);
}

// y[b] = sum_r A[b][r] x[neighbour_r(b)]: one workgroup per block, lane j
// computes row j; the nine input vectors pass through LDS.
template <class T>
__global__ void __launch_bounds__(64) coarse_matvec_kernel(const T* __restrict__ A, const int* __restrict__ bnbr,
                                                           int n, const double2* __restrict__ x,
                                                           double2* __restrict__ y) {
  __shared__ double2 xs[9 * 64];
  const int b = blockIdx.x;
  for (int i = threadIdx.x; i < 9 * n; i += 64) {
    const int r = i / n, k = i - r * n;
    const int src = r < 8 ? bnbr[(size_t)b * 8 + r] : b;
    xs[i] = x[(size_t)src * n + k];
  }
  __syncthreads();
  const int j = threadIdx.x;
  if (j >= n) return;
  double re = 0, im = 0;
  const T* Ab = A + (size_t)b * 9 * n * n;
  for (int r = 0; r < 9; ++r)
    for (int k = 0; k < n; ++k) {
      // each entry is read once per matvec: non-temporal loads (-10 % time in complex128)
      typedef typename std::conditional<sizeof(T) == 16, double, float>::type E;
      typedef E ev __attribute__((ext_vector_type(2)));
      const ev mv = __builtin_nontemporal_load(reinterpret_cast<const ev*>(Ab + ((size_t)r * n + k) * n + j));
      const T ms = {mv.x, mv.y};
      const double2 m = make_double2((double)ms.x, (double)ms.y);
      const double2 v = xs[r * n + k];
      re = fma(m.x, v.x, fma(-m.y, v.y, re));
      im = fma(m.x, v.y, fma(m.y, v.x, im));
    }
  y[(size_t)b * n + j] = make_double2(re, im);
}

// Fixed-order sums over the workgroup (wavefront shuffles, then the waves in
// order), valid on thread 0.
__device__ __forceinline__ void tree2(double& a, double& b) {
  __shared__ double red[2 * (CB / 64)];
  block_sum2(a, b, red);
}

// part[blk] (re) and part[CRED + blk] (im) of sum conj(x) y over n complex values
__global__ void __launch_bounds__(CB) cdot_kernel(long long n, const double2* __restrict__ x,
                                                  const double2* __restrict__ y, double* __restrict__ part) {
  double re = 0, im = 0;
  for (long long i = (long long)blockIdx.x * CB + threadIdx.x; i < n; i += (long long)CRED * CB) {
    const double2 a = x[i], b = y[i];
    re = fma(a.x, b.x, fma(a.y, b.y, re));
    im = fma(a.x, b.y, fma(-a.y, b.x, im));
  }
  tree2(re, im);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = re;
    part[CRED + blockIdx.x] = im;
  }
}

__global__ void __launch_bounds__(CB) csum_kernel(const double* __restrict__ part, double* __restrict__ out) {
  double re = 0, im = 0;
  for (int i = threadIdx.x; i < CRED; i += CB) {
    re += part[i];
    im += part[CRED + i];
  }
  tree2(re, im);
  if (threadIdx.x == 0) {
    out[0] = re;
    out[1] = im;
  }
}

// y = (ar + i ai) x + br y over n complex values (y not read when br == 0)
__global__ void __launch_bounds__(CB) caxpby_kernel(long long n, const double2* __restrict__ x, double ar, double ai,
                                                    double br, double2* y) {
  const long long i = (long long)blockIdx.x * CB + threadIdx.x;
  if (i >= n) return;
  double2 o = make_double2(0.0, 0.0);
  if (x) {
    const double2 v = x[i];
    o.x = ar * v.x - ai * v.y;
    o.y = ar * v.y + ai * v.x;
  }
  if (br != 0.0) {
    const double2 w = y[i];
    o.x += br * w.x;
    o.y += br * w.y;
  }
  y[i] = o;
}

// Device scalars of the coarse CG (one solve at a time).
enum CgSlot { CS_RR = 0, CS_QQ, CS_ALPHA, CS_STOP, CS_ACTIVE, CS_ITERS, CS_RRN, CS_BETA, CS_FLAG, CS_TMP, CS_N = 16 };

// cs[slot] = sum of the CRED real partials
__global__ void __launch_bounds__(CB) csum1_kernel(const double* __restrict__ part, double* __restrict__ cs, int slot) {
  double re = 0, im = 0;
  for (int i = threadIdx.x; i < CRED; i += CB) re += part[i];
  tree2(re, im);
  if (threadIdx.x == 0) cs[slot] = re;
}

__global__ void ccg_init_kernel(double* cs, double tol2) {
  const double bb = cs[CS_RR];
  cs[CS_STOP] = tol2 * bb;
  cs[CS_ACTIVE] = (bb > 0 && bb > cs[CS_STOP]) ? 1.0 : 0.0;
  cs[CS_ITERS] = 0;
  cs[CS_FLAG] = 0;
  cs[CS_ALPHA] = 0;
  cs[CS_BETA] = 0;
}

// alpha = |r|^2 / |A p|^2 while the solve is active, else 0 (the iteration is a no-op)
__global__ void ccg_alpha_kernel(double* cs) {
  double a = 0.0;
  if (cs[CS_ACTIVE] != 0.0) {
    a = cs[CS_RR] / cs[CS_QQ];
    if (!(cs[CS_QQ] > 0.0) || !isfinite(a)) {
      cs[CS_FLAG] = 1.0;
      cs[CS_ACTIVE] = 0.0;
      a = 0.0;
    }
  }
  cs[CS_ALPHA] = a;
}

// beta = |r_new|^2 / |r|^2; count the iteration; retire once |r_new|^2 <= tol^2 |b'|^2
__global__ void ccg_beta_kernel(double* cs) {
  if (cs[CS_ACTIVE] != 0.0) {
    const double rn = cs[CS_RRN];
    cs[CS_BETA] = rn / cs[CS_RR];
    cs[CS_RR] = rn;
    cs[CS_ITERS] += 1.0;
    if (!(rn > cs[CS_STOP])) cs[CS_ACTIVE] = 0.0;
  } else {
    cs[CS_BETA] = 0.0;
  }
}

// r -= alpha w with the partial sums of |r|^2
__global__ void __launch_bounds__(CB) caxpy_norm_kernel(long long n, const double2* __restrict__ w,
                                                        const double* __restrict__ cs, double2* __restrict__ r,
                                                        double* __restrict__ part) {
  const double a = cs[CS_ALPHA];
  double s = 0, dummy = 0;
  for (long long i = (long long)blockIdx.x * CB + threadIdx.x; i < n; i += (long long)CRED * CB) {
    const double2 v = w[i];
    double2 o = r[i];
    o.x -= a * v.x;
    o.y -= a * v.y;
    r[i] = o;
    s = fma(o.x, o.x, fma(o.y, o.y, s));
  }
  tree2(s, dummy);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// c += alpha p; p = r + beta p
__global__ void __launch_bounds__(CB) ccg_xp_kernel(long long n, double2* __restrict__ c, double2* __restrict__ p,
                                                    const double2* __restrict__ r, const double* __restrict__ cs) {
  const long long i = (long long)blockIdx.x * CB + threadIdx.x;
  if (i >= n) return;
  const double a = cs[CS_ALPHA], b = cs[CS_BETA];
  const double2 pv = p[i], rv = r[i];
  double2 cv = c[i];
  cv.x += a * pv.x;
  cv.y += a * pv.y;
  c[i] = cv;
  p[i] = make_double2(rv.x + b * pv.x, rv.y + b * pv.y);
}

unsigned blocks_for(long long n) { return (unsigned)((n + CB - 1) / CB); }

}  // namespace
}  // namespace dwf

// ---------------------------------------------------------------------------
// The solver object.
// ---------------------------------------------------------------------------
struct dwf_hdcr_s {
  dwf_context* h;
  int nvec, nk, nb;
  dwf_hdcr_params prm;
  const char* basis;   // caller's basis (packed both layout, nvec fields), set by dwf_hdcr_set_basis
  void* A;             // [nb][9][n][n], complex128 or complex64 (prm.coarse_prec)
  double2* coef;       // [9][nb][n]
  double2* cv[7];      // coarse vectors: d, c, r, p, q, w, b'
  double* part;        // [2][CRED] partials, 2 result doubles, then the coarse CG's CS_N scalars
  char* work;          // 9 both fields
  char* gb;            // GCR source Gamma_5 eta
  char* gr;            // GCR residual
  std::vector<char*> Z, W;
  size_t fb;           // bytes of a half field
  long long coarse_iters;
};

namespace {

constexpr size_t HALIGN = 256;
size_t hup(size_t n) { return (n + HALIGN - 1) / HALIGN * HALIGN; }

// A field of both parities: its even and odd halves.
struct BF {
  const char* e;
  const char* o;
};
struct BFm {
  char* e;
  char* o;
};
BFm whole(dwf_hdcr_s* hd, char* p) { return {p, p + hd->fb}; }
BF cwhole(const dwf_hdcr_s* hd, const char* p) { return {p, p + hd->fb}; }

size_t carve_hdcr(dwf_hdcr_s* d, const dwf_context* h, int nvec, int nk, char* base) {
  const size_t fb = field_bytes_rhs(h, DWF_F64);
  const size_t cvb = (size_t)h->nb * nvec * 16;
  size_t off = 0;
  auto take = [&](size_t n) -> char* {
    char* p = base ? base + off : nullptr;
    off += hup(n);
    return p;
  };
  dwf_hdcr_s tmp;
  dwf_hdcr_s* x = d ? d : &tmp;
  x->A = take((size_t)h->nb * 9 * nvec * nvec * 16);  // sized for complex128
  x->coef = reinterpret_cast<double2*>(take(9 * cvb));
  for (int i = 0; i < 7; ++i) x->cv[i] = reinterpret_cast<double2*>(take(cvb));
  x->part = reinterpret_cast<double*>(take((2 * CRED + 2 + CS_N) * sizeof(double)));
  x->work = take(9 * 2 * fb);
  x->gb = take(2 * fb);
  x->gr = take(2 * fb);
  x->Z.assign(nk, nullptr);
  x->W.assign(nk, nullptr);
  for (int i = 0; i < nk; ++i) {
    x->Z[i] = take(2 * fb);
    x->W[i] = take(2 * fb);
  }
  return off;
}

char* work_f(dwf_hdcr_s* hd, int i) { return hd->work + (size_t)i * 2 * hd->fb; }

// complex numbers in a both field of one rhs
long long both_len(const dwf_hdcr_s* hd) { return (long long)(2 * hd->fb / 16); }
long long coarse_len(const dwf_hdcr_s* hd) { return (long long)hd->nb * hd->nvec; }

hipError_t caxpby(dwf_hdcr_s* hd, long long n, const void* x, double ar, double ai, double br, void* y) {
  hipLaunchKernelGGL(caxpby_kernel, dim3(blocks_for(n)), dim3(CB), 0, hd->h->stream, n,
                     reinterpret_cast<const double2*>(x), ar, ai, br, reinterpret_cast<double2*>(y));
  return hipGetLastError();
}

// <x, y> over n complex values (synchronous)
int cdot(dwf_hdcr_s* hd, long long n, const void* x, const void* y, double& re, double& im) {
  hipLaunchKernelGGL(cdot_kernel, dim3(CRED), dim3(CB), 0, hd->h->stream, n, reinterpret_cast<const double2*>(x),
                     reinterpret_cast<const double2*>(y), hd->part);
  hipLaunchKernelGGL(csum_kernel, dim3(1), dim3(CB), 0, hd->h->stream, hd->part, hd->part + 2 * CRED);
  HIP_TRY(hipGetLastError());
  double r[2];
  HIP_TRY(hipMemcpyAsync(r, hd->part + 2 * CRED, sizeof r, hipMemcpyDeviceToHost, hd->h->stream));
  HIP_TRY(hipStreamSynchronize(hd->h->stream));
  re = r[0];
  im = r[1];
  return DWF_OK;
}

int cnorm2(dwf_hdcr_s* hd, long long n, const void* x, double& nn) {
  double im;
  return cdot(hd, n, x, x, nn, im);
}

// out = D_DW in (dag = 0) or D_DW^dag in: one hop launch per output parity
hipError_t ddw1(dwf_context* c, BF in, BFm out, int dag) {
  for (int p = 0; p < 2; ++p) {
    HopArgs a{};
    a.in = p ? in.e : in.o;
    a.x = p ? in.o : in.e;
    a.out = p ? out.o : out.e;
    a.alpha = -0.5;
    hipError_t e = launch_hop(c, DWF_F64, a, p, dag, EPI_M5, 1);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// out = ca D^dag D in + cb y + cc z + cw w (out may alias z or w); tmp = D in
hipError_t ddagd_step(dwf_context* c, BF in, BFm out, BF y, BF z, double ca, double cb, double cc, BF w, double cw,
                      BFm tmp) {
  hipError_t e = ddw1(c, in, tmp, 0);
  if (e != hipSuccess) return e;
  for (int p = 0; p < 2; ++p) {
    HopArgs b{};
    b.in = p ? tmp.e : tmp.o;
    b.x = p ? tmp.o : tmp.e;
    b.y = p ? y.o : y.e;
    b.z = p ? z.o : z.e;
    b.w = w.e ? (p ? w.o : w.e) : nullptr;
    b.out = p ? out.o : out.e;
    b.alpha = -0.5;
    b.ca = ca;
    b.cb = cb;
    b.cc = cc;
    b.cw = cw;
    e = launch_hop(c, DWF_F64, b, p, 1, EPI_CHEB, 1);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t g5_combine(dwf_hdcr_s* hd, const char* a, const char* b, double cb, char* out) {
  const long long nsite = 2 * hd->h->g.V4h;
  const long long n = nsite * 12 * hd->h->g.Ls;
  hipLaunchKernelGGL(g5_combine_kernel, dim3(blocks_for(n)), dim3(CB), 0, hd->h->stream, nsite, hd->h->g.Ls,
                     reinterpret_cast<const double2*>(a), reinterpret_cast<const double2*>(b), cb,
                     reinterpret_cast<double2*>(out));
  return hipGetLastError();
}

// out = r0 - H_DW x   (tmp: a both field)
int residual(dwf_hdcr_s* hd, const char* r0, const char* x, char* out, char* tmp) {
  HIP_TRY(ddw1(hd->h, cwhole(hd, x), whole(hd, tmp), 0));
  HIP_TRY(g5_combine(hd, r0, tmp, -1.0, out));
  return DWF_OK;
}

void smoother_coefficients(double lo, double hi, int N, std::vector<double>& c) {
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

// out = S_cheb([lo, hi], N) r with M = H_DW (uses work fields 0..3; out distinct from them and r)
int smoother(dwf_hdcr_s* hd, const char* r, char* out) {
  dwf_context* c = hd->h;
  const int N = hd->prm.smoother_order;
  const double lo = hd->prm.smoother_lo, hi = hd->prm.smoother_hi, wd = hi - lo;
  std::vector<double> cf;
  smoother_coefficients(lo, hi, N, cf);
  char* tmp = work_f(hd, 0);
  char* Wv = work_f(hd, 1);
  char* B1 = work_f(hd, 2);
  char* B2 = work_f(hd, 3);
  const long long n = both_len(hd);
  HIP_TRY(ddw1(c, cwhole(hd, r), whole(hd, tmp), 0));
  HIP_TRY(g5_combine(hd, nullptr, tmp, 1.0, Wv));               // w = H_DW r = M^dag r
  HIP_TRY(caxpby(hd, n, Wv, cf[N], 0.0, 0.0, B1));              // b_N = c_N w
  HIP_TRY(caxpby(hd, n, nullptr, 0.0, 0.0, 0.0, B2));           // b_{N+1} = 0
  for (int k = N - 1; k >= 1; --k) {
    // b_k = (4/wd) A b_{k+1} - (2(lo+hi)/wd) b_{k+1} - b_{k+2} + c_k w, over b_{k+2}
    HIP_TRY(ddagd_step(c, cwhole(hd, B1), whole(hd, B2), cwhole(hd, B1), cwhole(hd, B2), 4.0 / wd,
                       -2.0 * (hi + lo) / wd, -1.0, cwhole(hd, Wv), cf[k], whole(hd, tmp)));
    std::swap(B1, B2);
  }
  // out = x(A) b_1 - b_2 + c_0 w / 2
  HIP_TRY(ddagd_step(c, cwhole(hd, B1), whole(hd, out), cwhole(hd, B1), cwhole(hd, B2), 2.0 / wd, -(hi + lo) / wd,
                     -1.0, cwhole(hd, Wv), 0.5 * cf[0], whole(hd, tmp)));
  return DWF_OK;
}

hipError_t coarse_matvec(dwf_hdcr_s* hd, const double2* x, double2* y) {
  if (hd->prm.coarse_prec == DWF_F32)
    hipLaunchKernelGGL(coarse_matvec_kernel<float2>, dim3(hd->nb), dim3(64), 0, hd->h->stream,
                       reinterpret_cast<const float2*>(hd->A), hd->h->bnbr, hd->nvec, x, y);
  else
    hipLaunchKernelGGL(coarse_matvec_kernel<double2>, dim3(hd->nb), dim3(64), 0, hd->h->stream,
                       reinterpret_cast<const double2*>(hd->A), hd->h->bnbr, hd->nvec, x, y);
  return hipGetLastError();
}

// c = A^{-1} d by CG on A^2 c = A d from c = 0; stops when |A d - A^2 c| <= tol |A d|.
// The scalars stay on the device: once converged the remaining iterations of a batch
// are no-ops (alpha = 0), and the host looks at the state every CG_BATCH iterations,
// or sooner when the fall of |r|^2 over the last batch predicts convergence within it.
constexpr int CG_BATCH = 8;

int coarse_cgnr(dwf_hdcr_s* hd, const double2* d, double2* cvec, double tol, int maxiter, int* iters) {
  dwf_context* c = hd->h;
  const long long n = coarse_len(hd);
  double2 *r = hd->cv[2], *p = hd->cv[3], *q = hd->cv[4], *w = hd->cv[5], *bp = hd->cv[6];
  double* cs = hd->part + 2 * CRED + 2;
  auto norm_into = [&](const double2* v, int slot) {
    hipLaunchKernelGGL(cdot_kernel, dim3(CRED), dim3(CB), 0, c->stream, n, v, v, hd->part);
    hipLaunchKernelGGL(csum1_kernel, dim3(1), dim3(CB), 0, c->stream, hd->part, cs, slot);
  };
  HIP_TRY(coarse_matvec(hd, d, bp));
  HIP_TRY(caxpby(hd, n, nullptr, 0, 0, 0, cvec));
  HIP_TRY(caxpby(hd, n, bp, 1, 0, 0, r));
  HIP_TRY(caxpby(hd, n, bp, 1, 0, 0, p));
  norm_into(r, CS_RR);
  hipLaunchKernelGGL(ccg_init_kernel, dim3(1), dim3(1), 0, c->stream, cs, tol * tol);
  HIP_TRY(hipGetLastError());
  double st[CS_N];
  auto read_state = [&]() -> int {
    HIP_TRY(hipMemcpyAsync(st, cs, sizeof st, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return DWF_OK;
  };
  if (int rc = read_state()) return rc;
  const unsigned gb = blocks_for(n);
  int batch_size = CG_BATCH;
  for (int done = 0; st[CS_ACTIVE] != 0.0 && done < maxiter;) {
    const int batch = std::min(batch_size, maxiter - done);
    const double rr_before = st[CS_RR];
    for (int k = 0; k < batch; ++k) {
      HIP_TRY(coarse_matvec(hd, p, q));                       // q = A p
      norm_into(q, CS_QQ);                                    // |q|^2 = p.A^2 p
      hipLaunchKernelGGL(ccg_alpha_kernel, dim3(1), dim3(1), 0, c->stream, cs);
      HIP_TRY(coarse_matvec(hd, q, w));                       // w = A^2 p
      hipLaunchKernelGGL(caxpy_norm_kernel, dim3(CRED), dim3(CB), 0, c->stream, n, w, cs, r, hd->part);
      hipLaunchKernelGGL(csum1_kernel, dim3(1), dim3(CB), 0, c->stream, hd->part, cs, (int)CS_RRN);
      hipLaunchKernelGGL(ccg_beta_kernel, dim3(1), dim3(1), 0, c->stream, cs);
      hipLaunchKernelGGL(ccg_xp_kernel, dim3(gb), dim3(CB), 0, c->stream, n, cvec, p, r, cs);
      HIP_TRY(hipGetLastError());
    }
    done += batch;
    if (int rc = read_state()) return rc;
    if (st[CS_FLAG] != 0.0) return fail(DWF_EBREAKDOWN, "coarse CG breakdown");
    // iterations still needed at the rate |r|^2 fell over this batch
    batch_size = CG_BATCH;
    const double now = st[CS_RR], goal = st[CS_STOP];
    if (rr_before > 0.0 && now > 0.0 && now < rr_before && goal > 0.0 && now > goal) {
      const double left = std::log(goal / now) / (std::log(now / rr_before) / batch);
      if (left < CG_BATCH) batch_size = std::max(1, (int)std::ceil(left));
    }
  }
  const int it = (int)st[CS_ITERS];
  if (iters) *iters = it;
  hd->coarse_iters += it;
  return DWF_OK;
}

// out = Q r = P A^{-1} P^dag r
int coarse_correction(dwf_hdcr_s* hd, const char* r, char* out) {
  dwf_context* c = hd->h;
  HIP_TRY(launch_block_dot(c, DWF_F64, hd->basis, hd->nvec, r, 1, reinterpret_cast<double*>(hd->cv[0]), false));
  if (int rc = coarse_cgnr(hd, hd->cv[0], hd->cv[1], hd->prm.coarse_tol, hd->prm.coarse_maxiter, nullptr)) return rc;
  HIP_TRY(launch_block_prolong(c, DWF_F64, hd->basis, hd->nvec, reinterpret_cast<const double*>(hd->cv[1]), 1, out));
  return DWF_OK;
}

// x = V(1,1) r0 from x0 = 0 (uses work fields 0..6)
int vcycle(dwf_hdcr_s* hd, const char* r0, char* x) {
  const long long n = both_len(hd);
  char* rk = work_f(hd, 4);
  char* add = work_f(hd, 5);
  char* tmp = work_f(hd, 6);
  if (int rc = smoother(hd, r0, x)) return rc;               // x1 = S r0
  if (int rc = residual(hd, r0, x, rk, tmp)) return rc;      // r1 = r0 - M x1
  if (int rc = coarse_correction(hd, rk, add)) return rc;    // Q r1
  HIP_TRY(caxpby(hd, n, add, 1, 0, 1, x));                   // x2 = x1 + Q r1
  if (int rc = residual(hd, r0, x, rk, tmp)) return rc;      // r2 = r0 - M x2
  if (int rc = smoother(hd, rk, add)) return rc;             // S r2
  HIP_TRY(caxpby(hd, n, add, 1, 0, 1, x));                   // x3 = x2 + S r2
  return DWF_OK;
}

// v <- T_order(x(D^dag D)) v in place, x(A) = 2 (A - lo)/(hi - lo) - 1 (work fields 0, 1)
int filter_one(dwf_hdcr_s* hd, int order, double lo, double hi, BFm v) {
  if (order == 0) return DWF_OK;
  dwf_context* c = hd->h;
  const double w = hi - lo;
  const BFm tmp = whole(hd, work_f(hd, 0));
  const BF vc{v.e, v.o};
  // T_1 = x(A) v, then T_{j+1} = 2 x(A) T_j - T_{j-1} over the older buffer
  HIP_TRY(ddagd_step(c, vc, whole(hd, work_f(hd, 1)), vc, vc, 2.0 / w, -(hi + lo) / w, 0.0, BF{nullptr, nullptr},
                     0.0, tmp));
  BFm prev = v, cur = whole(hd, work_f(hd, 1));
  for (int j = 1; j < order; ++j) {
    HIP_TRY(ddagd_step(c, BF{cur.e, cur.o}, prev, BF{cur.e, cur.o}, BF{prev.e, prev.o}, 4.0 / w, -2.0 * (hi + lo) / w,
                       -1.0, BF{nullptr, nullptr}, 0.0, tmp));
    std::swap(prev, cur);
  }
  if (cur.e != v.e) {
    const long long nh = (long long)(hd->fb / 16);
    HIP_TRY(caxpby(hd, nh, cur.e, 1, 0, 0, v.e));
    HIP_TRY(caxpby(hd, nh, cur.o, 1, 0, 0, v.o));
  }
  return DWF_OK;
}

int check_hd(dwf_hdcr hd, bool need_basis) {
  if (!hd) return fail(DWF_EINVAL, "null HDCR handle");
  const dwf_context* h = hd->h;
  if (!h->coarse_both || h->nb != hd->nb)
    return fail(DWF_EINVAL, "HDCR: the handle's blocks changed since dwf_hdcr_create (need the same DWF_BOTH blocks)");
  if (need_basis && !hd->basis) return fail(DWF_EINVAL, "HDCR: call dwf_hdcr_set_basis first");
  return DWF_OK;
}

}  // namespace

extern "C" {

int dwf_hdw(dwf_handle h, const void* in, void* out, int nrhs) {
  if (int r = check_h(h)) return r;
  if (!in || !out || in == out || nrhs < 1) return fail(DWF_EINVAL, "dwf_hdw: in and out must be distinct, nrhs >= 1");
  if (h->prec != DWF_F64 || h->max_cg_rhs < 1)
    return fail(DWF_EINVAL, "dwf_hdw: needs a DWF_F64 handle with max_cg_rhs >= 1 (its FP64 work fields)");
  // D_DW into the handle's FP64 work fields, then Gamma_5 (which pairs s with
  // Ls-1-s, hence out of place) into out
  const size_t fb = field_bytes_rhs(h, DWF_F64);
  const char* src = reinterpret_cast<const char*>(in);
  char* dst = reinterpret_cast<char*>(out);
  const long long nsite = h->g.V4h;
  const long long n = nsite * 12 * h->g.Ls;
  for (int r = 0; r < nrhs; ++r) {
    // rhs r of a both-layout array: even half at r, odd half at nrhs + r
    const BF i{src + (size_t)r * fb, src + (size_t)(nrhs + r) * fb};
    const BFm t{h->r64, h->p64};
    HIP_TRY(ddw1(h, i, t, 0));
    for (int p = 0; p < 2; ++p) {
      hipLaunchKernelGGL(g5_combine_kernel, dim3(blocks_for(n)), dim3(CB), 0, h->stream, nsite, h->g.Ls, nullptr,
                         reinterpret_cast<const double2*>(p ? t.o : t.e), 1.0,
                         reinterpret_cast<double2*>(dst + (size_t)(p * nrhs + r) * fb));
      HIP_TRY(hipGetLastError());
    }
  }
  return DWF_OK;
}

size_t dwf_hdcr_workspace_bytes(dwf_handle h, int nvec, int nkrylov) {
  if (!h || !h->coarse_both || h->nb <= 0 || nvec < 1 || nvec > 64 || nkrylov < 1 || nkrylov > 64) return 0;
  return carve_hdcr(nullptr, h, nvec, nkrylov, nullptr) + HALIGN;
}

int dwf_hdcr_create(dwf_handle h, int nvec, const dwf_hdcr_params* prm, void* ws, size_t ws_bytes, dwf_hdcr* out) {
  if (int r = check_h(h)) return r;
  if (!out || !prm || !ws) return fail(DWF_EINVAL, "dwf_hdcr_create: NULL argument");
  *out = nullptr;
  if (h->prec != DWF_F64) return fail(DWF_EINVAL, "dwf_hdcr_create: needs a DWF_F64 handle");
  if (!h->coarse_both || h->nb <= 0) return fail(DWF_EINVAL, "dwf_hdcr_create: call dwf_set_blocks_ex with DWF_BOTH first");
  if (nvec < 1 || nvec > 64) return fail(DWF_EINVAL, "dwf_hdcr_create: nvec must be in [1, 64]");
  if (prm->nkrylov < 1 || prm->nkrylov > 64) return fail(DWF_EINVAL, "dwf_hdcr_create: nkrylov must be in [1, 64]");
  if (prm->coarse_prec != DWF_F64 && prm->coarse_prec != DWF_F32)
    return fail(DWF_EINVAL, "dwf_hdcr_create: coarse_prec must be DWF_F64 or DWF_F32");
  if (prm->smoother_order < 1 || !(prm->smoother_lo > 0) || !(prm->smoother_hi > prm->smoother_lo))
    return fail(DWF_EINVAL, "dwf_hdcr_create: smoother needs order >= 1 and 0 < lo < hi");
  if (!(prm->coarse_tol > 0) || prm->coarse_maxiter < 1)
    return fail(DWF_EINVAL, "dwf_hdcr_create: coarse_tol must be > 0 and coarse_maxiter >= 1");
  const size_t need = dwf_hdcr_workspace_bytes(h, nvec, prm->nkrylov);
  if (ws_bytes < need) return fail(DWF_ENOMEM, "dwf_hdcr_create: workspace %zu bytes < %zu needed", ws_bytes, need);
  dwf_hdcr_s* d = new (std::nothrow) dwf_hdcr_s();
  if (!d) return fail(DWF_ENOMEM, "dwf_hdcr_create: host allocation failed");
  d->h = h;
  d->nvec = nvec;
  d->nk = prm->nkrylov;
  d->nb = h->nb;
  d->prm = *prm;
  d->basis = nullptr;
  d->fb = field_bytes_rhs(h, DWF_F64);
  d->coarse_iters = 0;
  char* base = reinterpret_cast<char*>(ws);
  base += (HALIGN - reinterpret_cast<uintptr_t>(base) % HALIGN) % HALIGN;
  carve_hdcr(d, h, nvec, d->nk, base);
  *out = d;
  return DWF_OK;
}

int dwf_hdcr_destroy(dwf_hdcr hd) {
  delete hd;
  return DWF_OK;
}

int dwf_hdcr_set_basis(dwf_hdcr hd, const void* basis) {
  if (int r = check_hd(hd, false)) return r;
  if (!basis) return fail(DWF_EINVAL, "dwf_hdcr_set_basis: basis is NULL");
  dwf_context* c = hd->h;
  hd->basis = reinterpret_cast<const char*>(basis);
  const int n = hd->nvec;
  CoarsenArgs a{};
  a.g = c->g;
  for (int i = 0; i < 4; ++i) a.blk[i] = c->blk[i];
  a.d = 5.0 - c->M5;
  a.mf = c->mf;
  a.links = reinterpret_cast<const double2*>(c->links64);
  a.nbr = c->nbr;
  a.out = hd->work;
  a.fb = hd->fb;
  const long long threads = 2 * c->g.V4h * c->g.Ls;
  for (int k = 0; k < n; ++k) {
    a.phi_e = hd->basis + (size_t)k * hd->fb;
    a.phi_o = hd->basis + (size_t)(n + k) * hd->fb;
    hipLaunchKernelGGL(coarsen_kernel, dim3(blocks_for(threads)), dim3(CB), 0, c->stream, a);
    HIP_TRY(hipGetLastError());
    // the nine fields as a both-layout array of 9 rhs: restrict all of them
    HIP_TRY(launch_block_dot(c, DWF_F64, hd->basis, n, hd->work, 9, reinterpret_cast<double*>(hd->coef), false));
    const long long m = (long long)9 * hd->nb * n;
    if (hd->prm.coarse_prec == DWF_F32)
      hipLaunchKernelGGL(coarse_scatter_kernel<float2>, dim3(blocks_for(m)), dim3(CB), 0, c->stream, hd->coef,
                         reinterpret_cast<float2*>(hd->A), hd->nb, n, k);
    else
      hipLaunchKernelGGL(coarse_scatter_kernel<double2>, dim3(blocks_for(m)), dim3(CB), 0, c->stream, hd->coef,
                         reinterpret_cast<double2*>(hd->A), hd->nb, n, k);
    HIP_TRY(hipGetLastError());
  }
  return sync(c);
}

const void* dwf_hdcr_coarse_data(dwf_hdcr hd) { return hd ? hd->A : nullptr; }

int dwf_hdcr_coarse_apply(dwf_hdcr hd, const void* x, void* y) {
  if (int r = check_hd(hd, true)) return r;
  if (!x || !y || x == y) return fail(DWF_EINVAL, "dwf_hdcr_coarse_apply: x and y must be distinct");
  HIP_TRY(coarse_matvec(hd, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y)));
  return DWF_OK;
}

int dwf_hdcr_coarse_solve(dwf_hdcr hd, const void* d, void* c, double tol, int maxiter, int* iters) {
  if (int r = check_hd(hd, true)) return r;
  if (!d || !c || d == c || !(tol > 0) || maxiter < 0) return fail(DWF_EINVAL, "dwf_hdcr_coarse_solve: bad argument");
  return coarse_cgnr(hd, reinterpret_cast<const double2*>(d), reinterpret_cast<double2*>(c), tol, maxiter, iters);
}

int dwf_hdcr_filter(dwf_hdcr hd, int order, double lo, double hi, void* vecs, int nvecs) {
  if (int r = check_hd(hd, false)) return r;
  if (!vecs || nvecs < 1 || order < 0 || !(hi > lo)) return fail(DWF_EINVAL, "dwf_hdcr_filter: bad argument");
  char* V = reinterpret_cast<char*>(vecs);
  for (int k = 0; k < nvecs; ++k)
    if (int rc = filter_one(hd, order, lo, hi, BFm{V + (size_t)k * hd->fb, V + (size_t)(nvecs + k) * hd->fb})) return rc;
  return DWF_OK;
}

int dwf_hdcr_series(dwf_hdcr hd, int m, double lam_lo, double lam_max, int delta, int nvec, const void* eta,
                    void* out_series) {
  if (int r = check_hd(hd, false)) return r;
  if (!eta || !out_series || eta == out_series || m < 0 || delta < 1 || nvec < 1 || !(lam_max > lam_lo) ||
      !(lam_max > 0))
    return fail(DWF_EINVAL, "dwf_hdcr_series: bad argument");
  dwf_context* c = hd->h;
  const size_t fb = hd->fb;
  const long long nh = (long long)(fb / 16);
  char* S = reinterpret_cast<char*>(out_series);
  auto slot = [&](int k) { return BFm{S + (size_t)k * fb, S + (size_t)(nvec + k) * fb}; };
  auto cp = [&](BF from, BFm to) -> hipError_t {
    hipError_t e = caxpby(hd, nh, from.e, 1, 0, 0, to.e);
    return e != hipSuccess ? e : caxpby(hd, nh, from.o, 1, 0, 0, to.o);
  };
  const char* e = reinterpret_cast<const char*>(eta);
  // phi_0 = T_m(x_[lam_lo, lam_max](A)) eta
  const BFm s0 = slot(0);
  HIP_TRY(cp(BF{e, e + fb}, s0));
  if (int rc = filter_one(hd, m, lam_lo, lam_max, s0)) return rc;
  if (nvec == 1) return DWF_OK;
  // phi_k = T_{k delta}(2A/lam_max - 1) phi_0 from a second recurrence
  const BF s0c{s0.e, s0.o};
  BFm prev = whole(hd, work_f(hd, 1)), cur = whole(hd, work_f(hd, 2));
  const BFm tmp = whole(hd, work_f(hd, 0));
  HIP_TRY(cp(s0c, prev));
  HIP_TRY(ddagd_step(c, s0c, cur, s0c, s0c, 2.0 / lam_max, -1.0, 0.0, BF{nullptr, nullptr}, 0.0, tmp));
  int recorded = 1;
  for (int n = 1; recorded < nvec; ++n) {
    if (n % delta == 0) {
      HIP_TRY(cp(BF{cur.e, cur.o}, slot(recorded)));
      if (++recorded == nvec) break;
    }
    HIP_TRY(ddagd_step(c, BF{cur.e, cur.o}, prev, BF{cur.e, cur.o}, BF{prev.e, prev.o}, 4.0 / lam_max, -2.0, -1.0,
                       BF{nullptr, nullptr}, 0.0, tmp));
    std::swap(prev, cur);
  }
  return DWF_OK;
}

int dwf_hdcr_smoother(dwf_hdcr hd, const void* r, void* out) {
  if (int rc = check_hd(hd, false)) return rc;
  if (!r || !out || r == out) return fail(DWF_EINVAL, "dwf_hdcr_smoother: r and out must be distinct");
  return smoother(hd, reinterpret_cast<const char*>(r), reinterpret_cast<char*>(out));
}

int dwf_hdcr_vcycle(dwf_hdcr hd, const void* r, void* x, int* coarse_iters) {
  if (int rc = check_hd(hd, true)) return rc;
  if (!r || !x || r == x) return fail(DWF_EINVAL, "dwf_hdcr_vcycle: r and x must be distinct");
  const long long before = hd->coarse_iters;
  if (int rc = vcycle(hd, reinterpret_cast<const char*>(r), reinterpret_cast<char*>(x))) return rc;
  if (coarse_iters) *coarse_iters = (int)(hd->coarse_iters - before);
  return sync(hd->h);
}

int dwf_hdcr_solve(dwf_hdcr hd, const void* eta, void* psi, double tol, int maxiter, int* iters,
                   double* true_rel_resid, int* coarse_iters) {
  if (int rc = check_hd(hd, true)) return rc;
  if (!eta || !psi || eta == psi) return fail(DWF_EINVAL, "dwf_hdcr_solve: eta and psi must be distinct");
  if (!(tol > 0) || maxiter < 0) return fail(DWF_EINVAL, "dwf_hdcr_solve: tol must be > 0 and maxiter >= 0");
  dwf_context* c = hd->h;
  const long long n = both_len(hd);
  const long long before = hd->coarse_iters;
  char* x = reinterpret_cast<char*>(psi);
  char* b = hd->gb;
  char* r = hd->gr;
  char* tmp = work_f(hd, 7);
  HIP_TRY(g5_combine(hd, nullptr, reinterpret_cast<const char*>(eta), 1.0, b));  // b = Gamma_5 eta
  if (int rc = residual(hd, b, x, r, tmp)) return rc;
  double bb = 0, rr = 0;
  if (int rc = cnorm2(hd, n, b, bb)) return rc;
  if (int rc = cnorm2(hd, n, r, rr)) return rc;
  const double bn = std::sqrt(bb);
  double rn = std::sqrt(rr);
  int it = 0, last = 0;
  bool converged = bb == 0 || rn <= tol * bn, stopped = false;
  while (!converged && !stopped && it < maxiter) {
    for (int k = 0; k < hd->nk; ++k) {
      char* z = hd->Z[k];
      char* w = hd->W[k];
      if (int rc = vcycle(hd, r, z)) return rc;
      HIP_TRY(ddw1(c, cwhole(hd, z), whole(hd, tmp), 0));
      HIP_TRY(g5_combine(hd, nullptr, tmp, 1.0, w));  // w = M z
      for (int i = 0; i < k; ++i) {  // modified Gram-Schmidt against the earlier w_i (unit norm)
        double br = 0, bi = 0;
        if (int rc = cdot(hd, n, hd->W[i], w, br, bi)) return rc;
        HIP_TRY(caxpby(hd, n, hd->W[i], -br, -bi, 1, w));
        HIP_TRY(caxpby(hd, n, hd->Z[i], -br, -bi, 1, z));
      }
      double ww = 0;
      if (int rc = cnorm2(hd, n, w, ww)) return rc;
      if (!(ww > 0) || !std::isfinite(ww)) return fail(DWF_EBREAKDOWN, "dwf_hdcr_solve: GCR breakdown (M z = 0)");
      const double inv = 1.0 / std::sqrt(ww);
      HIP_TRY(caxpby(hd, n, w, inv, 0, 0, w));
      HIP_TRY(caxpby(hd, n, z, inv, 0, 0, z));
      double ar = 0, ai = 0;
      if (int rc = cdot(hd, n, w, r, ar, ai)) return rc;
      HIP_TRY(caxpby(hd, n, z, ar, ai, 1, x));
      HIP_TRY(caxpby(hd, n, w, -ar, -ai, 1, r));
      if (int rc = cnorm2(hd, n, r, rr)) return rc;
      rn = std::sqrt(rr);
      ++it;
      if (c->progress_fn && it - last >= c->progress_every) {
        last = it;
        const double rel = rn / bn;
        if (c->progress_fn(c->progress_user, it, 1, &rel)) stopped = true;
      }
      if (!std::isfinite(rn)) return fail(DWF_EBREAKDOWN, "dwf_hdcr_solve: non-finite residual");
      converged = rn <= tol * bn;
      if (converged || stopped || it >= maxiter) break;
    }
    if (!converged && !stopped && it < maxiter) {  // restart from the true residual
      if (int rc = residual(hd, b, x, r, tmp)) return rc;
    }
  }
  if (int rc = residual(hd, b, x, r, tmp)) return rc;
  double tr = 0;
  if (int rc = cnorm2(hd, n, r, tr)) return rc;
  const double rel = bb > 0 ? std::sqrt(tr / bb) : 0.0;
  if (iters) *iters = it;
  if (true_rel_resid) *true_rel_resid = rel;
  if (coarse_iters) *coarse_iters = (int)(hd->coarse_iters - before);
  if (!std::isfinite(rel)) return fail(DWF_EBREAKDOWN, "dwf_hdcr_solve: non-finite residual");
  if (stopped) return fail(DWF_ENOCONV, "dwf_hdcr_solve: stopped by the progress callback");
  if (!converged) return fail(DWF_ENOCONV, "dwf_hdcr_solve: no convergence in %d iterations", maxiter);
  return DWF_OK;
}

}  // extern "C"
