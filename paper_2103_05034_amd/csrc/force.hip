// Gauge-link gradient of the pseudofermion action S = phi^dag (M_pc^dag M_pc)^{-1} phi.
//
// With a = (Y on even, W on odd) and b = (X on even, Z on odd) the variation
// is dS = -Re(a^dag dD_hop b), so the link U_mu(x) receives
//   G_mu(x) = -sum_s sum_spin [ a(x,s) ((1-g_mu) b(x+mu,s))^dag + ((1+g_mu) b(x,s)) a(x+mu,s)^dag ]
// (colour outer products), in the convention G = dS/dRe U + i dS/dIm U.
//
// For Ls <= 64 one pass forms both terms, with the four directions on four
// groups of lanes, and sums over s with wavefront swizzles (or LDS); longer
// s-columns take one pass per term.
#include "dwf_internal.hpp"
#include "kernels.hpp"

namespace dwf {

// Both terms have the form sum_spin (P y(x))_i conj(z(x+mu)_j) or
// sum_spin y(x)_i conj((P z(x+mu))_j) with P = 1 + sigma g_mu (term 0: y = a,
// z = b, sigma = -1; term 1: y = b, z = a, sigma = +1).  P is Hermitian and
// P psi = (h, sigma B^dag h) with h = u + sigma B l and B unitary, so either
// form equals sum_{n=0,1} h_y[n]_i conj(h_z[n]_j): an outer product of two
// half spinors, half the work of the full spin sum.
template <int MU, int SIGMA>
__device__ __forceinline__ void term_outer(const cplx<double> y[12], const cplx<double> zn[12], cplx<double> g[9]) {
  cplx<double> hy[6], hz[6];
  project<MU, SIGMA>(y, hy);
  project<MU, SIGMA>(zn, hz);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cplx<double> acc = {0, 0};
#pragma unroll
      for (int n = 0; n < 2; ++n) acc = cfma_conj(hz[3 * n + j], hy[3 * n + i], acc);  // hy_i conj(hz_j)
      g[3 * i + j] = {-acc.re, -acc.im};
    }
}

// One butterfly step on a double with a DPP lane swizzle (two 32-bit moves).
template <int CTRL>
__device__ __forceinline__ double dpp_swap(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Sum of v over each group of `width` consecutive lanes (width a power of two
// up to 64), returned in every lane of the group; a fixed order for a given
// width.  Within a row of 16 lanes the partners come from DPP swizzles (row
// mirror, half-row mirror, then the quad permutations of lane xor 2 and xor
// 1), which pair every lane with one of the other half at each step; wider
// groups first add across rows with shuffles.
__device__ __forceinline__ double group_sum(double v, int width) {
  for (int off = width >> 1; off >= 16; off >>= 1) v += __shfl_xor(v, off, width);
  if (width >= 16) v += dpp_swap<0x140>(v);  // row_mirror: lane i <-> 15 - i
  if (width >= 8) v += dpp_swap<0x141>(v);   // row_half_mirror: lane i <-> 7 - i within 8
  if (width >= 4) v += dpp_swap<0x4e>(v);    // quad_perm [2, 3, 0, 1]
  if (width >= 2) v += dpp_swap<0xb1>(v);    // quad_perm [1, 0, 3, 2]
  return v;
}

struct ForceArgs {
  const char* y[2];  // per-term passes: own spinor of the term, on even and odd sites (one pass: a)
  const char* z[2];  // per-term passes: neighbour spinor of the term (one pass: b)
  const int* nbr;    // [2][8][V4h]
  double2* grad;     // natural [T][Z][Y][X][4][3][3]
  Geom g;
  int spb, nblocks, nb8;
  int accumulate;    // 0: grad = term; 1: grad += term
};

// One workgroup owns `spb` sites of one parity and all their s slices, and
// loops over the four directions: the form for Ls > 64, where four lanes per
// (site, s) would not fit a workgroup.  The sum over s runs through LDS.
template <int SIGMA>
__global__ void __launch_bounds__(256) force_kernel(ForceArgs fa) {
  extern __shared__ char smem_raw[];
  cplx<double>* buf = reinterpret_cast<cplx<double>*>(smem_raw);  // [spb][Ls][9]
  const int Ls = fa.g.Ls;
  const int bidx = blockIdx.x;
  const int logical = (bidx & 7) * fa.nb8 + (bidx >> 3);
  if (logical >= fa.nblocks) return;
  const int p = blockIdx.y;
  const int tid = threadIdx.x;
  const int sl = tid / Ls;
  const int s = tid - sl * Ls;
  const long long V4h = fa.g.V4h;
  const long long h0 = (long long)logical * fa.spb;
  const long long h = h0 + sl;
  const bool valid = (sl < fa.spb) && (h < V4h);
  cplx<double> y[12];
  if (valid) Store<DWF_F64>::load(fa.y[p], V4h, Ls, h, s, y);
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    cplx<double> gm[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) gm[k] = {0, 0};
    if (valid) {
      const long long nh = fa.nbr[((size_t)p * 8 + 2 * mu) * V4h + h];
      cplx<double> zn[12];
      Store<DWF_F64>::load(fa.z[1 - p], V4h, Ls, nh, s, zn);
      switch (mu) {
        case 0: term_outer<0, SIGMA>(y, zn, gm); break;
        case 1: term_outer<1, SIGMA>(y, zn, gm); break;
        case 2: term_outer<2, SIGMA>(y, zn, gm); break;
        default: term_outer<3, SIGMA>(y, zn, gm); break;
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) buf[((size_t)sl * Ls + s) * 9 + k] = gm[k];
    }
    __syncthreads();
    for (int idx = tid; idx < fa.spb * 9; idx += blockDim.x) {
      const int sl2 = idx / 9;
      const int k = idx - 9 * sl2;
      const long long h2 = h0 + sl2;
      if (h2 >= V4h) continue;
      // four interleaved partial sums over s, added in a fixed order
      cplx<double> p4[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
      int s2 = 0;
      for (; s2 + 3 < Ls; s2 += 4)
#pragma unroll
        for (int q = 0; q < 4; ++q) p4[q] = cadd(p4[q], buf[((size_t)sl2 * Ls + s2 + q) * 9 + k]);
      for (; s2 < Ls; ++s2) p4[0] = cadd(p4[0], buf[((size_t)sl2 * Ls + s2) * 9 + k]);
      cplx<double> acc = cadd(cadd(p4[0], p4[1]), cadd(p4[2], p4[3]));
      int x2, y2, z2, t2;
      site_coords(fa.g, p, h2, x2, y2, z2, t2);
      const long long site2 = x2 + (long long)fa.g.X * (y2 + (long long)fa.g.Y * (z2 + (long long)fa.g.Z * t2));
      double2* out = fa.grad + (site2 * 4 + mu) * 9 + k;
      if (fa.accumulate) {
        const double2 o = *out;
        acc = {o.x + acc.re, o.y + acc.im};
      }
      *out = make_double2(acc.re, acc.im);
    }
    __syncthreads();
  }
}

// Both terms in one pass, with the four directions on four groups of lanes:
// lane (mu, site, s) with mu slowest, so a wave holds one direction when
// spb * Ls is a multiple of 64.  The direction-0 lanes load a(x) and b(x) of
// their (site, s) once into LDS ([12][spb * Ls] each, so a wave's reads are
// contiguous); every lane loads its two neighbours a(x + mu), b(x + mu)
// together, so the four directions' loads are in flight at once, and forms
// term 0 (a(x) with b(x + mu)) and then term 1 (b(x) with a(x + mu)) from half
// spinors.  Used for Ls <= 64.
template <bool SHUFFLE>
__global__ void __launch_bounds__(256) force_dir_kernel(ForceArgs fa) {
  extern __shared__ char smem_raw[];
  const int Ls = fa.g.Ls;
  const int spb = fa.spb;
  const int bidx = blockIdx.x;
  const int logical = (bidx & 7) * fa.nb8 + (bidx >> 3);
  if (logical >= fa.nblocks) return;
  const int p = blockIdx.y;
  const int tid = threadIdx.x;
  const int per_dir = spb * Ls;
  const int mu = tid / per_dir;
  const int rem = tid - mu * per_dir;
  const int sl = rem / Ls;
  const int s = rem - sl * Ls;
  const long long V4h = fa.g.V4h;
  const long long h0 = (long long)logical * spb;
  const long long h = h0 + sl;
  const bool valid = h < V4h;
  // LDS: [4][spb][Ls][9] sums (without shuffles), then a(x) and b(x)
  cplx<double>* buf = reinterpret_cast<cplx<double>*>(smem_raw);
  cplx<double>* abuf = buf + (SHUFFLE ? 0 : (size_t)4 * per_dir * 9);
  cplx<double>* bbuf = abuf + (size_t)12 * per_dir;
  cplx<double> an[12], bn[12];
  if (valid) {
    const long long nh = fa.nbr[((size_t)p * 8 + 2 * mu) * V4h + h];
    Store<DWF_F64>::load(fa.y[1 - p], V4h, Ls, nh, s, an);
    Store<DWF_F64>::load(fa.z[1 - p], V4h, Ls, nh, s, bn);
  }
  if (mu == 0 && valid) {
    cplx<double> t[12];
    Store<DWF_F64>::load(fa.y[p], V4h, Ls, h, s, t);
#pragma unroll
    for (int c = 0; c < 12; ++c) abuf[(size_t)c * per_dir + rem] = t[c];
    Store<DWF_F64>::load(fa.z[p], V4h, Ls, h, s, t);
#pragma unroll
    for (int c = 0; c < 12; ++c) bbuf[(size_t)c * per_dir + rem] = t[c];
  }
  __syncthreads();
  cplx<double> gm[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) gm[k] = {0, 0};
  if (valid) {
    cplx<double> own[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) own[c] = abuf[(size_t)c * per_dir + rem];
    switch (mu) {  // term 0: a(x) with (1 - g_mu) b(x + mu)
      case 0: term_outer<0, -1>(own, bn, gm); break;
      case 1: term_outer<1, -1>(own, bn, gm); break;
      case 2: term_outer<2, -1>(own, bn, gm); break;
      default: term_outer<3, -1>(own, bn, gm); break;
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) own[c] = bbuf[(size_t)c * per_dir + rem];
    cplx<double> g1[9];
    switch (mu) {  // term 1: (1 + g_mu) b(x) with a(x + mu)
      case 0: term_outer<0, +1>(own, an, g1); break;
      case 1: term_outer<1, +1>(own, an, g1); break;
      case 2: term_outer<2, +1>(own, an, g1); break;
      default: term_outer<3, +1>(own, an, g1); break;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) gm[k] = cadd(gm[k], g1[k]);
  }
  if constexpr (SHUFFLE) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      gm[k].re = group_sum(gm[k].re, Ls);
      gm[k].im = group_sum(gm[k].im, Ls);
    }
    if (valid && s == 0) {
      int x, y1, z, t;
      site_coords(fa.g, p, h, x, y1, z, t);
      const long long site = x + (long long)fa.g.X * (y1 + (long long)fa.g.Y * (z + (long long)fa.g.Z * t));
      double2* out = fa.grad + (site * 4 + mu) * 9;
#pragma unroll
      for (int k = 0; k < 9; ++k) out[k] = make_double2(gm[k].re, gm[k].im);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) buf[(size_t)tid * 9 + k] = gm[k];
    __syncthreads();
    for (int idx = tid; idx < 4 * spb * 9; idx += blockDim.x) {
      const int g = idx / 9;  // (mu, site) group
      const int k = idx - 9 * g;
      const int mu2 = g / spb;
      const int sl2 = g - mu2 * spb;
      const long long h2 = h0 + sl2;
      if (h2 >= V4h) continue;
      // four interleaved partial sums over s, added in a fixed order
      cplx<double> p4[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
      const cplx<double>* col = buf + (size_t)g * Ls * 9 + k;
      int s2 = 0;
      for (; s2 + 3 < Ls; s2 += 4)
#pragma unroll
        for (int q = 0; q < 4; ++q) p4[q] = cadd(p4[q], col[(size_t)(s2 + q) * 9]);
      for (; s2 < Ls; ++s2) p4[0] = cadd(p4[0], col[(size_t)s2 * 9]);
      const cplx<double> acc = cadd(cadd(p4[0], p4[1]), cadd(p4[2], p4[3]));
      int x2, y2, z2, t2;
      site_coords(fa.g, p, h2, x2, y2, z2, t2);
      const long long site2 = x2 + (long long)fa.g.X * (y2 + (long long)fa.g.Y * (z2 + (long long)fa.g.Z * t2));
      fa.grad[(site2 * 4 + mu2) * 9 + k] = make_double2(acc.re, acc.im);
    }
  }
}

hipError_t launch_force(dwf_context* ctx, const char* a_even, const char* a_odd, const char* b_even,
                        const char* b_odd, double* grad_U) {
  ForceArgs fa;
  fa.nbr = ctx->nbr;
  fa.grad = reinterpret_cast<double2*>(grad_U);
  fa.g = ctx->g;
  const int Ls = ctx->g.Ls;
  if (Ls <= 64) {  // one pass, lanes (mu, site, s): 4 Ls threads per site
    int spb = 256 / (4 * Ls);
    if (spb < 1) spb = 1;
    fa.spb = spb;
    fa.nblocks = (int)((ctx->g.V4h + spb - 1) / spb);
    fa.nb8 = (fa.nblocks + 7) / 8;
    fa.y[0] = a_even;
    fa.y[1] = a_odd;
    fa.z[0] = b_even;
    fa.z[1] = b_odd;
    fa.accumulate = 0;
    const bool shuffle = (Ls & (Ls - 1)) == 0;
    const size_t lds = ((shuffle ? 0 : (size_t)4 * spb * Ls * 9) + (size_t)2 * spb * Ls * 12) * sizeof(cplx<double>);
    const dim3 grid(fa.nb8 * 8, 2), block(4 * spb * Ls);
    if (shuffle)
      hipLaunchKernelGGL((force_dir_kernel<true>), grid, block, lds, ctx->stream, fa);
    else
      hipLaunchKernelGGL((force_dir_kernel<false>), grid, block, lds, ctx->stream, fa);
    return hipGetLastError();
  }
  // Ls > 64: one lane per (site, s) looping over directions, one pass per term
  int spb = 256 / Ls;
  if (spb < 1) spb = 1;
  fa.spb = spb;
  fa.nblocks = (int)((ctx->g.V4h + spb - 1) / spb);
  fa.nb8 = (fa.nblocks + 7) / 8;
  const size_t lds = (size_t)spb * Ls * 9 * sizeof(cplx<double>);
  const dim3 grid(fa.nb8 * 8, 2), block(spb * Ls);
  // term 0: a(x) with (1 - g_mu) b(x + mu); term 1: (1 + g_mu) b(x) with a(x + mu), added
  for (int term = 0; term < 2; ++term) {
    fa.y[0] = term ? b_even : a_even;
    fa.y[1] = term ? b_odd : a_odd;
    fa.z[0] = term ? a_even : b_even;
    fa.z[1] = term ? a_odd : b_odd;
    fa.accumulate = term;
    if (term == 0)
      hipLaunchKernelGGL((force_kernel<-1>), grid, block, lds, ctx->stream, fa);
    else
      hipLaunchKernelGGL((force_kernel<+1>), grid, block, lds, ctx->stream, fa);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace dwf
