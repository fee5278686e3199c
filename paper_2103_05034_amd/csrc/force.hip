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

struct ForceArgs {
  const char* y[2];  // per-term passes: own spinor of the term, on even and odd sites (one pass: a)
  const char* z[2];  // per-term passes: neighbour spinor of the term (one pass: b)
  const int* nbr;    // [2][8][V4h]
  const int* order;  // [2][V4h] traversal order of the sites of each parity, or null (lexicographic)
  double2* grad;     // natural [T][Z][Y][X][4][3][3]
  Geom g;
  int spb;
  int nblocks;  // site blocks of spb sites per parity
  int nb8;      // workgroups per XCD (per parity and grid row in the per-term form)
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

// g -= sum_{n=0,1} hy[n]_i conj(hz[n]_j): one term of the gradient from the two
// projected half spinors (negated, as in term_outer).
__device__ __forceinline__ void outer_sub(const cplx<double> hy[6], const cplx<double> hz[6], cplx<double> g[9]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cplx<double> acc = g[3 * i + j];
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        const cplx<double> y = hy[3 * n + i], z = hz[3 * n + j];
        acc.re = fma(-y.re, z.re, acc.re);
        acc.re = fma(-y.im, z.im, acc.re);
        acc.im = fma(-y.im, z.re, acc.im);
        acc.im = fma(y.re, z.im, acc.im);
      }
      g[3 * i + j] = acc;
    }
}

// (1 + sg g_mu) projection of a spinor held in LDS (component c at
// own[c * stride]) for a direction mu known only at run time: h = u + sg B_mu l
// with the lower spin picked by address and the factor of B_mu (+-1 or +-i)
// applied as (cr, ci); one of cr, ci is zero, so each component is a single
// rounded add, as in the compile-time projection.
__device__ __forceinline__ void project_lds(const cplx<double>* own, int stride, int mu, double sg,
                                            cplx<double> h[6]) {
  // B_x l = (i l1, i l0), B_y l = (-l1, l0), B_z l = (i l0, -i l1), B_t l = (l0, l1)
  const int first = mu < 2 ? 9 : 6;   // lower spin feeding h[0..2]
  const int second = mu < 2 ? 6 : 9;  // lower spin feeding h[3..5]
  const double c0r = mu == 1 ? -sg : (mu == 3 ? sg : 0.0), c0i = (mu == 0 || mu == 2) ? sg : 0.0;
  const double c1r = (mu == 1 || mu == 3) ? sg : 0.0, c1i = mu == 0 ? sg : (mu == 2 ? -sg : 0.0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cplx<double> u0 = own[(size_t)a * stride], u1 = own[(size_t)(3 + a) * stride];
    const cplx<double> l = own[(size_t)(first + a) * stride], m = own[(size_t)(second + a) * stride];
    h[a] = {fma(c0r, l.re, fma(-c0i, l.im, u0.re)), fma(c0r, l.im, fma(c0i, l.re, u0.im))};
    h[3 + a] = {fma(c1r, m.re, fma(-c1i, m.im, u1.re)), fma(c1r, m.im, fma(c1i, m.re, u1.im))};
  }
}

// Both terms in one pass, with the four directions on four groups of lanes:
// lane (mu, site, s) with mu slowest, so a wave holds one direction when
// spb * Ls is a multiple of 64.  Every lane loads its two neighbours a(x + mu),
// b(x + mu) together, so the four directions' loads are in flight at once, and
// three of the twelve components of the site's own a(x) and b(x) (lane group mu
// takes components 3 mu .. 3 mu + 2) into LDS ([12][spb * Ls] each, so a
// wave's reads are contiguous).  Used for Ls <= 64.
template <bool SHUFFLE>
__global__ void __launch_bounds__(256) force_dir_kernel(ForceArgs fa) {
  extern __shared__ char smem_raw[];
  const int Ls = fa.g.Ls;
  const int spb = fa.spb;
  // one grid over (site block, parity) with the parity fastest, so the two
  // parities' workgroups of neighbouring sites run together and a spinor read
  // as a site's own is still in L2 when the other parity reads it as a neighbour
  const int bidx = blockIdx.x;
  const int both = (bidx & 7) * fa.nb8 + (bidx >> 3);
  if (both >= 2 * fa.nblocks) return;
  const int p = both & 1;
  const int logical = both >> 1;
  const int tid = threadIdx.x;
  const int per_dir = spb * Ls;
  const int mu = tid / per_dir;
  const int rem = tid - mu * per_dir;
  const int sl = rem / Ls;
  const int s = rem - sl * Ls;
  const long long V4h = fa.g.V4h;
  const long long h0 = (long long)logical * spb;
  const long long hq = h0 + sl;  // processing index
  const bool valid = hq < V4h;
  const long long h = fa.order && valid ? (long long)fa.order[(size_t)p * V4h + hq] : hq;
  // LDS: [4][spb][Ls][9] sums (without shuffles), then a(x) and b(x)
  cplx<double>* buf = reinterpret_cast<cplx<double>*>(smem_raw);
  cplx<double>* abuf = buf + (SHUFFLE ? 0 : (size_t)4 * per_dir * 9);
  cplx<double>* bbuf = abuf + (size_t)12 * per_dir;
  cplx<double> an[12], bn[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) an[c] = bn[c] = {0, 0};
  if (valid) {
    const long long nh = fa.nbr[((size_t)p * 8 + 2 * mu) * V4h + h];
    Store<DWF_F64>::load(fa.y[1 - p], V4h, Ls, nh, s, an);
    Store<DWF_F64>::load(fa.z[1 - p], V4h, Ls, nh, s, bn);
    const double2* pa = reinterpret_cast<const double2*>(fa.y[p]) + h * 12 * Ls + s;
    const double2* pb = reinterpret_cast<const double2*>(fa.z[p]) + h * 12 * Ls + s;
    double2 ta[3], tb[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ta[k] = pa[(size_t)(3 * mu + k) * Ls];
      tb[k] = pb[(size_t)(3 * mu + k) * Ls];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      abuf[(size_t)(3 * mu + k) * per_dir + rem] = {ta[k].x, ta[k].y};
      bbuf[(size_t)(3 * mu + k) * per_dir + rem] = {tb[k].x, tb[k].y};
    }
  }
  __syncthreads();
  // neighbours projected as soon as they are in: term 0 takes (1 - g_mu) b(x + mu),
  // term 1 (1 + g_mu) a(x + mu)
  cplx<double> hz0[6], hz1[6];
  switch (mu) {
    case 0: project<0, -1>(bn, hz0); project<0, +1>(an, hz1); break;
    case 1: project<1, -1>(bn, hz0); project<1, +1>(an, hz1); break;
    case 2: project<2, -1>(bn, hz0); project<2, +1>(an, hz1); break;
    default: project<3, -1>(bn, hz0); project<3, +1>(an, hz1); break;
  }
  cplx<double> gm[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) gm[k] = {0, 0};
  if (valid) {
    cplx<double> hy[6];
    project_lds(abuf + rem, per_dir, mu, -1.0, hy);  // term 0: a(x)
    outer_sub(hy, hz0, gm);
    project_lds(bbuf + rem, per_dir, mu, +1.0, hy);  // term 1: (1 + g_mu) b(x)
    outer_sub(hy, hz1, gm);
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
      const long long hq2 = h0 + sl2;
      if (hq2 >= V4h) continue;
      const long long h2 = fa.order ? (long long)fa.order[(size_t)p * V4h + hq2] : hq2;
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

// Lie-algebra force of every link, one thread per link: with M = U G^dag,
// F^a = -Im tr(T^a M), T^a = lambda^a / 2 and tr(lambda^a M) = sum_ij lambda^a_ij M_ji
// for the Gell-Mann matrices lambda^1 .. lambda^8.
__global__ void lie_force_kernel(const double2* __restrict__ U, const double2* __restrict__ G,
                                 double* __restrict__ F, long long nlinks) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nlinks) return;
  cplx<double> u[9], g[9], m[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double2 a = U[i * 9 + k], b = G[i * 9 + k];
    u[k] = {a.x, a.y};
    g[k] = {b.x, b.y};
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cplx<double> acc = {0, 0};
#pragma unroll
      for (int b = 0; b < 3; ++b) acc = cfma_conj(g[3 * c + b], u[3 * a + b], acc);  // U_ab conj(G_cb)
      m[3 * a + c] = acc;
    }
  auto M = [&](int r, int c) { return m[3 * r + c]; };
  double* f = F + i * 8;
  f[0] = -0.5 * (M(1, 0).im + M(0, 1).im);
  f[1] = -0.5 * (M(0, 1).re - M(1, 0).re);
  f[2] = -0.5 * (M(0, 0).im - M(1, 1).im);
  f[3] = -0.5 * (M(2, 0).im + M(0, 2).im);
  f[4] = -0.5 * (M(0, 2).re - M(2, 0).re);
  f[5] = -0.5 * (M(2, 1).im + M(1, 2).im);
  f[6] = -0.5 * (M(1, 2).re - M(2, 1).re);
  f[7] = -0.5 / sqrt(3.0) * (M(0, 0).im + M(1, 1).im - 2.0 * M(2, 2).im);
}

hipError_t launch_lie_force(dwf_context* ctx, const void* U, const void* G, double* F) {
  const long long nlinks = 2 * ctx->g.V4h * 4;
  const unsigned grid = (unsigned)((nlinks + 255) / 256);
  hipLaunchKernelGGL(lie_force_kernel, dim3(grid), dim3(256), 0, ctx->stream, reinterpret_cast<const double2*>(U),
                     reinterpret_cast<const double2*>(G), F, nlinks);
  return hipGetLastError();
}

hipError_t launch_force(dwf_context* ctx, const char* a_even, const char* a_odd, const char* b_even,
                        const char* b_odd, double* grad_U) {
  ForceArgs fa;
  fa.nbr = ctx->nbr;
  fa.order = nullptr;
  fa.grad = reinterpret_cast<double2*>(grad_U);
  fa.g = ctx->g;
  const int Ls = ctx->g.Ls;
  if (Ls <= 64) {  // one pass, lanes (mu, site, s): 4 Ls threads per site
    int spb = 256 / (4 * Ls);
    if (spb < 1) spb = 1;
    fa.spb = spb;
    fa.nblocks = (int)((ctx->g.V4h + spb - 1) / spb);
    fa.nb8 = (2 * fa.nblocks + 7) / 8;  // both parities in one interleaved grid
    fa.y[0] = a_even;
    fa.y[1] = a_odd;
    fa.z[0] = b_even;
    fa.z[1] = b_odd;
    fa.accumulate = 0;
    fa.order = ctx->order_mode ? ctx->order : nullptr;  // the hop kernels' site order
    const bool shuffle = (Ls & (Ls - 1)) == 0;
    const size_t lds = ((shuffle ? 0 : (size_t)4 * spb * Ls * 9) + (size_t)2 * spb * Ls * 12) * sizeof(cplx<double>);
    const dim3 grid(fa.nb8 * 8), block(4 * spb * Ls);
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
