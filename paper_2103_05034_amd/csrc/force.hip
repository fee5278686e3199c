// Gauge-link gradient of the pseudofermion action S = phi^dag (M_pc^dag M_pc)^{-1} phi.
//
// With a = (Y on even, W on odd) and b = (X on even, Z on odd) the variation
// is dS = -Re(a^dag dD_hop b), so the link U_mu(x) receives
//   G_mu(x) = -sum_s sum_spin [ a(x,s) ((1-g_mu) b(x+mu,s))^dag + ((1+g_mu) b(x,s)) a(x+mu,s)^dag ]
// (colour outer products), in the convention G = dS/dRe U + i dS/dIm U.
//
// One workgroup owns `spb` sites of one parity and all their s slices; each
// lane forms its slice's outer products and the s-sum runs through LDS.
#include "dwf_internal.hpp"
#include "kernels.hpp"

namespace dwf {

// full (1 + sigma g_mu) psi via the half-spinor identity
template <int MU, int SIGMA>
__device__ __forceinline__ void full_projection(const cplx<double> p[12], cplx<double> out[12]) {
  cplx<double> h[6];
  project<MU, SIGMA>(p, h);
#pragma unroll
  for (int c = 0; c < 12; ++c) out[c] = {0, 0};
  reconstruct<MU, SIGMA>(h, out);
}

template <int MU>
__device__ __forceinline__ void link_terms(const cplx<double> a[12], const cplx<double> b[12],
                                           const cplx<double> an[12], const cplx<double> bn[12],
                                           cplx<double> g[9]) {
  cplx<double> pb_n[12], pb[12];
  full_projection<MU, -1>(bn, pb_n);  // (1 - g_mu) b(x+mu)
  full_projection<MU, +1>(b, pb);     // (1 + g_mu) b(x)
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cplx<double> acc = {0, 0};
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        acc = cfma_conj(pb_n[3 * sp + j], a[3 * sp + i], acc);  // a_i conj(pb_n_j)
        acc = cfma_conj(an[3 * sp + j], pb[3 * sp + i], acc);   // pb_i conj(an_j)
      }
      g[3 * i + j] = {-acc.re, -acc.im};
    }
}

struct ForceArgs {
  const char* a[2];  // a on even, odd
  const char* b[2];
  const int* nbr;    // [2][8][V4h]
  double2* grad;     // natural [T][Z][Y][X][4][3][3]
  Geom g;
  int spb, nblocks, nb8;
};

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
  cplx<double> a[12], b[12];
  if (valid) {
    Store<DWF_F64>::load(fa.a[p], V4h, Ls, h, s, a);
    Store<DWF_F64>::load(fa.b[p], V4h, Ls, h, s, b);
  }
  int x = 0, y = 0, z = 0, t = 0;
  if (valid) site_coords(fa.g, p, h, x, y, z, t);
  const long long site = x + (long long)fa.g.X * (y + (long long)fa.g.Y * (z + (long long)fa.g.Z * t));
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    cplx<double> gm[9];
    if (valid) {
      const long long nh = fa.nbr[((size_t)p * 8 + 2 * mu) * V4h + h];
      cplx<double> an[12], bn[12];
      Store<DWF_F64>::load(fa.a[1 - p], V4h, Ls, nh, s, an);
      Store<DWF_F64>::load(fa.b[1 - p], V4h, Ls, nh, s, bn);
      switch (mu) {
        case 0: link_terms<0>(a, b, an, bn, gm); break;
        case 1: link_terms<1>(a, b, an, bn, gm); break;
        case 2: link_terms<2>(a, b, an, bn, gm); break;
        default: link_terms<3>(a, b, an, bn, gm); break;
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
      cplx<double> acc = {0, 0};
      for (int s2 = 0; s2 < Ls; ++s2) acc = cadd(acc, buf[((size_t)sl2 * Ls + s2) * 9 + k]);
      int x2, y2, z2, t2;
      site_coords(fa.g, p, h2, x2, y2, z2, t2);
      const long long site2 = x2 + (long long)fa.g.X * (y2 + (long long)fa.g.Y * (z2 + (long long)fa.g.Z * t2));
      fa.grad[(site2 * 4 + mu) * 9 + k] = make_double2(acc.re, acc.im);
    }
    __syncthreads();
  }
  (void)site;
}

hipError_t launch_force(dwf_context* ctx, const char* a_even, const char* a_odd, const char* b_even,
                        const char* b_odd, double* grad_U) {
  ForceArgs fa;
  fa.a[0] = a_even;
  fa.a[1] = a_odd;
  fa.b[0] = b_even;
  fa.b[1] = b_odd;
  fa.nbr = ctx->nbr;
  fa.grad = reinterpret_cast<double2*>(grad_U);
  fa.g = ctx->g;
  const int Ls = ctx->g.Ls;
  int spb = 256 / Ls;
  if (spb > 64) spb = 64;
  if (spb < 1) spb = 1;
  fa.spb = spb;
  fa.nblocks = (int)((ctx->g.V4h + spb - 1) / spb);
  fa.nb8 = (fa.nblocks + 7) / 8;
  const size_t lds = (size_t)spb * Ls * 9 * sizeof(cplx<double>);
  hipLaunchKernelGGL(force_kernel, dim3(fa.nb8 * 8, 2), dim3(spb * Ls), lds, ctx->stream, fa);
  return hipGetLastError();
}

}  // namespace dwf
