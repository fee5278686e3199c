// Layout conversion: natural lattice order <-> checkerboarded, site-fastest
// packed fields; link packing (double-stored per output parity, backward links
// pre-conjugated) and the nearest-neighbour tables.
#include "dwf_internal.hpp"
#include "kernels.hpp"

namespace dwf {

// Links of output parity po, direction dir = 2 mu + back, entry k = 3a + b:
//   forward  (back = 0): U_mu(x)[a][b]
//   backward (back = 1): (U_mu(x - mu)^dag)[a][b] = conj(U_mu(x - mu)[b][a])
__global__ void pack_links_kernel(Geom g, const double2* __restrict__ U, double2* __restrict__ l64,
                                  float2* __restrict__ l32) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * g.V4h) return;
  const int po = (int)(i / g.V4h);
  const long long h = i - po * g.V4h;
  int x, y, z, t;
  site_coords(g, po, h, x, y, z, t);
  const int L[4] = {g.X, g.Y, g.Z, g.T};
  for (int mu = 0; mu < 4; ++mu) {
    int c[4] = {x, y, z, t};
    for (int back = 0; back < 2; ++back) {
      if (back) c[mu] = (c[mu] - 1 + L[mu]) % L[mu];
      const long long site = c[0] + (long long)g.X * (c[1] + (long long)g.Y * (c[2] + (long long)g.Z * c[3]));
      const double2* u = U + (site * 4 + mu) * 9;
      const int dir = 2 * mu + back;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double2 v = back ? make_double2(u[3 * b + a].x, -u[3 * b + a].y) : u[3 * a + b];
          const size_t o = (((size_t)po * 8 + dir) * 9 + 3 * a + b) * g.V4h + h;
          l64[o] = v;
          if (l32) l32[o] = make_float2((float)v.x, (float)v.y);
        }
    }
  }
}

// nbr[po][dir][h] = half index (in the other parity) of the neighbour x +- mu
__global__ void neighbour_kernel(Geom g, int* __restrict__ nbr) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * g.V4h) return;
  const int po = (int)(i / g.V4h);
  const long long h = i - po * g.V4h;
  int x, y, z, t;
  site_coords(g, po, h, x, y, z, t);
  const int L[4] = {g.X, g.Y, g.Z, g.T};
  for (int mu = 0; mu < 4; ++mu)
    for (int back = 0; back < 2; ++back) {
      int c[4] = {x, y, z, t};
      c[mu] = back ? (c[mu] - 1 + L[mu]) % L[mu] : (c[mu] + 1) % L[mu];
      nbr[((size_t)po * 8 + 2 * mu + back) * g.V4h + h] = (int)half_index(g, c[0], c[1], c[2], c[3]);
    }
}

// natural [rhs][Ls][T][Z][Y][X][4][3] complex128 <-> packed half fields.
// grid: x over V4h * Ls spinors, y over rhs, z over the parities moved.
template <int PREC, bool UNPACK>
__global__ void pack_kernel(Geom g, double2* __restrict__ nat, char* __restrict__ packed, int nrhs, int p0,
                            size_t stride) {
  using R = typename Store<PREC>::real;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.V4h * g.Ls) return;
  const int rhs = blockIdx.y;
  const int pidx = blockIdx.z;
  const int p = p0 + pidx;
  const long long h = i / g.Ls;
  const int s = (int)(i - h * g.Ls);
  int x, y, z, t;
  site_coords(g, p, h, x, y, z, t);
  const long long nat_site =
      ((((long long)rhs * g.Ls + s) * g.T + t) * g.Z + z) * (long long)g.Y * g.X + (long long)y * g.X + x;
  double2* np = nat + nat_site * 12;
  char* base = packed + ((size_t)pidx * nrhs + rhs) * stride;
  cplx<R> v[12];
  if (!UNPACK) {
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = {(R)np[c].x, (R)np[c].y};
    Store<PREC>::store(base, g.V4h, g.Ls, h, s, v);
  } else {
    Store<PREC>::load(base, g.V4h, g.Ls, h, s, v);
#pragma unroll
    for (int c = 0; c < 12; ++c) np[c] = make_double2((double)v[c].re, (double)v[c].im);
  }
}

hipError_t launch_pack_links(dwf_context* ctx, const void* U) {
  const int bs = 256;
  const long long n = 2 * ctx->g.V4h;
  hipLaunchKernelGGL(pack_links_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, ctx->stream, ctx->g,
                     reinterpret_cast<const double2*>(U), reinterpret_cast<double2*>(ctx->links64),
                     reinterpret_cast<float2*>(ctx->links32));
  return hipGetLastError();
}

hipError_t launch_neighbours(dwf_context* ctx) {
  const int bs = 256;
  const long long n = 2 * ctx->g.V4h;
  hipLaunchKernelGGL(neighbour_kernel, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, ctx->stream, ctx->g,
                     ctx->nbr);
  return hipGetLastError();
}

template <int PREC>
static hipError_t launch_pack_p(dwf_context* ctx, const void* natural, char* packed, int nrhs, int parity,
                                bool unpack) {
  const int bs = 256;
  const long long n = ctx->g.V4h * ctx->g.Ls;
  const int np = parity == DWF_BOTH ? 2 : 1;
  const int p0 = parity == DWF_BOTH ? 0 : parity;
  dim3 grid((unsigned)((n + bs - 1) / bs), nrhs, np);
  const size_t stride = field_bytes_rhs(ctx, PREC);
  double2* nat = const_cast<double2*>(reinterpret_cast<const double2*>(natural));
  if (unpack)
    hipLaunchKernelGGL((pack_kernel<PREC, true>), grid, dim3(bs), 0, ctx->stream, ctx->g, nat, packed, nrhs, p0,
                       stride);
  else
    hipLaunchKernelGGL((pack_kernel<PREC, false>), grid, dim3(bs), 0, ctx->stream, ctx->g, nat, packed, nrhs, p0,
                       stride);
  return hipGetLastError();
}

hipError_t launch_pack(dwf_context* ctx, int prec, const void* natural, char* packed, int nrhs, int parity,
                       bool unpack) {
  switch (prec) {
    case DWF_F64: return launch_pack_p<DWF_F64>(ctx, natural, packed, nrhs, parity, unpack);
    case DWF_F32: return launch_pack_p<DWF_F32>(ctx, natural, packed, nrhs, parity, unpack);
    default: return launch_pack_p<DWF_F16S>(ctx, natural, packed, nrhs, parity, unpack);
  }
}

}  // namespace dwf
