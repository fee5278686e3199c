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
// component are contiguous along s; the workgroup's links (shared by the Ls
// lanes of a site) are staged once in LDS; the M5D / M5D^{-1} epilogues see
// whole s-columns of a site.  The eight neighbour-spinor loads are software
// pipelined DEPTH directions deep, so a wave keeps several directions of
// loads in flight instead of draining the memory queue per direction.
// Workgroups are remapped so that each XCD (workgroups are dealt round-robin
// over the 8 XCDs) sweeps one contiguous range of sites, which keeps the
// stencil's neighbour reuse inside one L2.
#include <algorithm>
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

// One direction: project the neighbour spinor, rotate by the link (read from
// the LDS copy, layout [dir*9 + k][spb]) and reconstruct into acc.
template <class R, bool DAG, int D>
__device__ __forceinline__ void hop_compute(const cplx<R> psi[12], const cplx<R>* __restrict__ ll, int spb, int sl,
                                            cplx<R> acc[12]) {
  constexpr int MU = D / 2;
  constexpr int BACK = D % 2;
  constexpr int SIGMA = DAG ? (BACK ? -1 : +1) : (BACK ? +1 : -1);
  cplx<R> hs[6];
  project<MU, SIGMA>(psi, hs);
  cplx<R> chi[6];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const cplx<R> u0 = ll[(D * 9 + 3 * i + 0) * spb + sl];
    const cplx<R> u1 = ll[(D * 9 + 3 * i + 1) * spb + sl];
    const cplx<R> u2 = ll[(D * 9 + 3 * i + 2) * spb + sl];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      cplx<R> v = cmul(u0, hs[3 * sp + 0]);
      v = cfma(u1, hs[3 * sp + 1], v);
      v = cfma(u2, hs[3 * sp + 2], v);
      chi[3 * sp + i] = v;
    }
  }
  reconstruct<MU, SIGMA>(chi, acc);
}

// The same direction for an FP16 + scale neighbour, without unpacking it:
// the projection reads the halves directly (each real is one mixed-precision
// FMA, f16 * (+-1) + f16 in FP32; `one` is 1.0 passed at run time so that the
// FMA is not folded into an add of two conversions), the link multiply runs on
// the unscaled half spinor, and the site's scale enters the reconstruction's
// FMAs.  48 fewer vector instructions per direction than unpack + project.
template <int MU, int SIGMA>
__device__ __forceinline__ void project_f16(const typename Store<DWF_F16S>::Raw& r, float one, cplx<float> h[6]) {
  const float sg = SIGMA > 0 ? one : -one;
  auto re = [&](int c) { return r.q[c / 4][2 * (c % 4)]; };
  auto im = [&](int c) { return r.q[c / 4][2 * (c % 4) + 1]; };
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int u0 = a, u1 = 3 + a, l0 = 6 + a, l1 = 9 + a;
    if (MU == 0) {  // u0 + sg i l1, u1 + sg i l0
      h[a] = {fmaf((float)im(l1), -sg, (float)re(u0)), fmaf((float)re(l1), sg, (float)im(u0))};
      h[3 + a] = {fmaf((float)im(l0), -sg, (float)re(u1)), fmaf((float)re(l0), sg, (float)im(u1))};
    } else if (MU == 1) {  // u0 - sg l1, u1 + sg l0
      h[a] = {fmaf((float)re(l1), -sg, (float)re(u0)), fmaf((float)im(l1), -sg, (float)im(u0))};
      h[3 + a] = {fmaf((float)re(l0), sg, (float)re(u1)), fmaf((float)im(l0), sg, (float)im(u1))};
    } else if (MU == 2) {  // u0 + sg i l0, u1 - sg i l1
      h[a] = {fmaf((float)im(l0), -sg, (float)re(u0)), fmaf((float)re(l0), sg, (float)im(u0))};
      h[3 + a] = {fmaf((float)im(l1), sg, (float)re(u1)), fmaf((float)re(l1), -sg, (float)im(u1))};
    } else {  // u0 + sg l0, u1 + sg l1
      h[a] = {fmaf((float)re(l0), sg, (float)re(u0)), fmaf((float)im(l0), sg, (float)im(u0))};
      h[3 + a] = {fmaf((float)re(l1), sg, (float)re(u1)), fmaf((float)im(l1), sg, (float)im(u1))};
    }
  }
}

template <bool DAG, int D>
__device__ __forceinline__ void hop_compute_f16(const typename Store<DWF_F16S>::Raw& r, float one,
                                                const cplx<float>* __restrict__ ll, int spb, int sl,
                                                cplx<float> acc[12]) {
  constexpr int MU = D / 2;
  constexpr int BACK = D % 2;
  constexpr int SIGMA = DAG ? (BACK ? -1 : +1) : (BACK ? +1 : -1);
  cplx<float> hs[6];
  project_f16<MU, SIGMA>(r, one, hs);
  cplx<float> chi[6];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const cplx<float> u0 = ll[(D * 9 + 3 * i + 0) * spb + sl];
    const cplx<float> u1 = ll[(D * 9 + 3 * i + 1) * spb + sl];
    const cplx<float> u2 = ll[(D * 9 + 3 * i + 2) * spb + sl];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      cplx<float> v = cmul(u0, hs[3 * sp + 0]);
      v = cfma(u1, hs[3 * sp + 1], v);
      v = cfma(u2, hs[3 * sp + 2], v);
      chi[3 * sp + i] = v;
    }
  }
  // acc += scale * (chi, sigma B^dag chi): the lower half as in reconstruct, with the scale in the FMA
  cplx<float> t[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) t[c] = {0.f, 0.f};
  reconstruct<MU, SIGMA>(chi, t);
  const float sc = r.scale;
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = {fmaf(sc, t[c].re, acc[c].re), fmaf(sc, t[c].im, acc[c].im)};
}

// Pipeline step K handles direction dir_at(K) = K (+x, -x, +y, ...): the +x and
// -x neighbours of a wave's consecutive sites share most of their cache lines,
// which then meet in L1.
__host__ __device__ constexpr int dir_at(int k) { return k; }

// Number of load slots of the neighbour pipeline: FP16 + scale keeps one spare
// slot, so the neighbour DEPTH steps ahead is loaded into a free slot before
// the packed one in use is computed (no register copy); the wider precisions
// compute a slot in place and then refill it.
template <int PREC, int DEPTH>
struct Slots {
  static constexpr int n = PREC == DWF_F16S ? DEPTH + 1 : DEPTH;
};

// compute the direction of step K from its slot; the neighbour of step
// K + DEPTH goes into slot (K + DEPTH) % NS
template <int PREC, bool DAG, int K, int DEPTH, int NS>
__device__ __forceinline__ void hop_pipeline(const char* in, long long V4h, int Ls, int s, const int nh[8],
                                             const cplx<typename Store<PREC>::real>* __restrict__ ll, int spb,
                                             int sl, typename Store<PREC>::Raw (&buf)[NS],
                                             cplx<typename Store<PREC>::real> acc[12], float one) {
  if constexpr (K < 8) {
    constexpr int DN = dir_at(K + DEPTH);
    if constexpr (PREC == DWF_F16S) {
      if constexpr (K + DEPTH < 8) Store<PREC>::load_raw(in, V4h, Ls, nh[DN], s, buf[(K + DEPTH) % NS]);
      hop_compute_f16<DAG, dir_at(K)>(buf[K % NS], one, ll, spb, sl, acc);
    } else {
      cplx<typename Store<PREC>::real> psi[12];
      Store<PREC>::unpack(buf[K % NS], psi);
      hop_compute<typename Store<PREC>::real, DAG, dir_at(K)>(psi, ll, spb, sl, acc);
      if constexpr (K + DEPTH < 8) Store<PREC>::load_raw(in, V4h, Ls, nh[DN], s, buf[(K + DEPTH) % NS]);
    }
    hop_pipeline<PREC, DAG, K + 1, DEPTH, NS>(in, V4h, Ls, s, nh, ll, spb, sl, buf, acc, one);
  }
}

template <int PREC, int J, int DEPTH, int NS>
__device__ __forceinline__ void hop_prologue(const char* in, long long V4h, int Ls, int s, const int nh[8],
                                             typename Store<PREC>::Raw (&buf)[NS]) {
  if constexpr (J < DEPTH) {
    Store<PREC>::load_raw(in, V4h, Ls, nh[dir_at(J)], s, buf[J]);
    hop_prologue<PREC, J + 1, DEPTH, NS>(in, V4h, Ls, s, nh, buf);
  }
}

// (M5D x)_s or (M5D^dag x)_s for one lane.  Per chirality only one neighbour
// slice enters: P_+ couples to s-1 (s+1 for the adjoint), P_- to s+1 (s-1),
// with the wrapped coupling +m instead of -1.  `up` holds the six upper-spin
// components of the P_+ neighbour, `lo` the six lower-spin components of the
// P_- neighbour.
template <class R>
__device__ __forceinline__ void m5d_combine(const cplx<R> xs[12], const cplx<R> up[6], const cplx<R> lo[6], R cu,
                                            R cl, R d, cplx<R> out[12]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    out[c] = {d * xs[c].re + cu * up[c].re, d * xs[c].im + cu * up[c].im};
    out[6 + c] = {d * xs[6 + c].re + cl * lo[c].re, d * xs[6 + c].im + cl * lo[c].im};
  }
}

// load the six components c0..c0+5 of the spinor at (h, s)
template <int PREC>
__device__ __forceinline__ void load_half(const char* base, long long V4h, int Ls, long long h, int s, int c0,
                                          cplx<typename Store<PREC>::real> v[6]) {
  using R = typename Store<PREC>::real;
  if constexpr (PREC == DWF_F64) {
    const double2* p = reinterpret_cast<const double2*>(base) + (h * 12 + c0) * Ls + s;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      double2 t = p[(size_t)c * Ls];
      v[c] = {t.x, t.y};
    }
  } else if constexpr (PREC == DWF_F32) {
    const float4* p = reinterpret_cast<const float4*>(base) + (h * 6 + c0 / 2) * Ls + s;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      float4 t = p[(size_t)j * Ls];
      v[2 * j] = {t.x, t.y};
      v[2 * j + 1] = {t.z, t.w};
    }
  } else {
    cplx<R> full[12];
    Store<PREC>::load(base, V4h, Ls, h, s, full);
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = full[c0 + c];
  }
}

// In-LDS inverse of M5D (or M5D^dag) on the columns of a workgroup.  buf is
// [spb][12][LP] with LP = Ls + 1.  Per chirality the matrix is d - S with S a
// cyclic shift whose wrap carries -m (lower shift for P_+, upper for P_-;
// transposed for the adjoint).  With y_{-1} := -m y_{Ls-1} the solve is the
// recursion y_j = (v_j + y_{j-1}) / d along the shift direction; the start
// value follows from Z = sum_j d^{-(Ls-j)} v_j as y_{-1} = corner * Z with
// corner = -m / (1 + m d^{-Ls}).
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
    R w = inv_d;  // d^{-(Ls - j)} for j = Ls-1, Ls-2, ...
    for (int j = Ls - 1; j >= 0; --j) {
      const int sj = fwd ? j : Ls - 1 - j;
      z = {fma(w, col[sj].re, z.re), fma(w, col[sj].im, z.im)};
      w *= inv_d;
    }
    cplx<R> y = {corner * z.re, corner * z.im};
    for (int j = 0; j < Ls; ++j) {
      const int sj = fwd ? j : Ls - 1 - j;
      y = {(col[sj].re + y.re) * inv_d, (col[sj].im + y.im) * inv_d};
      col[sj] = y;
    }
  }
}

// MULTI: the workgroup loops over rpb right-hand sides (links staged once);
// without it the body runs once, which keeps the loop-carried addresses out of
// the register budget of the common single-rhs launches.
// Minimum waves per SIMD the compiler must leave room for.  The single-rhs
// FP32 and FP16S kernels gain from holding three (fewer registers, more
// waves); the FP64 kernels keep the scheduler's own choice, which holds more
// loads in flight per wave and measured faster than any cap, and so do the
// multi-rhs kernels, which would spill under it.
template <int PREC, bool MULTI>
struct HopOccupancy {
  static constexpr int waves = (PREC == DWF_F64 || MULTI) ? 1 : 3;
};

// PREC is the storage of the output (and of y, z, w), PIN that of the
// neighbour input and PX that of the site-local operand x; all three share the
// arithmetic type.  The mixed forms (FP16 + scale in, FP32 out, or FP16 + scale
// x) let the low-precision CG keep its search direction in FP16 + scale while
// the operator's intermediate fields stay FP32.
template <int PREC, int PIN, int PX, bool DAG, int EPI, int DEPTH, bool MULTI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(HopOccupancy<PREC, MULTI>::waves)))
hop_kernel(HopArgs a) {
  using R = typename Store<PREC>::real;
  static_assert(sizeof(typename Store<PIN>::real) == sizeof(R) && sizeof(typename Store<PX>::real) == sizeof(R),
                "one arithmetic type per launch");
  using V = typename LinkT<R>::vec;
  extern __shared__ char smem_raw[];
  const int Ls = a.Ls;
  const int spb = a.spb;
  cplx<R>* ll = reinterpret_cast<cplx<R>*>(smem_raw);  // links [72][spb], kept for all rhs of the workgroup
  char* scratch = smem_raw + (size_t)spb * 72 * sizeof(cplx<R>);  // M5D^{-1} columns, x, reduction
  const int b = blockIdx.x;
  const int logical = (b & 7) * a.nb8 + (b >> 3);
  if (logical >= a.nblocks) return;  // whole workgroup leaves together
  const int tid = threadIdx.x;
  const int sl = tid / Ls;
  const int s = tid - sl * Ls;
  const long long V4h = a.V4h;
  const long long h0 = (long long)logical * spb;  // first processing index of the workgroup
  const bool valid = (sl < spb) && (h0 + sl < V4h);
  // index loads are unconditional (clamped to site 0 on idle lanes), so the
  // eight neighbour indices are fetched in one round trip instead of eight
  const long long hq = valid ? h0 + sl : 0;
  const long long h = a.order ? (long long)a.order[hq] : hq;

  int nh[8];
#pragma unroll
  for (int d = 0; d < 8; ++d) nh[d] = a.nbr[(size_t)d * V4h + h];
  // The workgroup's site indices go through LDS, so that the link loads below
  // carry no dependent lookup of the traversal order.
  __shared__ int site_h[256];
  if (s == 0 && sl < spb) site_h[sl] = valid ? (int)h : -1;
  __syncthreads();
  // Stage this workgroup's links once; every rhs the workgroup handles reuses
  // them.  A thread issues all its link loads (up to eight) before its first
  // LDS store, so the staging costs one memory round trip.
  {
    // element (dk, site) of the [72][spb] copy is staged by thread dk % Ls * spb + site
    // (blockDim = spb * Ls), so a thread's site and its first dk come from one division
    constexpr int U = 8;
    const V* lg = reinterpret_cast<const V*>(a.links);
    const int q0 = tid / spb;
    const int r0 = tid - q0 * spb;
    const int h2 = site_h[r0];
    for (int dk0 = 0; dk0 < 72; dk0 += U * Ls) {
      V t[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int dk = dk0 + u * Ls + q0;
        t[u] = V{0, 0};
        if (dk < 72 && h2 >= 0) {
          if constexpr (PREC == DWF_F64) {  // each site's links are read by its own workgroup only
            typedef double dv2 __attribute__((ext_vector_type(2)));
            const dv2 q = __builtin_nontemporal_load(reinterpret_cast<const dv2*>(lg + (size_t)dk * V4h + h2));
            t[u] = V{q.x, q.y};
          } else {  // 8-byte links: plain loads (non-temporal ones were slower)
            t[u] = lg[(size_t)dk * V4h + h2];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int dk = dk0 + u * Ls + q0;
        if (dk < 72) ll[dk * spb + r0] = {t[u].x, t[u].y};
      }
    }
  }
  const R alpha = (R)a.alpha;
  const int nrr = MULTI ? a.rpb : 1;
  for (int rr = 0; rr < nrr; ++rr) {
    const int rhs = blockIdx.y * nrr + rr;
    if (rhs >= a.nrhs) break;  // uniform across the workgroup
    const size_t off = (size_t)rhs * a.stride;
    const char* in = a.in + (size_t)rhs * a.in_stride;
    const char* xb = a.x ? a.x + (size_t)rhs * a.x_stride : nullptr;
    constexpr int NS = Slots<PIN, DEPTH>::n;
    typename Store<PIN>::Raw buf[NS];
    if (valid) hop_prologue<PIN, 0, DEPTH, NS>(in, V4h, Ls, s, nh, buf);
    __syncthreads();  // links staged (first rhs); scratch free (later rhs)
    cplx<R> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = {0, 0};
    if (valid) hop_pipeline<PIN, DAG, 0, DEPTH, NS>(in, V4h, Ls, s, nh, ll, spb, sl, buf, acc, a.one);

    char* out = a.out + off;
    cplx<R> v[12];
    if (EPI == EPI_LIN || EPI == EPI_M5INV) {
#pragma unroll
      for (int c = 0; c < 12; ++c) v[c] = cscale(alpha, acc[c]);
      const bool x_after = EPI == EPI_M5INV && a.x_after;
      if (xb != nullptr && valid && !x_after) {
        cplx<R> xv[12];
        Store<PX>::load(xb, V4h, Ls, h, s, xv);
        const R beta = (R)a.beta;
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = {v[c].re + beta * xv[c].re, v[c].im + beta * xv[c].im};
      }
      if (EPI == EPI_M5INV) {
        cplx<R>* col = reinterpret_cast<cplx<R>*>(scratch);
        const int LP = Ls + 1;
        if (valid) {
#pragma unroll
          for (int c = 0; c < 12; ++c) col[(size_t)(sl * 12 + c) * LP + s] = v[c];
        }
        __syncthreads();
        m5inv_columns<R, DAG>(col, spb, Ls, h0, V4h, (R)a.inv_d, (R)a.corner);
        __syncthreads();
        if (valid) {
#pragma unroll
          for (int c = 0; c < 12; ++c) v[c] = col[(size_t)(sl * 12 + c) * LP + s];
          if (x_after && xb != nullptr) {  // second Schur form: x + M5D^{-1}(alpha Dhop in)
            cplx<R> xv[12];
            Store<PX>::load(xb, V4h, Ls, h, s, xv);
            const R beta = (R)a.beta;
#pragma unroll
            for (int c = 0; c < 12; ++c) v[c] = {v[c].re + beta * xv[c].re, v[c].im + beta * xv[c].im};
          }
        }
      }
    } else {  // EPI_M5, EPI_CHEB, EPI_CGR
      // x(s) goes through LDS, [12][lanes], so that the s+-1 halves of M5D come
      // from the neighbouring lanes of the same site instead of a second pass
      // over cache lines whose fill may still be in flight
      cplx<R>* xl = reinterpret_cast<cplx<R>*>(scratch);
      const int nl = spb * Ls;
      cplx<R> xs[12];
      if (valid) {
        Store<PX>::load_nt(xb, V4h, Ls, h, s, xs);
#pragma unroll
        for (int c = 0; c < 12; ++c) xl[c * nl + tid] = xs[c];
      }
      __syncthreads();
      if (valid) {
        const int s_lo = (s == 0) ? Ls - 1 : s - 1;
        const int s_hi = (s == Ls - 1) ? 0 : s + 1;
        const R m_lo = (s == 0) ? (R)a.mf : (R)-1;       // coupling to slice s-1
        const R m_hi = (s == Ls - 1) ? (R)a.mf : (R)-1;  // coupling to slice s+1
        // M5D: P_+ from s-1, P_- from s+1; M5D^dag: P_+ from s+1, P_- from s-1
        const int t_up = sl * Ls + (DAG ? s_hi : s_lo);
        const int t_lo = sl * Ls + (DAG ? s_lo : s_hi);
        cplx<R> up[6], lo[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          up[c] = xl[c * nl + t_up];
          lo[c] = xl[(6 + c) * nl + t_lo];
        }
        m5d_combine<R>(xs, up, lo, DAG ? m_hi : m_lo, DAG ? m_lo : m_hi, (R)a.d, v);
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = {v[c].re + alpha * acc[c].re, v[c].im + alpha * acc[c].im};
        if (EPI == EPI_CHEB) {
          cplx<R> yv[12], zv[12];
          Store<PREC>::load_nt(a.y + off, V4h, Ls, h, s, yv);
          Store<PREC>::load_nt(a.z + off, V4h, Ls, h, s, zv);
          const R ca = (R)a.ca, cb = (R)a.cb, cc = (R)a.cc;
#pragma unroll
          for (int c = 0; c < 12; ++c) {
            v[c].re = ca * v[c].re + cb * yv[c].re + cc * zv[c].re;
            v[c].im = ca * v[c].im + cb * yv[c].im + cc * zv[c].im;
          }
          if (a.w != nullptr) {
            Store<PREC>::load_nt(a.w + off, V4h, Ls, h, s, yv);
            const R cw = (R)a.cw;
#pragma unroll
            for (int c = 0; c < 12; ++c) v[c] = {v[c].re + cw * yv[c].re, v[c].im + cw * yv[c].im};
          }
        }
      }
    }
    if constexpr (EPI == EPI_CGR) {
      // CG residual update with the operator output never written: r -= alpha q,
      // r unchanged for a right-hand side that has stopped (alpha = 0); the
      // partials below are then |r|^2
      const double al = a.scal[(size_t)rhs * NSCAL + S_ALPHA];
      if (valid) {
        cplx<R> rv[12];
        Store<PREC>::load_nt(out, V4h, Ls, h, s, rv);
        if (al != 0.0) {
#pragma unroll
          for (int c = 0; c < 12; ++c) rv[c] = {fma((R)-al, v[c].re, rv[c].re), fma((R)-al, v[c].im, rv[c].im)};
          Store<PREC>::store(out, V4h, Ls, h, s, rv);
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = rv[c];
      }
    } else {
      if (valid) {
        // non-temporal stores: M_pc^dag M_pc -4 % in FP64, -6 % in FP32; +3 % in FP16S, which keeps plain ones
        if constexpr (PREC == DWF_F16S)
          Store<PREC>::store(out, V4h, Ls, h, s, v);
        else
          Store<PREC>::store_nt(out, V4h, Ls, h, s, v);
      }
    }
    if (a.partial != nullptr) {
      // |out|^2 per site (FP64): p.Ap = |M_pc p|^2, or CG's |r|^2.  The s-slices of a
      // site are added in a fixed order (an in-wave butterfly for Ls a power of two, in
      // order through LDS otherwise) and the sum is stored at the site's own index, so
      // the totals do not depend on the launch shape or the traversal order.
      if (EPI != EPI_LIN) __syncthreads();  // scratch still holds x or the M5D^{-1} columns
      double n2 = 0;
      if (valid) {
#pragma unroll
        for (int c = 0; c < 12; ++c) n2 += (double)v[c].re * v[c].re + (double)v[c].im * v[c].im;
      }
      if ((Ls & (Ls - 1)) == 0 && Ls <= 64) {
        // a site's lanes are one aligned group of Ls lanes inside a wave
        const double tot = group_sum(n2, Ls);
        if (valid && s == 0) a.partial[(size_t)rhs * V4h + h] = tot;
      } else {
        double* red = reinterpret_cast<double*>(scratch);
        red[tid] = n2;
        __syncthreads();
        if (valid && s == 0) {
          double tot = 0;
          for (int k = 0; k < Ls; ++k) tot += red[sl * Ls + k];
          a.partial[(size_t)rhs * V4h + h] = tot;
        }
        __syncthreads();  // the next rhs of the workgroup reuses scratch
      }
    }
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
    const R m_lo = (s == 0) ? (R)a.mf : (R)-1;
    const R m_hi = (s == Ls - 1) ? (R)a.mf : (R)-1;
    cplx<R> xs[12], up[6], lo[6], v[12];
    Store<PREC>::load(in, a.V4h, Ls, h, s, xs);
    load_half<PREC>(in, a.V4h, Ls, h, DAG ? s_hi : s_lo, 0, up);
    load_half<PREC>(in, a.V4h, Ls, h, DAG ? s_lo : s_hi, 6, lo);
    m5d_combine<R>(xs, up, lo, DAG ? m_hi : m_lo, DAG ? m_lo : m_hi, (R)a.d, v);
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
static size_t cplx_bytes(int prec) { return prec == DWF_F64 ? 16 : 8; }

// LDS bytes of a hop launch: the link copy (kept for all rhs of a workgroup)
// followed by a scratch region for the M5D^{-1} columns, the x copy of the
// M5D epilogue, or the reduction
static size_t hop_lds(int prec, int spb, int Ls, int epi, bool reduce) {
  size_t scratch = 0;
  if (epi == EPI_M5INV) scratch = (size_t)spb * 12 * (Ls + 1) * cplx_bytes(prec);
  if (epi == EPI_M5 || epi == EPI_CHEB || epi == EPI_CGR) scratch = (size_t)spb * 12 * Ls * cplx_bytes(prec);
  if (reduce) scratch = std::max(scratch, (size_t)256 * sizeof(double));
  return (size_t)spb * 72 * cplx_bytes(prec) + scratch;
}

void fill_shape(const dwf_context* ctx, HopArgs& a) {
  const int Ls = ctx->g.Ls;
  int spb = ctx->spb;
  if (spb <= 0) {
    spb = 256 / Ls;
    if (spb > 64) spb = 64;
  }
  if (spb * Ls > 256) spb = 256 / Ls;
  if (spb < 1) spb = 1;
  // every staging buffer must fit 64 KiB of LDS
  while (spb > 1 && hop_lds(DWF_F64, spb, Ls, EPI_M5INV, true) > 65536) --spb;
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

template <int PREC, int PIN, int PX, bool DAG, int EPI, int DEPTH>
static hipError_t launch_hop_t(const HopArgs& a, int nrhs, hipStream_t st) {
  dim3 grid(a.nb8 * 8, (nrhs + a.rpb - 1) / a.rpb);
  dim3 block(a.spb * a.Ls);
  const size_t lds = std::max(hop_lds(PREC, a.spb, a.Ls, EPI, a.partial != nullptr), (size_t)a.lds_floor);
  if (a.rpb > 1)
    hipLaunchKernelGGL((hop_kernel<PREC, PIN, PX, DAG, EPI, DEPTH, true>), grid, block, lds, st, a);
  else
    hipLaunchKernelGGL((hop_kernel<PREC, PIN, PX, DAG, EPI, DEPTH, false>), grid, block, lds, st, a);
  return hipGetLastError();
}

template <int PREC, int PIN, int PX, bool DAG, int EPI>
static hipError_t launch_hop_d(const HopArgs& a, int depth, int nrhs, hipStream_t st) {
  switch (depth) {
    case 1: return launch_hop_t<PREC, PIN, PX, DAG, EPI, 1>(a, nrhs, st);
    case 3: return launch_hop_t<PREC, PIN, PX, DAG, EPI, 3>(a, nrhs, st);
    default: return launch_hop_t<PREC, PIN, PX, DAG, EPI, 2>(a, nrhs, st);
  }
}

template <int PREC>
static hipError_t launch_hop_p(const HopArgs& a, int dag, int epi, int depth, int nrhs, hipStream_t st) {
  switch (epi * 2 + (dag ? 1 : 0)) {
    case EPI_LIN * 2 + 0: return launch_hop_d<PREC, PREC, PREC, false, EPI_LIN>(a, depth, nrhs, st);
    case EPI_LIN * 2 + 1: return launch_hop_d<PREC, PREC, PREC, true, EPI_LIN>(a, depth, nrhs, st);
    case EPI_M5INV * 2 + 0: return launch_hop_d<PREC, PREC, PREC, false, EPI_M5INV>(a, depth, nrhs, st);
    case EPI_M5INV * 2 + 1: return launch_hop_d<PREC, PREC, PREC, true, EPI_M5INV>(a, depth, nrhs, st);
    case EPI_M5 * 2 + 0: return launch_hop_d<PREC, PREC, PREC, false, EPI_M5>(a, depth, nrhs, st);
    case EPI_M5 * 2 + 1: return launch_hop_d<PREC, PREC, PREC, true, EPI_M5>(a, depth, nrhs, st);
    case EPI_CHEB * 2 + 0: return launch_hop_d<PREC, PREC, PREC, false, EPI_CHEB>(a, depth, nrhs, st);
    case EPI_CHEB * 2 + 1: return launch_hop_d<PREC, PREC, PREC, true, EPI_CHEB>(a, depth, nrhs, st);
    case EPI_CGR * 2 + 1:
      if constexpr (PREC != DWF_F16S) return launch_hop_d<PREC, PREC, PREC, true, EPI_CGR>(a, depth, nrhs, st);
      break;
  }
  return hipErrorInvalidValue;
}

// The two mixed-storage forms: FP16 + scale neighbour input with FP32 output
// (t = M5D^{-1} D_hop p, no x), and FP32 neighbour input with an FP16 + scale
// site-local operand (u = M5D p - D_hop t / 4).
static hipError_t launch_hop_mixed(const HopArgs& a, int pin, int px, int dag, int epi, int depth, int nrhs,
                                   hipStream_t st) {
  if (pin == DWF_F16S && epi == EPI_M5INV && a.x == nullptr)
    return dag ? launch_hop_d<DWF_F32, DWF_F16S, DWF_F32, true, EPI_M5INV>(a, depth, nrhs, st)
               : launch_hop_d<DWF_F32, DWF_F16S, DWF_F32, false, EPI_M5INV>(a, depth, nrhs, st);
  if (pin == DWF_F32 && px == DWF_F16S && epi == EPI_M5)
    return dag ? launch_hop_d<DWF_F32, DWF_F32, DWF_F16S, true, EPI_M5>(a, depth, nrhs, st)
               : launch_hop_d<DWF_F32, DWF_F32, DWF_F16S, false, EPI_M5>(a, depth, nrhs, st);
  return hipErrorInvalidValue;
}

hipError_t launch_hop_ex(dwf_context* ctx, int prec, int pin, int px, HopArgs a, int out_parity, int dag, int epi,
                         int nrhs) {
  if (prec != DWF_F64 && ctx->links32 == nullptr) return hipErrorInvalidValue;  // FP64 handles hold no FP32 links
  fill_shape(ctx, a);
  const long long V4h = ctx->g.V4h;
  a.nbr = ctx->nbr + (size_t)out_parity * 8 * V4h;
  const size_t link_elems = (size_t)out_parity * 8 * 9 * V4h;
  if (prec == DWF_F64)
    a.links = reinterpret_cast<const double2*>(ctx->links64) + link_elems;
  else
    a.links = reinterpret_cast<const float2*>(ctx->links32) + link_elems;
  a.stride = field_bytes_rhs(ctx, prec);
  a.in_stride = field_bytes_rhs(ctx, pin);
  a.x_stride = field_bytes_rhs(ctx, px);
  a.order = ctx->order_mode ? ctx->order + (size_t)out_parity * V4h : nullptr;
  a.lds_floor = ctx->lds_floor;
  a.one = 1.0f;
  a.nrhs = nrhs;
  a.rpb = std::max(1, std::min(ctx->rpb, nrhs));
  const int depth = ctx->depth[pin];
  timing_begin(ctx);
  hipError_t e;
  if (pin != prec || px != prec) {
    e = (prec == DWF_F32) ? launch_hop_mixed(a, pin, px, dag, epi, depth, nrhs, ctx->stream) : hipErrorInvalidValue;
  } else {
    switch (prec) {
      case DWF_F64: e = launch_hop_p<DWF_F64>(a, dag, epi, depth, nrhs, ctx->stream); break;
      case DWF_F32: e = launch_hop_p<DWF_F32>(a, dag, epi, depth, nrhs, ctx->stream); break;
      default: e = launch_hop_p<DWF_F16S>(a, dag, epi, depth, nrhs, ctx->stream); break;
    }
  }
  timing_end(ctx);
  return e;
}

hipError_t launch_hop(dwf_context* ctx, int prec, HopArgs a, int out_parity, int dag, int epi, int nrhs) {
  return launch_hop_ex(ctx, prec, prec, prec, a, out_parity, dag, epi, nrhs);
}

template <int PREC, bool DAG, bool INV>
static hipError_t launch_site5_t(const HopArgs& a, int nrhs, hipStream_t st) {
  dim3 grid(a.nb8 * 8, nrhs);
  dim3 block(a.spb * a.Ls);
  size_t lds = INV ? (size_t)a.spb * 12 * (a.Ls + 1) * cplx_bytes(PREC) : 0;
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
