// Internal definitions shared by the libdwf translation units: the handle,
// field storage traits, complex arithmetic and the spin algebra of the
// hopping term in the chiral basis.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "dwf.h"

namespace dwf {

// ---------------------------------------------------------------------------
// Complex numbers (plain structs; HIP has no device std::complex).
// ---------------------------------------------------------------------------
template <class R>
struct cplx {
  R re, im;
};

template <class R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R>
__device__ __forceinline__ cplx<R> cscale(R s, cplx<R> a) { return {s * a.re, s * a.im}; }
// a * b
template <class R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// acc + a * b
template <class R>
__device__ __forceinline__ cplx<R> cfma(cplx<R> a, cplx<R> b, cplx<R> acc) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
  return acc;
}
// acc + conj(a) * b
template <class R>
__device__ __forceinline__ cplx<R> cfma_conj(cplx<R> a, cplx<R> b, cplx<R> acc) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
  return acc;
}
// i * a
template <class R>
__device__ __forceinline__ cplx<R> ctimesi(cplx<R> a) { return {-a.im, a.re}; }

// ---------------------------------------------------------------------------
// Deterministic workgroup sums built on wavefront shuffles.  A wave folds its
// 64 lanes in a fixed butterfly (the last wave of a workgroup may hold fewer
// lanes; only those that exist are added), then thread 0 adds the waves' sums
// in wave order.  The order depends only on blockDim, so results are bitwise
// reproducible.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int wave_lanes_present() {
  const int first = (int)(threadIdx.x & ~63u);
  const int n = (int)blockDim.x - first;
  return n < 64 ? n : 64;
}

// sum of v over the calling wave's lanes, valid in its lane 0
__device__ __forceinline__ double wave_sum(double v) {
  const int lane = (int)(threadIdx.x & 63u);
  const int present = wave_lanes_present();
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_down(v, off, 64);
    if (lane + off < present) v += o;
  }
  return v;
}

// sums of a and b over the workgroup, valid on thread 0; red holds 2 * (blockDim / 64) doubles
// (LDS).  Contains one barrier, which every thread of the workgroup must reach.
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = (int)(threadIdx.x >> 6);
  const int nw = (int)((blockDim.x + 63) >> 6);
  if ((threadIdx.x & 63u) == 0) {
    red[w] = a;
    red[nw + w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = red[0], tb = red[nw];
    for (int k = 1; k < nw; ++k) {
      ta += red[k];
      tb += red[nw + k];
    }
    a = ta;
    b = tb;
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

// ---------------------------------------------------------------------------
// Field storage.  A packed half field of one right-hand side holds the 12
// spin-colour components (c = 3 spin + colour) of every (site h, slice s),
// grouped so that one lane moves 16 bytes per load:
//   FP64 : [V4h][12][Ls]      complex128            (1 component per 16 B)
//   FP32 : [V4h][6][Ls][2]    complex64, c = 2j + k (2 components per 16 B)
//   FP16S: [V4h][3][Ls][8]    halves (4 components per 16 B), then [V4h][Ls] FP32 scales
// In each case s runs fastest across lanes, so a wave's load is contiguous.
// ---------------------------------------------------------------------------
template <int PREC>
struct Store;

template <>
struct Store<DWF_F64> {
  using real = double;
  static constexpr size_t bytes_per_spinor = 192;
  struct Raw {
    cplx<double> v[12];
  };
  __device__ static void load_raw(const char* base, size_t V4h, int Ls, size_t h, int s, Raw& r) {
    load(base, V4h, Ls, h, s, r.v);
  }
  __device__ static void unpack(const Raw& r, cplx<double> v[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = r.v[c];
  }
  __device__ static void load(const char* base, size_t V4h, int Ls, size_t h, int s, cplx<double> v[12]) {
    const double2* p = reinterpret_cast<const double2*>(base) + h * 12 * Ls + s;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      double2 t = p[(size_t)c * Ls];
      v[c] = {t.x, t.y};
    }
  }
  __device__ static void store(char* base, size_t V4h, int Ls, size_t h, int s, const cplx<double> v[12]) {
    double2* p = reinterpret_cast<double2*>(base) + h * 12 * Ls + s;
#pragma unroll
    for (int c = 0; c < 12; ++c) p[(size_t)c * Ls] = make_double2(v[c].re, v[c].im);
  }
  // non-temporal load of a field that the reading kernel uses once
  __device__ static void load_nt(const char* base, size_t V4h, int Ls, size_t h, int s, cplx<double> v[12]) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    const d2v* p = reinterpret_cast<const d2v*>(base) + h * 12 * Ls + s;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const d2v t = __builtin_nontemporal_load(p + (size_t)c * Ls);
      v[c] = {t.x, t.y};
    }
  }
  // The same with non-temporal stores, for an output that the kernel writing it
  // does not read back: it then displaces less of the neighbour data in L2.
  __device__ static void store_nt(char* base, size_t V4h, int Ls, size_t h, int s, const cplx<double> v[12]) {
    typedef double d2v __attribute__((ext_vector_type(2)));
    d2v* p = reinterpret_cast<d2v*>(base) + h * 12 * Ls + s;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      d2v t;
      t.x = v[c].re;
      t.y = v[c].im;
      __builtin_nontemporal_store(t, p + (size_t)c * Ls);
    }
  }
};

template <>
struct Store<DWF_F32> {
  using real = float;
  static constexpr size_t bytes_per_spinor = 96;
  struct Raw {
    cplx<float> v[12];
  };
  __device__ static void load_raw(const char* base, size_t V4h, int Ls, size_t h, int s, Raw& r) {
    load(base, V4h, Ls, h, s, r.v);
  }
  __device__ static void unpack(const Raw& r, cplx<float> v[12]) {
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = r.v[c];
  }
  __device__ static void load(const char* base, size_t V4h, int Ls, size_t h, int s, cplx<float> v[12]) {
    const float4* p = reinterpret_cast<const float4*>(base) + h * 6 * Ls + s;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      float4 t = p[(size_t)j * Ls];
      v[2 * j] = {t.x, t.y};
      v[2 * j + 1] = {t.z, t.w};
    }
  }
  __device__ static void store(char* base, size_t V4h, int Ls, size_t h, int s, const cplx<float> v[12]) {
    float4* p = reinterpret_cast<float4*>(base) + h * 6 * Ls + s;
#pragma unroll
    for (int j = 0; j < 6; ++j) p[(size_t)j * Ls] = make_float4(v[2 * j].re, v[2 * j].im, v[2 * j + 1].re, v[2 * j + 1].im);
  }  __device__ static void load_nt(const char* base, size_t V4h, int Ls, size_t h, int s, cplx<float> v[12]) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    const f4v* p = reinterpret_cast<const f4v*>(base) + h * 6 * Ls + s;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const f4v t = __builtin_nontemporal_load(p + (size_t)j * Ls);
      v[2 * j] = {t.x, t.y};
      v[2 * j + 1] = {t.z, t.w};
    }
  }
  // non-temporal, as for FP64
  __device__ static void store_nt(char* base, size_t V4h, int Ls, size_t h, int s, const cplx<float> v[12]) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    f4v* p = reinterpret_cast<f4v*>(base) + h * 6 * Ls + s;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      f4v t;
      t.x = v[2 * j].re;
      t.y = v[2 * j].im;
      t.z = v[2 * j + 1].re;
      t.w = v[2 * j + 1].im;
      __builtin_nontemporal_store(t, p + (size_t)j * Ls);
    }
  }
};

// FP16 values v * (1 / scale) (round to nearest even) plus one FP32 scale =
// max |v| per (site, s).  Data [V4h][3][Ls] groups of 8 halves (16 bytes per
// lane and load: components 4j .. 4j+3 as re, im pairs), then the scale array
// [V4h][Ls] of the same rhs.
typedef _Float16 half8v __attribute__((ext_vector_type(8)));

template <>
struct Store<DWF_F16S> {
  using real = float;
  static constexpr size_t bytes_per_spinor = 52;
  // the stored form of one spinor, as loaded: 3 x 16 bytes and the scale
  struct Raw {
    half8v q[3];
    float scale;
  };
  __device__ static void load_raw(const char* base, size_t V4h, int Ls, size_t h, int s, Raw& r) {
    const half8v* p = reinterpret_cast<const half8v*>(base) + h * 3 * Ls + s;
#pragma unroll
    for (int j = 0; j < 3; ++j) r.q[j] = p[(size_t)j * Ls];
    r.scale = reinterpret_cast<const float*>(base + V4h * Ls * 48)[h * Ls + s];
  }
  __device__ static void unpack(const Raw& r, cplx<float> v[12]) {
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 4; ++k) v[4 * j + k] = {(float)r.q[j][2 * k] * r.scale, (float)r.q[j][2 * k + 1] * r.scale};
  }
  __device__ static void load(const char* base, size_t V4h, int Ls, size_t h, int s, cplx<float> v[12]) {
    Raw r;
    load_raw(base, V4h, Ls, h, s, r);
    unpack(r, v);
  }
  __device__ static void load_nt(const char* base, size_t V4h, int Ls, size_t h, int s, cplx<float> v[12]) {
    load(base, V4h, Ls, h, s, v);  // plain loads: the scale array makes it two streams per spinor
  }
  __device__ static void store(char* base, size_t V4h, int Ls, size_t h, int s, const cplx<float> v[12]) {
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
    half8v* p = reinterpret_cast<half8v*>(base) + h * 3 * Ls + s;
    reinterpret_cast<float*>(base + V4h * Ls * 48)[h * Ls + s] = m;
    const float r = 1.f / ((m > 0.f) ? m : 1.f);  // one correctly rounded division per spinor
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      half8v t;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        t[2 * k] = (_Float16)(v[4 * j + k].re * r);
        t[2 * k + 1] = (_Float16)(v[4 * j + k].im * r);
      }
      p[(size_t)j * Ls] = t;
    }
  }
};

__host__ __device__ inline size_t spinor_bytes(int prec) {
  return prec == DWF_F64 ? 192 : prec == DWF_F32 ? 96 : 52;
}

// ---------------------------------------------------------------------------
// Spin algebra of the hopping term.  In the chiral basis each gamma_mu is
// [[0, B_mu], [B_mu^dag, 0]] with 2x2 blocks, so for sigma = +-1
//   (1 + sigma g_mu) psi = (h, sigma B_mu^dag h),  h = u + sigma B_mu l,
// with u = spins (0,1) and l = spins (2,3).  B_x = [[0,i],[i,0]],
// B_y = [[0,-1],[1,0]], B_z = diag(i,-i), B_t = 1.
// ---------------------------------------------------------------------------
template <int MU, int SIGMA, class R>
__device__ __forceinline__ void project(const cplx<R> p[12], cplx<R> h[6]) {
  const R sg = (R)SIGMA;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<R> u0 = p[a], u1 = p[3 + a], l0 = p[6 + a], l1 = p[9 + a];
    if (MU == 0) {  // B l = (i l1, i l0)
      h[a] = cadd(u0, cscale(sg, ctimesi(l1)));
      h[3 + a] = cadd(u1, cscale(sg, ctimesi(l0)));
    } else if (MU == 1) {  // B l = (-l1, l0)
      h[a] = csub(u0, cscale(sg, l1));
      h[3 + a] = cadd(u1, cscale(sg, l0));
    } else if (MU == 2) {  // B l = (i l0, -i l1)
      h[a] = cadd(u0, cscale(sg, ctimesi(l0)));
      h[3 + a] = csub(u1, cscale(sg, ctimesi(l1)));
    } else {  // B l = l
      h[a] = cadd(u0, cscale(sg, l0));
      h[3 + a] = cadd(u1, cscale(sg, l1));
    }
  }
}

// acc += (chi, sigma B^dag chi) for the colour-rotated half spinor chi.
template <int MU, int SIGMA, class R>
__device__ __forceinline__ void reconstruct(const cplx<R> chi[6], cplx<R> acc[12]) {
  const R sg = (R)SIGMA;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx<R> c0 = chi[a], c1 = chi[3 + a];
    acc[a] = cadd(acc[a], c0);
    acc[3 + a] = cadd(acc[3 + a], c1);
    if (MU == 0) {  // B^dag chi = (-i c1, -i c0)
      acc[6 + a] = csub(acc[6 + a], cscale(sg, ctimesi(c1)));
      acc[9 + a] = csub(acc[9 + a], cscale(sg, ctimesi(c0)));
    } else if (MU == 1) {  // B^dag chi = (c1, -c0)
      acc[6 + a] = cadd(acc[6 + a], cscale(sg, c1));
      acc[9 + a] = csub(acc[9 + a], cscale(sg, c0));
    } else if (MU == 2) {  // B^dag chi = (-i c0, i c1)
      acc[6 + a] = csub(acc[6 + a], cscale(sg, ctimesi(c0)));
      acc[9 + a] = cadd(acc[9 + a], cscale(sg, ctimesi(c1)));
    } else {  // B^dag chi = chi
      acc[6 + a] = cadd(acc[6 + a], cscale(sg, c0));
      acc[9 + a] = cadd(acc[9 + a], cscale(sg, c1));
    }
  }
}

// ---------------------------------------------------------------------------
// Lattice geometry shared by host and device.
// ---------------------------------------------------------------------------
struct Geom {
  int X, Y, Z, T;
  int Ls;
  long long V4, V4h;
};

// Coordinates of half-lattice site h of parity p.
__host__ __device__ inline void site_coords(const Geom& g, int p, long long h, int& x, int& y, int& z,
                                            int& t) {
  int Xh = g.X / 2;
  long long xh = h % Xh;
  long long rest = h / Xh;
  y = (int)(rest % g.Y);
  rest /= g.Y;
  z = (int)(rest % g.Z);
  t = (int)(rest / g.Z);
  x = 2 * (int)xh + ((p + y + z + t) & 1);
}

__host__ __device__ inline long long half_index(const Geom& g, int x, int y, int z, int t) {
  return ((long long)x + (long long)g.X * (y + (long long)g.Y * (z + (long long)g.Z * t))) / 2;
}

// ---------------------------------------------------------------------------
// Kernel parameter blocks.
// ---------------------------------------------------------------------------
enum Epilogue {
  EPI_LIN = 0,    // out = alpha * Dhop(in) + beta * x             (x optional)
  EPI_M5INV = 1,  // out = M5D^{-1} [alpha * Dhop(in) + beta * x]  (x optional)
  EPI_M5 = 2,     // out = M5D x + alpha * Dhop(in)
  EPI_CHEB = 3,   // out = ca * (M5D x + alpha * Dhop(in)) + cb * y + cc * z (+ cw * w)
  EPI_CGR = 4,    // q = M5D x + alpha * Dhop(in) kept in registers; out -= alpha_cg * q  (CG residual, FP64/FP32)
};

struct HopArgs {
  const char* in;     // other parity, rhs stride in_stride
  char* out;          // out parity
  const char* x;      // out parity (EPI_LIN/M5INV optional, EPI_M5/EPI_CHEB required)
  const char* y;      // EPI_CHEB
  const char* z;      // EPI_CHEB (may alias out)
  const char* w;      // EPI_CHEB optional fourth term (may alias out)
  const void* links;  // packed links of out parity: [dir][9][V4h] complex
  const int* nbr;     // neighbour table of out parity: [dir][V4h]
  size_t stride;      // bytes per rhs of out, y, z and w
  size_t in_stride;   // bytes per rhs of in
  size_t x_stride;    // bytes per rhs of x
  long long V4h;
  int Ls;
  int spb;            // sites per workgroup
  int nblocks;        // workgroups along the site axis (before XCD padding)
  int nb8;            // workgroups per XCD slot
  double alpha, beta, ca, cb, cc, cw;
  double d, inv_d, corner;  // 5 - M5, 1/d, -mf / (1 + mf d^{-Ls})
  double mf;
  double* partial;    // optional per-site FP64 |out|^2 sums, [rhs][V4h] (reductions)
  const int* order;   // optional traversal order of the out parity: processing index -> site h
  int lds_floor;      // minimum dynamic LDS of the launch (occupancy cap), bytes
  int nrhs;           // right-hand sides of the launch
  int rpb;            // right-hand sides per workgroup (looped, sharing the LDS links)
  const double* scal; // EPI_CGR: per-rhs solver scalars, alpha_cg = scal[rhs * NSCAL + S_ALPHA]
  int x_after;        // EPI_M5INV: add beta * x after the inverse instead of before
  float one;          // 1.0, passed at run time (keeps the FP16 projection FMAs as mixed-precision FMAs)
};

// ---------------------------------------------------------------------------
// The handle.
// ---------------------------------------------------------------------------
struct EventPair {
  hipEvent_t a, b;
};

}  // namespace dwf

struct dwf_context {
  dwf::Geom g;
  double M5, mf;
  int prec;
  int max_nrhs;
  int max_cg_rhs;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  // carved workspace
  void* links64;     // [2][8][9][V4h] complex128
  void* links32;     // [2][8][9][V4h] complex64 (prec != F64)
  int* nbr;          // [2][8][V4h]
  char* t_buf;       // odd half field, max_nrhs, handle precision
  char* u_buf;       // even half field, max_nrhs, handle precision
  char* t64;         // FP64 odd temporary (aliases t_buf for F64 handles)
  char* u64;         // FP64 even temporary (aliases u_buf for F64 handles)
  char* r64;         // FP64 CG vectors, max_nrhs
  char* p64;
  char* q64;
  char* b64;         // FP64 even field for the red-black source
  char* dir64;       // two more FP64 search directions per CG rhs (F64 handles)
  char* lo_r;        // low-precision CG vectors (F32/F16S handles)
  char* lo_p;
  char* lo_q;
  char* lo_x;        // FP32 accumulator of the low-precision solution
  char* cheb_a;      // Chebyshev partner set, handle precision, max(max_nrhs, 2)
  double* partials;  // reduction partials
  double* scalars;   // device scalars (per rhs)
  unsigned* counters;  // per-rhs completion counts of the per-site reductions (zero between launches)
  double* coef;      // Gram-Schmidt projection coefficients
  size_t partial_count;
  // launch shape of the hop kernels (sites per workgroup; load-pipeline depth per precision)
  int spb;
  int depth[3];
  int rpb;
  double* hop_partials;  // per-site |M_pc p|^2 (or |r|^2) sums of CG, [max_cg_rhs][V4h]
  int* order;            // site traversal order per out parity, [2][V4h] (device)
  int order_mode;        // 0: lexicographic (no table); 1: XCD octants; 2: XCD t-slabs; 3: boxes of order_box
  int order_box[3];      // the (x, y, z) cut of order 3
  int order_explicit;    // the caller chose the order (the autotuner then keeps it)
  int lds_floor;         // minimum LDS bytes requested by a hop launch (caps workgroups per CU)
  int schur_form;  // 1: M_ee - M_eo M_oo^{-1} M_oe; 2: 1 - M_ee^{-1} M_eo M_oo^{-1} M_oe
  double lam_max;  // lambda_max of M_pc^dag M_pc last measured by dwf_power (0: none since the operator changed)
  // coarse-space blocks: extents, count, sites per block and their indices [nb][nsb] (even sites
  // for even-parity fields; all sites, odd ones as h + V4h, for fields of both parities), and the
  // neighbouring block in each of the 8 hop directions [nb][8]
  int blk[4];
  int nb, nsb;
  int coarse_both;
  int* bsite;
  int* bnbr;
  // progress reporting of the synchronous solvers
  dwf_progress_fn progress_fn;
  void* progress_user;
  int progress_every;
  // low-precision CG: pinned host copies of the scalars (two slots of max_cg_rhs * 16 doubles)
  // and an event per slot, so the host reads an iteration's scalars while the next one runs
  double* pin_scal;
  hipEvent_t pin_ev[2];
  // timing of hopping kernels
  bool timing;
  std::vector<dwf::EventPair> ev_pool;
  size_t ev_used;
  double ev_ms;
  long long ev_launches;
  int ev_stride;       // time every ev_stride-th hop launch (1: all)
  long long ev_seq;    // hop launches seen since timing was enabled
  bool ev_open;        // the current launch is being timed
};
