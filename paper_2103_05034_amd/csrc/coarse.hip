// Coarse-space transfer of the two-level method.
//
// Blocks (Two level preconditioner section): 4D boxes of bx*by*bz*bt sites
// tiling the lattice, each taken with all Ls slices.  On even-parity fields a
// block holds nsb = bx*by*bz*bt/2 even sites, listed in `bsite[b * nsb + j]`
// (half-lattice index, block-local lexicographic order).  On fields of both
// parities (packed "both" layout: the even halves of all n fields, then the
// odd halves) a block lists all nsb = bx*by*bz*bt sites, an odd site h as
// h + V4h; its data lies n half fields further on (the parity stride).  The
// blocked basis phi_k^b is a field phi_k restricted to block b.
//
// * chiral_split: P+- v = (v +- Gamma_5 v)/2 with (Gamma_5 v)_s = gamma_5
//   v_{Ls-1-s}: the five-dimensional chirality used when the domain-wall
//   operator is coarsened (Deflation basis setup section).
// * block_dot: c[r][b][k] = <phi_k^b, v_r>, the restrictor applied to nrhs
//   fields; with v = the basis itself it is the Gram matrix of every block.
// * block_combine: out_r = sum_k c[r][b][k] phi_k^b (prolongator), or the
//   in-place map phi_k <- sum_{j<=k} W[b][j][k] phi_j^b used to
//   orthonormalise (W = R^{-1} of the block's Cholesky factor).
// * block_cholesky: per block G = R^dag R, then W = R^{-1}.
//
// One workgroup owns one block; its lane p = j * Ls + s holds one 5D site of
// the block (blocks of more than 512 5D sites: lane p also holds site p + 512).  Spinor loads are contiguous along s as in every other kernel.
// Sums over a block are reduced in a fixed order (wavefront shuffles, then
// the waves in index order), so results are reproducible run to run.
#include <algorithm>

#include "dwf_internal.hpp"
#include "kernels.hpp"

namespace dwf {

constexpr int KG = 4;  // basis vectors per reduction batch of block_dot

// (P+ v, P- v) for one lane: upper spins take (v_s + v_r)/2 and (v_s - v_r)/2,
// lower spins (gamma_5 = -1) the other way round; r = Ls - 1 - s
template <int P>
__global__ void __launch_bounds__(256) chiral_split_kernel(Geom g, const char* __restrict__ in, char* __restrict__ out,
                                                            size_t stride) {
  using R = typename Store<P>::real;
  const long long n = g.V4h * g.Ls;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = blockIdx.y;
  const long long h = i / g.Ls;
  const int s = (int)(i - h * g.Ls);
  const char* v = in + (size_t)k * stride;
  cplx<R> a[12], b[12], p[12], m[12];
  Store<P>::load(v, g.V4h, g.Ls, h, s, a);
  Store<P>::load(v, g.V4h, g.Ls, h, g.Ls - 1 - s, b);
  const R half = (R)0.5;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const cplx<R> sum = {(a[c].re + b[c].re) * half, (a[c].im + b[c].im) * half};
    const cplx<R> dif = {(a[c].re - b[c].re) * half, (a[c].im - b[c].im) * half};
    p[c] = c < 6 ? sum : dif;
    m[c] = c < 6 ? dif : sum;
  }
  Store<P>::store(out + (size_t)(2 * k) * stride, g.V4h, g.Ls, h, s, p);
  Store<P>::store(out + (size_t)(2 * k + 1) * stride, g.V4h, g.Ls, h, s, m);
}

// Fixed-order sum of NV doubles over the workgroup; thread 0 gets the totals.
// red holds (blockDim / 64) * NV doubles.
template <int NV>
__device__ __forceinline__ void group_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double x = v[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    v[i] = x;
  }
  __syncthreads();  // red is free
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i * nw + wave] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double t = 0;
      for (int w = 0; w < nw; ++w) t += red[i * nw + w];
      v[i] = t;
    }
  }
}

struct BlockArgs {
  Geom g;
  const int* bsite;  // [nb][nsb]; odd sites (fields of both parities) as h + V4h
  int nsb, nb;
  size_t basis_ps, v_ps, out_ps;  // byte offset of the odd halves (fields of both parities)
  const char* basis;  // nvec fields, stride `stride`
  int nvec;
  size_t stride;
  const char* v;  // block_dot: nrhs fields, stride `stride`
  char* out;      // block_combine: output fields (or the basis itself, in place)
  int nrhs;
  double* coef;        // block_dot output / block_combine input, complex [nrhs][nb][nvec]
  int per_block;       // block_dot: lay coef out as [nb][nrhs][nvec] (each block's Gram matrix contiguous)
  const double* wmat;  // block_combine in-place mode: complex [nb][nvec][nvec], W[j][k] at (j * nvec + k)
};

// Half-lattice site and parity of a block-table entry.
__device__ __forceinline__ int split_site(long long V4h, long long& h) {
  const int par = h >= V4h ? 1 : 0;
  h -= par * V4h;
  return par;
}

// c[r][b][k] = <phi_k^b, v_r> for the RT right-hand sides r = blockIdx.y * RT + ...
// A lane holds PP of the block's 5D sites (p = lane + q * blockDim.x), so a block
// may have up to PP * 512 of them.
template <int P, int RT, int PP>
__global__ void __launch_bounds__(512) block_dot_kernel(BlockArgs a) {
  using R = typename Store<P>::real;
  extern __shared__ double red[];
  const int b = blockIdx.x;
  const int r0 = blockIdx.y * RT;
  const int np = a.nsb * a.g.Ls;
  bool live[PP];
  long long h[PP];
  int s[PP], par[PP];
#pragma unroll
  for (int q = 0; q < PP; ++q) {
    const int p = threadIdx.x + q * blockDim.x;
    live[q] = p < np;
    h[q] = 0;
    s[q] = 0;
    par[q] = 0;
    if (live[q]) {
      const int j = p / a.g.Ls;
      s[q] = p - j * a.g.Ls;
      h[q] = a.bsite[(size_t)b * a.nsb + j];
      par[q] = split_site(a.g.V4h, h[q]);
    }
  }
  cplx<R> v[PP][RT][12];
#pragma unroll
  for (int q = 0; q < PP; ++q)
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const bool use = live[q] && (r0 + r < a.nrhs);
#pragma unroll
      for (int c = 0; c < 12; ++c) v[q][r][c] = {0, 0};
      if (use) Store<P>::load(a.v + par[q] * a.v_ps + (size_t)(r0 + r) * a.stride, a.g.V4h, a.g.Ls, h[q], s[q], v[q][r]);
    }
  // a Gram matrix (per_block) is Hermitian and its Cholesky factorisation reads
  // only the entries with basis index <= rhs index: stop at the tile's last rhs
  const int kend = a.per_block ? min(a.nvec, r0 + RT) : a.nvec;
  for (int k0 = 0; k0 < kend; k0 += KG) {
    double acc[2 * RT * KG];
#pragma unroll
    for (int i = 0; i < 2 * RT * KG; ++i) acc[i] = 0;
#pragma unroll
    for (int kk = 0; kk < KG; ++kk) {
#pragma unroll
      for (int q = 0; q < PP; ++q) {
        if (live[q] && k0 + kk < kend) {
          cplx<R> f[12];
          Store<P>::load(a.basis + par[q] * a.basis_ps + (size_t)(k0 + kk) * a.stride, a.g.V4h, a.g.Ls, h[q], s[q], f);
#pragma unroll
          for (int r = 0; r < RT; ++r) {
            double re = acc[2 * (r * KG + kk)], im = acc[2 * (r * KG + kk) + 1];
#pragma unroll
            for (int c = 0; c < 12; ++c) {  // conj(f) v
              re = fma((double)f[c].re, (double)v[q][r][c].re, re);
              re = fma((double)f[c].im, (double)v[q][r][c].im, re);
              im = fma((double)f[c].re, (double)v[q][r][c].im, im);
              im = fma(-(double)f[c].im, (double)v[q][r][c].re, im);
            }
            acc[2 * (r * KG + kk)] = re;
            acc[2 * (r * KG + kk) + 1] = im;
          }
        }
      }
    }
    group_sum<2 * RT * KG>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int kk = 0; kk < KG; ++kk)
          if (r0 + r < a.nrhs && k0 + kk < kend) {
            const size_t row = a.per_block ? (size_t)b * a.nrhs + r0 + r : (size_t)(r0 + r) * a.nb + b;
            double* o = a.coef + 2 * (row * a.nvec + k0 + kk);
            o[0] = acc[2 * (r * KG + kk)];
            o[1] = acc[2 * (r * KG + kk) + 1];
          }
    }
  }
}

// Gram matrix of every block, G[b][k][j] = <phi_j^b, phi_k^b> for j <= k, with
// each basis vector read once: the block's rows (5D site x colour-spin
// component) pass through LDS in chunks of `chunk` 5D sites, all nvec
// vectors at once, and every thread accumulates 2 x 2 tiles of (j, k) pairs
// in FP64 from the staged rows.
constexpr int GRAM_TPT = 4;  // tiles per thread: (n/2)(n/2+1)/2 <= 528 for n <= 64

template <int P>
__global__ void __launch_bounds__(256) block_gram_kernel(BlockArgs a, int chunk) {
  using R = typename Store<P>::real;
  extern __shared__ char smem[];
  cplx<R>* sm = reinterpret_cast<cplx<R>*>(smem);  // [chunk * 12][n]
  const int b = blockIdx.x;
  const int n = a.nvec;
  const int Ls = a.g.Ls;
  const int np = a.nsb * Ls;
  const int half = (n + 1) / 2;
  const int ntiles = half * (half + 1) / 2;
  double acc[GRAM_TPT][8];
  int ta[GRAM_TPT], tb[GRAM_TPT];
#pragma unroll
  for (int q = 0; q < GRAM_TPT; ++q) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[q][i] = 0;
    // tile index -> (ta <= tb): row-major over the upper triangle
    int t = threadIdx.x + q * blockDim.x, row = 0;
    while (t >= half - row && row < half) {
      t -= half - row;
      ++row;
    }
    ta[q] = row;
    tb[q] = row + t;
  }
  for (int p0 = 0; p0 < np; p0 += chunk) {
    const int cs = min(chunk, np - p0);
    __syncthreads();  // previous chunk consumed
    for (int item = threadIdx.x; item < cs * n; item += blockDim.x) {
      const int j = item / cs, pl = item - j * cs;  // consecutive threads: consecutive 5D sites
      const int p = p0 + pl;
      const int site = p / Ls, s = p - site * Ls;
      long long h = a.bsite[(size_t)b * a.nsb + site];
      const int par = split_site(a.g.V4h, h);
      cplx<R> f[12];
      Store<P>::load(a.basis + par * a.basis_ps + (size_t)j * a.stride, a.g.V4h, Ls, h, s, f);
#pragma unroll
      for (int c = 0; c < 12; ++c) sm[(size_t)(pl * 12 + c) * n + j] = f[c];
    }
    __syncthreads();
    const int rows = cs * 12;
#pragma unroll
    for (int q = 0; q < GRAM_TPT; ++q) {
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
  // G[b][k][j] = <phi_j, phi_k>, j <= k
  double* G = a.coef + 2 * (size_t)b * n * n;
#pragma unroll
  for (int q = 0; q < GRAM_TPT; ++q) {
    if (threadIdx.x + q * blockDim.x >= ntiles) continue;
    const int j0 = 2 * ta[q], k0 = 2 * tb[q];
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
      for (int dk = 0; dk < 2; ++dk) {
        const int j = j0 + dj, k = k0 + dk;
        if (j >= n || k >= n || j > k) continue;
        G[2 * (k * n + j)] = acc[q][2 * (2 * dj + dk)];
        G[2 * (k * n + j) + 1] = acc[q][2 * (2 * dj + dk) + 1];
      }
  }
}

// INPLACE = false: out_r = sum_k coef[r][b][k] phi_k^b for the KT right-hand
//   sides r = blockIdx.y * KT + ...
// INPLACE = true: phi_k <- sum_{j<=k} W[b][j][k] phi_j^b for every k, one
//   workgroup per block taking the k tiles from the top down, so that the
//   phi_j a tile still needs (j below the tile) are not yet overwritten; every
//   lane reads and writes only its own 5D site.
template <int P, int KT, bool INPLACE>
__global__ void __launch_bounds__(512) block_combine_kernel(BlockArgs a) {
  using R = typename Store<P>::real;
  extern __shared__ double cs[];  // complex coefficients of the workgroup
  const int b = blockIdx.x;
  const int np = a.nsb * a.g.Ls;
  const int n = a.nvec;
  if (INPLACE) {
    for (int i = threadIdx.x; i < n * n; i += blockDim.x) {
      cs[2 * i] = a.wmat[2 * ((size_t)b * n * n + i)];
      cs[2 * i + 1] = a.wmat[2 * ((size_t)b * n * n + i) + 1];
    }
  } else {
    const int r0 = blockIdx.y * KT;
    for (int i = threadIdx.x; i < KT * n; i += blockDim.x) {
      const int r = i / n, k = i - r * n;
      double re = 0, im = 0;
      if (r0 + r < a.nrhs) {
        const double* c = a.coef + 2 * (((size_t)(r0 + r) * a.nb + b) * n + k);
        re = c[0];
        im = c[1];
      }
      cs[2 * i] = re;
      cs[2 * i + 1] = im;
    }
  }
  __syncthreads();
  // every lane handles the block's 5D sites p = lane, lane + blockDim.x, ...
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    const int jsite = p / a.g.Ls;
    const int s = p - jsite * a.g.Ls;
    long long h = a.bsite[(size_t)b * a.nsb + jsite];
    const int par = split_site(a.g.V4h, h);
    const char* bb = a.basis + par * a.basis_ps;
    char* ob = a.out + par * a.out_ps;
    const int ntiles = INPLACE ? (n + KT - 1) / KT : 1;
    for (int tile = ntiles - 1; tile >= 0; --tile) {
      const int k0 = tile * KT;                         // INPLACE: outputs k0 .. k0+KT-1
      const int jmax = INPLACE ? min(n, k0 + KT) : n;  // inputs j < jmax
      cplx<double> acc[KT][12];
#pragma unroll
      for (int t = 0; t < KT; ++t)
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[t][c] = {0, 0};
      for (int j = 0; j < jmax; ++j) {
        cplx<R> f[12];
        Store<P>::load(bb + (size_t)j * a.stride, a.g.V4h, a.g.Ls, h, s, f);
#pragma unroll
        for (int t = 0; t < KT; ++t) {
          // coefficient of phi_j in output t
          const int idx = INPLACE ? (j * n + k0 + t) : (t * n + j);
          if (INPLACE && (k0 + t >= n || j > k0 + t)) continue;
          const double cr = cs[2 * idx], ci = cs[2 * idx + 1];
#pragma unroll
          for (int c = 0; c < 12; ++c) {
            acc[t][c].re = fma(cr, (double)f[c].re, fma(-ci, (double)f[c].im, acc[t][c].re));
            acc[t][c].im = fma(cr, (double)f[c].im, fma(ci, (double)f[c].re, acc[t][c].im));
          }
        }
      }
#pragma unroll
      for (int t = 0; t < KT; ++t) {
        const int k = INPLACE ? k0 + t : blockIdx.y * KT + t;
        if (k >= (INPLACE ? n : a.nrhs)) continue;
        cplx<R> o[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) o[c] = {(R)acc[t][c].re, (R)acc[t][c].im};
        Store<P>::store(ob + (size_t)k * a.stride, a.g.V4h, a.g.Ls, h, s, o);
      }
    }
  }
}

// Per block: Cholesky G = R^dag R of the Hermitian Gram matrix
// G[k][j] = <phi_j, phi_k> (as block_dot lays it out, row = rhs = k; only
// j <= k is read), then W = R^{-1}, upper triangular, stored W[j][k] at
// (j * n + k).  One wave per block, lane k owning column k: row j of R is
// R[j][k] = (G_jk - sum_{i<j} conj(R[i][j]) R[i][k]) / R[j][j], computed by
// all lanes k >= j at once from column j (finished by lane j in the step
// before); column k of R^{-1} then needs only R and the lane's own column.
// A non-positive or non-finite pivot raises *flag.
__global__ void __launch_bounds__(64) block_cholesky_kernel(const double* __restrict__ gram, double* __restrict__ w,
                                                            int nb, int n, int* flag) {
  extern __shared__ double rs[];  // R, complex [n][n]
  const int b = blockIdx.x;
  const int k = threadIdx.x;
  const double* G = gram + 2 * (size_t)b * n * n;
  double* W = w + 2 * (size_t)b * n * n;
  for (int i = k; i < n * n; i += 64) {
    rs[2 * i] = 0.0;
    rs[2 * i + 1] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (k == j) {
      double d = G[2 * (j * n + j)];
      for (int i = 0; i < j; ++i) d -= rs[2 * (i * n + j)] * rs[2 * (i * n + j)] + rs[2 * (i * n + j) + 1] * rs[2 * (i * n + j) + 1];
      if (!(d > 0.0) || !isfinite(d)) {
        *flag = 1;
        d = 1.0;
      }
      rs[2 * (j * n + j)] = sqrt(d);
    }
    __syncthreads();
    if (k > j && k < n) {
      double re = G[2 * (k * n + j)], im = G[2 * (k * n + j) + 1];  // G_jk = <phi_j, phi_k>
      for (int i = 0; i < j; ++i) {
        const double ar = rs[2 * (i * n + j)], ai = -rs[2 * (i * n + j) + 1];  // conj(R[i][j])
        const double br = rs[2 * (i * n + k)], bi = rs[2 * (i * n + k) + 1];
        re -= ar * br - ai * bi;
        im -= ar * bi + ai * br;
      }
      const double inv = 1.0 / rs[2 * (j * n + j)];
      rs[2 * (j * n + k)] = re * inv;
      rs[2 * (j * n + k) + 1] = im * inv;
    }
    __syncthreads();
  }
  if (k >= n) return;
  // column k of R^{-1}: W[k][k] = 1 / R[k][k]; W[j][k] = -(sum_{i=j+1..k} R[j][i] W[i][k]) / R[j][j]
  for (int j = k + 1; j < n; ++j) {
    W[2 * (j * n + k)] = 0.0;
    W[2 * (j * n + k) + 1] = 0.0;
  }
  W[2 * (k * n + k)] = 1.0 / rs[2 * (k * n + k)];
  W[2 * (k * n + k) + 1] = 0.0;
  for (int j = k - 1; j >= 0; --j) {
    double re = 0, im = 0;
    for (int i = j + 1; i <= k; ++i) {
      const double ar = rs[2 * (j * n + i)], ai = rs[2 * (j * n + i) + 1];
      const double br = W[2 * (i * n + k)], bi = W[2 * (i * n + k) + 1];
      re += ar * br - ai * bi;
      im += ar * bi + ai * br;
    }
    const double inv = -1.0 / rs[2 * (j * n + j)];
    W[2 * (j * n + k)] = re * inv;
    W[2 * (j * n + k) + 1] = im * inv;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static int lanes_of(const dwf_context* c) { return c->nsb * c->g.Ls; }
// workgroup of a per-block kernel: one lane per 5D site of the block, at most 512
static int group_of(int lanes) { return std::min(512, (lanes + 63) / 64 * 64); }

hipError_t launch_chiral_split(dwf_context* c, int prec, const char* in, char* out, int nvec) {
  const long long n = c->g.V4h * c->g.Ls;
  dim3 grid((unsigned)((n + 255) / 256), nvec);
  const size_t st = field_bytes_rhs(c, prec);
  // fields of both parities: the even halves, then the odd halves (nvec in, 2 nvec out)
  for (int par = 0; par < (c->coarse_both ? 2 : 1); ++par) {
    const char* i = in + (size_t)par * nvec * st;
    char* o = out + (size_t)par * 2 * nvec * st;
    switch (prec) {
      case DWF_F64: hipLaunchKernelGGL(chiral_split_kernel<DWF_F64>, grid, dim3(256), 0, c->stream, c->g, i, o, st); break;
      case DWF_F32: hipLaunchKernelGGL(chiral_split_kernel<DWF_F32>, grid, dim3(256), 0, c->stream, c->g, i, o, st); break;
      default: hipLaunchKernelGGL(chiral_split_kernel<DWF_F16S>, grid, dim3(256), 0, c->stream, c->g, i, o, st); break;
    }
  }
  return hipGetLastError();
}

static BlockArgs block_args(const dwf_context* c, int prec, const char* basis, int nvec) {
  BlockArgs a{};
  a.g = c->g;
  a.bsite = c->bsite;
  a.nsb = c->nsb;
  a.nb = c->nb;
  a.basis = basis;
  a.nvec = nvec;
  a.stride = field_bytes_rhs(c, prec);
  a.basis_ps = c->coarse_both ? (size_t)nvec * a.stride : 0;
  return a;
}

template <int P, int RT, int PP>
static void dot_t(const dwf_context* c, const BlockArgs& a) {
  const int lanes = group_of(lanes_of(c));
  const size_t lds = (size_t)(lanes / 64) * 2 * RT * KG * sizeof(double);
  hipLaunchKernelGGL((block_dot_kernel<P, RT, PP>), dim3(a.nb, (a.nrhs + RT - 1) / RT), dim3(lanes), lds, c->stream,
                     a);
}

// blocks of up to 512 5D sites: one site and two rhs per lane; up to 1024: two sites and one rhs
template <int P>
static void dot_p(const dwf_context* c, const BlockArgs& a) {
  if (lanes_of(c) <= 512)
    dot_t<P, 2, 1>(c, a);
  else
    dot_t<P, 1, 2>(c, a);
}

hipError_t launch_block_dot(dwf_context* c, int prec, const char* basis, int nvec, const char* v, int nrhs,
                            double* coef, bool per_block) {
  BlockArgs a = block_args(c, prec, basis, nvec);
  a.v = v;
  a.nrhs = nrhs;
  a.v_ps = c->coarse_both ? (size_t)nrhs * a.stride : 0;
  a.coef = coef;
  a.per_block = per_block ? 1 : 0;
  switch (prec) {
    case DWF_F64: dot_p<DWF_F64>(c, a); break;
    case DWF_F32: dot_p<DWF_F32>(c, a); break;
    default: dot_p<DWF_F16S>(c, a); break;
  }
  return hipGetLastError();
}

template <int P, int KT, bool INPLACE>
static void combine_t(const dwf_context* c, const BlockArgs& a) {
  const int lanes = group_of(lanes_of(c));
  const size_t lds = (INPLACE ? (size_t)a.nvec * a.nvec : (size_t)KT * a.nvec) * 2 * sizeof(double);
  const unsigned gy = INPLACE ? 1 : (unsigned)((a.nrhs + KT - 1) / KT);
  hipLaunchKernelGGL((block_combine_kernel<P, KT, INPLACE>), dim3(a.nb, gy), dim3(lanes), lds, c->stream, a);
}

hipError_t launch_block_prolong(dwf_context* c, int prec, const char* basis, int nvec, const double* coef, int nrhs,
                                char* out) {
  BlockArgs a = block_args(c, prec, basis, nvec);
  a.coef = const_cast<double*>(coef);
  a.nrhs = nrhs;
  a.out = out;
  a.out_ps = c->coarse_both ? (size_t)nrhs * a.stride : 0;
  switch (prec) {
    case DWF_F64: combine_t<DWF_F64, 2, false>(c, a); break;
    case DWF_F32: combine_t<DWF_F32, 2, false>(c, a); break;
    default: combine_t<DWF_F16S, 2, false>(c, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_block_apply(dwf_context* c, int prec, char* basis, int nvec, const double* wmat) {
  BlockArgs a = block_args(c, prec, basis, nvec);
  a.wmat = wmat;
  a.out = basis;
  a.out_ps = a.basis_ps;
  switch (prec) {
    case DWF_F64: combine_t<DWF_F64, 2, true>(c, a); break;
    case DWF_F32: combine_t<DWF_F32, 2, true>(c, a); break;
    default: combine_t<DWF_F16S, 2, true>(c, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_block_gram(dwf_context* c, int prec, const char* basis, int nvec, double* gram) {
  BlockArgs a = block_args(c, prec, basis, nvec);
  a.coef = gram;
  const size_t cb = prec == DWF_F64 ? 16 : 8;
  const size_t budget = 48 * 1024;
  int chunk = (int)(budget / (12 * (size_t)nvec * cb));  // 5D sites staged per pass
  if (chunk < 1) chunk = 1;
  const size_t lds = (size_t)chunk * 12 * nvec * cb;
  switch (prec) {
    case DWF_F64: hipLaunchKernelGGL(block_gram_kernel<DWF_F64>, dim3(a.nb), dim3(256), lds, c->stream, a, chunk); break;
    case DWF_F32: hipLaunchKernelGGL(block_gram_kernel<DWF_F32>, dim3(a.nb), dim3(256), lds, c->stream, a, chunk); break;
    default: hipLaunchKernelGGL(block_gram_kernel<DWF_F16S>, dim3(a.nb), dim3(256), lds, c->stream, a, chunk); break;
  }
  return hipGetLastError();
}

hipError_t launch_block_cholesky(dwf_context* c, const double* gram, double* w, int nvec, int* flag) {
  hipLaunchKernelGGL(block_cholesky_kernel, dim3(c->nb), dim3(64), (size_t)nvec * nvec * 2 * sizeof(double), c->stream,
                     gram, w, c->nb, nvec, flag);
  return hipGetLastError();
}

}  // namespace dwf
