// Host-side planning: argument checks, workspace layout, traversal orders,
// coarse-space block tables and the host arithmetic of the Cholesky QR (no
// device code).
#include "plan.hpp"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <tuple>

namespace dwf {
namespace plan {

namespace {
size_t round_up(size_t n) { return (n + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }
}  // namespace

bool valid_dims(const int dims[4], int Ls, int prec, int max_nrhs, int max_cg_rhs, std::string* why) {
  if (!dims) {
    *why = "dims is NULL";
    return false;
  }
  for (int i = 0; i < 4; ++i)
    if (dims[i] < 2 || (dims[i] & 1)) {
      char b[96];
      snprintf(b, sizeof b, "lattice extent %d (dim %d) must be even and >= 2", dims[i], i);
      *why = b;
      return false;
    }
  if (Ls < 1 || Ls > 128) {
    *why = "Ls must be in [1, 128]";
    return false;
  }
  if (prec != DWF_F64 && prec != DWF_F32 && prec != DWF_F16S) {
    *why = "unknown precision";
    return false;
  }
  if (max_nrhs < 1 || max_nrhs > 4096 || max_cg_rhs < 0 || max_cg_rhs > 4096) {
    *why = "max_nrhs must be in [1, 4096], max_cg_rhs in [0, 4096]";
    return false;
  }
  // the extents multiply in 64 bits: each is below 2^31, and the product of
  // the first two is checked before the next factor
  long long V4 = 1;
  for (int i = 0; i < 4; ++i) {
    if (V4 > (1LL << 32) / dims[i]) {
      *why = "lattice too large for 32-bit neighbour indices";
      return false;
    }
    V4 *= dims[i];
  }
  if (V4 / 2 > (1LL << 31) - 1) {
    *why = "lattice too large for 32-bit neighbour indices";
    return false;
  }
  return true;
}

Workspace plan_workspace(const int dims[4], int Ls, int prec, int max_nrhs, int max_cg_rhs) {
  const long long V4 = (long long)dims[0] * dims[1] * dims[2] * dims[3];
  const size_t V4h = (size_t)(V4 / 2);
  auto fb = [&](int p) { return SPINOR_BYTES[p] * (size_t)Ls * V4h; };
  Workspace w;
  for (int b = 0; b < B_COUNT; ++b) {
    w.offset[b] = ABSENT;
    w.bytes[b] = 0;
  }
  size_t off = 0;
  auto take = [&](Buffer b, size_t n) {
    w.offset[b] = off;
    w.bytes[b] = n;
    off += round_up(n);
  };
  const int chunk = max_nrhs > max_cg_rhs ? max_nrhs : max_cg_rhs;
  w.chunk = chunk;
  take(B_LINKS64, (size_t)2 * 8 * 9 * V4h * 16);
  if (prec != DWF_F64) take(B_LINKS32, (size_t)2 * 8 * 9 * V4h * 8);
  take(B_NBR, (size_t)2 * 8 * V4h * 4);
  take(B_T, fb(prec) * chunk);
  take(B_U, fb(prec) * chunk);
  take(B_CHEB, fb(prec) * (size_t)(max_nrhs > 2 ? max_nrhs : 2));
  if (max_cg_rhs > 0) {
    take(B_R64, fb(DWF_F64) * max_cg_rhs);
    take(B_P64, fb(DWF_F64) * max_cg_rhs);
    take(B_Q64, fb(DWF_F64) * max_cg_rhs);
    take(B_B64, fb(DWF_F64) * max_cg_rhs);
    if (prec == DWF_F64) take(B_DIR64, 2 * fb(DWF_F64) * max_cg_rhs);
    if (prec != DWF_F64) {
      take(B_T64, fb(DWF_F64) * max_cg_rhs);
      take(B_U64, fb(DWF_F64) * max_cg_rhs);
      take(B_LO_R, fb(DWF_F32) * max_cg_rhs);
      take(B_LO_X, fb(DWF_F32) * max_cg_rhs);
      take(B_LO_P, fb(prec) * max_cg_rhs);
      take(B_LO_Q, fb(prec) * max_cg_rhs);
    }
  }
  take(B_ORDER, (size_t)2 * V4h * sizeof(int));
  take(B_BSITE, (size_t)2 * V4h * sizeof(int));
  take(B_BNBR, (size_t)8 * V4h * sizeof(int));
  if (max_cg_rhs > 0) take(B_HOP_PARTIALS, (size_t)max_cg_rhs * V4h * sizeof(double));
  take(B_PARTIALS, (size_t)chunk * RED_BLOCKS * 2 * sizeof(double));
  take(B_SCALARS, (size_t)chunk * NSCAL * sizeof(double));
  take(B_COEF, (size_t)(4 * GS_MAX + 8) * sizeof(double));
  take(B_COUNTERS, (size_t)chunk * sizeof(unsigned));
  w.total = off;
  return w;
}

bool build_box_order(int X, int Y, int Z, int T, int nx, int ny, int nz, std::vector<int>& ord) {
  const size_t V4h = (size_t)X * Y * Z * T / 2;
  ord.assign(2 * V4h, 0);
  if (nx < 1 || ny < 1 || nz < 1 || X % nx || Y % ny || Z % nz) return false;
  const int bx = X / nx, by = Y / ny, bz = Z / nz;
  if (bx % 2) return false;
  for (int p = 0; p < 2; ++p) {
    size_t k = (size_t)p * V4h;
    for (int rz = 0; rz < nz; ++rz)
      for (int ry = 0; ry < ny; ++ry)
        for (int rx = 0; rx < nx; ++rx) {
          const int ox = rx * bx, oy = ry * by, oz = rz * bz;
          for (int t = 0; t < T; ++t)
            for (int z = oz; z < oz + bz; ++z)
              for (int y = oy; y < oy + by; ++y)
                for (int x = ox; x < ox + bx; ++x)
                  if (((x + y + z + t) & 1) == p) ord[k++] = (int)half_index(X, Y, Z, x, y, z, t);
        }
    if (k != (size_t)(p + 1) * V4h) return false;
  }
  return true;
}

bool build_order(int X, int Y, int Z, int T, int mode, std::vector<int>& ord) {
  const size_t V4h = (size_t)X * Y * Z * T / 2;
  ord.assign(2 * V4h, 0);
  if (mode == 1) {
    if (X % 4 || Y % 4 || Z % 4) return false;
    return build_box_order(X, Y, Z, T, 2, 2, 2, ord);
  }
  if (mode == 2) {
    if (T % 8) return false;
    const int st = T / 8;
    for (int p = 0; p < 2; ++p) {
      size_t k = (size_t)p * V4h;
      for (int slab = 0; slab < 8; ++slab)
        for (int y = 0; y < Y; ++y)
          for (int z = 0; z < Z; ++z)
            for (int x = 0; x < X; ++x)
              for (int t = slab * st; t < (slab + 1) * st; ++t)
                if (((x + y + z + t) & 1) == p) ord[k++] = (int)half_index(X, Y, Z, x, y, z, t);
      if (k != (size_t)(p + 1) * V4h) return false;
    }
    return true;
  }
  return false;
}

bool build_blocks(int X, int Y, int Z, int T, int Ls, const int block[4], bool both, std::vector<int>& sites,
                  std::vector<int>& nbrs, int* nblocks, int* sites_per_block, std::string* why) {
  char b[160];
  const int ext[4] = {X, Y, Z, T};
  for (int i = 0; i < 4; ++i)
    if (block[i] < 1 || ext[i] % block[i]) {
      snprintf(b, sizeof b, "block extent %d (dim %d) must divide the lattice extent %d", block[i], i, ext[i]);
      *why = b;
      return false;
    }
  const long long vol = (long long)block[0] * block[1] * block[2] * block[3];
  if (vol % 2) {
    *why = "the block volume must be even";
    return false;
  }
  const long long nsb = both ? vol : vol / 2;
  if (nsb * Ls > 1024) {
    snprintf(b, sizeof b, "%s per block x Ls = %lld exceeds 1024", both ? "sites" : "even sites", nsb * Ls);
    *why = b;
    return false;
  }
  const long long V4h = (long long)X * Y * Z * T / 2;
  if (both && 2 * V4h > (1LL << 31) - 1) {
    *why = "lattice too large for DWF_BOTH";
    return false;
  }
  const int n[4] = {X / block[0], Y / block[1], Z / block[2], T / block[3]};
  const long long nb = (long long)n[0] * n[1] * n[2] * n[3];
  sites.assign((size_t)(nb * nsb), 0);
  nbrs.assign((size_t)nb * 8, 0);
  for (int bt = 0; bt < n[3]; ++bt)
    for (int bz = 0; bz < n[2]; ++bz)
      for (int by = 0; by < n[1]; ++by)
        for (int bx = 0; bx < n[0]; ++bx) {
          const long long blk = ((long long)(bt * n[2] + bz) * n[1] + by) * n[0] + bx;
          const int bc[4] = {bx, by, bz, bt};
          for (int d = 0; d < 8; ++d) {
            int c[4] = {bc[0], bc[1], bc[2], bc[3]};
            const int mu = d / 2;
            c[mu] = (c[mu] + (d % 2 ? n[mu] - 1 : 1)) % n[mu];
            nbrs[(size_t)blk * 8 + d] = (int)(((long long)(c[3] * n[2] + c[2]) * n[1] + c[1]) * n[0] + c[0]);
          }
          long long j = 0, odd = 0;
          for (int t = bt * block[3]; t < (bt + 1) * block[3]; ++t)
            for (int z = bz * block[2]; z < (bz + 1) * block[2]; ++z)
              for (int y = by * block[1]; y < (by + 1) * block[1]; ++y)
                for (int x = bx * block[0]; x < (bx + 1) * block[0]; ++x) {
                  const int par = (x + y + z + t) & 1;
                  odd += par;
                  if (par && !both) continue;
                  if (j == nsb) {
                    *why = "blocks must hold equal even/odd counts";
                    return false;
                  }
                  sites[(size_t)(blk * nsb + j++)] = (int)(half_index(X, Y, Z, x, y, z, t) + par * V4h);
                }
          if (2 * odd != vol) {
            *why = "blocks must hold equal even/odd counts";
            return false;
          }
        }
  *nblocks = (int)nb;
  *sites_per_block = (int)nsb;
  return true;
}

std::string format_tune_line(const TuneKey& k, const TuneEntry& e) {
  char b[512];
  snprintf(b, sizeof b, "%s %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %d %.17g", k.arch.c_str(), k.dims[0],
           k.dims[1], k.dims[2], k.dims[3], k.Ls, k.nrhs, k.prec, k.order, k.lds_floor, k.schur_form, e.spb, e.depth,
           e.rpb, e.order, e.box[0], e.box[1], e.box[2], e.ms);
  return b;
}

bool parse_tune_line(const std::string& line, TuneKey* k, TuneEntry* e) {
  std::istringstream in(line);
  TuneKey kk;
  TuneEntry ee;
  if (!(in >> kk.arch >> kk.dims[0] >> kk.dims[1] >> kk.dims[2] >> kk.dims[3] >> kk.Ls >> kk.nrhs >> kk.prec >>
        kk.order >> kk.lds_floor >> kk.schur_form >> ee.spb >> ee.depth >> ee.rpb >> ee.order >> ee.box[0] >>
        ee.box[1] >> ee.box[2] >> ee.ms))
    return false;
  std::string rest;
  if (in >> rest) return false;  // trailing fields: not a line of this format
  if (ee.spb < 1 || ee.spb * kk.Ls > 256 || ee.depth < 1 || ee.depth > 3 || ee.rpb < 1 || ee.rpb > 64 ||
      !(ee.ms >= 0) || ee.order < 0 || ee.order > 3 || ee.box[0] < 0 || ee.box[1] < 0 || ee.box[2] < 0)
    return false;  // a shape the launchers would refuse
  *k = kk;
  *e = ee;
  return true;
}

namespace {
using KeyTuple = std::tuple<std::string, int, int, int, int, int, int, int, int, int, int>;
KeyTuple as_tuple(const TuneKey& k) {
  return KeyTuple(k.arch, k.dims[0], k.dims[1], k.dims[2], k.dims[3], k.Ls, k.nrhs, k.prec, k.order, k.lds_floor,
                  k.schur_form);
}
std::mutex g_tune_mu;
std::map<KeyTuple, TuneEntry> g_tune;
bool g_tune_loaded = false;
}  // namespace

bool tune_lookup(const TuneKey& k, TuneEntry* e, const char* path) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  if (!g_tune_loaded) {
    g_tune_loaded = true;
    if (path && *path) {
      std::ifstream f(path);
      std::string line;
      while (std::getline(f, line)) {
        TuneKey fk;
        TuneEntry fe;
        if (parse_tune_line(line, &fk, &fe)) g_tune[as_tuple(fk)] = fe;
      }
    }
  }
  auto it = g_tune.find(as_tuple(k));
  if (it == g_tune.end()) return false;
  *e = it->second;
  return true;
}

void tune_store(const TuneKey& k, const TuneEntry& e, const char* path) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[as_tuple(k)] = e;
  if (path && *path) {
    std::ofstream f(path, std::ios::app);
    if (f) f << format_tune_line(k, e) << "\n";
  }
}

void tune_clear() {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
  g_tune_loaded = false;
}

bool cholesky_upper(const std::vector<double>& G, int n, std::vector<double>& R, double min_ratio) {
  R.assign((size_t)2 * n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = G[2 * ((size_t)j * n + j)];
    const double djj = d;
    for (int i = 0; i < j; ++i) d -= R[2 * ((size_t)i * n + j)] * R[2 * ((size_t)i * n + j)] +
                                      R[2 * ((size_t)i * n + j) + 1] * R[2 * ((size_t)i * n + j) + 1];
    if (!(d > min_ratio * djj) || !std::isfinite(d)) return false;
    const double rjj = std::sqrt(d);
    R[2 * ((size_t)j * n + j)] = rjj;
    for (int k = j + 1; k < n; ++k) {
      double re = G[2 * ((size_t)k * n + j)], im = G[2 * ((size_t)k * n + j) + 1];  // <v_j, v_k>
      for (int i = 0; i < j; ++i) {  // - conj(R_ij) R_ik
        const double ar = R[2 * ((size_t)i * n + j)], ai = R[2 * ((size_t)i * n + j) + 1];
        const double br = R[2 * ((size_t)i * n + k)], bi = R[2 * ((size_t)i * n + k) + 1];
        re -= ar * br + ai * bi;
        im -= ar * bi - ai * br;
      }
      R[2 * ((size_t)j * n + k)] = re / rjj;
      R[2 * ((size_t)j * n + k) + 1] = im / rjj;
    }
  }
  return true;
}

void invert_upper(const std::vector<double>& R, int n, std::vector<double>& W) {
  W.assign((size_t)2 * n * n, 0.0);
  for (int k = 0; k < n; ++k) {
    W[2 * ((size_t)k * n + k)] = 1.0 / R[2 * ((size_t)k * n + k)];
    for (int j = k - 1; j >= 0; --j) {
      double re = 0, im = 0;
      for (int i = j + 1; i <= k; ++i) {  // sum R_ji W_ik
        const double ar = R[2 * ((size_t)j * n + i)], ai = R[2 * ((size_t)j * n + i) + 1];
        const double br = W[2 * ((size_t)i * n + k)], bi = W[2 * ((size_t)i * n + k) + 1];
        re += ar * br - ai * bi;
        im += ar * bi + ai * br;
      }
      const double rjj = R[2 * ((size_t)j * n + j)];
      W[2 * ((size_t)j * n + k)] = -re / rjj;
      W[2 * ((size_t)j * n + k) + 1] = -im / rjj;
    }
  }
}

void multiply_upper(const std::vector<double>& A, const std::vector<double>& B, int n, std::vector<double>& C) {
  C.assign((size_t)2 * n * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int k = j; k < n; ++k) {
      double re = 0, im = 0;
      for (int i = j; i <= k; ++i) {
        const double ar = A[2 * ((size_t)j * n + i)], ai = A[2 * ((size_t)j * n + i) + 1];
        const double br = B[2 * ((size_t)i * n + k)], bi = B[2 * ((size_t)i * n + k) + 1];
        re += ar * br - ai * bi;
        im += ar * bi + ai * br;
      }
      C[2 * ((size_t)j * n + k)] = re;
      C[2 * ((size_t)j * n + k) + 1] = im;
    }
}

}  // namespace plan
}  // namespace dwf
