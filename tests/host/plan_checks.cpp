// Host checks of the workspace plan, the argument checks, the traversal
// orders and the coarse block tables, built with AddressSanitizer and UBSan
// (see test_host_sanitizers.py).  Every table is written into a heap buffer of
// exactly the capacity the workspace gives it, so an overrun is a sanitizer
// report; the tuning cache's line parser also takes random input.  Prints
// "all checks passed" and one "total" line per planned shape.  argv[1]: a
// directory for the tuning-cache file.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "plan.hpp"

using namespace dwf;

static int g_fail = 0;
#define CHECK(cond, ...)                      \
  do {                                        \
    if (!(cond)) {                            \
      std::printf("FAIL %s:%d: ", __FILE__, __LINE__); \
      std::printf(__VA_ARGS__);               \
      std::printf("\n");                      \
      ++g_fail;                               \
    }                                         \
  } while (0)

static void check_valid_dims() {
  std::string why;
  const int ok[4] = {4, 4, 4, 8};
  CHECK(plan::valid_dims(ok, 8, DWF_F64, 1, 0, &why), "valid lattice rejected: %s", why.c_str());
  CHECK(!plan::valid_dims(nullptr, 8, DWF_F64, 1, 0, &why), "null dims accepted");
  const int bad[][4] = {{3, 4, 4, 4}, {0, 4, 4, 4}, {-2, 4, 4, 4}, {4, 4, 4, 1}, {4, 4, 4, 7}};
  for (const auto& d : bad) CHECK(!plan::valid_dims(d, 8, DWF_F64, 1, 0, &why), "bad extents accepted");
  CHECK(!plan::valid_dims(ok, 0, DWF_F64, 1, 0, &why), "Ls 0 accepted");
  CHECK(!plan::valid_dims(ok, 129, DWF_F64, 1, 0, &why), "Ls 129 accepted");
  CHECK(plan::valid_dims(ok, 128, DWF_F16S, 4096, 4096, &why), "Ls 128, 4096 rhs rejected");
  CHECK(!plan::valid_dims(ok, 8, 3, 1, 0, &why), "precision 3 accepted");
  CHECK(!plan::valid_dims(ok, 8, -1, 1, 0, &why), "precision -1 accepted");
  CHECK(!plan::valid_dims(ok, 8, DWF_F64, 0, 0, &why), "max_nrhs 0 accepted");
  CHECK(!plan::valid_dims(ok, 8, DWF_F64, 4097, 0, &why), "max_nrhs 4097 accepted");
  CHECK(!plan::valid_dims(ok, 8, DWF_F64, 1, -1, &why), "max_cg_rhs -1 accepted");
  // sizes around the 32-bit half-lattice index limit, and products that would
  // overflow 64 bits if multiplied out unchecked
  const int edge_ok[4] = {32768, 16384, 2, 2};      // V4h = 2^30
  const int edge_bad[4] = {32768, 32768, 2, 2};     // V4h = 2^31
  const int huge[4] = {1 << 30, 1 << 30, 1 << 30, 1 << 30};
  const int big_last[4] = {2, 2, 2, 2147483646};
  CHECK(plan::valid_dims(edge_ok, 1, DWF_F64, 1, 0, &why), "V4h = 2^30 rejected: %s", why.c_str());
  CHECK(!plan::valid_dims(edge_bad, 1, DWF_F64, 1, 0, &why), "V4h = 2^31 accepted");
  CHECK(!plan::valid_dims(huge, 1, DWF_F64, 1, 0, &why), "2^120 sites accepted");
  CHECK(!plan::valid_dims(big_last, 1, DWF_F64, 1, 0, &why), "2^34 sites accepted");
}

static void check_workspace(const int dims[4], int Ls, int prec, int max_nrhs, int max_cg_rhs) {
  std::string why;
  if (!plan::valid_dims(dims, Ls, prec, max_nrhs, max_cg_rhs, &why)) {
    CHECK(false, "shape rejected: %s", why.c_str());
    return;
  }
  const plan::Workspace w = plan::plan_workspace(dims, Ls, prec, max_nrhs, max_cg_rhs);
  const size_t V4h = (size_t)dims[0] * dims[1] * dims[2] * dims[3] / 2;
  const size_t fb = SPINOR_BYTES[prec] * (size_t)Ls * V4h;
  const int chunk = std::max(max_nrhs, max_cg_rhs);
  CHECK(w.chunk == chunk, "chunk %d != %d", w.chunk, chunk);
  CHECK(w.total % WS_ALIGN == 0, "total not aligned");
  // presence
  const bool cg = max_cg_rhs > 0, low = prec != DWF_F64;
  const bool want[plan::B_COUNT] = {true, low, true, true, true, true, cg, cg, cg, cg, cg && !low, cg && low, cg && low,
                                    cg && low, cg && low, cg && low, cg && low, true, true, true, cg, true, true, true,
                                    true};
  // least sizes the kernels rely on
  size_t need[plan::B_COUNT] = {};
  need[plan::B_LINKS64] = 2 * 8 * 9 * V4h * 16;
  need[plan::B_LINKS32] = 2 * 8 * 9 * V4h * 8;
  need[plan::B_NBR] = 2 * 8 * V4h * 4;
  need[plan::B_T] = need[plan::B_U] = fb * chunk;
  need[plan::B_CHEB] = fb * std::max(max_nrhs, 2);
  for (int b : {plan::B_R64, plan::B_P64, plan::B_Q64, plan::B_B64, plan::B_T64, plan::B_U64})
    need[b] = SPINOR_BYTES[DWF_F64] * (size_t)Ls * V4h * max_cg_rhs;
  need[plan::B_DIR64] = 2 * SPINOR_BYTES[DWF_F64] * (size_t)Ls * V4h * max_cg_rhs;
  need[plan::B_LO_R] = need[plan::B_LO_X] = SPINOR_BYTES[DWF_F32] * (size_t)Ls * V4h * max_cg_rhs;
  need[plan::B_LO_P] = need[plan::B_LO_Q] = fb * max_cg_rhs;
  need[plan::B_ORDER] = need[plan::B_BSITE] = 2 * V4h * sizeof(int);
  need[plan::B_BNBR] = 8 * V4h * sizeof(int);
  need[plan::B_HOP_PARTIALS] = (size_t)max_cg_rhs * V4h * sizeof(double);
  need[plan::B_PARTIALS] = (size_t)chunk * RED_BLOCKS * 2 * sizeof(double);
  need[plan::B_SCALARS] = (size_t)chunk * NSCAL * sizeof(double);
  need[plan::B_COEF] = (4 * GS_MAX + 8) * sizeof(double);
  need[plan::B_COUNTERS] = (size_t)chunk * sizeof(unsigned);
  std::vector<std::pair<size_t, size_t>> spans;
  for (int b = 0; b < plan::B_COUNT; ++b) {
    const bool present = w.offset[b] != plan::ABSENT;
    CHECK(present == want[b], "buffer %d present=%d expected %d (prec %d, cg rhs %d)", b, present, want[b], prec,
          max_cg_rhs);
    if (!present) {
      CHECK(w.bytes[b] == 0, "absent buffer %d has bytes", b);
      continue;
    }
    CHECK(w.offset[b] % WS_ALIGN == 0, "buffer %d misaligned", b);
    CHECK(w.bytes[b] >= need[b], "buffer %d: %zu bytes < %zu needed", b, w.bytes[b], need[b]);
    CHECK(w.offset[b] + w.bytes[b] <= w.total, "buffer %d ends past the workspace", b);
    spans.push_back({w.offset[b], w.offset[b] + w.bytes[b]});
  }
  std::sort(spans.begin(), spans.end());
  for (size_t i = 1; i < spans.size(); ++i) CHECK(spans[i].first >= spans[i - 1].second, "buffers overlap");
  std::printf("total %d %d %d %d %d %d %d %d %zu\n", dims[0], dims[1], dims[2], dims[3], Ls, prec, max_nrhs,
              max_cg_rhs, w.total);
}

// parity and coordinates of half-lattice site h (x fastest, x = 2 xh or 2 xh + 1)
static void decode(const int d[4], int p, long long h, int c[4]) {
  const int Xh = d[0] / 2;
  long long r = h;
  const int xh = (int)(r % Xh);
  r /= Xh;
  c[1] = (int)(r % d[1]);
  r /= d[1];
  c[2] = (int)(r % d[2]);
  c[3] = (int)(r / d[2]);
  c[0] = 2 * xh + ((p + c[1] + c[2] + c[3]) & 1);
}

static void check_orders(const int d[4]) {
  const size_t V4h = (size_t)d[0] * d[1] * d[2] * d[3] / 2;
  for (int mode = -1; mode <= 4; ++mode) {
    std::vector<int> ord;
    const bool ok = plan::build_order(d[0], d[1], d[2], d[3], mode, ord);
    const bool admits = (mode == 1 && d[0] % 4 == 0 && d[1] % 4 == 0 && d[2] % 4 == 0) || (mode == 2 && d[3] % 8 == 0);
    CHECK(ok == admits, "order %d on %dx%dx%dx%d: built=%d expected %d", mode, d[0], d[1], d[2], d[3], ok, admits);
    if (!ok) continue;
    CHECK(ord.size() == 2 * V4h, "order table size");
    // copied into a buffer of exactly the workspace capacity ([2][V4h] int)
    int* cap = static_cast<int*>(std::malloc(2 * V4h * sizeof(int)));
    std::memcpy(cap, ord.data(), ord.size() * sizeof(int));
    for (int p = 0; p < 2; ++p) {
      std::vector<char> seen(V4h, 0);
      for (size_t k = 0; k < V4h; ++k) {
        const int h = cap[p * V4h + k];
        if (h < 0 || (size_t)h >= V4h) {
          CHECK(false, "order %d: index %d out of range", mode, h);
          continue;
        }
        CHECK(!seen[h], "order %d parity %d: site %d twice", mode, p, h);
        seen[h] = 1;
        int c[4];
        decode(d, p, h, c);
        CHECK(((c[0] + c[1] + c[2] + c[3]) & 1) == p, "order %d: wrong parity", mode);
      }
      // XCD k runs the k-th eighth: octants (mode 1) hold one (x, y, z) sub-box each
      if (mode == 1)
        for (int r = 0; r < 8; ++r)
          for (size_t k = r * V4h / 8; k < (r + 1) * V4h / 8; ++k) {
            int c[4];
            decode(d, p, cap[p * V4h + k], c);
            const int ox = (r & 1) * d[0] / 2, oy = ((r >> 1) & 1) * d[1] / 2, oz = ((r >> 2) & 1) * d[2] / 2;
            CHECK(c[0] >= ox && c[0] < ox + d[0] / 2 && c[1] >= oy && c[1] < oy + d[1] / 2 && c[2] >= oz &&
                      c[2] < oz + d[2] / 2,
                  "octant %d holds a site outside its box", r);
          }
    }
    std::free(cap);
  }
}

// box orders: a permutation per parity; the k-th eighth of the order (XCD k) holds whole
// boxes when the box count is a multiple of 8; x rows stay whole with nx = 1
static void check_box_orders(const int d[4]) {
  const size_t V4h = (size_t)d[0] * d[1] * d[2] * d[3] / 2;
  static const int extra[2][3] = {{3, 1, 1}, {0, 1, 1}};  // an odd cut of x, and a zero cut
  for (int c = 0; c < plan::NUM_BOX_CANDIDATES + 2; ++c) {
    const int* cut = c < plan::NUM_BOX_CANDIDATES ? plan::BOX_CANDIDATES[c] : extra[c - plan::NUM_BOX_CANDIDATES];
    std::vector<int> ord;
    const bool ok = plan::build_box_order(d[0], d[1], d[2], d[3], cut[0], cut[1], cut[2], ord);
    const bool admits = cut[0] >= 1 && d[0] % cut[0] == 0 && d[1] % cut[1] == 0 && d[2] % cut[2] == 0 &&
                        (d[0] / cut[0]) % 2 == 0;
    CHECK(ok == admits, "box %d,%d,%d on %dx%dx%dx%d: built=%d expected %d", cut[0], cut[1], cut[2], d[0], d[1],
          d[2], d[3], ok, admits);
    if (!ok) continue;
    const int bx = d[0] / cut[0], by = d[1] / cut[1], bz = d[2] / cut[2];
    const int nbox = cut[0] * cut[1] * cut[2];
    const size_t per_box = V4h / nbox;
    for (int p = 0; p < 2; ++p) {
      std::vector<char> seen(V4h, 0);
      for (size_t k = 0; k < V4h; ++k) {
        const int h = ord[p * V4h + k];
        if (h < 0 || (size_t)h >= V4h) {
          CHECK(false, "box order index out of range");
          continue;
        }
        CHECK(!seen[h], "box order: site twice");
        seen[h] = 1;
        int cc[4];
        decode(d, p, h, cc);
        CHECK(((cc[0] + cc[1] + cc[2] + cc[3]) & 1) == p, "box order: wrong parity");
        // the k-th site lies in box k / per_box (boxes numbered x fastest)
        const int b = (int)(k / per_box);
        const int rx = b % cut[0], ry = (b / cut[0]) % cut[1], rz = b / (cut[0] * cut[1]);
        CHECK(cc[0] / bx == rx && cc[1] / by == ry && cc[2] / bz == rz, "box order: site outside its box");
      }
    }
  }
  // mode 1 is the 2 x 2 x 2 cut
  std::vector<int> a, b;
  if (plan::build_order(d[0], d[1], d[2], d[3], 1, a)) {
    CHECK(plan::build_box_order(d[0], d[1], d[2], d[3], 2, 2, 2, b) && a == b, "mode 1 differs from the 2x2x2 cut");
  }
}

static void check_blocks(const int d[4], int Ls, const int blk[4], bool both, bool expect_ok) {
  const size_t V4h = (size_t)d[0] * d[1] * d[2] * d[3] / 2;
  std::vector<int> sites, nbrs;
  int nb = -1, nsb = -1;
  std::string why;
  const bool ok = plan::build_blocks(d[0], d[1], d[2], d[3], Ls, blk, both, sites, nbrs, &nb, &nsb, &why);
  CHECK(ok == expect_ok, "blocks %dx%dx%dx%d (both %d): built=%d expected %d (%s)", blk[0], blk[1], blk[2], blk[3],
        both, ok, expect_ok, why.c_str());
  if (!ok) {
    CHECK(!why.empty(), "no reason given");
    return;
  }
  // the workspace holds [2][V4h] site and [8][V4h] neighbour entries
  CHECK(sites.size() == (size_t)nb * nsb && sites.size() <= 2 * V4h, "site table size");
  CHECK(nbrs.size() == (size_t)nb * 8 && nbrs.size() <= 8 * V4h, "neighbour table size");
  int* st = static_cast<int*>(std::malloc(2 * V4h * sizeof(int)));
  int* nt = static_cast<int*>(std::malloc(8 * V4h * sizeof(int)));
  std::memcpy(st, sites.data(), sites.size() * sizeof(int));
  std::memcpy(nt, nbrs.data(), nbrs.size() * sizeof(int));
  const int n[4] = {d[0] / blk[0], d[1] / blk[1], d[2] / blk[2], d[3] / blk[3]};
  std::vector<char> seen(2 * V4h, 0);
  for (int b = 0; b < nb; ++b) {
    const int bc[4] = {b % n[0], (b / n[0]) % n[1], (b / (n[0] * n[1])) % n[2], b / (n[0] * n[1] * n[2])};
    for (int j = 0; j < nsb; ++j) {
      const int e = st[(size_t)b * nsb + j];
      const int p = e >= (long long)V4h ? 1 : 0;
      CHECK(both || p == 0, "odd site in an even-only table");
      const long long h = e - p * (long long)V4h;
      if (h < 0 || (size_t)h >= V4h) {
        CHECK(false, "block site %d out of range", e);
        continue;
      }
      CHECK(!seen[e], "site listed twice");
      seen[e] = 1;
      int c[4];
      decode(d, p, h, c);
      for (int mu = 0; mu < 4; ++mu)
        CHECK(c[mu] / blk[mu] == bc[mu], "block %d lists a site of another block", b);
    }
    for (int dd = 0; dd < 8; ++dd) {
      int c[4] = {bc[0], bc[1], bc[2], bc[3]};
      const int mu = dd / 2;
      c[mu] = (c[mu] + (dd % 2 ? n[mu] - 1 : 1)) % n[mu];
      const int want = ((c[3] * n[2] + c[2]) * n[1] + c[1]) * n[0] + c[0];
      CHECK(nt[(size_t)b * 8 + dd] == want, "block %d direction %d neighbour", b, dd);
    }
  }
  const size_t listed = (size_t)std::count(seen.begin(), seen.end(), 1);
  CHECK(listed == (both ? 2 * V4h : V4h), "blocks do not cover the lattice");
  std::free(st);
  std::free(nt);
}

static void check_tune_cache(const std::string& dir) {
  plan::TuneKey k{"gfx950:sramecc+:xnack-", {16, 16, 16, 32}, 16, 1, DWF_F64, 1, 0, 1};
  plan::TuneEntry e{8, 3, 1, 3, {1, 2, 4}, 0.6192718505859375};
  plan::TuneKey k2;
  plan::TuneEntry e2;
  CHECK(plan::parse_tune_line(plan::format_tune_line(k, e), &k2, &e2), "formatted line does not parse");
  CHECK(k2.arch == k.arch && std::memcmp(k2.dims, k.dims, sizeof k.dims) == 0 && k2.Ls == k.Ls && k2.nrhs == k.nrhs &&
            k2.prec == k.prec && k2.order == k.order && k2.lds_floor == k.lds_floor && k2.schur_form == k.schur_form,
        "key does not round-trip");
  CHECK(e2.spb == e.spb && e2.depth == e.depth && e2.rpb == e.rpb && e2.order == e.order && e2.box[0] == 1 &&
            e2.box[1] == 2 && e2.box[2] == 4 && e2.ms == e.ms,
        "entry does not round-trip");
  const char* bad[] = {"", "gfx950", "gfx950 16 16 16 32 16 1 0 -1 0 1 8 3 1 3 1 2 4",          // too short
                       "gfx950 16 16 16 32 16 1 0 -1 0 1 8 3 1 3 1 2 4 0.5 extra",                // trailing field
                       "gfx950 16 16 16 32 16 1 0 -1 0 1 8 3 1 0.5",                              // the older format
                       "gfx950 16 16 16 32 16 1 0 -1 0 1 32 3 1 3 1 2 4 0.5",                     // 32 x 16 lanes
                       "gfx950 16 16 16 32 16 1 0 -1 0 1 8 0 1 3 1 2 4 0.5",
                       "gfx950 16 16 16 32 16 1 0 -1 0 1 8 4 1 3 1 2 4 0.5",
                       "gfx950 16 16 16 32 16 1 0 -1 0 1 8 3 0 3 1 2 4 0.5",
                       "gfx950 16 16 16 32 16 1 0 -1 0 1 8 3 65 3 1 2 4 0.5",
                       "gfx950 16 16 16 32 16 1 0 -1 0 1 8 3 1 4 1 2 4 0.5",                      // order 4
                       "gfx950 16 16 16 32 16 1 0 -1 0 1 8 3 1 3 -1 2 4 0.5",
                       "gfx950 16 16 16 32 16 1 0 -1 0 1 8 3 1 3 1 2 4 nan",
                       "gfx950 16 16 16 32 16 1 0 -1 0 1 8 3 1 3 1 2 4 -1",
                       "gfx950 x 16 16 32 16 1 0 -1 0 1 8 3 1 3 1 2 4 0.5",
                       "gfx950 16 16 16 32 16 1 0 -1 0 1 8 3 1 3 1 2 4 1e999x"};
  for (const char* line : bad) CHECK(!plan::parse_tune_line(line, &k2, &e2), "bad line parsed: '%s'", line);
  // random bytes and numbers: the parser must reject or accept cleanly
  unsigned seed = 12345;
  auto rnd = [&]() { return seed = seed * 1103515245u + 12345u, (seed >> 16) & 0x7fff; };
  for (int i = 0; i < 3000; ++i) {
    std::string line;
    const int n = rnd() % 120;
    for (int j = 0; j < n; ++j) {
      const int c = rnd() % 6;
      line += c == 0 ? ' ' : c == 1 ? (char)('0' + rnd() % 10) : c == 2 ? '-' : c == 3 ? (char)(rnd() % 256) : 'e';
    }
    plan::parse_tune_line(line, &k2, &e2);
  }
  // the process cache and its file
  const std::string path = dir + "/tune_cache.txt";
  std::remove(path.c_str());
  plan::tune_clear();
  CHECK(!plan::tune_lookup(k, &e2, path.c_str()), "hit in an empty cache");
  plan::tune_store(k, e, path.c_str());
  plan::TuneKey k3 = k;
  k3.nrhs = 40;
  k3.prec = DWF_F32;
  plan::tune_store(k3, plan::TuneEntry{16, 3, 2, 1, {0, 0, 0}, 3.125}, path.c_str());
  {
    FILE* f = std::fopen(path.c_str(), "a");
    std::fputs("this line is not an entry\n", f);
    std::fclose(f);
  }
  plan::tune_clear();  // forget: the next lookup reads the file
  CHECK(plan::tune_lookup(k, &e2, path.c_str()) && e2.spb == 8 && e2.depth == 3 && e2.order == 3 && e2.box[2] == 4 &&
            e2.ms == e.ms,
        "entry not read back from the file");
  CHECK(plan::tune_lookup(k3, &e2, path.c_str()) && e2.spb == 16 && e2.rpb == 2, "second entry not read back");
  plan::TuneKey k4 = k;
  k4.order = 2;
  CHECK(!plan::tune_lookup(k4, &e2, path.c_str()), "a different traversal order hit the cache");
  plan::tune_clear();
  CHECK(!plan::tune_lookup(k, &e2, nullptr), "hit after clearing, with no file");
  std::remove(path.c_str());
}

// Host arithmetic of the Cholesky QR: R^dag R reproduces the Gram matrix of a
// random complex set (norms spread over e^{+-3}, a near-parallel pair), R W = 1,
// the triangular product against a full product, and the breakdown answers.
static void check_cholesky() {
  unsigned long long st = 12345;
  auto rnd = [&]() {  // uniform in (-1, 1) from a 64-bit LCG
    st = st * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(st >> 11) / (double)(1ULL << 52) - 1.0;
  };
  using C = std::complex<double>;
  for (int n : {1, 2, 5, 17, 40, 64}) {
    const int m = 3 * n + 7;
    std::vector<C> V((size_t)m * n);
    for (int k = 0; k < n; ++k) {
      const double sc = std::exp(-3.0 + 6.0 * k / std::max(1, n - 1));
      for (int i = 0; i < m; ++i) V[(size_t)i * n + k] = sc * C(rnd(), rnd());
    }
    if (n > 3)
      for (int i = 0; i < m; ++i) V[(size_t)i * n + 2] += 40.0 * V[(size_t)i * n + 1];
    std::vector<double> G((size_t)2 * n * n, 0.0), R, W, P;
    double gmax = 0;
    for (int k = 0; k < n; ++k)
      for (int j = 0; j <= k; ++j) {
        C g = 0;
        for (int i = 0; i < m; ++i) g += std::conj(V[(size_t)i * n + j]) * V[(size_t)i * n + k];
        G[2 * ((size_t)k * n + j)] = g.real();
        G[2 * ((size_t)k * n + j) + 1] = g.imag();
        gmax = std::max(gmax, std::abs(g));
      }
    CHECK(plan::cholesky_upper(G, n, R, 1e-14), "cholesky rejected a well-posed set, n %d", n);
    auto at = [&](const std::vector<double>& A, int r, int c) { return C(A[2 * ((size_t)r * n + c)], A[2 * ((size_t)r * n + c) + 1]); };
    double err = 0, low = 0, diag_ok = 1;
    for (int j = 0; j < n; ++j) {
      if (!(at(R, j, j).real() > 0) || at(R, j, j).imag() != 0) diag_ok = 0;
      for (int k = 0; k < n; ++k) {
        if (k < j) low = std::max(low, std::abs(at(R, j, k)));
        if (k < j) continue;
        C s = 0;  // (R^dag R)_{jk} = sum_i conj(R_ij) R_ik
        for (int i = 0; i <= j; ++i) s += std::conj(at(R, i, j)) * at(R, i, k);
        err = std::max(err, std::abs(s - at(G, k, j)));
      }
    }
    CHECK(err < 1e-13 * gmax, "R^dag R != G (n %d, error %g of %g)", n, err, gmax);
    CHECK(low == 0 && diag_ok, "R not upper triangular with a positive real diagonal (n %d)", n);
    plan::invert_upper(R, n, W);
    double ierr = 0;
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        C s = 0;
        for (int i = 0; i < n; ++i) s += at(R, j, i) * at(W, i, k);
        ierr = std::max(ierr, std::abs(s - (j == k ? 1.0 : 0.0)));
      }
    CHECK(ierr < 1e-10, "R W != 1 (n %d, error %g)", n, ierr);
    plan::multiply_upper(R, W, n, P);
    double perr = 0;
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) perr = std::max(perr, std::abs(at(P, j, k) - (j == k ? 1.0 : 0.0)));
    CHECK(perr < 1e-10, "multiply_upper(R, R^-1) != 1 (n %d, error %g)", n, perr);
    if (n >= 2) {  // a repeated vector: no positive second pivot
      std::vector<double> Gs = G;
      Gs[2 * ((size_t)1 * n + 1)] = G[0];
      Gs[2 * ((size_t)1 * n + 0)] = G[0];
      Gs[2 * ((size_t)1 * n + 0) + 1] = 0;
      CHECK(!plan::cholesky_upper(Gs, n, R, 1e-14), "cholesky accepted a singular Gram matrix (n %d)", n);
    }
  }
  std::vector<double> neg = {-1.0, 0.0}, R;
  CHECK(!plan::cholesky_upper(neg, 1, R, 0.0), "cholesky accepted a negative pivot");
  std::vector<double> nan1 = {std::nan(""), 0.0};
  CHECK(!plan::cholesky_upper(nan1, 1, R, 0.0), "cholesky accepted a NaN pivot");
}

int main(int argc, char** argv) {
  check_valid_dims();
  check_cholesky();
  check_tune_cache(argc > 1 ? argv[1] : ".");
  const int shapes[][4] = {{2, 2, 2, 2}, {4, 4, 6, 8}, {8, 4, 4, 8}, {16, 16, 16, 32}, {24, 24, 24, 48}, {6, 2, 10, 4}};
  for (const auto& d : shapes)
    for (int prec = 0; prec < 3; ++prec)
      for (int Ls : {1, 16, 24})
        for (int cg : {0, 1, 2}) check_workspace(d, Ls, prec, cg == 2 ? 40 : 1, cg);
  const int small[][4] = {{2, 2, 2, 2}, {4, 4, 4, 8}, {8, 4, 4, 8}, {4, 8, 12, 16}, {6, 2, 10, 4}, {16, 16, 16, 32}};
  for (const auto& d : small) check_orders(d);
  const int boxed[][4] = {{16, 16, 16, 32}, {24, 24, 24, 8}, {8, 4, 4, 8}, {12, 6, 8, 4}, {2, 2, 2, 2}};
  for (const auto& d : boxed) check_box_orders(d);
  const int d1[4] = {8, 4, 4, 8};
  const int b_ok[][4] = {{2, 2, 2, 2}, {4, 2, 4, 2}, {4, 4, 4, 4}, {2, 1, 1, 1}, {1, 1, 1, 2}};
  for (const auto& b : b_ok) {
    check_blocks(d1, 4, b, false, true);
    check_blocks(d1, 4, b, true, true);
  }
  const int b_bad[][4] = {{3, 2, 2, 2}, {1, 1, 1, 1}, {0, 2, 2, 2}, {8, 4, 4, 8}};
  check_blocks(d1, 4, b_bad[0], false, false);  // does not divide
  check_blocks(d1, 4, b_bad[1], false, false);  // odd volume
  check_blocks(d1, 4, b_bad[2], false, false);  // zero extent
  check_blocks(d1, 8, b_bad[3], false, false);  // 512 even sites x Ls 8 > 1024
  if (g_fail) {
    std::printf("%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("all checks passed\n");
  return 0;
}
