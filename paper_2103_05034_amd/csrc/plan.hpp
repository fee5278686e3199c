// Host-side planning behind the entry points: argument checks, the layout of
// a handle's workspace, the site traversal orders of the hop kernels and the
// host arithmetic of the Cholesky QR.
// Plain C++17 with no HIP dependency, so the same source also builds into a
// host-only test program under AddressSanitizer and UBSan.
#pragma once

#include <cstddef>
#include <string>
#include <vector>

#include "dwf.h"

namespace dwf {

constexpr size_t WS_ALIGN = 256;  // alignment of every carved buffer (and of the workspace)
constexpr int NSCAL = 16;         // device scalars per rhs
constexpr int RED_BLOCKS = 1024;  // reduction partial sums per rhs
constexpr int GS_MAX = 256;       // most vectors one Gram-Schmidt call orthonormalises

// Bytes of one packed 5D spinor (12 complex components) per storage
// precision: FP64 complex, FP32 complex, 24 FP16 values plus one FP32 scale.
constexpr size_t SPINOR_BYTES[3] = {192, 96, 52};

namespace plan {

// Checks the lattice and capacity arguments of dwf_create and its sizing
// calls; on failure fills *why with the reason.
bool valid_dims(const int dims[4], int Ls, int prec, int max_nrhs, int max_cg_rhs, std::string* why);

// The buffers carved out of a handle's workspace, in carving order.
enum Buffer {
  B_LINKS64,      // [2][8][9][V4h] complex128
  B_LINKS32,      // [2][8][9][V4h] complex64 (handles below FP64)
  B_NBR,          // [2][8][V4h] int
  B_T,            // odd half field x chunk, handle precision
  B_U,            // even half field x chunk, handle precision
  B_CHEB,         // Chebyshev partner set, max(max_nrhs, 2) rhs
  B_R64,          // FP64 CG vectors (max_cg_rhs > 0)
  B_P64,
  B_Q64,
  B_B64,
  B_DIR64,        // two more FP64 search directions per CG rhs (FP64 handles): x is
                  // updated once per four iterations from the last four directions
  B_T64,          // FP64 temporaries of low-precision handles
  B_U64,
  B_LO_R,         // FP32 CG vectors of low-precision handles
  B_LO_X,
  B_LO_P,         // handle-precision search direction and product
  B_LO_Q,
  B_ORDER,        // [2][V4h] int
  B_BSITE,        // [2][V4h] int
  B_BNBR,         // [8][V4h] int
  B_HOP_PARTIALS, // [max_cg_rhs][V4h] double
  B_PARTIALS,     // [chunk][RED_BLOCKS][2] double
  B_SCALARS,      // [chunk][NSCAL] double
  B_COEF,         // [4 GS_MAX + 8] double
  B_COUNTERS,     // [chunk] unsigned: completion counts of the per-site reductions
  B_COUNT
};

constexpr size_t ABSENT = (size_t)-1;

struct Workspace {
  size_t offset[B_COUNT];  // byte offset of each buffer, or ABSENT
  size_t bytes[B_COUNT];   // bytes asked for (0 when absent)
  size_t total;            // workspace bytes, a multiple of WS_ALIGN
  int chunk;               // rhs capacity of the temporaries: max(max_nrhs, max_cg_rhs)
};

// Layout for arguments that passed valid_dims.  FP64 handles alias their
// FP64 temporaries to B_T / B_U (B_T64 / B_U64 absent).
Workspace plan_workspace(const int dims[4], int Ls, int prec, int max_nrhs, int max_cg_rhs);

// Half-lattice index of the site (x, y, z, t): its lexicographic index
// (x fastest) halved.
inline long long half_index(int X, int Y, int Z, int x, int y, int z, int t) {
  return ((long long)x + (long long)X * (y + (long long)Y * (z + (long long)Z * t))) / 2;
}

// Site traversal order of the hop kernels for each parity, [2][V4h]: mode 1
// cuts the (x, y, z) box into 2 x 2 x 2 sub-boxes, one per XCD, each streamed
// with t slowest; mode 2 cuts t into eight slabs, one per XCD, each streamed
// with t fastest, then x, z, y.  Returns false when the lattice does not admit
// the mode (mode 0, lexicographic, needs no table).
bool build_order(int X, int Y, int Z, int T, int mode, std::vector<int>& ord);

// Traversal order in boxes: the (x, y, z) volume cut into nx x ny x nz equal
// boxes (x extent even), numbered x fastest and dealt to the XCDs in
// contiguous groups (XCD k runs the k-th eighth of the order); inside a box
// the sites run with t slowest, then z, y, x.  nx = 1 keeps whole x rows, so a
// workgroup's ±x neighbours stay inside its row; (2, 2, 2) is mode 1.  Returns
// false when the cut does not divide the lattice.
bool build_box_order(int X, int Y, int Z, int T, int nx, int ny, int nz, std::vector<int>& ord);

// The box cuts the autotuner times (besides modes 0 and 2), in order; those a
// lattice does not admit are skipped.
constexpr int BOX_CANDIDATES[][3] = {{2, 2, 2}, {1, 2, 4}, {1, 4, 2}, {1, 4, 4}, {1, 2, 8}, {1, 4, 8},
                                     {1, 3, 8}, {1, 6, 4}, {1, 6, 8}, {1, 8, 1}, {1, 8, 8}};
constexpr int NUM_BOX_CANDIDATES = sizeof(BOX_CANDIDATES) / sizeof(BOX_CANDIDATES[0]);

// Coarse-space blocks of extents block[4] over the lattice: `sites` gets, per
// block (numbered x fastest), its sites in lexicographic order (even sites
// only, as half-lattice indices, unless `both`; with `both`, odd sites as
// V4h + their half index), `nbrs` the neighbouring block in each of the 8 hop
// directions (2 mu forward, 2 mu + 1 backward).  Returns false with *why set
// when the extents do not tile the lattice into blocks of equal even and odd
// counts holding at most 1024 5D sites.
bool build_blocks(int X, int Y, int Z, int T, int Ls, const int block[4], bool both, std::vector<int>& sites,
                  std::vector<int>& nbrs, int* nblocks, int* sites_per_block, std::string* why);

// Launch shapes found by the autotuner, kept per (GPU architecture, lattice,
// Ls, rhs count, precision, traversal order or "tuned", occupancy cap, Schur form) for
// the life of the process and, when a file path is given, in that file (one
// entry per line, appended as found; lines that do not parse are skipped).
struct TuneKey {
  std::string arch;  // the device's architecture name, without spaces
  int dims[4];
  int Ls, nrhs, prec;
  int order;  // -1: the traversal order is tuned too; else the code of the order the caller set
  int lds_floor, schur_form;
};
struct TuneEntry {
  int spb, depth, rpb;
  int order;      // traversal order mode chosen (0, 1, 2, or 3 for boxes)
  int box[3];     // the box cut of order 3
  double ms;      // time per M_pc^dag M_pc measured when the shape was tuned
};
std::string format_tune_line(const TuneKey& k, const TuneEntry& e);
bool parse_tune_line(const std::string& line, TuneKey* k, TuneEntry* e);
// Looks the key up in the process cache, first loading the file at `path`
// (null or empty: none) if it has not been read yet.
bool tune_lookup(const TuneKey& k, TuneEntry* e, const char* path);
// Records an entry in the process cache and appends it to the file at `path`.
void tune_store(const TuneKey& k, const TuneEntry& e, const char* path);
// Empties the process cache; the file is left as it is and read again on the
// next lookup.
void tune_clear();

// Host side of the Cholesky QR of dwf_gram_schmidt.  Complex n x n matrices as
// interleaved (re, im) doubles, row-major.  From the lower triangle of a Gram
// matrix, G[k][j] = <v_j, v_k> for j <= k, the upper R with G = R^dag R and a real
// positive diagonal; false when a pivot is not above min_ratio times its diagonal
// entry of G (or is not finite).
bool cholesky_upper(const std::vector<double>& G, int n, std::vector<double>& R, double min_ratio);
// W = R^{-1} for upper triangular R with a real positive diagonal.
void invert_upper(const std::vector<double>& R, int n, std::vector<double>& W);
// C = A B for upper triangular A and B.
void multiply_upper(const std::vector<double>& A, const std::vector<double>& B, int n, std::vector<double>& C);

}  // namespace plan
}  // namespace dwf
