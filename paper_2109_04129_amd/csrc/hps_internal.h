// Internal host-side structures of the hps library (not part of the ABI).
#pragma once

#include <complex>
#include <functional>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hps.h"

namespace hps {

using cplx = std::complex<double>;

struct Error {
  hps_status code;
  std::string msg;
};

// ---------------------------------------------------------------- mesh / RWG
struct Mesh {
  std::vector<double> xyz;     // nv * 3
  std::vector<int32_t> tri;    // nt * 3
  int64_t nv = 0, nt = 0;
  // per triangle
  std::vector<double> cen;     // nt * 3, (v0 + v1 + v2) / 3
  std::vector<double> area;    // nt
  std::vector<double> nrm;     // nt * 3, unit normal from the vertex order (outward if counter-clockwise)
  double hmax = 0.0;           // longest edge
  bool open = false;           // built with rim edges allowed (open sheet)
  // per RWG unknown (RWG order)
  int64_t N = 0;
  std::vector<int32_t> edge;   // N * 2 (min, max vertex)
  std::vector<int32_t> tp, tm; // T+, T-
  std::vector<int32_t> vp, vm; // free vertices
  std::vector<double> len;     // edge length
};

// Validates and builds the RWG functions; throws Error on bad meshes.  With
// allow_open, edges of one triangle (the rim of an open sheet) are accepted
// and carry no unknown.
void build_rwg(Mesh &m, bool allow_open = false);

// ---------------------------------------------------------------- octree
struct TreeNode {
  int depth;
  int64_t ijk[3];
  int64_t lo, hi;              // range in tree order
  int32_t first_child = -1, n_child = 0;
  int32_t leaf = -1;           // leaf (group) ordinal or -1
};

struct Tree {
  std::vector<TreeNode> nodes; // depth-first preorder; children contiguous by construction
  std::vector<int32_t> child;  // child node ids per node (first_child indexes here)
  std::vector<int64_t> perm;   // tree position -> RWG index
  std::vector<int32_t> leaf_node;
};

// box_min > 0: cells narrower than box_min (metres) are never created.
void build_tree(const Mesh &m, int leaf_max, double box_min, Tree &t);
bool cells_touch(const TreeNode &a, const TreeNode &b);
// eq. (10): eta dist >= min(dia) for the two cells
bool admissible(const TreeNode &a, const TreeNode &b, double eta);
void block_partition(const Tree &t, double eta, std::vector<std::pair<int32_t, int32_t>> &near_leaves,
                     std::vector<std::pair<int32_t, int32_t>> &far_nodes);

// ---------------------------------------------------------------- H-matrix (host copy)
struct HMatrix {
  int64_t N = 0, M = 0;
  // false: symmetric (EFIE), near blocks t <= s, far blocks applied both ways.
  // true (CFIE): every ordered near pair, every far block one way only.
  bool nonsym = false;
  std::vector<int64_t> perm;          // tree position -> RWG
  std::vector<int64_t> gptr;          // M + 1
  std::vector<int32_t> near_ts;       // 2 * n_near, t <= s unless nonsym
  std::vector<int64_t> near_off;      // n_near + 1
  std::vector<cplx> near_vals;        // row-major blocks
  std::vector<int64_t> far_rng;       // 4 * n_far
  std::vector<int32_t> far_rank;
  std::vector<int64_t> far_off;       // n_far + 1, U then V column-major
  std::vector<cplx> far_uv;
  int64_t n_near() const { return (int64_t)near_ts.size() / 2; }
  int64_t n_far() const { return (int64_t)far_rank.size(); }
};

// Entries of the Galerkin matrix: the EFIE (symmetric by construction) or,
// with cfie, alpha EFIE + eta0 (1 - alpha) MFIE (eq. 8, not symmetric).
struct Galerkin {
  const Mesh *mesh;
  double k, omega, h;
  cplx cA, cPhi;
  bool cfie = false;
  double alpha = 1.0;
  Galerkin(const Mesh &m, double freq_hz, bool cfie_ = false, double alpha_ = 1.0);
  cplx entry(int64_t m, int64_t n) const;
  cplx efie_entry(int64_t m, int64_t n) const;
  cplx mfie_entry(int64_t m, int64_t n) const;
  // Z[rows[i], cols[j]] into out (row-major rows x cols)
  void block(const int64_t *rows, int64_t nr, const int64_t *cols, int64_t nc, cplx *out) const;
};

// Re-compressed ACA of one admissible block; U (m x r) and V (n x r)
// column-major with block ~= U V^T.
void aca_block(const Galerkin &op, const int64_t *rows, int64_t m, const int64_t *cols, int64_t n,
               double eps, std::vector<cplx> &U, std::vector<cplx> &V, int &rank);

// Fills H.near_vals (sized from H.near_off) from the near block list of H;
// called on its own host thread while the far blocks are compressed.
using NearFill = std::function<void(HMatrix &H)>;

// Unrecompressed ACA factors of the far blocks [b0, b1): block b has
// rank[b - b0] terms (U m x k then V n x k, column-major, at
// uv[off[b - b0]]), or rank -1 when it is left to the host ACA (rank limit,
// term cap).
struct FarChunk {
  int64_t b0 = 0, b1 = 0;
  bool final = false;     // true: factors already recompressed (rank = final rank)
  std::vector<int32_t> rank;
  std::vector<int64_t> off;
  std::vector<cplx> uv;
};
using FarEmit = std::function<void(FarChunk &&chunk)>;
// Hands every far block of H (far_rng set) to emit, in chunks of increasing
// block index.
using FarSample = std::function<void(const HMatrix &H, const FarEmit &emit)>;

// With near_fill / far_sample the ACA sampling of the far blocks and then the
// near blocks run there (the device, on one host thread, in that order); host
// threads recompress each chunk of far blocks as it arrives.  Without them
// everything runs on host threads.
void build_hmatrix(const Mesh &mesh, const hps_params &p, HMatrix &H, const NearFill *near_fill = nullptr,
                   const FarSample *far_sample = nullptr);

// Small dense complex linear algebra used by the ACA recompression.
void householder_qr(int64_t m, int64_t n, cplx *A /* m x n col-major, in/out */,
                    std::vector<cplx> &Q /* m x k */, std::vector<cplx> &R /* k x n */, int64_t &k);
// T_U, T_V (k x r, column-major) of the recompressed factors U T_U, V T_V of a
// block U V^T, from G_U = U^H U and G_V = V^H V (k x k, column-major); r by
// the recompression's truncation rule at eps.
void recompress_from_grams(int64_t k, const cplx *GU, const cplx *GV, double eps, std::vector<cplx> &TU,
                           std::vector<cplx> &TV, int &rank);
void jacobi_svd(int64_t n, const cplx *A /* n x n col-major */, std::vector<cplx> &W,
                std::vector<double> &s, std::vector<cplx> &Y);  // A = W diag(s) Y^H, s descending

// ---------------------------------------------------------------- symbolic plan
struct Plan {
  int64_t M = 0, N = 0;
  std::vector<int32_t> order;        // elimination index -> group
  std::vector<int32_t> pos;          // group -> elimination index
  std::vector<int64_t> size;         // per elimination index: n_e
  std::vector<int64_t> uoff;         // per elimination index: first unknown (elimination order)
  std::vector<int64_t> later_ptr;    // CSR: N+(e) over elimination indices (sorted)
  std::vector<int32_t> later;
  std::vector<int64_t> col_off;      // per CSR entry: column offset of block (e, f) in panel e
  std::vector<int64_t> width;        // panel width W_e = n_e + sum n_f
  std::vector<int64_t> panel_off;    // element offset of panel e (n_e x W_e column-major)
  int64_t panel_elems = 0;
  std::vector<int32_t> level;        // etree level per elimination index
  int32_t n_levels = 0;
  std::vector<int64_t> level_ptr;    // pivots grouped by level
  std::vector<int32_t> level_piv;
  int64_t n_upper_blocks = 0, n_U = 0, n_D = 0;
  double setup_flops = 0.0;          // algorithmic (8 flops per complex MAC)
};

// gseg[P+1]: the groups of problem p are [gseg[p], gseg[p+1]) (one entry pair
// {0, M} for a single problem).  Each problem is ordered on its own and the
// problems follow each other, so every problem owns a contiguous range of
// elimination positions; the elimination-tree levels are shared.
void make_plan(const HMatrix &H, const Mesh &mesh, int ordering, const std::vector<int64_t> &gseg, Plan &P);

// ---------------------------------------------------------------- batches
// Several independent problems as one block-diagonal system: vertices,
// triangles, RWG unknowns, tree positions and groups of problem p follow
// those of problems 0..p-1, and no near or far block couples two problems.
// nseg[P+1] / gseg[P+1] receive the unknown / group offsets.
void merge_problems(const std::vector<Mesh> &meshes, const std::vector<HMatrix> &Hs, Mesh &mesh, HMatrix &H,
                    std::vector<int64_t> &nseg, std::vector<int64_t> &gseg);

// Cut groups larger than max_size unknowns into consecutive sub-groups
// (near blocks cut to match, far blocks unchanged).
void split_groups(HMatrix &H, int64_t max_size);
constexpr int64_t kMaxPivot = 128;   // largest pivot block of the setup kernels

}  // namespace hps
