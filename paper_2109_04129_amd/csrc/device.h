// Device side of the hps library: buffers, schedules and launches.
// Only host types appear here; the kernels live in device.hip.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "hps_internal.h"

namespace hps {

// One output tile of a grouped GEMM: C[r0:r0+32, c0:c0+32] of a block with
// m x n valid entries at C + c_off (column-major, leading dimension ldc),
// accumulated over terms [t_begin, t_end).
struct Tile {
  int64_t c_off;
  int32_t ldc, r0, c0, m, n, t_begin, t_end;
};

// c0 == TILE_PACKED marks a packed tile (the pipelined shapes 11 and 12 only,
// in the setup's Schur updates): rows r0 .. r0 + 31 of targets that share
// one row band (m rows, leading dimension ldc) and one term, whose A rows
// (terms[t_begin]; its b_off and ldb unused) multiply n <= 4 column blocks of
// up to 16 columns, one per wave.  Block w is terms[t_begin + 1 + w]: a_off =
// element offset of its first C column, b_off = of its first B column, ldb =
// B's leading dimension, lda = its valid columns (1..16), k = the term's k;
// t_end = t_begin + 1 + n, c_off unused.
constexpr int32_t TILE_PACKED = -2;

// One term op(A) B: A at a_off (column-major, lda), B at b_off (column-major,
// ldb), contraction length k; trans = 1 uses A^T (never the conjugate).
// sidx >= 0: A is a 16-bit far factor whose values are multiplied by
// scales[sidx] (precision form); -1 otherwise.
struct Term {
  int64_t a_off, b_off;
  int32_t lda, ldb, k, trans;
  int32_t sidx = -1, pad = 0;   // 16-bit A: scale index, or -2 for the per-row scale of the target's rows
};

// A batch of tiles for one launch: C = alpha * sum op(A) B + beta * C with
// mode 0: C = sum, 1: C -= sum, 2: C += sum.
struct GemmBatch {
  int mode = 0;
  int a_buf = 0, b_buf = 0, c_buf = 0;   // buffer ids (see DeviceState::buf)
  std::vector<Tile> tiles;
  std::vector<Term> terms;
  // device copies
  void *d_tiles = nullptr, *d_terms = nullptr;
  double flops = 0.0;                     // algorithmic, 8 per complex MAC
};

// Launch classes of the grouped GEMM whose tile shape is chosen by the
// tuning table (solve: sweeps, D^-1, far stages, near product; setup: Schur
// updates), and one entry of the table: `shape` for launches of class `cls`
// with at most rhs_max columns on a problem whose mean pivot size is at
// most group_max unknowns (and, when given, solve precision `precision`).
// Shapes 0-4: workgroup tiles of 32 rows x 32, 64, 64, 128, 128 columns
// (waves of 16 x 16, 16 x 32, 32 x 16, 32 x 32, 16 x 64); shape 5: 32 x 64
// with the operands staged in LDS, double-buffered (FP64; the FP32 kernels
// take shape 2 for it); shape 6: a vector-ALU matrix-vector kernel for
// one-column FP64 solves (any other launch takes shape 0 for it); shapes 7
// and 8: shapes 2 and 1 built for 3 waves per SIMD (FP64; FP32 takes 2, 1);
// shape 9: shape 0 built for 5 waves per SIMD (FP64; FP32 takes 0); shape
// 10: shape 3 built for 4 waves per SIMD (FP32; FP64 takes 3).  The FP64
// shape 0 itself is built for 4.  Shapes 11 and 12: the tile of shape 7 with
// every full 16-k chunk staged in LDS one chunk ahead by direct-to-LDS loads
// (FP64: 11 stages the target tile in LDS too, 12 fetches it after the
// products; FP32 launches with FP32 factors take the pipelined FP32 kernel
// for both, those with 16-bit factors take 2).
enum { TC_SWEEP = 0, TC_DINV, TC_FAR1, TC_FAR2, TC_NEAR, TC_SCHUR, TC_COUNT };
constexpr int TUNE_SHAPES = 13;
struct TuneEntry {
  int cls;
  int64_t rhs_max;
  double group_max;
  int shape;
  int precision = -1;     // solve arithmetic the entry applies to (0 FP64, 1-2 FP32); -1 any
};

// A tuning table: tile shapes per launch class, and the sweeps' pull
// threshold (the longest contraction a sweep target takes in one tile set;
// -1: the built-in value).
struct TuneTable {
  std::vector<TuneEntry> entries;
  int64_t sweep_pull_kmax = -1;
};

// Reads a tuning table (JSON, see tune.cpp); throws Error.
TuneTable read_tuning(const std::string &path);

struct StageTimes {
  double setup_ms = 0, inverse_ms = 0, coef_ms = 0, schur_ms = 0, symbolic_ms = 0;
  double solve_ms = 0, rhs_ms = 0, sweep_ms = 0, far_ms = 0, rcs_ms = 0;
};

class DeviceState {
 public:
  DeviceState(int device, void *stream);
  ~DeviceState();
  // nseg[P+1]: unknown offsets of the P independent problems of a batch
  // ({0, N} for one problem); outputs are laid out per problem.
  void upload(const Mesh &mesh, const HMatrix &H, const hps_params &p, const std::vector<int64_t> &nseg);
  void setup(const Plan &P, const HMatrix &H);         // throws Error
  int precision = 0;        // 0 FP64; 1 FP32 + BF16 far; 2 FP32 + FP16 far
  int refine = 0;           // residual-correction passes (precision form)
  int graphs = 1;           // replay the solve's device work from captured HIP graphs
  // RHS in elimination order into buffer `dst` (N x R), from plane waves.
  void solve_planewaves(int64_t R, const double *khat, const double *pol, void *X, double *rcs,
                        double *ratio);
  void solve_rhs(int64_t R, const void *B, void *X, double *ratio);
  void excitation(int64_t R, const double *khat, const double *pol, void *B);
  void hmatvec(int64_t R, const void *X, void *Y);
  // hmatvec with its work vectors in the fixed scratch array (no allocation)
  void hmatvec_noalloc(int64_t R, const void *X, void *Y);
  std::string stats_json() const;
  // EFIE entries of the near blocks of H (structure set, values sized) on the
  // device, copied into H.near_vals; synchronous.
  // cfie / alpha select the entries (EFIE, or the CFIE of eq. 8)
  void near_fill(const Mesh &m, double freq_hz, int cfie, double alpha, HMatrix &H);
  // Raw ACA factors of every far block of H (far_rng set), chunk by chunk
  // to emit, see FarChunk.
  void far_sample(const Mesh &m, double freq_hz, int cfie, double alpha, const HMatrix &H, double eps,
                  const FarEmit &emit);
  void set_profiling(bool on);
  // tile-shape table (applies from the next hps_setup / solve) and where it came from
  void set_tuning(const TuneTable &t, const std::string &src);
  TuneTable tune;
  std::string tune_src = "built-in (all 32 x 32)";

  int device;
  void *stream;     // hipStream_t
  bool own_stream;
  StageTimes times;
  int terms = 2;
  double last_solve_flops = 0.0;
  // setup schedule: ms until every level was built, ms the launching thread
  // waited for builds, ms it spent staging and enqueueing, tiles, terms, and
  // the Schur tiles' 16-column block slots x 16-k chunks, all and used
  double sched_split[7] = {0, 0, 0, 0, 0, 0, 0};

  struct Impl;
  std::unique_ptr<Impl> impl;
};

}  // namespace hps
