// HIP kernels and device schedules for gfx950 (CDNA4, wave64).
//
// Setup (Sec. III.A, eqs. 16-23), level by level of the elimination tree:
//   k_inverse   Gauss-Jordan inverse with partial pivoting of each scaled
//               diagonal block D_e = Z~_ee (held in registers, one block per
//               workgroup);
//   k_gemm      C_eN = D_e^-1 Z~_eN (the right scaling coefficients) and the
//               Schur updates Z~_jk -= Z~_ej^T C_ek (eq. 21, incl. fill-in).
// Solve (eqs. 25-36): plane-wave RHS, forward sweep with C^T (eq. 25), D^-1
// (eq. 32), back sweep with C (eq. 26), far field U (V^T x) in both
// directions, ratio of eq. (45), combination of the series terms, RCS.
//
// Every contraction goes through one grouped complex GEMM kernel driven by
// host-built tile and term lists, so each output tile is owned by exactly one
// workgroup and sums its terms in a fixed order (deterministic, no atomics).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <type_traits>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <sstream>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>

#include "device.h"

#define HIP_CHECK(x)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess)                                                                 \
      throw ::hps::Error{HPS_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)};   \
  } while (0)

namespace hps {

typedef double2 c2;

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ c2 cmul(c2 a, c2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ void cmac(c2 &acc, c2 a, c2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
__device__ __forceinline__ c2 cinv(c2 a) {
  const double r = 1.0 / (a.x * a.x + a.y * a.y);
  return make_double2(a.x * r, -a.y * r);
}

// ------------------------------------------------------------------ grouped GEMM
// Complex FP64 on the matrix cores: a workgroup of 4 waves owns a tile of 32
// rows and TN columns and accumulates op(A) B with V_MFMA_F64_16X16X4_F64 in
// the real 3M split (Gauss: Ar Br, Ai Bi and (Ar + Ai)(Br + Bi) in three
// accumulators; re = rr - ii, im = ss - rr - ii), three products per complex
// step instead of four.  Tile shape (template WR, NB): WR waves along the 32
// rows (WR = 2: a wave takes 16 rows; WR = 1: a wave takes all 32 as two
// 16-row blocks, so one B fragment serves two MFMA rows) and 4 / WR waves
// along the columns, NB column blocks of 16 each; TN = 16 NB (4 / WR).
// Operand layout of the instruction: lane l supplies A[l % 16][k slot l / 16]
// and B[k slot l / 16][l % 16]; result register r of lane l is
// D[l / 16 + 4 r][l % 16].  In step s of a chunk of 16 the lane groups take
// k = k0 + 4 s + l / 16, so one load instruction reads four consecutive
// elements of each of 16 rows (A) or columns (B).  Operands come straight
// from L2; the read-modify-write modes of the multi-wave builds stage their
// C sub-tile in LDS (below).  The tile shape of each launch class is a run-time choice
// (a tuning table written by the autotuner); every shape gives bitwise the
// same result (each output element sums the same products in the same order).
// WPE > 1 builds the kernel for at least WPE waves per SIMD (registers capped
// accordingly; the C tile of the read-modify-write modes then goes through
// LDS instead of registers).
constexpr int TM = 32;
constexpr int SUB_Y = 16;     // workgroups per whole-block tile (each loops over its share of sub-tiles)
typedef double d4 __attribute__((ext_vector_type(4)));

// tile shapes: (WR, NB) and the workgroup tile's column count
static_assert(TUNE_SHAPES == 13, "tile shapes 0-12");
__host__ __device__ constexpr int shape_wr(int v) {
  return v == 2 || v == 3 || v == 5 || v == 7 || v == 10 || v == 11 || v == 12 ? 1 : 2;
}
__host__ __device__ constexpr int shape_nb(int v) { return v == 1 || v == 3 || v == 8 || v == 10 ? 2 : (v == 4 ? 4 : 1); }
__host__ __device__ constexpr int shape_tn(int v) { return 16 * shape_nb(v) * (4 / shape_wr(v)); }

template <int MODE, int WR, int NB, int WPE = 1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_gemm(const c2 *__restrict__ A, const c2 *__restrict__ B,
                                              c2 *__restrict__ C, const Tile *__restrict__ tiles,
                                              const Term *__restrict__ terms, int ncols, int ntiles, int ny,
                                              int xcd_order) {
  constexpr int RB = 2 / WR;           // 16-row blocks per wave
  constexpr int WC = 4 / WR;           // waves along the columns
  constexpr int TN = 16 * NB * WC;
  // Workgroup -> (tile bx, part by).  Plain order: grid (ntiles, ny), tile
  // = blockIdx.x.  XCD-aware order: a one-dimensional grid of
  // 8 ceil(ntiles / 8) ny workgroups; consecutive workgroups go to the 8
  // XCDs in turn, so workgroup w takes tile 8 (q / ny) + w % 8 and part
  // q % ny, q = w / 8: the ny workgroups of one tile (the RHS column tiles
  // of a solve, which read the same factor rows) run one after another on
  // one XCD and share its L2.
  int bx = (int)blockIdx.x, by = (int)blockIdx.y;
  if (xcd_order) {
    const int q = (int)(blockIdx.x >> 3);
    by = q % ny;
    bx = 8 * (q / ny) + (int)(blockIdx.x & 7);
    if (bx >= ntiles) return;
  }
  const Tile t = tiles[bx];
  // r0 < 0: the tile stands for the whole m x n block; workgroup y takes its
  // sub-tiles y, y + ny, ...  c0 < 0: one row tile over ncols columns, y
  // picks the column tile.  Else one explicit tile (TN = 32 shapes only).
  int rb0 = t.r0, cb0 = t.c0, tn = t.n, nsub = 1, nsc = 1, st0 = 0, sstep = 1;
  if (t.r0 < 0) {
    nsc = (t.n + TN - 1) / TN;
    nsub = ((t.m + TM - 1) / TM) * nsc;
    st0 = by;
    sstep = ny;
  } else if (t.c0 < 0) {
    tn = ncols;
    cb0 = by * TN;
    if (cb0 >= tn) return;
  } else if (by > 0) {
    return;
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int li = lane & 15, lg = lane >> 4;
  const int wr = WR == 2 ? (wave >> 1) : 0, wc = WR == 2 ? (wave & 1) : wave;
  // The read-modify-write modes built for several waves per SIMD stage the
  // wave's C sub-tile (16 RB rows x 16 NB columns) in LDS with direct-to-LDS
  // loads issued before the products, so its latency hides behind them with
  // no registers held, and read it back after them.  Load q of the wave
  // fills slots 64 q .. 64 q + 63, lane l slot 64 q + l; element (c, r) of
  // the sub-tile sits at slot c RW + (r + 2 c) mod RW (the rotation spreads
  // the read-back of one row over the banks).
  constexpr bool LDS_C = MODE != 0 && WPE > 1;
  constexpr int RW = 16 * RB, CW = 16 * NB, NQ = RW * CW / 64;
  __shared__ c2 cbuf[LDS_C ? 4 * RW * CW : 1];
  c2 *const cw = cbuf + (LDS_C ? wave * RW * CW : 0);
  for (int st = st0; st < nsub; st += sstep) {
    int rb = rb0, cb = cb0;
    if (t.r0 < 0) {
      rb = (st / nsc) * TM;
      cb = (st % nsc) * TN;
    }
    const int row0 = rb + 16 * RB * wr, col0 = cb + 16 * NB * wc;
    if (row0 >= t.m || col0 >= tn) continue;           // wave-uniform
    bool arow_ok[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) arow_ok[i] = row0 + 16 * i + li < t.m;
    // a wave of two 16-row blocks whose second block lies wholly past the
    // target's edge computes the first only (wave-uniform choice)
    const bool one_rb = RB > 1 && row0 + 16 >= t.m;
    // read-modify-write modes: fetch C now, so its latency hides behind the
    // products (after them when the kernel is built for more waves per SIMD:
    // fewer registers live through the products)
    c2 cold[RB][NB][4];
    auto fetch_c = [&]() {
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const int ccol = col0 + 16 * j + li;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int crow = row0 + 16 * i + lg + 4 * r;
            cold[i][j][r] = make_double2(0.0, 0.0);
            if (ccol < tn && crow < t.m) cold[i][j][r] = C[t.c_off + (int64_t)ccol * t.ldc + crow];
          }
        }
    };
    if (MODE != 0 && WPE == 1) fetch_c();
    if constexpr (LDS_C) {
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");    // the previous sub-tile's read-back is done
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int e = 64 * q + lane, c = e / RW, r = (e - c * RW - 2 * c) & (RW - 1);
        const int ccol = col0 + c, crow = row0 + r;
        if (ccol < tn && crow < t.m)
          __builtin_amdgcn_global_load_lds((const void *)(C + t.c_off + (int64_t)ccol * t.ldc + crow),
                                           (__attribute__((address_space(3))) void *)(cw + 64 * q), 16, 0, 0);
      }
    }
    d4 rr[RB][NB], ii[RB][NB], ss[RB][NB];      // 3M: Ar Br, Ai Bi, (Ar + Ai)(Br + Bi)
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) rr[i][j] = ii[i][j] = ss[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    auto products = [&](auto rbe) {
      constexpr int RBE = decltype(rbe)::value;
      for (int q = t.t_begin; q < t.t_end; ++q) {
        const Term tm = terms[q];
        const c2 *Ab = A + tm.a_off;
        // full chunks of 16: in step s lane group g reads k = k0 + 4 s + g
        const int kfull = tm.k & ~15;
        for (int k0 = 0; k0 < kfull; k0 += 16) {
          c2 av[RB][4], bv[NB][4];
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int k = k0 + 4 * s + lg;
#pragma unroll
            for (int i = 0; i < RBE; ++i) {
              const int arow = row0 + 16 * i + li;
              av[i][s] = make_double2(0.0, 0.0);
              if (arow_ok[i]) av[i][s] = tm.trans ? Ab[(int64_t)arow * tm.lda + k] : Ab[(int64_t)k * tm.lda + arow];
            }
#pragma unroll
            for (int j = 0; j < NB; ++j) {
              const int bcol = col0 + 16 * j + li;
              bv[j][s] = make_double2(0.0, 0.0);
              if (bcol < tn) bv[j][s] = B[tm.b_off + (int64_t)bcol * tm.ldb + k];
            }
          }
#pragma unroll
          for (int s = 0; s < 4; ++s) {
#pragma unroll
            for (int j = 0; j < NB; ++j) {
              const double bs = bv[j][s].x + bv[j][s].y;
#pragma unroll
              for (int i = 0; i < RBE; ++i) {
                rr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][s].x, bv[j][s].x, rr[i][j], 0, 0, 0);
                ii[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][s].y, bv[j][s].y, ii[i][j], 0, 0, 0);
                ss[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][s].x + av[i][s].y, bs, ss[i][j], 0, 0, 0);
              }
            }
          }
        }
        // tail (k % 16): steps of 4, lane group g takes k = kt + g; empty steps skipped
        for (int kt = kfull; kt < tm.k; kt += 4) {
          const int k = kt + lg;
          const bool kok = k < tm.k;
          c2 av[RB];
#pragma unroll
          for (int i = 0; i < RBE; ++i) {
            const int arow = row0 + 16 * i + li;
            av[i] = make_double2(0.0, 0.0);
            if (kok && arow_ok[i]) av[i] = tm.trans ? Ab[(int64_t)arow * tm.lda + k] : Ab[(int64_t)k * tm.lda + arow];
          }
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            const int bcol = col0 + 16 * j + li;
            c2 bv = make_double2(0.0, 0.0);
            if (kok && bcol < tn) bv = B[tm.b_off + (int64_t)bcol * tm.ldb + k];
#pragma unroll
            for (int i = 0; i < RBE; ++i) {
              rr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, bv.x, rr[i][j], 0, 0, 0);
              ii[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].y, bv.y, ii[i][j], 0, 0, 0);
              ss[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x + av[i].y, bv.x + bv.y, ss[i][j], 0, 0, 0);
            }
          }
        }
      }
    };
    if (one_rb)
      products(std::integral_constant<int, 1>{});
    else
      products(std::integral_constant<int, RB>{});
    if constexpr (LDS_C) {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");      // the staged C sub-tile has landed
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int c = 16 * j + li, rw = 16 * i + lg + 4 * r;
            cold[i][j][r] = cw[c * RW + ((rw + 2 * c) & (RW - 1))];
          }
    } else if (MODE != 0 && WPE > 1) {
      fetch_c();
    }
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int ccol = col0 + 16 * j + li;
        if (ccol >= tn) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int crow = row0 + 16 * i + lg + 4 * r;
          if (crow >= t.m) continue;
          const c2 acc = make_double2(rr[i][j][r] - ii[i][j][r], ss[i][j][r] - rr[i][j][r] - ii[i][j][r]);
          c2 *p = C + t.c_off + (int64_t)ccol * t.ldc + crow;
          if (MODE == 0) {
            *p = acc;
          } else if (MODE == 1) {
            *p = make_double2(cold[i][j][r].x - acc.x, cold[i][j][r].y - acc.y);
          } else {
            *p = make_double2(cold[i][j][r].x + acc.x, cold[i][j][r].y + acc.y);
          }
        }
      }
  }
}

// LDS-staged variant (tile shape 5): a workgroup tile of 32 rows x 64
// columns, waves 1 x 4 (each 32 rows x 16 columns).  Per chunk of 16 k the
// 256 threads stage A (32 x 16) and B (16 x 64) in LDS with coalesced loads
// (A column-major: along the rows; A^T and B: along k), double-buffered: the
// next chunk's global loads are in flight while the waves run the current
// chunk's MFMAs from LDS, one barrier per chunk.  A is read from L2 once per
// workgroup instead of once per wave.  Each output element sums the same
// products in the same order as k_gemm (steps k0 + 4 s + l / 16, zero
// operands past k), so the results are bitwise those of the other shapes.
// Every wave takes part in the loads and barriers, also where its columns
// lie past the block; only the stores are masked.
template <int MODE>
__global__ __launch_bounds__(256) void k_gemm_lds(const c2 *__restrict__ A, const c2 *__restrict__ B,
                                                  c2 *__restrict__ C, const Tile *__restrict__ tiles,
                                                  const Term *__restrict__ terms, int ncols, int ntiles, int ny,
                                                  int xcd_order) {
  constexpr int TN = 64, KC = 16, AP = TM + 1, BP = KC + 1;   // LDS row pitches (c2), padded
  __shared__ c2 sA[2][KC * AP];        // [k][row]
  __shared__ c2 sB[2][TN * BP];        // [col][k]
  int bx = (int)blockIdx.x, by = (int)blockIdx.y;
  if (xcd_order) {
    const int q = (int)(blockIdx.x >> 3);
    by = q % ny;
    bx = 8 * (q / ny) + (int)(blockIdx.x & 7);
    if (bx >= ntiles) return;            // whole workgroup: uniform
  }
  const Tile t = tiles[bx];
  int rb0 = t.r0, cb0 = t.c0, tn = t.n, nsub = 1, nsc = 1, st0 = 0, sstep = 1;
  if (t.r0 < 0) {
    nsc = (t.n + TN - 1) / TN;
    nsub = ((t.m + TM - 1) / TM) * nsc;
    st0 = by;
    sstep = ny;
  } else if (t.c0 < 0) {
    tn = ncols;
    cb0 = by * TN;
    if (cb0 >= tn) return;
  } else if (by > 0) {
    return;
  }
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lg = lane >> 4;
  for (int st = st0; st < nsub; st += sstep) {
    int rb = rb0, cb = cb0;
    if (t.r0 < 0) {
      rb = (st / nsc) * TM;
      cb = (st % nsc) * TN;
    }
    const int col0 = cb + 16 * wave;                 // this wave's 16 columns
    c2 cold[2][4];
    if (MODE != 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int crow = rb + 16 * i + lg + 4 * r, ccol = col0 + li;
          cold[i][r] = make_double2(0.0, 0.0);
          if (ccol < tn && crow < t.m) cold[i][r] = C[t.c_off + (int64_t)ccol * t.ldc + crow];
        }
    }
    d4 rr[2], ii[2], ss[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) rr[i] = ii[i] = ss[i] = d4{0.0, 0.0, 0.0, 0.0};
    // chunk cursor: term q, first k k0 (terms with k = 0 contribute nothing)
    int q = t.t_begin, k0 = 0;
    while (q < t.t_end && terms[q].k <= 0) ++q;
    c2 ra[2], rbv[4];                                  // staged global loads of one chunk
    auto gload = [&](int qq, int kk0) {
      const Term tm = terms[qq];
      const c2 *Ab = A + tm.a_off;
      if (tm.trans) {                                  // A^T[row][k] = Ab[row lda + k]: along k
        const int kk = tid & 15, row = tid >> 4;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int rr_ = rb + row + 16 * h, k = kk0 + kk;
          ra[h] = (rr_ < t.m && k < tm.k) ? Ab[(int64_t)rr_ * tm.lda + k] : make_double2(0.0, 0.0);
        }
      } else {                                         // A[row][k] = Ab[k lda + row]: along the rows
        const int row = tid & 31, kk = tid >> 5;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int rr_ = rb + row, k = kk0 + kk + 8 * h;
          ra[h] = (rr_ < t.m && k < tm.k) ? Ab[(int64_t)k * tm.lda + rr_] : make_double2(0.0, 0.0);
        }
      }
      const int kk = tid & 15, cl = tid >> 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = cb + cl + 16 * j, k = kk0 + kk;
        rbv[j] = (col < tn && k < tm.k) ? B[tm.b_off + (int64_t)col * tm.ldb + k] : make_double2(0.0, 0.0);
      }
    };
    auto lstore = [&](int buf, int trans) {
      if (trans) {
        const int kk = tid & 15, row = tid >> 4;
        sA[buf][kk * AP + row] = ra[0];
        sA[buf][kk * AP + row + 16] = ra[1];
      } else {
        const int row = tid & 31, kk = tid >> 5;
        sA[buf][kk * AP + row] = ra[0];
        sA[buf][(kk + 8) * AP + row] = ra[1];
      }
      const int kk = tid & 15, cl = tid >> 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) sB[buf][(cl + 16 * j) * BP + kk] = rbv[j];
    };
    int buf = 0;
    if (q < t.t_end) {
      gload(q, 0);
      lstore(0, terms[q].trans);
    }
    __syncthreads();
    while (q < t.t_end) {
      // next chunk
      int nq = q, nk0 = k0 + KC;
      if (nk0 >= terms[q].k) {
        nk0 = 0;
        ++nq;
        while (nq < t.t_end && terms[nq].k <= 0) ++nq;
      }
      const bool more = nq < t.t_end;
      if (more) gload(nq, nk0);                        // in flight during the products
      const c2 *pa = sA[buf], *pb = sB[buf];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = 4 * s + lg;
        const c2 bv = pb[(16 * wave + li) * BP + kk];
        const double bs = bv.x + bv.y;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const c2 av = pa[kk * AP + 16 * i + li];
          rr[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x, bv.x, rr[i], 0, 0, 0);
          ii[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.y, bv.y, ii[i], 0, 0, 0);
          ss[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av.x + av.y, bs, ss[i], 0, 0, 0);
        }
      }
      if (more) lstore(buf ^ 1, terms[nq].trans);
      __syncthreads();
      buf ^= 1;
      q = nq;
      k0 = nk0;
    }
    // the next sub-tile's first stores must not overwrite LDS still being read
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ccol = col0 + li;
      if (ccol >= tn) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int crow = rb + 16 * i + lg + 4 * r;
        if (crow >= t.m) continue;
        const c2 acc = make_double2(rr[i][r] - ii[i][r], ss[i][r] - rr[i][r] - ii[i][r]);
        c2 *p = C + t.c_off + (int64_t)ccol * t.ldc + crow;
        if (MODE == 0) {
          *p = acc;
        } else if (MODE == 1) {
          *p = make_double2(cold[i][r].x - acc.x, cold[i][r].y - acc.y);
        } else {
          *p = make_double2(cold[i][r].x + acc.x, cold[i][r].y + acc.y);
        }
      }
    }
  }
}

// Pipelined variant (tile shapes 11 and 12): the 32 x 64 workgroup tile of
// shape 7 (four waves of 32 rows x 16 columns), with every full 16-k chunk
// of a term staged in LDS by direct-to-LDS loads one chunk ahead, so the
// loads of chunk c + 1 are in flight while the products of chunk c run.
// The workgroup shares the A chunk (32 rows x 16 k, each wave loads a
// quarter); each wave loads its own B chunk (16 k x 16 columns); both are
// double-buffered.  LDS slots of a load instruction are consecutive (lane l
// writes slot 64 q + l), so the layouts follow the coalesced lane order:
//   A, plain (A read along its columns): slot k 32 + r;
//   A^T (A read along k): slot r 16 + (k + r) mod 16;
//   B: slot c 16 + (k + c) mod 16 of the wave's block;
// the rotations keep the MFMA operand reads (16 rows or columns at one k)
// on distinct banks.  Rows and columns past the tile's edge are not loaded:
// their slots feed only outputs that are never stored.  The k % 16 tail and
// the target tile are handled as in k_gemm (CL = 1: the target tile staged
// in LDS too, CL = 0: fetched after the products).  The products are
// k_gemm's, in the same order, so the results are bitwise the same.  Every
// wave of the workgroup takes part in every barrier (the chunk loop and its
// bounds are uniform over the workgroup); waves past the tile's last column
// skip their loads of B, their products and their stores.
template <int MODE, int CL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gemm_pipe(
    const c2 *__restrict__ A, const c2 *__restrict__ B, c2 *__restrict__ C, const Tile *__restrict__ tiles,
    const Term *__restrict__ terms, int ncols, int ntiles, int ny, int xcd_order) {
  constexpr int RB = 2, TN = 64;
  __shared__ c2 abuf[2][512];
  __shared__ c2 bbuf[2][4][256];
  __shared__ c2 cbuf[CL ? 4 * 512 : 1];
  typedef __attribute__((address_space(3))) void *lds_ptr;
  int bx = (int)blockIdx.x, by = (int)blockIdx.y;
  if (xcd_order) {
    const int q = (int)(blockIdx.x >> 3);
    by = q % ny;
    bx = 8 * (q / ny) + (int)(blockIdx.x & 7);
    if (bx >= ntiles) return;
  }
  const Tile t = tiles[bx];
  const bool packed = t.c0 == TILE_PACKED;
  int rb0 = t.r0, cb0 = t.c0, tn = t.n, nsub = 1, nsc = 1, st0 = 0, sstep = 1;
  if (packed) {
    if (by > 0) return;
  } else if (t.r0 < 0) {
    nsc = (t.n + TN - 1) / TN;
    nsub = ((t.m + TM - 1) / TM) * nsc;
    st0 = by;
    sstep = ny;
  } else if (t.c0 < 0) {
    tn = ncols;
    cb0 = by * TN;
    if (cb0 >= tn) return;
  } else if (by > 0) {
    return;
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int li = lane & 15, lg = lane >> 4;
  c2 *const cw = cbuf + (CL ? wave * 512 : 0);
  // A packed tile gives each wave a column block of its own (C and B start,
  // B's leading dimension, valid columns): one term's A rows times blocks of
  // several targets.  Otherwise the wave's columns start at col0 of t.c_off.
  int64_t cbase = t.c_off, wb_off = 0;
  int wldb = 0, q_end = t.t_end;
  if (packed) {
    tn = 0;
    q_end = t.t_begin + 1;
    if (wave < t.n) {
      const Term wd = terms[t.t_begin + 1 + wave];
      cbase = wd.a_off;
      wb_off = wd.b_off;
      wldb = wd.ldb;
      tn = wd.lda;
    }
  }
  for (int st = st0; st < nsub; st += sstep) {
    int rb = rb0, cb = cb0;
    if (t.r0 < 0) {
      rb = (st / nsc) * TM;
      cb = (st % nsc) * TN;
    }
    const int row0 = rb, col0 = packed ? 0 : cb + 16 * wave;
    if (row0 >= t.m) continue;                          // uniform over the workgroup
    const bool cols = col0 < tn;                        // uniform over the wave
    __syncthreads();                                    // the previous sub-tile's LDS reads are done
    bool arow_ok[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) arow_ok[i] = row0 + 16 * i + li < t.m;
    const bool one_rb = row0 + 16 >= t.m;
    if (CL && MODE != 0 && cols) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = 64 * q + lane, c = e >> 5, r = (e - 32 * c - 2 * c) & 31;
        const int ccol = col0 + c, crow = row0 + r;
        if (ccol < tn && crow < t.m)
          __builtin_amdgcn_global_load_lds((const void *)(C + cbase + (int64_t)ccol * t.ldc + crow),
                                           (lds_ptr)(cw + 64 * q), 16, 0, 0);
      }
    }
    d4 rr[RB], ii[RB], ss[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) rr[i] = ii[i] = ss[i] = d4{0.0, 0.0, 0.0, 0.0};
    for (int q = t.t_begin; q < q_end; ++q) {
      const Term tm = terms[q];
      const c2 *Ab = A + tm.a_off;
      const c2 *Bw = B + (packed ? wb_off : tm.b_off);     // the wave's B columns start at column col0 of Bw
      const int ldb = packed ? wldb : tm.ldb;
      const int nchunk = tm.k >> 4;
      // chunk ch of this term into buffer b: the wave's quarter of A and its own B
      auto stage = [&](int ch, int b) {
        const int k0 = ch * 16;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int qa = 2 * wave + h, e = 64 * qa + lane;
          int r, k;
          if (tm.trans) {
            r = e >> 4;
            k = ((e & 15) - r) & 15;
          } else {
            k = e >> 5;
            r = e & 31;
          }
          if (row0 + r < t.m)
            __builtin_amdgcn_global_load_lds(
                (const void *)(tm.trans ? Ab + (int64_t)(row0 + r) * tm.lda + k0 + k
                                        : Ab + (int64_t)(k0 + k) * tm.lda + row0 + r),
                (lds_ptr)(&abuf[b][64 * qa]), 16, 0, 0);
        }
        if (cols) {
#pragma unroll
          for (int qb = 0; qb < 4; ++qb) {
            const int e = 64 * qb + lane, c = e >> 4, k = ((e & 15) - c) & 15;
            if (col0 + c < tn)
              __builtin_amdgcn_global_load_lds((const void *)(Bw + (int64_t)(col0 + c) * ldb + k0 + k),
                                               (lds_ptr)(&bbuf[b][wave][64 * qb]), 16, 0, 0);
          }
        }
      };
      __syncthreads();                                  // the previous term's chunk reads are done
      if (nchunk > 0) stage(0, 0);
      for (int ch = 0; ch < nchunk; ++ch) {
        const int b = ch & 1;
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's loads of chunk ch have landed
        __syncthreads();                                    // every wave's have; chunk ch - 1 is read
        if (ch + 1 < nchunk) stage(ch + 1, b ^ 1);
        if (cols) {
          auto prod = [&](auto rbe) {
            constexpr int RBE = decltype(rbe)::value;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              const int k = 4 * s + lg;
              c2 av[RB];
#pragma unroll
              for (int i = 0; i < RBE; ++i) {
                const int r = 16 * i + li;
                av[i] = tm.trans ? abuf[b][r * 16 + ((k + r) & 15)] : abuf[b][k * 32 + r];
              }
              const c2 bv = bbuf[b][wave][li * 16 + ((k + li) & 15)];
              const double bs = bv.x + bv.y;
#pragma unroll
              for (int i = 0; i < RBE; ++i) {
                rr[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, bv.x, rr[i], 0, 0, 0);
                ii[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].y, bv.y, ii[i], 0, 0, 0);
                ss[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x + av[i].y, bs, ss[i], 0, 0, 0);
              }
            }
          };
          if (one_rb)
            prod(std::integral_constant<int, 1>{});
          else
            prod(std::integral_constant<int, RB>{});
        }
      }
      // tail (k % 16): steps of 4 from global memory, as in k_gemm
      if (cols) {
        auto tail = [&](auto rbe) {
          constexpr int RBE = decltype(rbe)::value;
          for (int kt = nchunk * 16; kt < tm.k; kt += 4) {
            const int k = kt + lg;
            const bool kok = k < tm.k;
            c2 av[RB];
#pragma unroll
            for (int i = 0; i < RBE; ++i) {
              const int arow = row0 + 16 * i + li;
              av[i] = make_double2(0.0, 0.0);
              if (kok && arow_ok[i]) av[i] = tm.trans ? Ab[(int64_t)arow * tm.lda + k] : Ab[(int64_t)k * tm.lda + arow];
            }
            const int bcol = col0 + li;
            c2 bv = make_double2(0.0, 0.0);
            if (kok && bcol < tn) bv = Bw[(int64_t)bcol * ldb + k];
#pragma unroll
            for (int i = 0; i < RBE; ++i) {
              rr[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, bv.x, rr[i], 0, 0, 0);
              ii[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].y, bv.y, ii[i], 0, 0, 0);
              ss[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x + av[i].y, bv.x + bv.y, ss[i], 0, 0, 0);
            }
          }
        };
        if (one_rb)
          tail(std::integral_constant<int, 1>{});
        else
          tail(std::integral_constant<int, RB>{});
      }
    }
    if (!cols) continue;
    c2 cold[RB][4];
    if (MODE != 0) {
      if (CL) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rw = 16 * i + lg + 4 * r;
            cold[i][r] = cw[li * 32 + ((rw + 2 * li) & 31)];
          }
      } else {
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int crow = row0 + 16 * i + lg + 4 * r, ccol = col0 + li;
            cold[i][r] = make_double2(0.0, 0.0);
            if (ccol < tn && crow < t.m) cold[i][r] = C[cbase + (int64_t)ccol * t.ldc + crow];
          }
      }
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int ccol = col0 + li;
      if (ccol >= tn) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int crow = row0 + 16 * i + lg + 4 * r;
        if (crow >= t.m) continue;
        const c2 acc = make_double2(rr[i][r] - ii[i][r], ss[i][r] - rr[i][r] - ii[i][r]);
        c2 *p = C + cbase + (int64_t)ccol * t.ldc + crow;
        if (MODE == 0) {
          *p = acc;
        } else if (MODE == 1) {
          *p = make_double2(cold[i][r].x - acc.x, cold[i][r].y - acc.y);
        } else {
          *p = make_double2(cold[i][r].x + acc.x, cold[i][r].y + acc.y);
        }
      }
    }
  }
}

// One right-hand side (tile shape 6): a matrix-vector product per tile of
// 32 rows, on the vector ALU; with one column the MFMA tile would compute
// 31 padding columns and the product is bound by streaming A.  256 threads
// = 32 rows x 8 lanes along k; A^T terms (A read along k) take row = t / 8,
// plain terms (A read along its columns) row = t % 32, so every load of A is
// coalesced.  Each thread sums its share of k in order; the 8 partial sums
// of a row are added in a fixed order through LDS (deterministic).  Solve
// tiles only (c0 < 0, ncols = 1).
template <int MODE>
__global__ __launch_bounds__(256) void k_gemv(const c2 *__restrict__ A, const c2 *__restrict__ B,
                                              c2 *__restrict__ C, const Tile *__restrict__ tiles,
                                              const Term *__restrict__ terms, int ntiles) {
  __shared__ c2 part[2][TM][9];
  // one-dimensional grid of ntiles workgroups (the host launches it so)
  const int bx = (int)blockIdx.x;
  if (bx >= ntiles) return;
  const Tile t = tiles[bx];
  const int tid = threadIdx.x;
  const int rT = tid >> 3, kT = tid & 7;      // A^T terms
  const int rN = tid & 31, kN = tid >> 5;     // plain terms
  c2 accT = make_double2(0.0, 0.0), accN = make_double2(0.0, 0.0);
  const int rowT = t.r0 + rT, rowN = t.r0 + rN;
  for (int q = t.t_begin; q < t.t_end; ++q) {
    const Term tm = terms[q];
    const c2 *Ab = A + tm.a_off, *Bb = B + tm.b_off;
    if (tm.trans) {
      if (rowT < t.m) {
#pragma unroll 4
        for (int k = kT; k < tm.k; k += 8) cmac(accT, Ab[(int64_t)rowT * tm.lda + k], Bb[k]);
      }
    } else {
      if (rowN < t.m) {
#pragma unroll 4
        for (int k = kN; k < tm.k; k += 8) cmac(accN, Ab[(int64_t)k * tm.lda + rowN], Bb[k]);
      }
    }
  }
  part[0][rT][kT] = accT;
  part[1][rN][kN] = accN;
  __syncthreads();
  if (tid < TM) {
    const int row = t.r0 + tid;
    c2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      acc.x += part[0][tid][j].x;
      acc.y += part[0][tid][j].y;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      acc.x += part[1][tid][j].x;
      acc.y += part[1][tid][j].y;
    }
    if (row < t.m) {
      c2 *p = C + t.c_off + row;
      if (MODE == 0) *p = acc;
      else if (MODE == 1) *p = make_double2(p->x - acc.x, p->y - acc.y);
      else *p = make_double2(p->x + acc.x, p->y + acc.y);
    }
  }
}

// ------------------------------------------------------------------ precision form
// Complex FP32 products on V_MFMA_F32_16X16X4_F32 (3M split as k_gemm, FP32
// accumulation).  Same tile/term scheme and k permutation as k_gemm; the
// result register r of lane l is D[4 (l / 16) + r][l % 16] for this
// instruction.  AT selects the A operand: 0 complex FP32, 1 BF16 pairs,
// 2 FP16 pairs (16-bit far factors, multiplied by their block scale).
typedef float f4 __attribute__((ext_vector_type(4)));

template <int AT>
__device__ __forceinline__ float2 load_a(const void *__restrict__ A, int64_t i) {
  if (AT == 0) return reinterpret_cast<const float2 *>(A)[i];
  const uint32_t w = reinterpret_cast<const uint32_t *>(A)[i];
  if (AT == 1) return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
  const __half2 h = *reinterpret_cast<const __half2 *>(&w);
  return make_float2(__low2float(h), __high2float(h));
}

template <int MODE, int AT, int WR, int NB, int WPE = 1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_gemm32(const void *__restrict__ A, const float2 *__restrict__ B,
                                                float2 *__restrict__ C, const Tile *__restrict__ tiles,
                                                const Term *__restrict__ terms, const float *__restrict__ scales,
                                                const int32_t *__restrict__ rowpart, int ncols, int ntiles, int ny,
                                                int xcd_order) {
  constexpr int RB = 2 / WR, WC = 4 / WR;   // tile shapes as in k_gemm
  constexpr int TN = 16 * NB * WC;
  // workgroup -> (tile bx, part by): plain or XCD-aware order, as in k_gemm
  int bx = (int)blockIdx.x, by = (int)blockIdx.y;
  if (xcd_order) {
    const int q = (int)(blockIdx.x >> 3);
    by = q % ny;
    bx = 8 * (q / ny) + (int)(blockIdx.x & 7);
    if (bx >= ntiles) return;
  }
  const Tile t = tiles[bx];
  int rb = t.r0, cb = t.c0, tn = t.n;
  if (t.r0 < 0) {
    const int nsc = (t.n + TN - 1) / TN, nsr = (t.m + TM - 1) / TM;
    if (by >= nsr * nsc) return;
    rb = (by / nsc) * TM;
    cb = (by % nsc) * TN;
  } else if (t.c0 < 0) {             // one row tile over ncols columns, by picks the column tile
    tn = ncols;
    cb = by * TN;
    if (cb >= tn) return;
  } else if (by > 0) {
    return;
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int wr = WR == 2 ? (wave >> 1) : 0, wc = WR == 2 ? (wave & 1) : wave;
  const int row0 = rb + 16 * RB * wr, col0 = cb + 16 * NB * wc;
  if (row0 >= t.m || col0 >= tn) return;
  const int li = lane & 15, lg = lane >> 4;
  bool arow_ok[RB];
  // terms with sidx -2 (a factor group of the first far stage) scale each A
  // row by its own factor's scale: row arow of the target is T row c_off + arow
  float sc_row[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    const int arow = row0 + 16 * i + li;
    arow_ok[i] = arow < t.m;
    sc_row[i] = 1.0f;
    if (AT != 0 && rowpart != nullptr && arow_ok[i] && t.t_begin < t.t_end && terms[t.t_begin].sidx == -2)
      sc_row[i] = scales[rowpart[t.c_off + arow]];
  }
  // read-modify-write modes: fetch C now, so its latency hides behind the
  // products (after them in the builds for more waves per SIMD)
  float2 cold[RB][NB][4];
  auto fetch_c = [&]() {
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int ccol = col0 + 16 * j + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int crow = row0 + 16 * i + 4 * lg + r;
          cold[i][j][r] = make_float2(0.f, 0.f);
          if (ccol < tn && crow < t.m) cold[i][j][r] = C[t.c_off + (int64_t)ccol * t.ldc + crow];
        }
      }
  };
  if (MODE != 0 && WPE == 1) fetch_c();
  f4 rr[RB][NB], ii[RB][NB], ss[RB][NB];          // 3M: Ar Br, Ai Bi, (Ar + Ai)(Br + Bi)
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) rr[i][j] = ii[i][j] = ss[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  // a wave of two 16-row blocks whose second block lies wholly past the
  // target's edge computes the first only (wave-uniform choice)
  const bool one_rb = RB > 1 && row0 + 16 >= t.m;
  auto products = [&](auto rbe) {
    constexpr int RBE = decltype(rbe)::value;
    for (int q = t.t_begin; q < t.t_end; ++q) {
      const Term tm = terms[q];
      float sc[RB];
#pragma unroll
      for (int i = 0; i < RBE; ++i)
        sc[i] = AT == 0 ? 1.0f : (tm.sidx >= 0 ? scales[tm.sidx] : (tm.sidx == -2 ? sc_row[i] : 1.0f));
      const int kfull = tm.k & ~15;
      for (int k0 = 0; k0 < kfull; k0 += 16) {
        float2 av[RB][4], bv[NB][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int k = k0 + 4 * s + lg;
#pragma unroll
          for (int i = 0; i < RBE; ++i) {
            const int arow = row0 + 16 * i + li;
            av[i][s] = make_float2(0.f, 0.f);
            if (arow_ok[i]) {
              const int64_t idx =
                  tm.trans ? tm.a_off + (int64_t)arow * tm.lda + k : tm.a_off + (int64_t)k * tm.lda + arow;
              av[i][s] = load_a<AT>(A, idx);
              av[i][s].x *= sc[i];
              av[i][s].y *= sc[i];
            }
          }
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            const int bcol = col0 + 16 * j + li;
            bv[j][s] = make_float2(0.f, 0.f);
            if (bcol < tn) bv[j][s] = B[tm.b_off + (int64_t)bcol * tm.ldb + k];
          }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            const float bs = bv[j][s].x + bv[j][s].y;
#pragma unroll
            for (int i = 0; i < RBE; ++i) {
              rr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i][s].x, bv[j][s].x, rr[i][j], 0, 0, 0);
              ii[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i][s].y, bv[j][s].y, ii[i][j], 0, 0, 0);
              ss[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i][s].x + av[i][s].y, bs, ss[i][j], 0, 0, 0);
            }
          }
        }
      }
      for (int kt = kfull; kt < tm.k; kt += 4) {
        const int k = kt + lg;
        const bool kok = k < tm.k;
        float2 av[RB];
#pragma unroll
        for (int i = 0; i < RBE; ++i) {
          const int arow = row0 + 16 * i + li;
          av[i] = make_float2(0.f, 0.f);
          if (kok && arow_ok[i]) {
            const int64_t idx = tm.trans ? tm.a_off + (int64_t)arow * tm.lda + k : tm.a_off + (int64_t)k * tm.lda + arow;
            av[i] = load_a<AT>(A, idx);
            av[i].x *= sc[i];
            av[i].y *= sc[i];
          }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const int bcol = col0 + 16 * j + li;
          float2 bv = make_float2(0.f, 0.f);
          if (kok && bcol < tn) bv = B[tm.b_off + (int64_t)bcol * tm.ldb + k];
#pragma unroll
          for (int i = 0; i < RBE; ++i) {
            rr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x, bv.x, rr[i][j], 0, 0, 0);
            ii[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, bv.y, ii[i][j], 0, 0, 0);
            ss[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x + av[i].y, bv.x + bv.y, ss[i][j], 0, 0, 0);
          }
        }
      }
    }
  };
  if (one_rb)
    products(std::integral_constant<int, 1>{});
  else
    products(std::integral_constant<int, RB>{});
  if (MODE != 0 && WPE > 1) fetch_c();
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int ccol = col0 + 16 * j + li;
      if (ccol >= tn) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int crow = row0 + 16 * i + 4 * lg + r;
        if (crow >= t.m) continue;
        const float2 acc = make_float2(rr[i][j][r] - ii[i][j][r], ss[i][j][r] - rr[i][j][r] - ii[i][j][r]);
        float2 *p = C + t.c_off + (int64_t)ccol * t.ldc + crow;
        if (MODE == 0) {
          *p = acc;
        } else if (MODE == 1) {
          *p = make_float2(cold[i][j][r].x - acc.x, cold[i][j][r].y - acc.y);
        } else {
          *p = make_float2(cold[i][j][r].x + acc.x, cold[i][j][r].y + acc.y);
        }
      }
    }
}

// Pipelined FP32 variant (tile shapes 11 and 12 of launches with FP32 A
// operands): k_gemm32's 32 x 64 tile of four 32 x 16 waves, with every full
// 16-k chunk staged in LDS one chunk ahead as in k_gemm_pipe.  A lane's
// direct-to-LDS load moves 16 bytes, two complex floats: a pair of rows
// (plain A) or of k (A^T, and B).  LDS slot layouts (16-byte slots; slot e
// holds elements 2 e and 2 e + 1 of the buffer):
//   A, plain: slot k 16 + p holds rows 2 p, 2 p + 1 at k (element k 32 + r);
//   A^T: slot r 8 + (m + r) mod 8 holds k = 2 m, 2 m + 1 of row r;
//   B: slot c 8 + (m + c) mod 8 holds k = 2 m, 2 m + 1 of column c.
// A row pair that straddles the tile's last row takes a plain load of its
// valid row and an LDS store (no read past the operand).  The target tile is
// fetched after the products.  Same products in the same order as k_gemm32,
// so the results are bitwise the same.
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_gemm32_pipe(
    const float2 *__restrict__ A, const float2 *__restrict__ B, float2 *__restrict__ C,
    const Tile *__restrict__ tiles, const Term *__restrict__ terms, int ncols, int ntiles, int ny, int xcd_order) {
  constexpr int RB = 2, TN = 64;
  __shared__ float2 abuf[2][512];
  __shared__ float2 bbuf[2][4][256];
  typedef __attribute__((address_space(3))) void *lds_ptr;
  int bx = (int)blockIdx.x, by = (int)blockIdx.y;
  if (xcd_order) {
    const int q = (int)(blockIdx.x >> 3);
    by = q % ny;
    bx = 8 * (q / ny) + (int)(blockIdx.x & 7);
    if (bx >= ntiles) return;
  }
  const Tile t = tiles[bx];
  int rb = t.r0, cb = t.c0, tn = t.n;
  if (t.r0 < 0) {
    const int nsc = (t.n + TN - 1) / TN, nsr = (t.m + TM - 1) / TM;
    if (by >= nsr * nsc) return;
    rb = (by / nsc) * TM;
    cb = (by % nsc) * TN;
  } else if (t.c0 < 0) {
    tn = ncols;
    cb = by * TN;
    if (cb >= tn) return;
  } else if (by > 0) {
    return;
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int li = lane & 15, lg = lane >> 4;
  const int row0 = rb, col0 = cb + 16 * wave;
  if (row0 >= t.m) return;                              // uniform over the workgroup
  const bool cols = col0 < tn;                          // uniform over the wave
  bool arow_ok[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) arow_ok[i] = row0 + 16 * i + li < t.m;
  const bool one_rb = row0 + 16 >= t.m;
  f4 rr[RB], ii[RB], ss[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) rr[i] = ii[i] = ss[i] = f4{0.f, 0.f, 0.f, 0.f};
  for (int q = t.t_begin; q < t.t_end; ++q) {
    const Term tm = terms[q];
    const float2 *Ab = A + tm.a_off;
    const int nchunk = tm.k >> 4;
    auto stage = [&](int ch, int b) {
      const int k0 = ch * 16, e = 64 * wave + lane;          // this wave's 64 slots of A
      if (tm.trans) {
        const int r = e >> 3, m = ((e & 7) - r) & 7;
        if (row0 + r < t.m)
          __builtin_amdgcn_global_load_lds((const void *)(Ab + (int64_t)(row0 + r) * tm.lda + k0 + 2 * m),
                                           (lds_ptr)(&abuf[b][128 * wave]), 16, 0, 0);
      } else {
        const int k = e >> 4, r = 2 * (e & 15);
        if (row0 + r + 1 < t.m)
          __builtin_amdgcn_global_load_lds((const void *)(Ab + (int64_t)(k0 + k) * tm.lda + row0 + r),
                                           (lds_ptr)(&abuf[b][128 * wave]), 16, 0, 0);
        else if (row0 + r < t.m)
          abuf[b][2 * e] = Ab[(int64_t)(k0 + k) * tm.lda + row0 + r];
      }
      if (cols) {
#pragma unroll
        for (int qb = 0; qb < 2; ++qb) {
          const int eb = 64 * qb + lane, c = eb >> 3, m = ((eb & 7) - c) & 7;
          if (col0 + c < tn)
            __builtin_amdgcn_global_load_lds((const void *)(B + tm.b_off + (int64_t)(col0 + c) * tm.ldb + k0 + 2 * m),
                                             (lds_ptr)(&bbuf[b][wave][128 * qb]), 16, 0, 0);
        }
      }
    };
    __syncthreads();                                    // the previous term's chunk reads are done
    if (nchunk > 0) stage(0, 0);
    for (int ch = 0; ch < nchunk; ++ch) {
      const int b = ch & 1;
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's loads of chunk ch have landed
      __syncthreads();                                    // every wave's have; chunk ch - 1 is read
      if (ch + 1 < nchunk) stage(ch + 1, b ^ 1);
      if (cols) {
        auto prod = [&](auto rbe) {
          constexpr int RBE = decltype(rbe)::value;
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const int k = 4 * s + lg;
            float2 av[RB];
#pragma unroll
            for (int i = 0; i < RBE; ++i) {
              const int r = 16 * i + li;
              av[i] = tm.trans ? abuf[b][2 * (r * 8 + (((k >> 1) + r) & 7)) + (k & 1)] : abuf[b][k * 32 + r];
            }
            const float2 bv = bbuf[b][wave][2 * (li * 8 + (((k >> 1) + li) & 7)) + (k & 1)];
#pragma unroll
            for (int i = 0; i < RBE; ++i) {
              rr[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x, bv.x, rr[i], 0, 0, 0);
              ii[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, bv.y, ii[i], 0, 0, 0);
              ss[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x + av[i].y, bv.x + bv.y, ss[i], 0, 0, 0);
            }
          }
        };
        if (one_rb)
          prod(std::integral_constant<int, 1>{});
        else
          prod(std::integral_constant<int, RB>{});
      }
    }
    if (cols) {                                         // tail (k % 16) from global memory, as in k_gemm32
      auto tail = [&](auto rbe) {
        constexpr int RBE = decltype(rbe)::value;
        for (int kt = nchunk * 16; kt < tm.k; kt += 4) {
          const int k = kt + lg;
          const bool kok = k < tm.k;
          float2 av[RB];
#pragma unroll
          for (int i = 0; i < RBE; ++i) {
            const int arow = row0 + 16 * i + li;
            av[i] = make_float2(0.f, 0.f);
            if (kok && arow_ok[i]) av[i] = tm.trans ? Ab[(int64_t)arow * tm.lda + k] : Ab[(int64_t)k * tm.lda + arow];
          }
          const int bcol = col0 + li;
          float2 bv = make_float2(0.f, 0.f);
          if (kok && bcol < tn) bv = B[tm.b_off + (int64_t)bcol * tm.ldb + k];
#pragma unroll
          for (int i = 0; i < RBE; ++i) {
            rr[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x, bv.x, rr[i], 0, 0, 0);
            ii[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].y, bv.y, ii[i], 0, 0, 0);
            ss[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i].x + av[i].y, bv.x + bv.y, ss[i], 0, 0, 0);
          }
        }
      };
      if (one_rb)
        tail(std::integral_constant<int, 1>{});
      else
        tail(std::integral_constant<int, RB>{});
    }
  }
  if (!cols) return;
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    const int ccol = col0 + li;
    if (ccol >= tn) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int crow = row0 + 16 * i + 4 * lg + r;
      if (crow >= t.m) continue;
      const float2 acc = make_float2(rr[i][r] - ii[i][r], ss[i][r] - rr[i][r] - ii[i][r]);
      float2 *p = C + t.c_off + (int64_t)ccol * t.ldc + crow;
      if (MODE == 0) {
        *p = acc;
      } else {
        const float2 o = *p;
        *p = MODE == 1 ? make_float2(o.x - acc.x, o.y - acc.y) : make_float2(o.x + acc.x, o.y + acc.y);
      }
    }
  }
}


__global__ void k_to32(const c2 *__restrict__ in, float2 *__restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2((float)in[i].x, (float)in[i].y);
}
__global__ void k_to64(const float2 *__restrict__ in, c2 *__restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_double2((double)in[i].x, (double)in[i].y);
}
// y = a - b  (FP32 residual)
__global__ void k_sub32(const float2 *__restrict__ a, const float2 *__restrict__ b, float2 *__restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = make_float2(a[i].x - b[i].x, a[i].y - b[i].y);
}
// y += sgn * w  (FP32)
__global__ void k_axpy32(float2 *__restrict__ y, const float2 *__restrict__ w, float sgn, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = make_float2(fmaf(sgn, w[i].x, y[i].x), fmaf(sgn, w[i].y, y[i].y));
}
// Problem p of a batch owns unknowns [soff[p], soff[p + 1]) (elimination
// order and RWG order alike); nseg problems.
__device__ __forceinline__ int seg_of(const int64_t *__restrict__ soff, int nseg, int64_t q) {
  int lo = 0, hi = nseg;                  // soff[lo] <= q < soff[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (soff[mid] <= q) lo = mid; else hi = mid;
  }
  return lo;
}

// per-column, per-problem sum of |v|^2 (FP32 input, FP64 accumulation):
// block (r, p) writes out[p R + r]
__global__ __launch_bounds__(256) void k_colnorm32(const float2 *__restrict__ a, int64_t N,
                                                   const int64_t *__restrict__ soff, double *__restrict__ out) {
  const int64_t r = blockIdx.x, R = gridDim.x, p = blockIdx.y;
  __shared__ double sx[256];
  double x = 0.0;
  for (int64_t i = soff[p] + threadIdx.x; i < soff[p + 1]; i += 256) {
    const float2 u = a[r * N + i];
    x += (double)u.x * u.x + (double)u.y * u.y;
  }
  sx[threadIdx.x] = x;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sx[threadIdx.x] += sx[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p * R + r] = sx[0];
}

// Far factors to 16-bit pairs with one FP32 scale per factor per block:
// scale = largest |component|, stored values = component / scale.
struct FarPart {
  int64_t off, len;
};
__device__ __forceinline__ uint32_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
template <int AT>
__global__ __launch_bounds__(256) void k_far16(const c2 *__restrict__ in, uint32_t *__restrict__ out,
                                               float *__restrict__ scales, const FarPart *__restrict__ parts) {
  const FarPart pt = parts[blockIdx.x];
  __shared__ double sm[256];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < pt.len; i += 256) {
    const c2 v = in[pt.off + i];
    m = fmax(m, fmax(fabs(v.x), fabs(v.y)));
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  const double sc = sm[0] > 0.0 ? sm[0] : 1.0;
  if (threadIdx.x == 0) scales[blockIdx.x] = (float)sc;
  const double inv = 1.0 / sc;
  for (int64_t i = threadIdx.x; i < pt.len; i += 256) {
    const c2 v = in[pt.off + i];
    const float re = (float)(v.x * inv), im = (float)(v.y * inv);
    uint32_t w;
    if (AT == 1) {
      w = bf16_rne(re) | (bf16_rne(im) << 16);
    } else {
      const __half2 h = __floats2half2_rn(re, im);
      w = *reinterpret_cast<const uint32_t *>(&h);
    }
    out[pt.off + i] = w;
  }
}

// ------------------------------------------------------------------ inverse
// Gauss-Jordan inversion with partial pivoting (row interchanges recorded,
// not performed) of n x n blocks, n <= NC, one block per workgroup of 8 NC
// threads.  Equivalent to LU with partial pivoting followed by the inverse.
// A zero pivot column flags the block as singular.
//
// Tile layout: thread (rg, cg) with tid = rg + RB*cg owns rows rg*2, rg*2+1 and
// columns cg*CT..cg*CT+CT-1 (RB = NC/2 row groups, 16 column groups, CT = NC/16;
// a column group fills whole 16-lane rows of one wave).  One barrier per
// elimination step.
//
// The pivot row is not scaled at its step: every row r is kept multiplied by
// its own pivot piv_r from then on (row operations commute with that scaling),
// its pivot-column entry is stored as 1, and the store multiplies row r by
// 1 / piv_r.  So the step is one rank-1 update of all rows with the pivot
// row's multiplier set to zero.
//
// The chosen pivots are those of LU with partial pivoting (the rows not yet
// pivoted hold the Schur complement of the pivoted ones).  A block is
// flagged as numerically singular when a pivot's modulus falls below
// n eps max|D_ij| (eps = 2^-52, max over the block as loaded).

// 64-bit DPP move inside a wave; lanes outside the 16-lane row or the row
// mask read 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint64_t dpp64(uint64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROWMASK, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROWMASK, 0xF, true);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }

// Maximum over each group of RB consecutive lanes (RB = 16, 32 or 64), left
// in the group's last lane.  Every lane of the wave must be active.
template <int RB>
__device__ __forceinline__ uint64_t group_max(uint64_t k) {
  k = umax64(k, dpp64<0x111, 0xF>(k));                 // row_shr:1
  k = umax64(k, dpp64<0x112, 0xF>(k));                 // row_shr:2
  k = umax64(k, dpp64<0x114, 0xF>(k));                 // row_shr:4
  k = umax64(k, dpp64<0x118, 0xF>(k));                 // row_shr:8: lane 15 holds the row maximum
  if (RB >= 32) k = umax64(k, dpp64<0x142, 0xA>(k));   // row_bcast:15 into rows 1 and 3
  if (RB >= 64) k = umax64(k, dpp64<0x143, 0xC>(k));   // row_bcast:31 into rows 2 and 3
  return k;
}

// Value of lane src_lane (the same for the whole group) to every lane.
template <int RB>
__device__ __forceinline__ double group_bcast(double v, int src_lane) {
  if (RB == 64) {                     // one group per wave: the source lane is wave-uniform
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, src_lane);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src_lane);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
  }
  return __shfl(v, src_lane, 64);
}

// One Gauss-Jordan update: row PR of the source lane's pair is the pivot row
// (PR is block-uniform, so the caller branches instead of selecting per
// element); a[r][j] -= mi[r] rp[j].
template <int RT, int CT, int RB, int PR>
__device__ __forceinline__ void gj_update(c2 (&a)[RT][CT], const c2 (&mi)[RT], int src_lane) {
  c2 rp[CT];
#pragma unroll
  for (int j = 0; j < CT; ++j) {
    rp[j].x = group_bcast<RB>(a[PR][j].x, src_lane);
    rp[j].y = group_bcast<RB>(a[PR][j].y, src_lane);
  }
#pragma unroll
  for (int j = 0; j < CT; ++j)
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      a[r][j].x = fma(-mi[r].x, rp[j].x, fma(mi[r].y, rp[j].y, a[r][j].x));
      a[r][j].y = fma(-mi[r].x, rp[j].y, fma(-mi[r].y, rp[j].x, a[r][j].y));
    }
}

template <int NC>
__global__ __launch_bounds__(8 * NC) void k_inverse(const c2 *__restrict__ W, c2 *__restrict__ F,
                                                    const int64_t *__restrict__ off,
                                                    const int32_t *__restrict__ nsz,
                                                    const int32_t *__restrict__ ids,
                                                    int *__restrict__ status) {
  constexpr int RT = 2, RB = NC / RT, CT = NC / 16, GW = 64 / RB;
  static_assert(64 % RB == 0 && RB >= 16, "a column group must fill whole rows of one wave");
  static_assert(NC <= 128, "the row index is packed in 7 bits of the pivot key");
  const int blk = blockIdx.x;
  const int n = nsz[blk];
  const c2 *src = W + off[blk];
  c2 *dst = F + off[blk];
  const int tid = threadIdx.x, rg = tid % RB, cg = tid / RB;
  const int lane = tid & 63, wave = tid >> 6;
  const int gbase = lane - rg;          // first lane of my column group
  __shared__ c2 colbuf[2][NC];          // pivot column of the step (pivot row entry zeroed)
  __shared__ c2 pinv[2];
  __shared__ int pbuf[2];
  __shared__ int pivrow[NC], stepof[NC];
  __shared__ c2 rowinv[NC];             // 1 / pivot of each row
  __shared__ double wmax[8 * NC / 64];  // per-wave max |D_ij|^2
  c2 a[RT][CT];
  double amax = 0.0;
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int j = 0; j < CT; ++j) {
      const int row = rg * RT + r, col = cg * CT + j;
      a[r][j] = (row < n && col < n) ? src[(int64_t)col * n + row] : make_double2(0.0, 0.0);
      amax = fmax(amax, a[r][j].x * a[r][j].x + a[r][j].y * a[r][j].y);
    }
  // singularity threshold on |pivot|^2: (n eps max|D_ij|)^2
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
  if (lane == 0) wmax[wave] = amax;
  __syncthreads();
  for (int w = 0; w < 8 * NC / 64; ++w) amax = fmax(amax, wmax[w]);
  const double tol = (double)n * 0x1p-52;
  const double thr2 = tol * tol * amax;
  uint32_t used = 0;
#pragma unroll
  for (int r = 0; r < RT; ++r)
    if (rg * RT + r >= n) used |= 1u << r;
  // A wave whose columns all lie beyond the block (n below the size class)
  // holds zeros that every step leaves at zero: it skips the updates and
  // only joins the barriers.  Wave-uniform.
  const bool wave_live = wave * GW * CT < n;
  bool singular = false;
  // Steps in runs of CT, so that the pivot column's register slot kc is a
  // compile-time index (no select chains over the tile).
  for (int kb = 0; kb < n && !singular; kb += CT) {
    const int cgk = kb / CT;            // column group holding columns kb .. kb + CT - 1
#pragma unroll
    for (int kc = 0; kc < CT; ++kc) {
      const int k = kb + kc;
      if (k >= n) break;                // block-uniform
      const int s = k & 1;
      if (wave == cgk / GW) {
        // Pivot search on column k, at raised wave priority: the other waves
        // of this SIMD are still in the previous update.  Key = |z|^2 with
        // its last 7 mantissa bits replaced by (127 - row): largest modulus,
        // lowest row on ties.
        __builtin_amdgcn_s_setprio(3);
        const bool mine = (cg == cgk);
        uint64_t key = 0;
        c2 v[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          v[r] = a[r][kc];
          const int row = rg * RT + r;
          if (mine) colbuf[s][row] = v[r];
          const double m = v[r].x * v[r].x + v[r].y * v[r].y;
          const uint64_t kr = ((uint64_t)__double_as_longlong(m) & ~(uint64_t)0x7F) | (uint64_t)(0x7F - row);
          key = (mine && !((used >> r) & 1u)) ? umax64(key, kr) : key;
        }
        key = group_max<RB>(key);
        const uint32_t klo = __shfl((uint32_t)key, gbase + RB - 1, 64);
        const uint32_t khi = __shfl((uint32_t)(key >> 32), gbase + RB - 1, 64);
        const uint64_t K = ((uint64_t)khi << 32) | klo;
        // no pivot: the column is zero, or its largest |z|^2 (without the
        // row bits) is below the threshold
        const bool ok = (K >> 7) && __longlong_as_double((long long)(K & ~(uint64_t)0x7F)) >= thr2;
        const int p = ok ? 0x7F - (int)(K & 0x7F) : -1;
        if (mine) {
          // column k becomes 1 on the pivot row, 0 elsewhere; the update then
          // leaves -multiplier in the other rows
          const bool isp = (p >= 0) && (rg == p / RT);
#pragma unroll
          for (int r = 0; r < RT; ++r)
            a[r][kc] = (isp && r == p % RT) ? make_double2(1.0, 0.0) : make_double2(0.0, 0.0);
          if (isp) {
            const c2 iv = cinv((p % RT) ? v[1] : v[0]);
            pinv[s] = iv;
            rowinv[p] = iv;
            colbuf[s][p] = make_double2(0.0, 0.0);    // the pivot row is not updated
            pbuf[s] = p;
            pivrow[k] = p;
            stepof[p] = k;
          }
          if (p < 0 && rg == 0) pbuf[s] = -1;
        }
        __builtin_amdgcn_s_setprio(0);
      }
      __syncthreads();
      const int p = pbuf[s];
      if (p < 0) { singular = true; break; }
      const int pr = p % RT;
      if (wave_live) {
        const c2 inv = pinv[s];
        c2 mi[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) mi[r] = cmul(colbuf[s][rg * RT + r], inv);
        const int src_lane = gbase + p / RT;
        static_assert(RT == 2, "the update branches on the pivot row's slot");
        if (pr) gj_update<RT, CT, RB, 1>(a, mi, src_lane);
        else gj_update<RT, CT, RB, 0>(a, mi, src_lane);
      }
      if (rg == p / RT) used |= 1u << pr;
    }
  }
  if (singular) {
    if (tid == 0) atomicMax(status, ids[blk] + 1);
    return;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int row = rg * RT + r;
    const c2 ri = row < n ? rowinv[row] : make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < CT; ++j) {
      const int col = cg * CT + j;
      if (row < n && col < n) dst[(int64_t)pivrow[col] * n + stepof[row]] = cmul(a[r][j], ri);
    }
  }
}

// ------------------------------------------------------------------ small kernels
__global__ void k_fill(c2 *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_double2(0.0, 0.0);
}

// Sets one flag word from a kernel rather than a memset, so that the work
// around it can be captured into a graph.
__global__ void k_set_i32(int *p, int v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}

// Scatter the near blocks (row-major m x n, tree order) into the panels.
struct Scatter {
  int64_t src, dst;
  int32_t m, n, ld, trans;
};
__global__ void k_scatter(const c2 *__restrict__ near, c2 *__restrict__ W, const Scatter *__restrict__ d) {
  const Scatter s = d[blockIdx.x];
  const int64_t tot = (int64_t)s.m * s.n;
  for (int64_t i = threadIdx.x; i < tot; i += blockDim.x) {
    const int64_t a = i / s.n, b = i % s.n;   // row a of t, column b of s
    const c2 v = near[s.src + i];
    if (!s.trans)
      W[s.dst + b * s.ld + a] = v;           // panel of t: rows of t, columns of s
    else
      W[s.dst + a * s.ld + b] = v;           // panel of s: rows of s, columns of t
  }
}

// b[q, r] = sum over the 14 quadrature points of T+ and T- of
//           c (r_pt - v).pol exp(-j k khat.r_pt)
// Quadrature data per unknown, side and point (10 doubles): r (3), r - v (3),
// the weight (l / 2A) A w with the side's sign, and (r - v) x n (3).
constexpr int kQD = 10;

// b_m = sum over the 14 points of weight exp(-jk khat.r) [alpha (r - v).pol
//      + (1 - alpha) ((r - v) x n).(khat x pol)]: the EFIE excitation
// <f_m, E_inc> (alpha = 1) or the CFIE one of eq. (8), eta0 H_inc = khat x E_inc.
__global__ void k_rhs(const double *__restrict__ qd, const int64_t *__restrict__ dperm, int64_t N,
                      int64_t R, const double *__restrict__ kp, double k, double alpha, c2 *__restrict__ B) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * R) return;
  const int64_t q = idx % N, r = idx / N;
  const int64_t m = dperm[q];
  const double *w = kp + 6 * r;
  const double h[3] = {w[1] * w[5] - w[2] * w[4], w[2] * w[3] - w[0] * w[5], w[0] * w[4] - w[1] * w[3]};
  double re = 0.0, im = 0.0;
  for (int pt = 0; pt < 14; ++pt) {
    const double *d = qd + (m * 14 + pt) * kQD;
    const double ph = -k * (w[0] * d[0] + w[1] * d[1] + w[2] * d[2]);
    double g = d[3] * w[3] + d[4] * w[4] + d[5] * w[5];
    if (alpha != 1.0) g = alpha * g + (1.0 - alpha) * (d[7] * h[0] + d[8] * h[1] + d[9] * h[2]);
    const double f = d[6] * g;
    double sn, cs;
    sincos(ph, &sn, &cs);
    re = fma(f, cs, re);
    im = fma(f, sn, im);
  }
  B[idx] = make_double2(re, im);
}

// Monostatic RCS from the currents when the right-hand side is not the EFIE
// excitation (CFIE): amp = sum_q x_q <f_q, pol exp(-jk khat.r)>, block
// (r, p) -> out[p R + r] = coef |amp|^2 over the unknowns of problem p.
__global__ __launch_bounds__(256) void k_rcs_proj(const double *__restrict__ qd, const int64_t *__restrict__ dperm,
                                                  const c2 *__restrict__ X, int64_t N, const int64_t *__restrict__ soff,
                                                  const double *__restrict__ kp, double k, double coef,
                                                  double *__restrict__ out) {
  const int64_t r = blockIdx.x, R = gridDim.x, p = blockIdx.y;
  const double *w = kp + 6 * r;
  __shared__ double sx[256], sy[256];
  double ax = 0.0, ay = 0.0;
  for (int64_t i = soff[p] + threadIdx.x; i < soff[p + 1]; i += 256) {
    const int64_t m = dperm[i];
    double re = 0.0, im = 0.0;
    for (int pt = 0; pt < 14; ++pt) {
      const double *d = qd + (m * 14 + pt) * kQD;
      const double ph = -k * (w[0] * d[0] + w[1] * d[1] + w[2] * d[2]);
      const double f = d[6] * (d[3] * w[3] + d[4] * w[4] + d[5] * w[5]);
      double sn, cs;
      sincos(ph, &sn, &cs);
      re = fma(f, cs, re);
      im = fma(f, sn, im);
    }
    const c2 x = X[r * N + i];
    ax += re * x.x - im * x.y;
    ay += re * x.y + im * x.x;
  }
  sx[threadIdx.x] = ax;
  sy[threadIdx.x] = ay;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      sx[threadIdx.x] += sx[threadIdx.x + st];
      sy[threadIdx.x] += sy[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p * R + r] = coef * (sx[0] * sx[0] + sy[0] * sy[0]);
}

// Per-column, per-problem reductions, block (r, p) -> out[p R + r]:
// sum_q |a|^2 (mode 0) or coef * |sum_q a b|^2 (mode 1: monostatic RCS
// from b^T x), q over the unknowns of problem p.
__global__ __launch_bounds__(256) void k_colreduce(const c2 *__restrict__ a, const c2 *__restrict__ b,
                                                   int64_t N, const int64_t *__restrict__ soff, double coef,
                                                   int mode, double *__restrict__ out) {
  const int64_t r = blockIdx.x, R = gridDim.x, p = blockIdx.y;
  __shared__ double sx[256], sy[256];
  double x = 0.0, y = 0.0;
  for (int64_t i = soff[p] + threadIdx.x; i < soff[p + 1]; i += 256) {
    const c2 u = a[r * N + i];
    if (mode == 0) {
      x = fma(u.x, u.x, x);
      x = fma(u.y, u.y, x);
    } else {
      const c2 v = b[r * N + i];
      x = fma(u.x, v.x, x);
      x = fma(-u.y, v.y, x);
      y = fma(u.x, v.y, y);
      y = fma(u.y, v.x, y);
    }
  }
  sx[threadIdx.x] = x;
  sy[threadIdx.x] = y;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sx[threadIdx.x] += sx[threadIdx.x + s];
      sy[threadIdx.x] += sy[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p * R + r] = (mode == 0) ? sx[0] : coef * (sx[0] * sx[0] + sy[0] * sy[0]);
}

template <class T>
__global__ void k_copy(T *__restrict__ y, const T *__restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

// eq. (45) per problem and RHS: ||it_1|| / ||it_0|| from the squared norms
__global__ void k_ratio(const double *__restrict__ n0, const double *__restrict__ n1, double *__restrict__ out,
                        int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = sqrt(n1[i]) / sqrt(n0[i]);
}

// y += sgn * w
__global__ void k_axpy(c2 *__restrict__ y, const c2 *__restrict__ w, double sgn, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    c2 a = y[i];
    const c2 b = w[i];
    a.x = fma(sgn, b.x, a.x);
    a.y = fma(sgn, b.y, a.y);
    y[i] = a;
  }
}

// Between the internal N x R block (elimination order, leading dimension N)
// and the caller's layout, where problem p's N_p x R block (RWG order within
// the problem, leading dimension N_p) starts at element R soff[p]; for one
// problem that is the plain N x R block in RWG order.
// dir 0: caller -> internal; dir 1: internal -> caller.
__global__ void k_permute(const c2 *__restrict__ in, c2 *__restrict__ out, const int64_t *__restrict__ dperm,
                          const int64_t *__restrict__ soff, int nseg, int64_t N, int64_t R, int dir) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * R) return;
  const int64_t q = idx % N, r = idx / N;
  const int64_t n = dperm[q];
  const int p = seg_of(soff, nseg, n);
  const int64_t lo = soff[p];
  const int64_t o = R * lo + r * (soff[p + 1] - lo) + (n - lo);
  if (dir == 0)
    out[idx] = in[o];
  else
    out[o] = in[idx];
}

// ------------------------------------------------------------------ near-field fill
// EFIE Galerkin entries of the near blocks on the device (the host build's
// definition, eqs. 2-3 and 9 with e^{jwt}): each entry sums the four triangle
// pairs of its two RWG functions; the outer triangle is the one with the
// smaller id; shared vertex or centroid distance < 2h: 7-point outer rule,
// inner = closed-form 1/R and (r' - rho)/R integrals + 7 points on the
// bounded remainder (exp(-jkR) - 1)/R; < 4h: 7 x 7 points; else 3 x 3.
struct NearMesh {
  const double *xyz, *cen, *area, *len;
  const int32_t *tri, *tp, *tm, *vp, *vm;
  double k, h, cA, cPhi;          // cA = w mu / 4 and cPhi = -1 / (w eps) times j
  const double *nrm;              // unit triangle normals (CFIE)
  int cfie;                       // 0: EFIE entries; 1: alpha EFIE + eta0 (1 - alpha) MFIE
  double alpha, eta0;
};

__device__ __forceinline__ double ddot3(const double *a, const double *b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

template <int NQ>
__device__ void quad_points(const NearMesh &M, int32_t t, double (*p)[3]) {
  const double *v0 = M.xyz + 3 * M.tri[3 * t], *v1 = M.xyz + 3 * M.tri[3 * t + 1], *v2 = M.xyz + 3 * M.tri[3 * t + 2];
  if (NQ == 7) {
    const double s15 = sqrt(15.0);
    const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
    const double b1 = 1.0 - 2.0 * a1, b2 = 1.0 - 2.0 * a2;
    const double B[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {b1, a1, a1}, {a1, b1, a1}, {a1, a1, b1},
                            {b2, a2, a2}, {a2, b2, a2}, {a2, a2, b2}};
    for (int q = 0; q < 7; ++q)
      for (int d = 0; d < 3; ++d) p[q][d] = B[q][0] * v0[d] + B[q][1] * v1[d] + B[q][2] * v2[d];
  } else {
    for (int q = 0; q < 3; ++q)
      for (int d = 0; d < 3; ++d) {
        const double c0 = (q == 0) ? 2.0 / 3.0 : 1.0 / 6.0, c1 = (q == 1) ? 2.0 / 3.0 : 1.0 / 6.0,
                     c2_ = (q == 2) ? 2.0 / 3.0 : 1.0 / 6.0;
        p[q][d] = c0 * v0[d] + c1 * v1[d] + c2_ * v2[d];
      }
  }
}

__device__ __forceinline__ double quad_w(int nq, int q) {
  if (nq == 3) return 1.0 / 3.0;
  const double s15 = sqrt(15.0);
  return q == 0 ? 9.0 / 40.0 : (q < 4 ? (155.0 - s15) / 1200.0 : (155.0 + s15) / 1200.0);
}

// closed-form int_T 1/R dS' and int_T (r' - rho)/R dS' for observation point r
__device__ void tri_potentials(const NearMesh &M, int32_t t, const double *r, double &I1, double Ir[3],
                               double rho[3]) {
  const double *V[3] = {M.xyz + 3 * M.tri[3 * t], M.xyz + 3 * M.tri[3 * t + 1], M.xyz + 3 * M.tri[3 * t + 2]};
  double e1[3], e2[3], n[3];
  for (int d = 0; d < 3; ++d) { e1[d] = V[1][d] - V[0][d]; e2[d] = V[2][d] - V[0][d]; }
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double nn = sqrt(ddot3(n, n));
  for (int d = 0; d < 3; ++d) n[d] /= nn;
  double rv[3];
  for (int d = 0; d < 3; ++d) rv[d] = r[d] - V[0][d];
  const double h = ddot3(rv, n), ah = fabs(h);
  for (int d = 0; d < 3; ++d) rho[d] = r[d] - h * n[d];
  I1 = 0.0;
  Ir[0] = Ir[1] = Ir[2] = 0.0;
  for (int e = 0; e < 3; ++e) {
    const double *pa = V[e], *pb = V[(e + 1) % 3];
    double s[3], u[3], da[3], db[3];
    for (int d = 0; d < 3; ++d) s[d] = pb[d] - pa[d];
    const double ls = sqrt(ddot3(s, s));
    for (int d = 0; d < 3; ++d) s[d] /= ls;
    u[0] = s[1] * n[2] - s[2] * n[1];
    u[1] = s[2] * n[0] - s[0] * n[2];
    u[2] = s[0] * n[1] - s[1] * n[0];
    for (int d = 0; d < 3; ++d) { da[d] = pa[d] - rho[d]; db[d] = pb[d] - rho[d]; }
    const double lp = ddot3(db, s), lm = ddot3(da, s), t0 = ddot3(da, u);
    const double R0sq = t0 * t0 + h * h;
    const double Rp = sqrt(lp * lp + R0sq), Rm = sqrt(lm * lm + R0sq);
    double F = 0.0;
    if (R0sq > 0.0) F = (lp + lm >= 0.0) ? log((Rp + lp) / (Rm + lm)) : log((Rm - lm) / (Rp - lp));
    double beta = 0.0;
    const double dp = R0sq + ah * Rp, dm = R0sq + ah * Rm;
    if (dp > 0.0) beta += atan(t0 * lp / dp);
    if (dm > 0.0) beta -= atan(t0 * lm / dm);
    I1 += t0 * F - ah * beta;
    const double c = 0.5 * (R0sq * F + lp * Rp - lm * Rm);
    for (int d = 0; d < 3; ++d) Ir[d] += c * u[d];
  }
}

// (jw mu / 4) II (r - vO).(r' - vI) G - (j / (w eps)) II G over O x I, outer O
__device__ c2 pair_integral_dev(const NearMesh &M, int32_t O, const double *vO, int32_t I, const double *vI) {
  const int32_t *to = M.tri + 3 * O, *ti = M.tri + 3 * I;
  bool share = false;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) share |= (to[a] == ti[b]);
  double dc[3];
  for (int d = 0; d < 3; ++d) dc[d] = M.cen[3 * O + d] - M.cen[3 * I + d];
  const double d2 = ddot3(dc, dc);
  const double k = M.k, AO = M.area[O], AI = M.area[I];
  const double inv4pi = 1.0 / (4.0 * 3.14159265358979323846);
  double re = 0.0, im = 0.0;     // accumulated complex integral
  if (share || d2 < (2.0 * M.h) * (2.0 * M.h)) {
    double po[7][3], pi[7][3];
    quad_points<7>(M, O, po);
    quad_points<7>(M, I, pi);
    for (int a = 0; a < 7; ++a) {
      double I1, Ir[3], rho[3];
      tri_potentials(M, I, po[a], I1, Ir, rho);
      // s = I1 / 4pi + AI sum_b w_b g_b ; v = (Ir + (rho - vI) I1) / 4pi + AI sum_b w_b (pi_b - vI) g_b
      double s_re = I1 * inv4pi, s_im = 0.0;
      double v_re[3], v_im[3];
      for (int d = 0; d < 3; ++d) { v_re[d] = (Ir[d] + (rho[d] - vI[d]) * I1) * inv4pi; v_im[d] = 0.0; }
      double gs_re = 0.0, gs_im = 0.0, gv_re[3] = {0.0, 0.0, 0.0}, gv_im[3] = {0.0, 0.0, 0.0};
      for (int b = 0; b < 7; ++b) {
        double dd[3];
        for (int d = 0; d < 3; ++d) dd[d] = po[a][d] - pi[b][d];
        const double R = sqrt(ddot3(dd, dd));
        const double x = 0.5 * k * R;
        const double sinc = (x == 0.0) ? 1.0 : sin(x) / x;
        // (exp(-jkR) - 1) / (4 pi R) = -jk/(4 pi) sinc(kR/2) exp(-jkR/2)
        double sx, cx;
        sincos(x, &sx, &cx);
        const double amp = k * inv4pi * sinc;
        const double g_re = -amp * sx, g_im = -amp * cx;      // (-j amp)(cx - j sx)
        const double w = quad_w(7, b);
        gs_re += w * g_re;
        gs_im += w * g_im;
        for (int d = 0; d < 3; ++d) {
          const double f = w * (pi[b][d] - vI[d]);
          gv_re[d] += f * g_re;
          gv_im[d] += f * g_im;
        }
      }
      s_re += AI * gs_re;
      s_im += AI * gs_im;
      double dv_re = 0.0, dv_im = 0.0;
      for (int d = 0; d < 3; ++d) {
        v_re[d] += AI * gv_re[d];
        v_im[d] += AI * gv_im[d];
        dv_re += (po[a][d] - vO[d]) * v_re[d];
        dv_im += (po[a][d] - vO[d]) * v_im[d];
      }
      // cA j dotv + cPhi j s  (cA, cPhi real: the j factor is applied here)
      const double w = quad_w(7, a);
      re += w * (-M.cA * dv_im - M.cPhi * s_im);
      im += w * (M.cA * dv_re + M.cPhi * s_re);
    }
    return make_double2(AO * re, AO * im);
  }
  const int nq = (d2 < (4.0 * M.h) * (4.0 * M.h)) ? 7 : 3;
  double po[7][3], pi[7][3];
  if (nq == 7) {
    quad_points<7>(M, O, po);
    quad_points<7>(M, I, pi);
  } else {
    quad_points<3>(M, O, po);
    quad_points<3>(M, I, pi);
  }
  for (int a = 0; a < nq; ++a) {
    double ro[3];
    for (int d = 0; d < 3; ++d) ro[d] = po[a][d] - vO[d];
    double in_re = 0.0, in_im = 0.0;
    for (int b = 0; b < nq; ++b) {
      double dd[3], ri[3];
      for (int d = 0; d < 3; ++d) { dd[d] = po[a][d] - pi[b][d]; ri[d] = pi[b][d] - vI[d]; }
      const double R = sqrt(ddot3(dd, dd));
      double skr, ckr;
      sincos(k * R, &skr, &ckr);
      const double gr = ckr * (inv4pi / R), gi = -skr * (inv4pi / R);
      // G (j (cA ro.ri + cPhi)) = (gr + j gi) j c = -gi c + j gr c
      const double c = M.cA * ddot3(ro, ri) + M.cPhi;
      const double w = quad_w(nq, b);
      in_re += w * (-gi * c);
      in_im += w * (gr * c);
    }
    const double w = quad_w(nq, a);
    re += w * in_re;
    im += w * in_im;
  }
  return make_double2(AO * AI * re, AO * AI * im);
}

__device__ c2 efie_entry(const NearMesh &M, int64_t m_, int64_t n_) {
  const int64_t a = m_ < n_ ? m_ : n_, b = m_ < n_ ? n_ : m_;
  const int32_t ta[2] = {M.tp[a], M.tm[a]}, tb[2] = {M.tp[b], M.tm[b]};
  const int32_t va[2] = {M.vp[a], M.vm[a]}, vb[2] = {M.vp[b], M.vm[b]};
  double zr = 0.0, zi = 0.0;
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q) {
      const int32_t P = ta[p], Q = tb[q];
      const double *vP = M.xyz + 3 * va[p], *vQ = M.xyz + 3 * vb[q];
      const c2 I = (P <= Q) ? pair_integral_dev(M, P, vP, Q, vQ) : pair_integral_dev(M, Q, vQ, P, vP);
      const double f = ((p == q) ? 1.0 : -1.0) * M.len[a] * M.len[b] / (M.area[P] * M.area[Q]);
      zr += f * I.x;
      zi += f * I.y;
    }
  return make_double2(zr, zi);
}

// int_T (r - r') / R^3 dS' for observation point r: sum_i u_i F_i (the
// divergence theorem on grad'_s (1/R)) plus n sign(d) sum_i beta_i (the
// arctangent terms of tri_potentials).
__device__ void tri_grad_potential(const NearMesh &M, int32_t t, const double *r, double out[3]) {
  const double *V[3] = {M.xyz + 3 * M.tri[3 * t], M.xyz + 3 * M.tri[3 * t + 1], M.xyz + 3 * M.tri[3 * t + 2]};
  double e1[3], e2[3], n[3];
  for (int d = 0; d < 3; ++d) { e1[d] = V[1][d] - V[0][d]; e2[d] = V[2][d] - V[0][d]; }
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double nn = sqrt(ddot3(n, n));
  for (int d = 0; d < 3; ++d) n[d] /= nn;
  double rv[3], rho[3];
  for (int d = 0; d < 3; ++d) rv[d] = r[d] - V[0][d];
  const double h = ddot3(rv, n), ah = fabs(h);
  for (int d = 0; d < 3; ++d) rho[d] = r[d] - h * n[d];
  out[0] = out[1] = out[2] = 0.0;
  double bsum = 0.0;
  for (int e = 0; e < 3; ++e) {
    const double *pa = V[e], *pb = V[(e + 1) % 3];
    double sv[3], u[3], da[3], db[3];
    for (int d = 0; d < 3; ++d) sv[d] = pb[d] - pa[d];
    const double ls = sqrt(ddot3(sv, sv));
    for (int d = 0; d < 3; ++d) sv[d] /= ls;
    u[0] = sv[1] * n[2] - sv[2] * n[1];
    u[1] = sv[2] * n[0] - sv[0] * n[2];
    u[2] = sv[0] * n[1] - sv[1] * n[0];
    for (int d = 0; d < 3; ++d) { da[d] = pa[d] - rho[d]; db[d] = pb[d] - rho[d]; }
    const double lp = ddot3(db, sv), lm = ddot3(da, sv), t0 = ddot3(da, u);
    const double R0sq = t0 * t0 + h * h;
    const double Rp = sqrt(lp * lp + R0sq), Rm = sqrt(lm * lm + R0sq);
    double F = 0.0;
    if (R0sq > 0.0) F = (lp + lm >= 0.0) ? log((Rp + lp) / (Rm + lm)) : log((Rm - lm) / (Rp - lp));
    double beta = 0.0;
    const double dp = R0sq + ah * Rp, dm = R0sq + ah * Rm;
    if (dp > 0.0) beta += atan(t0 * lp / dp);
    if (dm > 0.0) beta -= atan(t0 * lm / dm);
    for (int d = 0; d < 3; ++d) out[d] += u[d] * F;
    bsum += beta;
  }
  const double sg = (h > 0.0) ? 1.0 : (h < 0.0 ? -1.0 : 0.0);
  for (int d = 0; d < 3; ++d) out[d] += n[d] * sg * bsum;
}

// MFIE pair term int_P (r - vP) . [n_P x ((r - vQ) x W_Q(r))] dS, P != Q,
// W_Q(r) = int_Q (r - r') (1 + jkR) exp(-jkR) / (4 pi R^3) dS', written as
// (a.b)(n.W) - (a.W)(n.b).  Same rules as pair_integral_dev: touching or
// < 2h: 7-point outer, closed-form static part + 7 points on the remainder;
// < 4h: 7 x 7; else 3 x 3.
__device__ c2 mfie_pair_dev(const NearMesh &M, int32_t P, const double *vP, int32_t Q, const double *vQ) {
  const int32_t *tp = M.tri + 3 * P, *tq = M.tri + 3 * Q;
  bool share = false;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) share |= (tp[a] == tq[b]);
  double dc[3];
  for (int d = 0; d < 3; ++d) dc[d] = M.cen[3 * P + d] - M.cen[3 * Q + d];
  const double d2 = ddot3(dc, dc);
  const int rule = (share || d2 < (2.0 * M.h) * (2.0 * M.h)) ? 0 : (d2 < (4.0 * M.h) * (4.0 * M.h) ? 1 : 2);
  const int nq = rule == 2 ? 3 : 7;
  double po[7][3], pi[7][3];
  if (nq == 7) {
    quad_points<7>(M, P, po);
    quad_points<7>(M, Q, pi);
  } else {
    quad_points<3>(M, P, po);
    quad_points<3>(M, Q, pi);
  }
  const double *nP = M.nrm + 3 * P;
  const double AQ = M.area[Q], inv4pi = 1.0 / (4.0 * 3.14159265358979323846);
  double acc_re = 0.0, acc_im = 0.0;
  for (int a = 0; a < nq; ++a) {
    double W_re[3] = {0.0, 0.0, 0.0}, W_im[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < nq; ++b) {
      double dd[3];
      for (int d = 0; d < 3; ++d) dd[d] = po[a][d] - pi[b][d];
      const double R = sqrt(ddot3(dd, dd));
      const double x = M.k * R;
      double sx, cx;
      sincos(x, &sx, &cx);
      const double den = inv4pi / (R * R * R);
      // (1 + jx) e^{-jx} - 1, plus 1 for the full kernel
      const double nre = (cx - 1.0 + x * sx) + (rule == 0 ? 0.0 : 1.0), nim = x * cx - sx;
      const double f = quad_w(nq, b) * AQ * den;
      for (int d = 0; d < 3; ++d) {
        W_re[d] += f * nre * dd[d];
        W_im[d] += f * nim * dd[d];
      }
    }
    if (rule == 0) {
      double V[3];
      tri_grad_potential(M, Q, po[a], V);
      for (int d = 0; d < 3; ++d) W_re[d] += V[d] * inv4pi;
    }
    double am[3], bn[3];
    for (int d = 0; d < 3; ++d) { am[d] = po[a][d] - vP[d]; bn[d] = po[a][d] - vQ[d]; }
    const double ab = ddot3(am, bn), nb = ddot3(nP, bn);
    const double nW_re = ddot3(nP, W_re), nW_im = ddot3(nP, W_im);
    const double aW_re = ddot3(am, W_re), aW_im = ddot3(am, W_im);
    const double w = quad_w(nq, a);
    acc_re += w * (ab * nW_re - aW_re * nb);
    acc_im += w * (ab * nW_im - aW_im * nb);
  }
  return make_double2(M.area[P] * acc_re, M.area[P] * acc_im);
}

// MFIE entry (eqs. 6-7): 1/2 <f_m, f_n> - <f_m, n x int f_n x grad' G>, over
// the triangle pairs (+,+), (+,-), (-,+), (-,-) of (m, n).
__device__ __noinline__ c2 mfie_entry(const NearMesh &M, int64_t m_, int64_t n_) {
  const int32_t tm_[2] = {M.tp[m_], M.tm[m_]}, tn_[2] = {M.tp[n_], M.tm[n_]};
  const int32_t vm_[2] = {M.vp[m_], M.vm[m_]}, vn_[2] = {M.vp[n_], M.vm[n_]};
  double zr = 0.0, zi = 0.0;
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q) {
      const int32_t P = tm_[p], Q = tn_[q];
      const double *vP = M.xyz + 3 * vm_[p], *vQ = M.xyz + 3 * vn_[q];
      const double c = ((p == q) ? 1.0 : -1.0) * M.len[m_] * M.len[n_] / (4.0 * M.area[P] * M.area[Q]);
      double vr, vi;
      if (P == Q) {
        double pts[7][3];
        quad_points<7>(M, P, pts);
        double acc = 0.0;
        for (int a = 0; a < 7; ++a) {
          double am[3], bn[3];
          for (int d = 0; d < 3; ++d) { am[d] = pts[a][d] - vP[d]; bn[d] = pts[a][d] - vQ[d]; }
          acc += quad_w(7, a) * ddot3(am, bn);
        }
        vr = 0.5 * M.area[P] * acc;
        vi = 0.0;
      } else {
        const c2 t = mfie_pair_dev(M, P, vP, Q, vQ);
        vr = -t.x;
        vi = -t.y;
      }
      zr += c * vr;
      zi += c * vi;
    }
  return make_double2(zr, zi);
}

// Galerkin entry Z_mn: the EFIE, or (CFIE) the combination of eq. (8).
template <bool CFIE>
__device__ c2 galerkin_entry(const NearMesh &M, int64_t m_, int64_t n_) {
  const c2 e = efie_entry(M, m_, n_);
  if (!CFIE) return e;
  c2 z = make_double2(M.alpha * e.x, M.alpha * e.y);
  if (M.alpha != 1.0) {
    const c2 h = mfie_entry(M, m_, n_);
    const double f = M.eta0 * (1.0 - M.alpha);
    z.x += f * h.x;
    z.y += f * h.y;
  }
  return z;
}

// One workgroup per near block (row-major m x n, rows of group t, columns of s).
template <bool CFIE>
__global__ __launch_bounds__(256) void k_near(NearMesh M, const int64_t *__restrict__ perm,
                                              const int64_t *__restrict__ gptr, const int32_t *__restrict__ ts,
                                              const int64_t *__restrict__ off, c2 *__restrict__ out) {
  const int64_t b = blockIdx.x;
  const int32_t t = ts[2 * b], s = ts[2 * b + 1];
  const int64_t m = gptr[t + 1] - gptr[t], n = gptr[s + 1] - gptr[s];
  for (int64_t i = threadIdx.x; i < m * n; i += blockDim.x) {
    const int64_t r = i / n, c = i % n;
    out[off[b] + i] = galerkin_entry<CFIE>(M, perm[gptr[t] + r], perm[gptr[s] + c]);
  }
}

// ------------------------------------------------------------------ ACA on the device
// Partial-pivoting ACA of one far block per workgroup, the host build's
// rule: first pivot row 0; pivot column = largest residual modulus in the
// row (lowest index on ties); v = row / row[j]; u = residual column j; the
// squared Frobenius norm of the running approximation is updated with the
// cross terms; stop when |u| |v| <= eps ||S||_F; next row = largest |u| over
// unused rows; zero residual rows are skipped.  The raw factors (rank k)
// stay in the workgroup's scratch; rank -1 hands the block back to the host
// (rank limit m n / (m + n) reached, more than kAcaCap terms, or m too
// large for the row bitmap).  Recompression happens on the host.
constexpr int kAcaCap = 96;
constexpr int kAcaMaxRows = 65536;

struct AcaBlock {
  int64_t tlo, m, slo, n, scratch;    // scratch: U (m x cap) then V (n x cap), column-major
};

__device__ __forceinline__ double cabs2(c2 a) { return a.x * a.x + a.y * a.y; }

// block-wide argmax of (value, index): largest value, lowest index on ties
__device__ void block_argmax(double &v, int &i, double *sv, int *si) {
  const int t = threadIdx.x;
  sv[t] = v;
  si[t] = i;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (t < s) {
      const double ov = sv[t + s];
      const int oi = si[t + s];
      if (ov > sv[t] || (ov == sv[t] && oi < si[t])) { sv[t] = ov; si[t] = oi; }
    }
    __syncthreads();
  }
  v = sv[0];
  i = si[0];
  __syncthreads();
}

// block-wide sum of a complex value
__device__ c2 block_csum(c2 a, double *sx, double *sy) {
  const int t = threadIdx.x;
  sx[t] = a.x;
  sy[t] = a.y;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (t < s) { sx[t] += sx[t + s]; sy[t] += sy[t + s]; }
    __syncthreads();
  }
  const c2 r = make_double2(sx[0], sy[0]);
  __syncthreads();
  return r;
}

template <bool CFIE>
__global__ __launch_bounds__(256) void k_aca(NearMesh M, const int64_t *__restrict__ perm,
                                             const AcaBlock *__restrict__ blocks, double eps, c2 *__restrict__ scratch,
                                             int32_t *__restrict__ rank_out) {
  const AcaBlock B = blocks[blockIdx.x];
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ uint32_t used[kAcaMaxRows / 32];
  __shared__ double sv[256], sw[256];
  __shared__ int si[256];
  __shared__ double xpart[4][kAcaCap][4];     // per-wave cross-term sums
  const int64_t m = B.m, n = B.n;
  if (m > kAcaMaxRows) {
    if (tid == 0) rank_out[blockIdx.x] = -1;
    return;
  }
  c2 *U = scratch + B.scratch, *V = U + m * kAcaCap;
  const int64_t *rows = perm + B.tlo, *cols = perm + B.slo;
  for (int64_t w = tid; w < (m + 31) / 32; w += nt) used[w] = 0u;
  __syncthreads();
  const double limit = (double)(m * n) / (double)(m + n);
  int k = 0, result = -2;      // -2: running
  int64_t i = 0;
  double norm2 = 0.0;
  while (result == -2) {
    if ((double)(k + 1) >= limit || k >= kAcaCap) { result = -1; break; }
    // residual row i into V[:, k]
    for (int64_t j = tid; j < n; j += nt) {
      c2 z = galerkin_entry<CFIE>(M, rows[i], cols[j]);
      for (int l = 0; l < k; ++l) {
        const c2 u = U[l * m + i], v = V[l * n + j];
        z.x -= u.x * v.x - u.y * v.y;
        z.y -= u.x * v.y + u.y * v.x;
      }
      V[k * n + j] = z;
    }
    if (tid == 0) used[i >> 5] |= 1u << (i & 31);
    double best = -1.0;
    int jp = 0x7fffffff;
    for (int64_t j = tid; j < n; j += nt) {
      const double a = sqrt(cabs2(V[k * n + j]));
      if (a > best) { best = a; jp = (int)j; }
    }
    block_argmax(best, jp, sv, si);       // also orders the row writes and the bitmap update
    if (best == 0.0) {                    // zero residual row: next unused row, if any
      int nx = 0x7fffffff;
      double one = -1.0;
      for (int64_t a = tid; a < m; a += nt)
        if (!((used[a >> 5] >> (a & 31)) & 1u) && (int)a < nx) { nx = (int)a; one = 1.0; }
      block_argmax(one, nx, sv, si);
      if (one < 0.0) { result = k; break; }
      i = nx;
      continue;
    }
    const c2 piv = V[k * n + jp];
    const double pd = cabs2(piv);
    const c2 pinv = make_double2(piv.x / pd, -piv.y / pd);
    // residual column jp into U[:, k]
    for (int64_t a = tid; a < m; a += nt) {
      c2 z = galerkin_entry<CFIE>(M, rows[a], cols[jp]);
      for (int l = 0; l < k; ++l) {
        const c2 v = V[l * n + jp], u = U[l * m + a];
        z.x -= v.x * u.x - v.y * u.y;
        z.y -= v.x * u.y + v.y * u.x;
      }
      U[k * m + a] = z;
    }
    for (int64_t j = tid; j < n; j += nt) {
      const c2 r = V[k * n + j];
      V[k * n + j] = make_double2(r.x * pinv.x - r.y * pinv.y, r.x * pinv.y + r.y * pinv.x);
    }
    __syncthreads();
    double pu = 0.0, pv = 0.0;
    for (int64_t a = tid; a < m; a += nt) pu += cabs2(U[k * m + a]);
    for (int64_t j = tid; j < n; j += nt) pv += cabs2(V[k * n + j]);
    const c2 s2 = block_csum(make_double2(pu, pv), sv, sw);
    const double nu2 = s2.x, nv2 = s2.y;
    // cross terms sum_l (U_l^H u)(V_l^H v): wave sums into LDS, one barrier
    {
      const int wv = tid >> 6, ln = tid & 63;
      for (int l = 0; l < k; ++l) {
        double q[4] = {0.0, 0.0, 0.0, 0.0};      // U_l^H u (re, im), V_l^H v (re, im)
        for (int64_t a = tid; a < m; a += nt) {
          const c2 x = U[l * m + a], y = U[k * m + a];
          q[0] += x.x * y.x + x.y * y.y;
          q[1] += x.x * y.y - x.y * y.x;
        }
        for (int64_t j = tid; j < n; j += nt) {
          const c2 x = V[l * n + j], y = V[k * n + j];
          q[2] += x.x * y.x + x.y * y.y;
          q[3] += x.x * y.y - x.y * y.x;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
          for (int w = 32; w > 0; w >>= 1) q[c] += __shfl_xor(q[c], w, 64);
        if (ln == 0)
          for (int c = 0; c < 4; ++c) xpart[wv][l][c] = q[c];
      }
    }
    __syncthreads();
    double cross = 0.0;
    for (int l = 0; l < k; ++l) {
      double q[4] = {0.0, 0.0, 0.0, 0.0};
      for (int w = 0; w < 4; ++w)
        for (int c = 0; c < 4; ++c) q[c] += xpart[w][l][c];
      cross += q[0] * q[2] - q[1] * q[3];
    }
    norm2 += 2.0 * cross + nu2 * nv2;
    ++k;
    if (sqrt(nu2 * nv2) <= eps * sqrt(norm2)) { result = k; break; }
    // next row: largest |u| over unused rows
    double bu = -1.0;
    int nx = 0x7fffffff;
    for (int64_t a = tid; a < m; a += nt)
      if (!((used[a >> 5] >> (a & 31)) & 1u)) {
        const double av = sqrt(cabs2(U[(k - 1) * m + a]));
        if (av > bu || (av == bu && (int)a < nx)) { bu = av; nx = (int)a; }
      }
    block_argmax(bu, nx, sv, si);
    if (bu < 0.0) { result = k; break; }   // every row used
    i = nx;
  }
  if (tid == 0) rank_out[blockIdx.x] = result;
}

// Raw factors of the finished blocks into one packed array: U (m x k) then
// V (n x k) per block at pack[b].
__global__ void k_aca_pack(const AcaBlock *__restrict__ blocks, const int32_t *__restrict__ rank,
                           const int64_t *__restrict__ pack, const c2 *__restrict__ scratch, c2 *__restrict__ out) {
  const AcaBlock B = blocks[blockIdx.x];
  const int k = rank[blockIdx.x];
  if (k <= 0) return;
  const c2 *U = scratch + B.scratch, *V = U + B.m * kAcaCap;
  c2 *o = out + pack[blockIdx.x];
  for (int64_t e = threadIdx.x; e < B.m * k; e += blockDim.x) o[e] = U[e];
  for (int64_t e = threadIdx.x; e < B.n * k; e += blockDim.x) o[B.m * k + e] = V[e];
}

// Recompression on the device, step 1: Gram matrices G_U = U^H U and
// G_V = V^H V (k x k, column-major) of each block's packed ACA factors (U
// m x k then V n x k at pack[b]), into gram[goff[b]] (G_U then G_V).  Each
// wave takes entries (p, c), p <= c, in turn; lanes stride over the rows and
// the wave sums them in a fixed order; the lower triangle is the conjugate.
__global__ __launch_bounds__(256) void k_gram(const AcaBlock *__restrict__ blocks, const int32_t *__restrict__ rank,
                                              const int64_t *__restrict__ pack, const int64_t *__restrict__ goff,
                                              const c2 *__restrict__ packed, c2 *__restrict__ gram) {
  const AcaBlock B = blocks[blockIdx.x];
  const int k = rank[blockIdx.x];
  if (k <= 0) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ne = k * (k + 1) / 2;
  for (int side = 0; side < 2; ++side) {
    const c2 *F = packed + pack[blockIdx.x] + (side ? B.m * k : 0);
    const int64_t rows = side ? B.n : B.m;
    c2 *G = gram + goff[blockIdx.x] + (int64_t)side * k * k;
    for (int e = wave; e < ne; e += 4) {
      // e -> (p, c), p <= c, column by column
      int c = 0;
      while ((c + 1) * (c + 2) / 2 <= e) ++c;
      const int p = e - c * (c + 1) / 2;
      const c2 *fp = F + (int64_t)p * rows, *fc = F + (int64_t)c * rows;
      double re = 0.0, im = 0.0;
      for (int64_t i = lane; i < rows; i += 64) {      // conj(f_p) f_c
        const c2 a = fp[i], b = fc[i];
        re = fma(a.x, b.x, re);
        re = fma(a.y, b.y, re);
        im = fma(a.x, b.y, im);
        im = fma(-a.y, b.x, im);
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_xor(re, off);
        im += __shfl_xor(im, off);
      }
      if (lane == 0) {
        G[(int64_t)c * k + p] = make_double2(re, im);
        G[(int64_t)p * k + c] = make_double2(re, -im);
      }
    }
  }
}

// Step 3 (after the host has formed T_U, T_V from the Gram matrices): the
// recompressed factors U' = U T_U (m x r) and V' = V T_V (n x r) into
// out[fpack[b]] (U' then V').  T at tofs[b]: T_U (k x r) then T_V (k x r).
// One row of U or V per thread; T is read from L1 (the same for every row).
__global__ __launch_bounds__(256) void k_apply(const AcaBlock *__restrict__ blocks, const int32_t *__restrict__ rank,
                                               const int32_t *__restrict__ rnew, const int64_t *__restrict__ pack,
                                               const int64_t *__restrict__ tofs, const int64_t *__restrict__ fpack,
                                               const c2 *__restrict__ packed, const c2 *__restrict__ T,
                                               c2 *__restrict__ out) {
  const AcaBlock B = blocks[blockIdx.x];
  const int k = rank[blockIdx.x], r = rnew[blockIdx.x];
  if (k <= 0 || r <= 0) return;
  for (int side = 0; side < 2; ++side) {
    const c2 *F = packed + pack[blockIdx.x] + (side ? B.m * k : 0);
    const c2 *Ts = T + tofs[blockIdx.x] + (int64_t)side * k * r;
    const int64_t rows = side ? B.n : B.m;
    c2 *o = out + fpack[blockIdx.x] + (side ? B.m * r : 0);
    for (int64_t i = threadIdx.x; i < rows; i += blockDim.x)
      for (int c = 0; c < r; ++c) {
        c2 acc = make_double2(0.0, 0.0);
        for (int q = 0; q < k; ++q) cmac(acc, F[(int64_t)q * rows + i], Ts[(int64_t)c * k + q]);
        o[(int64_t)c * rows + i] = acc;
      }
  }
}

// ------------------------------------------------------------------ host side
namespace {

template <class T>
struct DevArray {
  T *p = nullptr;
  size_t n = 0;
  void alloc(size_t count) {
    if (count <= n && p) return;
    release();
    if (count == 0) return;
    HIP_CHECK(hipMalloc((void **)&p, count * sizeof(T)));
    n = count;
  }
  void upload(const std::vector<T> &v, hipStream_t s) {
    alloc(v.size());
    if (!v.empty()) HIP_CHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  DevArray() = default;
  DevArray(const DevArray &) = delete;            // owns its allocation
  DevArray &operator=(const DevArray &) = delete;
  DevArray(DevArray &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevArray &operator=(DevArray &&o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevArray() { release(); }
};

// Pinned host array (hipHostMalloc), grow-only; the source of asynchronous
// uploads that must not wait for earlier work on the stream.  Growing frees
// the old block, so callers synchronise with the device before reusing a
// chunk across calls (every setup ends with a synchronisation).
template <class T>
struct PinnedArray {
  T *p = nullptr;
  size_t n = 0;
  void alloc(size_t count) {
    if (count <= n && p) return;
    release();
    if (count == 0) return;
    HIP_CHECK(hipHostMalloc((void **)&p, count * sizeof(T), hipHostMallocDefault));
    n = count;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
  }
  PinnedArray() = default;
  PinnedArray(const PinnedArray &) = delete;
  PinnedArray &operator=(const PinnedArray &) = delete;
  PinnedArray(PinnedArray &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  PinnedArray &operator=(PinnedArray &&o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~PinnedArray() { release(); }
};

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Host-side bounds check of a tile/term batch against the element counts of
// the A, B and C buffers: every index a kernel can form must be in range.
// Bounds of every tile and term against buffer sizes na, nb, nc (elements).
// A tile with n < 0 covers a run-time number of columns: it is checked for
// one column, with nb / nc the per-column buffer sizes, and its leading
// dimensions must equal them, so that the check holds for any column count.
void validate(const Tile *tiles, size_t ntiles, const std::vector<Term> &terms, int64_t na, int64_t nb,
              int64_t nc, const char *what) {
  for (size_t it = 0; it < ntiles; ++it) {
    const Tile &t0 = tiles[it];
    if (t0.c0 == TILE_PACKED) {
      if (t0.m <= 0 || t0.ldc < t0.m || t0.r0 < 0 || t0.r0 >= t0.m || t0.n < 1 || t0.n > 4 || t0.t_begin < 0 ||
          t0.t_end != t0.t_begin + 1 + t0.n || t0.t_end > (int64_t)terms.size())
        throw Error{HPS_EINVAL, std::string("internal: packed tile in ") + what};
      const Term &a = terms[t0.t_begin];
      const int64_t amax = a.trans ? a.a_off + (int64_t)(t0.m - 1) * a.lda + (a.k - 1)
                                   : a.a_off + (int64_t)(a.k - 1) * a.lda + (t0.m - 1);
      if (a.k <= 0 || a.a_off < 0 || amax >= na || (a.trans ? a.lda < a.k : a.lda < t0.m))
        throw Error{HPS_EINVAL, std::string("internal descriptor out of range (packed A) in ") + what};
      for (int w = 0; w < t0.n; ++w) {
        const Term &d = terms[t0.t_begin + 1 + w];
        if (d.lda < 1 || d.lda > 16 || d.k != a.k || d.ldb < a.k || d.a_off < 0 || d.b_off < 0 ||
            d.a_off + (int64_t)(d.lda - 1) * t0.ldc + (t0.m - 1) >= nc ||
            d.b_off + (int64_t)(d.lda - 1) * d.ldb + (a.k - 1) >= nb)
          throw Error{HPS_EINVAL, std::string("internal descriptor out of range (packed block) in ") + what};
      }
      continue;
    }
    Tile t = t0;
    if (t0.n < 0) {
      if (t0.ldc != nc) throw Error{HPS_EINVAL, std::string("internal: column stride of C in ") + what};
      t.n = 1;
      for (int32_t q = t0.t_begin; q < t0.t_end; ++q)
        if (q >= 0 && q < (int64_t)terms.size() && terms[q].ldb != nb)
          throw Error{HPS_EINVAL, std::string("internal: column stride of B in ") + what};
    }
    if (t.m <= 0 || t.n <= 0) continue;
    if (t.c_off < 0 || t.ldc < t.m || t.c_off + (int64_t)(t.n - 1) * t.ldc + (t.m - 1) >= nc ||
        t.t_begin < 0 || t.t_end > (int64_t)terms.size() || t.t_begin > t.t_end)
      throw Error{HPS_EINVAL, std::string("internal descriptor out of range (C) in ") + what};
    for (int32_t q = t.t_begin; q < t.t_end; ++q) {
      const Term &m = terms[q];
      if (m.k <= 0) continue;
      const int64_t amax = m.trans ? m.a_off + (int64_t)(t.m - 1) * m.lda + (m.k - 1)
                                   : m.a_off + (int64_t)(m.k - 1) * m.lda + (t.m - 1);
      const int64_t bmax = m.b_off + (int64_t)(t.n - 1) * m.ldb + (m.k - 1);
      const bool lda_ok = m.trans ? (m.lda >= m.k) : (m.lda >= t.m);
      if (m.a_off < 0 || m.b_off < 0 || amax >= na || bmax >= nb || !lda_ok || m.ldb < m.k)
        throw Error{HPS_EINVAL, std::string("internal descriptor out of range (A/B) in ") + what};
    }
  }
}

}  // namespace

// Launch of the grouped GEMM in tile shape `shape` (see shape_wr / shape_nb).
template <int MODE>
static void gemm64_launch(int shape, dim3 g, hipStream_t s, const c2 *A, const c2 *B, c2 *C, const Tile *tiles,
                          const Term *terms, int ncols, int nt, int ny, int xo) {
  const dim3 blk(256);
  switch (shape) {
    case 1: hipLaunchKernelGGL((k_gemm<MODE, 2, 2>), g, blk, 0, s, A, B, C, tiles, terms, ncols, nt, ny, xo); break;
    case 2: hipLaunchKernelGGL((k_gemm<MODE, 1, 1>), g, blk, 0, s, A, B, C, tiles, terms, ncols, nt, ny, xo); break;
    case 3: hipLaunchKernelGGL((k_gemm<MODE, 1, 2>), g, blk, 0, s, A, B, C, tiles, terms, ncols, nt, ny, xo); break;
    case 4: hipLaunchKernelGGL((k_gemm<MODE, 2, 4>), g, blk, 0, s, A, B, C, tiles, terms, ncols, nt, ny, xo); break;
    case 5: hipLaunchKernelGGL((k_gemm_lds<MODE>), g, blk, 0, s, A, B, C, tiles, terms, ncols, nt, ny, xo); break;
    case 7: hipLaunchKernelGGL((k_gemm<MODE, 1, 1, 3>), g, blk, 0, s, A, B, C, tiles, terms, ncols, nt, ny, xo); break;
    case 8: hipLaunchKernelGGL((k_gemm<MODE, 2, 2, 3>), g, blk, 0, s, A, B, C, tiles, terms, ncols, nt, ny, xo); break;
    case 9: hipLaunchKernelGGL((k_gemm<MODE, 2, 1, 5>), g, blk, 0, s, A, B, C, tiles, terms, ncols, nt, ny, xo); break;
    case 10: hipLaunchKernelGGL((k_gemm<MODE, 1, 2>), g, blk, 0, s, A, B, C, tiles, terms, ncols, nt, ny, xo); break;
    case 11: hipLaunchKernelGGL((k_gemm_pipe<MODE, 1>), g, blk, 0, s, A, B, C, tiles, terms, ncols, nt, ny, xo); break;
    case 12: hipLaunchKernelGGL((k_gemm_pipe<MODE, 0>), g, blk, 0, s, A, B, C, tiles, terms, ncols, nt, ny, xo); break;
    default: hipLaunchKernelGGL((k_gemm<MODE, 2, 1, 4>), g, blk, 0, s, A, B, C, tiles, terms, ncols, nt, ny, xo); break;
  }
}
template <int MODE, int AT>
static void gemm32_launch(int shape, dim3 g, hipStream_t s, const void *A, const float2 *B, float2 *C,
                          const Tile *tiles, const Term *terms, const float *sc, const int32_t *rp, int ncols, int nt,
                          int ny, int xo) {
  const dim3 blk(256);
  switch (shape) {
    case 1:
    case 8:
      hipLaunchKernelGGL((k_gemm32<MODE, AT, 2, 2>), g, blk, 0, s, A, B, C, tiles, terms, sc, rp, ncols, nt, ny, xo);
      break;
    case 11:      // the pipelined shapes: FP32 A operands only, else the same tile unpipelined
    case 12:
      if (AT == 0) {
        hipLaunchKernelGGL((k_gemm32_pipe<MODE>), g, blk, 0, s, (const float2 *)A, B, C, tiles, terms, ncols, nt, ny,
                           xo);
        break;
      }
      [[fallthrough]];
    case 2:
    case 5:       // the LDS-staged shape has no FP32 kernel: the same 32 x 64 tile without LDS
    case 7:       // FP32 kernels are not built for 3 waves per SIMD: the same tile
      hipLaunchKernelGGL((k_gemm32<MODE, AT, 1, 1>), g, blk, 0, s, A, B, C, tiles, terms, sc, rp, ncols, nt, ny, xo);
      break;
    case 3:
      hipLaunchKernelGGL((k_gemm32<MODE, AT, 1, 2>), g, blk, 0, s, A, B, C, tiles, terms, sc, rp, ncols, nt, ny, xo);
      break;
    case 10:      // shape 3 built for 4 waves per SIMD
      hipLaunchKernelGGL((k_gemm32<MODE, AT, 1, 2, 4>), g, blk, 0, s, A, B, C, tiles, terms, sc, rp, ncols, nt, ny, xo);
      break;
    case 4:
      hipLaunchKernelGGL((k_gemm32<MODE, AT, 2, 4>), g, blk, 0, s, A, B, C, tiles, terms, sc, rp, ncols, nt, ny, xo);
      break;
    default:
      hipLaunchKernelGGL((k_gemm32<MODE, AT, 2, 1>), g, blk, 0, s, A, B, C, tiles, terms, sc, rp, ncols, nt, ny, xo);
      break;
  }
}

struct DeviceState::Impl {
  hipStream_t s;
  void *scratch = nullptr;         // this device's address of the file-scope scratch array
  // problem
  int64_t N = 0, M = 0, R_cap = 0;
  int nseg = 1;                    // independent problems (batch)
  std::vector<int64_t> soff;       // nseg + 1 unknown offsets
  DevArray<int64_t> dsoff;
  double k = 0.0, coef_rcs = 0.0, ratio_warn = 0.1;
  int terms = 2;
  double series_tol = 0.0;         // > 0: stop the series once max ||it_t|| / ||it_0|| < series_tol
  int terms_used = 0;              // terms of the last series
  uint64_t mem_cap = 0;
  // H-matrix on device
  DevArray<c2> near, faruv;
  DevArray<double> quad;           // N x 14 x kQD (RWG order)
  bool nonsym = false;             // CFIE: left coefficients kept, far blocks one way
  double alpha = 1.0;              // CFIE alpha (1: EFIE right-hand side)
  HMatrix hcopy;                   // structure (values not needed after upload)
  std::vector<int64_t> far_m, far_n;
  // Far factors on the device are grouped by the cluster they multiply in
  // stage 1 (dir 0: V_b over the source range of block b; dir 1: U_b over
  // its target range): the factors of one group are contiguous, each still
  // column-major (cluster size x rank), so the group reads as one row-major
  // (sum of ranks) x (cluster size) matrix V^T / U^T.  fu / fv: device
  // offsets of U_b and V_b.
  struct FarGroup { int64_t lo, hi, off, rows; int32_t m0, m1; };
  std::vector<FarGroup> fgroups;
  std::vector<std::pair<int32_t, int32_t>> fmembers;   // (block, dir), group by group
  std::vector<int64_t> fu, fv;
  // plan
  bool ready = false;
  Plan P;
  DevArray<int64_t> dperm;         // elimination position -> RWG
  DevArray<c2> F;                  // factor panels
  DevArray<c2> Wk;                 // working panels (Z~ during the setup)
  std::vector<int64_t> tree2elim;  // tree position -> elimination position
  // solve schedules (independent of R: terms; tiles rebuilt per R)
  struct Sched {
    std::vector<Term> terms;
    std::vector<std::pair<int64_t, int32_t>> targets;   // (c_off, m) per target, rows
    std::vector<int32_t> t_ptr;                          // terms per target
    std::vector<int32_t> ld;                             // ldc per target
    int mode = 0;
  };
  std::vector<Sched> fwd, bwd;     // per level
  Sched dinv, far1, far2, nearmv;
  std::vector<int64_t> toff;       // far intermediate offsets (per block, dir), in units of R
  int64_t t_rows = 0;
  // vector buffers
  DevArray<c2> vB, vY, vW, vS, vI, vX;
  DevArray<c2> vT;
  DevArray<double> red;            // squared norms (2 x nseg x R), then RCS (nseg x R)
  DevArray<double> rat;            // eq. (45) ratios, nseg x R
  DevArray<double> dkp;            // plane waves: khat, pol per RHS
  DevArray<int> status;
  // Captured solve stages (device work only, fixed buffers) per RHS count.
  bool use_graphs = true;
  struct Graph {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    int64_t R = -1;
    int64_t pending = -1;          // R of the last eager run: captured if it comes again
    void reset() {
      if (x) (void)hipGraphExecDestroy(x);
      if (g) (void)hipGraphDestroy(g);
      x = nullptr;
      g = nullptr;
      R = -1;
      pending = -1;
    }
    ~Graph() { reset(); }
  };
  Graph g_pw, g_rhs;
  void drop_graphs() {
    g_pw.reset();
    g_rhs.reset();
  }
  // Flat tile / term arrays shared by many launches: one upload each.
  struct Pool {
    std::vector<Tile> tiles;
    std::vector<Term> terms;
    DevArray<Tile> dtiles;
    DevArray<Term> dterms;
    void clear() {
      tiles.clear();
      terms.clear();
    }
    void upload(hipStream_t st) {
      dtiles.upload(tiles, st);
      dterms.upload(terms, st);
    }
  };
  struct Built {
    int64_t t0 = 0, n_tiles = 0;
    int cls = TC_SWEEP;                // launch class (tile shape from the tuning table)
    // per-RHS sums: sum m k over terms (m = rows of the target), sum m over
    // targets, sum k over terms
    double smk = 0.0, sm = 0.0, sk = 0.0;
    double flops = 0.0, bytes = 0.0;   // for R RHS; algorithmic: each term's A and B once, C read + written once
    void at(int64_t R) {
      flops = 8.0 * (double)R * smk;
      bytes = 32.0 * sm * (double)R + 16.0 * (smk + sk * (double)R);
    }
  };
  // staging and device copies of one chunk of setup levels (grow-only, kept
  // across setups)
  struct Chunk {
    PinnedArray<Tile> h_tiles;
    PinnedArray<Term> h_terms;
    PinnedArray<int64_t> h_inv_off;
    PinnedArray<int32_t> h_inv_n, h_inv_id;
    DevArray<Tile> d_tiles;
    DevArray<Term> d_terms;
    DevArray<int64_t> d_inv_off;
    DevArray<int32_t> d_inv_n, d_inv_id;
    void reserve(int64_t nt, int64_t nm, int64_t ni) {
      h_tiles.alloc((size_t)nt);
      h_terms.alloc((size_t)nm);
      h_inv_off.alloc((size_t)ni);
      h_inv_n.alloc((size_t)ni);
      h_inv_id.alloc((size_t)ni);
      d_tiles.alloc((size_t)nt);
      d_terms.alloc((size_t)nm);
      d_inv_off.alloc((size_t)ni);
      d_inv_n.alloc((size_t)ni);
      d_inv_id.alloc((size_t)ni);
    }
    void upload(int64_t nt, int64_t nm, int64_t ni, hipStream_t st) {
      if (nt) HIP_CHECK(hipMemcpyAsync(d_tiles.p, h_tiles.p, nt * sizeof(Tile), hipMemcpyHostToDevice, st));
      if (nm) HIP_CHECK(hipMemcpyAsync(d_terms.p, h_terms.p, nm * sizeof(Term), hipMemcpyHostToDevice, st));
      if (ni) {
        HIP_CHECK(hipMemcpyAsync(d_inv_off.p, h_inv_off.p, ni * sizeof(int64_t), hipMemcpyHostToDevice, st));
        HIP_CHECK(hipMemcpyAsync(d_inv_n.p, h_inv_n.p, ni * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIP_CHECK(hipMemcpyAsync(d_inv_id.p, h_inv_id.p, ni * sizeof(int32_t), hipMemcpyHostToDevice, st));
      }
    }
  };
  std::deque<Chunk> chunks;       // a deque: growing never relocates the arrays
  // second stream of the setup (default priority) and per-level events
  hipStream_t s2 = nullptr;
  std::vector<hipEvent_t> lev_ev;  // 2 per level: coefficients done, far Schur part done
  void setup_streams(int L) {
    if (!s2) HIP_CHECK(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
    while ((int)lev_ev.size() < 2 * L) {
      hipEvent_t e;
      HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      lev_ev.push_back(e);
    }
  }
  ~Impl() {
    // captured graphs go first: they were recorded on s2 and the level events
    srec.reset();
    drop_graphs();
    for (hipEvent_t e : lev_ev) (void)hipEventDestroy(e);
    if (s2) {
      (void)hipStreamSynchronize(s2);
      (void)hipStreamDestroy(s2);
    }
  }
  // One elimination level of the setup as launches over device arrays: the
  // inverses of its pivots by size class, the right coefficients, and the
  // Schur updates into rows of the next level (main stream) and of the
  // levels after it (second stream).
  struct LevelLaunch {
    struct Inv { int nc; int64_t count; const int64_t *off; const int32_t *n, *id; double flops; };
    std::vector<Inv> inv;
    const Term *terms = nullptr;
    const Tile *coef = nullptr, *schur = nullptr, *schur2 = nullptr;
    int64_t n_coef = 0, n_schur = 0, n_schur2 = 0;
    int sub = 1, sub2 = 1;
    double f_coef = 0.0, b_coef = 0.0, f_schur = 0.0, b_schur = 0.0, f_schur2 = 0.0, b_schur2 = 0.0;
  };
  // Orders between the streams: S2(l) after COEF(l); INV(l) after S2(l - 2)
  // (the last update of its rows from the second stream); S1(l) after
  // S2(l - 1) (both write rows of level l + 1).
  void launch_level(const LevelLaunch &v, int l, c2 *Wd, int shape) {
    if (l >= 2) HIP_CHECK(hipStreamWaitEvent(s, lev_ev[2 * (l - 2) + 1], 0));
    for (const LevelLaunch::Inv &li : v.inv) {
      const unsigned nb = (unsigned)li.count;
      const int64_t pr = prof_begin(3, li.flops, 0.0, li.count);
      if (li.nc == 32)
        hipLaunchKernelGGL(k_inverse<32>, dim3(nb), dim3(256), 0, s, Wd, F.p, li.off, li.n, li.id, status.p);
      else if (li.nc == 64)
        hipLaunchKernelGGL(k_inverse<64>, dim3(nb), dim3(512), 0, s, Wd, F.p, li.off, li.n, li.id, status.p);
      else
        hipLaunchKernelGGL(k_inverse<128>, dim3(nb), dim3(1024), 0, s, Wd, F.p, li.off, li.n, li.id, status.p);
      HIP_CHECK(hipGetLastError());
      prof_end(pr);
    }
    launch_tiles(v.coef, v.terms, v.n_coef, 0, F.p, Wd, F.p, 1, v.f_coef, v.b_coef);
    HIP_CHECK(hipEventRecord(lev_ev[2 * l], s));
    if (l >= 1) HIP_CHECK(hipStreamWaitEvent(s, lev_ev[2 * (l - 1) + 1], 0));
    launch_tiles(v.schur, v.terms, v.n_schur, 1, Wd, F.p, Wd, std::min(v.sub, SUB_Y), v.f_schur, v.b_schur, false, 0,
                 shape, TC_SCHUR);
    HIP_CHECK(hipStreamWaitEvent(s2, lev_ev[2 * l], 0));
    const hipStream_t main_s = s;
    s = s2;                          // launch_tiles and its timing events use s
    try {
      launch_tiles(v.schur2, v.terms, v.n_schur2, 1, Wd, F.p, Wd, std::min(v.sub2, SUB_Y), v.f_schur2, v.b_schur2,
                   false, 0, shape, TC_SCHUR);
    } catch (...) {
      s = main_s;
      throw;
    }
    s = main_s;
    HIP_CHECK(hipEventRecord(lev_ev[2 * l + 1], s2));
  }
  // The setup's device work before the levels: panels cleared, near blocks
  // scattered into them, the singular-block flag cleared.
  DevArray<Scatter> dsc;           // scatter descriptors of the last setup
  int64_t n_scatter = 0;
  void setup_front(c2 *Wd, int64_t PEt) {
    hipLaunchKernelGGL(k_fill, dim3((unsigned)cdiv(PEt, 256)), dim3(256), 0, s, Wd, PEt);
    HIP_CHECK(hipGetLastError());
    if (n_scatter > 0) {
      hipLaunchKernelGGL(k_scatter, dim3((unsigned)n_scatter), dim3(256), 0, s, near.p, Wd, dsc.p);
      HIP_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(64), 0, s, status.p, 0);
    HIP_CHECK(hipGetLastError());
  }
  // Precision form, after the levels: FP32 copies of the factor panels, near
  // blocks and far factors, and the 16-bit far factors with one FP32 scale
  // per factor and block (buffers allocated by the caller).
  DevArray<FarPart> dparts;        // far-factor parts of the last setup
  int64_t n_parts = 0;
  void precision_convert(int64_t PEt) {
    hipLaunchKernelGGL(k_to32, dim3((unsigned)cdiv(PEt, 256)), dim3(256), 0, s, F.p, F32.p, PEt);
    HIP_CHECK(hipGetLastError());
    const int64_t nn = std::max<int64_t>((int64_t)near.n, 1);
    hipLaunchKernelGGL(k_to32, dim3((unsigned)cdiv(nn, 256)), dim3(256), 0, s, near.p, near32.p, (int64_t)near.n);
    HIP_CHECK(hipGetLastError());
    if (faruv.n) {
      hipLaunchKernelGGL(k_to32, dim3((unsigned)cdiv((int64_t)faruv.n, 256)), dim3(256), 0, s, faruv.p, farf32.p,
                         (int64_t)faruv.n);
      HIP_CHECK(hipGetLastError());
    }
    if (n_parts > 0) {
      if (precision == 1)
        hipLaunchKernelGGL(k_far16<1>, dim3((unsigned)n_parts), dim3(256), 0, s, faruv.p, far16.p, fscale.p, dparts.p);
      else
        hipLaunchKernelGGL(k_far16<2>, dim3((unsigned)n_parts), dim3(256), 0, s, faruv.p, far16.p, fscale.p, dparts.p);
      HIP_CHECK(hipGetLastError());
    }
  }
  // Setup replay (graphs == 2): the launches of the last eager setup, over
  // device arrays that stay allocated, with what they were built from.  A
  // later setup with the same plan, H-matrix structure, buffers, form and
  // tile shape runs the same launches on the values now in the buffers, from
  // one graph captured at its first replay.
  bool setup_graphs = false;
  struct SetupRec {
    bool valid = false;
    std::vector<LevelLaunch> levels;
    Plan plan;
    HMatrix hs;                      // structure only
    std::vector<int64_t> soff;
    const void *near_p = nullptr, *faruv_p = nullptr;
    size_t near_n = 0, faruv_n = 0;
    int64_t PEt = 0;
    int precision = 0, shape = 0;
    int64_t kpull = 0;
    bool nonsym = false;
    double flops = 0.0;
    int64_t replays = 0;
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    void reset() {
      if (x) (void)hipGraphExecDestroy(x);
      if (g) (void)hipGraphDestroy(g);
      x = nullptr;
      g = nullptr;
      valid = false;
      levels.clear();
      plan = Plan();
      hs = HMatrix();
      soff.clear();
    }
    ~SetupRec() { reset(); }
  } srec;
  bool setup_replayable(const Plan &P, int shape) const {
    const Plan &a = srec.plan;
    const HMatrix &h = srec.hs;
    return setup_graphs && !prof && srec.valid && srec.precision == precision && srec.shape == shape &&
           srec.kpull == sweep_pull_kmax &&
           srec.nonsym == nonsym && srec.near_p == (const void *)near.p && srec.near_n == near.n &&
           srec.faruv_p == (const void *)faruv.p && srec.faruv_n == faruv.n && srec.soff == soff &&
           h.N == hcopy.N && h.M == hcopy.M && h.nonsym == hcopy.nonsym && h.perm == hcopy.perm &&
           h.gptr == hcopy.gptr && h.near_ts == hcopy.near_ts && h.near_off == hcopy.near_off &&
           h.far_rng == hcopy.far_rng && h.far_rank == hcopy.far_rank && h.far_off == hcopy.far_off &&
           a.M == P.M && a.N == P.N && a.order == P.order && a.pos == P.pos && a.size == P.size && a.uoff == P.uoff &&
           a.later_ptr == P.later_ptr && a.later == P.later && a.col_off == P.col_off && a.width == P.width &&
           a.panel_off == P.panel_off && a.panel_elems == P.panel_elems && a.level == P.level &&
           a.n_levels == P.n_levels && a.level_ptr == P.level_ptr && a.level_piv == P.level_piv &&
           a.n_upper_blocks == P.n_upper_blocks;
  }
  // The whole device part of a setup whose level launches are recorded.
  void setup_device_work() {
    c2 *Wd = Wk.p;
    setup_front(Wd, srec.PEt);
    const int L = (int)srec.levels.size();
    for (int l = 0; l < L; ++l) launch_level(srec.levels[l], l, Wd, srec.shape);
    if (L > 0) HIP_CHECK(hipStreamWaitEvent(s, lev_ev[2 * (L - 1) + 1], 0));   // join the second stream
    if (precision > 0) precision_convert(srec.PEt);
  }
  Pool spool;                      // solve schedules (independent of R)
  int64_t built_R = -1;
  std::vector<Built> b_fwd, b_bwd;
  Built b_dinv, b_far1, b_far2, b_near;
  std::vector<double> solve_flops_parts;

  // Append the tiles of schedule sc (one per 32 target rows; the RHS
  // columns are split over blockIdx.y at launch) and its terms to pool pl.
  // na: elements of A; nb, nc: per-column sizes of the B and C buffers.
  void build(const Sched &sc, Pool &pl, Built &out, int64_t na, int64_t nb, int64_t nc, const char *what, int cls) {
    const int32_t base = (int32_t)pl.terms.size();
    pl.terms.insert(pl.terms.end(), sc.terms.begin(), sc.terms.end());
    out = Built();
    out.cls = cls;
    out.t0 = (int64_t)pl.tiles.size();
    for (size_t t = 0; t < sc.targets.size(); ++t) {
      const int64_t coff = sc.targets[t].first;
      const int32_t m = sc.targets[t].second;
      const int32_t tb = sc.t_ptr[t], te = sc.t_ptr[t + 1];
      for (int64_t r0 = 0; r0 < m; r0 += TM)
        pl.tiles.push_back(Tile{coff, sc.ld[t], (int32_t)r0, -1, m, -1, base + tb, base + te});
      out.sm += m;
      for (int32_t q = tb; q < te; ++q) {
        out.smk += (double)m * sc.terms[q].k;
        out.sk += sc.terms[q].k;
      }
    }
    out.n_tiles = (int64_t)pl.tiles.size() - out.t0;
    validate(pl.tiles.data() + out.t0, (size_t)out.n_tiles, pl.terms, na, nb, nc, what);
  }
  // host side of the solve schedules; upload_solve_pool() copies them
  // nF: length of the factor panels (F may still be allocated by another
  // thread while this runs)
  void build_solve_pool(int64_t nF) {
    spool.clear();
    b_fwd.assign(fwd.size(), Built());
    b_bwd.assign(bwd.size(), Built());
    const int64_t nT = std::max<int64_t>(t_rows, 1);
    for (size_t l = 0; l < fwd.size(); ++l) build(fwd[l], spool, b_fwd[l], nF, N, N, "forward sweep", TC_SWEEP);
    for (size_t l = 0; l < bwd.size(); ++l) build(bwd[l], spool, b_bwd[l], nF, N, N, "back sweep", TC_SWEEP);
    build(dinv, spool, b_dinv, nF, N, N, "D^-1", TC_DINV);
    build(far1, spool, b_far1, (int64_t)faruv.n, N, nT, "far stage 1", TC_FAR1);
    build(far2, spool, b_far2, (int64_t)faruv.n, nT, N, "far stage 2", TC_FAR2);
    build(nearmv, spool, b_near, (int64_t)near.n, N, N, "near matvec", TC_NEAR);
    built_R = -1;
  }
  void upload_solve_pool() { spool.upload(s); }

  // ---- optional per-launch timing with HIP events on the library stream
  // kinds: 0..2 = k_gemm<mode>, 3 = k_inverse
  bool prof = false;
  struct ProfRec { hipEvent_t a, b; int kind; double flops, bytes; int64_t units; int cls; };
  struct LaunchLog { int kind; int64_t units; double flops, bytes, ms; int cls; };
  std::vector<LaunchLog> launch_log;   // every timed launch since profiling was switched on
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> ev_free;
  struct KStat { int64_t launches = 0; double ms = 0.0, flops = 0.0, bytes = 0.0; };
  KStat kstat[4];
  hipEvent_t ev_get() {
    if (ev_free.empty()) {
      hipEvent_t e;
      HIP_CHECK(hipEventCreate(&e));
      return e;
    }
    hipEvent_t e = ev_free.back();
    ev_free.pop_back();
    return e;
  }
  // index of the new record (events on the current stream), -1 when off
  int64_t prof_begin(int kind, double flops, double bytes = 0.0, int64_t units = 0, int cls = -1) {
    if (!prof) return -1;
    prof_recs.push_back(ProfRec{ev_get(), ev_get(), kind, flops, bytes, units, cls});
    HIP_CHECK(hipEventRecord(prof_recs.back().a, s));
    return (int64_t)prof_recs.size() - 1;
  }
  void prof_end(int64_t r) {
    if (r >= 0) HIP_CHECK(hipEventRecord(prof_recs[(size_t)r].b, s));
  }
  void prof_collect() {     // after a stream synchronisation
    for (ProfRec &r : prof_recs) {
      float ms = 0.f;
      HIP_CHECK(hipEventElapsedTime(&ms, r.a, r.b));
      kstat[r.kind].launches += 1;
      kstat[r.kind].ms += ms;
      kstat[r.kind].flops += r.flops;
      kstat[r.kind].bytes += r.bytes;
      if (launch_log.size() < 100000)
        launch_log.push_back(LaunchLog{r.kind, r.units, r.flops, r.bytes, (double)ms, r.cls});
      ev_free.push_back(r.a);
      ev_free.push_back(r.b);
    }
    prof_recs.clear();
  }

  void launch_tiles(const Tile *tiles, const Term *terms, int64_t n_tiles, int mode, const c2 *A, const c2 *B,
                    c2 *C, int sub = 1, double flops = 0.0, double bytes = 0.0, bool wide = false, int ncols = 0,
                    int shape = 0, int cls = -1) {
    if (n_tiles == 0) return;
    // The store-mode launches of a solve (far field, D^-1: long term lists
    // over shared factor rows) take the kernel's XCD-aware order on a
    // one-dimensional grid, where it measured faster; the sweeps and the
    // setup keep the plain (ntiles, sub) grid
    const int xo = (wide && mode == 0) ? 1 : 0;
    const int64_t nwg = cdiv(n_tiles, 8) * 8 * (int64_t)sub;
    if (n_tiles > INT32_MAX || nwg * 256 > (int64_t)UINT32_MAX) throw Error{HPS_EINVAL, "launch too large"};
    dim3 g = xo ? dim3((unsigned)nwg) : dim3((unsigned)n_tiles, (unsigned)sub);
    const int nt = (int)n_tiles;
    const int64_t pr = prof_begin(mode, flops, bytes, n_tiles, cls);
    if (shape == 6 && !(wide && ncols == 1)) shape = 0;    // the vector kernel serves one-column solve tiles only
    if (shape == 6) {
      const dim3 g1((unsigned)n_tiles), blk(256);
      if (mode == 0) hipLaunchKernelGGL(k_gemv<0>, g1, blk, 0, s, A, B, C, tiles, terms, nt);
      else if (mode == 1) hipLaunchKernelGGL(k_gemv<1>, g1, blk, 0, s, A, B, C, tiles, terms, nt);
      else hipLaunchKernelGGL(k_gemv<2>, g1, blk, 0, s, A, B, C, tiles, terms, nt);
    } else if (mode == 0)
      gemm64_launch<0>(shape, g, s, A, B, C, tiles, terms, ncols, nt, sub, xo);
    else if (mode == 1)
      gemm64_launch<1>(shape, g, s, A, B, C, tiles, terms, ncols, nt, sub, xo);
    else
      gemm64_launch<2>(shape, g, s, A, B, C, tiles, terms, ncols, nt, sub, xo);
    HIP_CHECK(hipGetLastError());
    prof_end(pr);
  }
  // Tile shape of each launch class for the current RHS count (solve
  // classes) or for the setup (TC_SCHUR), from the tuning table: the first
  // entry of the class whose rhs_max and group_max bound R and the mean
  // pivot size; shape 0 (32 x 32) when none does.
  std::vector<TuneEntry> tune;
  int64_t sweep_pull_kmax = 0;     // sweep targets with a contraction up to this take one tile set (pull)
  int shape_of[TC_COUNT] = {0, 0, 0, 0, 0, 0};
  int pick_shape(int cls, int64_t R) const {
    const double g = P.M > 0 ? (double)N / (double)P.M : 0.0;
    const int pr = cls == TC_SCHUR ? 0 : precision;     // the setup is FP64 in every form
    for (const TuneEntry &e : tune)
      if (e.cls == cls && R <= e.rhs_max && g <= e.group_max && (e.precision < 0 || e.precision == pr))
        return e.shape;
    return 0;
  }
  void launch(const Built &b, int mode, const c2 *A, const c2 *B, c2 *C) {
    const int sh = shape_of[b.cls];
    launch_tiles(spool.dtiles.p + b.t0, spool.dterms.p, b.n_tiles, mode, A, B, C, (int)cdiv(cur_R, shape_tn(sh)),
                 b.flops, b.bytes, true, (int)cur_R, sh, b.cls);
  }

  // Sizes the vectors for R RHS and the launches' work counts; the tile
  // lists do not depend on R.
  int64_t cur_R = 0;
  void ensure_R(int64_t R) {
    if (R == built_R) return;
    if (R > (int64_t)INT32_MAX / 2 || cdiv(R, TM) > 65535) throw Error{HPS_EINVAL, "too many right-hand sides"};
    drop_graphs();
    cur_R = R;
    for (int c = 0; c < TC_SCHUR; ++c) shape_of[c] = pick_shape(c, R);
    solve_flops_parts.assign(4, 0.0);
    for (auto &b : b_fwd) { b.at(R); solve_flops_parts[0] += b.flops; }
    for (auto &b : b_bwd) { b.at(R); solve_flops_parts[1] += b.flops; }
    b_dinv.at(R);
    solve_flops_parts[2] = b_dinv.flops;
    b_far1.at(R);
    b_far2.at(R);
    solve_flops_parts[3] = b_far1.flops + b_far2.flops;
    b_near.at(R);
    const int64_t NR = N * R;
    vB.alloc(NR); vY.alloc(NR); vW.alloc(NR); vS.alloc(NR); vI.alloc(NR); vX.alloc(NR);
    vT.alloc((size_t)std::max<int64_t>(t_rows, 1) * R);
    red.alloc(3 * R * nseg + 8);
    rat.alloc(R * nseg + 8);
    dkp.alloc(6 * R);
    if (precision) ensure32(R);
    built_R = R;
  }

  // ---- precision form (FP32 solve operands, 16-bit far factors)
  int precision = 0, refine = 0;
  DevArray<float2> F32, near32;
  DevArray<float2> farf32;     // FP32 copy of the far factors (residual pass)
  DevArray<uint32_t> far16;
  DevArray<float> fscale;
  DevArray<int32_t> rowpart;   // first far stage, precision form: scale index of each T row
  DevArray<float2> wB, wY, wW, wS, wI, wX, wT, wR, wZ;

  template <int MODE>
  void g32(const Tile *tiles, const Term *terms, int64_t n, int at, const void *A, const float2 *B, float2 *C,
           double flops, double bytes, int64_t ncols, int shape, int cls) {
    if (n == 0) return;
    if (ncols < 0) ncols = cur_R;
    const int64_t pr = prof_begin(MODE, flops, bytes, n, cls);
    // store mode (far field, D^-1) in the XCD-aware order, as in launch_tiles
    if (shape == 6) shape = 0;                          // no FP32 vector kernel: the 32 x 32 tile
    const int ny = (int)cdiv(ncols, shape_tn(shape)), xo = MODE == 0 ? 1 : 0;
    const int64_t nwg = cdiv(n, 8) * 8 * (int64_t)ny;
    if (n > INT32_MAX || nwg * 256 > (int64_t)UINT32_MAX) throw Error{HPS_EINVAL, "launch too large"};
    dim3 g = xo ? dim3((unsigned)nwg) : dim3((unsigned)n, (unsigned)ny);
    const int nc = (int)ncols, nt = (int)n;
    if (at == 0)
      gemm32_launch<MODE, 0>(shape, g, s, A, B, C, tiles, terms, fscale.p, rowpart.p, nc, nt, ny, xo);
    else if (at == 1)
      gemm32_launch<MODE, 1>(shape, g, s, A, B, C, tiles, terms, fscale.p, rowpart.p, nc, nt, ny, xo);
    else
      gemm32_launch<MODE, 2>(shape, g, s, A, B, C, tiles, terms, fscale.p, rowpart.p, nc, nt, ny, xo);
    HIP_CHECK(hipGetLastError());
    prof_end(pr);
  }
  void launch32(const Built &b, int mode, int at, const void *A, const float2 *B, float2 *C, int64_t ncols = -1,
                int shape = -1) {
    const Tile *t = spool.dtiles.p + b.t0;
    const int sh = shape >= 0 ? shape : shape_of[b.cls];
    if (mode == 0) g32<0>(t, spool.dterms.p, b.n_tiles, at, A, B, C, b.flops, b.bytes, ncols, sh, b.cls);
    else if (mode == 1) g32<1>(t, spool.dterms.p, b.n_tiles, at, A, B, C, b.flops, b.bytes, ncols, sh, b.cls);
    else g32<2>(t, spool.dterms.p, b.n_tiles, at, A, B, C, b.flops, b.bytes, ncols, sh, b.cls);
  }
  void ensure32(int64_t R) {
    const int64_t NR = N * R;
    wB.alloc(NR); wY.alloc(NR); wW.alloc(NR); wS.alloc(NR); wI.alloc(NR); wX.alloc(NR); wR.alloc(NR); wZ.alloc(NR);
    wT.alloc((size_t)std::max<int64_t>(t_rows, 1) * R);
  }
  // Far field in FP32 arithmetic: with the 16-bit factors (at = precision)
  // or with their FP32 copies (at = 0).
  void far32(const float2 *y, float2 *out, int mode, int at) {
    const void *f = at == 0 ? (const void *)farf32.p : (const void *)far16.p;
    launch32(b_far1, 0, at, f, y, wT.p);
    launch32(b_far2, mode, at, f, wT.p, out);
  }
  // out = power series applied to in (FP32); in is kept.  With want_ratio
  // the eq. (45) ratios go to rat (device).  No host synchronisation.
  // far_at: far factors of the series (precision: 16-bit, 0: FP32).
  void series32(int64_t R, const float2 *in, float2 *out, bool want_ratio, int nterms, int far_at) {
    const int64_t NR = N * R, RP = R * nseg;
    const unsigned gb = (unsigned)cdiv(NR, 256);
    const dim3 gn((unsigned)R, (unsigned)nseg);
    copy(wS.p, in, NR);
    for (size_t l = 0; l < b_fwd.size(); ++l) launch32(b_fwd[l], 1, 0, F32.p, wS.p, wS.p);
    launch32(b_dinv, 0, 0, F32.p, wS.p, wI.p);
    const bool adapt = want_ratio && series_tol > 0.0;
    if (want_ratio && nterms > 1) {
      hipLaunchKernelGGL(k_colnorm32, gn, dim3(256), 0, s, wI.p, N, dsoff.p, red.p);
      HIP_CHECK(hipGetLastError());
    }
    copy(out, (const float2 *)wI.p, NR);
    for (int64_t l = (int64_t)b_bwd.size() - 1; l >= 0; --l) launch32(b_bwd[l], 1, 0, F32.p, out, out);
    const float2 *wprev = out;
    float2 *wa = wW.p, *wb = wX.p;
    if (want_ratio) terms_used = 1;
    for (int t = 1; t < nterms; ++t) {
      far32(wprev, wS.p, 0, far_at);
      for (size_t l = 0; l < b_fwd.size(); ++l) launch32(b_fwd[l], 1, 0, F32.p, wS.p, wS.p);
      launch32(b_dinv, 0, 0, F32.p, wS.p, wI.p);
      if (want_ratio && (t == 1 || adapt)) {
        hipLaunchKernelGGL(k_colnorm32, gn, dim3(256), 0, s, wI.p, N, dsoff.p, red.p + RP);
        HIP_CHECK(hipGetLastError());
        if (t == 1) ratio_kernel(RP);
      }
      copy(wa, (const float2 *)wI.p, NR);
      for (int64_t l = (int64_t)b_bwd.size() - 1; l >= 0; --l) launch32(b_bwd[l], 1, 0, F32.p, wa, wa);
      hipLaunchKernelGGL(k_axpy32, dim3(gb), dim3(256), 0, s, out, wa, (t & 1) ? -1.0f : 1.0f, NR);
      HIP_CHECK(hipGetLastError());
      wprev = wa;
      std::swap(wa, wb);
      if (want_ratio) terms_used = t + 1;
      if (adapt && converged(RP)) break;
    }
  }
  // H x in FP32 arithmetic with FP32 near blocks and FP32 far factors.
  void hmatvec32(const float2 *x, float2 *out) {
    launch32(b_near, 0, 0, near32.p, x, out);
    far32(x, out, 2, 0);
  }
  // Precision form of the solve: x = P16 b (the series with 16-bit far
  // factors), then refine passes x <- x + P32 (b - H x), where the residual
  // and the correction series use the FP32 far factors.  In exact arithmetic
  // one pass gives the four-term series; the far-factor rounding of the first
  // pass, x1 - P b = dP b, leaves the pass as (I - P H) dP b = K^2 dP b, so
  // the pass removes it where the series contracts (||K|| < 1) and cannot
  // where it does not.  b in wB, x left in wY.
  void solve32(int64_t R) {
    const int64_t NR = N * R;
    const unsigned gb = (unsigned)cdiv(NR, 256);
    series32(R, wB.p, wY.p, true, terms, precision);
    for (int it = 0; it < refine; ++it) {
      hmatvec32(wY.p, wZ.p);
      hipLaunchKernelGGL(k_sub32, dim3(gb), dim3(256), 0, s, wB.p, wZ.p, wR.p, NR);
      HIP_CHECK(hipGetLastError());
      series32(R, wR.p, wZ.p, false, terms_used, 0);   // the residual pass uses as many terms
      hipLaunchKernelGGL(k_axpy32, dim3(gb), dim3(256), 0, s, wY.p, wZ.p, 1.0f, NR);
      HIP_CHECK(hipGetLastError());
    }
  }

  // FP64 series (plain) or precision form; B in vB, x in vY (FP64), ratios
  // in rat.  Device work only (capturable).
  void solve_any(int64_t R) {
    if (precision == 0) {
      series(R);
      return;
    }
    const int64_t NR = N * R;
    const unsigned gb = (unsigned)cdiv(NR, 256);
    hipLaunchKernelGGL(k_to32, dim3(gb), dim3(256), 0, s, vB.p, wB.p, NR);
    HIP_CHECK(hipGetLastError());
    solve32(R);
    hipLaunchKernelGGL(k_to64, dim3(gb), dim3(256), 0, s, wY.p, vY.p, NR);
    HIP_CHECK(hipGetLastError());
  }

  // Plane-wave solve on the device: RHS from dkp into vB, solve, monostatic
  // RCS of every problem and RHS into red[2 RP, 3 RP).
  void core_pw(int64_t R) {
    const int64_t NR = N * R, RP = R * nseg;
    hipLaunchKernelGGL(k_rhs, dim3((unsigned)cdiv(NR, 256)), dim3(256), 0, s, quad.p, dperm.p, N, R, dkp.p, k, alpha,
                       vB.p);
    HIP_CHECK(hipGetLastError());
    solve_any(R);
    if (alpha == 1.0)          // the right-hand side is the EFIE excitation: sigma from b^T x
      hipLaunchKernelGGL(k_colreduce, dim3((unsigned)R, (unsigned)nseg), dim3(256), 0, s, vB.p, vY.p, N, dsoff.p,
                         coef_rcs, 1, red.p + 2 * RP);
    else
      hipLaunchKernelGGL(k_rcs_proj, dim3((unsigned)R, (unsigned)nseg), dim3(256), 0, s, quad.p, dperm.p, vY.p, N,
                         dsoff.p, dkp.p, k, coef_rcs, red.p + 2 * RP);
    HIP_CHECK(hipGetLastError());
  }
  void core_rhs(int64_t R) { solve_any(R); }

  // Run fn(R) on the stream.  The first solve with a given R after a setup
  // launches directly; a second one captures a graph, which later solves
  // with that R replay.  Direct launches when graphs are off or kernels are
  // timed.
  void run(Graph &g, int64_t R, void (Impl::*fn)(int64_t)) {
    const bool capturable = use_graphs && !prof && series_tol <= 0.0;
    if (!capturable || (!(g.x && g.R == R) && g.pending != R)) {
      if (capturable && !(g.x && g.R == R)) {
        g.reset();
        g.pending = R;
      }
      (this->*fn)(R);
      return;
    }
    if (g.R != R || !g.x) {
      g.reset();
      HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      try {
        (this->*fn)(R);
      } catch (...) {
        hipGraph_t tmp = nullptr;
        (void)hipStreamEndCapture(s, &tmp);
        if (tmp) (void)hipGraphDestroy(tmp);
        throw;
      }
      HIP_CHECK(hipStreamEndCapture(s, &g.g));
      HIP_CHECK(hipGraphInstantiate(&g.x, g.g, nullptr, nullptr, 0));
      g.R = R;
    }
    HIP_CHECK(hipGraphLaunch(g.x, s));
  }

  template <class T>
  void copy(T *y, const T *x, int64_t n) {
    hipLaunchKernelGGL(k_copy<T>, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, y, x, n);
    HIP_CHECK(hipGetLastError());
  }
  void ratio_kernel(int64_t RP) {
    hipLaunchKernelGGL(k_ratio, dim3((unsigned)cdiv(RP, 256)), dim3(256), 0, s, red.p, red.p + RP, rat.p, RP);
    HIP_CHECK(hipGetLastError());
  }

  void sweep_fwd(c2 *v) {
    for (size_t l = 0; l < b_fwd.size(); ++l) launch(b_fwd[l], 1, F.p, v, v);
  }
  void sweep_bwd(c2 *v) {
    for (int64_t l = (int64_t)b_bwd.size() - 1; l >= 0; --l) launch(b_bwd[l], 1, F.p, v, v);
  }
  void far_apply(const c2 *y, c2 *out, int mode) {
    launch(b_far1, 0, faruv.p, y, vT.p);
    launch(b_far2, mode, faruv.p, vT.p, out);
  }
  void colnorm2(const c2 *v, int64_t R, double *dst) {     // nseg x R values
    hipLaunchKernelGGL(k_colreduce, dim3((unsigned)R, (unsigned)nseg), dim3(256), 0, s, v, v, N, dsoff.p, 0.0, 0,
                       dst);
    HIP_CHECK(hipGetLastError());
  }

  // Adaptive series: squared norms of it_0 (red[0, RP)) and it_t (red[RP,
  // 2 RP)) to the host; true when every problem and RHS has
  // ||it_t|| / ||it_0|| < series_tol.  Synchronises the stream.
  bool converged(int64_t RP) {
    std::vector<double> n(2 * RP);
    HIP_CHECK(hipMemcpyAsync(n.data(), red.p, 2 * RP * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    double q = 0.0;
    for (int64_t i = 0; i < RP; ++i) q = std::max(q, n[RP + i] > 0.0 ? std::sqrt(n[RP + i] / n[i]) : 0.0);
    return q < series_tol;
  }

  // Power series (eqs. 25-36) on vB (elimination order, N x R): result in
  // vY, eq. (45) ratios in rat.  Device work only (capturable) unless the
  // term count is adaptive.
  void series(int64_t R) {
    const int64_t NR = N * R, RP = R * nseg;
    const unsigned gb = (unsigned)cdiv(NR, 256);
    copy(vS.p, (const c2 *)vB.p, NR);
    sweep_fwd(vS.p);                               // b~ = A^T b            (eq. 25)
    launch(b_dinv, 0, F.p, vS.p, vI.p);            // it_0 = b_o = D^-1 b~  (eq. 32)
    if (terms > 1) colnorm2(vI.p, R, red.p);
    copy(vY.p, (const c2 *)vI.p, NR);
    sweep_bwd(vY.p);                               // w_0 = A it_0          (eq. 26)
    const c2 *wprev = vY.p;
    terms_used = 1;
    for (int t = 1; t < terms; ++t) {
      far_apply(wprev, vS.p, 0);                   // s = Z_F w_{t-1}
      sweep_fwd(vS.p);                             // A^T s
      launch(b_dinv, 0, F.p, vS.p, vI.p);          // it_t = D^-1 A^T Z_F A it_{t-1}  (eq. 31)
      if (t == 1 || series_tol > 0.0) colnorm2(vI.p, R, red.p + RP);
      if (t == 1) ratio_kernel(RP);                // ||it_1|| / ||it_0||   (eq. 45)
      copy(vW.p, (const c2 *)vI.p, NR);
      sweep_bwd(vW.p);                             // w_t = A it_t
      hipLaunchKernelGGL(k_axpy, dim3(gb), dim3(256), 0, s, vY.p, vW.p, (t & 1) ? -1.0 : 1.0, NR);
      HIP_CHECK(hipGetLastError());
      // keep w_t for the next term
      std::swap(vW.p, vX.p);
      std::swap(vW.n, vX.n);
      wprev = vX.p;
      terms_used = t + 1;
      if (series_tol > 0.0 && converged(RP)) break;
    }
  }
};

// ------------------------------------------------------------------ fixed scratch
// Work vectors of the allocation-free H-matrix product (hmatvec_noalloc):
// one file-scope array per device, held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in); it takes each device's address from hipGetSymbolAddress once,
// with that device current, and uses that address everywhere.
static __device__ __align__(256) unsigned char scratch[HPS_SCRATCH_BYTES];

static void *scratch_address(int dev) {
  static std::mutex mu;
  static std::map<int, void *> addr;       // device ordinal -> address of its copy
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it != addr.end()) return it->second;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    throw Error{HPS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
  addr[dev] = ptr;
  return ptr;
}

DeviceState::DeviceState(int dev, void *strm) : device(dev), stream(strm), own_stream(false) {
  HIP_CHECK(hipSetDevice(dev));
  impl.reset(new Impl());
  if (!strm) {
    hipStream_t s;
    HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    stream = s;
    own_stream = true;
  }
  impl->s = (hipStream_t)stream;
  impl->status.alloc(1);
  impl->scratch = scratch_address(dev);
}

DeviceState::~DeviceState() {
  if (impl) {
    (void)hipStreamSynchronize(impl->s);
    impl.reset();
  }
  if (own_stream && stream) (void)hipStreamDestroy((hipStream_t)stream);
}

void DeviceState::upload(const Mesh &mesh, const HMatrix &H, const hps_params &p, const std::vector<int64_t> &nseg) {
  Impl &I = *impl;
  HIP_CHECK(hipSetDevice(device));
  if (nseg.size() < 2 || nseg.front() != 0 || nseg.back() != H.N) throw Error{HPS_EINVAL, "internal: bad problem offsets"};
  for (size_t q = 0; q + 1 < nseg.size(); ++q)
    if (nseg[q + 1] <= nseg[q]) throw Error{HPS_EINVAL, "internal: empty problem in a batch"};
  I.N = H.N;
  I.M = H.M;
  I.nseg = (int)nseg.size() - 1;
  I.soff = nseg;
  I.dsoff.upload(nseg, I.s);
  I.ready = false;
  I.built_R = -1;
  const double pi = 3.14159265358979323846, c0 = 299792458.0, mu0 = 4.0e-7 * pi;
  I.k = 2.0 * pi * p.freq_hz / c0;
  const double eta = mu0 * c0;
  I.coef_rcs = I.k * I.k * eta * eta / (4.0 * pi);
  I.terms = std::max(1, p.terms);
  I.series_tol = p.series_tol;
  terms = I.terms;
  I.precision = p.precision;
  I.refine = std::max(0, p.refine_passes);
  precision = I.precision;
  refine = I.refine;
  I.ratio_warn = p.ratio_warn;
  I.mem_cap = p.device_mem_cap;
  I.use_graphs = p.graphs != 0;
  I.setup_graphs = p.graphs == 2;
  graphs = p.graphs;
  I.drop_graphs();
  const uint64_t need = (H.near_vals.size() + H.far_uv.size()) * sizeof(c2) + (uint64_t)H.N * 14 * kQD * 8;
  if (I.mem_cap && need > I.mem_cap) throw Error{HPS_ENOMEM, "H-matrix exceeds device_mem_cap"};
  // complex<double> and double2 share their layout: copy straight from the host arrays
  I.near.alloc(H.near_vals.size());
  if (!H.near_vals.empty())
    HIP_CHECK(hipMemcpyAsync(I.near.p, H.near_vals.data(), H.near_vals.size() * sizeof(c2), hipMemcpyHostToDevice, I.s));
  {
    const int64_t nf = H.n_far();
    const int ndir = H.nonsym ? 1 : 2;
    std::map<std::pair<int64_t, int64_t>, std::vector<std::pair<int32_t, int32_t>>> grp;
    for (int64_t b = 0; b < nf; ++b) {
      if (H.far_rank[b] == 0) continue;
      for (int dir = 0; dir < ndir; ++dir) {
        const int64_t lo = H.far_rng[4 * b + (dir == 0 ? 2 : 0)], hi = H.far_rng[4 * b + (dir == 0 ? 3 : 1)];
        grp[{lo, hi}].push_back({(int32_t)b, dir});
      }
    }
    I.fu.assign(nf, 0);
    I.fv.assign(nf, 0);
    I.fgroups.clear();
    I.fmembers.clear();
    std::vector<char> placed_u(nf, 0), placed_v(nf, 0);
    int64_t off = 0;
    for (const auto &g : grp) {
      Impl::FarGroup fg{g.first.first, g.first.second, off, 0, (int32_t)I.fmembers.size(), 0};
      for (const auto &bd : g.second) {
        const int64_t b = bd.first, r = H.far_rank[b];
        const int64_t len = (g.first.second - g.first.first) * r;
        if (bd.second == 0) { I.fv[b] = off; placed_v[b] = 1; }
        else { I.fu[b] = off; placed_u[b] = 1; }
        off += len;
        fg.rows += r;
        I.fmembers.push_back(bd);
      }
      fg.m1 = (int32_t)I.fmembers.size();
      I.fgroups.push_back(fg);
    }
    for (int64_t b = 0; b < nf; ++b) {       // factors stage 1 does not read (U_b of a one-way field; rank 0)
      const int64_t m = H.far_rng[4 * b + 1] - H.far_rng[4 * b], n = H.far_rng[4 * b + 3] - H.far_rng[4 * b + 2];
      if (!placed_u[b]) { I.fu[b] = off; off += m * H.far_rank[b]; }
      if (!placed_v[b]) { I.fv[b] = off; off += n * H.far_rank[b]; }
    }
    if (off != (int64_t)H.far_uv.size()) throw Error{HPS_EINVAL, "internal: far factor layout does not cover the factors"};
    std::vector<cplx> reord(H.far_uv.size());
    for (int64_t b = 0; b < nf; ++b) {
      const int64_t m = H.far_rng[4 * b + 1] - H.far_rng[4 * b], n = H.far_rng[4 * b + 3] - H.far_rng[4 * b + 2];
      const int64_t r = H.far_rank[b];
      std::copy(H.far_uv.begin() + H.far_off[b], H.far_uv.begin() + H.far_off[b] + m * r, reord.begin() + I.fu[b]);
      std::copy(H.far_uv.begin() + H.far_off[b] + m * r, H.far_uv.begin() + H.far_off[b] + (m + n) * r,
                reord.begin() + I.fv[b]);
    }
    I.faruv.alloc(reord.size());
    if (!reord.empty())
      HIP_CHECK(hipMemcpyAsync(I.faruv.p, reord.data(), reord.size() * sizeof(c2), hipMemcpyHostToDevice, I.s));
    HIP_CHECK(hipStreamSynchronize(I.s));
  }
  // structure copy without values
  I.hcopy = HMatrix();
  I.hcopy.N = H.N; I.hcopy.M = H.M; I.hcopy.perm = H.perm; I.hcopy.gptr = H.gptr; I.hcopy.nonsym = H.nonsym;
  I.hcopy.near_ts = H.near_ts; I.hcopy.near_off = H.near_off;
  I.hcopy.far_rng = H.far_rng; I.hcopy.far_rank = H.far_rank; I.hcopy.far_off = H.far_off;
  // quadrature data of the RWG functions for the excitation (7-point rule)
  I.nonsym = H.nonsym;
  I.alpha = p.formulation == 1 ? p.cfie_alpha : 1.0;
  if (H.nonsym && mesh.nrm.size() != 3 * (size_t)mesh.nt) throw Error{HPS_EINVAL, "internal: mesh normals missing"};
  std::vector<double> qd((size_t)H.N * 14 * kQD);
  {
    const double s15 = std::sqrt(15.0);
    const double a1 = (6.0 - s15) / 21.0, w1 = (155.0 - s15) / 1200.0;
    const double a2 = (6.0 + s15) / 21.0, w2 = (155.0 + s15) / 1200.0;
    const double b1 = 1.0 - 2.0 * a1, b2 = 1.0 - 2.0 * a2;
    const double Bc[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {b1, a1, a1}, {a1, b1, a1}, {a1, a1, b1},
                             {b2, a2, a2}, {a2, b2, a2}, {a2, a2, b2}};
    const double Wq[7] = {9.0 / 40.0, w1, w1, w1, w2, w2, w2};
    for (int64_t m = 0; m < H.N; ++m)
      for (int side = 0; side < 2; ++side) {
        const int32_t t = side ? mesh.tm[m] : mesh.tp[m];
        const int32_t v = side ? mesh.vm[m] : mesh.vp[m];
        const double sg = side ? -1.0 : 1.0;
        const double *P0 = &mesh.xyz[3 * mesh.tri[3 * t]], *P1 = &mesh.xyz[3 * mesh.tri[3 * t + 1]],
                     *P2 = &mesh.xyz[3 * mesh.tri[3 * t + 2]];
        const double *V = &mesh.xyz[3 * v];
        for (int q = 0; q < 7; ++q) {
          double *d = &qd[((size_t)m * 14 + side * 7 + q) * kQD];
          for (int c = 0; c < 3; ++c) {
            d[c] = Bc[q][0] * P0[c] + Bc[q][1] * P1[c] + Bc[q][2] * P2[c];
            d[3 + c] = d[c] - V[c];
          }
          d[6] = sg * mesh.len[m] / 2.0 * Wq[q];   // (l / 2A) * A * w
          const double *n = mesh.nrm.empty() ? nullptr : &mesh.nrm[3 * t];
          d[7] = n ? d[4] * n[2] - d[5] * n[1] : 0.0;     // (r - v) x n
          d[8] = n ? d[5] * n[0] - d[3] * n[2] : 0.0;
          d[9] = n ? d[3] * n[1] - d[4] * n[0] : 0.0;
        }
      }
  }
  I.quad.upload(qd, I.s);
  HIP_CHECK(hipStreamSynchronize(I.s));
}

void DeviceState::setup(const Plan &P, const HMatrix &H) {
  Impl &I = *impl;
  HIP_CHECK(hipSetDevice(device));
  hipStream_t s = I.s;
  I.P = P;
  I.tune = tune.entries;
  I.sweep_pull_kmax = tune.sweep_pull_kmax >= 0 ? tune.sweep_pull_kmax : 0;
  // the Schur updates' tile shape (explicit tiles: the one-column vector
  // kernel does not apply, the width is the shape's)
  const int schur_shape = I.pick_shape(TC_SCHUR, 0) == 6 ? 0 : I.pick_shape(TC_SCHUR, 0);
  const int64_t schur_tn = shape_tn(schur_shape);
  const bool schur_packed = schur_shape == 11 || schur_shape == 12;   // packed tiles: k_gemm_pipe only
  I.shape_of[TC_SCHUR] = schur_shape;
  if (I.setup_replayable(P, schur_shape)) {
    // same structure as the recorded setup: its launches on the current
    // values, from the graph (captured here the first time); the solve
    // schedules and captured solves stay valid
    I.ready = false;
    const auto th0 = std::chrono::steady_clock::now();
    if (!I.srec.x) {
      HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      try {
        I.setup_device_work();
      } catch (...) {
        hipGraph_t tmp = nullptr;
        (void)hipStreamEndCapture(s, &tmp);
        if (tmp) (void)hipGraphDestroy(tmp);
        throw;
      }
      HIP_CHECK(hipStreamEndCapture(s, &I.srec.g));
      HIP_CHECK(hipGraphInstantiate(&I.srec.x, I.srec.g, nullptr, nullptr, 0));
    }
    hipEvent_t e0, e1;
    HIP_CHECK(hipEventCreate(&e0));
    HIP_CHECK(hipEventCreate(&e1));
    HIP_CHECK(hipEventRecord(e0, s));
    HIP_CHECK(hipGraphLaunch(I.srec.x, s));
    HIP_CHECK(hipEventRecord(e1, s));
    HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    HIP_CHECK(hipEventDestroy(e0));
    HIP_CHECK(hipEventDestroy(e1));
    times.schur_ms = ms;
    times.inverse_ms = 0.0;
    sched_split[0] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - th0).count();
    for (int q = 1; q < 5; ++q) sched_split[q] = 0.0;
    int st = 0;
    HIP_CHECK(hipMemcpy(&st, I.status.p, sizeof(int), hipMemcpyDeviceToHost));
    if (st > 0) throw Error{HPS_ESINGULAR, "singular scaled diagonal block of group " + std::to_string(P.order[st - 1])};
    I.P.setup_flops = I.srec.flops;
    I.srec.replays += 1;
    I.ready = true;
    return;
  }
  I.srec.reset();
  I.drop_graphs();
  I.ready = false;
  I.built_R = -1;
  const int64_t N = I.N, M = I.M;
  // working and factor panels; a non-symmetric near field (CFIE) also keeps
  // the lower blocks, stored transposed in a second copy of the panel layout
  // at offset PE (Zt_ef = Z~_fe^T, and the left coefficients
  // Lt_ef = D_e^-T Zt_ef in place of C_ef)
  const int64_t PE = std::max<int64_t>(P.panel_elems, 1);
  const int64_t PEt = I.nonsym ? 2 * PE : PE;
  const uint64_t need = 2ull * (uint64_t)PEt * sizeof(c2);
  if (I.mem_cap && need + (I.near.n + I.faruv.n) * sizeof(c2) > I.mem_cap)
    throw Error{HPS_ENOMEM, "setup plan exceeds device_mem_cap"};
  // ---- solve schedules: host work only (the plan and the H-matrix
  // structure), on a thread of their own while the levels are built and run
  std::string sched_err;
  std::vector<int32_t> rowpart_host;
  std::thread sched_thread([&]() {
    try {
      const int L = P.n_levels;
      // ---- solve schedules (terms independent of R)
      auto add_target = [](Impl::Sched &sc, int64_t coff, int32_t m, int32_t ld) {
        sc.targets.push_back({coff, m});
        sc.ld.push_back(ld);
        sc.t_ptr.push_back((int32_t)sc.terms.size());
      };
      auto close = [](Impl::Sched &sc) { sc.t_ptr.push_back((int32_t)sc.terms.size()); };
      // Sweeps (eqs. 25-26), one launch per level.  A group whose whole
      // contraction in a sweep (the summed sizes of the groups it receives
      // terms from) is at most sweep_pull_kmax takes all its terms in one tile
      // set, in the launch before its own level is needed (pull: its rows are
      // read and written once); the others take one tile set per source level
      // (push: many short tiles).  Sources of a launch are final at its start
      // and no group of a launch is both a source and a target.
      //   forward, levels ascending, launch l: b_f -= C_ef^T b_e for e at level l
      //     and push targets f in N+(e); and for pull targets f at level l + 1,
      //     every e with f in N+(e), e ascending;
      //   back, levels descending, launch l: x_e -= C_ef x_f for f at level l
      //     and push targets e with f in N+(e); and for pull targets e at level
      //     l - 1, every f in N+(e), f ascending.
      std::vector<std::vector<std::pair<int32_t, int64_t>>> contrib(M);
      for (int64_t e = 0; e < M; ++e)
        for (int64_t a = P.later_ptr[e]; a < P.later_ptr[e + 1]; ++a) contrib[P.later[a]].push_back({(int32_t)e, P.col_off[a]});
      const int64_t kpull = I.sweep_pull_kmax;
      std::vector<char> pull_f(M, 0), pull_b(M, 0);
      for (int64_t g = 0; g < M; ++g) {
        int64_t kf = 0;
        for (const auto &ce : contrib[g]) kf += P.size[ce.first];
        pull_f[g] = kf > 0 && kf <= kpull;
        const int64_t kb = P.width[g] - P.size[g];
        pull_b[g] = kb > 0 && kb <= kpull;
      }
      auto fwd_term = [&](int32_t e, int64_t coff) {
        return Term{(I.nonsym ? PE : 0) + P.panel_off[e] + coff * P.size[e], P.uoff[e], (int32_t)P.size[e],
                    (int32_t)N, (int32_t)P.size[e], 1};
      };
      auto bwd_term = [&](int32_t e, int64_t coff, int32_t f) {
        return Term{P.panel_off[e] + coff * P.size[e], P.uoff[f], (int32_t)P.size[e], (int32_t)N,
                    (int32_t)P.size[f], 0};
      };
      I.fwd.assign(L, Impl::Sched());
      I.bwd.assign(L, Impl::Sched());
      std::vector<int32_t> slot(M, -1), tgt;
      std::vector<std::vector<Term>> bucket(M);
      auto flush = [&](Impl::Sched &sc) {
        for (int32_t g : tgt) {
          add_target(sc, P.uoff[g], (int32_t)P.size[g], (int32_t)N);
          std::vector<Term> &bk = bucket[slot[g]];
          sc.terms.insert(sc.terms.end(), bk.begin(), bk.end());
          bk.clear();
        }
        for (int32_t g : tgt) slot[g] = -1;
        tgt.clear();
        close(sc);
      };
      auto put = [&](int32_t g, const Term &t) {
        if (slot[g] < 0) { slot[g] = (int32_t)tgt.size(); tgt.push_back(g); }
        bucket[slot[g]].push_back(t);
      };
      for (int l = 0; l < L; ++l) {
        for (int64_t i = P.level_ptr[l]; i < P.level_ptr[l + 1]; ++i) {
          const int32_t e = P.level_piv[i];
          for (int64_t a = P.later_ptr[e]; a < P.later_ptr[e + 1]; ++a)
            if (!pull_f[P.later[a]]) put(P.later[a], fwd_term(e, P.col_off[a]));
        }
        if (l + 1 < L)
          for (int64_t i = P.level_ptr[l + 1]; i < P.level_ptr[l + 2]; ++i) {
            const int32_t f = P.level_piv[i];
            if (pull_f[f])
              for (const auto &ce : contrib[f]) put(f, fwd_term(ce.first, ce.second));
          }
        flush(I.fwd[l]);
        for (int64_t i = P.level_ptr[l]; i < P.level_ptr[l + 1]; ++i) {
          const int32_t f = P.level_piv[i];
          for (const auto &ce : contrib[f])
            if (!pull_b[ce.first]) put(ce.first, bwd_term(ce.first, ce.second, f));
        }
        if (l >= 1)
          for (int64_t i = P.level_ptr[l - 1]; i < P.level_ptr[l]; ++i) {
            const int32_t e = P.level_piv[i];
            if (pull_b[e])
              for (int64_t a = P.later_ptr[e]; a < P.later_ptr[e + 1]; ++a) put(e, bwd_term(e, P.col_off[a], P.later[a]));
          }
        flush(I.bwd[l]);
      }
      I.dinv = Impl::Sched();
      for (int64_t e = 0; e < M; ++e) {
        add_target(I.dinv, P.uoff[e], (int32_t)P.size[e], (int32_t)N);
        I.dinv.terms.push_back(Term{P.panel_off[e], P.uoff[e], (int32_t)P.size[e], (int32_t)N, (int32_t)P.size[e], 0});
      }
      close(I.dinv);
      // far field: stage 1 targets = the rank rows of one factor group (FP64) or
      // of one (block, direction) (precision form: one 16-bit scale per factor
      // and term) x R; stage 2 targets = leaves
      const HMatrix &Hs = I.hcopy;
      const int64_t nf = Hs.n_far();
      I.far1 = Impl::Sched();
      I.far2 = Impl::Sched();
      I.toff.assign(2 * nf, -1);
      int64_t trow = 0;
      auto leaves_in = [&](int64_t lo, int64_t hi, std::vector<int64_t> &out) {
        out.clear();
        int64_t g = std::upper_bound(Hs.gptr.begin(), Hs.gptr.end(), lo) - Hs.gptr.begin() - 1;
        for (; g < Hs.M && Hs.gptr[g] < hi; ++g) out.push_back(g);
      };
      std::vector<std::vector<Term>> leaf_terms(M);
      std::vector<int64_t> lv;
      // T is one column-major matrix of t_rows x R: rows [toff, toff + r) hold
      // T0 = V^T Y[s] (dir 0, feeds the rows of t) or T1 = U^T Y[t] (dir 1, rows of
      // s); a non-symmetric H-matrix stores both orders as separate blocks, each
      // applied in dir 0 only.  The rows of one factor group are contiguous.
      const int ndir = I.nonsym ? 1 : 2;
      for (const Impl::FarGroup &fg : I.fgroups)
        for (int32_t q = fg.m0; q < fg.m1; ++q) {
          const auto bd = I.fmembers[q];
          I.toff[2 * bd.first + bd.second] = trow;
          trow += Hs.far_rank[bd.first];
        }
      I.t_rows = trow;
      const int32_t ldT = (int32_t)std::max<int64_t>(trow, 1);
      for (const Impl::FarGroup &fg : I.fgroups) {
        const int32_t clen = (int32_t)(fg.hi - fg.lo);
        leaves_in(fg.lo, fg.hi, lv);
        // one target: rows of every factor of the group, terms over the leaves;
        // the precision form scales each row by its factor's 16-bit scale
        const auto first = I.fmembers[fg.m0];
        add_target(I.far1, I.toff[2 * first.first + first.second], (int32_t)fg.rows, ldT);
        for (int64_t g : lv) {
          Term tm{fg.off + (Hs.gptr[g] - fg.lo), P.uoff[P.pos[g]], clen, (int32_t)N,
                  (int32_t)(Hs.gptr[g + 1] - Hs.gptr[g]), 1};
          tm.sidx = -2;
          I.far1.terms.push_back(tm);
        }
      }
      if (I.precision > 0) {
        std::vector<int32_t> rp((size_t)std::max<int64_t>(trow, 1), 0);
        for (const Impl::FarGroup &fg : I.fgroups)
          for (int32_t q = fg.m0; q < fg.m1; ++q) {
            const int64_t bb = I.fmembers[q].first;
            const int dir = I.fmembers[q].second;
            for (int64_t i = 0; i < Hs.far_rank[bb]; ++i)
              rp[I.toff[2 * bb + dir] + i] = (int32_t)(2 * bb + (dir == 0 ? 1 : 0));
          }
        rowpart_host = std::move(rp);
      }
      for (int64_t b = 0; b < nf; ++b) {
        const int64_t tlo = Hs.far_rng[4 * b], thi = Hs.far_rng[4 * b + 1];
        const int64_t slo = Hs.far_rng[4 * b + 2], shi = Hs.far_rng[4 * b + 3];
        const int64_t m = thi - tlo, n = shi - slo, r = Hs.far_rank[b];
        if (r == 0) continue;
        const int64_t uo = I.fu[b], vo = I.fv[b];
        leaves_in(tlo, thi, lv);
        for (int64_t g : lv) {
          Term tmu{uo + (Hs.gptr[g] - tlo), I.toff[2 * b], (int32_t)m, ldT, (int32_t)r, 0};
          tmu.sidx = (int32_t)(2 * b);
          leaf_terms[g].push_back(tmu);
        }
        if (ndir == 2) {
          leaves_in(slo, shi, lv);
          for (int64_t g : lv) {
            Term tmv{vo + (Hs.gptr[g] - slo), I.toff[2 * b + 1], (int32_t)n, ldT, (int32_t)r, 0};
            tmv.sidx = (int32_t)(2 * b + 1);
            leaf_terms[g].push_back(tmv);
          }
        }
      }
      close(I.far1);
      for (int64_t g = 0; g < M; ++g) {
        add_target(I.far2, P.uoff[P.pos[g]], (int32_t)(Hs.gptr[g + 1] - Hs.gptr[g]), (int32_t)N);
        I.far2.terms.insert(I.far2.terms.end(), leaf_terms[g].begin(), leaf_terms[g].end());
      }
      close(I.far2);
      // near-field matvec (both triangles of every stored near block; every
      // ordered block once when the field is not symmetric)
      I.nearmv = Impl::Sched();
      std::vector<std::vector<Term>> nt(M);
      for (int64_t b = 0; b < Hs.n_near(); ++b) {
        const int32_t t = Hs.near_ts[2 * b], u = Hs.near_ts[2 * b + 1];
        const int64_t mt = Hs.gptr[t + 1] - Hs.gptr[t], mu = Hs.gptr[u + 1] - Hs.gptr[u];
        // row-major mt x mu == column-major mu x mt with ld mu
        nt[t].push_back(Term{Hs.near_off[b], P.uoff[P.pos[u]], (int32_t)mu, (int32_t)N, (int32_t)mu, 1});
        if (t != u && !I.nonsym)
          nt[u].push_back(Term{Hs.near_off[b], P.uoff[P.pos[t]], (int32_t)mu, (int32_t)N, (int32_t)mt, 0});
      }
      for (int64_t g = 0; g < M; ++g) {
        add_target(I.nearmv, P.uoff[P.pos[g]], (int32_t)(Hs.gptr[g + 1] - Hs.gptr[g]), (int32_t)N);
        I.nearmv.terms.insert(I.nearmv.terms.end(), nt[g].begin(), nt[g].end());
      }
      close(I.nearmv);
      I.build_solve_pool(PEt);
    } catch (const Error &e) {
      sched_err = e.msg;
    } catch (const std::exception &e) {
      sched_err = e.what();
    }
  });
  struct SchedJoin {
    std::thread &t;
    ~SchedJoin() {
      if (t.joinable()) t.join();
    }
  } sched_join{sched_thread};

  // ---- per-level schedules: built per level on host threads (levels are
  // independent), then concatenated in level order into one pool.  The
  // workers start first, so the first levels are built while this thread
  // prepares the panels below.
  const auto th0 = std::chrono::steady_clock::now();
  const int L = P.n_levels;
  I.setup_streams(L);
  struct InvLaunch { int nc; int64_t start, count; int level; double flops; };
  struct GemmLaunch { int64_t t0, n; int sub = 1; double flops = 0.0, bytes = 0.0; };
  struct LevelOut {
    std::vector<int64_t> inv_off[3];
    std::vector<int32_t> inv_n[3], inv_id[3];
    double inv_flops[3] = {0, 0, 0};
    std::vector<Tile> ctiles, stiles, stiles2;   // stiles: targets in rows of the next level; stiles2: the rest
    std::vector<Term> cterms, sterms;
    GemmLaunch coef, schur, schur2;
    double flops = 0.0;
    double col_slots = 0.0, col_active = 0.0;    // Schur tiles: 16-column block slots x 16-k chunks, and the used ones
    std::string err;
  };
  std::vector<LevelOut> lv_out(L);
  const int64_t n_up = P.n_upper_blocks;
  auto build_level = [&](int l, std::vector<double> &tflop, std::vector<int32_t> &slot, std::vector<int32_t> &tgt,
                         std::vector<int32_t> &tcount,
                         std::vector<int32_t> &tjrow, std::vector<int32_t> &pair_id, std::vector<Term> &pair_term) {
    LevelOut &o = lv_out[l];
    for (int64_t i = P.level_ptr[l]; i < P.level_ptr[l + 1]; ++i) {
      const int32_t e = P.level_piv[i];
      const int64_t n = P.size[e];
      if (n > 128) throw Error{HPS_EINVAL, "group larger than 128 unknowns is not supported"};
      const int cls = n <= 32 ? 0 : (n <= 64 ? 1 : 2);
      if (P.panel_off[e] + n * n > P.panel_elems) throw Error{HPS_EINVAL, "internal descriptor out of range (inverse)"};
      o.inv_off[cls].push_back(P.panel_off[e]);
      o.inv_n[cls].push_back((int32_t)n);
      o.inv_id[cls].push_back(e);
      o.inv_flops[cls] += 8.0 * n * n * n;
    }
    // right scaling coefficients C_eN = D_e^-1 Z~_eN (eq. 16)
    for (int64_t i = P.level_ptr[l]; i < P.level_ptr[l + 1]; ++i) {
      const int32_t e = P.level_piv[i];
      const int64_t n = P.size[e], nF = P.width[e] - n;
      if (nF == 0) continue;
      const int32_t tb = (int32_t)o.cterms.size();
      o.cterms.push_back(Term{P.panel_off[e], P.panel_off[e] + n * n, (int32_t)n, (int32_t)n, (int32_t)n, 0});
      for (int64_t r0 = 0; r0 < n; r0 += TM)
        for (int64_t c0 = 0; c0 < nF; c0 += TM)
          o.ctiles.push_back(Tile{P.panel_off[e] + n * n, (int32_t)n, (int32_t)r0, (int32_t)c0, (int32_t)n,
                                  (int32_t)nF, tb, tb + 1});
      o.flops += 8.0 * n * n * nF;
      o.coef.flops += 8.0 * n * n * nF;
      o.coef.bytes += 16.0 * (n * n + 2.0 * n * nF);
      if (I.nonsym) {            // left coefficients (eq. 18), transposed: Lt_eN = D_e^-T Zt_eN
        const int32_t tl = (int32_t)o.cterms.size();
        o.cterms.push_back(Term{P.panel_off[e], PE + P.panel_off[e] + n * n, (int32_t)n, (int32_t)n, (int32_t)n, 1});
        for (int64_t r0 = 0; r0 < n; r0 += TM)
          for (int64_t c0 = 0; c0 < nF; c0 += TM)
            o.ctiles.push_back(Tile{PE + P.panel_off[e] + n * n, (int32_t)n, (int32_t)r0, (int32_t)c0, (int32_t)n,
                                    (int32_t)nF, tl, tl + 1});
        o.flops += 8.0 * n * n * nF;
        o.coef.flops += 8.0 * n * n * nF;
        o.coef.bytes += 16.0 * (n * n + 2.0 * n * nF);
      }
    }
    // Schur targets (j <= k), eq. (21): id = CSR index of (j, k), or n_up + j
    // for (j, j).  Terms are grouped per target by a counting sort in the
    // order of first touch; one whole-block tile per target.  Symmetric:
    // Z~_jk -= Z~_ej^T C_ek.  Non-symmetric: Z~_jk -= Zt_ej^T C_ek for j <= k,
    // and the lower block, stored as Zt_jk = Z~_kj^T, -= Z~_ej^T Lt_ek for
    // k > j (id n_up + M + CSR index).
    pair_id.clear();
    pair_term.clear();
    for (int64_t i = P.level_ptr[l]; i < P.level_ptr[l + 1]; ++i) {
      const int32_t e = P.level_piv[i];
      const int64_t n = P.size[e];
      for (int64_t a = P.later_ptr[e]; a < P.later_ptr[e + 1]; ++a) {
        const int32_t j = P.later[a];
        int64_t q = P.later_ptr[j];
        for (int64_t b = a; b < P.later_ptr[e + 1]; ++b) {
          const int32_t kk = P.later[b];
          int64_t id;
          if (b == a) {
            id = n_up + j;
          } else {
            while (q < P.later_ptr[j + 1] && P.later[q] < kk) ++q;
            if (q >= P.later_ptr[j + 1] || P.later[q] != kk)
              throw Error{HPS_EINVAL, "internal: fill pattern not closed"};
            id = q;
          }
          if (slot[id] < 0) {
            slot[id] = (int32_t)tgt.size();
            tgt.push_back((int32_t)id);
            tcount.push_back(0);
            tjrow.push_back(j);
            tflop.push_back(0.0);
          }
          tcount[slot[id]]++;
          pair_id.push_back(slot[id]);
          pair_term.push_back(Term{(I.nonsym ? PE : 0) + P.panel_off[e] + P.col_off[a] * n,
                                   P.panel_off[e] + P.col_off[b] * n, (int32_t)n, (int32_t)n, (int32_t)n, 1});
          const double f = 8.0 * n * P.size[j] * P.size[kk];
          o.flops += f;
          tflop[slot[id]] += f;
          if (I.nonsym && b != a) {
            const int64_t lid = n_up + M + id;
            if (slot[lid] < 0) {
              slot[lid] = (int32_t)tgt.size();
              tgt.push_back((int32_t)lid);
              tcount.push_back(0);
              tjrow.push_back(j);
              tflop.push_back(0.0);
            }
            tcount[slot[lid]]++;
            pair_id.push_back(slot[lid]);
            pair_term.push_back(Term{P.panel_off[e] + P.col_off[a] * n, PE + P.panel_off[e] + P.col_off[b] * n,
                                     (int32_t)n, (int32_t)n, (int32_t)n, 1});
            o.flops += f;
            tflop[slot[lid]] += f;
          }
        }
      }
    }
    std::vector<int32_t> start(tgt.size() + 1, 0);
    for (size_t x = 0; x < tgt.size(); ++x) start[x + 1] = start[x] + tcount[x];
    o.sterms.resize(start[tgt.size()]);
    std::vector<int32_t> fillp(start.begin(), start.end() - 1);
    for (size_t x = 0; x < pair_id.size(); ++x) o.sterms[fillp[pair_id[x]]++] = pair_term[x];
    // Packed tiles (pipelined shapes): the 16-column blocks of the targets
    // with a single term are grouped by that term's A (one pivot, one row
    // band: the targets of one row band are consecutive here, and a
    // non-symmetric field interleaves two such groups, upper and lower
    // blocks) and dealt four to a tile, one per wave, so a target whose width
    // is not a multiple of 64 leaves no wave of the launch idle.
    struct PackRun {
      int64_t a_off = -1, j = -1;
      bool next = false;
      Term at{};
      std::vector<Term> blocks;
    };
    std::vector<PackRun> runs;          // the open groups of the current row band
    int64_t runs_j = -1;
    auto flush = [&](PackRun &run) {
      if (run.blocks.empty()) return;
      std::vector<Tile> &tl = run.next ? o.stiles : o.stiles2;
      const int64_t mj = P.size[run.j];
      for (size_t i = 0; i < run.blocks.size(); i += 4) {
        const int32_t nw = (int32_t)std::min<size_t>(4, run.blocks.size() - i);
        const int32_t tb = (int32_t)o.sterms.size();
        o.sterms.push_back(run.at);
        for (int32_t w = 0; w < nw; ++w) o.sterms.push_back(run.blocks[i + w]);
        for (int64_t r0 = 0; r0 < mj; r0 += TM)
          tl.push_back(Tile{run.blocks[i].a_off, (int32_t)mj, (int32_t)r0, TILE_PACKED, (int32_t)mj, nw, tb,
                            tb + 1 + nw});
        const double ch = (double)((run.at.k + 15) / 16) * (double)cdiv(mj, TM);
        o.col_slots += 4.0 * ch;
        o.col_active += nw * ch;
      }
      run.blocks.clear();
    };
    auto flush_all = [&]() {
      for (PackRun &r : runs) flush(r);
      runs.clear();
    };
    for (size_t x = 0; x < tgt.size(); ++x) {
      const int64_t id = tgt[x], j = tjrow[x];
      int64_t coff, cols;
      if (id >= n_up + M) {                 // lower block of a non-symmetric field
        const int64_t q = id - n_up - M;
        coff = PE + P.panel_off[j] + P.col_off[q] * P.size[j];
        cols = P.size[P.later[q]];
      } else if (id >= n_up) {
        coff = P.panel_off[j];
        cols = P.size[j];
      } else {
        coff = P.panel_off[j] + P.col_off[id] * P.size[j];
        cols = P.size[P.later[id]];
      }
      // targets in rows of the next level are needed by its pivots first
      const bool next = P.level[j] == l + 1;
      std::vector<Tile> &tl = next ? o.stiles : o.stiles2;
      GemmLaunch &gl = next ? o.schur : o.schur2;
      if (schur_packed && start[x + 1] - start[x] == 1) {
        const Term tm = o.sterms[start[x]];
        if (j != runs_j) {
          flush_all();
          runs_j = j;
        }
        size_t r = 0;
        while (r < runs.size() && runs[r].a_off != tm.a_off) ++r;
        if (r == runs.size()) {
          runs.emplace_back();
          runs[r].a_off = tm.a_off;
          runs[r].j = j;
          runs[r].next = next;
          runs[r].at = tm;
        }
        PackRun &run = runs[r];
        for (int64_t c0 = 0; c0 < cols; c0 += 16)
          run.blocks.push_back(Term{coff + c0 * P.size[j], tm.b_off + c0 * tm.ldb,
                                    (int32_t)std::min<int64_t>(16, cols - c0), tm.ldb, tm.k, 0});
      } else {
        // one explicit tile per (32 x shape-width) sub-tile of the target, so
        // every workgroup of the launch has work (a whole-block tile would be
        // given as many workgroups as the launch's largest target needs)
        for (int64_t r0 = 0; r0 < P.size[j]; r0 += TM)
          for (int64_t c0 = 0; c0 < cols; c0 += schur_tn)
            tl.push_back(Tile{coff, (int32_t)P.size[j], (int32_t)r0, (int32_t)c0, (int32_t)P.size[j],
                              (int32_t)cols, start[x], start[x + 1]});
        double ch = 0.0;
        for (int32_t q = start[x]; q < start[x + 1]; ++q) ch += (double)((o.sterms[q].k + 15) / 16);
        ch *= (double)cdiv(P.size[j], TM);
        o.col_slots += (double)(cdiv(cols, schur_tn) * (schur_tn / 16)) * ch;
        o.col_active += (double)cdiv(cols, 16) * ch;
      }
      gl.flops += tflop[x];
      for (int32_t q = start[x]; q < start[x + 1]; ++q)
        gl.bytes += 16.0 * o.sterms[q].k * ((double)P.size[j] + (double)cols);
      gl.bytes += 32.0 * P.size[j] * cols;
      slot[id] = -1;
    }
    flush_all();
    tgt.clear();
    tcount.clear();
    tjrow.clear();
    tflop.clear();
  };
  // Levels are built on worker threads in level order while this thread
  // uploads and launches them in chunks of growing size (1, 2, 4, ... levels),
  // so the device starts on the first levels while later ones are built.
  std::mutex mu;
  std::condition_variable cv;
  std::vector<char> built(L, 0);
  std::atomic<int> next{0};
  auto worker = [&]() {
    std::vector<int32_t> slot((I.nonsym ? 2 * n_up : n_up) + M, -1), tgt, tcount, tjrow, pair_id;
    std::vector<Term> pair_term;
    std::vector<double> tflop;
    while (true) {
      const int l = next.fetch_add(1);
      if (l >= L) break;
      try {
        build_level(l, tflop, slot, tgt, tcount, tjrow, pair_id, pair_term);
        LevelOut &o = lv_out[l];
        validate(o.ctiles.data(), o.ctiles.size(), o.cterms, PEt, PEt, PEt, "setup");
        validate(o.stiles.data(), o.stiles.size(), o.sterms, PEt, PEt, PEt, "setup");
        validate(o.stiles2.data(), o.stiles2.size(), o.sterms, PEt, PEt, PEt, "setup");
      } catch (const Error &e) {
        lv_out[l].err = e.msg;
      }
      std::lock_guard<std::mutex> lk(mu);
      built[l] = 1;
      cv.notify_all();
    }
  };
  const int nthreads = std::max(1, std::min<int>((int)std::thread::hardware_concurrency(), 16));
  std::vector<std::thread> pool_threads;
  struct Joiner {
    std::vector<std::thread> &t;
    std::atomic<int> &next;
    int L;
    ~Joiner() {
      next.store(L);                    // on an early exit the workers stop after their level
      for (auto &th : t)
        if (th.joinable()) th.join();
    }
  } joiner{pool_threads, next, L};
  for (int t = 0; t < nthreads; ++t) pool_threads.emplace_back(worker);

  // elimination-order permutation
  std::vector<int64_t> dperm(N), t2e(N);
  for (int64_t e = 0; e < M; ++e) {
    const int32_t g = P.order[e];
    for (int64_t i = 0; i < P.size[e]; ++i) {
      dperm[P.uoff[e] + i] = H.perm[H.gptr[g] + i];
      t2e[H.gptr[g] + i] = P.uoff[e] + i;
    }
  }
  // every problem of a batch must own one contiguous range of elimination
  // positions (the per-problem reductions and layouts rely on it)
  for (int64_t e = 0; e < M; ++e) {
    const int64_t lo = H.gptr[P.order[e]];
    const int64_t p = std::upper_bound(I.soff.begin(), I.soff.end(), lo) - I.soff.begin() - 1;
    if (p < 0 || p >= I.nseg || P.uoff[e] < I.soff[p] || P.uoff[e] + P.size[e] > I.soff[p + 1] ||
        H.gptr[P.order[e] + 1] > I.soff[p + 1])
      throw Error{HPS_EINVAL, "internal: a problem of the batch is not contiguous in elimination order"};
  }
  I.tree2elim = t2e;
  I.dperm.upload(dperm, s);

  // column-offset lookup: block (e, f) of panel e
  auto col_of = [&](int64_t e, int64_t f) -> int64_t {
    if (e == f) return 0;
    const int32_t *b = &P.later[P.later_ptr[e]], *en = &P.later[P.later_ptr[e + 1]];
    const int32_t *it = std::lower_bound(b, en, (int32_t)f);
    if (it == en || *it != f) throw Error{HPS_EINVAL, "internal: block missing from fill pattern"};
    return P.col_off[it - &P.later[0]];
  };

  // ---- working panels and factor panels (kept across setups, grow-only)
  I.Wk.alloc(PEt);
  I.F.alloc(PEt);
  c2 *Wd = I.Wk.p;
  std::vector<Scatter> sc(H.n_near());
  for (int64_t b = 0; b < H.n_near(); ++b) {
    const int32_t t = H.near_ts[2 * b], u = H.near_ts[2 * b + 1];
    const int64_t et = P.pos[t], eu = P.pos[u];
    Scatter d;
    d.src = H.near_off[b];
    d.m = (int32_t)(H.gptr[t + 1] - H.gptr[t]);
    d.n = (int32_t)(H.gptr[u + 1] - H.gptr[u]);
    if (et <= eu) {
      d.dst = P.panel_off[et] + col_of(et, eu) * P.size[et];
      d.ld = (int32_t)P.size[et];
      d.trans = 0;
    } else {                     // Z_tu^T: the (u, t) upper block, or the lower block of a non-symmetric field
      d.dst = (I.nonsym ? PE : 0) + P.panel_off[eu] + col_of(eu, et) * P.size[eu];
      d.ld = (int32_t)P.size[eu];
      d.trans = 1;
    }
    const int64_t last = d.trans ? d.dst + (int64_t)(d.m - 1) * d.ld + (d.n - 1) : d.dst + (int64_t)(d.n - 1) * d.ld + (d.m - 1);
    if (d.src < 0 || d.src + (int64_t)d.m * d.n > (int64_t)I.near.n || d.dst < 0 || last >= PEt)
      throw Error{HPS_EINVAL, "internal descriptor out of range (scatter)"};
    sc[b] = d;
  }
  I.dsc.upload(sc, s);
  I.n_scatter = (int64_t)sc.size();
  I.setup_front(Wd, PEt);

  std::vector<int> cut{0};
  for (int w = 1; cut.back() < L; w *= 2) cut.push_back(std::min(L, cut.back() + w));
  const int n_chunks = (int)cut.size() - 1;
  if ((int)I.chunks.size() < n_chunks) I.chunks.resize(n_chunks);
  double flops = 0.0, wait_ms = 0.0, stage_ms = 0.0;
  int64_t n_tiles_all = 0, n_terms_all = 0;
  double col_slots = 0.0, col_active = 0.0;
  const int ncls[3] = {32, 64, 128};
  const bool record = I.setup_graphs && !I.prof;
  if (record) I.srec.levels.resize(L);
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  for (int c = 0; c < n_chunks; ++c) {
    const int lo = cut[c], hi = cut[c + 1];
    {
      const auto tw = std::chrono::steady_clock::now();
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&]() {
        for (int l = lo; l < hi; ++l)
          if (!built[l]) return false;
        return true;
      });
      wait_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tw).count();
    }
    for (int l = lo; l < hi; ++l)
      if (!lv_out[l].err.empty()) throw Error{HPS_EINVAL, lv_out[l].err};
    const auto tst = std::chrono::steady_clock::now();
    Impl::Chunk &ch = I.chunks[c];
    int64_t nt = 0, nm = 0, ni = 0;
    for (int l = lo; l < hi; ++l) {
      const LevelOut &o = lv_out[l];
      nt += (int64_t)(o.ctiles.size() + o.stiles.size() + o.stiles2.size());
      nm += (int64_t)(o.cterms.size() + o.sterms.size());
      for (int k = 0; k < 3; ++k) ni += (int64_t)o.inv_off[k].size();
    }
    ch.reserve(nt, nm, ni);
    // concatenate into the chunk's pinned staging arrays (term indices rebased)
    std::vector<InvLaunch> invl;
    std::vector<GemmLaunch> coefl(hi - lo), schurl(hi - lo), schur2l(hi - lo);
    int64_t ti = 0, mi_ = 0, ii = 0;
    for (int l = lo; l < hi; ++l) {
      LevelOut &o = lv_out[l];
      for (int k = 0; k < 3; ++k) {
        const int64_t cnt = (int64_t)o.inv_off[k].size();
        if (cnt == 0) continue;
        invl.push_back(InvLaunch{ncls[k], ii, cnt, l, o.inv_flops[k]});
        std::copy(o.inv_off[k].begin(), o.inv_off[k].end(), ch.h_inv_off.p + ii);
        std::copy(o.inv_n[k].begin(), o.inv_n[k].end(), ch.h_inv_n.p + ii);
        std::copy(o.inv_id[k].begin(), o.inv_id[k].end(), ch.h_inv_id.p + ii);
        ii += cnt;
      }
      auto append_terms = [&](std::vector<Term> &tm) {
        const int32_t base = (int32_t)mi_;
        std::copy(tm.begin(), tm.end(), ch.h_terms.p + mi_);
        mi_ += (int64_t)tm.size();
        std::vector<Term>().swap(tm);
        return base;
      };
      auto append_tiles = [&](std::vector<Tile> &tl, int32_t base, GemmLaunch &dst, const GemmLaunch &src) {
        dst = src;
        dst.t0 = ti;
        for (const Tile &t0 : tl) {
          Tile t = t0;
          t.t_begin += base;
          t.t_end += base;
          ch.h_tiles.p[ti++] = t;
        }
        dst.n = (int64_t)tl.size();
        std::vector<Tile>().swap(tl);
      };
      append_tiles(o.ctiles, append_terms(o.cterms), coefl[l - lo], o.coef);
      const int32_t sb = append_terms(o.sterms);
      append_tiles(o.stiles, sb, schurl[l - lo], o.schur);
      append_tiles(o.stiles2, sb, schur2l[l - lo], o.schur2);
      flops += o.flops;
      col_slots += o.col_slots;
      col_active += o.col_active;
    }
    ch.upload(nt, nm, ni, s);
    n_tiles_all += nt;
    n_terms_all += nm;
    stage_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tst).count();
    if (c == 0) HIP_CHECK(hipEventRecord(e0, s));
    size_t q = 0;
    for (int l = lo; l < hi; ++l) {
      Impl::LevelLaunch v;
      for (; q < invl.size() && invl[q].level == l; ++q) {
        const InvLaunch &li = invl[q];
        v.inv.push_back(Impl::LevelLaunch::Inv{li.nc, li.count, ch.d_inv_off.p + li.start, ch.d_inv_n.p + li.start,
                                               ch.d_inv_id.p + li.start, li.flops});
      }
      const GemmLaunch &cl = coefl[l - lo], &sl = schurl[l - lo], &sl2 = schur2l[l - lo];
      v.terms = ch.d_terms.p;
      v.coef = ch.d_tiles.p + cl.t0;
      v.n_coef = cl.n;
      v.f_coef = cl.flops;
      v.b_coef = cl.bytes;
      v.schur = ch.d_tiles.p + sl.t0;
      v.n_schur = sl.n;
      v.sub = sl.sub;
      v.f_schur = sl.flops;
      v.b_schur = sl.bytes;
      v.schur2 = ch.d_tiles.p + sl2.t0;
      v.n_schur2 = sl2.n;
      v.sub2 = sl2.sub;
      v.f_schur2 = sl2.flops;
      v.b_schur2 = sl2.bytes;
      I.launch_level(v, l, Wd, schur_shape);
      if (record) I.srec.levels[l] = std::move(v);
    }
  }
  if (L > 0) HIP_CHECK(hipStreamWaitEvent(s, I.lev_ev[2 * (L - 1) + 1], 0));   // join the second stream
  sched_split[0] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - th0).count();
  sched_split[1] = wait_ms;
  sched_split[2] = stage_ms;
  sched_split[3] = (double)n_tiles_all;
  sched_split[4] = (double)n_terms_all;
  sched_split[5] = col_slots;
  sched_split[6] = col_active;
  times.inverse_ms = wait_ms + stage_ms;
  HIP_CHECK(hipEventRecord(e1, s));

  sched_thread.join();
  if (!sched_err.empty()) throw Error{HPS_EINVAL, sched_err};
  if (I.precision > 0) I.rowpart.upload(rowpart_host, s);
  HIP_CHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
  times.schur_ms = ms;
  I.prof_collect();
  HIP_CHECK(hipEventDestroy(e0));
  HIP_CHECK(hipEventDestroy(e1));
  int st = 0;
  HIP_CHECK(hipMemcpy(&st, I.status.p, sizeof(int), hipMemcpyDeviceToHost));
  if (st > 0) throw Error{HPS_ESINGULAR, "singular scaled diagonal block of group " + std::to_string(P.order[st - 1])};
  I.P.setup_flops = flops;

  // ---- precision form: FP32 copies of the factor panels and near blocks,
  // far factors to 16-bit pairs with one FP32 scale per factor per block
  if (I.precision > 0) {
    I.F32.alloc(PEt);
    I.near32.alloc(std::max<int64_t>((int64_t)I.near.n, 1));
    const HMatrix &Hf = I.hcopy;
    std::vector<FarPart> parts(2 * Hf.n_far());
    for (int64_t b = 0; b < Hf.n_far(); ++b) {
      const int64_t m = Hf.far_rng[4 * b + 1] - Hf.far_rng[4 * b], n = Hf.far_rng[4 * b + 3] - Hf.far_rng[4 * b + 2];
      const int64_t r = Hf.far_rank[b];
      parts[2 * b] = FarPart{I.fu[b], m * r};
      parts[2 * b + 1] = FarPart{I.fv[b], n * r};
      if (I.fu[b] + m * r > (int64_t)I.faruv.n || I.fv[b] + n * r > (int64_t)I.faruv.n)
        throw Error{HPS_EINVAL, "internal descriptor out of range (far16)"};
    }
    I.farf32.alloc(std::max<int64_t>((int64_t)I.faruv.n, 1));
    I.far16.alloc(std::max<int64_t>((int64_t)I.faruv.n, 1));
    I.fscale.alloc(std::max<size_t>(parts.size(), 1));
    I.dparts.upload(parts, s);
    I.n_parts = (int64_t)parts.size();
    I.precision_convert(PEt);
    HIP_CHECK(hipStreamSynchronize(s));
  }
  if (record) {                  // what a later setup of the same structure replays
    Impl::SetupRec &r = I.srec;
    r.plan = P;
    r.hs.N = I.hcopy.N; r.hs.M = I.hcopy.M; r.hs.nonsym = I.hcopy.nonsym; r.hs.perm = I.hcopy.perm;
    r.hs.gptr = I.hcopy.gptr; r.hs.near_ts = I.hcopy.near_ts; r.hs.near_off = I.hcopy.near_off;
    r.hs.far_rng = I.hcopy.far_rng; r.hs.far_rank = I.hcopy.far_rank; r.hs.far_off = I.hcopy.far_off;
    r.soff = I.soff;
    r.near_p = I.near.p;
    r.near_n = I.near.n;
    r.faruv_p = I.faruv.p;
    r.faruv_n = I.faruv.n;
    r.PEt = PEt;
    r.precision = I.precision;
    r.shape = schur_shape;
    r.kpull = I.sweep_pull_kmax;
    r.nonsym = I.nonsym;
    r.flops = flops;
    r.valid = true;
  }
  I.upload_solve_pool();
  I.ready = true;
}

// ------------------------------------------------------------------ solves
namespace {
struct Ev {
  hipEvent_t e;
  Ev() { HIP_CHECK(hipEventCreate(&e)); }
  ~Ev() { (void)hipEventDestroy(e); }
};
float elapsed(const Ev &a, const Ev &b) {
  float ms = 0.f;
  HIP_CHECK(hipEventElapsedTime(&ms, a.e, b.e));
  return ms;
}
}  // namespace

// With a library-owned (non-blocking) stream the caller's work on the legacy
// default stream, which produced the inputs or allocated the outputs, must
// finish first.
static void order_after_caller(const DeviceState &d) {
  if (d.own_stream) HIP_CHECK(hipStreamSynchronize(nullptr));
}

static void check_ready(const DeviceState::Impl *I) {
  if (!I->ready) throw Error{HPS_ESTATE, "setup has not been run"};
}

// True for memory that kernels address directly (device or managed
// allocations); false for host memory, which is staged through a copy.
static bool device_pointer(const void *p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();          // plain host memory unknown to the runtime
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Caller block (its layout, N x R c128) -> internal order in dst; a host
// block is copied into stage first.
static void caller_to_internal(DeviceState::Impl &I, const void *src, c2 *dst, c2 *stage, int64_t R) {
  const int64_t N = I.N, NR = N * R;
  const c2 *in = (const c2 *)src;
  if (!device_pointer(src)) {
    HIP_CHECK(hipMemcpyAsync(stage, src, NR * sizeof(c2), hipMemcpyHostToDevice, I.s));
    in = stage;
  }
  hipLaunchKernelGGL(k_permute, dim3((unsigned)cdiv(NR, 256)), dim3(256), 0, I.s, in, dst, I.dperm.p, I.dsoff.p,
                     I.nseg, N, R, 0);
  HIP_CHECK(hipGetLastError());
}

// Internal src -> caller block dst (device, or host through stage).
static void internal_to_caller(DeviceState::Impl &I, const c2 *src, void *dst, c2 *stage, int64_t R) {
  const int64_t N = I.N, NR = N * R;
  const bool dev = device_pointer(dst);
  hipLaunchKernelGGL(k_permute, dim3((unsigned)cdiv(NR, 256)), dim3(256), 0, I.s, src, dev ? (c2 *)dst : stage,
                     I.dperm.p, I.dsoff.p, I.nseg, N, R, 1);
  HIP_CHECK(hipGetLastError());
  if (!dev) HIP_CHECK(hipMemcpyAsync(dst, stage, NR * sizeof(c2), hipMemcpyDeviceToHost, I.s));
}

static void upload_planewaves(DeviceState::Impl &I, int64_t R, const double *khat, const double *pol) {
  std::vector<double> kp(6 * R);
  for (int64_t r = 0; r < R; ++r)
    for (int d = 0; d < 3; ++d) {
      kp[6 * r + d] = khat[3 * r + d];
      kp[6 * r + 3 + d] = pol[3 * r + d];
    }
  HIP_CHECK(hipMemcpyAsync(I.dkp.p, kp.data(), kp.size() * sizeof(double), hipMemcpyHostToDevice, I.s));
  HIP_CHECK(hipStreamSynchronize(I.s));
}

void DeviceState::solve_planewaves(int64_t R, const double *khat, const double *pol, void *X, double *rcs,
                                   double *ratio) {
  Impl &I = *impl;
  check_ready(&I);
  HIP_CHECK(hipSetDevice(device));
  order_after_caller(*this);
  I.ensure_R(R);
  const int64_t N = I.N, NR = N * R, RP = R * I.nseg;
  upload_planewaves(I, R, khat, pol);
  Ev e0, e1, e2;
  HIP_CHECK(hipEventRecord(e0.e, I.s));
  I.run(I.g_pw, R, &Impl::core_pw);
  HIP_CHECK(hipEventRecord(e1.e, I.s));
  if (X) internal_to_caller(I, I.vY.p, X, I.vS.p, R);
  HIP_CHECK(hipEventRecord(e2.e, I.s));
  if (rcs) HIP_CHECK(hipMemcpyAsync(rcs, I.red.p + 2 * RP, RP * sizeof(double), hipMemcpyDeviceToHost, I.s));
  if (ratio && terms > 1) HIP_CHECK(hipMemcpyAsync(ratio, I.rat.p, RP * sizeof(double), hipMemcpyDeviceToHost, I.s));
  HIP_CHECK(hipStreamSynchronize(I.s));
  if (ratio && terms <= 1) std::fill(ratio, ratio + RP, 0.0);
  I.prof_collect();
  times.rhs_ms = 0.0;
  times.sweep_ms = elapsed(e0, e1);
  times.rcs_ms = elapsed(e1, e2);
  times.solve_ms = elapsed(e0, e2);
  last_solve_flops = 0.0;
  for (double f : I.solve_flops_parts) last_solve_flops += f;
}

void DeviceState::solve_rhs(int64_t R, const void *B, void *X, double *ratio) {
  Impl &I = *impl;
  check_ready(&I);
  HIP_CHECK(hipSetDevice(device));
  order_after_caller(*this);
  I.ensure_R(R);
  const int64_t N = I.N, NR = N * R, RP = R * I.nseg;
  Ev e0, e1;
  HIP_CHECK(hipEventRecord(e0.e, I.s));
  caller_to_internal(I, B, I.vB.p, I.vS.p, R);
  I.run(I.g_rhs, R, &Impl::core_rhs);
  internal_to_caller(I, I.vY.p, X, I.vS.p, R);
  HIP_CHECK(hipEventRecord(e1.e, I.s));
  if (ratio && terms > 1) HIP_CHECK(hipMemcpyAsync(ratio, I.rat.p, RP * sizeof(double), hipMemcpyDeviceToHost, I.s));
  HIP_CHECK(hipStreamSynchronize(I.s));
  if (ratio && terms <= 1) std::fill(ratio, ratio + RP, 0.0);
  I.prof_collect();
  times.solve_ms = elapsed(e0, e1);
}

void DeviceState::excitation(int64_t R, const double *khat, const double *pol, void *B) {
  Impl &I = *impl;
  check_ready(&I);
  HIP_CHECK(hipSetDevice(device));
  order_after_caller(*this);
  I.ensure_R(R);
  const int64_t N = I.N, NR = N * R;
  upload_planewaves(I, R, khat, pol);
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)cdiv(NR, 256)), dim3(256), 0, I.s, I.quad.p, I.dperm.p, N, R, I.dkp.p, I.k,
                     I.alpha,
                     I.vB.p);
  HIP_CHECK(hipGetLastError());
  internal_to_caller(I, I.vB.p, B, I.vS.p, R);
  HIP_CHECK(hipStreamSynchronize(I.s));
}

void DeviceState::hmatvec(int64_t R, const void *X, void *Y) {
  Impl &I = *impl;
  check_ready(&I);
  HIP_CHECK(hipSetDevice(device));
  order_after_caller(*this);
  I.ensure_R(R);
  const int64_t N = I.N, NR = N * R;
  const unsigned g = (unsigned)cdiv(NR, 256);
  caller_to_internal(I, X, I.vS.p, I.vW.p, R);
  if (I.precision == 0) {
    I.launch(I.b_near, 0, I.near.p, I.vS.p, I.vI.p);
    I.far_apply(I.vS.p, I.vI.p, 2);
  } else {                                  // FP32 near blocks and far factors
    I.ensure32(R);
    hipLaunchKernelGGL(k_to32, dim3(g), dim3(256), 0, I.s, I.vS.p, I.wS.p, NR);
    I.hmatvec32(I.wS.p, I.wI.p);
    hipLaunchKernelGGL(k_to64, dim3(g), dim3(256), 0, I.s, I.wI.p, I.vI.p, NR);
    HIP_CHECK(hipGetLastError());
  }
  internal_to_caller(I, I.vI.p, Y, I.vW.p, R);
  HIP_CHECK(hipStreamSynchronize(I.s));
}

// Scratch bytes hmatvec_noalloc needs for R columns (each part 256-byte
// aligned): FP64 x, y (internal order) and the far intermediate T; the
// precision form adds FP32 copies of x and y and keeps T in FP32.
static int64_t noalloc_bytes(const DeviceState::Impl &I, int64_t R, int64_t part[5]) {
  auto up = [](int64_t b) { return (b + 255) & ~(int64_t)255; };
  const int64_t NR = I.N * R, TR = std::max<int64_t>(I.t_rows, 1) * R;
  const bool f32 = I.precision != 0;
  part[0] = up(NR * (int64_t)sizeof(c2));                     // x
  part[1] = up(NR * (int64_t)sizeof(c2));                     // y
  part[2] = f32 ? up(NR * (int64_t)sizeof(float2)) : 0;       // x, FP32
  part[3] = f32 ? up(NR * (int64_t)sizeof(float2)) : 0;       // y, FP32
  part[4] = up(TR * (int64_t)(f32 ? sizeof(float2) : sizeof(c2)));
  return part[0] + part[1] + part[2] + part[3] + part[4];
}

// The product of hmatvec on the same kernels, with every work vector in
// the device's scratch array: no allocation, no host copy, no stream
// synchronisation (the result is in Y once the context's stream reaches
// this point).  X and Y must be device memory.
void DeviceState::hmatvec_noalloc(int64_t R, const void *X, void *Y) {
  Impl &I = *impl;
  check_ready(&I);
  HIP_CHECK(hipSetDevice(device));
  if (!device_pointer(X) || !device_pointer(Y))
    throw Error{HPS_EINVAL, "hps_hmatvec_noalloc: X and Y must be device memory"};
  if (cdiv(R, TM) > 65535 || R > (int64_t)INT32_MAX / 2) throw Error{HPS_EINVAL, "too many columns"};
  int64_t part[5];
  const int64_t need = noalloc_bytes(I, R, part);
  if (need > (int64_t)HPS_SCRATCH_BYTES) {
    std::ostringstream o;
    o << "hps_hmatvec_noalloc: " << R << " columns need " << need << " bytes of scratch, the limit is "
      << (int64_t)HPS_SCRATCH_BYTES << " (at most " << (int64_t)HPS_SCRATCH_BYTES * R / need
      << " columns for this problem)";
    throw Error{HPS_EINVAL, o.str()};
  }
  unsigned char *base = (unsigned char *)I.scratch;
  if (!base) throw Error{HPS_EDEVICE, "scratch address not set"};
  c2 *x = (c2 *)base, *y = (c2 *)(base + part[0]);
  float2 *xs = (float2 *)(base + part[0] + part[1]), *ys = (float2 *)(base + part[0] + part[1] + part[2]);
  void *T = base + part[0] + part[1] + part[2] + part[3];
  order_after_caller(*this);
  const bool prof_was = I.prof;        // no timing events here
  I.prof = false;
  try {
    const int64_t NR = I.N * R;
    const unsigned g = (unsigned)cdiv(NR, 256);
    hipLaunchKernelGGL(k_permute, dim3(g), dim3(256), 0, I.s, (const c2 *)X, x, I.dperm.p, I.dsoff.p, I.nseg,
                       I.N, R, 0);
    HIP_CHECK(hipGetLastError());
    // every tile of the near product and of far stage 1 is written in store
    // mode (every row has its diagonal block; T rows are all covered), so
    // nothing left in the scratch by an earlier call is read
    if (I.precision == 0) {
      const Tile *tl = I.spool.dtiles.p;
      const Term *tm = I.spool.dterms.p;
      // tile shapes of the classes for this R, as hmatvec would take them
      const int sn = I.pick_shape(TC_NEAR, R), s1 = I.pick_shape(TC_FAR1, R), s2 = I.pick_shape(TC_FAR2, R);
      I.launch_tiles(tl + I.b_near.t0, tm, I.b_near.n_tiles, 0, I.near.p, x, y, (int)cdiv(R, shape_tn(sn)), 0.0, 0.0,
                     true, (int)R, sn);
      I.launch_tiles(tl + I.b_far1.t0, tm, I.b_far1.n_tiles, 0, I.faruv.p, x, (c2 *)T, (int)cdiv(R, shape_tn(s1)), 0.0,
                     0.0, true, (int)R, s1);
      I.launch_tiles(tl + I.b_far2.t0, tm, I.b_far2.n_tiles, 2, I.faruv.p, (const c2 *)T, y,
                     (int)cdiv(R, shape_tn(s2)), 0.0, 0.0, true, (int)R, s2);
    } else {
      hipLaunchKernelGGL(k_to32, dim3(g), dim3(256), 0, I.s, (const c2 *)x, xs, NR);
      HIP_CHECK(hipGetLastError());
      I.launch32(I.b_near, 0, 0, I.near32.p, xs, ys, R, I.pick_shape(TC_NEAR, R));
      I.launch32(I.b_far1, 0, 0, I.farf32.p, xs, (float2 *)T, R, I.pick_shape(TC_FAR1, R));
      I.launch32(I.b_far2, 2, 0, I.farf32.p, (const float2 *)T, ys, R, I.pick_shape(TC_FAR2, R));
      hipLaunchKernelGGL(k_to64, dim3(g), dim3(256), 0, I.s, (const float2 *)ys, y, NR);
      HIP_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_permute, dim3(g), dim3(256), 0, I.s, (const c2 *)y, (c2 *)Y, I.dperm.p, I.dsoff.p,
                       I.nseg, I.N, R, 1);
    HIP_CHECK(hipGetLastError());
  } catch (...) {
    I.prof = prof_was;
    throw;
  }
  I.prof = prof_was;
}

namespace {
// Mesh arrays on the device for the entry kernels (freed with the object).
struct DevMesh {
  DevArray<double> xyz, cen, area, len, nrm;
  DevArray<int32_t> tri, tp, tm, vp, vm;
  NearMesh M;
  DevMesh(const Mesh &m, double freq_hz, hipStream_t st, int cfie = 0, double alpha = 1.0) {
    const double pi = 3.14159265358979323846, c0 = 299792458.0, mu0 = 4.0e-7 * pi, eps0 = 1.0 / (mu0 * c0 * c0);
    const double w = 2.0 * pi * freq_hz;
    xyz.upload(m.xyz, st); cen.upload(m.cen, st); area.upload(m.area, st); len.upload(m.len, st);
    tri.upload(m.tri, st); tp.upload(m.tp, st); tm.upload(m.tm, st); vp.upload(m.vp, st); vm.upload(m.vm, st);
    nrm.upload(m.nrm, st);
    M = NearMesh{xyz.p, cen.p, area.p, len.p, tri.p, tp.p, tm.p, vp.p, vm.p, w / c0, m.hmax, w * mu0 / 4.0,
                 -1.0 / (w * eps0), nrm.p, cfie, alpha, mu0 * c0};
  }
};
}  // namespace

void DeviceState::near_fill(const Mesh &m, double freq_hz, int cfie, double alpha, HMatrix &H) {
  HIP_CHECK(hipSetDevice(device));
  Impl &I = *impl;
  const int64_t nn = H.n_near();
  if (nn == 0) return;
  DevMesh dm(m, freq_hz, I.s, cfie, alpha);
  DevArray<int32_t> ts;
  DevArray<int64_t> perm, gptr, off;
  DevArray<c2> out;
  perm.upload(H.perm, I.s); gptr.upload(H.gptr, I.s); ts.upload(H.near_ts, I.s); off.upload(H.near_off, I.s);
  const int64_t total = H.near_off[nn];
  out.alloc((size_t)total);
  if (cfie)
    hipLaunchKernelGGL(k_near<true>, dim3((unsigned)nn), dim3(256), 0, I.s, dm.M, perm.p, gptr.p, ts.p, off.p, out.p);
  else
    hipLaunchKernelGGL(k_near<false>, dim3((unsigned)nn), dim3(256), 0, I.s, dm.M, perm.p, gptr.p, ts.p, off.p, out.p);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipMemcpyAsync((void *)H.near_vals.data(), out.p, (size_t)total * sizeof(c2), hipMemcpyDeviceToHost, I.s));
  HIP_CHECK(hipStreamSynchronize(I.s));
}

// f(q) for q in [0, n) on all host cores (blocks handed out in order).
template <class F>
static void parallel_blocks(int64_t n, F &&f) {
  const int nt = std::max(1, std::min<int>((int)std::thread::hardware_concurrency(), (int)((n + 63) / 64)));
  std::atomic<int64_t> next{0};
  std::exception_ptr err;
  std::mutex emu;
  auto work = [&]() {
    try {
      for (int64_t q; (q = next.fetch_add(1)) < n;) f(q);
    } catch (...) {
      std::lock_guard<std::mutex> lk(emu);
      if (!err) err = std::current_exception();
      next.store(n);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(work);
  work();
  for (auto &t : pool) t.join();
  if (err) std::rethrow_exception(err);
}

void DeviceState::far_sample(const Mesh &m, double freq_hz, int cfie, double alpha, const HMatrix &H, double eps,
                             const FarEmit &emit) {
  HIP_CHECK(hipSetDevice(device));
  Impl &I = *impl;
  const int64_t nf = H.n_far();
  if (nf == 0) return;
  DevMesh dm(m, freq_hz, I.s, cfie, alpha);
  DevArray<int64_t> perm;
  perm.upload(H.perm, I.s);
  // chunks: at most 4 GiB of scratch, and about a sixteenth of the blocks
  // (no fewer than 4096) so that the host recompression starts early
  const int64_t cap_elems = (int64_t)1 << 28;
  const int64_t cap_blocks = std::max<int64_t>(4096, (nf + 15) / 16);
  DevArray<c2> scratch, packed, gram, dT, finals;
  DevArray<AcaBlock> dblk;
  DevArray<int32_t> drank, drnew;
  DevArray<int64_t> dpack, dgoff, dtofs, dfpack;
  int64_t b0 = 0;
  while (b0 < nf) {
    std::vector<AcaBlock> blk;
    int64_t need = 0;
    int64_t b = b0;
    for (; b < nf && b - b0 < cap_blocks; ++b) {
      const int64_t mm = H.far_rng[4 * b + 1] - H.far_rng[4 * b], nn = H.far_rng[4 * b + 3] - H.far_rng[4 * b + 2];
      const int64_t e = (mm + nn) * kAcaCap;
      if (!blk.empty() && need + e > cap_elems) break;
      blk.push_back(AcaBlock{H.far_rng[4 * b], mm, H.far_rng[4 * b + 2], nn, need});
      need += e;
    }
    const int64_t nb = (int64_t)blk.size();
    scratch.alloc((size_t)need);
    dblk.upload(blk, I.s);
    drank.alloc((size_t)nb);
    if (cfie)
      hipLaunchKernelGGL(k_aca<true>, dim3((unsigned)nb), dim3(256), 0, I.s, dm.M, perm.p, dblk.p, eps, scratch.p,
                         drank.p);
    else
      hipLaunchKernelGGL(k_aca<false>, dim3((unsigned)nb), dim3(256), 0, I.s, dm.M, perm.p, dblk.p, eps, scratch.p,
                         drank.p);
    HIP_CHECK(hipGetLastError());
    FarChunk ch;
    ch.b0 = b0;
    ch.b1 = b;
    ch.rank.resize(nb);
    HIP_CHECK(hipMemcpyAsync(ch.rank.data(), drank.p, nb * sizeof(int32_t), hipMemcpyDeviceToHost, I.s));
    HIP_CHECK(hipStreamSynchronize(I.s));
    ch.off.assign(nb, 0);
    int64_t tot = 0;
    for (int64_t q = 0; q < nb; ++q) {
      ch.off[q] = tot;
      if (ch.rank[q] > 0) tot += (blk[q].m + blk[q].n) * ch.rank[q];
    }
    if (tot > 0) {
      dpack.upload(ch.off, I.s);
      packed.alloc((size_t)tot);
      hipLaunchKernelGGL(k_aca_pack, dim3((unsigned)nb), dim3(256), 0, I.s, dblk.p, drank.p, dpack.p, scratch.p,
                         packed.p);
      HIP_CHECK(hipGetLastError());
      // recompression: Gram matrices on the device, the k x k eigenproblems
      // on host threads, the recompressed factors U T_U, V T_V on the device
      std::vector<int64_t> goff(nb, 0);
      int64_t gtot = 0;
      for (int64_t q = 0; q < nb; ++q) {
        goff[q] = gtot;
        if (ch.rank[q] > 0) gtot += 2 * (int64_t)ch.rank[q] * ch.rank[q];
      }
      dgoff.upload(goff, I.s);
      gram.alloc((size_t)std::max<int64_t>(gtot, 1));
      hipLaunchKernelGGL(k_gram, dim3((unsigned)nb), dim3(256), 0, I.s, dblk.p, drank.p, dpack.p, dgoff.p, packed.p,
                         gram.p);
      HIP_CHECK(hipGetLastError());
      std::vector<cplx> hg((size_t)std::max<int64_t>(gtot, 1));
      HIP_CHECK(hipMemcpyAsync((void *)hg.data(), gram.p, (size_t)gtot * sizeof(c2), hipMemcpyDeviceToHost, I.s));
      HIP_CHECK(hipStreamSynchronize(I.s));
      std::vector<std::vector<cplx>> TU(nb), TV(nb);
      std::vector<int32_t> rnew(nb, 0);
      parallel_blocks(nb, [&](int64_t q) {
        const int k = ch.rank[q];
        if (k <= 0) return;
        int r = 0;
        recompress_from_grams(k, &hg[goff[q]], &hg[goff[q] + (int64_t)k * k], eps, TU[q], TV[q], r);
        rnew[q] = r;
      });
      std::vector<int64_t> tofs(nb, 0), fpack(nb, 0);
      int64_t ttot = 0, ftot = 0;
      for (int64_t q = 0; q < nb; ++q) {
        tofs[q] = ttot;
        fpack[q] = ftot;
        ttot += 2 * (int64_t)TU[q].size();
        ftot += (blk[q].m + blk[q].n) * (int64_t)rnew[q];
      }
      std::vector<c2> ht((size_t)std::max<int64_t>(ttot, 1));
      for (int64_t q = 0; q < nb; ++q) {
        std::memcpy(&ht[tofs[q]], TU[q].data(), TU[q].size() * sizeof(c2));
        std::memcpy(&ht[tofs[q] + (int64_t)TU[q].size()], TV[q].data(), TV[q].size() * sizeof(c2));
      }
      dT.upload(ht, I.s);
      dtofs.upload(tofs, I.s);
      dfpack.upload(fpack, I.s);
      drnew.upload(rnew, I.s);
      finals.alloc((size_t)std::max<int64_t>(ftot, 1));
      hipLaunchKernelGGL(k_apply, dim3((unsigned)nb), dim3(256), 0, I.s, dblk.p, drank.p, drnew.p, dpack.p, dtofs.p,
                         dfpack.p, packed.p, dT.p, finals.p);
      HIP_CHECK(hipGetLastError());
      ch.uv.resize(ftot);
      HIP_CHECK(hipMemcpyAsync((void *)ch.uv.data(), finals.p, (size_t)ftot * sizeof(c2), hipMemcpyDeviceToHost, I.s));
      for (int64_t q = 0; q < nb; ++q) {
        ch.off[q] = fpack[q];
        if (ch.rank[q] > 0) ch.rank[q] = rnew[q];
      }
    }
    ch.final = true;
    HIP_CHECK(hipStreamSynchronize(I.s));
    emit(std::move(ch));
    b0 = b;
  }
}

void DeviceState::set_tuning(const TuneTable &t, const std::string &src) {
  Impl &I = *impl;
  HIP_CHECK(hipStreamSynchronize(I.s));
  tune = t;
  tune_src = src;
  I.tune = t.entries;             // the sweep pull threshold applies from the next setup
  if (I.ready) {                 // re-resolve the solve shapes at the next solve (captured graphs dropped)
    I.drop_graphs();
    I.built_R = -1;
  }
}

void DeviceState::set_profiling(bool on) {
  Impl &I = *impl;
  HIP_CHECK(hipStreamSynchronize(I.s));
  I.prof_collect();
  I.prof = on;
  for (auto &k : I.kstat) k = Impl::KStat();
  I.launch_log.clear();
}

std::string DeviceState::stats_json() const {
  const Impl &I = *impl;
  std::ostringstream o;
  o.precision(9);
  o << "{\"N\": " << I.N << ", \"groups\": " << I.M;
  if (I.ready) {
    o << ", \"levels\": " << I.P.n_levels << ", \"upper_blocks\": " << I.P.n_upper_blocks
      << ", \"n_U\": " << I.P.n_U << ", \"n_D\": " << I.P.n_D
      << ", \"factor_bytes\": " << 16.0 * (double)I.P.panel_elems * (I.nonsym ? 2.0 : 1.0)
      << ", \"setup_flops\": " << I.P.setup_flops << ", \"far_T_rows\": " << I.t_rows;
  }
  o << ", \"near_elems\": " << I.near.n << ", \"far_elems\": " << I.faruv.n;
  {
    const char *cn[TC_COUNT] = {"sweep", "dinv", "far1", "far2", "near", "schur"};
    o << ", \"tuning\": {\"source\": \"" << tune_src << "\", \"entries\": " << tune.entries.size()
      << ", \"sweep_pull_kmax\": " << I.sweep_pull_kmax << ", \"shapes\": {";
    for (int c = 0; c < TC_COUNT; ++c) o << (c ? ", " : "") << "\"" << cn[c] << "\": " << I.shape_of[c];
    o << "}}";
  }
  o << ", \"terms\": " << I.terms << ", \"series_tol\": " << I.series_tol << ", \"terms_used\": " << I.terms_used;
  o << ", \"setup_replays\": " << I.srec.replays << ", \"setup_recorded\": " << (I.srec.valid ? "true" : "false");
  o << ", \"schedule_split\": {\"levels_built_ms\": " << sched_split[0] << ", \"wait_ms\": " << sched_split[1]
    << ", \"stage_ms\": " << sched_split[2] << ", \"tiles\": " << sched_split[3] << ", \"terms\": " << sched_split[4]
    << ", \"schur_col_slots\": " << sched_split[5] << ", \"schur_col_active\": " << sched_split[6] << "}";
  o << ", \"times_ms\": {\"setup_numeric\": " << times.schur_ms << ", \"setup_schedule\": " << times.inverse_ms
    << ", \"symbolic\": " << times.symbolic_ms
    << ", \"solve\": " << times.solve_ms << ", \"rhs\": " << times.rhs_ms << ", \"series\": " << times.sweep_ms
    << ", \"rcs\": " << times.rcs_ms << "}";
  {
    const char *names[4] = {"gemm_store", "gemm_sub", "gemm_add", "inverse"};
    o << ", \"kernels\": {";
    for (int k = 0; k < 4; ++k)
      o << (k ? ", " : "") << "\"" << names[k] << "\": {\"launches\": " << I.kstat[k].launches
        << ", \"ms\": " << I.kstat[k].ms << ", \"flops\": " << I.kstat[k].flops
        << ", \"bytes\": " << I.kstat[k].bytes << "}";
    o << ", \"profiling\": " << (I.prof ? 1 : 0) << "}";
    if (I.prof) {   // kind (0..2 GEMM mode, 3 inverse), work units (tiles / blocks), flops, algorithmic bytes, ms,
                    // tuning class (0 sweep, 1 D^-1, 2-3 far stages, 4 near product, 5 Schur; -1 none)
      o << ", \"launch_log\": [";
      for (size_t i = 0; i < I.launch_log.size(); ++i) {
        const auto &L = I.launch_log[i];
        o << (i ? ", " : "") << "[" << L.kind << ", " << L.units << ", " << L.flops << ", " << L.bytes << ", " << L.ms
          << ", " << L.cls << "]";
      }
      o << "]";
    }
  }
  if (I.built_R > 0) {
    o << ", \"solve_flops\": {\"fwd\": " << I.solve_flops_parts[0] << ", \"bwd\": " << I.solve_flops_parts[1]
      << ", \"dinv\": " << I.solve_flops_parts[2] << ", \"far\": " << I.solve_flops_parts[3]
      << ", \"R\": " << I.built_R << "}";
  }
  o << "}";
  return o.str();
}

}  // namespace hps
