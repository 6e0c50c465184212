/*
 * hps.h -- C ABI of the H-matrix power-series EFIE solver for MI355X (gfx950).
 *
 * Method: Negi, Balakrishnan, Rao, "Fast Power Series Solution of Large 3-D
 * Electrodynamic Integral Equation for PEC Scatterers" (arXiv:2109.04129).
 *
 *   Z x = b  (eq. 9), Z = Z_N + Z_F (eq. 13): dense near-field blocks between
 *   touching octree leaves and ACA low-rank far-field blocks (eqs. 10-12).
 *   Setup: right scaling coefficients alpha_i = I - sum_j E_ij Z~_ii^-1 Z~_ij
 *   by successive Schur steps with fill-in until the near field is block
 *   diagonal (eqs. 14-23).  Only the right coefficients are stored; the left
 *   ones are their transposes (Z_N = Z_N^T).
 *   Solve: b~ = A^T b (eq. 25), b_o = D^-1 b~ (eq. 32), x~ = b_o - U b_o
 *   (eqs. 31, 35-36, two terms), x = A x~ (eq. 26), with the per-RHS ratio
 *   ||U b_o|| / ||b_o|| of eq. (45).
 *
 * Conventions shared by every call:
 *   - complex numbers are interleaved (re, im) IEEE doubles ("c128");
 *   - unknowns are RWG functions, one per interior mesh edge, numbered by the
 *     edges sorted lexicographically on (min vertex id, max vertex id);
 *     T+ is the triangle that runs along the edge from the smaller to the
 *     larger vertex id in its counter-clockwise order;
 *   - an N x R block of vectors is column-major with leading dimension N;
 *   - time convention e^{j w t}, G = exp(-jkR)/(4 pi R), E0 = 1 V/m;
 *   - every function returns an hps_status; nothing throws or aborts across
 *     the ABI; after an error hps_last_error() describes it;
 *   - a context is not thread-safe: one host thread at a time.
 *
 * Call order:  hps_create -> hps_set_mesh -> (hps_build_hmatrix |
 *              hps_set_hmatrix) -> hps_setup -> hps_solve_* (any number).
 *   Calling out of order returns HPS_ESTATE.
 */
#ifndef HPS_H
#define HPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hps_ctx hps_ctx;

typedef enum {
  HPS_OK = 0,
  HPS_WRATIO = 1,       /* results written, but some ratio >= ratio_warn (eq. 45) */
  HPS_EINVAL = -1,      /* bad argument or mesh */
  HPS_ENOMEM = -2,      /* host or device allocation failed, or over device_mem_cap */
  HPS_EDEVICE = -3,     /* HIP runtime error, or no device in this context */
  HPS_ESINGULAR = -4,   /* a scaled diagonal block Z~_ii is singular */
  HPS_ESTATE = -5,      /* call order violated */
  HPS_EIO = -6          /* file error */
} hps_status;

typedef struct {
  double freq_hz;          /* > 0 */
  int32_t leaf_max;        /* max unknowns per octree leaf (group), 1..1024.  Groups
                              above 128 unknowns are eliminated as consecutive
                              sub-groups of at most 128 (the pivot blocks of the
                              setup); currents do not depend on it, the eq. (45)
                              ratio does */
  double aca_tol;          /* eps of eq. (12), Frobenius, per far block, in (0, 1) */
  int32_t precision;       /* 0: FP64 throughout.  1: FP32 solve (D^-1, scaling
                              blocks, vectors) with BF16 far factors and a per-block
                              FP32 scale, FP64 setup, plus refine_passes residual
                              passes in FP32.  2: as 1 with FP16 far factors.  The
                              residual passes (b - H x and the correction series)
                              use FP32 copies of the far factors */
  int32_t terms;           /* power-series terms, >= 1 (paper: 2) */
  int32_t refine_passes;   /* residual-correction passes (precision form), >= 0 */
  double ratio_warn;       /* HPS_WRATIO threshold on eq. (45) (paper: 0.1) */
  uint64_t device_mem_cap; /* bytes; 0 = none.  hps_setup fails with HPS_ENOMEM
                              before allocating if its plan needs more */
  int32_t host_threads;    /* threads for the host H-matrix build; 0 = all cores */
  int32_t ordering;        /* group elimination order: 0 = nested dissection (default),
                              1 = natural (tree order of the groups).  The currents do
                              not depend on it; the eq. (45) ratio, which is measured in
                              the scaled unknowns, does. */
  int32_t graphs;          /* 1 (default): the device part of a solve is captured once
                              per RHS count into a HIP graph and replayed; 0: every
                              kernel is launched from the host on each call.  2: as 1,
                              and the setup too: an hps_setup whose elimination plan,
                              H-matrix structure (groups, near and far block lists,
                              ranks), device buffers, form and tile shape equal those
                              of the last eager setup replays that setup's launches on
                              the values now installed (same structure, new values:
                              hps_set_hmatrix with arrays of the same sizes), from a
                              graph captured at the first replay; the solve schedules
                              and captured solves are kept.  Anything else runs the
                              setup eagerly and records it again.  Same results in
                              every mode.  Setups and solves run eagerly while
                              hps_profile is on. */
  int32_t verbose;         /* 1: the host H-matrix build reports its progress on
                              stderr; 0 (default): silent */
  double leaf_box_min;     /* metres; > 0: octree cells narrower than this are never
                              created, so leaves may hold more than leaf_max unknowns
                              (electrically sized leaves, Sec. V.A: about half a
                              wavelength for two-term convergence); 0 (default): off */
  double series_tol;       /* > 0: adaptive series, `terms` is the maximum; the series
                              stops after the first term t with ||it_t|| / ||it_0||
                              < series_tol for every RHS (eqs. 35-36, 45); the
                              precision form's residual pass uses as many terms.
                              Solves are then launched without graphs.  0 (default):
                              exactly `terms` terms */
  int32_t host_near;       /* 0 (default): with a device, hps_build_hmatrix computes the
                              near blocks, the ACA samples of the far blocks and
                              their recompression on it (host threads solve only
                              the k x k eigenproblems of the recompression, k <= 96);
                              1: the whole build on host threads */
  int32_t formulation;     /* 0 (default): EFIE (eqs. 2-3), symmetric matrix, right
                              coefficients only.  1: CFIE of eq. (8),
                              cfie_alpha EFIE + eta0 (1 - cfie_alpha) MFIE (eqs. 4-7),
                              closed surfaces only; the matrix is not symmetric, so
                              the setup also keeps the left coefficients of eq. (18)
                              (twice the factor memory) */
  double cfie_alpha;       /* alpha of eq. (8) in [0, 1] (paper: 0.5 for closed bodies) */
  double eta;              /* admissibility constant of eq. (10), >= 0: two octree
                              cells form a far block when eta dist >= min(dia), dia the
                              cell diagonal and dist the gap between the closed cells.
                              Any eta >= sqrt(3) (default 2) means "the cells do not
                              touch"; smaller values keep more leaf pairs near; 0 makes
                              every leaf pair near (no far field) */
} hps_params;

/* Fill *p with defaults: leaf_max 128, aca_tol 1e-3, precision 0, terms 2,
   refine_passes 0, ratio_warn 0.1, no cap, host_threads 0, ordering 0, graphs 1, verbose 0, leaf_box_min 0, series_tol 0, host_near 0,
   formulation 0 (EFIE), cfie_alpha 0.5, eta 2.
   freq_hz = 0 (must be set). */
hps_status hps_params_default(hps_params *p);

/* Create a context on HIP device `device` (>= 0), or a host-only context
   (device = -1) that can build and inspect H-matrices but not set up or solve.
   `stream` is a hipStream_t to run on, or NULL for a stream the context
   creates (default priority).  *out receives the context. */
hps_status hps_create(hps_ctx **out, int device, void *stream);

/* Release every host and device allocation of the context.  NULL is a no-op. */
void hps_destroy(hps_ctx *ctx);

/* Text of the last error on ctx (empty if none); valid until the next call.
   With ctx = NULL: the reason the last failed hps_create on this thread failed. */
const char *hps_last_error(const hps_ctx *ctx);

/* Triangle mesh: xyz (nv x 3 doubles, metres, host), tri (nt x 3 int32 vertex
   ids, host), counter-clockwise seen from outside.  Copied.  The mesh must be a
   closed, consistently oriented 2-manifold without degenerate triangles, else
   HPS_EINVAL.  Builds the RWG functions. */
hps_status hps_set_mesh(hps_ctx *ctx, const double *xyz, int64_t nv, const int32_t *tri,
                        int64_t nt);

/* Same for an open sheet (e.g. the square plate of Sec. V.C.2): edges that
   belong to one triangle only (the rim) are accepted and carry no unknown;
   the EFIE holds on open PEC surfaces.  Interior edges as in hps_set_mesh. */
hps_status hps_set_open_mesh(hps_ctx *ctx, const double *xyz, int64_t nv, const int32_t *tri,
                             int64_t nt);

/* Number of RWG unknowns of the current mesh. */
hps_status hps_num_unknowns(const hps_ctx *ctx, int64_t *N);

/* Build the H-matrix of the mesh (Sec. II): octree over edge midpoints with at
   most leaf_max unknowns per leaf; near blocks = touching leaf pairs (EFIE
   Galerkin quadrature, Z = Z^T exactly); far blocks = non-touching cluster
   pairs, re-compressed ACA to aca_tol (eqs. 10-12).  With a device (see
   host_near) the near blocks, the ACA sampling and the recompression run on
   it (recompression through the Gram matrices of the ACA factors: the same
   truncation rule as QR + SVD, to about 1e-8 of the block norm); the blocks
   are then held on both sides.  Not part of "setup". */
hps_status hps_build_hmatrix(hps_ctx *ctx, const hps_params *p);

/* Install an H-matrix built elsewhere instead (same meaning as above), all
   arrays on the host, copied:
     perm[N]          tree position -> RWG unknown (a permutation);
     group_ptr[M+1]   group g owns tree positions [group_ptr[g], group_ptr[g+1]);
     near_ts[2*n_near]  (t, s) group pairs, t <= s, each pair at most once, all
                      (g, g) present; near_off[n_near+1] element offsets into
                      near_vals (c128), block (t, s) is row-major
                      (size_t - size_s) x (size of s) with entry [a][b] =
                      Z(perm[lo_t + a], perm[lo_s + b]); block (s, t) is its
                      transpose;
     far_rng[4*n_far] (tlo, thi, slo, shi) tree-position ranges, disjoint from
                      the near pattern; far_rank[n_far] r_b >= 0;
                      far_off[n_far+1] element offsets into far_uv (c128);
                      block b stores U (m x r, column-major) then V (n x r,
                      column-major), m = thi - tlo, n = shi - slo, with
                      Z[t, s] ~= U V^T and Z[s, t] ~= V U^T.
   With p->formulation = 1 (CFIE, not symmetric) near_ts lists every ordered
   pair (t, s) of touching groups, t > s included, each block holding
   Z[t, s] only, and every far block b holds Z[t, s] ~= U V^T only (the
   (s, t) block is a separate entry).
   p supplies freq_hz (for excitation / RCS) and the solve options.  Groups of
   more than 128 unknowns are cut into consecutive sub-groups (near blocks cut
   to match), as after hps_build_hmatrix. */
hps_status hps_set_hmatrix(hps_ctx *ctx, const hps_params *p, int64_t N, const int64_t *perm,
                           int64_t M, const int64_t *group_ptr, int64_t n_near,
                           const int32_t *near_ts, const int64_t *near_off,
                           const double *near_vals, int64_t n_far, const int64_t *far_rng,
                           const int32_t *far_rank, const int64_t *far_off,
                           const double *far_uv);

/* Query the H-matrix structure.  Pass NULL for arrays not wanted; sizes first:
   *M, *n_near, *n_far, *near_elems (total near c128 entries), *far_elems. */
hps_status hps_hmatrix_sizes(const hps_ctx *ctx, int64_t *M, int64_t *n_near, int64_t *n_far,
                             int64_t *near_elems, int64_t *far_elems);
/* Copy out the structure (host arrays sized by hps_hmatrix_sizes, layout as
   in hps_set_hmatrix, groups as held, i.e. after any cut of groups above 128
   unknowns; any pointer may be NULL). */
hps_status hps_get_hmatrix(const hps_ctx *ctx, int64_t *perm, int64_t *group_ptr, int32_t *near_ts,
                           int64_t *near_off, double *near_vals, int64_t *far_rng,
                           int32_t *far_rank, int64_t *far_off, double *far_uv);

/* The RWG functions of the current mesh (Sec. II: one unknown per interior
   edge, with the two triangles sharing it), in RWG order, i.e. the order of
   the unknowns in X, B and the currents: edges sorted by (smaller vertex id,
   larger vertex id).  Host arrays of N x 2 int32 (N from hps_num_unknowns),
   caller-owned, any of them NULL if not wanted:
     edge_v[2n], edge_v[2n+1]  the edge's vertex ids, smaller first;
     tri_pm[2n], tri_pm[2n+1]  T+ (the triangle that runs along the edge from
                              the smaller to the larger vertex id) and T-;
     free_v[2n], free_v[2n+1]  the vertex of T+ and of T- opposite the edge.
   Batch contexts: the problems' functions in problem order, with vertex and
   triangle ids counted in the concatenation of the meshes.
   HPS_ESTATE before a mesh is set. */
hps_status hps_rwg(const hps_ctx *ctx, int32_t *edge_v, int32_t *tri_pm, int32_t *free_v);

/* Write the installed H-matrix and its parameters to a file, and read one
   back in place of hps_build_hmatrix / hps_set_hmatrix (same structure as
   hps_get_hmatrix).  Layout, little-endian: the 8 bytes "HPSHMAT1"; int64
   header N, M, n_near, near_elems, n_far, far_elems, nonsym (0/1),
   sizeof(hps_params); the hps_params struct as stored; then perm (N int64),
   group_ptr (M+1 int64), near_ts (2 n_near int32), near_off (n_near+1
   int64), near_vals (near_elems c128), far_rng (4 n_far int64), far_rank
   (n_far int32), far_off (n_far+1 int64), far_uv (far_elems c128).
   Single-problem contexts only (HPS_EINVAL for a batch).  Export: HPS_ESTATE
   without an H-matrix, HPS_EIO if the file cannot be written.  Import: needs
   the same mesh set first (N must match, else HPS_EINVAL); HPS_EIO for a
   missing, truncated or foreign file; the arrays are checked as in
   hps_set_hmatrix; a file or format error leaves the context as it was. */
hps_status hps_export_hmatrix(const hps_ctx *ctx, const char *path);
hps_status hps_import_hmatrix(hps_ctx *ctx, const char *path);

/* Setup ("setup time", Sec. III.A and IV.A): host symbolic phase (fill-reducing
   nested-dissection order of the groups, fill-in pattern, elimination-tree
   levels), then on the device, level by level: LU with partial pivoting and
   inverse of each scaled diagonal block Z~_ii (eq. 16), the right coefficients
   C_ij = Z~_ii^-1 Z~_ij, and the Schur updates Z~_jk -= Z~_ij^T C_ik including
   fill-in blocks (eq. 21).  Precision form: also converts the solve operands.
   HPS_ENOMEM, before any device allocation, when device_mem_cap is set and the
   plan's device memory (H-matrix, two panel sets, precision-form copies)
   exceeds it; this check runs on host-only contexts too (then HPS_EDEVICE
   follows only when the plan fits).
   HPS_ESINGULAR if a pivot block is numerically singular: LU with partial
   pivoting of Z~_ii meets a pivot of modulus below n eps max|Z~_ii|
   (n the block size, eps = 2^-52). */
hps_status hps_setup(hps_ctx *ctx);

/* Solve R plane-wave right-hand sides (Sec. V): wave r travels along khat[r]
   with polarisation pol[r] (host arrays R x 3, unit, orthogonal).  Writes:
     X     N x R c128 currents (RWG order), host or device pointer (found
           with hipPointerGetAttributes; a host block is staged through a
           device buffer of the context), or NULL;
     rcs   R doubles (host): monostatic co-polar RCS in m^2 in the direction
           -khat[r] (sigma = k^2 eta^2 / 4pi |b_r^T x_r|^2), or NULL;
     ratio R doubles (host): ||it_1|| / ||it_0|| of eq. (45), or NULL.
   Returns HPS_WRATIO (results written) when some ratio >= ratio_warn. */
hps_status hps_solve_planewaves(hps_ctx *ctx, int64_t R, const double *khat, const double *pol,
                                void *X, double *rcs, double *ratio);

/* Solve arbitrary right-hand sides: B and X are N x R c128 blocks in RWG
   order, host or device as X above (may not alias); ratio as above (host,
   nullable). */
hps_status hps_solve_rhs(hps_ctx *ctx, int64_t R, const void *B, void *X, double *ratio);

/* Plane-wave excitation only: B (N x R c128, host or device, RWG order) = <f_m, E_inc>
   (EFIE), or the CFIE right-hand side alpha <f_m, E_inc> + eta0 (1 - alpha)
   <f_m, n x H_inc> of eq. (8). */
hps_status hps_excitation(hps_ctx *ctx, int64_t R, const double *khat, const double *pol,
                          void *B);

/* Y = H X on the device (near blocks + both directions of every far block;
   for the CFIE every stored block in its own direction),
   X and Y N x R c128 blocks (host or device) in RWG order.  The precision
   form computes it in FP32 (FP32 near blocks and far factors).  Valid after hps_setup
   (its product schedules are built there); HPS_ESTATE before. */
hps_status hps_hmatvec(hps_ctx *ctx, int64_t R, const void *X, void *Y);

/* Size of the fixed device scratch array used by hps_hmatvec_noalloc (one
   copy per GPU the library runs on, held until the process ends). */
#define HPS_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the product
   of hps_hmatvec, Y = H X, with every work vector in a fixed device scratch
   array of HPS_SCRATCH_BYTES instead of context buffers sized on demand.  It
   calls no hipMalloc / hipFree and no host copy, and does not synchronise:
   the result is in Y once the context's stream reaches this call.
   X and Y: N x R c128, RWG order, caller-owned DEVICE memory (host memory
   gives HPS_EINVAL).  The results are bitwise those of hps_hmatvec.
   Scratch need: 16 (2 N R + t R) bytes for FP64 (t = far rank rows,
   hps_stats "device" "far_T_rows"), 8 (6 N R + t R) in the precision form, each
   part rounded up to 256 bytes; a larger
   R gives HPS_EINVAL naming the largest R that fits.  Every call on a GPU
   shares that GPU's array: calls that overlap on one GPU (two contexts, two
   streams, two host threads) race and give wrong results.  Valid after
   hps_setup; HPS_ESTATE before. */
hps_status hps_hmatvec_noalloc(hps_ctx *ctx, int64_t R, const void *X, void *Y);

/* Tile shapes of the grouped complex GEMM (batching form: tile shapes chosen
   by the project's autotuner, paper_2109_04129_amd/autotune.py).  path: a JSON
   table {"entries": [{"class": C, "rhs_max": R, "group_max": G, "precision": P,
   "shape": S}, ...]} (R, G, P optional: no bound / any precision), C one of "sweep", "dinv", "far1", "far2", "near" (solve launches),
   "schur" (setup Schur updates); S 0-4 = workgroup tiles of 32 rows x 32, 64,
   64, 128, 128 columns (waves of 16 x 16, 16 x 32, 32 x 16, 32 x 32,
   16 x 64 outputs), 5 = 32 x 64 with both operands staged in LDS,
   double-buffered (FP64 launches; FP32 ones take shape 2 for it), 6 = a
   vector-ALU matrix-vector kernel for one-column FP64 solves (other launches
   take shape 0 for it; its sums are in another order, so one-column results
   differ from the other shapes' by rounding), 7 and 8 = shapes 2 and 1 built
   for 3 waves per SIMD (FP64; FP32 launches take 2 and 1), 9 = shape 0
   built for 5 waves per SIMD (FP64; FP32 takes 0), 10 = shape 3 built for 4
   waves per SIMD (FP32; FP64 takes 3), 11 and 12 = the tile of shape 7 with
   every full 16-k chunk of a term staged in LDS one chunk ahead by
   direct-to-LDS loads (FP64: 11 also stages the target tile; FP32 launches
   with FP32 factors take the pipelined FP32 kernel for both, those with
   16-bit factors take 2).  A launch takes the first entry of its class whose
   rhs_max bounds its column count, whose group_max bounds the mean pivot
   size (unknowns per group) and whose precision (0, 1, 2 as in hps_params;
   the setup counts as 0) matches; shape 0 when none does.  NULL or "" restores
   the built-in table (shape 0 everywhere).  Every shape gives bitwise the
   same results.  An optional top-level "sweep_pull_kmax": K (integer >= 0,
   default 0) makes every sweep target whose summed contraction is at most K
   take all its terms in one tile set (pull) instead of one per source level
   (push); the sums then run in another order (results equal to rounding);
   it applies from the next hps_setup.  hps_create loads tuning/gfx950.json from the library's
   directory when that file exists (a malformed one fails hps_create with
   HPS_EINVAL).  Takes effect at the next hps_setup / solve.  Errors:
   HPS_EIO (file), HPS_EINVAL (content), HPS_EDEVICE (host-only context). */
hps_status hps_set_tuning(hps_ctx *ctx, const char *path);

/* Per-launch kernel timing: with enable != 0 every grouped-GEMM and inverse
   launch is bracketed by HIP events on the context's stream; hps_stats then
   reports launches, summed device ms, algorithmic flops and bytes per kernel
   class since the call, and a launch log ([kind, work units, flops,
   algorithmic bytes, ms, tuning class] per launch; kind 0-2 the grouped GEMM
   in store / subtract / add mode, 3 the inverse; tuning class as in
   hps_set_tuning: 0 sweep, 1 dinv, 2 far1, 3 far2, 4 near, 5 schur, -1 for
   launches without one).  Counters reset on every call.  Adds two event
   records per launch. */
hps_status hps_profile(hps_ctx *ctx, int enable);

/* JSON statistics (sizes, ranks, fill, bytes, per-stage device times of the
   last setup / solve in ms, the tile shapes in use, and the last setup's
   schedule: "schedule_split" with its build times, tile and term counts and
   the Schur tiles' 16-column block slots x 16-k chunks, all and used) into
   buf (NUL-terminated, truncated to len). */
hps_status hps_stats(const hps_ctx *ctx, char *buf, size_t len);

/* ------------------------------------------------------------------ batches
 * A batch context holds P independent scattering problems (separate meshes,
 * one set of parameters).  Their H-matrices are kept apart (no block couples
 * two problems) but the setup and the solve treat them as one block-diagonal
 * system: every elimination-tree level of every problem is processed in the
 * same launches, and every solve stage is one launch over all problems.
 * Results per problem are those of a single-problem context on the same
 * problem, up to rounding.
 *
 * Call order:  hps_batch_create -> hps_batch_set_mesh for p = 0..P-1 ->
 *   (hps_build_hmatrix | hps_batch_set_hmatrix for every p) -> hps_setup ->
 *   hps_solve_* ; hps_set_mesh / hps_set_hmatrix return HPS_EINVAL on a
 *   batch context.
 * Layouts on a batch context (all R plane waves or RHS columns apply to every
 *   problem): X, B and Y hold, for p = 0..P-1 in turn, problem p's N_p x R
 *   column-major block (RWG order of that mesh, leading dimension N_p),
 *   starting at element R * (N_0 + ... + N_{p-1}); rcs and ratio hold P x R
 *   doubles, problem-major (entry p * R + r).  hps_num_unknowns returns
 *   N_0 + ... + N_{P-1}; hps_get_hmatrix returns the merged block-diagonal
 *   H-matrix (tree positions and groups of problem p follow those of
 *   problems 0..p-1).  A single-problem context behaves as a batch of one. */

/* Create a batch context for n_problems (1..65535) problems; device and
   stream as in hps_create. */
hps_status hps_batch_create(hps_ctx **out, int device, void *hip_stream, int32_t n_problems);

/* Mesh of problem p (0 <= p < P); same rules as hps_set_mesh.  Invalidates
   the H-matrix and setup of the whole batch. */
hps_status hps_batch_set_mesh(hps_ctx *ctx, int32_t p, const double *xyz, int64_t nv,
                              const int32_t *tri, int64_t nt);

/* Install problem p's H-matrix (arguments as in hps_set_hmatrix, positions
   local to problem p).  params must be identical for every problem.  The
   batch becomes ready for hps_setup once every problem has one. */
hps_status hps_batch_set_hmatrix(hps_ctx *ctx, int32_t p, const hps_params *params, int64_t N,
                                 const int64_t *perm, int64_t M, const int64_t *group_ptr,
                                 int64_t n_near, const int32_t *near_ts, const int64_t *near_off,
                                 const double *near_vals, int64_t n_far, const int64_t *far_rng,
                                 const int32_t *far_rank, const int64_t *far_off,
                                 const double *far_uv);

/* Number of problems (1 for a single-problem context). */
hps_status hps_num_problems(const hps_ctx *ctx, int32_t *n_problems);

/* Unknowns N_p of problem p (after its mesh is set). */
hps_status hps_problem_unknowns(const hps_ctx *ctx, int32_t p, int64_t *N);

#ifdef __cplusplus
}
#endif
#endif /* HPS_H */
