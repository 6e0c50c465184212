// Re-compressed ACA (eqs. 11-12 and the recompression of refs. [20, 21]) and
// the H-matrix assembly on the host.
//
// ACA with partial pivoting: first pivot row 0; the pivot column maximises
// the residual row (lowest index on ties); v = row / row[j]; u = residual
// column j; the Frobenius norm of the running approximation is updated
// incrementally and the iteration stops when |u||v| <= eps ||S||_F; the next
// row maximises |u| over unused rows.  Zero residual rows are skipped.  When
// the rank would reach m n / (m + n) the block is formed in full and truncated
// by its SVD.  Recompression: QR of U and V, SVD of R_U R_V^T, truncation to
// the smallest rank whose discarded singular values have norm <= eps ||s||.
#include <cstdio>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <exception>
#include <mutex>
#include <thread>

#include "hps_internal.h"

namespace hps {

// ---------------------------------------------------------------- QR, SVD
void householder_qr(int64_t m, int64_t n, cplx *A, std::vector<cplx> &Q, std::vector<cplx> &R,
                    int64_t &kk) {
  const int64_t k = std::min(m, n);
  kk = k;
  std::vector<cplx> tau(k);
  for (int64_t j = 0; j < k; ++j) {
    cplx *x = A + j * m + j;
    const int64_t len = m - j;
    double nrm2 = 0.0;
    for (int64_t i = 0; i < len; ++i) nrm2 += std::norm(x[i]);
    const double nrm = std::sqrt(nrm2);
    if (nrm == 0.0) { tau[j] = 0.0; continue; }
    const double ax0 = std::abs(x[0]);
    const cplx phase = (ax0 == 0.0) ? cplx(1.0, 0.0) : x[0] / ax0;
    const cplx alpha = -phase * nrm;      // new diagonal value
    // v = x - alpha e1, normalised so v[0] = 1; H = I - tau v v^H
    const cplx v0 = x[0] - alpha;
    for (int64_t i = 1; i < len; ++i) x[i] /= v0;
    // tau = 2 / (v^H v) with v[0] = 1
    double vv = 1.0;
    for (int64_t i = 1; i < len; ++i) vv += std::norm(x[i]);
    tau[j] = 2.0 / vv;
    x[0] = alpha;
    // apply H to the remaining columns
    for (int64_t c = j + 1; c < n; ++c) {
      cplx *y = A + c * m + j;
      cplx w = y[0];
      for (int64_t i = 1; i < len; ++i) w += std::conj(x[i]) * y[i];
      w *= tau[j];
      y[0] -= w;
      for (int64_t i = 1; i < len; ++i) y[i] -= w * x[i];
    }
  }
  R.assign(k * n, 0.0);
  for (int64_t c = 0; c < n; ++c)
    for (int64_t i = 0; i <= std::min(c, k - 1); ++i) R[c * k + i] = A[c * m + i];
  Q.assign(m * k, 0.0);
  for (int64_t c = 0; c < k; ++c) Q[c * m + c] = 1.0;
  for (int64_t j = k - 1; j >= 0; --j) {
    const cplx *x = A + j * m + j;
    const int64_t len = m - j;
    for (int64_t c = 0; c < k; ++c) {
      cplx *y = &Q[c * m + j];
      cplx w = y[0];
      for (int64_t i = 1; i < len; ++i) w += std::conj(x[i]) * y[i];
      w *= tau[j];
      y[0] -= w;
      for (int64_t i = 1; i < len; ++i) y[i] -= w * x[i];
    }
  }
}

// One-sided (Hestenes) Jacobi SVD of an m x n matrix with m >= n:
// A = W diag(s) Y^H, W m x n, Y n x n, s descending.
static void jacobi_tall(int64_t m, int64_t n, std::vector<cplx> A, std::vector<cplx> &W,
                        std::vector<double> &s, std::vector<cplx> &Y) {
  Y.assign(n * n, 0.0);
  for (int64_t i = 0; i < n; ++i) Y[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int64_t p = 0; p < n - 1; ++p)
      for (int64_t q = p + 1; q < n; ++q) {
        cplx *ap = &A[p * m], *aq = &A[q * m];
        double al = 0.0, be = 0.0;
        cplx ga = 0.0;
        for (int64_t i = 0; i < m; ++i) {
          al += std::norm(ap[i]);
          be += std::norm(aq[i]);
          ga += std::conj(ap[i]) * aq[i];
        }
        const double g = std::abs(ga);
        if (g == 0.0 || g <= 1e-15 * std::sqrt(al * be)) continue;
        off = std::max(off, g / std::sqrt(al * be));
        const cplx ph = ga / g;               // e^{i phi}
        const double zeta = (be - al) / (2.0 * g);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int64_t i = 0; i < m; ++i) {
          const cplx x = ap[i], y = aq[i];
          ap[i] = c * x - sn * std::conj(ph) * y;
          aq[i] = sn * ph * x + c * y;
        }
        cplx *yp = &Y[p * n], *yq = &Y[q * n];
        for (int64_t i = 0; i < n; ++i) {
          const cplx x = yp[i], y = yq[i];
          yp[i] = c * x - sn * std::conj(ph) * y;
          yq[i] = sn * ph * x + c * y;
        }
      }
    if (off < 1e-15) break;
  }
  std::vector<double> nr(n);
  for (int64_t c = 0; c < n; ++c) {
    double t = 0.0;
    for (int64_t i = 0; i < m; ++i) t += std::norm(A[c * m + i]);
    nr[c] = std::sqrt(t);
  }
  std::vector<int64_t> idx(n);
  for (int64_t i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return nr[a] > nr[b]; });
  W.assign(m * n, 0.0);
  s.assign(n, 0.0);
  std::vector<cplx> Ys(n * n);
  for (int64_t c = 0; c < n; ++c) {
    const int64_t o = idx[c];
    s[c] = nr[o];
    for (int64_t i = 0; i < m; ++i) W[c * m + i] = (nr[o] > 0.0) ? A[o * m + i] / nr[o] : 0.0;
    for (int64_t i = 0; i < n; ++i) Ys[c * n + i] = Y[o * n + i];
  }
  Y.swap(Ys);
}

void jacobi_svd(int64_t n, const cplx *A, std::vector<cplx> &W, std::vector<double> &s,
                std::vector<cplx> &Y) {
  jacobi_tall(n, n, std::vector<cplx>(A, A + n * n), W, s, Y);
}

// General m x n: A = W diag(s) Y^H with k = min(m, n) columns in W and Y.
static void svd_general(int64_t m, int64_t n, const cplx *A, std::vector<cplx> &W,
                        std::vector<double> &s, std::vector<cplx> &Y) {
  if (m >= n) {
    jacobi_tall(m, n, std::vector<cplx>(A, A + m * n), W, s, Y);
    return;
  }
  // A^T = W' S Y'^H  =>  A = conj(Y') S conj(W')^H
  std::vector<cplx> At(n * m);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = 0; j < n; ++j) At[i * n + j] = A[j * m + i];
  std::vector<cplx> W2, Y2;
  jacobi_tall(n, m, At, W2, s, Y2);
  W.resize(m * m);
  Y.resize(n * m);
  for (size_t i = 0; i < W.size(); ++i) W[i] = std::conj(Y2[i]);
  for (size_t i = 0; i < Y.size(); ++i) Y[i] = std::conj(W2[i]);
}

static int64_t trunc_rank(const std::vector<double> &s, double eps) {
  double tot = 0.0;
  for (double v : s) tot += v * v;
  tot = std::sqrt(tot);
  if (tot == 0.0) return 0;
  const int64_t k = (int64_t)s.size();
  std::vector<double> tail(k + 1, 0.0);
  for (int64_t i = k - 1; i >= 0; --i) tail[i] = tail[i + 1] + s[i] * s[i];
  for (int64_t r = 0; r <= k; ++r)
    if (std::sqrt(tail[r]) <= eps * tot) return r;
  return k;
}

// U' = W_r diag(s_r), V' = conj(Y_r)  for block = W diag(s) Y^H
static void from_svd(int64_t m, int64_t n, const std::vector<cplx> &W, const std::vector<double> &s,
                     const std::vector<cplx> &Y, int64_t r, std::vector<cplx> &U, std::vector<cplx> &V) {
  U.assign(m * r, 0.0);
  V.assign(n * r, 0.0);
  for (int64_t c = 0; c < r; ++c) {
    for (int64_t i = 0; i < m; ++i) U[c * m + i] = W[c * m + i] * s[c];
    for (int64_t i = 0; i < n; ++i) V[c * n + i] = std::conj(Y[c * n + i]);
  }
}

static void recompress(int64_t m, int64_t n, int64_t k, std::vector<cplx> &U, std::vector<cplx> &V,
                       double eps, int &rank) {
  if (k == 0) { rank = 0; U.clear(); V.clear(); return; }
  std::vector<cplx> Qu, Ru, Qv, Rv;
  int64_t ku, kv;
  householder_qr(m, k, U.data(), Qu, Ru, ku);
  householder_qr(n, k, V.data(), Qv, Rv, kv);
  // S = Ru Rv^T  (ku x kv)
  std::vector<cplx> S(ku * kv, 0.0);
  for (int64_t j = 0; j < kv; ++j)
    for (int64_t i = 0; i < ku; ++i) {
      cplx acc = 0.0;
      for (int64_t l = 0; l < k; ++l) acc += Ru[l * ku + i] * Rv[l * kv + j];
      S[j * ku + i] = acc;
    }
  std::vector<cplx> W, Y;
  std::vector<double> s;
  svd_general(ku, kv, S.data(), W, s, Y);
  const int64_t r = trunc_rank(s, eps);
  const int64_t kk = (int64_t)s.size();
  std::vector<cplx> U2(m * r, 0.0), V2(n * r, 0.0);
  for (int64_t c = 0; c < r; ++c) {
    for (int64_t i = 0; i < m; ++i) {
      cplx acc = 0.0;
      for (int64_t l = 0; l < ku; ++l) acc += Qu[l * m + i] * W[c * ku + l];
      U2[c * m + i] = acc * s[c];
    }
    for (int64_t i = 0; i < n; ++i) {
      cplx acc = 0.0;
      for (int64_t l = 0; l < kv; ++l) acc += Qv[l * n + i] * std::conj(Y[c * kv + l]);
      V2[c * n + i] = acc;
    }
  }
  (void)kk;
  U.swap(U2);
  V.swap(V2);
  rank = (int)r;
}

// Recompression from the Gram matrices of the ACA factors (the device path,
// which forms G_U = U^H U and G_V = V^H V and then U T_U, V T_V).  With
// G_V = P diag(l) P^H (Jacobi), V = Q_V S P^H, S = diag(sqrt(l)), Q_V
// orthonormal; the block U V^T = B Q_V^T with B = U conj(P) S, and
// B^H B = S P^T G_U conj(P) S = Y diag(s^2) Y^H (Jacobi), s the singular
// values of the block.  The best rank-r approximation (the truncation rule
// of the QR + SVD route) is (B Y_r)(Q_V conj(Y_r))^T, so
//   T_U = conj(P) S Y_r,   T_V = P S^-1 conj(Y_r)   (k x r each).
// Directions of V with sqrt(l) <= 1e-12 of the largest carry no weight and
// are dropped (S^-1 = 0 there).  The squared conditioning of the Gram route
// limits the accuracy to about 1e-8 of the block norm, far below the ACA
// tolerance.
void recompress_from_grams(int64_t k, const cplx *GU, const cplx *GV, double eps, std::vector<cplx> &TU,
                           std::vector<cplx> &TV, int &rank) {
  TU.clear();
  TV.clear();
  rank = 0;
  if (k <= 0) return;
  std::vector<cplx> W, P, Y;
  std::vector<double> l;
  jacobi_svd(k, GV, W, l, P);               // Hermitian PSD: singular values = eigenvalues
  std::vector<double> sv(k), si(k);
  const double lmax = l.empty() ? 0.0 : std::max(l[0], 0.0);
  for (int64_t j = 0; j < k; ++j) {
    const double x = std::sqrt(std::max(l[j], 0.0));
    const bool keep = lmax > 0.0 && x > 1e-12 * std::sqrt(lmax);
    sv[j] = keep ? x : 0.0;
    si[j] = keep ? 1.0 / x : 0.0;
  }
  // H = S P^T G_U conj(P) S
  std::vector<cplx> T(k * k, 0.0), H(k * k, 0.0);
  for (int64_t c = 0; c < k; ++c)          // T = G_U conj(P)
    for (int64_t i = 0; i < k; ++i) {
      cplx acc = 0.0;
      for (int64_t q = 0; q < k; ++q) acc += GU[q * k + i] * std::conj(P[c * k + q]);
      T[c * k + i] = acc;
    }
  for (int64_t c = 0; c < k; ++c)
    for (int64_t i = 0; i < k; ++i) {
      cplx acc = 0.0;
      for (int64_t q = 0; q < k; ++q) acc += P[i * k + q] * T[c * k + q];     // (P^T)_iq = P_qi
      H[c * k + i] = sv[i] * acc * sv[c];
    }
  std::vector<double> s2;
  jacobi_svd(k, H.data(), W, s2, Y);
  std::vector<double> s(k);
  for (int64_t j = 0; j < k; ++j) s[j] = std::sqrt(std::max(s2[j], 0.0));
  const int64_t r = trunc_rank(s, eps);
  TU.assign(k * r, 0.0);
  TV.assign(k * r, 0.0);
  for (int64_t c = 0; c < r; ++c)
    for (int64_t i = 0; i < k; ++i) {
      cplx au = 0.0, av = 0.0;
      for (int64_t q = 0; q < k; ++q) {
        au += std::conj(P[q * k + i]) * sv[q] * Y[c * k + q];
        av += P[q * k + i] * si[q] * std::conj(Y[c * k + q]);
      }
      TU[c * k + i] = au;
      TV[c * k + i] = av;
    }
  rank = (int)r;
}

void aca_block(const Galerkin &op, const int64_t *rows, int64_t m, const int64_t *cols, int64_t n,
               double eps, std::vector<cplx> &U, std::vector<cplx> &V, int &rank) {
  const double limit = (double)(m * n) / (double)(m + n);
  std::vector<cplx> Uc, Vc;     // column-major growing factors
  std::vector<char> used(m, 0);
  std::vector<cplx> row(n), col(m);
  int64_t k = 0, i = 0;
  double norm2 = 0.0;
  bool full = false;
  while (true) {
    if ((double)(k + 1) >= limit) { full = true; break; }
    for (int64_t j = 0; j < n; ++j) {
      cplx z = op.entry(rows[i], cols[j]);
      for (int64_t l = 0; l < k; ++l) z -= Uc[l * m + i] * Vc[l * n + j];
      row[j] = z;
    }
    used[i] = 1;
    int64_t jp = 0;
    double best = std::abs(row[0]);
    for (int64_t j = 1; j < n; ++j) {
      const double a = std::abs(row[j]);
      if (a > best) { best = a; jp = j; }
    }
    if (best == 0.0) {
      int64_t nx = -1;
      for (int64_t r = 0; r < m; ++r) if (!used[r]) { nx = r; break; }
      if (nx < 0) break;
      i = nx;
      continue;
    }
    const cplx piv = row[jp];
    for (int64_t a = 0; a < m; ++a) {
      cplx z = op.entry(rows[a], cols[jp]);
      for (int64_t l = 0; l < k; ++l) z -= Vc[l * n + jp] * Uc[l * m + a];
      col[a] = z;
    }
    double nu2 = 0.0, nv2 = 0.0;
    for (int64_t a = 0; a < m; ++a) nu2 += std::norm(col[a]);
    std::vector<cplx> v(n);
    for (int64_t j = 0; j < n; ++j) { v[j] = row[j] / piv; nv2 += std::norm(v[j]); }
    cplx cross = 0.0;
    for (int64_t l = 0; l < k; ++l) {
      cplx uu = 0.0, vv = 0.0;
      for (int64_t a = 0; a < m; ++a) uu += std::conj(Uc[l * m + a]) * col[a];
      for (int64_t j = 0; j < n; ++j) vv += std::conj(Vc[l * n + j]) * v[j];
      cross += uu * vv;
    }
    norm2 += 2.0 * cross.real() + nu2 * nv2;
    Uc.insert(Uc.end(), col.begin(), col.end());
    Vc.insert(Vc.end(), v.begin(), v.end());
    ++k;
    if (std::sqrt(nu2 * nv2) <= eps * std::sqrt(norm2)) break;
    bool all = true;
    for (int64_t a = 0; a < m; ++a) all = all && used[a];
    if (all) break;
    int64_t nx = -1;
    double bu = -1.0;
    for (int64_t a = 0; a < m; ++a)
      if (!used[a]) {
        const double av = std::abs(col[a]);
        if (av > bu) { bu = av; nx = a; }
      }
    i = nx;
  }
  if (full) {
    std::vector<cplx> B(m * n);   // column-major
    for (int64_t j = 0; j < n; ++j)
      for (int64_t a = 0; a < m; ++a) B[j * m + a] = op.entry(rows[a], cols[j]);
    std::vector<cplx> W, Y;
    std::vector<double> s;
    svd_general(m, n, B.data(), W, s, Y);
    const int64_t r = trunc_rank(s, eps);
    from_svd(m, n, W, s, Y, r, U, V);
    rank = (int)r;
    return;
  }
  U.swap(Uc);
  V.swap(Vc);
  recompress(m, n, k, U, V, eps, rank);
}

// ---------------------------------------------------------------- assembly
// f(i) for i in [0, n) on `threads` host threads; with a label, every tenth
// of the items started is reported on stderr.
template <class F>
static void parallel_for(int64_t n, int threads, F &&f, const char *label = nullptr) {
  std::atomic<int64_t> next{0};
  const int64_t tenth = std::max<int64_t>(n / 10, 1);
  auto work = [&]() {
    while (true) {
      const int64_t i = next.fetch_add(1);
      if (i >= n) break;
      if (label && i % tenth == 0) {
        std::fprintf(stderr, "[hps] %s: %lld of %lld\n", label, (long long)i, (long long)n);
        std::fflush(stderr);
      }
      f(i);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < threads; ++t) pool.emplace_back(work);
  work();
  for (auto &th : pool) th.join();
}

void build_hmatrix(const Mesh &mesh, const hps_params &p, HMatrix &H, const NearFill *near_fill,
                   const FarSample *far_sample) {
  const auto t_start = std::chrono::steady_clock::now();
  auto stage = [&](const char *what) {
    if (!p.verbose) return;
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    std::fprintf(stderr, "[hps] %s at %.2f s\n", what, sec);
    std::fflush(stderr);
  };
  Tree T;
  build_tree(mesh, p.leaf_max, p.leaf_box_min, T);
  std::vector<std::pair<int32_t, int32_t>> near, far;
  block_partition(T, p.eta, near, far);
  if (p.formulation == 1) {            // CFIE: not symmetric, both orders of every block
    const size_t nn0 = near.size(), nf0 = far.size();
    for (size_t b = 0; b < nn0; ++b)
      if (near[b].first != near[b].second) near.emplace_back(near[b].second, near[b].first);
    for (size_t b = 0; b < nf0; ++b) far.emplace_back(far[b].second, far[b].first);
    std::sort(near.begin(), near.end());
    std::sort(far.begin(), far.end());
  }
  Galerkin op(mesh, p.freq_hz, p.formulation == 1, p.cfie_alpha);
  int threads = p.host_threads > 0 ? p.host_threads : (int)std::thread::hardware_concurrency();
  if (threads < 1) threads = 1;

  H.N = mesh.N;
  H.nonsym = p.formulation == 1;
  H.M = (int64_t)T.leaf_node.size();
  H.perm = T.perm;
  H.gptr.resize(H.M + 1);
  for (int64_t g = 0; g < H.M; ++g) H.gptr[g] = T.nodes[T.leaf_node[g]].lo;
  H.gptr[H.M] = H.N;

  const int64_t nn = (int64_t)near.size();
  H.near_ts.resize(2 * nn);
  H.near_off.assign(nn + 1, 0);
  for (int64_t b = 0; b < nn; ++b) {
    H.near_ts[2 * b] = near[b].first;
    H.near_ts[2 * b + 1] = near[b].second;
    const int64_t mt = H.gptr[near[b].first + 1] - H.gptr[near[b].first];
    const int64_t ms = H.gptr[near[b].second + 1] - H.gptr[near[b].second];
    H.near_off[b + 1] = H.near_off[b] + mt * ms;
  }
  H.near_vals.assign(H.near_off[nn], 0.0);
  const int64_t nf = (int64_t)far.size();
  H.far_rng.resize(4 * nf);
  H.far_rank.assign(nf, 0);
  for (int64_t b = 0; b < nf; ++b) {
    const TreeNode &a = T.nodes[far[b].first], &c = T.nodes[far[b].second];
    H.far_rng[4 * b] = a.lo; H.far_rng[4 * b + 1] = a.hi;
    H.far_rng[4 * b + 2] = c.lo; H.far_rng[4 * b + 3] = c.hi;
  }

  stage("tree and block partition done");
  // Device work on its own thread: the ACA sampling of the far blocks, chunk
  // by chunk, then the near blocks.  Host threads recompress each chunk as it
  // arrives (blocks the device left over get the host ACA).
  std::mutex mu;
  std::condition_variable cv;
  std::deque<FarChunk> chunks;              // stable element addresses
  std::vector<const cplx *> src(far_sample ? nf : 0);
  std::vector<int32_t> raw_rank(far_sample ? nf : 0);
  std::vector<char> is_final(far_sample ? nf : 0, 0);
  int64_t ready = 0;                        // far blocks [0, ready) have arrived
  bool dev_done = false;
  std::thread dev_thread;
  std::exception_ptr dev_error;
  if (near_fill || far_sample) {
    dev_thread = std::thread([&]() {
      try {
        if (far_sample) {
          (*far_sample)(H, [&](FarChunk &&ch) {
            std::lock_guard<std::mutex> lk(mu);
            if (ch.b0 != ready || ch.b1 < ch.b0 || ch.b1 > nf) throw Error{HPS_EINVAL, "internal: device ACA chunk order"};
            chunks.push_back(std::move(ch));
            const FarChunk &c = chunks.back();
            for (int64_t b = c.b0; b < c.b1; ++b) {
              raw_rank[b] = c.rank[b - c.b0];
              src[b] = c.uv.data() + c.off[b - c.b0];
              is_final[b] = (char)(c.final && raw_rank[b] >= 0);
            }
            ready = c.b1;
            cv.notify_all();
          });
          stage("device ACA sampling done");
        }
        if (near_fill) (*near_fill)(H);
        stage("device near blocks done");
      } catch (...) {
        dev_error = std::current_exception();
      }
      std::lock_guard<std::mutex> lk(mu);
      dev_done = true;
      cv.notify_all();
    });
  }
  struct Joiner {            // the device thread is joined on every path out
    std::thread &t;
    ~Joiner() { if (t.joinable()) t.join(); }
  } joiner{dev_thread};
  if (!near_fill) {
    parallel_for(nn, threads, [&](int64_t b) {
      const int64_t t = H.near_ts[2 * b], s = H.near_ts[2 * b + 1];
      op.block(&H.perm[H.gptr[t]], H.gptr[t + 1] - H.gptr[t], &H.perm[H.gptr[s]],
               H.gptr[s + 1] - H.gptr[s], &H.near_vals[H.near_off[b]]);
    }, p.verbose ? "near blocks" : nullptr);
  }
  std::vector<std::vector<cplx>> Us(nf), Vs(nf);
  if (far_sample) {
    int64_t next = 0;
    const int64_t tenth = std::max<int64_t>(nf / 10, 1);
    auto work = [&]() {
      while (true) {
        int64_t b;
        {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait(lk, [&]() { return next < ready || dev_done; });
          if (next >= ready) break;           // device finished (or failed) and nothing is left
          b = next++;
        }
        if (p.verbose && b % tenth == 0) {
          std::fprintf(stderr, "[hps] far blocks (recompression): %lld of %lld\n", (long long)b, (long long)nf);
          std::fflush(stderr);
        }
        const int64_t tlo = H.far_rng[4 * b], thi = H.far_rng[4 * b + 1];
        const int64_t slo = H.far_rng[4 * b + 2], shi = H.far_rng[4 * b + 3];
        const int64_t m = thi - tlo, n = shi - slo, k = raw_rank[b];
        int r = 0;
        if (is_final[b]) {                    // recompressed on the device: copy
          r = (int)k;
          const cplx *u = src[b];
          Us[b].assign(u, u + m * k);
          Vs[b].assign(u + m * k, u + (m + n) * k);
        } else if (k < 0) {
          aca_block(op, &H.perm[tlo], m, &H.perm[slo], n, p.aca_tol, Us[b], Vs[b], r);
        } else if (k > 0) {
          const cplx *u = src[b];
          Us[b].assign(u, u + m * k);
          Vs[b].assign(u + m * k, u + (m + n) * k);
          recompress(m, n, k, Us[b], Vs[b], p.aca_tol, r);
        }
        H.far_rank[b] = r;
      }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < threads; ++t) pool.emplace_back(work);
    work();
    for (auto &th : pool) th.join();
    dev_thread.join();
    if (dev_error) std::rethrow_exception(dev_error);
    if (ready != nf) throw Error{HPS_EINVAL, "internal: device ACA left far blocks out"};
    chunks.clear();
  } else {
    parallel_for(nf, threads, [&](int64_t b) {
      const int64_t tlo = H.far_rng[4 * b], thi = H.far_rng[4 * b + 1];
      const int64_t slo = H.far_rng[4 * b + 2], shi = H.far_rng[4 * b + 3];
      int r = 0;
      aca_block(op, &H.perm[tlo], thi - tlo, &H.perm[slo], shi - slo, p.aca_tol, Us[b], Vs[b], r);
      H.far_rank[b] = r;
    }, p.verbose ? "far blocks (ACA)" : nullptr);
  }
  stage("far blocks done");
  H.far_off.assign(nf + 1, 0);
  for (int64_t b = 0; b < nf; ++b) H.far_off[b + 1] = H.far_off[b] + (int64_t)(Us[b].size() + Vs[b].size());
  H.far_uv.resize(H.far_off[nf]);
  parallel_for(nf, threads, [&](int64_t b) {
    std::copy(Us[b].begin(), Us[b].end(), H.far_uv.begin() + H.far_off[b]);
    std::copy(Vs[b].begin(), Vs[b].end(), H.far_uv.begin() + H.far_off[b] + (int64_t)Us[b].size());
    std::vector<cplx>().swap(Us[b]);
    std::vector<cplx>().swap(Vs[b]);
  });
  if (dev_thread.joinable()) dev_thread.join();
  if (dev_error) std::rethrow_exception(dev_error);
  stage("far factors assembled");
}

}  // namespace hps
