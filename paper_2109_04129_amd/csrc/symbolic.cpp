// Symbolic phase of the setup (host, integer work only).
//
// The paper eliminates the groups one by one with Schur steps that keep every
// fill-in block (eqs. 16-23) and reduces fill with a graph ordering (Sloan's,
// Sec. III.A).  Here the order is a geometric nested dissection of the group
// graph (touching leaves): split the groups at the median of the longest axis
// of their centroids, take as separator the smaller of the two boundary sets,
// order both halves recursively and the separator last.  Any order gives the
// same two-term result in exact arithmetic; this one bounds fill and gives a
// balanced elimination tree, whose levels are the units of parallel work.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "hps_internal.h"

namespace hps {

namespace {

struct ND {
  const std::vector<std::vector<int32_t>> &adj;
  const std::vector<double> &cen;   // M * 3
  std::vector<int32_t> &order;
  std::vector<int32_t> mark;        // scratch side flags
  ND(const std::vector<std::vector<int32_t>> &a, const std::vector<double> &c, std::vector<int32_t> &o)
      : adj(a), cen(c), order(o), mark(a.size(), 0) {}

  void run(std::vector<int32_t> S) {
    if (S.empty()) return;
    if (S.size() <= 3) {
      std::sort(S.begin(), S.end());
      order.insert(order.end(), S.begin(), S.end());
      return;
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t g : S)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], cen[3 * g + d]);
        hi[d] = std::max(hi[d], cen[3 * g + d]);
      }
    int ax = 0;
    for (int d = 1; d < 3; ++d)
      if (hi[d] - lo[d] > hi[ax] - lo[ax]) ax = d;
    std::sort(S.begin(), S.end(), [&](int32_t a, int32_t b) {
      const double ca = cen[3 * a + ax], cb = cen[3 * b + ax];
      return ca < cb || (ca == cb && a < b);
    });
    const size_t h = S.size() / 2;
    std::vector<int32_t> L(S.begin(), S.begin() + h), R(S.begin() + h, S.end());
    for (int32_t g : L) mark[g] = 1;
    for (int32_t g : R) mark[g] = 2;
    std::vector<int32_t> sepL, sepR, restL, restR;
    for (int32_t g : L) {
      bool b = false;
      for (int32_t x : adj[g]) b = b || mark[x] == 2;
      (b ? sepL : restL).push_back(g);
    }
    for (int32_t g : R) {
      bool b = false;
      for (int32_t x : adj[g]) b = b || mark[x] == 1;
      (b ? sepR : restR).push_back(g);
    }
    for (int32_t g : S) mark[g] = 0;
    if (sepL.size() <= sepR.size()) {
      run(restL);
      run(R);
      std::sort(sepL.begin(), sepL.end());
      order.insert(order.end(), sepL.begin(), sepL.end());
    } else {
      run(L);
      run(restR);
      std::sort(sepR.begin(), sepR.end());
      order.insert(order.end(), sepR.begin(), sepR.end());
    }
  }
};

}  // namespace

void make_plan(const HMatrix &H, const Mesh &mesh, int ordering, const std::vector<int64_t> &gseg, Plan &P) {
  const int64_t M = H.M;
  P.M = M;
  P.N = H.N;
  std::vector<std::vector<int32_t>> adj(M);
  for (int64_t b = 0; b < H.n_near(); ++b) {
    const int32_t t = H.near_ts[2 * b], s = H.near_ts[2 * b + 1];
    if (t != s) { adj[t].push_back(s); adj[s].push_back(t); }
  }
  std::vector<double> cen(3 * M, 0.0);
  for (int64_t g = 0; g < M; ++g) {
    const int64_t n = H.gptr[g + 1] - H.gptr[g];
    for (int64_t p = H.gptr[g]; p < H.gptr[g + 1]; ++p) {
      const int64_t r = H.perm[p];
      for (int d = 0; d < 3; ++d)
        cen[3 * g + d] += 0.5 * (mesh.xyz[3 * mesh.edge[2 * r] + d] + mesh.xyz[3 * mesh.edge[2 * r + 1] + d]);
    }
    for (int d = 0; d < 3; ++d) cen[3 * g + d] /= (double)std::max<int64_t>(n, 1);
  }
  if (gseg.size() < 2 || gseg.front() != 0 || gseg.back() != M)
    throw Error{HPS_EINVAL, "internal: problem group ranges do not cover the groups"};
  P.order.clear();
  if (ordering == 1) {
    P.order.resize(M);
    std::iota(P.order.begin(), P.order.end(), 0);
  } else {
    ND nd(adj, cen, P.order);
    for (size_t q = 0; q + 1 < gseg.size(); ++q) {   // problems never couple: order each on its own
      std::vector<int32_t> grp(gseg[q + 1] - gseg[q]);
      std::iota(grp.begin(), grp.end(), (int32_t)gseg[q]);
      nd.run(grp);
    }
  }
  if ((int64_t)P.order.size() != M) throw Error{HPS_EINVAL, "internal: ordering lost groups"};
  P.pos.assign(M, -1);
  for (int64_t e = 0; e < M; ++e) P.pos[P.order[e]] = (int32_t)e;

  // symbolic elimination with the elimination tree
  std::vector<std::vector<int32_t>> children(M);
  std::vector<std::vector<int32_t>> str(M);
  std::vector<int32_t> marker(M, -1), parent(M, -1);
  P.level.assign(M, 0);
  for (int64_t e = 0; e < M; ++e) {
    std::vector<int32_t> &s = str[e];
    marker[e] = (int32_t)e;
    for (int32_t g : adj[P.order[e]]) {
      const int32_t f = P.pos[g];
      if (f > e && marker[f] != e) { marker[f] = (int32_t)e; s.push_back(f); }
    }
    int32_t lev = 0;
    for (int32_t c : children[e]) {
      for (int32_t f : str[c])
        if (f > e && marker[f] != e) { marker[f] = (int32_t)e; s.push_back(f); }
      lev = std::max(lev, P.level[c] + 1);
    }
    std::sort(s.begin(), s.end());
    P.level[e] = lev;
    if (!s.empty()) {
      parent[e] = s[0];
      children[s[0]].push_back((int32_t)e);
    }
  }
  P.size.resize(M);
  P.uoff.resize(M + 1);
  P.uoff[0] = 0;
  for (int64_t e = 0; e < M; ++e) {
    const int32_t g = P.order[e];
    P.size[e] = H.gptr[g + 1] - H.gptr[g];
    P.uoff[e + 1] = P.uoff[e] + P.size[e];
  }
  P.later_ptr.assign(M + 1, 0);
  for (int64_t e = 0; e < M; ++e) P.later_ptr[e + 1] = P.later_ptr[e] + (int64_t)str[e].size();
  P.later.resize(P.later_ptr[M]);
  P.col_off.resize(P.later_ptr[M]);
  P.width.resize(M);
  P.panel_off.resize(M + 1);
  P.panel_off[0] = 0;
  P.n_U = 0;
  P.n_D = 0;
  P.setup_flops = 0.0;
  for (int64_t e = 0; e < M; ++e) {
    int64_t c = P.size[e];
    double nF = 0.0, sq = 0.0;
    for (size_t i = 0; i < str[e].size(); ++i) {
      const int32_t f = str[e][i];
      P.later[P.later_ptr[e] + i] = f;
      P.col_off[P.later_ptr[e] + i] = c;
      c += P.size[f];
      nF += (double)P.size[f];
      sq += (double)P.size[f] * (double)P.size[f];
    }
    P.width[e] = c;
    P.panel_off[e + 1] = P.panel_off[e] + P.size[e] * c;
    P.n_D += P.size[e] * P.size[e];
    P.n_U += P.size[e] * (c - P.size[e]);
    const double ni = (double)P.size[e];
    P.setup_flops += 8.0 * (ni * ni * ni + ni * ni * nF + ni * (nF * nF + sq) / 2.0);
  }
  P.panel_elems = P.panel_off[M];
  P.n_upper_blocks = P.later_ptr[M];
  P.n_levels = 0;
  for (int64_t e = 0; e < M; ++e) P.n_levels = std::max(P.n_levels, P.level[e] + 1);
  P.level_ptr.assign(P.n_levels + 1, 0);
  for (int64_t e = 0; e < M; ++e) P.level_ptr[P.level[e] + 1]++;
  for (int l = 0; l < P.n_levels; ++l) P.level_ptr[l + 1] += P.level_ptr[l];
  P.level_piv.resize(M);
  std::vector<int64_t> fillp(P.level_ptr.begin(), P.level_ptr.end() - 1);
  for (int64_t e = 0; e < M; ++e) P.level_piv[fillp[P.level[e]]++] = (int32_t)e;
}

}  // namespace hps
