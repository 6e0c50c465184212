// Mesh validation and RWG construction (host).
//
// One RWG unknown per interior edge (Sec. II, Galerkin RWG discretisation).
// Edges are numbered in lexicographic order of (min vertex, max vertex); T+ is
// the triangle whose counter-clockwise boundary runs from the smaller to the
// larger vertex id along the edge.  f = +(l/2A+)(r - v+) on T+, -(l/2A-)(r - v-)
// on T-.
#include <algorithm>
#include <cmath>

#include "hps_internal.h"

namespace hps {

namespace {
struct EdgeRec {
  int32_t a, b;     // a < b
  int32_t t;        // triangle
  int32_t fwd;      // 1 if the triangle runs a -> b
};
}  // namespace

void build_rwg(Mesh &m, bool allow_open) {
  const int64_t nt = m.nt, nv = m.nv;
  if (nt <= 0 || nv <= 0) throw Error{HPS_EINVAL, "empty mesh"};
  for (int64_t i = 0; i < 3 * nt; ++i)
    if (m.tri[i] < 0 || m.tri[i] >= nv) throw Error{HPS_EINVAL, "vertex index out of range"};
  m.cen.assign(3 * nt, 0.0);
  m.area.assign(nt, 0.0);
  m.nrm.assign(3 * nt, 0.0);
  m.open = allow_open;
  double hmax = 0.0;
  for (int64_t t = 0; t < nt; ++t) {
    const double *p[3];
    for (int c = 0; c < 3; ++c) p[c] = &m.xyz[3 * m.tri[3 * t + c]];
    for (int d = 0; d < 3; ++d) m.cen[3 * t + d] = (p[0][d] + p[1][d] + p[2][d]) / 3.0;
    double u[3], v[3];
    for (int d = 0; d < 3; ++d) { u[d] = p[1][d] - p[0][d]; v[d] = p[2][d] - p[0][d]; }
    const double cx = u[1] * v[2] - u[2] * v[1];
    const double cy = u[2] * v[0] - u[0] * v[2];
    const double cz = u[0] * v[1] - u[1] * v[0];
    m.area[t] = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
    if (m.area[t] > 0.0) {
      m.nrm[3 * t] = cx / (2.0 * m.area[t]);
      m.nrm[3 * t + 1] = cy / (2.0 * m.area[t]);
      m.nrm[3 * t + 2] = cz / (2.0 * m.area[t]);
    }
    for (int e = 0; e < 3; ++e) {
      const double *a = p[e], *b = p[(e + 1) % 3];
      const double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
      hmax = std::max(hmax, std::sqrt((dx * dx + dy * dy) + dz * dz));
    }
    const int32_t *tv = &m.tri[3 * t];
    if (tv[0] == tv[1] || tv[1] == tv[2] || tv[0] == tv[2])
      throw Error{HPS_EINVAL, "degenerate triangle " + std::to_string(t)};
  }
  m.hmax = hmax;
  for (int64_t t = 0; t < nt; ++t)
    if (!(m.area[t] > 1e-12 * hmax * hmax))
      throw Error{HPS_EINVAL, "degenerate triangle " + std::to_string(t)};

  std::vector<EdgeRec> recs;
  recs.reserve(3 * nt);
  for (int64_t t = 0; t < nt; ++t)
    for (int e = 0; e < 3; ++e) {
      const int32_t a = m.tri[3 * t + e], b = m.tri[3 * t + (e + 1) % 3];
      recs.push_back({std::min(a, b), std::max(a, b), (int32_t)t, a < b ? 1 : 0});
    }
  std::sort(recs.begin(), recs.end(), [](const EdgeRec &x, const EdgeRec &y) {
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    return x.t < y.t;
  });
  m.edge.clear(); m.tp.clear(); m.tm.clear(); m.vp.clear(); m.vm.clear(); m.len.clear();
  size_t i = 0;
  while (i < recs.size()) {
    size_t j = i;
    while (j < recs.size() && recs[j].a == recs[i].a && recs[j].b == recs[i].b) ++j;
    const size_t cnt = j - i;
    if (cnt == 1) {
      if (!allow_open)
        throw Error{HPS_EINVAL, "open boundary edge (" + std::to_string(recs[i].a) + "," + std::to_string(recs[i].b) +
                                    ")"};
      i = j;               // rim of an open sheet: no unknown
      continue;
    }
    if (cnt > 2) throw Error{HPS_EINVAL, "non-manifold edge"};
    const EdgeRec &r0 = recs[i], &r1 = recs[i + 1];
    if (r0.fwd == r1.fwd) throw Error{HPS_EINVAL, "inconsistent triangle orientation"};
    const EdgeRec &P = r0.fwd ? r0 : r1;
    const EdgeRec &Q = r0.fwd ? r1 : r0;
    auto free_vertex = [&](int32_t t) {
      for (int c = 0; c < 3; ++c) {
        const int32_t v = m.tri[3 * t + c];
        if (v != r0.a && v != r0.b) return v;
      }
      return (int32_t)-1;
    };
    m.edge.push_back(r0.a);
    m.edge.push_back(r0.b);
    m.tp.push_back(P.t);
    m.tm.push_back(Q.t);
    m.vp.push_back(free_vertex(P.t));
    m.vm.push_back(free_vertex(Q.t));
    const double *pa = &m.xyz[3 * r0.a], *pb = &m.xyz[3 * r0.b];
    const double dx = pb[0] - pa[0], dy = pb[1] - pa[1], dz = pb[2] - pa[2];
    m.len.push_back(std::sqrt((dx * dx + dy * dy) + dz * dz));
    i = j;
  }
  m.N = (int64_t)m.tp.size();
}

}  // namespace hps
