// Batches of independent scattering problems merged into one block-diagonal
// system, so that every setup level and solve stage of all problems runs in
// the same launches.  Pure index arithmetic on the host.
#include <algorithm>

#include "hps_internal.h"

namespace hps {

void merge_problems(const std::vector<Mesh> &meshes, const std::vector<HMatrix> &Hs, Mesh &out, HMatrix &H,
                    std::vector<int64_t> &nseg, std::vector<int64_t> &gseg) {
  const size_t P = meshes.size();
  if (P == 0 || Hs.size() != P) throw Error{HPS_EINVAL, "empty batch"};
  nseg.assign(P + 1, 0);
  gseg.assign(P + 1, 0);
  int64_t nv = 0, nt = 0, N = 0, M = 0, nnear = 0, nfar = 0, ne = 0, fe = 0;
  for (size_t p = 0; p < P; ++p) {
    if (Hs[p].N != meshes[p].N) throw Error{HPS_EINVAL, "H-matrix does not match its mesh"};
    nv += meshes[p].nv;
    nt += meshes[p].nt;
    N += meshes[p].N;
    M += Hs[p].M;
    nnear += Hs[p].n_near();
    nfar += Hs[p].n_far();
    ne += (int64_t)Hs[p].near_vals.size();
    fe += (int64_t)Hs[p].far_uv.size();
    nseg[p + 1] = N;
    gseg[p + 1] = M;
  }
  if (N > INT32_MAX || M > INT32_MAX || nt > INT32_MAX || nv > INT32_MAX)
    throw Error{HPS_EINVAL, "batch too large for 32-bit indices"};
  Mesh m;
  m.nv = nv;
  m.nt = nt;
  m.N = N;
  m.xyz.reserve(3 * nv); m.tri.reserve(3 * nt); m.cen.reserve(3 * nt); m.area.reserve(nt);
  m.edge.reserve(2 * N); m.tp.reserve(N); m.tm.reserve(N); m.vp.reserve(N); m.vm.reserve(N); m.len.reserve(N);
  HMatrix h;
  h.N = N;
  h.M = M;
  h.perm.reserve(N); h.gptr.reserve(M + 1); h.near_ts.reserve(2 * nnear); h.near_off.reserve(nnear + 1);
  h.near_vals.reserve(ne); h.far_rng.reserve(4 * nfar); h.far_rank.reserve(nfar); h.far_off.reserve(nfar + 1);
  h.far_uv.reserve(fe);
  h.gptr.push_back(0);
  h.near_off.push_back(0);
  h.far_off.push_back(0);
  int32_t voff = 0, toff = 0;
  for (size_t p = 0; p < P; ++p) {
    const Mesh &a = meshes[p];
    const HMatrix &b = Hs[p];
    const int64_t no = nseg[p], go = gseg[p];
    m.xyz.insert(m.xyz.end(), a.xyz.begin(), a.xyz.end());
    for (int32_t v : a.tri) m.tri.push_back(v + voff);
    m.cen.insert(m.cen.end(), a.cen.begin(), a.cen.end());
    m.area.insert(m.area.end(), a.area.begin(), a.area.end());
    m.hmax = std::max(m.hmax, a.hmax);
    for (int32_t v : a.edge) m.edge.push_back(v + voff);
    for (int64_t n = 0; n < a.N; ++n) {
      m.tp.push_back(a.tp[n] + toff);
      m.tm.push_back(a.tm[n] + toff);
      m.vp.push_back(a.vp[n] + voff);
      m.vm.push_back(a.vm[n] + voff);
    }
    m.len.insert(m.len.end(), a.len.begin(), a.len.end());
    for (int64_t x : b.perm) h.perm.push_back(x + no);
    for (int64_t g = 1; g <= b.M; ++g) h.gptr.push_back(b.gptr[g] + no);
    const int64_t nbase = h.near_off.back(), fbase = h.far_off.back();
    for (int32_t x : b.near_ts) h.near_ts.push_back((int32_t)(x + go));
    for (int64_t i = 1; i < (int64_t)b.near_off.size(); ++i) h.near_off.push_back(b.near_off[i] + nbase);
    h.near_vals.insert(h.near_vals.end(), b.near_vals.begin(), b.near_vals.end());
    for (int64_t x : b.far_rng) h.far_rng.push_back(x + no);
    h.far_rank.insert(h.far_rank.end(), b.far_rank.begin(), b.far_rank.end());
    for (int64_t i = 1; i < (int64_t)b.far_off.size(); ++i) h.far_off.push_back(b.far_off[i] + fbase);
    h.far_uv.insert(h.far_uv.end(), b.far_uv.begin(), b.far_uv.end());
    voff += (int32_t)a.nv;
    toff += (int32_t)a.nt;
  }
  out = std::move(m);
  H = std::move(h);
}

}  // namespace hps
