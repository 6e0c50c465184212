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
  h.nonsym = !Hs.empty() && Hs[0].nonsym;
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
    m.nrm.insert(m.nrm.end(), a.nrm.begin(), a.nrm.end());
    m.open = m.open || a.open;
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

namespace hps {

// Pivot blocks are at most max_size unknowns (the register-resident inverse):
// a larger group is cut into consecutive sub-groups of near-equal size, which
// the setup eliminates one after the other like any other groups.  The near
// blocks are cut along the same lines (upper triangle of the group pattern
// kept, or every sub-block of a non-symmetric H-matrix); far blocks refer to
// tree-position ranges and are unchanged.
void split_groups(HMatrix &H, int64_t max_size) {
  const int64_t M = H.M;
  bool any = false;
  for (int64_t g = 0; g < M; ++g) any = any || (H.gptr[g + 1] - H.gptr[g] > max_size);
  if (!any) return;
  std::vector<int64_t> ng0(M + 1, 0), gptr{0};
  for (int64_t g = 0; g < M; ++g) {
    const int64_t s = H.gptr[g + 1] - H.gptr[g];
    const int64_t parts = (s + max_size - 1) / max_size, base = s / parts, extra = s % parts;
    int64_t pos = H.gptr[g];
    for (int64_t q = 0; q < parts; ++q) {
      pos += base + (q < extra ? 1 : 0);
      gptr.push_back(pos);
    }
    ng0[g + 1] = ng0[g] + parts;
  }
  std::vector<int32_t> ts;
  std::vector<int64_t> off{0};
  std::vector<cplx> vals;
  ts.reserve(H.near_ts.size());
  vals.reserve(H.near_vals.size());
  for (int64_t b = 0; b < H.n_near(); ++b) {
    const int32_t t = H.near_ts[2 * b], s = H.near_ts[2 * b + 1];
    const int64_t ns = H.gptr[s + 1] - H.gptr[s];
    const cplx *blk = H.near_vals.data() + H.near_off[b];
    for (int64_t ta = ng0[t]; ta < ng0[t + 1]; ++ta)
      for (int64_t sb = (t == s && !H.nonsym ? ta : ng0[s]); sb < ng0[s + 1]; ++sb) {
        const int64_t r0 = gptr[ta] - H.gptr[t], r1 = gptr[ta + 1] - H.gptr[t];
        const int64_t c0 = gptr[sb] - H.gptr[s], c1 = gptr[sb + 1] - H.gptr[s];
        for (int64_t r = r0; r < r1; ++r)
          vals.insert(vals.end(), blk + r * ns + c0, blk + r * ns + c1);
        ts.push_back((int32_t)ta);
        ts.push_back((int32_t)sb);
        off.push_back((int64_t)vals.size());
      }
  }
  if (ng0[M] > INT32_MAX) throw Error{HPS_EINVAL, "too many groups"};
  H.M = ng0[M];
  H.gptr = std::move(gptr);
  H.near_ts = std::move(ts);
  H.near_off = std::move(off);
  H.near_vals = std::move(vals);
}

}  // namespace hps
