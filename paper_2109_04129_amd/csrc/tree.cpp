// Octree clusters and the near / far split (host).
//
// Admissibility (eq. 10) on cubic cells, eta dist >= min(dia), with
// dia = sqrt(3) * side and dist = the Euclidean gap between the two closed
// cells, decided on integer cell coordinates (units of the finest grid):
// 3 s^2 <= eta^2 d^2 with s the smaller side and d^2 the squared gap.  Two
// cells that do not touch have a gap of at least the smaller side along some
// axis, so for eta >= sqrt(3) the test is "the cells do not touch"; eta = 0
// admits nothing (no far field).
//
// Cell coordinates: q = floor((p - lo) / s * 2^21), lo = per-axis minimum of
// the edge midpoints, s = largest extent * (1 + 2^-20).  A cell splits while it
// holds more than leaf_max points and its children would be at least box_min
// wide (electrically sized leaves, Sec. V.A); children in the order
// 4 bx + 2 by + bz;
// unknowns inside a leaf sorted by RWG index; tree order = depth-first.
#include <algorithm>
#include <cmath>

#include "hps_internal.h"

namespace hps {

static const int kDepth = 21;

void build_tree(const Mesh &m, int leaf_max, double box_min, Tree &T) {
  const int64_t N = m.N;
  std::vector<double> pt(3 * N);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t n = 0; n < N; ++n)
    for (int d = 0; d < 3; ++d) {
      const double v = 0.5 * (m.xyz[3 * m.edge[2 * n] + d] + m.xyz[3 * m.edge[2 * n + 1] + d]);
      pt[3 * n + d] = v;
      lo[d] = std::min(lo[d], v);
      hi[d] = std::max(hi[d], v);
    }
  double ext = 0.0;
  for (int d = 0; d < 3; ++d) ext = std::max(ext, hi[d] - lo[d]);
  const double s = ext * (1.0 + std::ldexp(1.0, -20));
  const double scale = (double)(1 << kDepth);
  // deepest level whose cells are at least box_min wide
  int depth_cap = kDepth;
  if (box_min > 0.0) {
    depth_cap = 0;
    while (depth_cap < kDepth && s / std::ldexp(1.0, depth_cap + 1) >= box_min) ++depth_cap;
  }
  std::vector<int64_t> q(3 * N);
  for (int64_t n = 0; n < N; ++n)
    for (int d = 0; d < 3; ++d) {
      int64_t v = (int64_t)std::floor((pt[3 * n + d] - lo[d]) / s * scale);
      v = std::max<int64_t>(0, std::min<int64_t>(v, (1 << kDepth) - 1));
      q[3 * n + d] = v;
    }

  // Recursive construction with explicit lists; nodes numbered depth-first.
  T.nodes.clear(); T.child.clear(); T.perm.clear(); T.leaf_node.clear();
  struct Item { int depth; int64_t ijk[3]; std::vector<int64_t> pts; int32_t parent; };
  // depth-first: process children in order immediately (stack in reverse).
  std::vector<Item> stack;
  Item root{0, {0, 0, 0}, {}, -1};
  root.pts.resize(N);
  for (int64_t n = 0; n < N; ++n) root.pts[n] = n;
  stack.push_back(std::move(root));
  std::vector<std::vector<int32_t>> kids;
  while (!stack.empty()) {
    Item it = std::move(stack.back());
    stack.pop_back();
    const int32_t id = (int32_t)T.nodes.size();
    TreeNode nd;
    nd.depth = it.depth;
    for (int d = 0; d < 3; ++d) nd.ijk[d] = it.ijk[d];
    nd.lo = nd.hi = -1;
    T.nodes.push_back(nd);
    kids.emplace_back();
    if (it.parent >= 0) kids[it.parent].push_back(id);
    if ((int64_t)it.pts.size() <= leaf_max || it.depth >= depth_cap) {
      std::sort(it.pts.begin(), it.pts.end());
      T.nodes[id].leaf = (int32_t)T.leaf_node.size();
      T.leaf_node.push_back(id);
      T.nodes[id].lo = (int64_t)T.perm.size();
      T.perm.insert(T.perm.end(), it.pts.begin(), it.pts.end());
      T.nodes[id].hi = (int64_t)T.perm.size();
      continue;
    }
    const int sh = kDepth - it.depth - 1;
    std::vector<int64_t> part[8];
    for (int64_t p : it.pts) {
      const int c = (int)(4 * ((q[3 * p] >> sh) & 1) + 2 * ((q[3 * p + 1] >> sh) & 1) +
                          ((q[3 * p + 2] >> sh) & 1));
      part[c].push_back(p);
    }
    for (int c = 7; c >= 0; --c) {
      if (part[c].empty()) continue;
      Item ch{it.depth + 1,
              {2 * it.ijk[0] + ((c >> 2) & 1), 2 * it.ijk[1] + ((c >> 1) & 1), 2 * it.ijk[2] + (c & 1)},
              std::move(part[c]), id};
      stack.push_back(std::move(ch));
    }
  }
  // children lists and ranges (post-order fill of lo/hi for inner nodes)
  for (size_t id = 0; id < T.nodes.size(); ++id) {
    T.nodes[id].first_child = (int32_t)T.child.size();
    T.nodes[id].n_child = (int32_t)kids[id].size();
    T.child.insert(T.child.end(), kids[id].begin(), kids[id].end());
  }
  for (int64_t id = (int64_t)T.nodes.size() - 1; id >= 0; --id) {
    TreeNode &nd = T.nodes[id];
    if (nd.n_child == 0) continue;
    nd.lo = T.nodes[T.child[nd.first_child]].lo;
    nd.hi = T.nodes[T.child[nd.first_child + nd.n_child - 1]].hi;
  }
}

bool cells_touch(const TreeNode &a, const TreeNode &b) {
  for (int d = 0; d < 3; ++d) {
    const int64_t alo = a.ijk[d] << (kDepth - a.depth), ahi = (a.ijk[d] + 1) << (kDepth - a.depth);
    const int64_t blo = b.ijk[d] << (kDepth - b.depth), bhi = (b.ijk[d] + 1) << (kDepth - b.depth);
    if (alo > bhi || blo > ahi) return false;
  }
  return true;
}

bool admissible(const TreeNode &a, const TreeNode &b, double eta) {
  int64_t d2 = 0;
  for (int d = 0; d < 3; ++d) {
    const int64_t alo = a.ijk[d] << (kDepth - a.depth), ahi = (a.ijk[d] + 1) << (kDepth - a.depth);
    const int64_t blo = b.ijk[d] << (kDepth - b.depth), bhi = (b.ijk[d] + 1) << (kDepth - b.depth);
    const int64_t gap = std::max<int64_t>(0, std::max(blo - ahi, alo - bhi));
    d2 += gap * gap;
  }
  const int64_t side = (int64_t)1 << (kDepth - std::max(a.depth, b.depth));
  return eta * eta * (double)d2 >= 3.0 * (double)(side * side);
}

void block_partition(const Tree &T, double eta, std::vector<std::pair<int32_t, int32_t>> &near,
                     std::vector<std::pair<int32_t, int32_t>> &far) {
  near.clear();
  far.clear();
  std::vector<std::pair<int32_t, int32_t>> st{{0, 0}};
  while (!st.empty()) {
    auto [t, s] = st.back();
    st.pop_back();
    const TreeNode &a = T.nodes[t], &b = T.nodes[s];
    if (admissible(a, b, eta)) {
      if (t < s) far.push_back({t, s});
      continue;
    }
    const bool la = a.n_child == 0, lb = b.n_child == 0;
    if (la && lb) {
      if (a.leaf <= b.leaf) near.push_back({a.leaf, b.leaf});
      continue;
    }
    auto split_a = [&]() {
      for (int c = 0; c < a.n_child; ++c) st.push_back({T.child[a.first_child + c], s});
    };
    auto split_b = [&]() {
      for (int c = 0; c < b.n_child; ++c) st.push_back({t, T.child[b.first_child + c]});
    };
    if (la) split_b();
    else if (lb) split_a();
    else if (a.depth < b.depth) split_a();
    else if (b.depth < a.depth) split_b();
    else {
      for (int c = 0; c < a.n_child; ++c)
        for (int e = 0; e < b.n_child; ++e)
          st.push_back({T.child[a.first_child + c], T.child[b.first_child + e]});
    }
  }
  std::sort(near.begin(), near.end());
  std::sort(far.begin(), far.end());
}

}  // namespace hps
