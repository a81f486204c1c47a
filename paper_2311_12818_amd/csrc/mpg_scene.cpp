// Host-side scene preparation: binned-SAH BVH with two-child 64-byte nodes,
// per-object area prefix sums for p_0, object xy bounds.
#include "mpg_scene.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>

namespace mpg_host {

namespace {

struct Box {
  float lo[3], hi[3];
  Box() {
    for (int a = 0; a < 3; ++a) { lo[a] = FLT_MAX; hi[a] = -FLT_MAX; }
  }
  void grow(const float* p) {
    for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], p[a]); hi[a] = std::max(hi[a], p[a]); }
  }
  void grow(const Box& b) {
    for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], b.lo[a]); hi[a] = std::max(hi[a], b.hi[a]); }
  }
  bool empty() const { return lo[0] > hi[0]; }
  float area() const {
    if (empty()) return 0.0f;
    float dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    return 2.0f * (dx * dy + dy * dz + dz * dx);
  }
};

struct TreeNode {
  Box box;
  int left = -1, right = -1;  // tree indices; -1 for leaves
  int start = 0, count = 0;   // leaf range in the reordered triangle list
  int depth = 1;
};

constexpr int kLeafMax = 4;
constexpr int kBins = 16;

}  // namespace

int build_bvh(const float* verts, const int32_t* tris, int n_tris, float pad, std::vector<float>& gpu_nodes,
              std::vector<int32_t>& order, std::vector<int32_t>& ranges, int* max_depth) {
  std::vector<Box> tb(n_tris);
  std::vector<float> cen(3 * (size_t)n_tris);
  for (int t = 0; t < n_tris; ++t) {
    for (int k = 0; k < 3; ++k) tb[t].grow(verts + 3 * (size_t)tris[3 * t + k]);
    for (int a = 0; a < 3; ++a) cen[3 * (size_t)t + a] = 0.5f * (tb[t].lo[a] + tb[t].hi[a]);
  }
  order.resize(n_tris);
  for (int t = 0; t < n_tris; ++t) order[t] = t;
  std::vector<TreeNode> tree;
  tree.reserve(2 * (size_t)n_tris / kLeafMax + 4);
  struct Job { int node, start, count; };
  std::vector<Job> jobs;
  tree.push_back(TreeNode());
  jobs.push_back({0, 0, n_tris});
  while (!jobs.empty()) {
    Job j = jobs.back();
    jobs.pop_back();
    TreeNode nd;
    nd.depth = tree[j.node].depth;
    Box cb;
    for (int i = j.start; i < j.start + j.count; ++i) {
      nd.box.grow(tb[order[i]]);
      cb.grow(&cen[3 * (size_t)order[i]]);
    }
    nd.start = j.start;
    nd.count = j.count;
    if (j.count <= kLeafMax) {
      tree[j.node] = nd;
      continue;
    }
    // binned SAH over the centroid bounds
    int best_axis = -1, best_split = -1;
    float best_cost = FLT_MAX;
    for (int a = 0; a < 3; ++a) {
      float ext = cb.hi[a] - cb.lo[a];
      if (!(ext > 0.0f)) continue;
      Box bb[kBins];
      int bc[kBins] = {0};
      for (int i = j.start; i < j.start + j.count; ++i) {
        int t = order[i];
        int b = std::min(kBins - 1, (int)((cen[3 * (size_t)t + a] - cb.lo[a]) / ext * kBins));
        bb[b].grow(tb[t]);
        bc[b]++;
      }
      Box lb[kBins], rb[kBins];
      int lc[kBins], rc[kBins];
      Box acc;
      int cnt = 0;
      for (int b = 0; b < kBins; ++b) { acc.grow(bb[b]); cnt += bc[b]; lb[b] = acc; lc[b] = cnt; }
      acc = Box();
      cnt = 0;
      for (int b = kBins - 1; b >= 0; --b) { acc.grow(bb[b]); cnt += bc[b]; rb[b] = acc; rc[b] = cnt; }
      for (int s = 0; s < kBins - 1; ++s) {
        if (lc[s] == 0 || rc[s + 1] == 0) continue;
        float cost = lc[s] * lb[s].area() + rc[s + 1] * rb[s + 1].area();
        if (cost < best_cost) { best_cost = cost; best_axis = a; best_split = s; }
      }
    }
    int mid;
    if (best_axis < 0) {
      mid = j.start + j.count / 2;  // coincident centroids: split by count
    } else {
      float ext = cb.hi[best_axis] - cb.lo[best_axis];
      auto it = std::partition(order.begin() + j.start, order.begin() + j.start + j.count, [&](int t) {
        int b = std::min(kBins - 1, (int)((cen[3 * (size_t)t + best_axis] - cb.lo[best_axis]) / ext * kBins));
        return b <= best_split;
      });
      mid = (int)(it - order.begin());
      if (mid == j.start || mid == j.start + j.count) mid = j.start + j.count / 2;
    }
    int l = (int)tree.size();
    tree.push_back(TreeNode());
    tree.push_back(TreeNode());
    tree[l].depth = tree[l + 1].depth = nd.depth + 1;
    nd.left = l;
    nd.right = l + 1;
    tree[j.node] = nd;
    jobs.push_back({l, j.start, mid - j.start});
    jobs.push_back({l + 1, mid, j.start + j.count - mid});
  }
  // emit GPU nodes: interior nodes only, each holding both child boxes
  std::vector<int> gidx(tree.size(), -1);
  int n_int = 0;
  int depth = 1;
  bool root_leaf = tree[0].left < 0;
  if (root_leaf) {
    n_int = 1;
  } else {
    for (size_t i = 0; i < tree.size(); ++i)
      if (tree[i].left >= 0) { gidx[i] = n_int++; depth = std::max(depth, tree[i].depth); }
  }
  gpu_nodes.assign((size_t)n_int * 16, 0.0f);
  ranges.assign((size_t)n_int * 4, 0);
  auto ref_of = [&](int ti) -> int32_t {
    const TreeNode& t = tree[ti];
    if (t.left >= 0) return gidx[ti];
    return (int32_t)(0x80000000u | ((uint32_t)t.count << 24) | (uint32_t)t.start);
  };
  auto put = [&](int g, const Box& L, const Box& R, int32_t lref, int32_t rref) {
    float* f = &gpu_nodes[(size_t)g * 16];
    Box l = L, r = R;
    for (int a = 0; a < 3; ++a) {
      if (!l.empty()) { l.lo[a] -= pad; l.hi[a] += pad; }
      if (!r.empty()) { r.lo[a] -= pad; r.hi[a] += pad; }
    }
    f[0] = l.lo[0]; f[1] = l.lo[1]; f[2] = l.lo[2]; f[3] = l.hi[0];
    f[4] = l.hi[1]; f[5] = l.hi[2]; f[6] = r.lo[0]; f[7] = r.lo[1];
    f[8] = r.lo[2]; f[9] = r.hi[0]; f[10] = r.hi[1]; f[11] = r.hi[2];
    std::memcpy(&f[12], &lref, 4);
    std::memcpy(&f[13], &rref, 4);
    int32_t z = 0;
    std::memcpy(&f[14], &z, 4);
    std::memcpy(&f[15], &z, 4);
  };
  if (root_leaf) {
    Box empty;
    int32_t lref = (int32_t)(0x80000000u | ((uint32_t)tree[0].count << 24) | (uint32_t)tree[0].start);
    int32_t rref = (int32_t)0x80000000u;  // empty leaf
    put(0, tree[0].box, empty, lref, rref);
    ranges[0] = tree[0].start;
    ranges[1] = tree[0].count;
  } else {
    for (size_t i = 0; i < tree.size(); ++i) {
      if (tree[i].left < 0) continue;
      put(gidx[i], tree[tree[i].left].box, tree[tree[i].right].box, ref_of(tree[i].left), ref_of(tree[i].right));
      int32_t* r = &ranges[(size_t)gidx[i] * 4];
      r[0] = tree[tree[i].left].start;
      r[1] = tree[tree[i].left].count;
      r[2] = tree[tree[i].right].start;
      r[3] = tree[tree[i].right].count;
    }
  }
  *max_depth = depth;
  return n_int;
}

}  // namespace mpg_host
