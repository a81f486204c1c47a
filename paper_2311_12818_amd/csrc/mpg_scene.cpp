// Host-side scene preparation: binned-SAH binary BVH collapsed into 4-wide
// 128-byte nodes (child boxes in structure-of-arrays order),
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
  // collapse the binary tree into 4-wide nodes: starting from a node's two
  // children, the interior child with the largest box is replaced by its own
  // two children until there are four or only leaves remain
  struct Wide {
    int child[4];  // tree indices, -1 = empty
    int level;
  };
  std::vector<Wide> wide;
  std::vector<int> stack_tree, stack_level, stack_slot;
  auto open_children = [&](int ti, int* out) {
    int list[4];
    int n = 0;
    if (tree[ti].left < 0) {
      list[n++] = ti;  // a leaf root: one leaf child
    } else {
      list[n++] = tree[ti].left;
      list[n++] = tree[ti].right;
      while (n < 4) {
        int best = -1;
        float area = -1.0f;
        for (int k = 0; k < n; ++k)
          if (tree[list[k]].left >= 0 && tree[list[k]].box.area() > area) { area = tree[list[k]].box.area(); best = k; }
        if (best < 0) break;
        int t = list[best];
        list[best] = tree[t].left;
        for (int k = n; k > best + 1; --k) list[k] = list[k - 1];
        list[best + 1] = tree[t].right;
        ++n;
      }
    }
    for (int k = 0; k < 4; ++k) out[k] = k < n ? list[k] : -1;
  };
  // depth-first emission, parents before children; pending (tree node, parent slot) pairs
  struct Pending {
    int tree, parent, slot, level;
  };
  std::vector<Pending> todo;
  todo.push_back({0, -1, -1, 1});
  std::vector<int32_t> child_ref;  // 4 per wide node, filled as children are emitted
  int levels = 1;
  while (!todo.empty()) {
    Pending pd = todo.back();
    todo.pop_back();
    int w = (int)wide.size();
    Wide nd;
    open_children(pd.tree, nd.child);
    nd.level = pd.level;
    levels = std::max(levels, pd.level);
    wide.push_back(nd);
    child_ref.resize((size_t)(w + 1) * 4, (int32_t)0x80000000u);
    if (pd.parent >= 0) child_ref[(size_t)pd.parent * 4 + pd.slot] = w;
    for (int k = 3; k >= 0; --k) {
      int c = nd.child[k];
      if (c < 0) continue;
      if (tree[c].left >= 0)
        todo.push_back({c, w, k, pd.level + 1});
      else
        child_ref[(size_t)w * 4 + k] =
            (int32_t)(0x80000000u | ((uint32_t)tree[c].count << 24) | (uint32_t)tree[c].start);
    }
  }
  const int n_wide = (int)wide.size();
  gpu_nodes.assign((size_t)n_wide * 32, 0.0f);
  ranges.assign((size_t)n_wide * 8, 0);
  for (int w = 0; w < n_wide; ++w) {
    float* f = &gpu_nodes[(size_t)w * 32];
    for (int k = 0; k < 4; ++k) {
      int c = wide[w].child[k];
      float lo[3], hi[3];
      if (c < 0) {
        for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = INFINITY; }  // never hit
      } else {
        for (int a = 0; a < 3; ++a) { lo[a] = tree[c].box.lo[a] - pad; hi[a] = tree[c].box.hi[a] + pad; }
        ranges[(size_t)w * 8 + 2 * k] = tree[c].start;
        ranges[(size_t)w * 8 + 2 * k + 1] = tree[c].count;
      }
      for (int a = 0; a < 3; ++a) {
        f[4 * a + k] = lo[a];
        f[12 + 4 * a + k] = hi[a];
      }
      int32_t ref = child_ref[(size_t)w * 4 + k];
      std::memcpy(&f[24 + k], &ref, 4);
    }
  }
  // near-first traversal pushes at most three children per level
  *max_depth = 3 * levels;
  return n_wide;
}

}  // namespace mpg_host
