// Host side of the paper's guide (Sec. 5.6): the binary tree over the 6-D
// configuration (x_D, x_L) and the per-leaf tables, built from the sample
// records in breadth-first order.  The per-lobe footprints (the quadratic
// nearest-direction search) and all sampling run on the GPU.
//
// Split rule: a node holding more than c sqrt(|S|) samples (and above the
// depth limit) is halved across its longest side (lowest axis on ties).
// Overlap: each child keeps the parent's samples that fall inside the child
// box widened by eps times the child's extent along the split axis; a sample
// is the node's own when it lies inside the unwidened box.  Leaf tables:
// total weight, weight per length, and the lobes grouped by (length, type)
// in increasing order, samples in increasing index order inside a group.
#include "mpg_stree_host.h"

#include <algorithm>
#include <cmath>

namespace mpg_host {

namespace {

struct Work {
  double lo[6], hi[6];
  int depth;
  std::vector<int> ids;
  std::vector<char> own;
};

bool record_ok(const float* r, const double* lo, const double* hi) {
  for (int a = 0; a < 12; ++a)
    if (!std::isfinite(r[a])) return false;
  if (!(r[9] > 0.0f)) return false;
  int n = (int)r[10];
  if (n < 1 || n > 8 || (float)n != r[10]) return false;
  for (int a = 0; a < 6; ++a)
    if (!((double)r[a] >= lo[a] && (double)r[a] <= hi[a])) return false;
  return true;
}

}  // namespace

int build_stree(const float* rec, int n_rec, const StreeParams& prm, StreeHost* out) {
  out->axis.clear(); out->mid.clear(); out->child.clear(); out->depth.clear();
  out->leaf_W.clear(); out->leaf_Wn.clear(); out->leaf_own.clear(); out->leaf_groups.clear();
  out->grp_key.clear(); out->grp_w.clear(); out->grp_lobes.clear();
  out->lobe_dir.clear(); out->lobe_cdf.clear(); out->lobe_sample.clear();
  std::vector<Work> nodes(1);
  Work& root = nodes[0];
  for (int a = 0; a < 6; ++a) { root.lo[a] = prm.lo[a]; root.hi[a] = prm.hi[a]; }
  root.depth = 0;
  for (int j = 0; j < n_rec; ++j)
    if (record_ok(rec + 16 * (size_t)j, prm.lo, prm.hi)) { root.ids.push_back(j); root.own.push_back(1); }
  const double limit = prm.thr_scale * std::sqrt((double)root.ids.size());
  // breadth-first splitting; a node's index is its position in `nodes`
  std::vector<int> axis(1, -1), child(1, -1);
  std::vector<double> mid(1, 0.0);
  for (size_t k = 0; k < nodes.size(); ++k) {
    if (!((double)nodes[k].ids.size() > limit) || nodes[k].depth >= prm.max_depth) continue;
    int ax = 0;
    for (int a = 1; a < 6; ++a)
      if (nodes[k].hi[a] - nodes[k].lo[a] > nodes[k].hi[ax] - nodes[k].lo[ax]) ax = a;
    const double m = 0.5 * (nodes[k].lo[ax] + nodes[k].hi[ax]);
    const double widen = prm.eps * (m - nodes[k].lo[ax]);
    Work left, right;
    for (int a = 0; a < 6; ++a) {
      left.lo[a] = right.lo[a] = nodes[k].lo[a];
      left.hi[a] = right.hi[a] = nodes[k].hi[a];
    }
    left.hi[ax] = m;
    right.lo[ax] = m;
    left.depth = right.depth = nodes[k].depth + 1;
    const double lo_edge = nodes[k].lo[ax], hi_edge = nodes[k].hi[ax];
    for (size_t e = 0; e < nodes[k].ids.size(); ++e) {
      const int j = nodes[k].ids[e];
      const double v = (double)rec[16 * (size_t)j + ax];
      const bool mine = nodes[k].own[e] != 0;
      if (v >= lo_edge - widen && v < m + widen) { left.ids.push_back(j); left.own.push_back(mine && v < m); }
      if (v >= m - widen && v < hi_edge + widen) { right.ids.push_back(j); right.own.push_back(mine && v >= m); }
    }
    axis[k] = ax;
    mid[k] = m;
    child[k] = (int)nodes.size();
    nodes[k].ids.clear();
    nodes[k].ids.shrink_to_fit();
    nodes[k].own.clear();
    nodes.push_back(std::move(left));
    nodes.push_back(std::move(right));
    axis.push_back(-1); axis.push_back(-1);
    child.push_back(-1); child.push_back(-1);
    mid.push_back(0.0); mid.push_back(0.0);
  }
  const int nn = (int)nodes.size();
  out->axis = axis;
  out->child = child;
  out->mid.resize(nn);
  out->depth.resize(nn);
  out->leaf_W.assign(nn, 0.0f);
  out->leaf_Wn.assign((size_t)nn * 8, 0.0f);
  out->leaf_own.assign(nn, 0);
  out->leaf_groups.assign(nn, std::pair<int, int>(0, 0));
  for (int k = 0; k < nn; ++k) {
    out->mid[k] = (float)mid[k];
    out->depth[k] = nodes[k].depth;
    if (axis[k] >= 0) continue;
    const Work& lf = nodes[k];
    double W = 0.0, Wn[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int own = 0;
    // (n, type, sample) order
    std::vector<std::pair<long long, int>> key(lf.ids.size());
    for (size_t e = 0; e < lf.ids.size(); ++e) {
      const float* r = rec + 16 * (size_t)lf.ids[e];
      const int n = (int)r[10], ty = (int)r[11] & 0xff;
      W += r[9];
      Wn[n - 1] += r[9];
      own += lf.own[e] ? 1 : 0;
      key[e] = {((long long)n << 40) | ((long long)ty << 32) | (long long)lf.ids[e], lf.ids[e]};
    }
    std::sort(key.begin(), key.end());
    out->leaf_W[k] = (float)W;
    for (int q = 0; q < 8; ++q) out->leaf_Wn[(size_t)k * 8 + q] = (float)Wn[q];
    out->leaf_own[k] = own;
    const int g0 = (int)out->grp_key.size();
    for (size_t i = 0; i < key.size();) {
      size_t e = i;
      const long long gk = key[i].first >> 32;
      while (e < key.size() && (key[e].first >> 32) == gk) ++e;
      const int first = (int)out->lobe_sample.size();
      double acc = 0.0;
      for (size_t a = i; a < e; ++a) {
        const float* r = rec + 16 * (size_t)key[a].second;
        double dx = r[6], dy = r[7], dz = r[8];
        double l = std::sqrt(dx * dx + dy * dy + dz * dz);
        out->lobe_dir.push_back((float)(dx / l));
        out->lobe_dir.push_back((float)(dy / l));
        out->lobe_dir.push_back((float)(dz / l));
        acc += r[9];
        out->lobe_cdf.push_back((float)acc);
        out->lobe_sample.push_back(key[a].second);
      }
      out->grp_key.push_back((int)((gk >> 8) & 0xff) | (int)((gk & 0xff) << 8));
      out->grp_w.push_back((float)acc);
      out->grp_lobes.push_back(std::pair<int, int>(first, (int)(e - i)));
      i = e;
    }
    out->leaf_groups[k] = std::pair<int, int>(g0, (int)out->grp_key.size() - g0);
  }
  return nn;
}

}  // namespace mpg_host
