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
#include <atomic>
#include <cmath>
#include <thread>

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

// f(i) for i in [0, n) on up to `threads` threads (work items taken in
// order from a shared counter; every item writes only its own outputs, so
// the result does not depend on the schedule)
template <class F>
void parallel_for(int n, int threads, F f) {
  threads = std::max(1, std::min(threads, n));
  if (threads == 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next(0);
  auto worker = [&]() {
    for (int i; (i = next.fetch_add(1)) < n;) f(i);
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < threads; ++t) pool.emplace_back(worker);
  worker();
  for (std::thread& th : pool) th.join();
}

int host_threads() {
  const unsigned h = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(h, 16u));
}

// one leaf's tables, before they are placed in the shared arrays
struct LeafOut {
  double W = 0.0, Wn[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int own = 0;
  std::vector<int> grp_key, grp_count;
  std::vector<float> grp_w, dir, cdf;
  std::vector<int> sample;
};

void leaf_tables(const float* rec, const Work& lf, LeafOut* o) {
  // (n, type, sample) order
  std::vector<std::pair<long long, int>> key(lf.ids.size());
  for (size_t e = 0; e < lf.ids.size(); ++e) {
    const float* r = rec + 16 * (size_t)lf.ids[e];
    const int n = (int)r[10], ty = (int)r[11] & 0xff;
    o->W += r[9];
    o->Wn[n - 1] += r[9];
    o->own += lf.own[e] ? 1 : 0;
    key[e] = {((long long)n << 40) | ((long long)ty << 32) | (long long)lf.ids[e], lf.ids[e]};
  }
  std::sort(key.begin(), key.end());
  o->dir.reserve(3 * key.size());
  o->cdf.reserve(key.size());
  o->sample.reserve(key.size());
  for (size_t i = 0; i < key.size();) {
    size_t e = i;
    const long long gk = key[i].first >> 32;
    while (e < key.size() && (key[e].first >> 32) == gk) ++e;
    double acc = 0.0;
    for (size_t a = i; a < e; ++a) {
      const float* r = rec + 16 * (size_t)key[a].second;
      double dx = r[6], dy = r[7], dz = r[8];
      double l = std::sqrt(dx * dx + dy * dy + dz * dz);
      o->dir.push_back((float)(dx / l));
      o->dir.push_back((float)(dy / l));
      o->dir.push_back((float)(dz / l));
      acc += r[9];
      o->cdf.push_back((float)acc);
      o->sample.push_back(key[a].second);
    }
    o->grp_key.push_back((int)((gk >> 8) & 0xff) | (int)((gk & 0xff) << 8));
    o->grp_w.push_back((float)acc);
    o->grp_count.push_back((int)(e - i));
    i = e;
  }
}

}  // namespace

int build_stree(const float* rec, int n_rec, const StreeParams& prm, StreeHost* out) {
  out->axis.clear(); out->mid.clear(); out->child.clear(); out->depth.clear();
  out->leaf_W.clear(); out->leaf_Wn.clear(); out->leaf_own.clear(); out->leaf_groups.clear();
  out->grp_key.clear(); out->grp_w.clear(); out->grp_lobes.clear();
  out->lobe_dir.clear(); out->lobe_cdf.clear(); out->lobe_sample.clear();
  const int threads = host_threads();
  std::vector<Work> nodes(1);
  Work& root = nodes[0];
  for (int a = 0; a < 6; ++a) { root.lo[a] = prm.lo[a]; root.hi[a] = prm.hi[a]; }
  root.depth = 0;
  for (int j = 0; j < n_rec; ++j)
    if (record_ok(rec + 16 * (size_t)j, prm.lo, prm.hi)) { root.ids.push_back(j); root.own.push_back(1); }
  const double limit = prm.thr_scale * std::sqrt((double)root.ids.size());
  // Breadth-first splitting, one level at a time: the children of the i-th
  // node split on a level are nodes end + 2i and end + 2i + 1 (end = first
  // index after the level), the order a one-node-at-a-time breadth-first
  // pass gives.  A node's entries are classified in chunks in parallel and
  // the chunks concatenated in order, so each child lists its samples in the
  // parent's order.
  std::vector<int> axis(1, -1), child(1, -1);
  std::vector<double> mid(1, 0.0);
  const size_t chunk = 1 << 15;
  for (size_t a = 0, b = 1; a < b; a = b, b = nodes.size()) {
    std::vector<int> split;
    for (size_t k = a; k < b; ++k)
      if ((double)nodes[k].ids.size() > limit && nodes[k].depth < prm.max_depth) split.push_back((int)k);
    if (split.empty()) break;
    struct Task { int s; size_t e0, e1; std::vector<int> lid, rid; std::vector<char> lown, rown; };
    std::vector<Task> tasks;
    std::vector<int> ax(split.size());
    std::vector<double> m(split.size()), widen(split.size());
    for (size_t i = 0; i < split.size(); ++i) {
      const Work& w = nodes[split[i]];
      int x = 0;
      for (int q = 1; q < 6; ++q)
        if (w.hi[q] - w.lo[q] > w.hi[x] - w.lo[x]) x = q;
      ax[i] = x;
      m[i] = 0.5 * (w.lo[x] + w.hi[x]);
      widen[i] = prm.eps * (m[i] - w.lo[x]);
      for (size_t e0 = 0; e0 < w.ids.size(); e0 += chunk)
        tasks.push_back(Task{(int)i, e0, std::min(w.ids.size(), e0 + chunk), {}, {}, {}, {}});
    }
    parallel_for((int)tasks.size(), threads, [&](int t) {
      Task& T = tasks[t];
      const Work& w = nodes[split[T.s]];
      const int x = ax[T.s];
      const double mm = m[T.s], wd = widen[T.s], lo_edge = w.lo[x], hi_edge = w.hi[x];
      T.lid.reserve(T.e1 - T.e0);
      T.lown.reserve(T.e1 - T.e0);
      T.rid.reserve(T.e1 - T.e0);
      T.rown.reserve(T.e1 - T.e0);
      for (size_t e = T.e0; e < T.e1; ++e) {
        const int j = w.ids[e];
        const double v = (double)rec[16 * (size_t)j + x];
        const bool mine = w.own[e] != 0;
        if (v >= lo_edge - wd && v < mm + wd) { T.lid.push_back(j); T.lown.push_back(mine && v < mm); }
        if (v >= mm - wd && v < hi_edge + wd) { T.rid.push_back(j); T.rown.push_back(mine && v >= mm); }
      }
    });
    nodes.resize(b + 2 * split.size());
    axis.resize(nodes.size(), -1);
    child.resize(nodes.size(), -1);
    mid.resize(nodes.size(), 0.0);
    // task ranges per split node (tasks are in split order)
    std::vector<size_t> t0(split.size() + 1, 0);
    for (const Task& T : tasks) ++t0[T.s + 1];
    for (size_t i = 0; i < split.size(); ++i) t0[i + 1] += t0[i];
    parallel_for((int)split.size(), threads, [&](int i) {
      Work& w = nodes[split[i]];
      Work& left = nodes[b + 2 * i];
      Work& right = nodes[b + 2 * i + 1];
      for (int q = 0; q < 6; ++q) {
        left.lo[q] = right.lo[q] = w.lo[q];
        left.hi[q] = right.hi[q] = w.hi[q];
      }
      left.hi[ax[i]] = m[i];
      right.lo[ax[i]] = m[i];
      left.depth = right.depth = w.depth + 1;
      for (size_t t = t0[i]; t < t0[i + 1]; ++t) {
        Task& T = tasks[t];
        left.ids.insert(left.ids.end(), T.lid.begin(), T.lid.end());
        left.own.insert(left.own.end(), T.lown.begin(), T.lown.end());
        right.ids.insert(right.ids.end(), T.rid.begin(), T.rid.end());
        right.own.insert(right.own.end(), T.rown.begin(), T.rown.end());
      }
      axis[split[i]] = ax[i];
      mid[split[i]] = m[i];
      child[split[i]] = (int)(b + 2 * i);
      std::vector<int>().swap(w.ids);
      std::vector<char>().swap(w.own);
    });
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
  std::vector<LeafOut> lo(nn);
  parallel_for(nn, threads, [&](int k) {
    if (axis[k] < 0) leaf_tables(rec, nodes[k], &lo[k]);
  });
  // place every leaf's groups and lobes in node order
  std::vector<size_t> g_off(nn + 1, 0), l_off(nn + 1, 0);
  for (int k = 0; k < nn; ++k) {
    g_off[k + 1] = g_off[k] + lo[k].grp_key.size();
    l_off[k + 1] = l_off[k] + lo[k].sample.size();
  }
  out->grp_key.resize(g_off[nn]);
  out->grp_w.resize(g_off[nn]);
  out->grp_lobes.resize(g_off[nn]);
  out->lobe_dir.resize(3 * l_off[nn]);
  out->lobe_cdf.resize(l_off[nn]);
  out->lobe_sample.resize(l_off[nn]);
  parallel_for(nn, threads, [&](int k) {
    out->mid[k] = (float)mid[k];
    out->depth[k] = nodes[k].depth;
    if (axis[k] >= 0) return;
    const LeafOut& L = lo[k];
    out->leaf_W[k] = (float)L.W;
    for (int q = 0; q < 8; ++q) out->leaf_Wn[(size_t)k * 8 + q] = (float)L.Wn[q];
    out->leaf_own[k] = L.own;
    out->leaf_groups[k] = std::pair<int, int>((int)g_off[k], (int)L.grp_key.size());
    size_t first = l_off[k];
    for (size_t g = 0; g < L.grp_key.size(); ++g) {
      out->grp_key[g_off[k] + g] = L.grp_key[g];
      out->grp_w[g_off[k] + g] = L.grp_w[g];
      out->grp_lobes[g_off[k] + g] = std::pair<int, int>((int)first, L.grp_count[g]);
      first += L.grp_count[g];
    }
    std::copy(L.dir.begin(), L.dir.end(), out->lobe_dir.begin() + 3 * l_off[k]);
    std::copy(L.cdf.begin(), L.cdf.end(), out->lobe_cdf.begin() + l_off[k]);
    std::copy(L.sample.begin(), L.sample.end(), out->lobe_sample.begin() + l_off[k]);
  });
  return nn;
}

}  // namespace mpg_host
