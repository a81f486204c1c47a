// The paper's guide tree (Sec. 5.6) built on the GPU from the sample records,
// level by level.
//
// Split rule: a node holding more than c sqrt(|S|) samples (and above the
// depth limit) is halved across its longest side (lowest axis on ties).
// Overlap: each child keeps the parent's samples that fall inside the child
// box widened by eps times the child's extent along the split axis; a sample
// is the node's own when it lies inside the unwidened box.  Leaf tables:
// total weight, weight per length, and the lobes grouped by (length, type)
// in increasing order, samples in increasing index order inside a group.
//
// The entries (sample index, own flag) of one level lie node after node in
// one buffer.  Per level: a classification kernel marks each entry for the
// left child, the right child or (node not split) the leaf buffer; exclusive
// scans of the three marks give every entry its place; the per-node counts
// come back to the host, which lays out the next level; a scatter kernel
// writes the children's entries in the parent's order and appends the
// leaves' entries to the leaf buffer.  The split decisions, planes and
// widened bounds are computed on the host in FP64 and the kernels only
// compare FP64 values with them, so the tree is the one a sequential FP64
// pass builds.  Leaf and group sums run sequentially per leaf / group in
// FP64 in entry order, as such a pass would.
#include "mpg_stree_build.h"

#include <hipcub/hipcub.hpp>

namespace {

struct RootBox {
  double lo[6], hi[6];
};

__device__ __forceinline__ bool record_ok(const float* r, const RootBox& B) {
  for (int a = 0; a < 12; ++a)
    if (!isfinite(r[a])) return false;
  if (!(r[9] > 0.0f)) return false;
  const int n = (int)r[10];
  if (n < 1 || n > 8 || (float)n != r[10]) return false;
  for (int a = 0; a < 6; ++a)
    if (!((double)r[a] >= B.lo[a] && (double)r[a] <= B.hi[a])) return false;
  return true;
}

__global__ void k_sb_valid(const float* rec, int n, RootBox B, int* flag) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) flag[j] = record_ok(rec + 16 * (size_t)j, B) ? 1 : 0;
  if (j == n) flag[j] = 0;
}

__global__ void k_sb_compact(const int* flag, const int* pos, int n, int* ids, uint8_t* own) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n && flag[j]) {
    ids[pos[j]] = j;
    own[pos[j]] = 1;
  }
}

// per node of a level: first entry, split axis (-1: leaf), the widened
// intervals of the two children and the plane
struct LevelNode {
  long long e0;
  int axis;
  double lo_l, hi_l, lo_r, hi_r, mid;
};

__device__ __forceinline__ int node_of(const LevelNode* nodes, int n_nodes, long long e) {
  int lo = 0, hi = n_nodes - 1;  // last node whose first entry is <= e
  while (lo < hi) {
    const int m = (lo + hi + 1) >> 1;
    if (nodes[m].e0 <= e) lo = m;
    else hi = m - 1;
  }
  return lo;
}

// marks: left child, right child, leaf buffer (index E holds 0 so that the
// exclusive scans end with the totals)
__global__ void k_sb_classify(const float* rec, const int* ids, long long E, const LevelNode* nodes, int n_nodes,
                              int* ml, int* mr, int* mf) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e > E) return;
  if (e == E) {
    ml[e] = mr[e] = mf[e] = 0;
    return;
  }
  const LevelNode& nd = nodes[node_of(nodes, n_nodes, e)];
  if (nd.axis < 0) {
    ml[e] = mr[e] = 0;
    mf[e] = 1;
    return;
  }
  const double v = (double)rec[16 * (size_t)ids[e] + nd.axis];
  ml[e] = v >= nd.lo_l && v < nd.hi_l ? 1 : 0;
  mr[e] = v >= nd.lo_r && v < nd.hi_r ? 1 : 0;
  mf[e] = 0;
}

// scan values at every node's first entry and at E
__global__ void k_sb_bounds(const LevelNode* nodes, int n_nodes, long long E, const int* sl, const int* sr,
                            const int* sf, int* bl, int* br, int* bf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n_nodes) return;
  const long long e = i == n_nodes ? E : nodes[i].e0;
  bl[i] = sl[e];
  br[i] = sr[e];
  bf[i] = sf[e];
}

// next-level place of a node's left / right child entries, and the leaf
// buffer offset of its leaf entries
struct LevelOut {
  long long left, right, leaf;
};

__global__ void k_sb_scatter(const float* rec, const int* ids, const uint8_t* own, long long E,
                             const LevelNode* nodes, int n_nodes, const LevelOut* out, const int* bl, const int* br,
                             const int* bf, const int* sl, const int* sr, const int* sf, int* next_ids,
                             uint8_t* next_own, int* leaf_ids, uint8_t* leaf_own) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int i = node_of(nodes, n_nodes, e);
  const LevelNode& nd = nodes[i];
  const int j = ids[e];
  const bool mine = own[e] != 0;
  if (nd.axis < 0) {
    const long long p = out[i].leaf + (sf[e] - bf[i]);
    leaf_ids[p] = j;
    leaf_own[p] = mine ? 1 : 0;
    return;
  }
  const double v = (double)rec[16 * (size_t)j + nd.axis];
  if (v >= nd.lo_l && v < nd.hi_l) {
    const long long p = out[i].left + (sl[e] - bl[i]);
    next_ids[p] = j;
    next_own[p] = mine && v < nd.mid ? 1 : 0;
  }
  if (v >= nd.lo_r && v < nd.hi_r) {
    const long long p = out[i].right + (sr[e] - br[i]);
    next_ids[p] = j;
    next_own[p] = mine && v >= nd.mid ? 1 : 0;
  }
}

__global__ void k_sb_zero(float* W, float* Wn, int* own, int2* lg, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  W[k] = 0.0f;
  for (int q = 0; q < 8; ++q) Wn[(size_t)k * 8 + q] = 0.0f;
  own[k] = 0;
  lg[k] = make_int2(0, 0);
}

// one thread per leaf: W, W_n and own count, summed in entry order in FP64
__global__ void k_sb_leaf_sums(const float* rec, const int* leaf_node, const long long* leaf_off, int n_leaves,
                               const int* leaf_ids, const uint8_t* leaf_own, float* W, float* Wn, int* own) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_leaves) return;
  double w = 0.0, wn[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int o = 0;
  for (long long p = leaf_off[l]; p < leaf_off[l + 1]; ++p) {
    const float* r = rec + 16 * (size_t)leaf_ids[p];
    const int n = (int)r[10];
    w += r[9];
    wn[n - 1] += r[9];
    o += leaf_own[p];
  }
  const int k = leaf_node[l];
  W[k] = (float)w;
  for (int q = 0; q < 8; ++q) Wn[(size_t)k * 8 + q] = (float)wn[q];
  own[k] = o;
}

// sort key of a leaf entry: (leaf rank, n, tau)
__global__ void k_sb_keys(const float* rec, const long long* leaf_off, int n_leaves, const int* leaf_ids,
                          long long total, unsigned long long* keys) {
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= total) return;
  int lo = 0, hi = n_leaves - 1;  // last leaf whose first entry is <= p
  while (lo < hi) {
    const int m = (lo + hi + 1) >> 1;
    if (leaf_off[m] <= p) lo = m;
    else hi = m - 1;
  }
  const float* r = rec + 16 * (size_t)leaf_ids[p];
  const unsigned long long n = (unsigned)(int)r[10], ty = (unsigned)((int)r[11] & 0xff);
  keys[p] = ((unsigned long long)lo << 16) | (n << 8) | ty;
}

// group starts (index total holds 0: the scan ends with the group count)
__global__ void k_sb_group_marks(const unsigned long long* keys, long long total, int* mark) {
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p > total) return;
  mark[p] = p < total && (p == 0 || keys[p] != keys[p - 1]) ? 1 : 0;
}

__global__ void k_sb_group_starts(const int* mark, const int* gidx, long long total, long long* gstart) {
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p > total) return;
  if (p == total) gstart[gidx[p]] = total;
  else if (mark[p]) gstart[gidx[p]] = p;
}

// one thread per group: key, lobes (unit directions in FP64) and the
// inclusive prefix of their weights in FP64, in lobe order
__global__ void k_sb_groups(const float* rec, const unsigned long long* keys, const int* sorted_ids,
                            const long long* gstart, int n_groups, int* grp_key, float* grp_w, int2* grp_lobes,
                            float4* lobe, float* lobe_cdf) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  const long long a = gstart[g], b = gstart[g + 1];
  const unsigned long long key = keys[a];
  const int n = (int)((key >> 8) & 0xff), ty = (int)(key & 0xff);
  double acc = 0.0;
  for (long long p = a; p < b; ++p) {
    const float* r = rec + 16 * (size_t)sorted_ids[p];
    const double dx = r[6], dy = r[7], dz = r[8];
    // products and sums rounded one by one (no contraction), as on the host
    const double l = sqrt(__dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz)));
    lobe[p] = make_float4((float)(dx / l), (float)(dy / l), (float)(dz / l), 0.0f);
    acc += r[9];
    lobe_cdf[p] = (float)acc;
  }
  grp_key[g] = n | (ty << 8);
  grp_w[g] = (float)acc;
  grp_lobes[g] = make_int2((int)a, (int)(b - a));
}

__global__ void k_sb_leaf_groups(const int* leaf_node, const long long* leaf_off, int n_leaves, const int* gidx,
                                 int2* lg) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_leaves) return;
  const int g0 = gidx[leaf_off[l]], g1 = gidx[leaf_off[l + 1]];
  lg[leaf_node[l]] = make_int2(g0, g1 - g0);
}

// device scratch released when the build returns
struct Scratch {
  std::vector<void*> p;
  template <class T>
  hipError_t get(T** q, size_t count) {
    return dalloc(p, q, count);
  }
  void release(void* q) {
    for (size_t i = 0; i < p.size(); ++i)
      if (p[i] == q) {
        (void)hipFree(q);
        p.erase(p.begin() + i);
        return;
      }
  }
  ~Scratch() { free_all(p); }
};

hipError_t exclusive_sum(Scratch& sc, const int* in, int* out, long long n, hipStream_t stream) {
  size_t bytes = 0;
  hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, n, stream);
  if (e != hipSuccess) return e;
  void* tmp = nullptr;
  if ((e = sc.get((char**)&tmp, bytes)) != hipSuccess) return e;
  e = hipcub::DeviceScan::ExclusiveSum(tmp, bytes, in, out, n, stream);
  return e;
}

inline unsigned blocks(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

struct HostNode {
  double lo[6], hi[6];
  int depth;
  long long e0, e1;
};

}  // namespace

mpg_status stree_build_gpu(const float* d_rec, int n_rec, const StreeBuildParams& prm, std::vector<void*>& allocs,
                           StreeBuilt* out, hipStream_t stream) {
  Scratch sc;
  RootBox B;
  for (int a = 0; a < 6; ++a) { B.lo[a] = prm.lo[a]; B.hi[a] = prm.hi[a]; }
  // samples of the root, in record order
  int *flag, *pos;
  HIP_TRY(sc.get(&flag, (size_t)n_rec + 1));
  HIP_TRY(sc.get(&pos, (size_t)n_rec + 1));
  hipLaunchKernelGGL(k_sb_valid, dim3(blocks((long long)n_rec + 1)), dim3(256), 0, stream, d_rec, n_rec, B, flag);
  HIP_TRY(hipGetLastError());
  HIP_TRY(exclusive_sum(sc, flag, pos, (long long)n_rec + 1, stream));
  int m0 = 0;
  HIP_TRY(hipMemcpyAsync(&m0, pos + n_rec, sizeof(int), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  int* ids;
  uint8_t* own;
  HIP_TRY(sc.get(&ids, (size_t)m0));
  HIP_TRY(sc.get(&own, (size_t)m0));
  hipLaunchKernelGGL(k_sb_compact, dim3(blocks(n_rec)), dim3(256), 0, stream, flag, pos, n_rec, ids, own);
  HIP_TRY(hipGetLastError());
  sc.release(flag);
  sc.release(pos);
  const double limit = prm.thr_scale * std::sqrt((double)m0);

  std::vector<int> axis, child;
  std::vector<float> mid;
  std::vector<int> leaf_node;
  std::vector<long long> leaf_off(1, 0);
  // leaf entries, appended level by level (leaves in node order)
  long long leaf_cap = std::max<long long>(2LL * m0, 1024), leaf_size = 0;
  int* leaf_ids;
  uint8_t* leaf_own;
  HIP_TRY(sc.get(&leaf_ids, (size_t)leaf_cap));
  HIP_TRY(sc.get(&leaf_own, (size_t)leaf_cap));

  std::vector<HostNode> level(1);
  for (int a = 0; a < 6; ++a) { level[0].lo[a] = prm.lo[a]; level[0].hi[a] = prm.hi[a]; }
  level[0].depth = 0;
  level[0].e0 = 0;
  level[0].e1 = m0;
  long long E = m0;
  int first = 0;  // index of the level's first node
  while (!level.empty()) {
    const int nl = (int)level.size();
    const int base = first + nl;  // index of the next level's first node
    std::vector<LevelNode> ln(nl);
    for (int i = 0; i < nl; ++i) {
      const HostNode& h = level[i];
      LevelNode& d = ln[i];
      d.e0 = h.e0;
      d.axis = -1;
      d.lo_l = d.hi_l = d.lo_r = d.hi_r = d.mid = 0.0;
      if (!((double)(h.e1 - h.e0) > limit) || h.depth >= prm.max_depth) continue;
      int ax = 0;
      for (int a = 1; a < 6; ++a)
        if (h.hi[a] - h.lo[a] > h.hi[ax] - h.lo[ax]) ax = a;
      const double m = 0.5 * (h.lo[ax] + h.hi[ax]);
      const double widen = prm.eps * (m - h.lo[ax]);
      d.axis = ax;
      d.mid = m;
      d.lo_l = h.lo[ax] - widen;
      d.hi_l = m + widen;
      d.lo_r = m - widen;
      d.hi_r = h.hi[ax] + widen;
    }
    LevelNode* d_nodes;
    int *ml, *mr, *mf, *sl, *sr, *sf, *bnd;
    HIP_TRY(sc.get(&d_nodes, nl));
    HIP_TRY(hipMemcpyAsync(d_nodes, ln.data(), nl * sizeof(LevelNode), hipMemcpyHostToDevice, stream));
    HIP_TRY(sc.get(&ml, (size_t)E + 1));
    HIP_TRY(sc.get(&mr, (size_t)E + 1));
    HIP_TRY(sc.get(&mf, (size_t)E + 1));
    HIP_TRY(sc.get(&sl, (size_t)E + 1));
    HIP_TRY(sc.get(&sr, (size_t)E + 1));
    HIP_TRY(sc.get(&sf, (size_t)E + 1));
    HIP_TRY(sc.get(&bnd, 3 * ((size_t)nl + 1)));
    hipLaunchKernelGGL(k_sb_classify, dim3(blocks(E + 1)), dim3(256), 0, stream, d_rec, ids, E, d_nodes, nl, ml, mr,
                       mf);
    HIP_TRY(hipGetLastError());
    HIP_TRY(exclusive_sum(sc, ml, sl, E + 1, stream));
    HIP_TRY(exclusive_sum(sc, mr, sr, E + 1, stream));
    HIP_TRY(exclusive_sum(sc, mf, sf, E + 1, stream));
    hipLaunchKernelGGL(k_sb_bounds, dim3(blocks((long long)nl + 1)), dim3(256), 0, stream, d_nodes, nl, E, sl, sr,
                       sf, bnd, bnd + nl + 1, bnd + 2 * (nl + 1));
    HIP_TRY(hipGetLastError());
    std::vector<int> hb(3 * ((size_t)nl + 1));
    HIP_TRY(hipMemcpyAsync(hb.data(), bnd, hb.size() * sizeof(int), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    const int* bl = hb.data();
    const int* br = bl + nl + 1;
    const int* bf = br + nl + 1;
    // the next level: children of the s-th split node are nodes base + 2s,
    // base + 2s + 1, their entries laid out in that order
    std::vector<HostNode> next;
    std::vector<LevelOut> lo(nl);
    long long ne = 0;
    for (int i = 0; i < nl; ++i) {
      const HostNode& h = level[i];
      axis.push_back(ln[i].axis);
      mid.push_back((float)ln[i].mid);
      lo[i].leaf = leaf_size + bf[i];
      lo[i].left = lo[i].right = 0;
      if (ln[i].axis < 0) {
        child.push_back(-1);
        leaf_node.push_back(first + i);
        leaf_off.push_back(leaf_size + bf[i + 1]);
        continue;
      }
      child.push_back(base + (int)next.size());
      const long long L = bl[i + 1] - bl[i], R = br[i + 1] - br[i];
      HostNode l = h, r = h;
      l.hi[ln[i].axis] = ln[i].mid;
      r.lo[ln[i].axis] = ln[i].mid;
      l.depth = r.depth = h.depth + 1;
      l.e0 = ne;
      l.e1 = ne + L;
      r.e0 = ne + L;
      r.e1 = ne + L + R;
      lo[i].left = l.e0;
      lo[i].right = r.e0;
      ne += L + R;
      next.push_back(l);
      next.push_back(r);
    }
    const long long nf = bf[nl];
    if (leaf_size + nf > leaf_cap) {  // grow the leaf buffer
      long long cap = std::max(2 * leaf_cap, leaf_size + nf);
      int* ni;
      uint8_t* no;
      HIP_TRY(sc.get(&ni, (size_t)cap));
      HIP_TRY(sc.get(&no, (size_t)cap));
      if (leaf_size) {
        HIP_TRY(hipMemcpyAsync(ni, leaf_ids, leaf_size * sizeof(int), hipMemcpyDeviceToDevice, stream));
        HIP_TRY(hipMemcpyAsync(no, leaf_own, leaf_size, hipMemcpyDeviceToDevice, stream));
      }
      HIP_TRY(hipStreamSynchronize(stream));
      sc.release(leaf_ids);
      sc.release(leaf_own);
      leaf_ids = ni;
      leaf_own = no;
      leaf_cap = cap;
    }
    LevelOut* d_out;
    int* nids = nullptr;
    uint8_t* nown = nullptr;
    HIP_TRY(sc.get(&d_out, nl));
    HIP_TRY(hipMemcpyAsync(d_out, lo.data(), nl * sizeof(LevelOut), hipMemcpyHostToDevice, stream));
    HIP_TRY(sc.get(&nids, (size_t)ne));
    HIP_TRY(sc.get(&nown, (size_t)ne));
    if (E > 0) {
      hipLaunchKernelGGL(k_sb_scatter, dim3(blocks(E)), dim3(256), 0, stream, d_rec, ids, own, E, d_nodes, nl, d_out,
                         bnd, bnd + nl + 1, bnd + 2 * (nl + 1), sl, sr, sf, nids, nown, leaf_ids, leaf_own);
      HIP_TRY(hipGetLastError());
    }
    // hipMemcpyAsync from pageable host memory returns once the source has
    // been read, so the host vectors may go; the device scratch of this level
    // is released after the stream has drained it
    HIP_TRY(hipStreamSynchronize(stream));
    for (void* q : {(void*)d_nodes, (void*)ml, (void*)mr, (void*)mf, (void*)sl, (void*)sr, (void*)sf, (void*)bnd,
                    (void*)d_out, (void*)ids, (void*)own})
      sc.release(q);
    leaf_size += nf;
    ids = nids;
    own = nown;
    E = ne;
    first = base;
    level.swap(next);
  }
  const int nn = (int)axis.size();
  const int n_leaves = (int)leaf_node.size();
  // node arrays
  HIP_TRY(dalloc(allocs, &out->axis, nn));
  HIP_TRY(dalloc(allocs, &out->mid, nn));
  HIP_TRY(dalloc(allocs, &out->child, nn));
  HIP_TRY(dalloc(allocs, &out->W, nn));
  HIP_TRY(dalloc(allocs, &out->Wn, (size_t)nn * 8));
  HIP_TRY(dalloc(allocs, &out->own, nn));
  HIP_TRY(dalloc(allocs, &out->leaf_groups, nn));
  HIP_TRY(hipMemcpyAsync(out->axis, axis.data(), nn * sizeof(int), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(out->mid, mid.data(), nn * sizeof(float), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(out->child, child.data(), nn * sizeof(int), hipMemcpyHostToDevice, stream));
  hipLaunchKernelGGL(k_sb_zero, dim3(blocks(nn)), dim3(256), 0, stream, out->W, out->Wn, out->own, out->leaf_groups,
                     nn);
  HIP_TRY(hipGetLastError());
  int* d_leaf_node;
  long long* d_leaf_off;
  HIP_TRY(sc.get(&d_leaf_node, n_leaves));
  HIP_TRY(sc.get(&d_leaf_off, (size_t)n_leaves + 1));
  HIP_TRY(hipMemcpyAsync(d_leaf_node, leaf_node.data(), n_leaves * sizeof(int), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(d_leaf_off, leaf_off.data(), (n_leaves + 1) * sizeof(long long), hipMemcpyHostToDevice,
                         stream));
  if (n_leaves > 0) {
    hipLaunchKernelGGL(k_sb_leaf_sums, dim3(blocks(n_leaves, 64)), dim3(64), 0, stream, d_rec, d_leaf_node,
                       d_leaf_off, n_leaves, leaf_ids, leaf_own, out->W, out->Wn, out->own);
    HIP_TRY(hipGetLastError());
  }
  // lobes: leaf entries stably sorted by (leaf rank, n, tau), grouped by key
  const long long total = leaf_size;
  unsigned long long *keys, *skeys;
  int *sids, *mark, *gidx;
  HIP_TRY(sc.get(&keys, (size_t)total));
  HIP_TRY(sc.get(&skeys, (size_t)total));
  HIP_TRY(sc.get(&sids, (size_t)total));
  HIP_TRY(sc.get(&mark, (size_t)total + 1));
  HIP_TRY(sc.get(&gidx, (size_t)total + 1));
  int n_groups = 0;
  if (total > 0) {
    hipLaunchKernelGGL(k_sb_keys, dim3(blocks(total)), dim3(256), 0, stream, d_rec, d_leaf_off, n_leaves, leaf_ids,
                       total, keys);
    HIP_TRY(hipGetLastError());
    int end_bit = 16;
    while (end_bit < 64 && (1LL << (end_bit - 16)) < (long long)n_leaves) ++end_bit;
    size_t bytes = 0;
    HIP_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, keys, skeys, leaf_ids, sids, total, 0, end_bit,
                                               stream));
    char* tmp;
    HIP_TRY(sc.get(&tmp, bytes));
    HIP_TRY(hipcub::DeviceRadixSort::SortPairs((void*)tmp, bytes, keys, skeys, leaf_ids, sids, total, 0, end_bit,
                                               stream));
  }
  hipLaunchKernelGGL(k_sb_group_marks, dim3(blocks(total + 1)), dim3(256), 0, stream, skeys, total, mark);
  HIP_TRY(hipGetLastError());
  HIP_TRY(exclusive_sum(sc, mark, gidx, total + 1, stream));
  HIP_TRY(hipMemcpyAsync(&n_groups, gidx + total, sizeof(int), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  long long* gstart;
  HIP_TRY(sc.get(&gstart, (size_t)n_groups + 1));
  hipLaunchKernelGGL(k_sb_group_starts, dim3(blocks(total + 1)), dim3(256), 0, stream, mark, gidx, total, gstart);
  HIP_TRY(hipGetLastError());
  HIP_TRY(dalloc(allocs, &out->grp_key, n_groups));
  HIP_TRY(dalloc(allocs, &out->grp_w, n_groups));
  HIP_TRY(dalloc(allocs, &out->grp_lobes, n_groups));
  HIP_TRY(dalloc(allocs, &out->lobe, (size_t)total));
  HIP_TRY(dalloc(allocs, &out->lobe_cdf, (size_t)total));
  if (n_groups > 0) {
    hipLaunchKernelGGL(k_sb_groups, dim3(blocks(n_groups, 64)), dim3(64), 0, stream, d_rec, skeys, sids, gstart,
                       n_groups, out->grp_key, out->grp_w, out->grp_lobes, out->lobe, out->lobe_cdf);
    HIP_TRY(hipGetLastError());
  }
  if (n_leaves > 0) {
    hipLaunchKernelGGL(k_sb_leaf_groups, dim3(blocks(n_leaves)), dim3(256), 0, stream, d_leaf_node, d_leaf_off,
                       n_leaves, gidx, out->leaf_groups);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(stream));
  out->n_nodes = nn;
  out->n_leaves = n_leaves;
  out->n_groups = n_groups;
  out->n_lobes = (int)total;
  return MPG_OK;
}
