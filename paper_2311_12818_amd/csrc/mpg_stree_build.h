// Device build of the paper's guide tree (Sec. 5.6): see mpg_stree_build.hip.
#pragma once
#include "mpg_internal.h"

#include <vector>

struct StreeBuildParams {
  double lo[6], hi[6];  // root box over (x_D, x_L)
  double eps;           // child overlap, relative to the child's extent along the split axis
  double thr_scale;     // leaf limit c in c sqrt(|S|)
  int max_depth;
};

// The built tree in device arrays (allocated into the caller's list, which
// owns them).  Nodes in breadth-first order: per node the split axis (-1 for
// a leaf), split plane and left child (right = left + 1); per leaf the
// weight W, the weight per length W_n (n = 1..8), the number of own samples
// and its range of groups (internal nodes: zeros); per group the key n | tau
// << 8, its weight and its range of lobes; per lobe the unit direction (w =
// 0, the footprint is set later) and the inclusive prefix of the lobe
// weights within its group.
struct StreeBuilt {
  int* axis = nullptr;
  float* mid = nullptr;
  int* child = nullptr;
  float* W = nullptr;
  float* Wn = nullptr;
  int* own = nullptr;
  int2* leaf_groups = nullptr;
  int* grp_key = nullptr;
  float* grp_w = nullptr;
  int2* grp_lobes = nullptr;
  float4* lobe = nullptr;
  float* lobe_cdf = nullptr;
  int n_nodes = 0, n_leaves = 0, n_groups = 0, n_lobes = 0;
};

// Records: device float [n_rec][16] = x_D (3), x_L (3), w_D (3), w, n, tau,
// 0 x 4.  Records with w <= 0, a non-finite value, n outside 1..8 or a
// configuration outside the root box are not samples.  Synchronises the
// stream (the level sizes steer the launches).
mpg_status stree_build_gpu(const float* d_rec, int n_rec, const StreeBuildParams& prm, std::vector<void*>& allocs,
                           StreeBuilt* out, hipStream_t stream);
