// Host-side builder of the paper's guide tree (see mpg_stree_host.cpp).
#pragma once
#include <utility>
#include <vector>

namespace mpg_host {

struct StreeParams {
  double lo[6], hi[6];  // root box over (x_D, x_L)
  double eps;           // child overlap, relative to the child's extent along the split axis
  double thr_scale;     // leaf limit c in c sqrt(|S|)
  int max_depth;
};

// Breadth-first tree: per node the split axis (-1 for a leaf), split plane
// and left child (right = left + 1); per leaf the weight W, the weight per
// length W_n (n = 1..8), the number of own samples and its range of groups;
// per group the key n | tau << 8, its weight and its range of lobes; per lobe
// the unit direction, the inclusive prefix of the lobe weights within its
// group and the sample index.
struct StreeHost {
  std::vector<int> axis, child, depth;
  std::vector<float> mid;
  std::vector<float> leaf_W, leaf_Wn;
  std::vector<int> leaf_own;
  std::vector<std::pair<int, int>> leaf_groups;
  std::vector<int> grp_key;
  std::vector<float> grp_w;
  std::vector<std::pair<int, int>> grp_lobes;
  std::vector<float> lobe_dir, lobe_cdf;
  std::vector<int> lobe_sample;
};

// Records: float [n_rec][16] = x_D (3), x_L (3), w_D (3), w, n, tau, 0 x 4.
// Records with w <= 0, a non-finite value, n outside 1..8 or a configuration
// outside the root box are not samples.  Returns the node count.
int build_stree(const float* rec, int n_rec, const StreeParams& prm, StreeHost* out);

}  // namespace mpg_host
