// C entry for the CPU tests of the host BVH builder (4-wide nodes).
#include <cstring>
#include <vector>

#include "../../paper_2311_12818_amd/csrc/mpg_scene.h"

extern "C" int bvh_build(const float* verts, const int* tris, int n_tris, float pad, int max_nodes, float* nodes,
                         int* order, int* ranges, int* max_depth) {
  std::vector<float> nd;
  std::vector<int32_t> ord, rg;
  int n = mpg_host::build_bvh(verts, tris, n_tris, pad, nd, ord, rg, max_depth);
  if (n > max_nodes) return -n;
  std::memcpy(nodes, nd.data(), nd.size() * sizeof(float));
  std::memcpy(order, ord.data(), ord.size() * sizeof(int));
  std::memcpy(ranges, rg.data(), rg.size() * sizeof(int));
  return n;
}
