// Host-side BVH builder interface.
#pragma once
#include <stdint.h>

#include <vector>

namespace mpg_host {

// Binned-SAH BVH (16 bins, leaves of <= 4 triangles).  Emits interior nodes
// only, 16 floats each: left box (lo, hi), right box (lo, hi), then the two
// child references as int bits (>= 0 interior node index; otherwise
// 0x80000000 | count << 24 | start into `order`).  Boxes are padded by `pad`.
// Returns the number of nodes; *max_depth is the deepest interior level.
// ranges receives, per node, the triangle ranges of its two children in
// `order` (left start, left count, right start, right count): every child box
// is the bounding box of its range, which is what a refit recomputes.
int build_bvh(const float* verts, const int32_t* tris, int n_tris, float pad, std::vector<float>& gpu_nodes,
              std::vector<int32_t>& order, std::vector<int32_t>& ranges, int* max_depth);

}  // namespace mpg_host
