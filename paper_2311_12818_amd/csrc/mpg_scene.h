// Host-side BVH builder interface.
#pragma once
#include <stdint.h>

#include <vector>

namespace mpg_host {

// Binned-SAH BVH (16 bins, leaves of <= 4 triangles), collapsed into 4-wide
// nodes of 32 floats: child boxes as lo.x[4], lo.y[4], lo.z[4], hi.x[4],
// hi.y[4], hi.z[4], then the four child references as int bits (>= 0 node
// index; otherwise 0x80000000 | count << 24 | start into `order`; an empty
// child has count 0 and a box at +infinity that no ray enters), then 4
// unused words.  Boxes are padded by `pad`.  Returns the number of nodes;
// *max_depth + 1 is the traversal stack depth a ray can need (three entries
// per level).
// ranges receives, per node, the triangle ranges of its four children in
// `order` (start, count pairs; 0, 0 when empty): every child box is the
// bounding box of its range, which is what a refit recomputes.
int build_bvh(const float* verts, const int32_t* tris, int n_tris, float pad, std::vector<float>& gpu_nodes,
              std::vector<int32_t>& order, std::vector<int32_t>& ranges, int* max_depth);

}  // namespace mpg_host
