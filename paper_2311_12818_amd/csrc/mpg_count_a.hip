// Counting walk kernels for NMAX 1-5.
#include "mpg_count.h"

count_kernel_t count_kernel_1to5(int nmax) {
  switch (nmax) {
    case 1: return k_walk_count<1>;
    case 2: return k_walk_count<2>;
    case 3: return k_walk_count<3>;
    case 4: return k_walk_count<4>;
    default: return k_walk_count<5>;
  }
}
