// Counting walk kernel for NMAX 8.
#include "mpg_count.h"

count_kernel_t count_kernel_8() { return k_walk_count<8>; }
