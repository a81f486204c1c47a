// Counting walk kernels for NMAX 6-7.
#include "mpg_count.h"

count_kernel_t count_kernel_6to7(int nmax) { return nmax <= 6 ? k_walk_count<6> : k_walk_count<7>; }
