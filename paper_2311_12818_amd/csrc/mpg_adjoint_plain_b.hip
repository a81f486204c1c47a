// Plain adjoint kernels for NMAX 6-7.
#include "mpg_adjoint_plain.h"

adj_kernel_t adjoint_kernel_6to7(int nmax) { return nmax <= 6 ? k_adjoint<6> : k_adjoint<7>; }
