// Plain adjoint kernel for NMAX 8.
#include "mpg_adjoint_plain.h"

adj_kernel_t adjoint_kernel_8() { return k_adjoint<8>; }
