// Plain adjoint kernels for NMAX 1-5.
#include "mpg_adjoint_plain.h"

adj_kernel_t adjoint_kernel_1to5(int nmax) {
  switch (nmax) {
    case 1: return k_adjoint<1>;
    case 2: return k_adjoint<2>;
    case 3: return k_adjoint<3>;
    case 4: return k_adjoint<4>;
    default: return k_adjoint<5>;
  }
}
