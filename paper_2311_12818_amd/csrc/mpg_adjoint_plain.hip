// Plain form of the adjoint: launch (the kernels are instantiated in
// mpg_adjoint_plain_*.hip).
#include "mpg_adjoint_plain.h"

static adj_kernel_t adjoint_kernel(int nmax) {
  if (nmax <= 5) return adjoint_kernel_1to5(nmax);
  if (nmax <= 7) return adjoint_kernel_6to7(nmax);
  return adjoint_kernel_8();
}


mpg_status launch_adjoint_plain(const mpg_scene* s, const WalkParams& P, const EpView& E, const AdjIO& io, int max_len,
                                hipStream_t stream) {
  const int threads = 256;  // k_adjoint's launch bound
  hipLaunchKernelGGL(adjoint_kernel(max_len), dim3((E.N + threads - 1) / threads), dim3(threads), 0, stream, s->dev,
                     P, E, io);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}
