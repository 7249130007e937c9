// FP64 instances of the fused stage kernels of degree 2 and 3.
#include "k_stage.inl"

namespace cteno {
template hipError_t stage_fused<double>(const DeviceMesh &m, const FluxLaunch &f, const int *done, int part,
                                     hipStream_t st, unsigned long long *fb_count);
}  // namespace cteno
