// FP64 instances of the reconstruction kernels of degree 2 and 3.
#include "k_recon.inl"

namespace cteno {
template hipError_t reconstruct_lo<double>(const DeviceMesh &m, const double *U, void *FV, uint8_t *delta, int dmode,
                                  const int *done, hipStream_t st, unsigned long long *fb_count);
}  // namespace cteno
