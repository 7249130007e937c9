// FP32 (mixed precision) instances of the reconstruction kernels of degree 4 to 6.
#include "k_recon_ho.inl"

namespace cteno {
template hipError_t reconstruct_hi<float>(const DeviceMesh &m, const double *U, void *FV, uint8_t *delta, int dmode,
                                  const int *done, hipStream_t st, unsigned long long *fb_count);
}  // namespace cteno
