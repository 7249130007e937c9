// Reconstruction of degree 2 and 3 (one lane per cell): the kernel and its
// launch, for one arithmetic type; instantiated per type by k_recon_f32.hip
// and k_recon_f64.hip.
#pragma once
#include "kernels_common.h"

namespace cteno {

// The FP64 march in conserved variables is held to two waves per SIMD (its
// directional coefficients wait in LDS); the other instances take the
// registers they need
template <typename real, int R, int NV, int SCHEME, int GFORM, int DMODE, int VARS>
__global__ __launch_bounds__(256, (std::is_same<real, double>::value && VARS == 0 && DMODE != 2) ? 2 : 1)
void k_reconstruct(const ReconArgs<real, (R + 1) * (R + 2) / 2 - 1> a) {
    constexpr int K = (R + 1) * (R + 2) / 2 - 1;
    constexpr bool F64 = std::is_same<real, double>::value;
    __shared__ real tab[F64 ? 1 : recon_tab_size<K>()];
    __shared__ double lad[F64 ? 3 * 2 * NV * 256 : 1];   // FP64: directional coefficients
    recon_tab_fill<real, K>(a, tab);
    __syncthreads();
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    if (a.done && *a.done) return;
    const ReconPtrs<real> ptr{a.U, a.slot, a.flags, a.P, a.FV, a.delta, a.fr, a.fb_count, tab, lad};
    real out[3][2][NV];
    recon_body<real, R, NV, SCHEME, GFORM, DMODE, VARS>(a, ptr, i, out);
    store_row<real, 3 * 2 * NV>(ptr.FV + i * 3 * 2 * NV, &out[0][0][0]);
}


template <typename real, int R, int NV, int VARS>
static void reconstruct_launch(const DeviceMesh &m, const ReconArgs<real, (R + 1) * (R + 2) / 2 - 1> &a, int dmode,
                               unsigned grid, hipStream_t st) {
#define CT_LAUNCH(SCH, GF, DM) \
    hipLaunchKernelGGL((k_reconstruct<real, R, NV, SCH, GF, DM, VARS>), dim3(grid), dim3(256), 0, st, a)
#define CT_DM(SCH, GF)                        \
    switch (dmode) {                          \
        case 0: CT_LAUNCH(SCH, GF, 0); break; \
        case 1: CT_LAUNCH(SCH, GF, 1); break; \
        default: CT_LAUNCH(SCH, GF, 2); break; \
    }
    if (m.scheme == CTENO_SCHEME_CTENOZ && m.gamma_form == CTENO_GAMMA_SCALED) { CT_DM(CTENO_SCHEME_CTENOZ, CTENO_GAMMA_SCALED); }
    else if (m.scheme == CTENO_SCHEME_CTENOZ) { CT_DM(CTENO_SCHEME_CTENOZ, CTENO_GAMMA_PAPER); }
    else if (m.scheme == CTENO_SCHEME_CWENO) { CT_DM(CTENO_SCHEME_CWENO, CTENO_GAMMA_PAPER); }
    else if (m.scheme == CTENO_SCHEME_TENO) { CT_DM(CTENO_SCHEME_TENO, CTENO_GAMMA_PAPER); }
    else if (m.gamma_form == CTENO_GAMMA_LAMBDA) { CT_DM(CTENO_SCHEME_CTENO, CTENO_GAMMA_LAMBDA); }
    else { CT_DM(CTENO_SCHEME_CTENO, CTENO_GAMMA_PAPER); }
#undef CT_DM
#undef CT_LAUNCH
}

template <typename real, int R, int NV>
static hipError_t reconstruct_t(const DeviceMesh &m, const double *U, void *FV, uint8_t *delta, int dmode,
                                const int *done, hipStream_t st, unsigned long long *fb_count) {
    constexpr int K = (R + 1) * (R + 2) / 2 - 1;
    ReconArgs<real, K> a;
    a.N = m.N;
    a.U = U;
    a.slot = m.slot;
    a.flags = m.flags;
    if constexpr (std::is_same<real, double>::value) a.P = m.P64;
    else a.P = m.P32;
    if (!a.P) return hipErrorInvalidValue;
    a.FV = (real *)FV;
    a.delta = delta;
    a.done = done;
    if constexpr (std::is_same<real, double>::value) a.fr = m.fr64;
    else a.fr = m.fr32;
    fill_recon_constants<real, K>(m, a);
    a.fb_count = fb_count;
    const unsigned grid = (unsigned)m.blocks();
    if (m.vars == CTENO_VARS_CHARACTERISTIC) {
        if constexpr (NV == 4) {
            if (!a.fr) return hipErrorInvalidValue;
            reconstruct_launch<real, R, NV, 1>(m, a, dmode, grid, st);
        } else {
            return hipErrorInvalidValue;
        }
    } else {
        reconstruct_launch<real, R, NV, 0>(m, a, dmode, grid, st);
    }
    return hipGetLastError();
}

template <typename real>
hipError_t reconstruct_lo(const DeviceMesh &m, const double *U, void *FV, uint8_t *delta, int dmode,
                          const int *done, hipStream_t st, unsigned long long *fb_count) {
    if (m.nv == 4) {
        switch (m.r) {
            case 2: return reconstruct_t<real, 2, 4>(m, U, FV, delta, dmode, done, st, fb_count);
            case 3: return reconstruct_t<real, 3, 4>(m, U, FV, delta, dmode, done, st, fb_count);
        }
    } else {
        switch (m.r) {
            case 2: return reconstruct_t<real, 2, 1>(m, U, FV, delta, dmode, done, st, fb_count);
            case 3: return reconstruct_t<real, 3, 1>(m, U, FV, delta, dmode, done, st, fb_count);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace cteno
