// Fused SSP-RK3 stage of degree 2 and 3 for one arithmetic type;
// instantiated per type by k_stage_f32.hip and k_stage_f64.hip.
//
// k_stage (part 0), one lane per cell, 256-cell blocks: the reconstruction of
// the block's cells (sec. 2.1-2.6) goes to LDS; after a block barrier each
// cell evaluates the fluxes (sec. 2.7) of its faces whose neighbour lies in
// the same block from LDS, and of its boundary faces, and -- when no face
// leads to another block -- applies its RK stage at once.  A cell with a
// face to another block (a cross cell) stores the values of those faces and
// its stage state from the other faces instead, both by its rank among the
// cross cells (so part 1 reads them contiguously), and k_stage_cross (part
// 1) adds the faces to other blocks.  Both cells of a face evaluate the same
// flux from the same values (LDS holds exactly the values the other cell
// computed), so the update stays conservative to FP64 round-off.  Face
// values of faces inside a block never leave the chip.
#pragma once
#include "kernels_common.h"

namespace cteno {

// FP64 in conserved variables is held to two waves per SIMD, like its
// reconstruction kernel
template <typename real, int R, int NV, int SCHEME, int GFORM, int VARS, int PHYS>
__global__ __launch_bounds__(256, (std::is_same<real, double>::value && VARS == 0) ? 2 : 1)
void k_stage(const ReconArgs<real, (R + 1) * (R + 2) / 2 - 1> ra, const FluxArgs<real> fa) {
    constexpr int NQ = 2, ROW = 3 * NQ * NV;
    constexpr bool F64 = std::is_same<real, double>::value;
    // the block's face-point values; in FP64 the same space first holds the
    // reconstruction's directional coefficients ([3][2][NV] x 256 doubles)
    __shared__ __align__(16) real lfv[256 * ROW];
    __shared__ __align__(16) double lterm[256 * 3 * NV]; // owners' terms of the faces inside the block
    constexpr int K = (R + 1) * (R + 2) / 2 - 1;
    __shared__ real tab[F64 ? 1 : recon_tab_size<K>()];
    __shared__ int wcross[4];                         // cross cells per wave
    static_assert(!F64 || ROW == 3 * 2 * NV, "the face-value rows hold the directional coefficients");
    recon_tab_fill<real, K>(ra, tab);
    __syncthreads();
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t i = blk * 256 + threadIdx.x;
    if (ra.done && *ra.done) return;           // uniform across the grid
    const bool live = i < fa.N;
    const FluxPtrs<real> ptr{fa.FV, fa.fr, fa.area, fa.Un, fa.Us, fa.Uout, fa.dt_ptr, nullptr, nullptr,
                             fa.nonphys, fa.dt_part != nullptr};
    real own[3][NQ][NV];
    real nx[3], ny[3], len[3];
    uint32_t code[3];
    double u0[NV], us[NV], ar = 1.0;
    if (live) {
        const ReconPtrs<real> rp{ra.U, ra.slot, ra.flags, ra.P, nullptr, nullptr, ra.fr, ra.fb_count, tab,
                                 F64 ? reinterpret_cast<double *>(lfv) : nullptr};
        recon_body<real, R, NV, SCHEME, GFORM, 0, VARS>(ra, rp, i, own);
    }
    if constexpr (F64) __syncthreads();     // every lane is done with the coefficients in lfv
    if (live) {
        store_row<real, ROW>(lfv + threadIdx.x * ROW, &own[0][0][0]);
        // the flux phase's operands, requested before the barrier
#pragma unroll
        for (int f = 0; f < 3; ++f) face_record<real>(fa.fr, i, f, nx[f], ny[f], len[f], code[f]);
        rk_load<real, NV>(ptr, i, u0, us, ar);
    }
    __syncthreads();
    // boundary faces and the faces inside the block that this cell owns;
    // the owners' terms go to LDS for the other cells of those faces
    double term[3][NV];
    bool bad = false;
    int kind[3];        // 0: computed here, 1: the owner's term, negated, 2: to another block
    if (live) {
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            real oth[NQ][NV];
            bool wallf = false;
            kind[f] = 0;
            if (code[f] & kNbBoundary) {
                wallf = boundary_state<real, NV, PHYS, 2, NQ>(fa, fa.dt_ptr, code[f], own[f], oth);
            } else {
                const int64_t j = code[f] & kNbIndexMask;
                if ((j >> 8) != blk) { kind[f] = 2; continue; }
                if (!(code[f] & kNbOwner)) { kind[f] = 1; continue; }
                const int g = (code[f] >> 28) & 3;
                load_row<real, NQ * NV>(lfv + (j & 255) * ROW + g * NQ * NV, &oth[0][0]);
            }
            face_term<real, NV, PHYS, NQ>(fa, own[f], oth, true, wallf, nx[f], ny[f], len[f], term[f], bad);
            if (!(code[f] & kNbBoundary)) {
#pragma unroll
                for (int v = 0; v < NV; ++v) lterm[(threadIdx.x * 3 + f) * NV + v] = term[f][v];
            }
        }
    }
    // a cross cell's rank among the block's cross cells (listed in ascending order)
    const bool cross = live && (kind[0] == 2 || kind[1] == 2 || kind[2] == 2);
    const unsigned long long cbal = __ballot(cross);
    if ((threadIdx.x & 63) == 0) wcross[threadIdx.x >> 6] = __popcll(cbal);
    __syncthreads();
    double dtc = INFINITY;
    if (live) {
        double acc[NV], nrm[3][3];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            nrm[f][0] = (double)nx[f]; nrm[f][1] = (double)ny[f]; nrm[f][2] = (double)len[f];
            if (kind[f] == 2) continue;
            if (kind[f] == 1) {
                // the owner evaluated F(owner side, this side; owner normal):
                // this cell's term is its exact negation
                const int64_t j = code[f] & kNbIndexMask;
                const int g = (code[f] >> 28) & 3;
#pragma unroll
                for (int v = 0; v < NV; ++v) term[f][v] = -lterm[((j & 255) * 3 + g) * NV + v];
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += term[f][v];
        }
        if (bad && fa.nonphys) atomicOr(fa.nonphys, 1);
        if (!cross) {
            dtc = rk_apply<real, NV, PHYS>(fa, ptr, i, acc, nrm, u0, us, ar);
        } else {
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
            int before = 0;
#pragma unroll
            for (int w = 0; w < 3; ++w) before += w < wv ? wcross[w] : 0;
            const int64_t t = (int64_t)fa.xbase[blk] + before + __popcll(cbal & ((1ull << lane) - 1));
            // only the values of the faces to other blocks leave the chip
#pragma unroll
            for (int f = 0; f < 3; ++f)
                if (kind[f] == 2)
                    store_row<real, NQ * NV>(const_cast<real *>(fa.FV) + t * ROW + f * NQ * NV, &own[f][0][0]);
            // the stage state from the faces inside the block; part 1 adds
            // dt times the residual of the others with rk_weight
            const double dt = ptr.dt_ptr ? *ptr.dt_ptr : fa.dt_value;
#pragma unroll
            for (int v = 0; v < NV; ++v) fa.xpart[t * NV + v] = rk_value(fa.stage, u0[v], us[v], dt * (-acc[v] / ar));
        }
    }
    if (fa.dt_part) {
        const double bm = block_min(dtc);
        if (threadIdx.x == 0) fa.dt_part[blockIdx.x] = bm;
    }
}

// part 1: one lane per cross cell, in cross-cell order: the faces to other
// blocks from both sides' stored values, added to the partial stage state
template <typename real, int NV, int PHYS>
__global__ __launch_bounds__(256) void k_stage_cross(const FluxArgs<real> fa) {
    constexpr int NQ = 2, ROW = 3 * NQ * NV;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (fa.ctrl && fa.ctrl->done) return;      // uniform across the grid
    double dtc = INFINITY;
    if (t < fa.n_cross) {
        const int64_t i = fa.xcells[t];
        const FluxPtrs<real> ptr{fa.FV, fa.fr, fa.area, fa.Un, fa.Us, fa.Uout, fa.dt_ptr, nullptr, nullptr,
                                 fa.nonphys, fa.dt_part != nullptr};
        double acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = 0.0;
        double nrm[3][3];
        bool bad = false;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            real nx, ny, len;
            uint32_t code;
            face_record<real>(fa.xfr, t, f, nx, ny, len, code);
            nrm[f][0] = (double)nx; nrm[f][1] = (double)ny; nrm[f][2] = (double)len;
            const int tn = fa.xnb[t * 3 + f];
            if (tn < 0) continue;                 // a boundary, or inside the block: in part 0's state
            const bool owner = (code & kNbOwner) != 0;
            const int g = (code >> 28) & 3;
            // both sides' values of this face, as part 0 stored them
            real mine[NQ][NV], oth[NQ][NV];
            load_row<real, NQ * NV>(fa.FV + t * ROW + f * NQ * NV, &mine[0][0]);
            load_row<real, NQ * NV>(fa.FV + (int64_t)tn * ROW + g * NQ * NV, &oth[0][0]);
            double term[NV];
            face_term<real, NV, PHYS, NQ>(fa, mine, oth, owner, false, nx, ny, len, term, bad);
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += term[v];
        }
        if (bad && fa.nonphys) atomicOr(fa.nonphys, 1);
        const double dt = ptr.dt_ptr ? *ptr.dt_ptr : fa.dt_value;
        const double ar = fa.xarea[t], w = rk_weight(fa.stage);
        double un[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) un[v] = fa.xpart[t * NV + v] + w * (dt * (-acc[v] / ar));
        dtc = rk_store<real, NV, PHYS>(fa, ptr, i, un, nrm, ar);
    }
    if (fa.dt_part) {
        const double bm = block_min(dtc);
        if (threadIdx.x == 0) fa.dt_part[fa.part_off + blockIdx.x] = bm;
    }
}

template <typename real, int R, int NV, int VARS, int PHYS>
static void stage_launch(const DeviceMesh &m, const ReconArgs<real, (R + 1) * (R + 2) / 2 - 1> &ra,
                         const FluxArgs<real> &fa, unsigned grid, hipStream_t st) {
#define ST_LAUNCH(SCH, GF) \
    hipLaunchKernelGGL((k_stage<real, R, NV, SCH, GF, VARS, PHYS>), dim3(grid), dim3(256), 0, st, ra, fa)
    if (m.scheme == CTENO_SCHEME_CTENOZ && m.gamma_form == CTENO_GAMMA_SCALED) ST_LAUNCH(CTENO_SCHEME_CTENOZ, CTENO_GAMMA_SCALED);
    else if (m.scheme == CTENO_SCHEME_CTENOZ) ST_LAUNCH(CTENO_SCHEME_CTENOZ, CTENO_GAMMA_PAPER);
    else if (m.scheme == CTENO_SCHEME_CWENO) ST_LAUNCH(CTENO_SCHEME_CWENO, CTENO_GAMMA_PAPER);
    else if (m.scheme == CTENO_SCHEME_TENO) ST_LAUNCH(CTENO_SCHEME_TENO, CTENO_GAMMA_PAPER);
    else if (m.gamma_form == CTENO_GAMMA_LAMBDA) ST_LAUNCH(CTENO_SCHEME_CTENO, CTENO_GAMMA_LAMBDA);
    else ST_LAUNCH(CTENO_SCHEME_CTENO, CTENO_GAMMA_PAPER);
#undef ST_LAUNCH
}

template <typename real, int R, int NV, int PHYS>
static hipError_t stage_t(const DeviceMesh &m, const FluxLaunch &f, const int *done, hipStream_t st,
                          unsigned long long *fb_count) {
    constexpr int K = (R + 1) * (R + 2) / 2 - 1;
    ReconArgs<real, K> ra;
    ra.N = m.N;
    ra.U = f.Us;
    ra.slot = m.slot;
    ra.flags = m.flags;
    if constexpr (std::is_same<real, double>::value) { ra.P = m.P64; ra.fr = m.fr64; }
    else { ra.P = m.P32; ra.fr = m.fr32; }
    if (!ra.P || !ra.fr) return hipErrorInvalidValue;
    ra.FV = nullptr;
    ra.delta = nullptr;
    ra.done = done;
    fill_recon_constants<real, K>(m, ra);
    ra.fb_count = fb_count;
    FluxArgs<real> fa;
    fill_flux_args<real>(m, f, fa);
    const unsigned grid = (unsigned)m.blocks();
    if (m.vars == CTENO_VARS_CHARACTERISTIC) {
        if constexpr (NV == 4) stage_launch<real, R, NV, 1, PHYS>(m, ra, fa, grid, st);
        else return hipErrorInvalidValue;
    } else {
        stage_launch<real, R, NV, 0, PHYS>(m, ra, fa, grid, st);
    }
    return hipGetLastError();
}

template <typename real>
hipError_t stage_fused(const DeviceMesh &m, const FluxLaunch &f, const int *done, int part, hipStream_t st,
                       unsigned long long *fb_count) {
    if (f.mode != 2 || m.r > 3 || m.tab.Nq != 2 || !f.xpart || !f.FV) return hipErrorInvalidValue;
    const void *xfr = std::is_same<real, double>::value ? (const void *)m.xfr64 : (const void *)m.xfr32;
    if (m.n_cross && (!m.xcells || !m.xbase || !m.xnb || !m.xarea || !xfr)) return hipErrorInvalidValue;
    if (part == 1) {
        if (m.n_cross == 0) return hipSuccess;
        FluxArgs<real> fa;
        fill_flux_args<real>(m, f, fa);
        const unsigned grid = (unsigned)m.cross_blocks();
        if (m.physics == CTENO_EULER)
            hipLaunchKernelGGL((k_stage_cross<real, 4, CTENO_EULER>), dim3(grid), dim3(256), 0, st, fa);
        else
            hipLaunchKernelGGL((k_stage_cross<real, 1, CTENO_ADVECTION>), dim3(grid), dim3(256), 0, st, fa);
        return hipGetLastError();
    }
    if (m.physics == CTENO_EULER) {
        if (m.nv != 4) return hipErrorInvalidValue;
        return m.r == 2 ? stage_t<real, 2, 4, CTENO_EULER>(m, f, done, st, fb_count)
                        : stage_t<real, 3, 4, CTENO_EULER>(m, f, done, st, fb_count);
    }
    if (m.nv != 1) return hipErrorInvalidValue;
    return m.r == 2 ? stage_t<real, 2, 1, CTENO_ADVECTION>(m, f, done, st, fb_count)
                    : stage_t<real, 3, 1, CTENO_ADVECTION>(m, f, done, st, fb_count);
}

}  // namespace cteno
