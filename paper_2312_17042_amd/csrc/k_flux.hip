// Flux / residual / RK stage kernels, step control, the batched serving
// kernels, layout conversions and utilities; the reconstruction dispatch.
#include "kernels_common.h"

#include <mutex>

namespace cteno {

hipError_t launch_reconstruct(const DeviceMesh &m, bool fp32, const double *U, void *FV, uint8_t *delta, int dmode,
                              const int *done, hipStream_t st, unsigned long long *fb_count) {
    if (m.r >= 4)
        return fp32 ? reconstruct_hi<float>(m, U, FV, delta, dmode, done, st, fb_count)
                    : reconstruct_hi<double>(m, U, FV, delta, dmode, done, st, fb_count);
    return fp32 ? reconstruct_lo<float>(m, U, FV, delta, dmode, done, st, fb_count)
                : reconstruct_lo<double>(m, U, FV, delta, dmode, done, st, fb_count);
}

template <typename real, int NV, int PHYS, int MODE, int NQ>
__global__ __launch_bounds__(256) void k_flux(const FluxArgs<real> a) {
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (a.ctrl && a.ctrl->done) return;        // uniform across the grid
    const FluxPtrs<real> ptr{a.FV, a.fr, a.area, a.Un, a.Us, a.Uout, a.dt_ptr, a.flux_out, a.resid, a.nonphys,
                             a.dt_part != nullptr};
    double dtc = INFINITY;
    if (i < a.N) dtc = flux_body<real, NV, PHYS, MODE, NQ>(a, ptr, i);
    if (MODE == 2 && a.dt_part) {
        const double bm = block_min(dtc);
        if (threadIdx.x == 0) a.dt_part[blockIdx.x] = bm;
    }
}

template <typename real, int NV, int PHYS>
static hipError_t flux_t(const DeviceMesh &m, const FluxLaunch &f, hipStream_t st) {
    FluxArgs<real> a;
    fill_flux_args<real>(m, f, a);
    const unsigned grid = (unsigned)m.blocks();
#define FX_LAUNCH(NQ)                                                                                         \
    switch (f.mode) {                                                                                         \
        case 0: hipLaunchKernelGGL((k_flux<real, NV, PHYS, 0, NQ>), dim3(grid), dim3(256), 0, st, a); break; \
        case 1: hipLaunchKernelGGL((k_flux<real, NV, PHYS, 1, NQ>), dim3(grid), dim3(256), 0, st, a); break; \
        default: hipLaunchKernelGGL((k_flux<real, NV, PHYS, 2, NQ>), dim3(grid), dim3(256), 0, st, a); break; \
    }
    switch (m.tab.Nq) {
        case 2: FX_LAUNCH(2); break;
        case 3: FX_LAUNCH(3); break;
        case 4: FX_LAUNCH(4); break;
        default: return hipErrorInvalidValue;
    }
#undef FX_LAUNCH
    return hipGetLastError();
}

hipError_t launch_stage(const DeviceMesh &m, bool fp32, const FluxLaunch &f, const int *done, int part,
                        hipStream_t st, unsigned long long *fb_count) {
    return fp32 ? stage_fused<float>(m, f, done, part, st, fb_count)
                : stage_fused<double>(m, f, done, part, st, fb_count);
}

hipError_t launch_flux(const DeviceMesh &m, bool fp32, const FluxLaunch &f, hipStream_t st) {
    if (m.physics == CTENO_EULER)
        return fp32 ? flux_t<float, 4, CTENO_EULER>(m, f, st) : flux_t<double, 4, CTENO_EULER>(m, f, st);
    return fp32 ? flux_t<float, 1, CTENO_ADVECTION>(m, f, st) : flux_t<double, 1, CTENO_ADVECTION>(m, f, st);
}

// ===========================================================================
// time-step control
// ===========================================================================

template <typename real, int NV, int PHYS>
__global__ __launch_bounds__(256) void k_dt_partials(int64_t N, const double *U, const real *fr, const double *area,
                                                     double gamma, double ax, double ay, double *part) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double dtc = INFINITY;
    if (i < N) {
        double u[NV], nrm[3][3];
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = U[i * NV + v];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            real nx, ny, len;
            uint32_t code;
            face_record<real>(fr, i, f, nx, ny, len, code);
            nrm[f][0] = nx; nrm[f][1] = ny; nrm[f][2] = len;
        }
        dtc = cell_dt_bound<NV, PHYS>(u, nrm, area[i], gamma, ax, ay);
    }
    const double bm = block_min(dtc);
    if (threadIdx.x == 0) part[blockIdx.x] = bm;
}

hipError_t launch_dt_partials(const DeviceMesh &m, bool fp32, const double *U, double *part, hipStream_t st) {
    const unsigned grid = (unsigned)m.blocks();
    const bool f32 = (fp32 && m.fr32) || m.fr64 == nullptr;
    if (m.physics == CTENO_EULER) {
        if (f32) hipLaunchKernelGGL((k_dt_partials<float, 4, CTENO_EULER>), dim3(grid), dim3(256), 0, st, m.N, U,
                                    m.fr32, m.area, m.gamma, m.ax, m.ay, part);
        else hipLaunchKernelGGL((k_dt_partials<double, 4, CTENO_EULER>), dim3(grid), dim3(256), 0, st, m.N, U,
                                m.fr64, m.area, m.gamma, m.ax, m.ay, part);
    } else {
        if (f32) hipLaunchKernelGGL((k_dt_partials<float, 1, CTENO_ADVECTION>), dim3(grid), dim3(256), 0, st, m.N, U,
                                    m.fr32, m.area, m.gamma, m.ax, m.ay, part);
        else hipLaunchKernelGGL((k_dt_partials<double, 1, CTENO_ADVECTION>), dim3(grid), dim3(256), 0, st, m.N, U,
                                m.fr64, m.area, m.gamma, m.ax, m.ay, part);
    }
    return hipGetLastError();
}

// Commits the pending step (t <- t_next), then decides the next one exactly
// as: stop when t >= t_final or the step budget is used; dt = cfl * bound;
// clip the last step onto t_final.
__device__ void control_logic(Ctrl *c, double bound, int commit_only) {
    if (c->pending) {
        c->t = c->t_next;
        c->step += 1;
        c->pending = 0;
    }
    if (commit_only || c->done) return;
    if (c->nonphysical || !(c->t < c->t_final) || c->step >= c->max_steps) {
        c->done = 1;
        return;
    }
    double dt = c->cfl * bound;
    double tn = c->t + dt;
    if (dt >= c->t_final - c->t) {
        dt = c->t_final - c->t;
        tn = c->t_final;
    }
    if (!(dt > 0.0)) {
        c->done = 1;
        c->nonphysical = 1;
        return;
    }
    c->dt = dt;
    c->t_next = tn;
    c->pending = 1;
}

// minimum of part[0..n) over the block (valid in thread 0)
__device__ __forceinline__ double block_min_array(const double *part, int64_t n, bool reduce) {
    __shared__ double red[16];
    double v = INFINITY;
    if (reduce)
        for (int64_t k = threadIdx.x; k < n; k += blockDim.x) v = fmin(v, part[k]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double bound = INFINITY;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) bound = fmin(bound, red[k]);
    return bound;
}

// Step control of one march, one block: the bound is the minimum of the
// per-block minima left by the last stage (or by k_dt_partials).
__global__ __launch_bounds__(1024) void k_control(Ctrl *c, const double *part, int64_t n_part, int commit_only) {
    const bool reduce = !commit_only && !c->done;
    const double bound = block_min_array(part, n_part, reduce);
    if (threadIdx.x == 0) control_logic(c, bound, commit_only);
}

hipError_t launch_control(Ctrl *ctrl, const double *part, int64_t n_part, int commit_only, hipStream_t st) {
    hipLaunchKernelGGL(k_control, dim3(1), dim3(1024), 0, st, ctrl, part, n_part, commit_only);
    return hipGetLastError();
}

// ===========================================================================
// batched serving kernels: one launch covers every active solve (slot)
// ===========================================================================

// slot of global block b: slots hold consecutive block ranges in table order
// (binary search for the first range that ends past b)
__device__ __forceinline__ int find_slot(const BatchSlot *tab, int n, int64_t b) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (tab[mid].block0 + tab[mid].nblocks > b) hi = mid;
        else lo = mid + 1;
    }
    return lo < n && b >= tab[lo].block0 ? lo : -1;
}

template <int R, int SCHEME, int GFORM>
__global__ __launch_bounds__(256) void k_reconstruct_batch(const ReconArgs<float, (R + 1) * (R + 2) / 2 - 1> a,
                                                           const BatchSlot *tab, const int *n_slots, int stage) {
    constexpr int K = (R + 1) * (R + 2) / 2 - 1;
    const int64_t b = blockIdx.x;
    const int s = find_slot(tab, *n_slots, b);
    if (s < 0) return;                        // uniform across the block
    const BatchSlot &t = tab[s];
    if (t.ctrl->done) return;
    __shared__ float ctab[recon_tab_size<K>()];
    recon_tab_fill<float, K>(a, ctab);
    __syncthreads();
    const int64_t i = (b - t.block0) * blockDim.x + threadIdx.x;
    if (i >= t.N) return;
    const ReconPtrs<float> ptr{t.U[stage], t.slot, t.flags, t.P, t.FV, nullptr, nullptr, &t.ctrl->fallbacks, ctab,
                               nullptr};
    float out[3][2][4];
    recon_body<float, R, 4, SCHEME, GFORM, 0, 0>(a, ptr, i, out);
    store_row<float, 3 * 2 * 4>(ptr.FV + i * 3 * 2 * 4, &out[0][0][0]);
}

__global__ __launch_bounds__(256) void k_flux_batch(const FluxArgs<float> a, const BatchSlot *tab, const int *n_slots) {
    const int64_t b = blockIdx.x;
    const int s = find_slot(tab, *n_slots, b);
    if (s < 0) return;
    const BatchSlot &t = tab[s];
    if (t.ctrl->done) return;                 // uniform across the block
    const int stage = a.stage;
    const int64_t local = b - t.block0;
    const int64_t i = local * blockDim.x + threadIdx.x;
    const FluxPtrs<float> ptr{t.FV, t.fr, t.area, t.U[0], t.U[stage], stage == 2 ? t.U[0] : t.U[stage + 1],
                              &t.ctrl->dt, nullptr, nullptr, &t.ctrl->nonphysical, stage == 2};
    double dtc = INFINITY;
    if (i < t.N) dtc = flux_body<float, 4, CTENO_EULER, 2, 2>(a, ptr, i);
    if (stage == 2) {
        const double bm = block_min(dtc);
        if (threadIdx.x == 0) t.dt_part[local] = bm;
    }
}

__global__ __launch_bounds__(1024) void k_control_batch(const BatchSlot *tab, const int *n_slots) {
    if ((int)blockIdx.x >= *n_slots) return;
    const BatchSlot &t = tab[blockIdx.x];
    const bool reduce = !t.ctrl->done;
    const double bound = block_min_array(t.dt_part, t.nblocks, reduce);
    if (threadIdx.x == 0) control_logic(t.ctrl, bound, 0);
}

template <int R>
static hipError_t batch_step_r(const DeviceMesh &proto, const BatchSlot *tab, const int *n_slots, int max_slots,
                               int64_t max_blocks, hipStream_t st) {
    constexpr int K = (R + 1) * (R + 2) / 2 - 1;
    ReconArgs<float, K> ra;
    std::memset(&ra, 0, sizeof ra);
    fill_recon_constants<float, K>(proto, ra);
    FluxArgs<float> fa{};
    std::memset(&fa, 0, sizeof fa);
    fa.gamma = (float)proto.gamma; fa.ax = (float)proto.ax; fa.ay = (float)proto.ay; fa.gamma64 = proto.gamma;
    fa.gw[0] = fa.gw[1] = 0.5f;
    fa.gw[2] = fa.gw[3] = 0.0f;
    hipLaunchKernelGGL(k_control_batch, dim3(max_slots), dim3(1024), 0, st, tab, n_slots);
    for (int stage = 0; stage < 3; ++stage) {
        if (proto.scheme == CTENO_SCHEME_CTENOZ && proto.gamma_form == CTENO_GAMMA_SCALED)
            hipLaunchKernelGGL((k_reconstruct_batch<R, CTENO_SCHEME_CTENOZ, CTENO_GAMMA_SCALED>), dim3(max_blocks),
                               dim3(256), 0, st, ra, tab, n_slots, stage);
        else if (proto.scheme == CTENO_SCHEME_CTENOZ)
            hipLaunchKernelGGL((k_reconstruct_batch<R, CTENO_SCHEME_CTENOZ, CTENO_GAMMA_PAPER>), dim3(max_blocks),
                               dim3(256), 0, st, ra, tab, n_slots, stage);
        else if (proto.scheme == CTENO_SCHEME_CWENO)
            hipLaunchKernelGGL((k_reconstruct_batch<R, CTENO_SCHEME_CWENO, CTENO_GAMMA_PAPER>), dim3(max_blocks),
                               dim3(256), 0, st, ra, tab, n_slots, stage);
        else if (proto.scheme == CTENO_SCHEME_TENO)
            hipLaunchKernelGGL((k_reconstruct_batch<R, CTENO_SCHEME_TENO, CTENO_GAMMA_PAPER>), dim3(max_blocks),
                               dim3(256), 0, st, ra, tab, n_slots, stage);
        else if (proto.gamma_form == CTENO_GAMMA_LAMBDA)
            hipLaunchKernelGGL((k_reconstruct_batch<R, CTENO_SCHEME_CTENO, CTENO_GAMMA_LAMBDA>), dim3(max_blocks),
                               dim3(256), 0, st, ra, tab, n_slots, stage);
        else
            hipLaunchKernelGGL((k_reconstruct_batch<R, CTENO_SCHEME_CTENO, CTENO_GAMMA_PAPER>), dim3(max_blocks),
                               dim3(256), 0, st, ra, tab, n_slots, stage);
        fa.stage = stage;
        hipLaunchKernelGGL(k_flux_batch, dim3(max_blocks), dim3(256), 0, st, fa, tab, n_slots);
    }
    return hipGetLastError();
}

hipError_t launch_batch_step(const DeviceMesh &proto, const BatchSlot *tab, const int *n_slots, int max_slots,
                             int64_t max_blocks, hipStream_t st) {
    if (proto.nv != 4 || proto.physics != CTENO_EULER) return hipErrorInvalidValue;
    switch (proto.r) {
        case 2: return batch_step_r<2>(proto, tab, n_slots, max_slots, max_blocks, st);
        case 3: return batch_step_r<3>(proto, tab, n_slots, max_slots, max_blocks, st);
        default: return hipErrorInvalidValue;
    }
}

// ===========================================================================
// layout conversions and utilities
// ===========================================================================

__global__ void k_user_to_state(int64_t N, int nv, const int32_t *perm, const double *user, double *state) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int64_t u = perm[k];
    for (int v = 0; v < nv; ++v) state[k * nv + v] = user[(int64_t)v * N + u];
}
__global__ void k_state_to_user(int64_t N, int nv, const int32_t *perm, const double *state, double *user) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int64_t u = perm[k];
    for (int v = 0; v < nv; ++v) user[(int64_t)v * N + u] = state[k * nv + v];
}
// rows of `width` elements, internal row k <-> caller row perm[k]
template <typename T>
__global__ void k_rows_to_user(int64_t N, int width, const int32_t *perm, const T *src, T *dst) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int64_t u = perm[k];
    for (int e = 0; e < width; ++e) dst[u * width + e] = src[k * width + e];
}
template <typename T>
__global__ void k_rows_from_user(int64_t N, int width, const int32_t *perm, const T *src, T *dst) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int64_t u = perm[k];
    for (int e = 0; e < width; ++e) dst[k * width + e] = src[u * width + e];
}

static unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_user_to_state(const DeviceMesh &m, const double *user, double *state, hipStream_t st) {
    hipLaunchKernelGGL(k_user_to_state, dim3(grid_for(m.N)), dim3(256), 0, st, m.N, m.nv, m.perm, user, state);
    return hipGetLastError();
}
hipError_t launch_state_to_user(const DeviceMesh &m, const double *state, double *user, hipStream_t st) {
    hipLaunchKernelGGL(k_state_to_user, dim3(grid_for(m.N)), dim3(256), 0, st, m.N, m.nv, m.perm, state, user);
    return hipGetLastError();
}
hipError_t launch_fv_to_user(const DeviceMesh &m, bool fp32, const void *fv, void *user, hipStream_t st) {
    const int w = 3 * m.tab.Nq * m.nv;
    if (fp32) hipLaunchKernelGGL(k_rows_to_user<float>, dim3(grid_for(m.N)), dim3(256), 0, st, m.N, w, m.perm, (const float *)fv, (float *)user);
    else hipLaunchKernelGGL(k_rows_to_user<double>, dim3(grid_for(m.N)), dim3(256), 0, st, m.N, w, m.perm, (const double *)fv, (double *)user);
    return hipGetLastError();
}
hipError_t launch_fv_from_user(const DeviceMesh &m, bool fp32, const void *user, void *fv, hipStream_t st) {
    const int w = 3 * m.tab.Nq * m.nv;
    if (fp32) hipLaunchKernelGGL(k_rows_from_user<float>, dim3(grid_for(m.N)), dim3(256), 0, st, m.N, w, m.perm, (const float *)user, (float *)fv);
    else hipLaunchKernelGGL(k_rows_from_user<double>, dim3(grid_for(m.N)), dim3(256), 0, st, m.N, w, m.perm, (const double *)user, (double *)fv);
    return hipGetLastError();
}
hipError_t launch_flux_to_user(const DeviceMesh &m, bool fp32, const void *fo, void *user, hipStream_t st) {
    const int w = 3 * m.nv;
    if (fp32) hipLaunchKernelGGL(k_rows_to_user<float>, dim3(grid_for(m.N)), dim3(256), 0, st, m.N, w, m.perm, (const float *)fo, (float *)user);
    else hipLaunchKernelGGL(k_rows_to_user<double>, dim3(grid_for(m.N)), dim3(256), 0, st, m.N, w, m.perm, (const double *)fo, (double *)user);
    return hipGetLastError();
}
hipError_t launch_delta_to_user(const DeviceMesh &m, const uint8_t *d, uint8_t *user, hipStream_t st) {
    hipLaunchKernelGGL(k_rows_to_user<uint8_t>, dim3(grid_for(m.N)), dim3(256), 0, st, m.N, m.delta_bytes(), m.perm, d,
                       user);
    return hipGetLastError();
}
hipError_t launch_delta_from_user(const DeviceMesh &m, const uint8_t *user, uint8_t *d, hipStream_t st) {
    hipLaunchKernelGGL(k_rows_from_user<uint8_t>, dim3(grid_for(m.N)), dim3(256), 0, st, m.N, m.delta_bytes(), m.perm,
                       user, d);
    return hipGetLastError();
}

__global__ void k_count_diff(int64_t n, const uint8_t *a, const uint8_t *b, unsigned long long *count) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c = (k < n && a[k] != b[k]) ? 1ull : 0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}
hipError_t launch_count_diff(const DeviceMesh &m, const uint8_t *a, const uint8_t *b, unsigned long long *count,
                             hipStream_t st) {
    const int64_t n = m.N * m.delta_bytes();
    hipLaunchKernelGGL(k_count_diff, dim3(grid_for(n)), dim3(256), 0, st, n, a, b, count);
    return hipGetLastError();
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, size_t n) {
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for((int64_t)n)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

__global__ void k_copy16(uint4 *dst, const uint4 *src, size_t n) {
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        dst[k] = src[k];
}
hipError_t launch_copy16(void *dst, const void *src, size_t n16, hipStream_t st) {
    unsigned grid = (unsigned)std::min<size_t>((n16 + 255) / 256, 256 * 64);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, st, (uint4 *)dst, (const uint4 *)src, n16);
    return hipGetLastError();
}

// ===========================================================================
// fixed device scratch of the allocation-free entry point
// ===========================================================================

// One static buffer per device for callers that cannot allocate device
// memory (cteno_flux_noalloc): the internal-order face-point values, face
// fluxes and the non-physical flag of one call.  Host code must use the
// address that hipGetSymbolAddress returns for the device, never the
// array's name, which on the host is only a stand-in.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;     // the device must be current
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

void *scratch_device_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

__global__ void k_gather_entries(int n, const int32_t *idx, int E, int VW, const double *s64, const float *s32,
                                 const int32_t *si, double *dst, int ct) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * E) return;
    const int a = (int)(t / E), e = (int)(t % E);
    const size_t src = ct == 64 ? avix(idx[a], e, E, VW) : hvix(idx[a], e, E, VW, ct);
    dst[t] = s64 ? s64[src] : (s32 ? (double)s32[src] : (double)si[src]);
}
hipError_t launch_gather_entries(int n, const int32_t *idx, int E, int VW, const double *src64, const float *src32,
                                 const int32_t *srci, double *dst, hipStream_t st, int ct) {
    hipLaunchKernelGGL(k_gather_entries, dim3(grid_for((int64_t)n * E)), dim3(256), 0, st, n, idx, E, VW, src64,
                       src32, srci, dst, ct);
    return hipGetLastError();
}

}  // namespace cteno
