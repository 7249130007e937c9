// Kernel launchers of the CTENO/CTENOZ library, implemented in k_precompute.hip
// (pseudo-inverses), k_recon_*.hip (reconstruction, per degree range and
// arithmetic type) and k_flux.hip (fluxes, RK stages, step control, serving
// batches, utilities); kernels_common.h holds the shared device code.
//
// HIP kernels (gfx950) of the CTENO/CTENOZ finite-volume hot path.
//
//   k_precompute   once per mesh, FP64: reference-space moments of every
//                  stencil cell (sec. 2.1), Householder QR of the M x K
//                  least-squares matrix and the pseudo-inverse
//                  P = R^-1 Q^T diag(|V'_m|), for the central stencil and
//                  the three directional stencils; FP32 copies on request.
//   k_reconstruct  per cell and stage: gather of neighbour averages, central
//                  and directional products P d, p_1 (eq. e17), smoothness
//                  indicators, CTENO (Algorithm 1) / CTENOZ (Algorithm 2)
//                  selection, final polynomial at the face Gauss points.
//   k_flux         per cell and stage: HLLC (sec. 2.6) or upwind flux at the
//                  Gauss points of its three faces, the residual of the
//                  semi-discrete form after eq. e1, and the SSP-RK3 stage;
//                  each interior face flux is evaluated identically by both
//                  of its cells (same operands, same order) so the update is
//                  conservative to FP64 round-off without atomics.
//   k_control      per RK step, one thread: time step from the reduced CFL
//                  bound, clipping to t_final, termination.
//
// Memory layout: per-cell static data (stencil slots, pseudo-inverses,
// face geometry) in 64-cell tiles, entry-major inside a tile, so a wave
// streams each entry as one contiguous 256/512-byte segment; the state and
// the face-point values are cell-major (array of structures) so a gather of
// one neighbour touches one cache line.
#pragma once

#include "cteno_internal.h"

namespace cteno {

struct DeviceMesh {
    int64_t N = 0, Np = 0;
    int r = 0, K = 0, S = 0, SP = 0, nv = 0, physics = 0;
    int scheme = 0, gamma_form = 0, precision = 0;
    int positivity = 0;            // 1: cell-average fallback for non-physical face states
    int vars = 0;                  // CTENO_VARS_CONSERVED | CTENO_VARS_CHARACTERISTIC
    int E64 = 0, E32 = 0;          // pseudo-inverse entries per cell (padded to the vector width)
    int Kd = 0, Md = 0, Nq = 2;    // directional basis size and members, Gauss points per face
    int stile = 64;                // cells per stream tile (r >= 4: 64 / nv)
    double gamma = 1.4, ax = 0, ay = 0, lam1p = 1e4, ct = 1e-6, eps = 1e-12;
    double Lx = 0, Ly = 0;
    int32_t *slot = nullptr;       // vector-tiled [SP], VW 4
    uint8_t *flags = nullptr;      // [Np]
    double *fr64 = nullptr;        // face records, vector-tiled [12], VW 2
    float *fr32 = nullptr;         // face records, vector-tiled [12], VW 4
    double *area = nullptr;        // [Np]
    double *P64 = nullptr;         // pseudo-inverse stream, vector-tiled [E64], VW 2
    float *P32 = nullptr;          // pseudo-inverse stream, vector-tiled [E32], VW 4
    int32_t *perm = nullptr;       // internal -> user [N]
    double *bface = nullptr;       // [n_inflow][4]: first vertex and edge vector of each inflow face
    int64_t n_inflow = 0;
    double bst[2][4] = {};         // inflow states behind / ahead of the moving line
    double bline[3] = {};          // x = bline[0] + bline[1] y + bline[2] t
    double *htab64 = nullptr;      // r >= 4: Gram matrix [K][K] and face basis [3][Nq][K], FP64
    float *htab32 = nullptr;       // the same in FP32
    RefTables tab;
    // fused stage (degree <= 3): cells with a face whose neighbour lies in
    // another 256-cell block ("cross cells"), ascending; per cross cell (in
    // that order) the cross index of the neighbour across each face, -1
    // where the face stays in the block or is a boundary, its area and its
    // face records (tiled like fr32 / fr64); per block the number of cross
    // cells in the blocks before it
    int32_t *xcells = nullptr;
    int64_t n_cross = 0;
    int32_t *xbase = nullptr;      // [blocks() + 1]
    int32_t *xnb = nullptr;        // [n_cross][3]
    double *xarea = nullptr;       // [n_cross]
    float *xfr32 = nullptr;        // [pad64(n_cross)][12], VW 4
    double *xfr64 = nullptr;       // [pad64(n_cross)][12], VW 2
    bool fused = false;            // the march runs the fused stage kernels
    int64_t blocks() const { return (N + 255) / 256; }
    int64_t cross_blocks() const { return (n_cross + 255) / 256; }
    // per-block CFL minima of one march step: both stage kernels' blocks
    int64_t dt_parts() const { return blocks() + (fused ? cross_blocks() : 0); }
    // selection bytes per cell: per variable, or per face and characteristic field
    int delta_bytes() const { return vars == CTENO_VARS_CHARACTERISTIC ? 3 * nv : nv; }
};

struct PrecomputeInputs {
    const double *verts;          // tiled [6]
    const uint8_t *slot_flag;     // tiled [S]
    const int8_t *slot_shift;     // tiled [2S]
    uint8_t *flags;               // [Np] in/out: inadmissible-by-rank bits cleared
    int *rank_fail;               // device counter of rank-deficient central systems
};

hipError_t launch_precompute(const DeviceMesh &m, const PrecomputeInputs &in, hipStream_t st);

// reconstruction of degree 2-3 (reconstruct_lo) and 4-6 (reconstruct_hi) in
// arithmetic `real` (float: mixed precision; double: FP64); instantiated in
// k_recon_f32/f64.hip and k_recon_ho_f32/f64.hip
template <typename real>
hipError_t reconstruct_lo(const DeviceMesh &m, const double *U, void *FV, uint8_t *delta, int dmode, const int *done,
                          hipStream_t st, unsigned long long *fb_count);
template <typename real>
hipError_t reconstruct_hi(const DeviceMesh &m, const double *U, void *FV, uint8_t *delta, int dmode, const int *done,
                          hipStream_t st, unsigned long long *fb_count);

// reconstruction; dmode: 0 none, 1 write delta, 2 forced delta
// fb_count (may be null) counts the cells that take the positivity fallback
hipError_t launch_reconstruct(const DeviceMesh &m, bool fp32, const double *U, void *FV, uint8_t *delta, int dmode,
                              const int *done, hipStream_t st, unsigned long long *fb_count = nullptr);

// flux / residual / RK stage.  mode: 0 outward face fluxes, 1 residual, 2 RK stage
struct FluxLaunch {
    int mode = 2;
    const void *FV = nullptr;
    const double *Un = nullptr, *Us = nullptr;
    double *Uout = nullptr;
    int stage = 0;
    const double *dt_ptr = nullptr;
    double dt_value = 0.0;
    void *flux_out = nullptr;    // AoS [Np][3][nv] of the precision type
    double *resid = nullptr;     // AoS [Np][nv]
    Ctrl *ctrl = nullptr;        // done / nonphysical (may be null); with dt_ptr also the march time
    int *nonphys = nullptr;      // non-physical flag when ctrl is null (may be null)
    double *dt_part = nullptr;   // per-block minima of the CFL bound (stage 2 of a march), or null
    double t_base = 0.0;         // time of the stage input when the march time is not on the device
    // fused stage: [n_cross][nv] stage states of the cross cells from their
    // faces inside the block (the faces to other blocks still to add)
    double *xpart = nullptr;
};
hipError_t launch_flux(const DeviceMesh &m, bool fp32, const FluxLaunch &f, hipStream_t st);

// Fused SSP-RK3 stage of degree <= 3 (f.mode 2): part 0 reconstructs each
// 256-cell block into LDS, evaluates the faces inside the block and updates
// the cells whose faces all lie inside it; the others store the values of
// their faces to other blocks (f.FV, by cross index) and their partial stage
// states (f.xpart), and part 1 finishes them with the faces to other
// blocks.  The two parts are launched in order, 0 then 1.
hipError_t launch_stage(const DeviceMesh &m, bool fp32, const FluxLaunch &f, const int *done, int part,
                        hipStream_t st, unsigned long long *fb_count);
template <typename real>
hipError_t stage_fused(const DeviceMesh &m, const FluxLaunch &f, const int *done, int part, hipStream_t st,
                       unsigned long long *fb_count);     // k_stage_f32.hip, k_stage_f64.hip

// per-block minima of the CFL bound of state U into dt_part[blocks()], from the
// face records of the stage kernels' precision (fp32) so a march's first step
// uses the same geometry as its later steps
hipError_t launch_dt_partials(const DeviceMesh &m, bool fp32, const double *U, double *dt_part, hipStream_t st);
// step control; reduces dt_part[n_part] unless commit_only
hipError_t launch_control(Ctrl *ctrl, const double *dt_part, int64_t n_part, int commit_only, hipStream_t st);

// device descriptor of one active serving slot (one independent solve)
struct BatchSlot {
    int64_t N, block0, nblocks;     // cells; first global block; blocks of 256 cells
    const int32_t *slot;
    const uint8_t *flags;
    const float *P;                 // FP32 pseudo-inverse stream
    const float *fr;                // FP32 face records
    const double *area;
    double *U[3];                   // U^n, U^(1), U^(2)
    float *FV;
    double *dt_part;                // [nblocks]
    Ctrl *ctrl;
};
// one SSP-RK3 step (control + 3 x (reconstruction, flux/RK)) of every slot in
// tab[0 .. *n_slots); grids of max_slots and max_blocks blocks (blocks past the
// active range exit at once).  FP32 reconstruction/flux, Euler, r = 2 or 3.
hipError_t launch_batch_step(const DeviceMesh &proto, const BatchSlot *tab, const int *n_slots, int max_slots,
                             int64_t max_blocks, hipStream_t st);

// layout conversions between caller order/layout and internal order/layout
hipError_t launch_user_to_state(const DeviceMesh &m, const double *user, double *state, hipStream_t st);
hipError_t launch_state_to_user(const DeviceMesh &m, const double *state, double *user, hipStream_t st);
hipError_t launch_fv_to_user(const DeviceMesh &m, bool fp32, const void *fv, void *user, hipStream_t st);
hipError_t launch_fv_from_user(const DeviceMesh &m, bool fp32, const void *user, void *fv, hipStream_t st);
hipError_t launch_flux_to_user(const DeviceMesh &m, bool fp32, const void *fo, void *user, hipStream_t st);
hipError_t launch_delta_to_user(const DeviceMesh &m, const uint8_t *d, uint8_t *user, hipStream_t st);
hipError_t launch_delta_from_user(const DeviceMesh &m, const uint8_t *user, uint8_t *d, hipStream_t st);
hipError_t launch_count_diff(const DeviceMesh &m, const uint8_t *a, const uint8_t *b, unsigned long long *count,
                             hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, size_t n, hipStream_t st);

// Fixed device scratch of the allocation-free entry point (one array per
// device, held until the process ends).  scratch_init records its device
// address for `device`, which must be the current device; it is called
// once per device by cteno_ctx_create.  scratch_device_ptr returns the
// recorded address, or null before scratch_init succeeded on that device.
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
hipError_t scratch_init(int device);
void *scratch_device_ptr(int device);
hipError_t launch_copy16(void *dst, const void *src, size_t n16, hipStream_t st);
// dst[a][e] = src[avix(idx[a], e, E, VW)] (ct = 64) or src[hvix(idx[a], e, E, VW, ct)]
// from exactly one of src64 / src32 / srci
hipError_t launch_gather_entries(int n, const int32_t *idx, int E, int VW, const double *src64, const float *src32,
                                 const int32_t *srci, double *dst, hipStream_t st, int ct = 64);

}  // namespace cteno
