// Internal declarations of the CTENO/CTENOZ MI355X library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <utility>
#include <string>
#include <vector>

#include "../../include/cteno.h"

namespace cteno {

// ---------------------------------------------------------------------------
// sizes
// ---------------------------------------------------------------------------
constexpr int kTile = 64;          // cells per tile of the tiled per-cell arrays (one wave)
constexpr int kNq = 2;             // Gauss points per face for degree <= 3
constexpr int kMaxR = 6;
constexpr int kMaxK = 27;          // K at degree 6
constexpr int kMaxS = 54;          // slots at degree 6
constexpr int kMaxNq = 4;          // Gauss points per face at degree 6
constexpr int kDirSlots = 4;       // M_d = 2 K_d with K_d = 2 (degree-1 directional, r <= 3)

inline int dims_K(int r) { return (r + 1) * (r + 2) / 2 - 1; }
inline int dims_M(int r) { return 2 * dims_K(r); }
// directional degree: 1 up to cubic, ceil(r/2) above (third-order directional
// stencils for the fifth-order scheme)
inline int dims_rd(int r) { return r <= 3 ? 1 : (r + 1) / 2; }
inline int dims_Kd(int r) { return dims_K(dims_rd(r)); }
inline int dims_Md(int r) { return 2 * dims_Kd(r); }
// Slots of a cell's stream.  Up to cubic (and at degree 6, where
// 3 M_d = M): the three directional groups of M_d slots first (a group's
// members, then other central cells or pads), then the rest of the central
// stencil.  At degrees 4 and 5 (M < 3 M_d; the directional stencils, subsets
// of the central one, hold at most M cells together): exactly the M central
// cells, the members of the three directional stencils first, one stencil
// after the other, then the central cells of no directional stencil.
inline bool ho_var_groups(int r) { return r >= 4 && dims_M(r) < 3 * dims_Md(r); }
inline int dims_S(int r) {
    if (ho_var_groups(r)) return dims_M(r);
    return dims_M(r) > 3 * dims_Md(r) ? dims_M(r) : 3 * dims_Md(r);
}
inline int dims_Nq(int r) { return (r + 2) / 2; }
// r >= 4: every slot carries K central and K_d directional entries, padded
// to a multiple of 4 so each slot is a whole number of 16-byte vectors
inline int ho_slot_entries(int r) { return (dims_K(r) + dims_Kd(r) + 3) / 4 * 4; }

// tiled index: per-cell array with E entries, 64-cell tiles, entry-major inside a tile
__host__ __device__ inline size_t tix(int64_t i, int e, int E) {
    return ((size_t)(i >> 6) * E + e) * kTile + (i & 63);
}
// vector-tiled index (array of structures of arrays): entries are grouped in
// vectors of VW consecutive entries per cell, vectors tiled like tix; a lane
// reads VW entries with one 16-byte load and a wave reads 1 KiB contiguously.
// E must be a multiple of VW.  Returns the scalar index of entry e.
__host__ __device__ inline size_t avix(int64_t i, int e, int E, int VW) {
    return ((((size_t)(i >> 6) * (E / VW) + e / VW) * kTile + (i & 63)) * VW) + (e % VW);
}
inline int64_t pad64(int64_t n) { return (n + kTile - 1) / kTile * kTile; }
inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

// pseudo-inverse stream of one cell, consumed slot by slot: for slot j the K
// central entries P_c[k][j], then (j < 12) the two directional entries
// P_d[j/4][c][j%4]
__host__ __device__ constexpr int pinv_offset(int j, int K) {
    return j <= 12 ? j * (K + 2) : 12 * (K + 2) + (j - 12) * K;
}
inline int pinv_entries(int r) {
    return r <= 3 ? pinv_offset(dims_S(r), dims_K(r)) : dims_S(r) * ho_slot_entries(r);
}
// r >= 4: vector-tiled stream with tiles of CT cells (CT = 64 / nv: one lane
// per cell and variable), VW = 4 (FP32) or 2 (FP64) entries per vector
__host__ __device__ inline size_t hvix(int64_t i, int e, int E, int VW, int CT) {
    return ((((size_t)(i / CT) * (E / VW) + e / VW) * CT + (i % CT)) * VW) + (e % VW);
}

// neighbour code per cell face: bit 31 set = boundary (bits 0..1 = kind),
// else bits 0..27 neighbour (internal index), 28..29 neighbour's local
// face, bit 30 = this cell owns the face
constexpr uint32_t kNbBoundary = 0x80000000u;
constexpr uint32_t kNbOwner = 0x40000000u;
constexpr uint32_t kNbIndexMask = 0x0FFFFFFFu;
// boundary faces: kind in bits 0-1; an inflow face's row in the inflow table in bits 2-29
constexpr uint32_t kNbInflowMask = 0x0FFFFFFFu;
// slot entries at degree >= 4: bits 0..27 the cell (internal index), bits
// 28..29 the directional stencil (face 0..2) that holds it, 3 for none
constexpr uint32_t kSlotIndexMask = 0x0FFFFFFFu;
constexpr int kSlotGroupShift = 28;
constexpr uint32_t kSlotNoGroup = 3u;

// allocator whose new elements are left uninitialised (default-initialised):
// for arrays that the parallel mesh layout writes in full, so that no serial
// zero fill runs first
template <typename T>
struct NoInitAlloc : std::allocator<T> {
    template <typename U> struct rebind { using other = NoInitAlloc<U>; };
    NoInitAlloc() = default;
    template <typename U> NoInitAlloc(const NoInitAlloc<U> &) noexcept {}
    template <typename U> void construct(U *p) noexcept { ::new (static_cast<void *>(p)) U; }
    template <typename U, typename... A> void construct(U *p, A &&...a) {
        ::new (static_cast<void *>(p)) U(std::forward<A>(a)...);
    }
};
template <typename T> using raw_vector = std::vector<T, NoInitAlloc<T>>;

// ---------------------------------------------------------------------------
// host mesh builder output (all in internal order unless noted)
// ---------------------------------------------------------------------------
struct HostMesh {
    int N = 0, r = 0, K = 0, M = 0, S = 0, nv = 0, Kd = 0, Md = 0, Nq = 0;
    int per_x = 0, per_y = 0;
    double Lx = 0, Ly = 0;
    int64_t n_faces = 0, n_boundary = 0;
    int n_inadmissible = 0;
    std::vector<int32_t> perm;     // internal -> user
    std::vector<int32_t> iperm;    // user -> internal
    // user-order stencils (for inspection)
    std::vector<int32_t> cen_user;     // [N][M] ascending user ids
    std::vector<int32_t> dir_user;     // [N][3][Md] user ids, -1 padded
    std::vector<int32_t> dirn_user;    // [N][3]
    // internal-order device inputs
    int SP = 0;                        // slots padded to a multiple of 4
    raw_vector<int32_t> slot;          // vector-tiled [SP] (VW 4): internal cell index (self for pads)
    raw_vector<uint8_t> slot_flag;     // tiled [S]: bit0 central member, bit1 directional member
    raw_vector<int8_t> slot_shift;     // tiled [2*S]: periodic image shift (x then y)
    raw_vector<uint8_t> flags;         // [Npad]: bit s = directional stencil of face s admissible
    raw_vector<double> verts;          // tiled [6]: CCW vertex coordinates x0,y0,x1,y1,x2,y2
    // face records: per local face (nx, ny, |A|, neighbour code), vector-tiled
    raw_vector<double> fr64;           // [12] entries, VW 2; code stored in the low bits of the double
    raw_vector<float> fr32;            // [12] entries, VW 4; code stored as the float's bits
    raw_vector<double> area;           // [Npad]
    // inflow faces: first vertex (x, y) and edge vector, rows in internal cell order
    std::vector<double> bface;         // [n_inflow][4]
    double bst[2][4] = {};             // prescribed states behind / ahead of the moving line
    double bline[3] = {};              // x = bline[0] + bline[1] y + bline[2] t
};

// host threads the calling thread's mesh builds may use (default 16)
void set_builder_threads(int n);
// returns CTENO_OK or an error (message in err)
cteno_status build_host_mesh(const cteno_mesh_desc &d, const cteno_scheme &s, HostMesh &hm, std::string &err);

// ---------------------------------------------------------------------------
// constant tables of the reference triangle (host-computed, FP64)
// ---------------------------------------------------------------------------
struct RefTables {
    int K = 0, Nq = 0;
    int ex[kMaxK][2];               // exponents of psi_k
    double mean[kMaxK];             // mean of psi_k over the reference triangle
    double gram[kMaxK][kMaxK];      // smoothness-indicator Gram matrix
    double basis[3][kMaxNq][kMaxK]; // phi_k at the face Gauss points
    double gq[kMaxNq], gw[kMaxNq];  // Gauss points and weights on [0, 1]
};
void make_ref_tables(int r, RefTables &t);

// ---------------------------------------------------------------------------
// device-side control block of a time march
// ---------------------------------------------------------------------------
struct Ctrl {
    double t, t_next, t_final, dt, cfl;
    unsigned long long dt_cand_bits;   // min over cells of the dt bound (bits of a positive double)
    long long step, max_steps;
    int done, pending, nonphysical, pad;
    unsigned long long fallbacks;      // cells x stages that took the positivity fallback
};

}  // namespace cteno
