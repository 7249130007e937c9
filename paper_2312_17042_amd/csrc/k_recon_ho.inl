// Reconstruction of degree 4 to 6 (orders 5 to 7; a quad of lanes per Euler
// cell, a lane per cell for advection) for one arithmetic type;
// instantiated per type by k_recon_ho_f32.hip and k_recon_ho_f64.hip.
#pragma once
#include "kernels_common.h"

namespace cteno {

template <typename real>
struct ReconHoArgs {
    int64_t N;
    const double *U;
    const int32_t *slot;
    const uint8_t *flags;
    const real *P;
    real *FV;                // AoS [Np][3][N_q][nv]
    uint8_t *delta;
    const int *done;
    const real *tab;
    const real *fr;          // face records (characteristic variables)
    real lams[5], lam_ratio[5];
    real lam1, ct, eps, gamma;
    int positivity;          // 1: cell-average fallback for non-physical face states
    unsigned long long *fb_count;   // cells that took the fallback (may be null)
    // the p_1 step's factors: (p_opt - p1_ls sum_s lambda_s p_s) / p1_l1,
    // (1, lambda_1) for the CTENO family, (0, 1) for TENO, which keeps p_opt
    real p1_ls, p1_l1;
};

// one lane's field (a conserved variable, or a characteristic field on one
// face): selection or CWENO weights and the final coefficients, in place in
// c1[K] (p_1 on entry); cd[3][K_d] the directional coefficients
template <typename real, int K, int KD, int SCHEME, int GFORM, int DMODE>
__device__ __forceinline__ int finish_field_ho(const ReconHoArgs<real> a, real (&c1)[K], const real (&cd)[3][KD],
                                               int fl, int adm, int st, real lams, real lratio, int forced) {
    int bits;
    if (DMODE == 2 && SCHEME != CTENO_SCHEME_CWENO) {
        bits = forced & adm;
    } else if (st == 1) {
        bits = 1;
    } else {
        real si[4];
        si[0] = 0;
#pragma unroll
        for (int p = 0; p < K; ++p) {
            real rp = 0;
#pragma unroll
            for (int q = 0; q < K; ++q) rp += a.tab[p * K + q] * c1[q];
            si[0] += c1[p] * rp;
        }
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            real sv = 0;
#pragma unroll
            for (int p = 0; p < KD; ++p) {
                real rp = 0;
#pragma unroll
                for (int q = 0; q < KD; ++q) rp += a.tab[p * K + q] * cd[s][q];
                sv += cd[s][p] * rp;
            }
            si[s + 1] = sv;
        }
        if constexpr (SCHEME == CTENO_SCHEME_CWENO) {
            // every admissible stencil contributes: sum_s omega_s p_s, in place
            bits = adm;
            real w[4];
            cweno_weights<real>(si, adm, lams, a.lam1, lratio, a.eps, w);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                real x = w[0] * c1[k];
                if (k < KD) {
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        if ((fl >> q) & 1) x += w[q + 1] * cd[q][k];
                }
                c1[k] = x;
            }
        } else {
            constexpr int SEL = SCHEME == CTENO_SCHEME_TENO ? CTENO_SCHEME_CTENO : SCHEME;
            constexpr int SGF = SCHEME == CTENO_SCHEME_TENO ? CTENO_GAMMA_PAPER : GFORM;
            bits = teno_bits<real, SEL, SGF>(si, adm, st, a.lam1, lams, lratio, a.ct, a.eps);
        }
    }
    // final coefficients: p_1, or the mean of the selected directional polynomials
    if (SCHEME != CTENO_SCHEME_CWENO && !(bits & 1)) {
        int cnt = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) c1[k] = 0;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            if ((bits >> (q + 1)) & 1) {
                ++cnt;
#pragma unroll
                for (int k = 0; k < KD; ++k) c1[k] += cd[q][k];
            }
#pragma unroll
        for (int k = 0; k < KD; ++k) c1[k] = fdiv(c1[k], (real)cnt);
    }
    return bits;
}

// value of x in lane u of each group of four lanes (a quad), by a DPP move
template <int u>
__device__ __forceinline__ float quad_bcast(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), u * 0x55, 0xF, 0xF, false));
}
template <int u>
__device__ __forceinline__ double quad_bcast(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xFFFFFFFFll), u * 0x55, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), u * 0x55, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
// the value that lane `owner` of the quad holds in x[v] for the calling lane's v
template <typename real, int owner>
__device__ __forceinline__ real quad_take(const real (&x)[4], int v) {
    const real x0 = quad_bcast<owner>(x[0]), x1 = quad_bcast<owner>(x[1]);
    const real x2 = quad_bcast<owner>(x[2]), x3 = quad_bcast<owner>(x[3]);
    return v == 0 ? x0 : v == 1 ? x1 : v == 2 ? x2 : x3;
}

// Coefficient e of the slot stream is accumulated by lane (e / VW) % 4 of
// the quad, in its round (e / VW) / 4, component e % VW, for the GF full
// rounds of four vectors; the four entries past them (the spread tail) by
// lane e - 4 GF VW.  These hand coefficients e0, e0 + 1, ... to the variable
// lanes.
template <typename real, int VW, int GF, int e>
__device__ __forceinline__ real ho_take1(const real (&acc)[GF][VW][4], const real (&acs)[4], int v) {
    if constexpr (e < 4 * GF * VW) return quad_take<real, (e / VW) % 4>(acc[e / VW / 4][e % VW], v);
    else return quad_take<real, e - 4 * GF * VW>(acs, v);
}

template <typename real, int VW, int GF, int e0, int n, int... k>
__device__ __forceinline__ void ho_take(const real (&acc)[GF][VW][4], const real (&acs)[4], int v, real (&out)[n],
                                        std::integer_sequence<int, k...>) {
    ((out[k] = ho_take1<real, VW, GF, e0 + k>(acc, acs, v)), ...);
}

// an empty asm statement that takes x and gives it back, so that x is
// computed here (not volatile: a volatile statement would count as a
// possible store and turn the uniform table loads after it into vector loads)
template <typename T>
__device__ __forceinline__ void opaque(T &x) { asm("" : "+v"(x)); }

// whether some lane of a quad holds a directional entry (e in [K, K + K_d))
// at component c of its vector in round t
template <int K, int KD, int VW>
constexpr bool ho_dir_any(int t, int c) {
    for (int u = 0; u < 4; ++u) {
        const int e = (4 * t + u) * VW + c;
        if (e >= K && e < K + KD) return true;
    }
    return false;
}

// a_opt = P_c d and a_s = P_s d for the four variables of a cell held by a
// quad of lanes.  The lanes split each slot's stream instead of each reading
// all of it: lane q loads the stream vectors q, q + 4, ... and accumulates
// their coefficients for all four variables (the differences d come from
// the variable lanes by DPP moves); the coefficients go to their variable
// lanes at the end (and, with fixed groups of M_d slots, at the end of each
// group).  Every coefficient sums its slots in slot order, as a lane per
// variable would.  With variable groups (degrees 4 and 5), where a slot's
// directional stencil comes with its index, the positions that hold a
// directional entry in some lane keep three sums, one per stencil: a
// directional entry enters the sum of its slot's stencil only, a central
// entry enters the first sum at every slot.
// Where the slot ends in a partial round of four scalars (r = 4 and 6: one
// float4 or two double2 vectors), lane q reads scalar q of it, so no lane
// multiplies a vector it does not own.
template <typename real, int R>
__device__ __forceinline__ void ho_contract_quad(const ReconHoArgs<real> a, int64_t i, int v, double U0,
                                                 real (&ao)[HoDims<R>::K], real (&ad)[3][HoDims<R>::KD]) {
    using D = HoDims<R>;
    constexpr int K = D::K, KD = D::KD, MD = D::MD, S = D::S, SP = D::SP, EPS = D::EPS, E = D::E;
    constexpr bool VARG = D::VARG;
    constexpr int CT = 16;
    using V = typename Vec<real>::T;
    constexpr int VW = Vec<real>::W;
    constexpr int SV = EPS / VW;          // stream vectors per slot
    constexpr int GF = SV / 4;            // full rounds of four vectors
    constexpr bool SPREAD = SV % 4 != 0;  // a tail of four scalars follows
    static_assert(!SPREAD || (SV % 4) * VW == 4, "a partial round must hold four scalars");
    const V *__restrict__ Pv = reinterpret_cast<const V *>(a.P) + (size_t)(i / CT) * (E / VW) * CT + (i % CT);
    // this lane's tail scalar of slot j: Pr[j * SV * CT * VW]
    const real *__restrict__ Pr =
        reinterpret_cast<const real *>(Pv) + ((4 * GF + v / VW) * CT) * VW + v % VW;
    const int32_t *__restrict__ Si = a.slot + (size_t)(i >> 6) * (SP / 4) * 256 + (i & 63) * 4;
    // acc: central sums and (fixed groups) the current group's directional
    // sums, or (variable groups) those of stencil 0; ag[0], ag[1]: those of
    // stencils 1 and 2 (variable groups, directional positions only)
    real acc[GF][VW][4], acs[4], ag[2][GF][VW][4], ags[2][4];
#pragma unroll
    for (int t = 0; t < GF; ++t)
#pragma unroll
        for (int c = 0; c < VW; ++c)
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[t][c][u] = ag[0][t][c][u] = ag[1][t][c][u] = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) acs[u] = ags[0][u] = ags[1][u] = 0;
    // this lane's entries that belong to a directional polynomial
    bool isdir[GF][VW];
#pragma unroll
    for (int t = 0; t < GF; ++t)
#pragma unroll
        for (int c = 0; c < VW; ++c) {
            const int e = (4 * t + v) * VW + c;
            isdir[t][c] = e >= K && e < K + KD;
        }
    const int es = 4 * GF * VW + v;
    const bool isdirs = es >= K && es < K + KD;
    constexpr bool DIRS = SPREAD && 4 * GF * VW + 3 >= K && 4 * GF * VW < K + KD;
    // Slot j's stream vectors and neighbour averages are requested when slot
    // j - 2 has been used and its entry when slot j - 4 has: the loop takes
    // the slots in pairs with a buffer per slot of the pair, so that no load
    // is waited for before its slot (a rotating buffer waits at the copy,
    // and the compiler had turned the earlier rotating version into loads
    // at the top of each slot, waited for at once).  The scheduling
    // barriers keep each pair's loads behind the slot that frees the buffer.
    static_assert(S % 2 == 0, "slots are taken in pairs (or one by one)");
    auto ld_stream = [&](int j, V (&b)[GF], real &bs) {
        const int jc = j < S ? j : S - 1;
#pragma unroll
        for (int t = 0; t < GF; ++t) b[t] = Pv[(jc * SV + 4 * t + v) * CT];
        if constexpr (SPREAD) bs = Pr[(size_t)jc * SV * CT * VW];
    };
    auto ld_entry = [&](int j) {
        const int jc = j < S ? j : S - 1;
        return (uint32_t)Si[(jc >> 2) * 256 + (jc & 3)];
    };
    const double *__restrict__ Ug = a.U;
    auto ld_avg = [Ug, v](uint32_t se) { return Ug[(int64_t)(se & kSlotIndexMask) * 4 + v]; };
    // one slot: differences of the quad's four variables, products with
    // this lane's stream vectors (b, bs), group sums (g: the slot's stencil)
    double uc = U0;                       // the cell's own average, loaded before the loop
    opaque(uc);                           // (pending at the loop it would cost a full wait per pair)
    auto slot_step = [&](const V (&b)[GF], real bs, double u, int g, int j) {
        const real dv = (real)(u - uc);
        const real d[4] = {quad_bcast<0>(dv), quad_bcast<1>(dv), quad_bcast<2>(dv), quad_bcast<3>(dv)};
#pragma unroll
        for (int t = 0; t < GF; ++t)
#pragma unroll
            for (int c = 0; c < VW; ++c) {
                const real p = comp(b[t], c);
                if (VARG && ho_dir_any<K, KD, VW>(t, c)) {
                    const real p0 = (isdir[t][c] && g != 0) ? (real)0 : p;
                    const real p1 = g == 1 ? p : (real)0, p2 = g == 2 ? p : (real)0;
#pragma unroll
                    for (int u4 = 0; u4 < 4; ++u4) {
                        acc[t][c][u4] += p0 * d[u4];
                        ag[0][t][c][u4] += p1 * d[u4];
                        ag[1][t][c][u4] += p2 * d[u4];
                    }
                } else {
#pragma unroll
                    for (int u4 = 0; u4 < 4; ++u4) acc[t][c][u4] += p * d[u4];
                }
            }
        if constexpr (SPREAD) {
            if constexpr (VARG && DIRS) {
                const real p0 = (isdirs && g != 0) ? (real)0 : bs;
                const real p1 = g == 1 ? bs : (real)0, p2 = g == 2 ? bs : (real)0;
#pragma unroll
                for (int u4 = 0; u4 < 4; ++u4) {
                    acs[u4] += p0 * d[u4];
                    ags[0][u4] += p1 * d[u4];
                    ags[1][u4] += p2 * d[u4];
                }
            } else {
#pragma unroll
                for (int u4 = 0; u4 < 4; ++u4) acs[u4] += bs * d[u4];
            }
        }
        if (!VARG && j % MD == MD - 1) {  // uniform: group j / MD is complete
            real x[KD];
            ho_take<real, VW, GF, K, KD>(acc, acs, v, x, std::make_integer_sequence<int, KD>{});
            const int s = j / MD;
            if (s == 0) {
#pragma unroll
                for (int k = 0; k < KD; ++k) ad[0][k] = x[k];
            } else if (s == 1) {
#pragma unroll
                for (int k = 0; k < KD; ++k) ad[1][k] = x[k];
            } else {
#pragma unroll
                for (int k = 0; k < KD; ++k) ad[2][k] = x[k];
            }
#pragma unroll
            for (int t = 0; t < GF; ++t)
#pragma unroll
                for (int c = 0; c < VW; ++c)
#pragma unroll
                    for (int u4 = 0; u4 < 4; ++u4) acc[t][c][u4] = isdir[t][c] ? (real)0 : acc[t][c][u4];
#pragma unroll
            for (int u4 = 0; u4 < 4; ++u4) acs[u4] = isdirs ? (real)0 : acs[u4];
        }
    };
    // FP64 at degree 6: one buffer (its second would cost a wave per SIMD)
    constexpr bool PAIRS = !(sizeof(real) == 8 && R == 6);
    V bA[GF], bB[GF];
    real sA = 0, sB = 0;
    ld_stream(0, bA, sA);
    uint32_t eA = ld_entry(0), eB = ld_entry(1);
    double uA = ld_avg(eA), uB = 0;
    int gA = (int)(eA >> kSlotGroupShift), gB = 0;
    if constexpr (PAIRS) {
        ld_stream(1, bB, sB);
        uB = ld_avg(eB);
        gB = (int)(eB >> kSlotGroupShift);
        eA = ld_entry(2);
        eB = ld_entry(3);
#pragma unroll 1
        for (int j = 0; j < S; j += 2) {
            slot_step(bA, sA, uA, gA, j);
            __builtin_amdgcn_sched_barrier(0);
            ld_stream(j + 2, bA, sA);
            gA = (int)(eA >> kSlotGroupShift);
            opaque(gA);                   // taken now: eA's register is free for the next entry
            uA = ld_avg(eA);
            eA = ld_entry(j + 4);
            __builtin_amdgcn_sched_barrier(0);
            slot_step(bB, sB, uB, gB, j + 1);
            __builtin_amdgcn_sched_barrier(0);
            ld_stream(j + 3, bB, sB);
            gB = (int)(eB >> kSlotGroupShift);
            opaque(gB);
            uB = ld_avg(eB);
            eB = ld_entry(j + 5);
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        eA = eB;
#pragma unroll 1
        for (int j = 0; j < S; ++j) {
            slot_step(bA, sA, uA, gA, j);
            __builtin_amdgcn_sched_barrier(0);
            ld_stream(j + 1, bA, sA);
            gA = (int)(eA >> kSlotGroupShift);
            opaque(gA);
            uA = ld_avg(eA);
            eA = ld_entry(j + 2);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if constexpr (VARG) {
        ho_take<real, VW, GF, K, KD>(acc, acs, v, ad[0], std::make_integer_sequence<int, KD>{});
        ho_take<real, VW, GF, K, KD>(ag[0], ags[0], v, ad[1], std::make_integer_sequence<int, KD>{});
        ho_take<real, VW, GF, K, KD>(ag[1], ags[1], v, ad[2], std::make_integer_sequence<int, KD>{});
    }
    ho_take<real, VW, GF, 0, K>(acc, acs, v, ao, std::make_integer_sequence<int, K>{});
}

template <typename real, int R, int NV, int SCHEME, int GFORM, int DMODE, int VARS>
__global__ __launch_bounds__(256) void k_reconstruct_ho(const ReconHoArgs<real> a) {
    using D = HoDims<R>;
    constexpr int K = D::K, KD = D::KD, MD = D::MD, S = D::S, SP = D::SP, EPS = D::EPS, E = D::E, NQ = D::NQ;
    constexpr int CT = 64 / NV;
    using V = typename Vec<real>::T;
    constexpr int VW = Vec<real>::W;
    constexpr int SV = EPS / VW;          // stream vectors per slot
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * (256 / NV) + threadIdx.x / NV;
    const int v = threadIdx.x % NV;
    if (i >= a.N) return;                 // all lanes of a cell leave together
    if (a.done && *a.done) return;
    const V *__restrict__ Pv = reinterpret_cast<const V *>(a.P) + (size_t)(i / CT) * (E / VW) * CT + (i % CT);
    const int32_t *__restrict__ Si = a.slot + (size_t)(i >> 6) * (SP / 4) * 256 + (i & 63) * 4;
    const double U0 = a.U[i * NV + v];

    real ao[K], ad[3][KD];
    if constexpr (NV == 4) {
        ho_contract_quad<real, R>(a, i, v, U0, ao, ad);
    } else {
    // a_opt = P_c d and a_s = P_s d, slot by slot (one lane per cell); the
    // next slot's stream vectors and entry are requested before the current
    // slot is used.  Variable groups: a slot's directional entries go to the
    // sums of the stencil its entry names
    real adt[KD];
#pragma unroll
    for (int k = 0; k < K; ++k) ao[k] = 0;
#pragma unroll
    for (int k = 0; k < KD; ++k) { adt[k] = 0; ad[0][k] = 0; ad[1][k] = 0; ad[2][k] = 0; }
    V cur[SV];
#pragma unroll
    for (int g = 0; g < SV; ++g) cur[g] = Pv[g * CT];
    uint32_t scur = (uint32_t)Si[0];
#pragma unroll 1
    for (int j = 0; j < S; ++j) {
        const int jn = j + 1 < S ? j + 1 : j;
        V nxt[SV];
#pragma unroll
        for (int g = 0; g < SV; ++g) nxt[g] = Pv[(jn * SV + g) * CT];
        const uint32_t sn = (uint32_t)Si[(jn >> 2) * 256 + (jn & 3)];
        const real d = (real)(a.U[(int64_t)(scur & kSlotIndexMask) * NV + v] - U0);
#pragma unroll
        for (int k = 0; k < K; ++k) ao[k] += comp(cur[k / VW], k % VW) * d;
        if constexpr (D::VARG) {
            const int gs = (int)(scur >> kSlotGroupShift);
            const real d0 = gs == 0 ? d : (real)0, d1 = gs == 1 ? d : (real)0, d2 = gs == 2 ? d : (real)0;
#pragma unroll
            for (int k = 0; k < KD; ++k) {
                const real p = comp(cur[(K + k) / VW], (K + k) % VW);
                ad[0][k] += p * d0;
                ad[1][k] += p * d1;
                ad[2][k] += p * d2;
            }
        } else {
#pragma unroll
            for (int k = 0; k < KD; ++k) adt[k] += comp(cur[(K + k) / VW], (K + k) % VW) * d;
            if (j % MD == MD - 1) {       // uniform: group j / MD is complete
                const int s = j / MD;
#pragma unroll
                for (int s2 = 0; s2 < 3; ++s2)
                    if (s2 == s)
#pragma unroll
                        for (int k = 0; k < KD; ++k) ad[s2][k] = adt[k];
#pragma unroll
                for (int k = 0; k < KD; ++k) adt[k] = 0;
            }
        }
#pragma unroll
        for (int g = 0; g < SV; ++g) cur[g] = nxt[g];
        scur = sn;
    }
    }

    const int fl = a.flags[i] & 7;
    const int adm = 1 | (fl << 1);
    const int st = 1 + __popc(fl);
    const real lams = st == 2 ? a.lams[2] : (st == 3 ? a.lams[3] : a.lams[4]);
    const real lratio = st == 2 ? a.lam_ratio[2] : (st == 3 ? a.lam_ratio[3] : a.lam_ratio[4]);
    // p_1 = (p_opt - sum_s lambda_s p_s) / lambda_1 (eq. e17), in place.
    // TENO keeps the central stencil's own polynomial: it runs the same step
    // with factors 0 and 1 from the arguments (exact: x - 0 y = x, x / 1 = x),
    // because without the step the compiler's schedule needs a third more
    // registers (110 instead of 81 VGPRs at r = 4, 187 instead of 145 at r = 6)
    {
        const real ls = lams * a.p1_ls, il1 = frcp(a.p1_l1);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            real sm = ao[k];
            if (k < KD && st > 1) {
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    if ((fl >> q) & 1) sm -= ls * ad[q][k];
            }
            ao[k] = st > 1 ? sm * il1 : sm;
        }
    }
    const real *Bt = a.tab + K * K;
    real out[3][NQ];
    constexpr int NB = VARS ? 3 : 1;              // selection bytes of this lane
    int dbyte[NB];
    if constexpr (VARS == 0) {
        dbyte[0] = finish_field_ho<real, K, KD, SCHEME, GFORM, DMODE>(a, ao, ad, fl, adm, st, lams, lratio,
                                                                      DMODE == 2 ? a.delta[i * NV + v] : 0);
        // face Gauss-point values
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                real val = 0;
#pragma unroll
                for (int k = 0; k < K; ++k) val += Bt[(f * NQ + q) * K + k] * ao[k];
                out[f][q] = (real)(U0 + (double)val);
            }
    } else {
        // characteristic fields per face, lane v reconstructs field v: the
        // coefficients are projected with row v of L_f using the cell's
        // other lanes, the face values come back through row v of R_f
        static_assert(NV == 4, "characteristic variables need the Euler equations");
        const int l0 = (threadIdx.x & 63) & ~3;
        const double Ud[4] = {__shfl(U0, l0, 64), __shfl(U0, l0 + 1, 64), __shfl(U0, l0 + 2, 64),
                              __shfl(U0, l0 + 3, 64)};
        const real rho = (real)Ud[0], uu = (real)(Ud[1] / Ud[0]), vv = (real)(Ud[2] / Ud[0]);
        const real q2 = (real)0.5 * (uu * uu + vv * vv);
        const real pr = (a.gamma - 1) * ((real)Ud[3] - rho * q2);
        const real cs = fsqrt(fdiv(a.gamma * pr, rho)), H = fdiv((real)Ud[3] + pr, rho);
        const real b1 = fdiv(a.gamma - 1, cs * cs), b2 = b1 * q2, ic = frcp(cs);
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            real nx, ny, len;
            uint32_t code;
            face_record<real>(a.fr, i, f, nx, ny, len, code);
            const real un = uu * nx + vv * ny, ut = -uu * ny + vv * nx;
            real Lr[4], Rr[4];      // row v of L_f and of R_f
            if (v == 0) {
                Lr[0] = (real)0.5 * (b2 + un * ic); Lr[1] = (real)-0.5 * (b1 * uu + nx * ic);
                Lr[2] = (real)-0.5 * (b1 * vv + ny * ic); Lr[3] = (real)0.5 * b1;
                Rr[0] = 1; Rr[1] = 1; Rr[2] = 0; Rr[3] = 1;
            } else if (v == 1) {
                Lr[0] = 1 - b2; Lr[1] = b1 * uu; Lr[2] = b1 * vv; Lr[3] = -b1;
                Rr[0] = uu - cs * nx; Rr[1] = uu; Rr[2] = -ny; Rr[3] = uu + cs * nx;
            } else if (v == 2) {
                Lr[0] = -ut; Lr[1] = -ny; Lr[2] = nx; Lr[3] = 0;
                Rr[0] = vv - cs * ny; Rr[1] = vv; Rr[2] = nx; Rr[3] = vv + cs * ny;
            } else {
                Lr[0] = (real)0.5 * (b2 - un * ic); Lr[1] = (real)-0.5 * (b1 * uu - nx * ic);
                Lr[2] = (real)-0.5 * (b1 * vv - ny * ic); Lr[3] = (real)0.5 * b1;
                Rr[0] = H - un * cs; Rr[1] = q2; Rr[2] = ut; Rr[3] = H + un * cs;
            }
            real c1[K], cd[3][KD];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                real x = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) x += Lr[u] * __shfl(ao[k], l0 + u, 64);
                c1[k] = x;
            }
#pragma unroll
            for (int s2 = 0; s2 < 3; ++s2)
#pragma unroll
                for (int k = 0; k < KD; ++k) {
                    real x = 0;
#pragma unroll
                    for (int u = 0; u < 4; ++u) x += Lr[u] * __shfl(ad[s2][k], l0 + u, 64);
                    cd[s2][k] = x;
                }
            dbyte[f] = finish_field_ho<real, K, KD, SCHEME, GFORM, DMODE>(
                a, c1, cd, fl, adm, st, lams, lratio, DMODE == 2 ? a.delta[(i * 3 + f) * NV + v] : 0);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                real w = 0;
#pragma unroll
                for (int k = 0; k < K; ++k) w += Bt[(f * NQ + q) * K + k] * c1[k];
                real x = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) x += Rr[u] * __shfl(w, l0 + u, 64);
                out[f][q] = (real)(U0 + (double)x);
            }
        }
    }
    if constexpr (NV == 4) if (a.positivity) {
        // optional positivity fallback (not in the paper; density or
        // pressure <= 0 at a Gauss point): the four lanes of the cell
        // exchange their values
        const int l0 = (threadIdx.x & 63) & ~3;
        bool bad = false;
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const real r0 = __shfl(out[f][q], l0, 64), r1 = __shfl(out[f][q], l0 + 1, 64);
                const real r2 = __shfl(out[f][q], l0 + 2, 64), r3 = __shfl(out[f][q], l0 + 3, 64);
                const real pr = euler_pressure(a.gamma, r0, r1, r2, r3);
                bad |= !(r0 > 0) || !(pr > 0);
            }
        if (bad) {
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int q = 0; q < NQ; ++q) out[f][q] = (real)U0;
#pragma unroll
            for (int k = 0; k < NB; ++k) dbyte[k] |= 0x80;
            if (v == 0 && a.fb_count) atomicAdd(a.fb_count, 1ull);
        }
    }
    if (DMODE == 1) {
        if constexpr (VARS == 0) a.delta[i * NV + v] = (uint8_t)dbyte[0];
        else {
#pragma unroll
            for (int f = 0; f < 3; ++f) a.delta[(i * 3 + f) * NV + v] = (uint8_t)dbyte[f];
        }
    }
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int q = 0; q < NQ; ++q) a.FV[((i * 3 + f) * NQ + q) * NV + v] = out[f][q];
}

template <typename real, int R, int NV>
static hipError_t reconstruct_ho_t(const DeviceMesh &m, const double *U, void *FV, uint8_t *delta, int dmode,
                                   const int *done, hipStream_t st, unsigned long long *fb_count) {
    using D = HoDims<R>;
    ReconHoArgs<real> a;
    a.N = m.N;
    a.U = U;
    a.slot = m.slot;
    a.flags = m.flags;
    if constexpr (std::is_same<real, double>::value) { a.P = m.P64; a.tab = m.htab64; }
    else { a.P = m.P32; a.tab = m.htab32; }
    if (!a.P || !a.tab || m.stile != 64 / NV || m.E64 != D::E) return hipErrorInvalidValue;
    if constexpr (std::is_same<real, double>::value) a.fr = m.fr64;
    else a.fr = m.fr32;
    if (m.vars == CTENO_VARS_CHARACTERISTIC && (NV != 4 || !a.fr)) return hipErrorInvalidValue;
    a.FV = (real *)FV;
    a.delta = delta;
    a.done = done;
    const double lam1 = 1.0 - 1.0 / m.lam1p;
    a.lam1 = (real)lam1;
    a.gamma = (real)m.gamma;
    a.ct = (real)m.ct;
    a.eps = (real)m.eps;
    a.positivity = m.positivity;
    a.fb_count = fb_count;
    for (int s = 0; s < 5; ++s) {
        const double ls = s >= 2 ? (1.0 - lam1) / (s - 1) : 0.0;
        a.lams[s] = (real)ls;
        a.lam_ratio[s] = s >= 2 ? (real)(lam1 / ls) : (real)1;
    }
    a.p1_ls = m.scheme == CTENO_SCHEME_TENO ? (real)0 : (real)1;
    a.p1_l1 = m.scheme == CTENO_SCHEME_TENO ? (real)1 : a.lam1;
    const unsigned grid = (unsigned)((m.N * NV + 255) / 256);
#define HO_LAUNCH(SCH, GF, DM)                                                                               \
    do {                                                                                                     \
        if constexpr (NV == 4)                                                                               \
            if (m.vars == CTENO_VARS_CHARACTERISTIC) {                                                       \
                hipLaunchKernelGGL((k_reconstruct_ho<real, R, NV, SCH, GF, DM, 1>), dim3(grid), dim3(256), 0, st, \
                                   a);                                                                       \
                break;                                                                                       \
            }                                                                                                \
        hipLaunchKernelGGL((k_reconstruct_ho<real, R, NV, SCH, GF, DM, 0>), dim3(grid), dim3(256), 0, st, a);   \
    } while (0)
#define HO_DM(SCH, GF)                        \
    switch (dmode) {                          \
        case 0: HO_LAUNCH(SCH, GF, 0); break; \
        case 1: HO_LAUNCH(SCH, GF, 1); break; \
        default: HO_LAUNCH(SCH, GF, 2); break; \
    }
    if (m.scheme == CTENO_SCHEME_CTENOZ && m.gamma_form == CTENO_GAMMA_SCALED) { HO_DM(CTENO_SCHEME_CTENOZ, CTENO_GAMMA_SCALED); }
    else if (m.scheme == CTENO_SCHEME_CTENOZ) { HO_DM(CTENO_SCHEME_CTENOZ, CTENO_GAMMA_PAPER); }
    else if (m.scheme == CTENO_SCHEME_CWENO) { HO_DM(CTENO_SCHEME_CWENO, CTENO_GAMMA_PAPER); }
    else if (m.scheme == CTENO_SCHEME_TENO) { HO_DM(CTENO_SCHEME_TENO, CTENO_GAMMA_PAPER); }
    else if (m.gamma_form == CTENO_GAMMA_LAMBDA) { HO_DM(CTENO_SCHEME_CTENO, CTENO_GAMMA_LAMBDA); }
    else { HO_DM(CTENO_SCHEME_CTENO, CTENO_GAMMA_PAPER); }
#undef HO_DM
#undef HO_LAUNCH
    return hipGetLastError();
}

template <typename real>
hipError_t reconstruct_hi(const DeviceMesh &m, const double *U, void *FV, uint8_t *delta, int dmode,
                          const int *done, hipStream_t st, unsigned long long *fb_count) {
    if (m.nv == 4) {
        switch (m.r) {
            case 4: return reconstruct_ho_t<real, 4, 4>(m, U, FV, delta, dmode, done, st, fb_count);
            case 5: return reconstruct_ho_t<real, 5, 4>(m, U, FV, delta, dmode, done, st, fb_count);
            case 6: return reconstruct_ho_t<real, 6, 4>(m, U, FV, delta, dmode, done, st, fb_count);
        }
    } else {
        switch (m.r) {
            case 4: return reconstruct_ho_t<real, 4, 1>(m, U, FV, delta, dmode, done, st, fb_count);
            case 5: return reconstruct_ho_t<real, 5, 1>(m, U, FV, delta, dmode, done, st, fb_count);
            case 6: return reconstruct_ho_t<real, 6, 1>(m, U, FV, delta, dmode, done, st, fb_count);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace cteno
