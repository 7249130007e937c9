// Device helpers shared by the kernel translation units of the CTENO/CTENOZ
// library: vector loads, face records, the XCD-aware block order, the
// reconstruction body of degree 2 and 3 (used by the single-mesh and the
// batched serving kernels), TENO-type selections, CWENO weights, HLLC and
// the flux / residual / RK body.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cstring>
#include <cmath>
#include <type_traits>
#include <utility>

#include "kernels.h"

namespace cteno {

// ===========================================================================
// small helpers
// ===========================================================================

template <typename real> struct Vec;
template <> struct Vec<float> { using T = float4; static constexpr int W = 4; };
template <> struct Vec<double> { using T = double2; static constexpr int W = 2; };

__device__ __forceinline__ float comp(const float4 &v, int c) { return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w; }
__device__ __forceinline__ double comp(const double2 &v, int c) { return c == 0 ? v.x : v.y; }
__device__ __forceinline__ int comp(const int4 &v, int c) { return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w; }

// Division, reciprocal and square root in the working precision.  FP64 keeps
// the IEEE operations (the fluxes multiply by an IEEE reciprocal where
// several quotients share a denominator: one more rounding).  FP32 takes the
// hardware reciprocal and square root (about 1 ulp each): a few ulps beside
// the correctly rounded sequences, at a fraction of their instruction count.
__device__ __forceinline__ float fdiv(float x, float y) { return x * __builtin_amdgcn_rcpf(y); }
__device__ __forceinline__ double fdiv(double x, double y) { return x / y; }
__device__ __forceinline__ float frcp(float y) { return __builtin_amdgcn_rcpf(y); }
__device__ __forceinline__ double frcp(double y) { return 1.0 / y; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }

// Pressure of a conserved Euler state (rho, m_x, m_y, E).  The positivity
// fallback of the reconstructions and the admissibility test of the fluxes
// evaluate it with this one sequence of roundings (contraction into fused
// operations is off here), so a face state that the fallback accepts is
// accepted by the flux: two formulas could disagree on a state whose
// pressure is within rounding of zero, which FP32 meets in strong shocks.
template <typename real>
__device__ __forceinline__ real euler_pressure(real g, real r, real mx, real my, real E) {
#pragma clang fp contract(off)
    const real q = (real)0.5 * (mx * mx + my * my);
    real ke;
    if constexpr (std::is_same<real, float>::value) ke = q * __builtin_amdgcn_rcpf(r);
    else ke = q / r;
    return (g - 1) * (E - ke);
}

// n consecutive reals from/to an aligned address with the widest vector the
// row size allows (16 bytes, else 8 bytes)
template <typename real, int n>
__device__ __forceinline__ void load_row(const real *__restrict__ p, real *out) {
    if constexpr ((n * sizeof(real)) % 16 == 0) {
        using V = typename Vec<real>::T;
        constexpr int W = Vec<real>::W;
#pragma unroll
        for (int k = 0; k < n / W; ++k) {
            const V v = reinterpret_cast<const V *>(p)[k];
#pragma unroll
            for (int c = 0; c < W; ++c) out[k * W + c] = comp(v, c);
        }
    } else if constexpr (std::is_same<real, float>::value && n % 2 == 0) {
#pragma unroll
        for (int k = 0; k < n / 2; ++k) {
            const float2 v = reinterpret_cast<const float2 *>(p)[k];
            out[2 * k] = v.x;
            out[2 * k + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < n; ++k) out[k] = p[k];
    }
}
template <typename real, int n>
__device__ __forceinline__ void store_row(real *__restrict__ p, const real *in) {
    if constexpr ((n * sizeof(real)) % 16 == 0) {
        if constexpr (std::is_same<real, float>::value) {
#pragma unroll
            for (int k = 0; k < n / 4; ++k)
                reinterpret_cast<float4 *>(p)[k] = make_float4(in[4 * k], in[4 * k + 1], in[4 * k + 2], in[4 * k + 3]);
        } else {
#pragma unroll
            for (int k = 0; k < n / 2; ++k) reinterpret_cast<double2 *>(p)[k] = make_double2(in[2 * k], in[2 * k + 1]);
        }
    } else if constexpr (std::is_same<real, float>::value && n % 2 == 0) {
#pragma unroll
        for (int k = 0; k < n / 2; ++k) reinterpret_cast<float2 *>(p)[k] = make_float2(in[2 * k], in[2 * k + 1]);
    } else {
#pragma unroll
        for (int k = 0; k < n; ++k) p[k] = in[k];
    }
}

// face record of local face f: unit normal, length, neighbour code
template <typename real>
__device__ __forceinline__ void face_record(const real *fr, int64_t i, int f, real &nx, real &ny, real &len,
                                            uint32_t &code) {
    if constexpr (std::is_same<real, float>::value) {
        const float4 r = reinterpret_cast<const float4 *>(fr)[(size_t)(i >> 6) * 3 * 64 + f * 64 + (i & 63)];
        nx = r.x; ny = r.y; len = r.z;
        code = (uint32_t)__float_as_int(r.w);
    } else {
        const double2 *b = reinterpret_cast<const double2 *>(fr) + (size_t)(i >> 6) * 6 * 64 + (i & 63);
        const double2 r0 = b[(2 * f) * 64], r1 = b[(2 * f + 1) * 64];
        nx = r0.x; ny = r0.y; len = r1.x;
        code = (uint32_t)__double_as_longlong(r1.y);
    }
}

// Work-groups are dispatched round-robin over the 8 XCDs; remap them so that
// each XCD (and its L2) works on one contiguous range of cells, which keeps
// the neighbour gathers of adjacent blocks in the same L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
    if (nb < 8) return b;
    const int64_t per = nb / 8, rem = nb % 8;
    const int64_t x = b % 8, pos = b / 8;
    return x < rem ? x * (per + 1) + pos : rem * (per + 1) + (x - rem) * per + pos;
}

// ===========================================================================
// reconstruction
// ===========================================================================

template <typename real>
__device__ __forceinline__ real pow6(real x) {
    const real x2 = x * x;
    return x2 * x2 * x2;
}

// d[v] = U[m][v] - U0[v], rounded to the working precision
template <int NV, typename real>
__device__ __forceinline__ void gather_diff(const double *__restrict__ U, int64_t m, const double *U0, real *d) {
    if constexpr (NV == 4) {
        const double2 u01 = reinterpret_cast<const double2 *>(U)[2 * m];
        const double2 u23 = reinterpret_cast<const double2 *>(U)[2 * m + 1];
        d[0] = (real)(u01.x - U0[0]); d[1] = (real)(u01.y - U0[1]);
        d[2] = (real)(u23.x - U0[2]); d[3] = (real)(u23.y - U0[3]);
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) d[v] = (real)(U[m * NV + v] - U0[v]);
    }
}

template <typename real, int K>
struct ReconArgs {
    int64_t N;
    const double *U;        // AoS [Np][NV]
    const int32_t *slot;    // vector-tiled [SP], VW 4
    const uint8_t *flags;   // [Np]
    const real *P;          // vector-tiled pseudo-inverse stream
    real *FV;               // AoS [Np][3][2][NV]
    uint8_t *delta;         // AoS [Np][NV] (characteristic variables: [Np][3][NV])
    const int *done;
    const real *fr;         // face records (characteristic variables)
    real gram[K][K];
    real basis[3][2][K];
    real lam1, ct, eps;
    real lams[5];           // lambda_s for s_t = 2, 3, 4 (index s_t)
    real gamma;             // ratio of specific heats (positivity check)
    real lam_ratio[5];      // lambda_1 / lambda_s (index s_t)
    int positivity;         // 1: cell-average fallback for non-physical face states
    unsigned long long *fb_count;   // cells that took the fallback (may be null)
};

// TENO selection bits for one variable: bit 0 central, bit 1+s directional s.
// FP64 follows Algorithms 1/2 literally; FP32 evaluates the same chi_s
// through ratios that cannot overflow (gamma_s reaches 1e72 in FP64 terms).
template <typename real, int SCHEME, int GFORM>
__device__ __forceinline__ int teno_bits(const real si[4], int adm, int st, real lam1, real lams, real lratio,
                                         real ct, real eps) {
    int bits = 0;
    if constexpr (std::is_same<real, double>::value) {
        double g[4], sum = 0.0;
        if (SCHEME == CTENO_SCHEME_CTENO) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const double lam = s == 0 ? (double)lam1 : (double)lams;
                g[s] = (GFORM == CTENO_GAMMA_LAMBDA ? lam : 1.0) / pow6(si[s] + eps);
            }
        } else {
            double tsum = 0.0;
#pragma unroll
            for (int s = 1; s < 4; ++s) if ((adm >> s) & 1) tsum += fabs(si[s] - si[0]);
            const double tau = pow6(tsum / (st - 1));
#pragma unroll
            for (int s = 0; s < 4; ++s)
                g[s] = 1.0 + (GFORM == CTENO_GAMMA_SCALED ? tau / pow6(si[s] + eps) : tau / (si[s] + eps));
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) if ((adm >> s) & 1) sum += g[s];
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if ((adm >> s) & 1) {
                const double chi = g[s] / sum;
                if (!(chi < ct)) bits |= 1 << s;
            }
    } else {
        // chi_s < C_T is decided as num_s < C_T sum_t num_t (sum > 0), with
        // one reciprocal per stencil and no division
        float e[4], re[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            e[s] = si[s] + eps;
            re[s] = frcp(e[s]);
        }
        if (SCHEME == CTENO_SCHEME_CTENO) {
            // chi_s = 1 / den_s, den_s = sum_t (lambda_t / lambda_s) (e_s / e_t)^6
            const float ilratio = frcp(lratio);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                if (!((adm >> s) & 1)) continue;
                float den = 0.0f;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (!((adm >> t) & 1)) continue;
                    float lr = 1.0f;
                    if (GFORM == CTENO_GAMMA_LAMBDA && s != t) lr = (t == 0) ? lratio : (s == 0 ? ilratio : 1.0f);
                    den += lr * pow6(e[s] * re[t]);
                }
                if (!(ct * den > 1.0f)) bits |= 1 << s;
            }
        } else {
            float tsum = 0.0f, emin = e[0], remin = re[0];
#pragma unroll
            for (int s = 1; s < 4; ++s)
                if ((adm >> s) & 1) {
                    tsum += fabsf(e[s] - e[0]);
                    emin = fminf(emin, e[s]);
                    remin = fmaxf(remin, re[s]);
                }
            const float mean = tsum * (st == 2 ? 1.0f : st == 3 ? 0.5f : 1.0f / 3.0f);
            float num[4], sum = 0.0f;
            if constexpr (GFORM == CTENO_GAMMA_SCALED) {
                // gamma_s = 1 + X^6 w_s^6 with X = mean |SI_s - SI_1| / emin
                const float X = mean * remin;
                if (X <= 1e5f) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) num[s] = 1.0f + pow6(X * (emin * re[s]));
                } else {
                    const float iX6 = pow6(frcp(X));
#pragma unroll
                    for (int s = 0; s < 4; ++s) num[s] = iX6 + pow6(emin * re[s]);
                }
            } else {
                const float tau = pow6(mean);
                const float G = tau * remin;       // gamma_s = 1 + G w_s, w_s = emin / e_s in (0, 1]
                if (G <= 1e30f) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) num[s] = 1.0f + G * (emin * re[s]);
                } else {
                    const float iG = frcp(G);
#pragma unroll
                    for (int s = 0; s < 4; ++s) num[s] = iG + emin * re[s];
                }
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) if ((adm >> s) & 1) sum += num[s];
            const float lim = ct * sum;
#pragma unroll
            for (int s = 0; s < 4; ++s)
                if ((adm >> s) & 1) {
                    if (!(num[s] < lim)) bits |= 1 << s;
                }
        }
    }
    return bits;
}

// CWENO nonlinear weights (sec. 2.2-2.3: the WENO weights with exponent 4 and
// the linear weights of eq. e18) of the admissible stencils.  FP64 follows
// the formula; FP32 evaluates w_s = 1 / sum_t (lambda_t / lambda_s)
// (e_s / e_t)^4, e = SI + eps, which cannot overflow into a NaN.
template <typename real>
__device__ __forceinline__ void cweno_weights(const real si[4], int adm, real lams, real lam1, real lratio, real eps,
                                              real w[4]) {
    if constexpr (std::is_same<real, double>::value) {
        double g[4], sum = 0.0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const double e = si[s] + eps, e2 = e * e;
            g[s] = ((adm >> s) & 1) ? (s == 0 ? lam1 : lams) / (e2 * e2) : 0.0;
            sum += g[s];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) w[s] = g[s] / sum;
    } else {
        float e[4], re[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            e[s] = si[s] + eps;
            re[s] = frcp(e[s]);
        }
        const float ilratio = frcp(lratio);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            float den = 0.0f;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (!((adm >> t) & 1)) continue;
                const float lr = (s == t) ? 1.0f : (t == 0 ? lratio : (s == 0 ? ilratio : 1.0f));
                const float q = e[s] * re[t], q2 = q * q;
                den += lr * (q2 * q2);
            }
            w[s] = ((adm >> s) & 1) ? frcp(den) : 0.0f;
        }
    }
}

// per-mesh arrays of one reconstruction (the constants stay in ReconArgs)
template <typename real>
struct ReconPtrs {
    const double *U;
    const int32_t *slot;
    const uint8_t *flags;
    const real *P;
    real *FV;
    uint8_t *delta;
    const real *fr;         // face records (characteristic variables only)
    unsigned long long *fb; // cells that took the positivity fallback (may be null)
    const real *tab;        // the block's LDS copy of the Gram matrix [K][K] and face basis [3][2][K]
    double *lad;            // FP64: the block's LDS space for directional coefficients, [3][2][NV] x 256
};

// Entries of the reconstruction's constant table (Gram matrix, then face
// basis values) and its LDS copy: lane 0 of the block writes it from the
// kernel arguments; the caller synchronises the block before use.  In LDS
// the FP32 constants cost no scalar registers in the epilogue, where they
// would not fit beside the kernel's other scalars (FP64 and characteristic
// variables read them from the arguments: as vector registers they would
// cost a wave).
template <int K>
constexpr int recon_tab_size() { return K * K + 6 * K; }
template <typename real, int K>
__device__ __forceinline__ void recon_tab_fill(const ReconArgs<real, K> a, real *tab) {
    if (std::is_same<real, float>::value && threadIdx.x == 0) {
#pragma unroll
        for (int p = 0; p < K; ++p)
#pragma unroll
            for (int q = 0; q < K; ++q) tab[p * K + q] = a.gram[p][q];
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int k = 0; k < K; ++k) tab[K * K + (f * 2 + q) * K + k] = a.basis[f][q][k];
    }
}

// selection (or CWENO weights) of NV fields and their final coefficients,
// in place: c1[K][NV] holds the p_1 coefficients on entry and the final
// polynomial's on exit, cd[3][2][NV] the degree-1 directional ones; forced
// (DMODE 2) points at the fields' forced selection bytes
template <typename real, int K, int NV, int SCHEME, int GFORM, int DMODE, bool LT, typename CD>
__device__ __forceinline__ void finish_fields(const ReconArgs<real, K> a, const real *tab, real (&c1)[K][NV],
                                              const CD cd, int fl, int adm, int st, real lams, real lratio,
                                              const uint8_t *forced, int (&bits)[NV]) {
    if (DMODE == 2 && SCHEME != CTENO_SCHEME_CWENO) {
#pragma unroll
        for (int v = 0; v < NV; ++v) bits[v] = forced[v] & adm;
    } else if (st == 1) {
#pragma unroll
        for (int v = 0; v < NV; ++v) bits[v] = 1;
    } else {
        // smoothness indicators: SI_1 = a1^T G a1, SI_s over the degree-1 block
        // of G.  FP64 sums the full quadratic form; FP32 its upper triangle,
        // whose off-diagonal entries the FP32 table holds doubled
        // (fill_recon_constants), at about half the products.
        constexpr bool SYM = std::is_same<real, float>::value;
        real si[NV][4];
#pragma unroll
        for (int v = 0; v < NV; ++v) si[v][0] = 0;
#pragma unroll
        for (int p = 0; p < K; ++p) {
            real rowp[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) rowp[v] = 0;
#pragma unroll
            for (int q = SYM ? p : 0; q < K; ++q) {
                const real g = LT ? tab[p * K + q] : a.gram[p][q];
#pragma unroll
                for (int v = 0; v < NV; ++v) rowp[v] += g * c1[q][v];
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) si[v][0] += c1[p][v] * rowp[v];
        }
        const real g00 = LT ? tab[0] : a.gram[0][0], g01 = LT ? tab[1] : a.gram[0][1];
        const real g10 = LT ? tab[K] : a.gram[1][0], g11 = LT ? tab[K + 1] : a.gram[1][1];
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const real x0 = cd(q, 0, v), x1 = cd(q, 1, v);
                if constexpr (SYM) si[v][q + 1] = x0 * (g00 * x0 + g01 * x1) + g11 * (x1 * x1);
                else si[v][q + 1] = x0 * (g00 * x0 + g01 * x1) + x1 * (g10 * x0 + g11 * x1);
            }
        if constexpr (SCHEME == CTENO_SCHEME_CWENO) {
            // every admissible stencil contributes; final coefficients, in
            // place: sum_s omega_s p_s
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                bits[v] = adm;
                real w[4];
                cweno_weights<real>(si[v], adm, lams, a.lam1, lratio, a.eps, w);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    real x = w[0] * c1[k][v];
                    if (k < 2) {
#pragma unroll
                        for (int q = 0; q < 3; ++q)
                            if ((fl >> q) & 1) x += w[q + 1] * cd(q, k, v);
                    }
                    c1[k][v] = x;
                }
            }
        } else {
            constexpr int SEL = SCHEME == CTENO_SCHEME_TENO ? CTENO_SCHEME_CTENO : SCHEME;
            constexpr int SGF = SCHEME == CTENO_SCHEME_TENO ? CTENO_GAMMA_PAPER : GFORM;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                bits[v] = teno_bits<real, SEL, SGF>(si[v], adm, st, a.lam1, lams, lratio, a.ct, a.eps);
        }
    }
    // final coefficients, in place: p_1, or the mean of the selected
    // directional polynomials
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (SCHEME != CTENO_SCHEME_CWENO && !(bits[v] & 1)) {
            real s0 = 0, s1 = 0;
            int cnt = 0;
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if ((bits[v] >> (q + 1)) & 1) { s0 += cd(q, 0, v); s1 += cd(q, 1, v); ++cnt; }
            c1[0][v] = cnt == 1 ? s0 : cnt == 2 ? (real)0.5 * s0 : fdiv(s0, (real)3);
            c1[1][v] = cnt == 1 ? s1 : cnt == 2 ? (real)0.5 * s1 : fdiv(s1, (real)3);
#pragma unroll
            for (int k = 2; k < K; ++k) c1[k][v] = 0;
        }
    }
}

// the degree-1 directional coefficients cd(q, c, v) of a cell: in registers,
// or parked in LDS (FP64 reconstruction: the kernel provides [3][2][NV] x
// 256 doubles of block-shared space, one column per lane)
template <typename real, int NV>
struct CdRegs {
    const real (&a)[3][2][NV];
    __device__ __forceinline__ real operator()(int q, int c, int v) const { return a[q][c][v]; }
};
template <int NV>
struct CdLds {
    const double *p;
    __device__ __forceinline__ double operator()(int q, int c, int v) const {
        return p[((q * 2 + c) * NV + v) * 256 + threadIdx.x];
    }
};

// Reconstruction of cell i: its face Gauss-point values in out (and its
// selection bytes, DMODE 1); the caller stores them
template <typename real, int R, int NV, int SCHEME, int GFORM, int DMODE, int VARS>
__device__ __forceinline__ void recon_body(const ReconArgs<real, (R + 1) * (R + 2) / 2 - 1> a,
                                           const ReconPtrs<real> ptr, int64_t i, real (&out)[3][2][NV]) {
    // a and ptr by value: a reference to the kernel-argument struct would make
    // the compiler copy it to scratch memory
    constexpr int K = (R + 1) * (R + 2) / 2 - 1;
    constexpr int M = 2 * K;
    constexpr int S = M > 12 ? M : 12;
    constexpr int SP = (S + 3) / 4 * 4;
    using V = typename Vec<real>::T;
    constexpr int VW = Vec<real>::W;
    constexpr int E = (pinv_offset(S, K) + VW - 1) / VW * VW;

    // this cell's streams: vector g of the pseudo-inverse at Pv[g * 64]
    const V *__restrict__ Pv = reinterpret_cast<const V *>(ptr.P) + (size_t)(i >> 6) * (E / VW) * 64 + (i & 63);
    const int4 *__restrict__ Sv = reinterpret_cast<const int4 *>(ptr.slot) + (size_t)(i >> 6) * (SP / 4) * 64 + (i & 63);

    double U0[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) U0[v] = ptr.U[i * NV + v];

    real ao[K][NV], ad[3][2][NV];
    // FP64: the directional coefficients wait in LDS until the epilogue
    // (registers for two waves per SIMD); 256 lanes per block
    constexpr bool AD_LDS = std::is_same<real, double>::value;
    // FP32 in conserved variables reads the scheme constants from the block's
    // LDS table; the others from the arguments (their epilogues would hold
    // the loaded constants in vector registers and lose a wave per SIMD)
    constexpr bool LTAB = std::is_same<real, float>::value && VARS == 0;
    double *const lad = ptr.lad;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int v = 0; v < NV; ++v) ao[k][v] = 0;
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < NV; ++v) ad[s][c][v] = 0;

    // a_opt = P_c d and a_s = P_s d.  Slots 4s..4s+3 (directional group s)
    // hold K central and 2 directional entries each: 4 (K + 2) entries, a
    // whole number of vectors, loaded at once per group; then the remaining
    // slots with K central entries each.
    constexpr int GE = 4 * (K + 2);
    constexpr int GV = GE / VW;
    // all slot indices up front, so each group's gathers issue with its loads
    int4 slv[SP / 4];
#pragma unroll
    for (int g = 0; g < SP / 4; ++g) slv[g] = Sv[g * 64];
    constexpr int NVEC = E / VW;
    if constexpr (AD_LDS) {
        // FP64: half a group of stream vectors in flight per wave, loaded at
        // the top of its part, and the directional coefficients parked in
        // LDS, so that two waves fit on a SIMD
#pragma unroll 1
        for (int s = 0; s < 3; ++s) {
            int4 sl = slv[0];
#pragma unroll
            for (int s2 = 1; s2 < 3; ++s2)
                if (s2 == s) sl = slv[s2];
            real adt[2][NV];
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int v = 0; v < NV; ++v) adt[c][v] = 0;
            // the group in two halves of two slots (whole vectors)
            constexpr int PARTS = (GE / 2) % VW == 0 ? 2 : 1;
            constexpr int PVEC = GV / PARTS, PT = 4 / PARTS;
#pragma unroll
            for (int h = 0; h < PARTS; ++h) {
                V cur[PVEC];
#pragma unroll
                for (int g = 0; g < PVEC; ++g) cur[g] = Pv[(s * GV + h * PVEC + g) * 64];
#pragma unroll
                for (int t = h * PT; t < (h + 1) * PT; ++t) {
                    const int64_t m = comp(sl, t);
                    real d[NV];
                    gather_diff<NV>(ptr.U, m, U0, d);
#pragma unroll
                    for (int q = 0; q < K + 2; ++q) {
                        const int el = t * (K + 2) + q - h * PVEC * VW;
                        const real p = comp(cur[el / VW], el % VW);
                        if (q < K) {
#pragma unroll
                            for (int v = 0; v < NV; ++v) ao[q][v] += p * d[v];
                        } else {
#pragma unroll
                            for (int v = 0; v < NV; ++v) adt[q - K][v] += p * d[v];
                        }
                    }
                }
                if (PARTS > 1) __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int v = 0; v < NV; ++v) lad[((s * 2 + c) * NV + v) * 256 + threadIdx.x] = adt[c][v];
            __builtin_amdgcn_sched_barrier(0);   // keep the groups apart: bounded live registers
        }
        if constexpr (S > 12) {
            // remaining slots (K central entries each), from stream vector 3 GV
            // on, in parts of at most three slots
            constexpr int T0 = 12 * (K + 2);
            constexpr int NT = S - 12;
#pragma unroll
            for (int t0 = 0; t0 < NT; t0 += 3) {
                constexpr int PV = (3 * K + 2 * VW - 2) / VW;     // vectors that three slots can touch
                const int v0 = (T0 + t0 * K) / VW;
                V buf[PV];
#pragma unroll
                for (int g = 0; g < PV; ++g)
                    if (v0 + g < NVEC) buf[g] = Pv[(v0 + g) * 64];
#pragma unroll
                for (int t = t0; t < t0 + 3 && t < NT; ++t) {
                    const int j = 12 + t;
                    const int64_t m = comp(slv[j / 4], j % 4);
                    real d[NV];
                    gather_diff<NV>(ptr.U, m, U0, d);
#pragma unroll
                    for (int q = 0; q < K; ++q) {
                        const int e = T0 + t * K + q;
                        const real p = comp(buf[e / VW - v0], e % VW);
#pragma unroll
                        for (int v = 0; v < NV; ++v) ao[q][v] += p * d[v];
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    } else {
        // Rolled loop over the three directional groups with a two-deep load
        // pipeline: the GV vectors that follow group s (group s + 1, or the head
        // of the remaining slots) are requested before group s is computed, so a
        // wave keeps two groups of stream loads in flight.  With no remaining
        // slots (S = 12) the last iteration requests its own group again.
        static_assert(S == 12 || 4 * GV <= NVEC, "stream shorter than four groups");
        V cur[GV];
#pragma unroll
        for (int g = 0; g < GV; ++g) cur[g] = Pv[g * 64];
#pragma unroll 1
        for (int s = 0; s < 3; ++s) {
            int4 sl = slv[0];
#pragma unroll
            for (int s2 = 1; s2 < 3; ++s2)
                if (s2 == s) sl = slv[s2];
            const int gn = (S > 12 || s < 2 ? s + 1 : s) * GV;
            V nxt[GV];
#pragma unroll
            for (int g = 0; g < GV; ++g) nxt[g] = Pv[(gn + g) * 64];
            real adt[2][NV];
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int v = 0; v < NV; ++v) adt[c][v] = 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t m = comp(sl, t);
                real d[NV];
                gather_diff<NV>(ptr.U, m, U0, d);
#pragma unroll
                for (int q = 0; q < K + 2; ++q) {
                    const int el = t * (K + 2) + q;
                    const real p = comp(cur[el / VW], el % VW);
                    if (q < K) {
#pragma unroll
                        for (int v = 0; v < NV; ++v) ao[q][v] += p * d[v];
                    } else {
#pragma unroll
                        for (int v = 0; v < NV; ++v) adt[q - K][v] += p * d[v];
                    }
                }
            }
#pragma unroll
            for (int s2 = 0; s2 < 3; ++s2)
                if (s2 == s)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
#pragma unroll
                        for (int v = 0; v < NV; ++v) ad[s2][c][v] = adt[c][v];
#pragma unroll
            for (int g = 0; g < GV; ++g) cur[g] = nxt[g];
            __builtin_amdgcn_sched_barrier(0);   // keep the groups apart: bounded live registers
        }
        if constexpr (S > 12) {
            // remaining slots (K central entries each): cur holds stream vectors
            // [3 GV, 4 GV); the rest of the stream follows
            constexpr int T0 = 12 * (K + 2);
            constexpr int NT = S - 12;
            constexpr int RV = NVEC - 4 * GV;
            V rest[RV > 0 ? RV : 1];
#pragma unroll
            for (int g = 0; g < RV; ++g) rest[g] = Pv[(4 * GV + g) * 64];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int j = 12 + t;
                const int64_t m = comp(slv[j / 4], j % 4);
                real d[NV];
                gather_diff<NV>(ptr.U, m, U0, d);
#pragma unroll
                for (int q = 0; q < K; ++q) {
                    const int e = T0 + t * K + q;
                    const int gv = e / VW - 3 * GV;     // compile-time after unrolling
                    const real p = gv < GV ? comp(cur[gv < GV ? gv : 0], e % VW)
                                           : comp(rest[gv < GV ? 0 : gv - GV], e % VW);
#pragma unroll
                    for (int v = 0; v < NV; ++v) ao[q][v] += p * d[v];
                }
            }
        }
    }
    // the directional coefficients, wherever they wait
    auto adv = [&](int q, int c, int v) -> real {
        if constexpr (AD_LDS) return lad[((q * 2 + c) * NV + v) * 256 + threadIdx.x];
        else return ad[q][c][v];
    };
    const int fl = ptr.flags[i] & 7;
    const int adm = 1 | (fl << 1);
    const int st = 1 + __popc(fl);
    // static indices only: a dynamic index into the argument struct would
    // force it into scratch memory
    const real lams = st == 2 ? a.lams[2] : (st == 3 ? a.lams[3] : a.lams[4]);
    const real lratio = st == 2 ? a.lam_ratio[2] : (st == 3 ? a.lam_ratio[3] : a.lam_ratio[4]);
    // The epilogue works on all variables at once, phase by phase, so each
    // scheme constant (Gram matrix, face basis values) is used once and
    // dies, instead of staying live across a per-variable loop.
    // p_1 = (p_opt - sum_s lambda_s p_s) / lambda_1, in place of a_opt, with
    // one reciprocal of lambda_1
    const real ilam1 = frcp(a.lam1);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            real sm = ao[k][v];
            if (k < 2 && st > 1) {
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    if ((fl >> q) & 1) sm -= lams * adv(q, k, v);
            }
            // TENO keeps the central stencil's own polynomial
            if (SCHEME != CTENO_SCHEME_TENO) ao[k][v] = st > 1 ? sm * ilam1 : sm;
        }
    constexpr int NB = VARS ? 3 * NV : NV;       // selection bytes per cell
    uint8_t dbyte[NB];
    if constexpr (VARS == 0) {
        int bits[NV];
        if constexpr (AD_LDS)
            finish_fields<real, K, NV, SCHEME, GFORM, DMODE, LTAB>(a, ptr.tab, ao, CdLds<NV>{lad}, fl, adm, st,
                                                                   lams, lratio, ptr.delta + i * NV, bits);
        else
            finish_fields<real, K, NV, SCHEME, GFORM, DMODE, LTAB>(a, ptr.tab, ao, CdRegs<real, NV>{ad}, fl, adm,
                                                                   st, lams, lratio, ptr.delta + i * NV, bits);
#pragma unroll
        for (int v = 0; v < NV; ++v) dbyte[v] = (uint8_t)bits[v];
        // face Gauss-point values
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                real val[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) val[v] = 0;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const real b = LTAB ? ptr.tab[K * K + (f * 2 + q) * K + k] : a.basis[f][q][k];
#pragma unroll
                    for (int v = 0; v < NV; ++v) val[v] += b * ao[k][v];
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) out[f][q][v] = (real)(U0[v] + (double)val[v]);
            }
    } else {
        // characteristic fields per face: the least-squares coefficients are
        // linear in the data, so projecting them with L_f equals
        // reconstructing the projected averages W = L_f U; the face values
        // are U_0 + R_f (W(x_q) - W_0)
        static_assert(NV == 4, "characteristic variables need the Euler equations");
        const real rho = (real)U0[0], uu = (real)(U0[1] / U0[0]), vv = (real)(U0[2] / U0[0]);
        const real q2 = (real)0.5 * (uu * uu + vv * vv);
        const real pr = (a.gamma - 1) * ((real)U0[3] - rho * q2);
        const real cs = fsqrt(fdiv(a.gamma * pr, rho)), H = fdiv((real)U0[3] + pr, rho);
        const real b1 = fdiv(a.gamma - 1, cs * cs), b2 = b1 * q2, ic = frcp(cs);
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            real nx, ny, len;
            uint32_t code;
            face_record<real>(ptr.fr, i, f, nx, ny, len, code);
            const real un = uu * nx + vv * ny, ut = -uu * ny + vv * nx;
            const real L[4][4] = {{(real)0.5 * (b2 + un * ic), (real)-0.5 * (b1 * uu + nx * ic),
                                   (real)-0.5 * (b1 * vv + ny * ic), (real)0.5 * b1},
                                  {1 - b2, b1 * uu, b1 * vv, -b1},
                                  {-ut, -ny, nx, 0},
                                  {(real)0.5 * (b2 - un * ic), (real)-0.5 * (b1 * uu - nx * ic),
                                   (real)-0.5 * (b1 * vv - ny * ic), (real)0.5 * b1}};
            const real Rm[4][4] = {{1, 1, 0, 1},
                                   {uu - cs * nx, uu, -ny, uu + cs * nx},
                                   {vv - cs * ny, vv, nx, vv + cs * ny},
                                   {H - un * cs, q2, ut, H + un * cs}};
            real c1[K][4], cd[3][2][4];
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    real x = 0;
#pragma unroll
                    for (int v = 0; v < 4; ++v) x += L[j][v] * ao[k][v];
                    c1[k][j] = x;
                }
#pragma unroll
            for (int s2 = 0; s2 < 3; ++s2)
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        real x = 0;
#pragma unroll
                        for (int v = 0; v < 4; ++v) x += L[j][v] * adv(s2, k, v);
                        cd[s2][k][j] = x;
                    }
            int bits[4];
            finish_fields<real, K, 4, SCHEME, GFORM, DMODE, false>(a, ptr.tab, c1, CdRegs<real, 4>{cd}, fl, adm, st,
                                                                   lams, lratio, ptr.delta + (i * 3 + f) * 4, bits);
#pragma unroll
            for (int j = 0; j < 4; ++j) dbyte[f * 4 + j] = (uint8_t)bits[j];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                real w[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) w[j] = 0;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const real b = a.basis[f][q][k];
#pragma unroll
                    for (int j = 0; j < 4; ++j) w[j] += b * c1[k][j];
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    real x = 0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) x += Rm[v][j] * w[j];
                    out[f][q][v] = (real)(U0[v] + (double)x);
                }
            }
        }
    }
    if constexpr (NV == 4) if (a.positivity) {
        // optional positivity fallback (not in the paper): a cell with a
        // non-physical state (density or pressure <= 0) at any of its Gauss
        // points uses its cell average at all of them; reported with bit 7
        // of its selection bytes and counted.  Without it the flux reports
        // the state.
        bool bad = false;
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const real rho = out[f][q][0];
                const real pr = euler_pressure(a.gamma, rho, out[f][q][1], out[f][q][2], out[f][q][3]);
                bad |= !(rho > 0) || !(pr > 0);
            }
        if (bad) {
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int v = 0; v < NV; ++v) out[f][q][v] = (real)U0[v];
#pragma unroll
            for (int k = 0; k < NB; ++k) dbyte[k] |= 0x80;
            if (ptr.fb) atomicAdd(ptr.fb, 1ull);
        }
    }
    if (DMODE == 1) {
#pragma unroll
        for (int k = 0; k < NB; ++k) ptr.delta[i * NB + k] = dbyte[k];
    }
}


// scheme constants of the reconstruction (tables of the reference triangle,
// linear weights of eq. e18 for every admissible-stencil count)
template <typename real, int K>
inline void fill_recon_constants(const DeviceMesh &m, ReconArgs<real, K> &a) {
    a.N = m.N;
    // FP64: the Gram matrix; FP32: its upper triangle with the off-diagonal
    // entries doubled (finish_fields sums the quadratic form over it), the
    // lower triangle as is
    constexpr bool sym = std::is_same<real, float>::value;
    for (int p = 0; p < K; ++p)
        for (int q = 0; q < K; ++q) a.gram[p][q] = (real)((sym && q > p ? 2.0 : 1.0) * m.tab.gram[p][q]);
    for (int f = 0; f < 3; ++f)
        for (int q = 0; q < 2; ++q)
            for (int k = 0; k < K; ++k) a.basis[f][q][k] = (real)m.tab.basis[f][q][k];
    const double lam1 = 1.0 - 1.0 / m.lam1p;
    a.lam1 = (real)lam1;
    a.gamma = (real)m.gamma;
    a.ct = (real)m.ct;
    a.eps = (real)m.eps;
    a.positivity = m.positivity;
    a.fb_count = nullptr;
    for (int s = 0; s < 5; ++s) {
        const double ls = s >= 2 ? (1.0 - lam1) / (s - 1) : 0.0;
        a.lams[s] = (real)ls;
        a.lam_ratio[s] = s >= 2 ? (real)(lam1 / ls) : (real)1;
    }
}

template <int R>
struct HoDims {
    static constexpr int K = (R + 1) * (R + 2) / 2 - 1;
    static constexpr int RD = (R + 1) / 2;
    static constexpr int KD = (RD + 1) * (RD + 2) / 2 - 1;
    static constexpr int MD = 2 * KD;
    static constexpr int M = 2 * K;
    // variable groups (degrees 4 and 5): the slots are the M central cells,
    // each directional stencil's members contiguous, their stencil in the
    // slot entry; else three groups of M_d slots
    static constexpr bool VARG = M < 3 * MD;
    static constexpr int S = VARG ? M : 3 * MD;
    static constexpr int SP = (S + 3) / 4 * 4;
    static constexpr int EPS = (K + KD + 3) / 4 * 4;
    static constexpr int E = S * EPS;
    static constexpr int NQ = (R + 2) / 2;
    static_assert(S >= 2 * K, "the directional groups must hold the central stencil");
    static_assert(S <= 64, "one lane per least-squares row");
};

// ===========================================================================
// fluxes, residual, Runge-Kutta
// ===========================================================================

// HLLC with Roe-averaged signal speeds (sec. 2.7), in the face-normal frame
// (u normal, w tangential velocity); F returned in the global frame.
template <typename real>
__device__ __forceinline__ bool hllc(real g, const real *UL, const real *UR, real nx, real ny, real *F) {
    // one reciprocal per denominator, shared by the quotients over it
    const real rl = UL[0], rr = UR[0];
    const real irl = frcp(rl), irr = frcp(rr);
    const real ul = (UL[1] * nx + UL[2] * ny) * irl, wl = (-UL[1] * ny + UL[2] * nx) * irl;
    const real ur = (UR[1] * nx + UR[2] * ny) * irr, wr = (-UR[1] * ny + UR[2] * nx) * irr;
    const real El = UL[3], Er = UR[3];
    const real h = (real)0.5;
    const real pl = euler_pressure(g, rl, UL[1], UL[2], El);
    const real pr = euler_pressure(g, rr, UR[1], UR[2], Er);
    const bool ok = rl > 0 && rr > 0 && pl > 0 && pr > 0;
    const real cl = fsqrt((g * pl) * irl), cr = fsqrt((g * pr) * irr);
    const real Hl = (El + pl) * irl, Hr = (Er + pr) * irr;
    const real D = fsqrt(rr * irl);
    const real iD = frcp(1 + D);
    const real ut = (ul + ur * D) * iD;
    const real wt = (wl + wr * D) * iD;
    const real Ht = (Hl + Hr * D) * iD;
    const real ct = fsqrt((g - 1) * (Ht - h * (ut * ut + wt * wt)));
    const real SL = fmin(ul - cl, ut - ct);
    const real SR = fmax(ur + cr, ut + ct);
    const real SM = fdiv(rr * ur * (SR - ur) - rl * ul * (SL - ul) + pl - pr, rr * (SR - ur) - rl * (SL - ul));
    const real ps = rl * (ul - SL) * (ul - SM) + pl;
    real Fn[4];
    if (SL > 0) {
        Fn[0] = rl * ul; Fn[1] = rl * ul * ul + pl; Fn[2] = rl * ul * wl; Fn[3] = ul * (El + pl);
    } else if (0 < SM) {
        const real id = frcp(SL - SM);
        const real Us0 = (rl * (SL - ul)) * id;
        const real Us1 = ((SL - ul) * rl * ul + ps - pl) * id;
        const real Us2 = ((SL - ul) * rl * wl) * id;
        const real Us3 = ((SL - ul) * El - pl * ul + ps * SM) * id;
        Fn[0] = rl * ul + SL * (Us0 - rl);
        Fn[1] = (rl * ul * ul + pl) + SL * (Us1 - rl * ul);
        Fn[2] = rl * ul * wl + SL * (Us2 - rl * wl);
        Fn[3] = ul * (El + pl) + SL * (Us3 - El);
    } else if (0 < SR) {
        const real id = frcp(SR - SM);
        const real Us0 = (rr * (SR - ur)) * id;
        const real Us1 = ((SR - ur) * rr * ur + ps - pr) * id;
        const real Us2 = ((SR - ur) * rr * wr) * id;
        const real Us3 = ((SR - ur) * Er - pr * ur + ps * SM) * id;
        Fn[0] = rr * ur + SR * (Us0 - rr);
        Fn[1] = (rr * ur * ur + pr) + SR * (Us1 - rr * ur);
        Fn[2] = rr * ur * wr + SR * (Us2 - rr * wr);
        Fn[3] = ur * (Er + pr) + SR * (Us3 - Er);
    } else {
        Fn[0] = rr * ur; Fn[1] = rr * ur * ur + pr; Fn[2] = rr * ur * wr; Fn[3] = ur * (Er + pr);
    }
    F[0] = Fn[0];
    F[1] = Fn[1] * nx - Fn[2] * ny;
    F[2] = Fn[1] * ny + Fn[2] * nx;
    F[3] = Fn[3];
    return ok;
}

// HLLC through a wall, i.e. against the mirror image of the inside state:
// the Roe-averaged normal velocity and the contact speed are zero, so the
// flux is the star pressure on the normal, p* = p + rho u_n (u_n - S_L),
// with S_L = min(u_n - c, -c~) and c~^2 = (gamma - 1)(H - w^2 / 2).  Written
// out, the mass and energy fluxes through the wall are exactly zero in
// either precision (the star-region formulas leave a rounding residue).
template <typename real>
__device__ __forceinline__ bool wall_flux(real g, const real *UL, real nx, real ny, real *F) {
    const real r = UL[0];
    const real ir = frcp(r);
    const real u = (UL[1] * nx + UL[2] * ny) * ir, w = (-UL[1] * ny + UL[2] * nx) * ir;
    const real E = UL[3];
    const real p = euler_pressure(g, r, UL[1], UL[2], E);
    const bool ok = r > 0 && p > 0;
    const real c = fsqrt((g * p) * ir);
    const real H = (E + p) * ir;
    const real ct = fsqrt((g - 1) * (H - (real)0.5 * w * w));
    const real SL = fmin(u - c, -ct);
    const real ps = r * (u - SL) * u + p;
    F[0] = 0;
    F[1] = ps * nx;
    F[2] = ps * ny;
    F[3] = 0;
    return ok;
}

template <typename real>
struct FluxArgs {
    int64_t N;
    const real *FV;
    const real *fr;         // face records (nx, ny, |A|, code), vector-tiled
    const double *area;
    const double *Un, *Us;
    double *Uout;
    const double *dt_ptr;
    double dt_value;
    real *flux_out;
    double *resid;
    Ctrl *ctrl;             // time march: done flag and time (may be null)
    int *nonphys;           // set when a face state is non-physical (may be null)
    double *dt_part;
    real gamma, ax, ay;
    real gw[4];             // Gauss weights on [0, 1]
    double gamma64;
    int stage;
    // prescribed-state (inflow) boundary faces
    const double *bface;    // [n_inflow][4]: first vertex (x, y) and edge vector of each inflow face
    double bst[2][4];       // outside states behind / ahead of the moving line (conserved variables)
    double bline[3];        // the line x = bline[0] + bline[1] y + bline[2] t
    double gq[4];           // Gauss nodes on [0, 1]
    double t_base;          // time of the stage input when tctrl is null
    const Ctrl *tctrl;      // time march: the stage input's time is tctrl->t, its step *dt_ptr
    // fused stage: cells with a face whose neighbour lies in another
    // 256-cell block (cross cells) finish in a second kernel from their
    // partial stage states; their data in cross-cell order
    double *xpart;          // [n_cross][NV] stage states from the faces inside the block
    const int32_t *xcells;  // the cross cells, ascending
    int64_t n_cross;
    const int32_t *xbase;   // [blocks + 1] cross cells before each block
    const int32_t *xnb;     // [n_cross][3] the neighbour's cross index across a face to another block, else -1
    const double *xarea;    // [n_cross]
    const real *xfr;        // [n_cross] face records, tiled like fr
    int64_t part_off;       // offset of the second kernel's block minima in dt_part
};

// the launch arguments of a flux / residual / RK stage (MODE f.mode)
template <typename real>
inline void fill_flux_args(const DeviceMesh &m, const FluxLaunch &f, FluxArgs<real> &a) {
    a = FluxArgs<real>{};
    a.N = m.N;
    a.FV = (const real *)f.FV;
    if constexpr (std::is_same<real, double>::value) a.fr = m.fr64;
    else a.fr = m.fr32;
    a.area = m.area;
    a.Un = f.Un; a.Us = f.Us; a.Uout = f.Uout;
    a.dt_ptr = f.dt_ptr; a.dt_value = f.dt_value;
    a.flux_out = (real *)f.flux_out;
    a.resid = f.resid;
    a.ctrl = f.ctrl;
    a.nonphys = f.nonphys ? f.nonphys : (f.ctrl ? &f.ctrl->nonphysical : nullptr);
    a.dt_part = f.dt_part;
    a.gamma = (real)m.gamma; a.ax = (real)m.ax; a.ay = (real)m.ay;
    a.gamma64 = m.gamma;
    a.stage = f.mode == 2 ? f.stage : 0;
    for (int q = 0; q < 4; ++q) a.gw[q] = q < m.tab.Nq ? (real)m.tab.gw[q] : (real)0;
    a.bface = m.bface;
    for (int k = 0; k < 2; ++k)
        for (int v = 0; v < 4; ++v) a.bst[k][v] = m.bst[k][v];
    for (int k = 0; k < 3; ++k) a.bline[k] = m.bline[k];
    for (int q = 0; q < 4; ++q) a.gq[q] = q < m.tab.Nq ? m.tab.gq[q] : 0.0;
    a.t_base = f.t_base;
    a.tctrl = f.ctrl && f.dt_ptr ? f.ctrl : nullptr;
    a.xpart = f.xpart;
    a.xcells = m.xcells;
    a.n_cross = m.n_cross;
    a.xbase = m.xbase;
    a.xnb = m.xnb;
    a.xarea = m.xarea;
    if constexpr (std::is_same<real, double>::value) a.xfr = m.xfr64;
    else a.xfr = m.xfr32;
    a.part_off = m.blocks();
}

template <int NV, int PHYS>
__device__ __forceinline__ double cell_dt_bound(const double *U, const double nrm[3][3], double area, double gamma,
                                                double ax, double ay) {
    double sum = 0.0;
    if (PHYS == CTENO_EULER) {
        const double rho = U[0], u = U[1] / rho, v = U[2] / rho;
        const double p = (gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v));
        const double c = sqrt(gamma * p / rho);
#pragma unroll
        for (int f = 0; f < 3; ++f) sum += nrm[f][2] * (fabs(u * nrm[f][0] + v * nrm[f][1]) + c);
    } else {
#pragma unroll
        for (int f = 0; f < 3; ++f) sum += nrm[f][2] * fabs(ax * nrm[f][0] + ay * nrm[f][1]);
    }
    return 2.0 * area / sum;
}

// minimum over the block (all threads call it; result valid in thread 0)
__device__ __forceinline__ double block_min(double v) {
    __shared__ double red[16];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = INFINITY;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r = fmin(r, red[k]);
    return r;
}

// per-mesh arrays of one flux / residual / RK launch (constants stay in FluxArgs)
template <typename real>
struct FluxPtrs {
    const real *FV;
    const real *fr;
    const double *area;
    const double *Un, *Us;
    double *Uout;
    const double *dt_ptr;
    real *flux_out;
    double *resid;
    int *nonphys;           // set when a face state is non-physical (may be null)
    bool want_dt;
};

// Outside values of a boundary face at its Gauss points, oth[NQ-1-q]
// paired with ownf[q]: a prescribed (inflow) state on the Gauss point's side
// of the moving line at the stage time (t, t + dt, t + dt/2 for the three
// stages), or the inside state (transmissive).  Returns true for a wall of
// the Euler equations, whose flux comes in closed form from the inside state.
template <typename real, int NV, int PHYS, int MODE, int NQ>
__device__ __forceinline__ bool boundary_state(const FluxArgs<real> a, const double *dt_ptr, uint32_t code,
                                               const real (&ownf)[NQ][NV], real (&oth)[NQ][NV]) {
    const uint32_t kind = code & 3u;
    if (PHYS == CTENO_EULER && kind == CTENO_WALL) return true;
    if (kind == CTENO_INFLOW) {
        const double *e = a.bface + 4 * (int64_t)((code >> 2) & kNbInflowMask);
        const double t0 = a.tctrl ? a.tctrl->t : a.t_base;
        const double dts = MODE == 2 ? (dt_ptr ? *dt_ptr : a.dt_value) : 0.0;
        const double ts = t0 + (a.stage == 1 ? dts : a.stage == 2 ? 0.5 * dts : 0.0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const double px = e[0] + a.gq[q] * e[2], py = e[1] + a.gq[q] * e[3];
            const int side = px < a.bline[0] + a.bline[1] * py + a.bline[2] * ts ? 0 : 1;
#pragma unroll
            for (int v = 0; v < NV; ++v) oth[NQ - 1 - q][v] = (real)a.bst[side][v];
        }
    } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int v = 0; v < NV; ++v) oth[NQ - 1 - q][v] = ownf[q][v];
    }
    return false;
}

// A cell's outward flux through one face, |A| sum_q w_q F_q, with its sign.
// Both cells of a face evaluate F(owner side, other side; owner normal) at
// the owner's Gauss points in the owner's order, so the two terms are
// bitwise negatives of each other.
template <typename real, int NV, int PHYS, int NQ>
__device__ __forceinline__ void face_term(const FluxArgs<real> a, const real (&ownf)[NQ][NV],
                                          const real (&oth)[NQ][NV], bool owner, bool wallf, real nx, real ny,
                                          real len, double (&term)[NV], bool &bad) {
    const real fx = owner ? nx : -nx, fy = owner ? ny : -ny;
    real sumF[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) sumF[v] = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        real A[NV], B[NV], F[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            A[v] = owner ? ownf[q][v] : oth[q][v];
            B[v] = owner ? oth[NQ - 1 - q][v] : ownf[NQ - 1 - q][v];
        }
        if (PHYS == CTENO_EULER) {
            if (wallf) bad |= !wall_flux<real>(a.gamma, A, fx, fy, F);
            else bad |= !hllc<real>(a.gamma, A, B, fx, fy, F);
        } else {
            const real an = a.ax * fx + a.ay * fy;
            F[0] = an * (an >= 0 ? A[0] : B[0]);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) sumF[v] += a.gw[q] * F[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double val = (double)(len * sumF[v]);
        term[v] = owner ? val : -val;
    }
}

// U^n, the stage input and the area of cell i (the RK stage's operands)
template <typename real, int NV>
__device__ __forceinline__ void rk_load(const FluxPtrs<real> ptr, int64_t i, double (&u0)[NV], double (&us)[NV],
                                        double &ar) {
    ar = ptr.area[i];
    if constexpr (NV == 4) {
        const double2 *U2 = reinterpret_cast<const double2 *>(ptr.Un);
        const double2 *S2 = reinterpret_cast<const double2 *>(ptr.Us);
        const double2 x0 = U2[2 * i], x1 = U2[2 * i + 1], y0 = S2[2 * i], y1 = S2[2 * i + 1];
        u0[0] = x0.x; u0[1] = x0.y; u0[2] = x1.x; u0[3] = x1.y;
        us[0] = y0.x; us[1] = y0.y; us[2] = y1.x; us[3] = y1.y;
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) { u0[v] = ptr.Un[i * NV + v]; us[v] = ptr.Us[i * NV + v]; }
    }
}

// SSP-RK3 stage value from U^n, the stage input and dt times the residual
__device__ __forceinline__ double rk_value(int stage, double u0, double us, double dtR) {
    if (stage == 0) return us + dtR;
    if (stage == 1) return 0.75 * u0 + 0.25 * (us + dtR);
    return (1.0 / 3.0) * u0 + (2.0 / 3.0) * (us + dtR);
}
// the weight of dt times the residual in rk_value
__device__ __forceinline__ double rk_weight(int stage) { return stage == 0 ? 1.0 : stage == 1 ? 0.25 : 2.0 / 3.0; }

// writes the new state un of cell i; returns its CFL bound when requested, else +inf
template <typename real, int NV, int PHYS>
__device__ __forceinline__ double rk_store(const FluxArgs<real> a, const FluxPtrs<real> ptr, int64_t i,
                                           const double (&un)[NV], const double (&nrm)[3][3], double ar) {
    if constexpr (NV == 4) {
        double2 *O2 = reinterpret_cast<double2 *>(ptr.Uout);
        O2[2 * i] = make_double2(un[0], un[1]);
        O2[2 * i + 1] = make_double2(un[2], un[3]);
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) ptr.Uout[i * NV + v] = un[v];
    }
    return ptr.want_dt ? cell_dt_bound<NV, PHYS>(un, nrm, ar, a.gamma64, (double)a.ax, (double)a.ay) : INFINITY;
}

// SSP-RK3 stage of cell i from the sum acc of its outward face fluxes (the
// residual is -acc / |V_i|) and its loaded operands: writes the new state;
// returns its CFL bound when requested, else +inf
template <typename real, int NV, int PHYS>
__device__ __forceinline__ double rk_apply(const FluxArgs<real> a, const FluxPtrs<real> ptr, int64_t i,
                                           const double (&acc)[NV], const double (&nrm)[3][3],
                                           const double (&u0)[NV], const double (&us)[NV], double ar) {
    const double dt = ptr.dt_ptr ? *ptr.dt_ptr : a.dt_value;
    double un[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) un[v] = rk_value(a.stage, u0[v], us[v], dt * (-acc[v] / ar));
    return rk_store<real, NV, PHYS>(a, ptr, i, un, nrm, ar);
}

template <typename real, int NV, int PHYS>
__device__ __forceinline__ double rk_update(const FluxArgs<real> a, const FluxPtrs<real> ptr, int64_t i,
                                            const double (&acc)[NV], const double (&nrm)[3][3]) {
    double u0[NV], us[NV], ar;
    rk_load<real, NV>(ptr, i, u0, us, ar);
    return rk_apply<real, NV, PHYS>(a, ptr, i, acc, nrm, u0, us, ar);
}

// one cell's three faces, residual and (MODE 2) RK stage; returns the cell's
// CFL bound of the new state when requested, else +inf
template <typename real, int NV, int PHYS, int MODE, int NQ>
__device__ __forceinline__ double flux_body(const FluxArgs<real> a, const FluxPtrs<real> ptr, int64_t i) {
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    double nrm[3][3];
    bool bad = false;
    real own[3][NQ][NV];
    load_row<real, 3 * NQ * NV>(ptr.FV + i * 3 * NQ * NV, &own[0][0][0]);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        real nx, ny, len;
        uint32_t code;
        face_record<real>(ptr.fr, i, f, nx, ny, len, code);
        nrm[f][0] = (double)nx; nrm[f][1] = (double)ny; nrm[f][2] = (double)len;
        real oth[NQ][NV];
        bool owner = true, wallf = false;
        if (code & kNbBoundary) {
            wallf = boundary_state<real, NV, PHYS, MODE, NQ>(a, ptr.dt_ptr, code, own[f], oth);
        } else {
            owner = (code & kNbOwner) != 0;
            const int64_t j = code & kNbIndexMask;
            const int g = (code >> 28) & 3;
            load_row<real, NQ * NV>(ptr.FV + (j * 3 + g) * NQ * NV, &oth[0][0]);
        }
        double term[NV];
        face_term<real, NV, PHYS, NQ>(a, own[f], oth, owner, wallf, nx, ny, len, term, bad);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            acc[v] += term[v];
            if (MODE == 0) ptr.flux_out[(i * 3 + f) * NV + v] = (real)term[v];
        }
    }
    if (bad && ptr.nonphys) atomicOr(ptr.nonphys, 1);
    if (MODE == 1) {
#pragma unroll
        for (int v = 0; v < NV; ++v) ptr.resid[i * NV + v] = -acc[v] / ptr.area[i];
    }
    if (MODE == 2) return rk_update<real, NV, PHYS>(a, ptr, i, acc, nrm);
    return INFINITY;
}

}  // namespace cteno
