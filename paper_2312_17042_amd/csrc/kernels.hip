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
// precompute (FP64)
// ===========================================================================

struct QuadRule {
    double s[16], t[16], w[16];     // collapsed Gauss-Legendre 4x4 on the reference triangle
};

template <int R>
struct PreArgs {
    static constexpr int K = (R + 1) * (R + 2) / 2 - 1;
    static constexpr int M = 2 * K;
    static constexpr int S = M > 12 ? M : 12;
    static constexpr int SP = (S + 3) / 4 * 4;
    int64_t N;
    const double *verts;
    const int32_t *slot;
    const uint8_t *slot_flag;
    const int8_t *slot_shift;
    uint8_t *flags;
    int *rank_fail;
    double *P64;
    float *P32;
    int E64, E32;
    double Lx, Ly;
    int ex[K][2];
    double mean[K];
    QuadRule q;
};

template <int R>
__global__ __launch_bounds__(64) void k_precompute(const PreArgs<R> a) {
    constexpr int K = PreArgs<R>::K;
    constexpr int S = PreArgs<R>::S;
    constexpr int SP = PreArgs<R>::SP;
    __shared__ double sA[K * S][64];      // least-squares matrix, column-major, one column of lanes per cell
    __shared__ double sQ[3][K][64];       // Householder v0, beta, and diag(R)
    const int lane = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    if (i >= a.N) return;                 // lanes only touch their own LDS column: no barriers needed
    auto put = [&](int e, double v) {
        a.P64[avix(i, e, a.E64, 2)] = v;
        if (a.P32) a.P32[avix(i, e, a.E32, 4)] = (float)v;
    };

    const double x0 = a.verts[tix(i, 0, 6)], y0 = a.verts[tix(i, 1, 6)];
    const double ja = a.verts[tix(i, 2, 6)] - x0, jc = a.verts[tix(i, 3, 6)] - y0;
    const double jb = a.verts[tix(i, 4, 6)] - x0, jd = a.verts[tix(i, 5, 6)] - y0;
    const double det = ja * jd - jb * jc;

    double wrow[S];
    double dA[3][4][2], dW[3][4];
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const uint8_t fl = a.slot_flag[tix(i, j, S)];
        double row[K];
#pragma unroll
        for (int k = 0; k < K; ++k) row[k] = 0.0;
        double w = 0.0;
        if (fl & 1) {
            const int64_t m = a.slot[avix(i, j, SP, 4)];
            const double sx = a.slot_shift[tix(i, 2 * j, 2 * S)] * a.Lx;
            const double sy = a.slot_shift[tix(i, 2 * j + 1, 2 * S)] * a.Ly;
            double X[3], Y[3];
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                const double px = (a.verts[tix(m, 2 * v, 6)] + sx) - x0;
                const double py = (a.verts[tix(m, 2 * v + 1, 6)] + sy) - y0;
                X[v] = (jd * px - jb * py) / det;
                Y[v] = (-jc * px + ja * py) / det;
            }
            const double ar = 0.5 * fabs((X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]));
            double mom[K];
#pragma unroll
            for (int k = 0; k < K; ++k) mom[k] = 0.0;
#pragma unroll
            for (int p = 0; p < 16; ++p) {
                const double xi = X[0] + a.q.s[p] * (X[1] - X[0]) + a.q.t[p] * (X[2] - X[0]);
                const double et = Y[0] + a.q.s[p] * (Y[1] - Y[0]) + a.q.t[p] * (Y[2] - Y[0]);
                double px[R + 1], py[R + 1];
                px[0] = py[0] = 1.0;
#pragma unroll
                for (int e = 1; e <= R; ++e) { px[e] = px[e - 1] * xi; py[e] = py[e - 1] * et; }
#pragma unroll
                for (int k = 0; k < K; ++k) mom[k] += a.q.w[p] * (px[a.ex[k][0]] * py[a.ex[k][1]]);
            }
            // int_{V'_m} psi_k = 2 |V'_m| sum_p w_p psi_k(x_p);  A_mk = that - |V'_m| mean(psi_k)
#pragma unroll
            for (int k = 0; k < K; ++k) row[k] = 2.0 * ar * mom[k] - ar * a.mean[k];
            w = ar;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) sA[k * S + j][lane] = row[k];
        wrow[j] = w;
        if (j < 12) {
            const bool dm = (fl & 2) != 0;
            dA[j / 4][j % 4][0] = dm ? row[0] : 0.0;
            dA[j / 4][j % 4][1] = dm ? row[1] : 0.0;
            dW[j / 4][j % 4] = dm ? w : 0.0;
        }
    }

    // Householder QR of the S x K matrix (zero rows for padding slots)
    double rmax = 0.0;
    for (int j = 0; j < K; ++j) {
        double nrm2 = 0.0;
        for (int r2 = j; r2 < S; ++r2) { const double x = sA[j * S + r2][lane]; nrm2 += x * x; }
        const double nrm = sqrt(nrm2);
        const double xj = sA[j * S + j][lane];
        const double alpha = xj > 0 ? -nrm : nrm;
        const double v0 = xj - alpha;
        double vv = v0 * v0;
        for (int r2 = j + 1; r2 < S; ++r2) { const double x = sA[j * S + r2][lane]; vv += x * x; }
        const double beta = vv > 0 ? 2.0 / vv : 0.0;
        sQ[0][j][lane] = v0;
        sQ[1][j][lane] = beta;
        sQ[2][j][lane] = alpha;
        rmax = fmax(rmax, fabs(alpha));
        for (int k2 = j + 1; k2 < K; ++k2) {
            double s = v0 * sA[k2 * S + j][lane];
            for (int r2 = j + 1; r2 < S; ++r2) s += sA[j * S + r2][lane] * sA[k2 * S + r2][lane];
            s *= beta;
            sA[k2 * S + j][lane] -= s * v0;
            for (int r2 = j + 1; r2 < S; ++r2) sA[k2 * S + r2][lane] -= s * sA[j * S + r2][lane];
        }
    }
    bool rank_ok = rmax > 0.0;
    for (int j = 0; j < K; ++j) rank_ok = rank_ok && fabs(sQ[2][j][lane]) > 1e-12 * rmax;
    if (!rank_ok) atomicAdd(a.rank_fail, 1);

    // P(:, m) = R^-1 Q^T (w_m e_m)
#pragma unroll 1
    for (int m = 0; m < S; ++m) {
        double b[S];
#pragma unroll
        for (int r2 = 0; r2 < S; ++r2) b[r2] = (r2 == m) ? wrow[r2] : 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const double v0 = sQ[0][j][lane];
            double s = v0 * b[j];
#pragma unroll
            for (int r2 = j + 1; r2 < S; ++r2) s += sA[j * S + r2][lane] * b[r2];
            s *= sQ[1][j][lane];
            b[j] -= s * v0;
#pragma unroll
            for (int r2 = j + 1; r2 < S; ++r2) b[r2] -= s * sA[j * S + r2][lane];
        }
        double x[K];
#pragma unroll
        for (int j = K - 1; j >= 0; --j) {
            double s = b[j];
#pragma unroll
            for (int k2 = j + 1; k2 < K; ++k2) s -= sA[k2 * S + j][lane] * x[k2];
            x[j] = s / sQ[2][j][lane];
        }
        const int off = pinv_offset(m, K);
#pragma unroll
        for (int k = 0; k < K; ++k) put(off + k, rank_ok ? x[k] : 0.0);
    }

    // directional 4 x 2 systems in registers
    uint8_t fl = a.flags[i];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        double A[4][2], v0[2], bt[2], rd[2];
#pragma unroll
        for (int t = 0; t < 4; ++t) { A[t][0] = dA[s][t][0]; A[t][1] = dA[s][t][1]; }
        double dmax = 0.0;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            double nrm2 = 0.0;
#pragma unroll
            for (int r2 = j; r2 < 4; ++r2) nrm2 += A[r2][j] * A[r2][j];
            const double nrm = sqrt(nrm2);
            const double alpha = A[j][j] > 0 ? -nrm : nrm;
            const double vj = A[j][j] - alpha;
            double vv = vj * vj;
#pragma unroll
            for (int r2 = j + 1; r2 < 4; ++r2) vv += A[r2][j] * A[r2][j];
            const double beta = vv > 0 ? 2.0 / vv : 0.0;
            v0[j] = vj; bt[j] = beta; rd[j] = alpha;
            dmax = fmax(dmax, fabs(alpha));
#pragma unroll
            for (int k2 = j + 1; k2 < 2; ++k2) {
                double sm = vj * A[j][k2];
#pragma unroll
                for (int r2 = j + 1; r2 < 4; ++r2) sm += A[r2][j] * A[r2][k2];
                sm *= beta;
                A[j][k2] -= sm * vj;
#pragma unroll
                for (int r2 = j + 1; r2 < 4; ++r2) A[r2][k2] -= sm * A[r2][j];
            }
        }
        bool ok = ((fl >> s) & 1) && dmax > 0.0 && fabs(rd[0]) > 1e-12 * dmax && fabs(rd[1]) > 1e-12 * dmax;
        if (!ok) fl &= (uint8_t)~(1u << s);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            double b[4];
#pragma unroll
            for (int r2 = 0; r2 < 4; ++r2) b[r2] = (r2 == m) ? dW[s][r2] : 0.0;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                double sm = v0[j] * b[j];
#pragma unroll
                for (int r2 = j + 1; r2 < 4; ++r2) sm += A[r2][j] * b[r2];
                sm *= bt[j];
                b[j] -= sm * v0[j];
#pragma unroll
                for (int r2 = j + 1; r2 < 4; ++r2) b[r2] -= sm * A[r2][j];
            }
            const double x1 = ok ? b[1] / rd[1] : 0.0;
            const double x0v = ok ? (b[0] - A[0][1] * x1) / rd[0] : 0.0;
            const int off = pinv_offset(4 * s + m, K) + K;
            put(off, x0v);
            put(off + 1, x1);
        }
    }
    a.flags[i] = fl;
}

static void gauss_legendre4(double x[4], double w[4]) {
    // roots of P_4 by Newton iteration from the Chebyshev guesses
    for (int k = 0; k < 4; ++k) {
        double z = cos(M_PI * (k + 0.75) / 4.5);
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int n = 2; n <= 4; ++n) { double p2 = ((2 * n - 1) * z * p1 - (n - 1) * p0) / n; p0 = p1; p1 = p2; }
            double dp = 4 * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-17) break;
        }
        double p0 = 1.0, p1 = z;
        for (int n = 2; n <= 4; ++n) { double p2 = ((2 * n - 1) * z * p1 - (n - 1) * p0) / n; p0 = p1; p1 = p2; }
        double dp = 4 * (z * p1 - p0) / (z * z - 1.0);
        x[k] = z;
        w[k] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// collapsed 4 x 4 Gauss-Legendre rule on the reference triangle (exact to
// degree 6, the highest monomial degree of the basis)
static void fill_quad_rule(QuadRule &q) {
    double x[4], w[4];
    gauss_legendre4(x, w);
    int p = 0;
    for (int u = 0; u < 4; ++u)
        for (int v = 0; v < 4; ++v) {
            double su = 0.5 * (x[u] + 1.0), sv = 0.5 * (x[v] + 1.0);
            q.s[p] = su;
            q.t[p] = sv * (1.0 - su);
            q.w[p] = 0.25 * w[u] * w[v] * (1.0 - su);
            ++p;
        }
}

template <int R>
static hipError_t precompute_ho_r(const DeviceMesh &m, const PrecomputeInputs &in, hipStream_t st);

template <int R>
static hipError_t precompute_r(const DeviceMesh &m, const PrecomputeInputs &in, hipStream_t st) {
    PreArgs<R> a;
    a.N = m.N;
    a.verts = in.verts; a.slot = m.slot; a.slot_flag = in.slot_flag; a.slot_shift = in.slot_shift;
    a.flags = in.flags; a.rank_fail = in.rank_fail;
    a.P64 = m.P64; a.P32 = m.P32; a.E64 = m.E64; a.E32 = m.E32;
    a.Lx = m.Lx; a.Ly = m.Ly;
    for (int k = 0; k < PreArgs<R>::K; ++k) {
        a.ex[k][0] = m.tab.ex[k][0];
        a.ex[k][1] = m.tab.ex[k][1];
        a.mean[k] = m.tab.mean[k];
    }
    fill_quad_rule(a.q);
    const unsigned grid = (unsigned)((m.N + 63) / 64);
    hipLaunchKernelGGL(k_precompute<R>, dim3(grid), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_precompute(const DeviceMesh &m, const PrecomputeInputs &in, hipStream_t st) {
    switch (m.r) {
        case 2: return precompute_r<2>(m, in, st);
        case 3: return precompute_r<3>(m, in, st);
        case 4: return precompute_ho_r<4>(m, in, st);
        case 5: return precompute_ho_r<5>(m, in, st);
        case 6: return precompute_ho_r<6>(m, in, st);
        default: return hipErrorInvalidValue;
    }
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
            for (int s = 0; s < 4; ++s) g[s] = 1.0 + tau / (si[s] + eps);
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
        float e[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) e[s] = si[s] + eps;
        if (SCHEME == CTENO_SCHEME_CTENO) {
            // chi_s = 1 / sum_t (lambda_t / lambda_s) (e_s / e_t)^6
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                if (!((adm >> s) & 1)) continue;
                float den = 0.0f;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (!((adm >> t) & 1)) continue;
                    float lr = 1.0f;
                    if (GFORM == CTENO_GAMMA_LAMBDA && s != t) lr = (t == 0) ? lratio : (s == 0 ? 1.0f / lratio : 1.0f);
                    den += lr * pow6(e[s] / e[t]);
                }
                const float chi = 1.0f / den;
                if (!(chi < ct)) bits |= 1 << s;
            }
        } else {
            float tsum = 0.0f, emin = e[0];
#pragma unroll
            for (int s = 1; s < 4; ++s)
                if ((adm >> s) & 1) { tsum += fabsf(e[s] - e[0]); emin = fminf(emin, e[s]); }
            const float tau = pow6(tsum / (float)(st - 1));
            const float G = tau / emin;            // gamma_s = 1 + G w_s, w_s = emin / e_s in (0, 1]
            float num[4], sum = 0.0f;
            if (G <= 1e30f) {
#pragma unroll
                for (int s = 0; s < 4; ++s) num[s] = 1.0f + G * (emin / e[s]);
            } else {
                const float iG = 1.0f / G;
#pragma unroll
                for (int s = 0; s < 4; ++s) num[s] = iG + emin / e[s];
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) if ((adm >> s) & 1) sum += num[s];
#pragma unroll
            for (int s = 0; s < 4; ++s)
                if ((adm >> s) & 1) {
                    const float chi = num[s] / sum;
                    if (!(chi < ct)) bits |= 1 << s;
                }
        }
    }
    return bits;
}

// CWENO nonlinear weights (sec. 2.2: the WENO weights with exponent 4 and
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
        float e[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) e[s] = si[s] + eps;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            float den = 0.0f;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (!((adm >> t) & 1)) continue;
                const float lr = (s == t) ? 1.0f : (t == 0 ? lratio : (s == 0 ? 1.0f / lratio : 1.0f));
                const float q = e[s] / e[t], q2 = q * q;
                den += lr * (q2 * q2);
            }
            w[s] = ((adm >> s) & 1) ? 1.0f / den : 0.0f;
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
};

// selection (or CWENO weights) of NV fields and their final coefficients,
// in place: c1[K][NV] holds the p_1 coefficients on entry and the final
// polynomial's on exit, cd[3][2][NV] the degree-1 directional ones; forced
// (DMODE 2) points at the fields' forced selection bytes
template <typename real, int K, int NV, int SCHEME, int GFORM, int DMODE>
__device__ __forceinline__ void finish_fields(const ReconArgs<real, K> a, real (&c1)[K][NV], const real (&cd)[3][2][NV],
                                              int fl, int adm, int st, real lams, real lratio, const uint8_t *forced,
                                              int (&bits)[NV]) {
    if (DMODE == 2 && SCHEME != CTENO_SCHEME_CWENO) {
#pragma unroll
        for (int v = 0; v < NV; ++v) bits[v] = forced[v] & adm;
    } else if (st == 1) {
#pragma unroll
        for (int v = 0; v < NV; ++v) bits[v] = 1;
    } else {
        // smoothness indicators: SI_1 = a1^T G a1, SI_s over the degree-1 block of G
        real si[NV][4];
#pragma unroll
        for (int v = 0; v < NV; ++v) si[v][0] = 0;
#pragma unroll
        for (int p = 0; p < K; ++p) {
            real rowp[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) rowp[v] = 0;
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const real g = a.gram[p][q];
#pragma unroll
                for (int v = 0; v < NV; ++v) rowp[v] += g * c1[q][v];
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) si[v][0] += c1[p][v] * rowp[v];
        }
        const real g00 = a.gram[0][0], g01 = a.gram[0][1], g10 = a.gram[1][0], g11 = a.gram[1][1];
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const real x0 = cd[q][0][v], x1 = cd[q][1][v];
                si[v][q + 1] = x0 * (g00 * x0 + g01 * x1) + x1 * (g10 * x0 + g11 * x1);
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
                            if ((fl >> q) & 1) x += w[q + 1] * cd[q][k][v];
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
                if ((bits[v] >> (q + 1)) & 1) { s0 += cd[q][0][v]; s1 += cd[q][1][v]; ++cnt; }
            c1[0][v] = s0 / (real)cnt;
            c1[1][v] = s1 / (real)cnt;
#pragma unroll
            for (int k = 2; k < K; ++k) c1[k][v] = 0;
        }
    }
}

template <typename real, int R, int NV, int SCHEME, int GFORM, int DMODE, int VARS>
__device__ __forceinline__ void recon_body(const ReconArgs<real, (R + 1) * (R + 2) / 2 - 1> a,
                                           const ReconPtrs<real> ptr, int64_t i) {
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
    // Rolled loop over the three directional groups with a two-deep load
    // pipeline: the GV vectors that follow group s (group s + 1, or the head
    // of the remaining slots) are requested before group s is computed, so a
    // wave keeps two groups of stream loads in flight.  With no remaining
    // slots (S = 12) the last iteration requests its own group again.
    constexpr int NVEC = E / VW;
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
    // p_1 = (p_opt - sum_s lambda_s p_s) / lambda_1, in place of a_opt
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            real sm = ao[k][v];
            if (k < 2 && st > 1) {
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    if ((fl >> q) & 1) sm -= lams * ad[q][k][v];
            }
            // TENO keeps the central stencil's own polynomial
            if (SCHEME != CTENO_SCHEME_TENO) ao[k][v] = st > 1 ? sm / a.lam1 : sm;
        }
    real out[3][2][NV];
    constexpr int NB = VARS ? 3 * NV : NV;       // selection bytes per cell
    uint8_t dbyte[NB];
    if constexpr (VARS == 0) {
        int bits[NV];
        finish_fields<real, K, NV, SCHEME, GFORM, DMODE>(a, ao, ad, fl, adm, st, lams, lratio, ptr.delta + i * NV,
                                                         bits);
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
                    const real b = a.basis[f][q][k];
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
        const real cs = sqrt(a.gamma * pr / rho), H = ((real)U0[3] + pr) / rho;
        const real b1 = (a.gamma - 1) / (cs * cs), b2 = b1 * q2, ic = (real)1 / cs;
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
                        for (int v = 0; v < 4; ++v) x += L[j][v] * ad[s2][k][v];
                        cd[s2][k][j] = x;
                    }
            int bits[4];
            finish_fields<real, K, 4, SCHEME, GFORM, DMODE>(a, c1, cd, fl, adm, st, lams, lratio,
                                                            ptr.delta + (i * 3 + f) * 4, bits);
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
    if constexpr (NV == 4) {
        // positivity fallback: a cell with a non-physical state (density or
        // pressure <= 0) at any of its Gauss points uses its cell average at
        // all of them; reported with bit 7 of its selection bytes
        bool bad = false;
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const real rho = out[f][q][0];
                const real pr = (a.gamma - 1) * (out[f][q][3] - (real)0.5 * (out[f][q][1] * out[f][q][1] +
                                                                             out[f][q][2] * out[f][q][2]) / rho);
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
        }
    }
    if (DMODE == 1) {
#pragma unroll
        for (int k = 0; k < NB; ++k) ptr.delta[i * NB + k] = dbyte[k];
    }
    store_row<real, 3 * 2 * NV>(ptr.FV + i * 3 * 2 * NV, &out[0][0][0]);
}

template <typename real, int R, int NV, int SCHEME, int GFORM, int DMODE, int VARS>
__global__ __launch_bounds__(256) void k_reconstruct(const ReconArgs<real, (R + 1) * (R + 2) / 2 - 1> a) {
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    if (a.done && *a.done) return;
    const ReconPtrs<real> ptr{a.U, a.slot, a.flags, a.P, a.FV, a.delta, a.fr};
    recon_body<real, R, NV, SCHEME, GFORM, DMODE, VARS>(a, ptr, i);
}

// scheme constants of the reconstruction (tables of the reference triangle,
// linear weights of eq. e18 for every admissible-stencil count)
template <typename real, int K>
static void fill_recon_constants(const DeviceMesh &m, ReconArgs<real, K> &a) {
    a.N = m.N;
    for (int p = 0; p < K; ++p)
        for (int q = 0; q < K; ++q) a.gram[p][q] = (real)m.tab.gram[p][q];
    for (int f = 0; f < 3; ++f)
        for (int q = 0; q < 2; ++q)
            for (int k = 0; k < K; ++k) a.basis[f][q][k] = (real)m.tab.basis[f][q][k];
    const double lam1 = 1.0 - 1.0 / m.lam1p;
    a.lam1 = (real)lam1;
    a.gamma = (real)m.gamma;
    a.ct = (real)m.ct;
    a.eps = (real)m.eps;
    for (int s = 0; s < 5; ++s) {
        const double ls = s >= 2 ? (1.0 - lam1) / (s - 1) : 0.0;
        a.lams[s] = (real)ls;
        a.lam_ratio[s] = s >= 2 ? (real)(lam1 / ls) : (real)1;
    }
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
    if (m.scheme == CTENO_SCHEME_CTENOZ) { CT_DM(CTENO_SCHEME_CTENOZ, CTENO_GAMMA_PAPER); }
    else if (m.scheme == CTENO_SCHEME_CWENO) { CT_DM(CTENO_SCHEME_CWENO, CTENO_GAMMA_PAPER); }
    else if (m.scheme == CTENO_SCHEME_TENO) { CT_DM(CTENO_SCHEME_TENO, CTENO_GAMMA_PAPER); }
    else if (m.gamma_form == CTENO_GAMMA_LAMBDA) { CT_DM(CTENO_SCHEME_CTENO, CTENO_GAMMA_LAMBDA); }
    else { CT_DM(CTENO_SCHEME_CTENO, CTENO_GAMMA_PAPER); }
#undef CT_DM
#undef CT_LAUNCH
}

template <typename real, int R, int NV>
static hipError_t reconstruct_t(const DeviceMesh &m, const double *U, void *FV, uint8_t *delta, int dmode,
                                const int *done, hipStream_t st) {
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
static hipError_t reconstruct_p(const DeviceMesh &m, const double *U, void *FV, uint8_t *delta, int dmode,
                                const int *done, hipStream_t st) {
    if (m.nv == 4) {
        switch (m.r) {
            case 2: return reconstruct_t<real, 2, 4>(m, U, FV, delta, dmode, done, st);
            case 3: return reconstruct_t<real, 3, 4>(m, U, FV, delta, dmode, done, st);
        }
    } else {
        switch (m.r) {
            case 2: return reconstruct_t<real, 2, 1>(m, U, FV, delta, dmode, done, st);
            case 3: return reconstruct_t<real, 3, 1>(m, U, FV, delta, dmode, done, st);
        }
    }
    return hipErrorInvalidValue;
}

template <typename real>
static hipError_t reconstruct_ho_p(const DeviceMesh &m, const double *U, void *FV, uint8_t *delta, int dmode,
                                   const int *done, hipStream_t st);

hipError_t launch_reconstruct(const DeviceMesh &m, bool fp32, const double *U, void *FV, uint8_t *delta, int dmode,
                              const int *done, hipStream_t st) {
    if (m.r >= 4)
        return fp32 ? reconstruct_ho_p<float>(m, U, FV, delta, dmode, done, st)
                    : reconstruct_ho_p<double>(m, U, FV, delta, dmode, done, st);
    return fp32 ? reconstruct_p<float>(m, U, FV, delta, dmode, done, st)
                : reconstruct_p<double>(m, U, FV, delta, dmode, done, st);
}

// ===========================================================================
// orders 5 to 7 (r = 4..6)
// ===========================================================================
// The pseudo-inverse stream of a cell has S = 3 M_d slots (the three
// directional groups cover the whole central stencil) of EPS entries: K
// central, K_d directional, zero padding to a multiple of 4.  It is
// vector-tiled with tiles of CT = 64 / nv cells: the reconstruction runs one
// lane per (cell, variable), so a wave covers CT cells and its lanes of one
// cell read the same 16-byte vector.

// sum over the wave; the butterfly adds the same pairs in every lane, so all
// lanes hold bitwise the same result
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

template <int R>
struct HoDims {
    static constexpr int K = (R + 1) * (R + 2) / 2 - 1;
    static constexpr int RD = (R + 1) / 2;
    static constexpr int KD = (RD + 1) * (RD + 2) / 2 - 1;
    static constexpr int MD = 2 * KD;
    static constexpr int S = 3 * MD;
    static constexpr int SP = (S + 3) / 4 * 4;
    static constexpr int EPS = (K + KD + 3) / 4 * 4;
    static constexpr int E = S * EPS;
    static constexpr int NQ = (R + 2) / 2;
    static_assert(S >= 2 * K, "the directional groups must hold the central stencil");
    static_assert(S <= 64, "one lane per least-squares row");
};

template <int R>
struct PreHoArgs {
    using D = HoDims<R>;
    int64_t N;
    const double *verts;
    const int32_t *slot;
    const uint8_t *slot_flag;
    const int8_t *slot_shift;
    uint8_t *flags;
    int *rank_fail;
    double *P64;
    float *P32;
    int ct;                  // cells per stream tile
    double Lx, Ly;
    int ex[D::K][2];
    double mean[D::K];
    QuadRule q;
};

// One wave per cell, one lane per least-squares row (slot).  Householder QR
// (sec. 2.1) of the S x K central system and of the three M_d x K_d
// directional systems; P = R^-1 Q^T diag(|V'_m|), column by column.
template <int R>
__global__ __launch_bounds__(256) void k_precompute_ho(const PreHoArgs<R> a) {
    using D = HoDims<R>;
    constexpr int K = D::K, KD = D::KD, MD = D::MD, S = D::S, SP = D::SP, EPS = D::EPS, E = D::E;
    __shared__ double sA[4][K][64];       // central system, column-major, row = lane
    __shared__ double sD[4][KD][64];      // directional systems (disjoint rows)
    __shared__ double sH[4][3][K];        // central v0, beta, diag(R)
    __shared__ double sHd[4][3][3][KD];   // directional v0, beta, diag(R)
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + wv;
    if (i >= a.N) return;                 // whole waves; a wave only touches its own LDS
    double (*cA)[64] = sA[wv];
    double (*cD)[64] = sD[wv];
    auto put = [&](int e, double v) {
        a.P64[hvix(i, e, E, 2, a.ct)] = v;
        if (a.P32) a.P32[hvix(i, e, E, 4, a.ct)] = (float)v;
    };

    // reference map of cell i: v0 and J = [v1 - v0, v2 - v0]
    const double x0 = a.verts[tix(i, 0, 6)], y0 = a.verts[tix(i, 1, 6)];
    const double ja = a.verts[tix(i, 2, 6)] - x0, jc = a.verts[tix(i, 3, 6)] - y0;
    const double jb = a.verts[tix(i, 4, 6)] - x0, jd = a.verts[tix(i, 5, 6)] - y0;
    const double det = ja * jd - jb * jc;

    // row of slot `lane`: A_mk = int_{V'_m} psi_k - |V'_m| mean(psi_k)
    uint8_t fl = 0;
    double w = 0.0;
    double row[K];
#pragma unroll
    for (int k = 0; k < K; ++k) row[k] = 0.0;
    if (lane < S) {
        fl = a.slot_flag[tix(i, lane, S)];
        if (fl & 1) {
            const int64_t m = a.slot[avix(i, lane, SP, 4)];
            const double sx = a.slot_shift[tix(i, 2 * lane, 2 * S)] * a.Lx;
            const double sy = a.slot_shift[tix(i, 2 * lane + 1, 2 * S)] * a.Ly;
            double X[3], Y[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double px = (a.verts[tix(m, 2 * c, 6)] + sx) - x0;
                const double py = (a.verts[tix(m, 2 * c + 1, 6)] + sy) - y0;
                X[c] = (jd * px - jb * py) / det;
                Y[c] = (-jc * px + ja * py) / det;
            }
            const double ar = 0.5 * fabs((X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]));
            double mom[K];
#pragma unroll
            for (int k = 0; k < K; ++k) mom[k] = 0.0;
#pragma unroll 1
            for (int p = 0; p < 16; ++p) {
                const double xi = X[0] + a.q.s[p] * (X[1] - X[0]) + a.q.t[p] * (X[2] - X[0]);
                const double et = Y[0] + a.q.s[p] * (Y[1] - Y[0]) + a.q.t[p] * (Y[2] - Y[0]);
                double px[R + 1], py[R + 1];
                px[0] = py[0] = 1.0;
#pragma unroll
                for (int e = 1; e <= R; ++e) { px[e] = px[e - 1] * xi; py[e] = py[e - 1] * et; }
#pragma unroll
                for (int k = 0; k < K; ++k) mom[k] += a.q.w[p] * (px[a.ex[k][0]] * py[a.ex[k][1]]);
            }
#pragma unroll
            for (int k = 0; k < K; ++k) row[k] = 2.0 * ar * mom[k] - ar * a.mean[k];
            w = ar;
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) cA[k][lane] = row[k];
#pragma unroll
    for (int k = 0; k < KD; ++k) cD[k][lane] = (fl & 2) ? row[k] : 0.0;
    const double wc = w, wd = (fl & 2) ? w : 0.0;
    __builtin_amdgcn_wave_barrier();

    // central Householder QR; column k's tail (rows > k) keeps the reflector
    double amax = 0.0;
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
        const double x = lane >= k ? cA[k][lane] : 0.0;
        const double nrm = sqrt(wave_sum(x * x));
        const double xk = cA[k][k];
        const double alpha = xk > 0 ? -nrm : nrm;
        const double v = lane == k ? xk - alpha : x;
        const double vv = wave_sum(v * v);
        const double beta = vv > 0 ? 2.0 / vv : 0.0;
        if (lane == 0) { sH[wv][0][k] = xk - alpha; sH[wv][1][k] = beta; sH[wv][2][k] = alpha; }
        amax = fmax(amax, fabs(alpha));
#pragma unroll 1
        for (int c = k + 1; c < K; ++c) {
            const double y = cA[c][lane];
            const double sm = beta * wave_sum(v * y);
            cA[c][lane] = y - sm * v;
        }
        __builtin_amdgcn_wave_barrier();
    }
    bool rank_ok = amax > 0.0;
#pragma unroll 1
    for (int k = 0; k < K; ++k) rank_ok = rank_ok && fabs(sH[wv][2][k]) > 1e-12 * amax;
    if (!rank_ok && lane == 0) atomicAdd(a.rank_fail, 1);

    // column m of P: apply the reflectors to w_m e_m, then back-substitute;
    // lane k ends with coefficient k
#pragma unroll 1
    for (int m = 0; m < S; ++m) {
        double b = lane == m ? wc : 0.0;
#pragma unroll 1
        for (int k = 0; k < K; ++k) {
            const double v = lane > k ? cA[k][lane] : (lane == k ? sH[wv][0][k] : 0.0);
            b -= sH[wv][1][k] * wave_sum(v * b) * v;
        }
        double xo = 0.0;
#pragma unroll 1
        for (int k = K - 1; k >= 0; --k) {
            const double xk = __shfl(b, k, 64) / sH[wv][2][k];
            if (lane == k) xo = xk;
            if (lane < k) b -= cA[k][lane] * xk;
        }
        if (lane < K) put(m * EPS + lane, rank_ok ? xo : 0.0);
    }

    // directional systems: group s owns rows [s M_d, (s+1) M_d); its members
    // come first, in directional-list order
    uint8_t flg = a.flags[i];
#pragma unroll 1
    for (int s = 0; s < 3; ++s) {
        const int base = s * MD;
        const bool in = lane >= base && lane < base + MD;
        double dmax = 0.0;
#pragma unroll 1
        for (int k = 0; k < KD; ++k) {
            const int pk = base + k;
            const double x = (in && lane >= pk) ? cD[k][lane] : 0.0;
            const double nrm = sqrt(wave_sum(x * x));
            const double xk = cD[k][pk];
            const double alpha = xk > 0 ? -nrm : nrm;
            const double v = lane == pk ? xk - alpha : x;
            const double vv = wave_sum(v * v);
            const double beta = vv > 0 ? 2.0 / vv : 0.0;
            if (lane == 0) { sHd[wv][s][0][k] = xk - alpha; sHd[wv][s][1][k] = beta; sHd[wv][s][2][k] = alpha; }
            dmax = fmax(dmax, fabs(alpha));
#pragma unroll 1
            for (int c = k + 1; c < KD; ++c) {
                const double y = cD[c][lane];
                const double sm = beta * wave_sum(v * y);
                if (in) cD[c][lane] = y - sm * v;
            }
            __builtin_amdgcn_wave_barrier();
        }
        bool ok = ((flg >> s) & 1) && dmax > 0.0;
#pragma unroll 1
        for (int k = 0; k < KD; ++k) ok = ok && fabs(sHd[wv][s][2][k]) > 1e-12 * dmax;
        if (!ok) flg &= (uint8_t)~(1u << s);
#pragma unroll 1
        for (int t = 0; t < MD; ++t) {
            const int mrow = base + t;
            double b = lane == mrow ? wd : 0.0;
#pragma unroll 1
            for (int k = 0; k < KD; ++k) {
                const double v = (in && lane > base + k) ? cD[k][lane] : (lane == base + k ? sHd[wv][s][0][k] : 0.0);
                b -= sHd[wv][s][1][k] * wave_sum(v * b) * v;
            }
            double xo = 0.0;
#pragma unroll 1
            for (int k = KD - 1; k >= 0; --k) {
                const double xk = __shfl(b, base + k, 64) / sHd[wv][s][2][k];
                if (lane == base + k) xo = xk;
                if (lane >= base && lane < base + k) b -= cD[k][lane] * xk;
            }
            if (lane >= base && lane < base + KD) put(mrow * EPS + K + (lane - base), ok ? xo : 0.0);
        }
    }
    if (lane == 0) a.flags[i] = flg;
}

template <int R>
static hipError_t precompute_ho_r(const DeviceMesh &m, const PrecomputeInputs &in, hipStream_t st) {
    using D = HoDims<R>;
    if (m.S != D::S || m.E64 != D::E || m.E32 != D::E || m.SP != D::SP) return hipErrorInvalidValue;
    PreHoArgs<R> a;
    a.N = m.N;
    a.verts = in.verts; a.slot = m.slot; a.slot_flag = in.slot_flag; a.slot_shift = in.slot_shift;
    a.flags = in.flags; a.rank_fail = in.rank_fail;
    a.P64 = m.P64; a.P32 = m.P32; a.ct = m.stile;
    a.Lx = m.Lx; a.Ly = m.Ly;
    for (int k = 0; k < D::K; ++k) {
        a.ex[k][0] = m.tab.ex[k][0];
        a.ex[k][1] = m.tab.ex[k][1];
        a.mean[k] = m.tab.mean[k];
    }
    fill_quad_rule(a.q);
    const unsigned grid = (unsigned)((m.N + 3) / 4);
    hipLaunchKernelGGL(k_precompute_ho<R>, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

// scheme constants of the higher-order reconstruction: linear weights, and a
// device table (Gram matrix [K][K], then face basis [3][N_q][K])
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
        for (int k = 0; k < KD; ++k) c1[k] /= (real)cnt;
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

// a_opt = P_c d and a_s = P_s d for the four variables of a cell held by a
// quad of lanes.  The lanes split each slot's stream instead of each reading
// all of it: lane q loads the stream vectors q, q + 4, ... and accumulates
// their coefficients for all four variables (the differences d come from
// the variable lanes by DPP moves); at the end of each directional group
// and of the loop the coefficients go to their variable lanes.  Every
// coefficient sums its slots in slot order, as a lane per variable would.
// Where the slot ends in a partial round of four scalars (r = 4 and 6: one
// float4 or two double2 vectors), lane q reads scalar q of it, so no lane
// multiplies a vector it does not own.
template <typename real, int R>
__device__ __forceinline__ void ho_contract_quad(const ReconHoArgs<real> a, int64_t i, int v, double U0,
                                                 real (&ao)[HoDims<R>::K], real (&ad)[3][HoDims<R>::KD]) {
    using D = HoDims<R>;
    constexpr int K = D::K, KD = D::KD, MD = D::MD, S = D::S, SP = D::SP, EPS = D::EPS, E = D::E;
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
    real acc[GF][VW][4], acs[4];
#pragma unroll
    for (int t = 0; t < GF; ++t)
#pragma unroll
        for (int c = 0; c < VW; ++c)
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[t][c][u] = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) acs[u] = 0;
    // this lane's entries that belong to a directional polynomial
    bool keep[GF][VW];
#pragma unroll
    for (int t = 0; t < GF; ++t)
#pragma unroll
        for (int c = 0; c < VW; ++c) {
            const int e = (4 * t + v) * VW + c;
            keep[t][c] = !(e >= K && e < K + KD);
        }
    const int es = 4 * GF * VW + v;
    const bool keeps = !(es >= K && es < K + KD);
    V cur[GF], nxt[GF];
    real cs = 0, ns = 0;
#pragma unroll
    for (int t = 0; t < GF; ++t) cur[t] = Pv[(4 * t + v) * CT];
    if constexpr (SPREAD) cs = Pr[0];
    // neighbour averages GD slots ahead (a ring), the next index one more:
    // four in FP32, where the dependent index -> average -> product chain
    // bounds the order-7 kernel (-11 %); one in FP64, where the ring's
    // registers would cost a wave per SIMD
    constexpr int GD = sizeof(real) == 4 ? 4 : 1;
    auto slot_index = [&](int j) { const int jc = j < S ? j : S - 1; return Si[(jc >> 2) * 256 + (jc & 3)]; };
    double ring[GD];
#pragma unroll
    for (int k = 0; k < GD; ++k) ring[k] = a.U[(int64_t)slot_index(k) * 4 + v];
    int mnext = slot_index(GD);
#pragma unroll 1
    for (int j = 0; j < S; ++j) {
        const int jn = j + 1 < S ? j + 1 : j;
#pragma unroll
        for (int t = 0; t < GF; ++t) nxt[t] = Pv[(jn * SV + 4 * t + v) * CT];
        if constexpr (SPREAD) ns = Pr[(size_t)jn * SV * CT * VW];
        const double ucur = ring[0];
#pragma unroll
        for (int k = 0; k < GD - 1; ++k) ring[k] = ring[k + 1];
        ring[GD - 1] = a.U[(int64_t)mnext * 4 + v];
        mnext = slot_index(j + GD + 1);
        const real dv = (real)(ucur - U0);
        const real d[4] = {quad_bcast<0>(dv), quad_bcast<1>(dv), quad_bcast<2>(dv), quad_bcast<3>(dv)};
#pragma unroll
        for (int t = 0; t < GF; ++t)
#pragma unroll
            for (int c = 0; c < VW; ++c)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[t][c][u] += comp(cur[t], c) * d[u];
        if constexpr (SPREAD) {
#pragma unroll
            for (int u = 0; u < 4; ++u) acs[u] += cs * d[u];
        }
        if (j % MD == MD - 1) {           // uniform: group j / MD is complete
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
                    for (int u = 0; u < 4; ++u) acc[t][c][u] = keep[t][c] ? acc[t][c][u] : (real)0;
#pragma unroll
            for (int u = 0; u < 4; ++u) acs[u] = keeps ? acs[u] : (real)0;
        }
#pragma unroll
        for (int t = 0; t < GF; ++t) cur[t] = nxt[t];
        cs = ns;
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
    // next slot's stream vectors and index are requested before the current
    // slot is used
    real adt[KD];
#pragma unroll
    for (int k = 0; k < K; ++k) ao[k] = 0;
#pragma unroll
    for (int k = 0; k < KD; ++k) { adt[k] = 0; ad[0][k] = 0; ad[1][k] = 0; ad[2][k] = 0; }
    V cur[SV];
#pragma unroll
    for (int g = 0; g < SV; ++g) cur[g] = Pv[g * CT];
    int mcur = Si[0];
#pragma unroll 1
    for (int j = 0; j < S; ++j) {
        const int jn = j + 1 < S ? j + 1 : j;
        V nxt[SV];
#pragma unroll
        for (int g = 0; g < SV; ++g) nxt[g] = Pv[(jn * SV + g) * CT];
        const int mn = Si[(jn >> 2) * 256 + (jn & 3)];
        const real d = (real)(a.U[(int64_t)mcur * NV + v] - U0);
#pragma unroll
        for (int k = 0; k < K; ++k) ao[k] += comp(cur[k / VW], k % VW) * d;
#pragma unroll
        for (int k = 0; k < KD; ++k) adt[k] += comp(cur[(K + k) / VW], (K + k) % VW) * d;
        if (j % MD == MD - 1) {           // uniform: group j / MD is complete
            const int s = j / MD;
#pragma unroll
            for (int s2 = 0; s2 < 3; ++s2)
                if (s2 == s)
#pragma unroll
                    for (int k = 0; k < KD; ++k) ad[s2][k] = adt[k];
#pragma unroll
            for (int k = 0; k < KD; ++k) adt[k] = 0;
        }
#pragma unroll
        for (int g = 0; g < SV; ++g) cur[g] = nxt[g];
        mcur = mn;
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
        const real ls = lams * a.p1_ls;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            real sm = ao[k];
            if (k < KD && st > 1) {
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    if ((fl >> q) & 1) sm -= ls * ad[q][k];
            }
            ao[k] = st > 1 ? sm / a.p1_l1 : sm;
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
        const real cs = sqrt(a.gamma * pr / rho), H = ((real)Ud[3] + pr) / rho;
        const real b1 = (a.gamma - 1) / (cs * cs), b2 = b1 * q2, ic = (real)1 / cs;
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
    if constexpr (NV == 4) {
        // positivity fallback (density or pressure <= 0 at a Gauss point):
        // the four lanes of the cell exchange their values
        const int l0 = (threadIdx.x & 63) & ~3;
        bool bad = false;
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const real r0 = __shfl(out[f][q], l0, 64), r1 = __shfl(out[f][q], l0 + 1, 64);
                const real r2 = __shfl(out[f][q], l0 + 2, 64), r3 = __shfl(out[f][q], l0 + 3, 64);
                const real pr = (a.gamma - 1) * (r3 - (real)0.5 * (r1 * r1 + r2 * r2) / r0);
                bad |= !(r0 > 0) || !(pr > 0);
            }
        if (bad) {
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int q = 0; q < NQ; ++q) out[f][q] = (real)U0;
#pragma unroll
            for (int k = 0; k < NB; ++k) dbyte[k] |= 0x80;
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
                                   const int *done, hipStream_t st) {
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
    if (m.scheme == CTENO_SCHEME_CTENOZ) { HO_DM(CTENO_SCHEME_CTENOZ, CTENO_GAMMA_PAPER); }
    else if (m.scheme == CTENO_SCHEME_CWENO) { HO_DM(CTENO_SCHEME_CWENO, CTENO_GAMMA_PAPER); }
    else if (m.scheme == CTENO_SCHEME_TENO) { HO_DM(CTENO_SCHEME_TENO, CTENO_GAMMA_PAPER); }
    else if (m.gamma_form == CTENO_GAMMA_LAMBDA) { HO_DM(CTENO_SCHEME_CTENO, CTENO_GAMMA_LAMBDA); }
    else { HO_DM(CTENO_SCHEME_CTENO, CTENO_GAMMA_PAPER); }
#undef HO_DM
#undef HO_LAUNCH
    return hipGetLastError();
}

template <typename real>
static hipError_t reconstruct_ho_p(const DeviceMesh &m, const double *U, void *FV, uint8_t *delta, int dmode,
                                   const int *done, hipStream_t st) {
    if (m.nv == 4) {
        switch (m.r) {
            case 4: return reconstruct_ho_t<real, 4, 4>(m, U, FV, delta, dmode, done, st);
            case 5: return reconstruct_ho_t<real, 5, 4>(m, U, FV, delta, dmode, done, st);
            case 6: return reconstruct_ho_t<real, 6, 4>(m, U, FV, delta, dmode, done, st);
        }
    } else {
        switch (m.r) {
            case 4: return reconstruct_ho_t<real, 4, 1>(m, U, FV, delta, dmode, done, st);
            case 5: return reconstruct_ho_t<real, 5, 1>(m, U, FV, delta, dmode, done, st);
            case 6: return reconstruct_ho_t<real, 6, 1>(m, U, FV, delta, dmode, done, st);
        }
    }
    return hipErrorInvalidValue;
}

// ===========================================================================
// fluxes, residual, Runge-Kutta
// ===========================================================================

// HLLC with Roe-averaged signal speeds (sec. 2.6), in the face-normal frame
// (u normal, w tangential velocity); F returned in the global frame.
template <typename real>
__device__ __forceinline__ bool hllc(real g, const real *UL, const real *UR, real nx, real ny, real *F) {
    const real rl = UL[0], rr = UR[0];
    const real ul = (UL[1] * nx + UL[2] * ny) / rl, wl = (-UL[1] * ny + UL[2] * nx) / rl;
    const real ur = (UR[1] * nx + UR[2] * ny) / rr, wr = (-UR[1] * ny + UR[2] * nx) / rr;
    const real El = UL[3], Er = UR[3];
    const real h = (real)0.5;
    const real pl = (g - 1) * (El - h * rl * (ul * ul + wl * wl));
    const real pr = (g - 1) * (Er - h * rr * (ur * ur + wr * wr));
    const bool ok = rl > 0 && rr > 0 && pl > 0 && pr > 0;
    const real cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
    const real Hl = (El + pl) / rl, Hr = (Er + pr) / rr;
    const real D = sqrt(rr / rl);
    const real ut = (ul + ur * D) / (1 + D);
    const real wt = (wl + wr * D) / (1 + D);
    const real Ht = (Hl + Hr * D) / (1 + D);
    const real ct = sqrt((g - 1) * (Ht - h * (ut * ut + wt * wt)));
    const real SL = fmin(ul - cl, ut - ct);
    const real SR = fmax(ur + cr, ut + ct);
    const real SM = (rr * ur * (SR - ur) - rl * ul * (SL - ul) + pl - pr) / (rr * (SR - ur) - rl * (SL - ul));
    const real ps = rl * (ul - SL) * (ul - SM) + pl;
    real Fn[4];
    if (SL > 0) {
        Fn[0] = rl * ul; Fn[1] = rl * ul * ul + pl; Fn[2] = rl * ul * wl; Fn[3] = ul * (El + pl);
    } else if (0 < SM) {
        const real d = SL - SM;
        const real Us0 = rl * (SL - ul) / d;
        const real Us1 = ((SL - ul) * rl * ul + ps - pl) / d;
        const real Us2 = (SL - ul) * rl * wl / d;
        const real Us3 = ((SL - ul) * El - pl * ul + ps * SM) / d;
        Fn[0] = rl * ul + SL * (Us0 - rl);
        Fn[1] = (rl * ul * ul + pl) + SL * (Us1 - rl * ul);
        Fn[2] = rl * ul * wl + SL * (Us2 - rl * wl);
        Fn[3] = ul * (El + pl) + SL * (Us3 - El);
    } else if (0 < SR) {
        const real d = SR - SM;
        const real Us0 = rr * (SR - ur) / d;
        const real Us1 = ((SR - ur) * rr * ur + ps - pr) / d;
        const real Us2 = (SR - ur) * rr * wr / d;
        const real Us3 = ((SR - ur) * Er - pr * ur + ps * SM) / d;
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
    const real u = (UL[1] * nx + UL[2] * ny) / r, w = (-UL[1] * ny + UL[2] * nx) / r;
    const real E = UL[3];
    const real p = (g - 1) * (E - (real)0.5 * r * (u * u + w * w));
    const bool ok = r > 0 && p > 0;
    const real c = sqrt(g * p / r);
    const real H = (E + p) / r;
    const real ct = sqrt((g - 1) * (H - (real)0.5 * w * w));
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
    Ctrl *ctrl;
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
};

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
    Ctrl *ctrl;
    bool want_dt;
};

// one cell's three faces, residual and (MODE 2) RK stage; returns the cell's
// CFL bound of the new state when requested, else +inf
template <typename real, int NV, int PHYS, int MODE, int NQ>
__device__ __forceinline__ double flux_body(const FluxArgs<real> a, const FluxPtrs<real> ptr, int64_t i) {
    double dtc = INFINITY;
    {
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
            bool owner;
            bool wallf = false;
            if (code & kNbBoundary) {
                owner = true;
                const uint32_t kind = code & 3u;
                wallf = PHYS == CTENO_EULER && kind == CTENO_WALL;
                if (wallf) {
                    // the flux comes from wall_flux; no outside state needed
                } else if (kind == CTENO_INFLOW) {
                    // prescribed state on the Gauss point's side of the moving line
                    // at the stage time (t, t + dt, t + dt/2 for the three stages)
                    const double *e = a.bface + 4 * (int64_t)((code >> 2) & kNbInflowMask);
                    const double t0 = a.tctrl ? a.tctrl->t : a.t_base;
                    const double dts = MODE == 2 ? (ptr.dt_ptr ? *ptr.dt_ptr : a.dt_value) : 0.0;
                    const double ts = t0 + (a.stage == 1 ? dts : a.stage == 2 ? 0.5 * dts : 0.0);
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        const double px = e[0] + a.gq[q] * e[2], py = e[1] + a.gq[q] * e[3];
                        const int side = px < a.bline[0] + a.bline[1] * py + a.bline[2] * ts ? 0 : 1;
#pragma unroll
                        for (int v = 0; v < NV; ++v) oth[NQ - 1 - q][v] = (real)a.bst[side][v];
                    }
                } else {
                    // transmissive: the inside state at the same Gauss point
                    // (oth[NQ-1-q] pairs with own[q])
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
#pragma unroll
                        for (int v = 0; v < NV; ++v) oth[NQ - 1 - q][v] = own[f][q][v];
                }
            } else {
                owner = (code & kNbOwner) != 0;
                const int64_t j = code & kNbIndexMask;
                const int g = (code >> 28) & 3;
                load_row<real, NQ * NV>(ptr.FV + (j * 3 + g) * NQ * NV, &oth[0][0]);
            }
            // both cells of a face evaluate F(owner side, other side; owner normal)
            // at the owner's Gauss points in the owner's order
            const real fx = owner ? nx : -nx, fy = owner ? ny : -ny;
            real sumF[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) sumF[v] = 0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                real A[NV], B[NV], F[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    A[v] = owner ? own[f][q][v] : oth[q][v];
                    B[v] = owner ? oth[NQ - 1 - q][v] : own[f][NQ - 1 - q][v];
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
                const double out = owner ? val : -val;
                acc[v] += out;
                if (MODE == 0) ptr.flux_out[(i * 3 + f) * NV + v] = (real)out;
            }
        }
        if (bad && ptr.ctrl) atomicOr(&ptr.ctrl->nonphysical, 1);
        if (MODE == 1) {
#pragma unroll
            for (int v = 0; v < NV; ++v) ptr.resid[i * NV + v] = -acc[v] / ptr.area[i];
        }
        if (MODE == 2) {
            const double dt = ptr.dt_ptr ? *ptr.dt_ptr : a.dt_value;
            const double ar = ptr.area[i];
            double u0[NV], us[NV], un[NV];
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
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double R = -acc[v] / ar;
                double r;
                if (a.stage == 0) r = us[v] + dt * R;
                else if (a.stage == 1) r = 0.75 * u0[v] + 0.25 * (us[v] + dt * R);
                else r = (1.0 / 3.0) * u0[v] + (2.0 / 3.0) * (us[v] + dt * R);
                un[v] = r;
            }
            if constexpr (NV == 4) {
                double2 *O2 = reinterpret_cast<double2 *>(ptr.Uout);
                O2[2 * i] = make_double2(un[0], un[1]);
                O2[2 * i + 1] = make_double2(un[2], un[3]);
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v) ptr.Uout[i * NV + v] = un[v];
            }
            if (ptr.want_dt) dtc = cell_dt_bound<NV, PHYS>(un, nrm, ar, a.gamma64, (double)a.ax, (double)a.ay);
        }
    }
    return dtc;
}

template <typename real, int NV, int PHYS, int MODE, int NQ>
__global__ __launch_bounds__(256) void k_flux(const FluxArgs<real> a) {
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (a.ctrl && a.ctrl->done) return;        // uniform across the grid
    const FluxPtrs<real> ptr{a.FV, a.fr, a.area, a.Un, a.Us, a.Uout, a.dt_ptr, a.flux_out, a.resid, a.ctrl,
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
    FluxArgs<real> a{};
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
__device__ __forceinline__ int find_slot(const BatchSlot *tab, int n, int64_t b) {
    for (int k = 0; k < n; ++k)
        if (b < tab[k].block0 + tab[k].nblocks) return b >= tab[k].block0 ? k : -1;
    return -1;
}

template <int R, int SCHEME, int GFORM>
__global__ __launch_bounds__(256) void k_reconstruct_batch(const ReconArgs<float, (R + 1) * (R + 2) / 2 - 1> a,
                                                           const BatchSlot *tab, const int *n_slots, int stage) {
    const int64_t b = blockIdx.x;
    const int s = find_slot(tab, *n_slots, b);
    if (s < 0) return;
    const BatchSlot &t = tab[s];
    if (t.ctrl->done) return;
    const int64_t i = (b - t.block0) * blockDim.x + threadIdx.x;
    if (i >= t.N) return;
    const ReconPtrs<float> ptr{t.U[stage], t.slot, t.flags, t.P, t.FV, nullptr, nullptr};
    recon_body<float, R, 4, SCHEME, GFORM, 0, 0>(a, ptr, i);
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
                              &t.ctrl->dt, nullptr, nullptr, t.ctrl, stage == 2};
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
        if (proto.scheme == CTENO_SCHEME_CTENOZ)
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
