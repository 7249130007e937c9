// Precompute kernels (once per mesh, FP64): reference-space moments of every
// stencil cell (sec. 2.1), Householder QR of the least-squares systems and
// the pseudo-inverses P = R^-1 Q^T diag(|V'_m|), for the central stencil and
// the three directional stencils; FP32 copies on request.  Degree 2 and 3:
// one lane per cell; degree 4 to 6: one wave per cell.
#include "kernels_common.h"

namespace cteno {

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
// orders 5 to 7 (r = 4..6)
// ===========================================================================
// The pseudo-inverse stream of a cell has S slots of EPS entries: K central,
// K_d directional (those of the directional stencil that holds the slot's
// cell; zero for a cell of none), zero padding to a multiple of 4.  At
// degrees 4 and 5 the slots are exactly the M central cells; at degree 6
// (M = 3 M_d) three groups of M_d slots, each group's members first.  It is
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
    constexpr int K = D::K, KD = D::KD, S = D::S, SP = D::SP, EPS = D::EPS, E = D::E;
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
    // the slot's directional stencil (3: none); each stencil's rows are contiguous
    int gl = (int)kSlotNoGroup;
    if (lane < S) {
        fl = a.slot_flag[tix(i, lane, S)];
        const uint32_t se = (uint32_t)a.slot[avix(i, lane, SP, 4)];
        gl = (int)(se >> kSlotGroupShift);
        if (fl & 1) {
            const int64_t m = se & kSlotIndexMask;
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

    // directional systems: stencil s owns the contiguous rows [base, base +
    // n) of the slots that name it, in directional-list order (the other
    // rows' directional entries stay zero from the stream's clearing)
    uint8_t flg = a.flags[i];
#pragma unroll 1
    for (int s = 0; s < 3; ++s) {
        const unsigned long long mk = __ballot(gl == s);
        const int nmem = __popcll(mk);
        if (nmem == 0) {                  // uniform: no stencil on this face
            flg &= (uint8_t)~(1u << s);
            continue;
        }
        const int base = __ffsll((long long)mk) - 1;
        const bool in = gl == s;
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
        for (int t = 0; t < nmem; ++t) {
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

}  // namespace cteno
