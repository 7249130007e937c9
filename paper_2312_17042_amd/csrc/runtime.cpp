// C ABI implementation: contexts, mesh upload, solution state, stage calls
// and the device-driven SSP-RK3 time march.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "cteno_internal.h"
#include "kernels.h"

using namespace cteno;

namespace {
thread_local std::string g_err;
cteno_status fail(cteno_status s, const std::string &m) {
    g_err = m;
    return s;
}
}  // namespace

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail(CTENO_ERR_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

extern "C" const char *cteno_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct cteno_ctx {
    int device = 0;
    hipStream_t user_stream = nullptr;
    hipStream_t own_stream = nullptr;
    cteno_alloc_fn alloc = nullptr;
    cteno_free_fn free_fn = nullptr;
    void *user = nullptr;
    bool timing = false;
    bool fused_stage = true;    // degree <= 3: the fused stage kernels (else reconstruction + flux)
    int64_t launches[3] = {0, 0, 0};
    double total_ms[3] = {0, 0, 0};
    struct Pending { int kernel; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> event_pool;
    hipStream_t stream() const { return user_stream ? user_stream : own_stream; }
};

namespace {

void *dev_alloc(cteno_ctx *c, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (c->alloc) return c->alloc(bytes, c->user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}
void dev_free(cteno_ctx *c, void *p) {
    if (!p) return;
    if (c->free_fn) c->free_fn(p, c->user);
    else (void)hipFree(p);
}

hipEvent_t take_event(cteno_ctx *c) {
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// drains recorded timing events (call after a stream synchronisation)
void collect_timing(cteno_ctx *c) {
    for (auto &p : c->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->launches[p.kernel] += 1;
            c->total_ms[p.kernel] += ms;
        }
        c->event_pool.push_back(p.a);
        c->event_pool.push_back(p.b);
    }
    c->pending.clear();
}

// launches fn on the context stream, bracketed by timing events when enabled
template <class F>
hipError_t timed(cteno_ctx *c, int kernel, F &&fn) {
    if (!c->timing) return fn();
    hipEvent_t a = take_event(c), b = take_event(c);
    (void)hipEventRecord(a, c->stream());
    hipError_t e = fn();
    (void)hipEventRecord(b, c->stream());
    c->pending.push_back({kernel, a, b});
    if (c->pending.size() > 4096) {
        (void)hipEventSynchronize(b);
        collect_timing(c);
    }
    return e;
}

struct DevBuf {
    cteno_ctx *ctx = nullptr;
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(cteno_ctx *c, size_t n) : ctx(c), bytes(n) { p = dev_alloc(c, n); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : ctx(o.ctx), p(o.p), bytes(o.bytes) { o.p = nullptr; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        reset();
        ctx = o.ctx; p = o.p; bytes = o.bytes; o.p = nullptr;
        return *this;
    }
    ~DevBuf() { reset(); }
    void reset() {
        if (p && ctx) dev_free(ctx, p);
        p = nullptr;
    }
    template <class T> T *as() const { return (T *)p; }
};

}  // namespace

extern "C" cteno_status cteno_ctx_create(int device, void *stream, cteno_alloc_fn alloc, cteno_free_fn free_fn,
                                         void *user, cteno_ctx **out) {
    if (!out) return fail(CTENO_ERR_INVALID, "out is NULL");
    if ((alloc == nullptr) != (free_fn == nullptr)) return fail(CTENO_ERR_INVALID, "alloc and free must be given together");
    int n = 0;
    HIP_TRY(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(CTENO_ERR_INVALID, "no such device");
    HIP_TRY(hipSetDevice(device));
    HIP_TRY(scratch_init(device));       // address of this device's fixed scratch
    auto c = std::make_unique<cteno_ctx>();
    c->device = device;
    c->user_stream = (hipStream_t)stream;
    c->alloc = alloc;
    c->free_fn = free_fn;
    c->user = user;
    HIP_TRY(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
    *out = c.release();
    return CTENO_OK;
}

extern "C" void cteno_ctx_destroy(cteno_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream());
    collect_timing(c);
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
}

extern "C" cteno_status cteno_ctx_set_stream(cteno_ctx *c, void *stream) {
    if (!c) return fail(CTENO_ERR_INVALID, "ctx is NULL");
    c->user_stream = (hipStream_t)stream;
    return CTENO_OK;
}

extern "C" cteno_status cteno_ctx_synchronize(cteno_ctx *c) {
    if (!c) return fail(CTENO_ERR_INVALID, "ctx is NULL");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipStreamSynchronize(c->stream()));
    collect_timing(c);
    return CTENO_OK;
}

extern "C" cteno_status cteno_ctx_set_fused_stage(cteno_ctx *c, int32_t on) {
    if (!c) return fail(CTENO_ERR_INVALID, "ctx is NULL");
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(hipStreamSynchronize(c->stream()));
    c->fused_stage = on != 0;
    return CTENO_OK;
}

extern "C" cteno_status cteno_ctx_set_timing(cteno_ctx *c, int32_t on) {
    if (!c) return fail(CTENO_ERR_INVALID, "ctx is NULL");
    c->timing = on != 0;
    return CTENO_OK;
}

extern "C" cteno_status cteno_ctx_kernel_stats(cteno_ctx *c, int32_t kernel, int64_t *launches, double *total_ms) {
    if (!c || kernel < 0 || kernel > 2) return fail(CTENO_ERR_INVALID, "bad kernel id");
    HIP_TRY(hipStreamSynchronize(c->stream()));
    collect_timing(c);
    if (launches) *launches = c->launches[kernel];
    if (total_ms) *total_ms = c->total_ms[kernel];
    return CTENO_OK;
}

extern "C" cteno_status cteno_ctx_reset_stats(cteno_ctx *c) {
    if (!c) return fail(CTENO_ERR_INVALID, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->stream()));
    collect_timing(c);
    for (int k = 0; k < 3; ++k) { c->launches[k] = 0; c->total_ms[k] = 0; }
    return CTENO_OK;
}

// ---------------------------------------------------------------------------
// mesh
// ---------------------------------------------------------------------------
struct cteno_mesh {
    cteno_ctx *ctx = nullptr;
    cteno_scheme scheme{};
    HostMesh host;
    DeviceMesh dm;
    std::vector<DevBuf> bufs;
    int64_t bytes = 0;
    template <class T> T *alloc(size_t count) {
        bufs.emplace_back(ctx, count * sizeof(T));
        if (!bufs.back().p) return nullptr;
        bytes += (int64_t)(count * sizeof(T));
        return bufs.back().as<T>();
    }
};

namespace {
template <class T, class A>
hipError_t h2d(T *dst, const std::vector<T, A> &src, hipStream_t st) {
    return hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st);
}
}  // namespace

static cteno_status check_scheme(const cteno_scheme &s) {
    if (s.physics != CTENO_ADVECTION && s.physics != CTENO_EULER) return fail(CTENO_ERR_INVALID, "bad physics");
    if (s.scheme < CTENO_SCHEME_CTENO || s.scheme > CTENO_SCHEME_TENO) return fail(CTENO_ERR_INVALID, "bad scheme");
    if (s.degree < 2 || s.degree > kMaxR) return fail(CTENO_ERR_INVALID, "degree must be 2..6");
    if (s.precision < 1 || s.precision > 3) return fail(CTENO_ERR_INVALID, "bad precision");
    if (!(s.lambda1_prime > 1.0) || !(s.c_t > 0 && s.c_t < 1) || !(s.eps > 0))
        return fail(CTENO_ERR_INVALID, "bad lambda1_prime, c_t or eps");
    if (s.physics == CTENO_EULER && !(s.gamma > 1.0)) return fail(CTENO_ERR_INVALID, "bad gamma");
    if (s.variables != CTENO_VARS_CONSERVED && s.variables != CTENO_VARS_CHARACTERISTIC)
        return fail(CTENO_ERR_INVALID, "bad variables");
    if (s.variables == CTENO_VARS_CHARACTERISTIC && s.physics != CTENO_EULER)
        return fail(CTENO_ERR_INVALID, "characteristic variables need the Euler equations");
    if (s.gamma_form < CTENO_GAMMA_PAPER || s.gamma_form > CTENO_GAMMA_SCALED)
        return fail(CTENO_ERR_INVALID, "bad gamma_form");
    if (s.gamma_form == CTENO_GAMMA_SCALED && s.scheme != CTENO_SCHEME_CTENOZ)
        return fail(CTENO_ERR_INVALID, "the scaled gamma form belongs to CTENOZ");
    if (s.positivity != 0 && s.positivity != 1) return fail(CTENO_ERR_INVALID, "positivity must be 0 or 1");
    return CTENO_OK;
}

// Uploads a host-built mesh: device arrays, FP64 precompute of the
// pseudo-inverses (plus the FP32 copy for MIXED), admissibility fix-up.
// Allocations are appended to bufs; their size is added to bytes.
static cteno_status upload_device_mesh(cteno_ctx *ctx, hipStream_t st, HostMesh &hm, const cteno_scheme &s,
                                       DeviceMesh &dm, std::vector<DevBuf> &bufs, int64_t &bytes, bool keep_fr64) {
    auto alloc_raw = [&](size_t n) -> void * {
        bufs.emplace_back(ctx, n);
        if (!bufs.back().p) return nullptr;
        bytes += (int64_t)n;
        return bufs.back().p;
    };
    auto allocator = [&](auto *tag, size_t count) { return (decltype(tag))alloc_raw(count * sizeof(*tag)); };
#define alloc_T(T, n) allocator((T *)nullptr, (n))
    dm.N = hm.N; dm.Np = pad64(hm.N);
    dm.r = hm.r; dm.K = hm.K; dm.S = hm.S; dm.nv = hm.nv;
    dm.Kd = hm.Kd; dm.Md = hm.Md; dm.Nq = hm.Nq;
    dm.stile = hm.r >= 4 ? kTile / hm.nv : kTile;
    dm.physics = s.physics; dm.scheme = s.scheme; dm.gamma_form = s.gamma_form; dm.precision = s.precision;
    dm.vars = s.variables;
    dm.positivity = s.physics == CTENO_EULER ? s.positivity : 0;
    dm.gamma = s.gamma; dm.ax = s.ax; dm.ay = s.ay; dm.lam1p = s.lambda1_prime; dm.ct = s.c_t; dm.eps = s.eps;
    dm.Lx = hm.Lx; dm.Ly = hm.Ly;
    make_ref_tables(hm.r, dm.tab);
    const size_t Np = (size_t)dm.Np, S = hm.S;
    dm.SP = hm.SP;
    dm.E64 = round_up(pinv_entries(hm.r), 2);
    dm.E32 = round_up(pinv_entries(hm.r), 4);
    dm.slot = alloc_T(int32_t, Np * hm.SP);
    dm.flags = alloc_T(uint8_t, Np);
    dm.fr64 = keep_fr64 ? alloc_T(double, Np * 12) : nullptr;
    dm.area = alloc_T(double, Np);
    dm.perm = alloc_T(int32_t, (size_t)hm.N);
    dm.n_inflow = (int64_t)(hm.bface.size() / 4);
    if (dm.n_inflow) {
        dm.bface = alloc_T(double, hm.bface.size());
        if (!dm.bface) return fail(CTENO_ERR_NOMEM, "device allocation failed");
        HIP_TRY(h2d(dm.bface, hm.bface, st));
    }
    for (int k = 0; k < 2; ++k)
        for (int v = 0; v < 4; ++v) dm.bst[k][v] = hm.bst[k][v];
    for (int k = 0; k < 3; ++k) dm.bline[k] = hm.bline[k];
    if (s.precision & CTENO_MIXED) {
        dm.fr32 = alloc_T(float, Np * 12);
        dm.P32 = alloc_T(float, Np * dm.E32);
    }
    if (!dm.slot || !dm.flags || (keep_fr64 && !dm.fr64) || !dm.area || !dm.perm ||
        ((s.precision & CTENO_MIXED) && (!dm.fr32 || !dm.P32)))
        return fail(CTENO_ERR_NOMEM, "device allocation failed");
    if (hm.r >= 4) {
        // Gram matrix [K][K] and face basis [3][Nq][K] of the higher-order kernels
        const int K = hm.K, ntab = K * K + 3 * hm.Nq * K;
        std::vector<double> t64(ntab);
        std::vector<float> t32(ntab);
        for (int p = 0; p < K; ++p)
            for (int q = 0; q < K; ++q) t64[p * K + q] = dm.tab.gram[p][q];
        for (int f = 0; f < 3; ++f)
            for (int q = 0; q < hm.Nq; ++q)
                for (int k = 0; k < K; ++k) t64[K * K + (f * hm.Nq + q) * K + k] = dm.tab.basis[f][q][k];
        for (int e = 0; e < ntab; ++e) t32[e] = (float)t64[e];
        dm.htab64 = alloc_T(double, ntab);
        dm.htab32 = alloc_T(float, ntab);
        if (!dm.htab64 || !dm.htab32) return fail(CTENO_ERR_NOMEM, "device allocation failed");
        HIP_TRY(h2d(dm.htab64, t64, st));
        HIP_TRY(h2d(dm.htab32, t32, st));
    }
    // FP64 pseudo-inverses are always computed; kept only when FP64 is resident
    DevBuf p64(ctx, Np * dm.E64 * sizeof(double));
    DevBuf verts(ctx, Np * 6 * sizeof(double)), sflag(ctx, Np * S), sshift(ctx, Np * 2 * S), rfail(ctx, sizeof(int));
    if (!p64.p || !verts.p || !sflag.p || !sshift.p || !rfail.p)
        return fail(CTENO_ERR_NOMEM, "device allocation failed (precompute)");
    dm.P64 = p64.as<double>();

    HIP_TRY(h2d(dm.slot, hm.slot, st));
    HIP_TRY(h2d(dm.flags, hm.flags, st));
    if (dm.fr64) HIP_TRY(h2d(dm.fr64, hm.fr64, st));
    if (dm.fr32) HIP_TRY(h2d(dm.fr32, hm.fr32, st));
    HIP_TRY(h2d(dm.area, hm.area, st));
    HIP_TRY(h2d(dm.perm, hm.perm, st));
    HIP_TRY(h2d(verts.as<double>(), hm.verts, st));
    HIP_TRY(h2d(sflag.as<uint8_t>(), hm.slot_flag, st));
    HIP_TRY(h2d(sshift.as<int8_t>(), hm.slot_shift, st));
    HIP_TRY(hipMemsetAsync(rfail.p, 0, sizeof(int), st));
    // padding entries of the streams stay zero
    HIP_TRY(hipMemsetAsync(dm.P64, 0, Np * dm.E64 * sizeof(double), st));
    if (dm.P32) HIP_TRY(hipMemsetAsync(dm.P32, 0, Np * dm.E32 * sizeof(float), st));

    PrecomputeInputs in{verts.as<double>(), sflag.as<uint8_t>(), sshift.as<int8_t>(), dm.flags, rfail.as<int>()};
    // kernel timing belongs to the context's own stream and thread
    if (st == ctx->stream()) HIP_TRY(timed(ctx, 2, [&] { return launch_precompute(dm, in, st); }));
    else HIP_TRY(launch_precompute(dm, in, st));
    int rank_fail = 0;
    std::vector<uint8_t> flags(Np);
    HIP_TRY(hipMemcpyAsync(&rank_fail, rfail.p, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(flags.data(), dm.flags, Np, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (st == ctx->stream()) collect_timing(ctx);
    if (rank_fail) return fail(CTENO_ERR_STENCIL, std::to_string(rank_fail) + " rank-deficient central stencils");
    // directional stencils found rank-deficient on the device become inadmissible
    for (int k = 0; k < hm.N; ++k) {
        const int u = hm.perm[k];
        for (int f = 0; f < 3; ++f)
            if (((hm.flags[k] >> f) & 1) && !((flags[k] >> f) & 1)) {
                hm.dirn_user[3 * (size_t)u + f] = 0;
                for (int a = 0; a < hm.Md; ++a) hm.dir_user[((size_t)u * 3 + f) * hm.Md + a] = -1;
                hm.n_inadmissible++;
            }
        hm.flags[k] = flags[k];
    }
    if (s.precision & CTENO_FP64) {
        bytes += (int64_t)p64.bytes;
        bufs.push_back(std::move(p64));
    } else {
        dm.P64 = nullptr;
    }
    // fused stage (degree <= 3; single meshes -- the batched serving kernels
    // keep the reconstruction + flux pair): the cells with a face whose
    // neighbour lies in another 256-cell block, from the face codes
    dm.fused = keep_fr64 && hm.r <= 3 && hm.Nq == 2;
    if (dm.fused) {
        std::vector<int32_t> xc;
        for (int64_t k = 0; k < hm.N; ++k)
            for (int f = 0; f < 3; ++f) {
                uint32_t code;
                std::memcpy(&code, &hm.fr32[avix(k, 4 * f + 3, 12, 4)], sizeof code);
                if (!(code & kNbBoundary) && ((int64_t)(code & kNbIndexMask) >> 8) != (k >> 8)) {
                    xc.push_back((int32_t)k);
                    break;
                }
            }
        dm.n_cross = (int64_t)xc.size();
        if (dm.n_cross) {
            // in cross-cell order: the neighbour's cross index across each
            // face to another block, the area and the face records; per
            // block the number of cross cells before it
            const int64_t nx = dm.n_cross, nxp = pad64(nx), nb = dm.blocks();
            std::vector<int32_t> xbase(nb + 1, 0), xidx(hm.N, -1), xnb(3 * nx, -1);
            std::vector<double> xar(nx), xf64(keep_fr64 ? nxp * 12 : 0);
            std::vector<float> xf32(dm.fr32 ? nxp * 12 : 0);
            for (int64_t t = 0; t < nx; ++t) {
                xbase[(xc[t] >> 8) + 1]++;
                xidx[xc[t]] = (int32_t)t;
            }
            for (int64_t b = 0; b < nb; ++b) xbase[b + 1] += xbase[b];
            for (int64_t t = 0; t < nx; ++t) {
                const int64_t k = xc[t];
                xar[t] = hm.area[k];
                for (int f = 0; f < 3; ++f) {
                    uint32_t code;
                    std::memcpy(&code, &hm.fr32[avix(k, 4 * f + 3, 12, 4)], sizeof code);
                    const int64_t j = code & kNbIndexMask;
                    if (!(code & kNbBoundary) && (j >> 8) != (k >> 8)) xnb[3 * t + f] = xidx[j];
                }
                for (int e = 0; e < 12; ++e) {
                    if (!xf32.empty()) xf32[avix(t, e, 12, 4)] = hm.fr32[avix(k, e, 12, 4)];
                    if (!xf64.empty()) xf64[avix(t, e, 12, 2)] = hm.fr64[avix(k, e, 12, 2)];
                }
            }
            dm.xcells = alloc_T(int32_t, xc.size());
            dm.xbase = alloc_T(int32_t, xbase.size());
            dm.xnb = alloc_T(int32_t, xnb.size());
            dm.xarea = alloc_T(double, xar.size());
            if (!xf32.empty()) dm.xfr32 = alloc_T(float, xf32.size());
            if (!xf64.empty()) dm.xfr64 = alloc_T(double, xf64.size());
            if (!dm.xcells || !dm.xbase || !dm.xnb || !dm.xarea || (!xf32.empty() && !dm.xfr32) ||
                (!xf64.empty() && !dm.xfr64))
                return fail(CTENO_ERR_NOMEM, "device allocation failed");
            HIP_TRY(h2d(dm.xcells, xc, st));
            HIP_TRY(h2d(dm.xbase, xbase, st));
            HIP_TRY(h2d(dm.xnb, xnb, st));
            HIP_TRY(h2d(dm.xarea, xar, st));
            if (!xf32.empty()) HIP_TRY(h2d(dm.xfr32, xf32, st));
            if (!xf64.empty()) HIP_TRY(h2d(dm.xfr64, xf64, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
    }
    // release host-only copies that the device now holds
    hm.slot.clear(); hm.slot.shrink_to_fit();
    hm.slot_flag.clear(); hm.slot_flag.shrink_to_fit();
    hm.slot_shift.clear(); hm.slot_shift.shrink_to_fit();
    hm.verts.clear(); hm.verts.shrink_to_fit();
    hm.fr64.clear(); hm.fr64.shrink_to_fit();
    hm.fr32.clear(); hm.fr32.shrink_to_fit();
#undef alloc_T
    return CTENO_OK;
}

extern "C" cteno_status cteno_mesh_upload(cteno_ctx *ctx, const cteno_mesh_desc *desc, const cteno_scheme *scheme,
                                          cteno_mesh **out) {
    if (!ctx || !desc || !scheme || !out) return fail(CTENO_ERR_INVALID, "NULL argument");
    const cteno_scheme &s = *scheme;
    if (cteno_status rc = check_scheme(s)) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    auto m = std::make_unique<cteno_mesh>();
    m->ctx = ctx;
    m->scheme = s;
    std::string err;
    cteno_status rc = build_host_mesh(*desc, s, m->host, err);
    if (rc != CTENO_OK) return fail(rc, err);
    rc = upload_device_mesh(ctx, ctx->stream(), m->host, s, m->dm, m->bufs, m->bytes, true);
    if (rc != CTENO_OK) return rc;
    *out = m.release();
    return CTENO_OK;
}

extern "C" cteno_status cteno_mesh_info_get(const cteno_mesh *m, cteno_mesh_info *info) {
    if (!m || !info) return fail(CTENO_ERR_INVALID, "NULL argument");
    info->n_cells = m->host.N;
    info->n_faces = m->host.n_faces;
    info->n_boundary_faces = m->host.n_boundary;
    info->K = m->host.K;
    info->M = m->host.M;
    info->slots = m->host.S;
    info->nv = m->host.nv;
    info->nq = m->host.Nq;
    info->Kd = m->host.Kd;
    info->Md = m->host.Md;
    info->n_inadmissible = m->host.n_inadmissible;
    info->device_bytes = m->bytes;
    info->n_cross_cells = m->dm.n_cross;
    return CTENO_OK;
}

extern "C" cteno_status cteno_mesh_stencils(const cteno_mesh *m, int32_t *central, int32_t *directional,
                                            int32_t *dir_count) {
    if (!m) return fail(CTENO_ERR_INVALID, "mesh is NULL");
    const HostMesh &h = m->host;
    if (central) std::memcpy(central, h.cen_user.data(), h.cen_user.size() * sizeof(int32_t));
    if (directional) std::memcpy(directional, h.dir_user.data(), h.dir_user.size() * sizeof(int32_t));
    if (dir_count) std::memcpy(dir_count, h.dirn_user.data(), h.dirn_user.size() * sizeof(int32_t));
    return CTENO_OK;
}

extern "C" cteno_status cteno_mesh_pinv(cteno_ctx *ctx, const cteno_mesh *m, int32_t which, int32_t n,
                                        const int32_t *cells, double *central, double *directional) {
    if (!ctx || !m || n < 0 || (n && !cells)) return fail(CTENO_ERR_INVALID, "bad arguments");
    const DeviceMesh &dm = m->dm;
    const HostMesh &hm = m->host;
    const bool f32 = which == CTENO_MIXED;
    if (which != CTENO_FP64 && which != CTENO_MIXED) return fail(CTENO_ERR_INVALID, "which must be FP64 or MIXED");
    if (!(dm.precision & which)) return fail(CTENO_ERR_INVALID, "requested pseudo-inverse copy is not resident");
    if (n == 0) return CTENO_OK;
    std::vector<int32_t> idx(n);
    for (int a = 0; a < n; ++a) {
        if (cells[a] < 0 || cells[a] >= hm.N) return fail(CTENO_ERR_INVALID, "cell out of range");
        idx[a] = hm.iperm[cells[a]];
    }
    // slot tables are not kept on the host; rebuild the column maps from the stencils
    const int K = hm.K, S = hm.S, M = hm.M, Kd = hm.Kd, Md = hm.Md;
    const int E = f32 ? dm.E32 : dm.E64, VW = f32 ? 4 : 2;
    HIP_TRY(hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream();
    DevBuf didx(ctx, n * sizeof(int32_t)), op(ctx, (size_t)n * E * sizeof(double)),
        dslot(ctx, (size_t)n * dm.SP * sizeof(double));
    if (!didx.p || !op.p || !dslot.p) return fail(CTENO_ERR_NOMEM, "device allocation failed");
    HIP_TRY(hipMemcpyAsync(didx.p, idx.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_gather_entries(n, didx.as<int32_t>(), E, VW, f32 ? nullptr : dm.P64, f32 ? dm.P32 : nullptr,
                                  nullptr, op.as<double>(), st, dm.stile));
    HIP_TRY(launch_gather_entries(n, didx.as<int32_t>(), dm.SP, 4, nullptr, nullptr, dm.slot, dslot.as<double>(), st));
    std::vector<double> pe((size_t)n * E), slotd((size_t)n * dm.SP);
    HIP_TRY(hipMemcpyAsync(pe.data(), op.p, pe.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(slotd.data(), dslot.p, slotd.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int a = 0; a < n; ++a) {
        const int u = cells[a];
        const int32_t *cen = hm.cen_user.data() + (size_t)u * M;
        const int32_t *dr = hm.dir_user.data() + (size_t)u * 3 * Md;
        if (central) std::fill(central + (size_t)a * K * M, central + (size_t)(a + 1) * K * M, 0.0);
        if (directional)
            std::fill(directional + (size_t)a * 3 * Kd * Md, directional + (size_t)(a + 1) * 3 * Kd * Md, 0.0);
        for (int j = 0; j < S; ++j) {
            // degree >= 4: the slot entry also names the slot's directional stencil
            const uint32_t se = (uint32_t)(int64_t)slotd[(size_t)a * dm.SP + j];
            const int src_k = hm.r >= 4 ? (int)(se & kSlotIndexMask) : (int)se;
            const int grp = hm.r >= 4 ? (int)(se >> kSlotGroupShift) : (j < 3 * Md ? j / Md : 3);
            if (src_k == idx[a]) continue;   // padding slot (the cell itself)
            const int src_u = hm.perm[src_k];
            int cpos = -1;
            for (int q = 0; q < M; ++q) if (cen[q] == src_u) cpos = q;
            if (cpos < 0) return fail(CTENO_ERR_DEVICE, "slot not in stencil");
            // slot j: K central entries, then (slots of the directional groups) K_d directional ones
            const int off = hm.r >= 4 ? j * ho_slot_entries(hm.r) : pinv_offset(j, K);
            if (central)
                for (int k = 0; k < K; ++k) central[((size_t)a * K + k) * M + cpos] = pe[(size_t)a * E + off + k];
            if (grp < 3 && directional) {
                const int s = grp;
                int dpos = -1;
                for (int q = 0; q < Md; ++q) if (dr[s * Md + q] == src_u) dpos = q;
                if (dpos >= 0)
                    for (int c = 0; c < Kd; ++c)
                        directional[(((size_t)a * 3 + s) * Kd + c) * Md + dpos] = pe[(size_t)a * E + off + K + c];
            }
        }
    }
    return CTENO_OK;
}

extern "C" cteno_status cteno_stencils_host(const cteno_mesh_desc *desc, const cteno_scheme *scheme,
                                            int32_t *central, int32_t *directional, int32_t *dir_count) {
    if (!desc || !scheme) return fail(CTENO_ERR_INVALID, "NULL argument");
    if (scheme->degree < 2 || scheme->degree > kMaxR) return fail(CTENO_ERR_INVALID, "degree must be 2..6");
    HostMesh hm;
    std::string err;
    cteno_scheme s = *scheme;
    s.reorder = 0;
    cteno_status rc = build_host_mesh(*desc, s, hm, err);
    if (rc != CTENO_OK) return fail(rc, err);
    if (central) std::memcpy(central, hm.cen_user.data(), hm.cen_user.size() * sizeof(int32_t));
    if (directional) std::memcpy(directional, hm.dir_user.data(), hm.dir_user.size() * sizeof(int32_t));
    if (dir_count) std::memcpy(dir_count, hm.dirn_user.data(), hm.dirn_user.size() * sizeof(int32_t));
    return CTENO_OK;
}

extern "C" void cteno_mesh_destroy(cteno_mesh *m) {
    if (!m) return;
    (void)hipSetDevice(m->ctx->device);
    (void)hipStreamSynchronize(m->ctx->stream());
    delete m;
}

// ---------------------------------------------------------------------------
// solution state
// ---------------------------------------------------------------------------
struct cteno_sol {
    cteno_ctx *ctx = nullptr;
    const cteno_mesh *mesh = nullptr;
    DevBuf U[3];              // U^n, U^(1), U^(2): AoS [Np][nv]
    DevBuf FV[2];             // face-point values, FP64 / FP32
    DevBuf ctrl;              // Ctrl
    DevBuf dt_part;           // per-block minima of the CFL bound
    DevBuf status;            // SolStatus: fallback count, non-physical flag of stage calls
    DevBuf xpart;             // fused stage: partial stage states of the cross cells
    double t = 0.0;
    Ctrl *h_ctrl = nullptr;   // pinned host mirror
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    bool graph_fused[2] = {false, false};   // stage kernels a captured graph holds
    ~cteno_sol() {
        for (auto &g : graph) if (g) (void)hipGraphExecDestroy(g);
        if (h_ctrl) (void)hipHostFree(h_ctrl);
    }
    void *fv(bool f32) {
        DevBuf &b = FV[f32 ? 1 : 0];
        if (!b.p) {
            const DeviceMesh &dm = mesh->dm;
            b = DevBuf(ctx, (size_t)dm.Np * 3 * dm.Nq * dm.nv * (f32 ? sizeof(float) : sizeof(double)));
        }
        return b.p;
    }
};

// device-side counters of a solution, written by its reconstructions and stage calls
struct SolStatus {
    unsigned long long fallbacks;   // cells x stages that took the positivity fallback
    int nonphysical;                // a stage call met a non-physical face state
    int pad;
};

namespace {
SolStatus *sol_status(const cteno_sol *s) { return s->status.as<SolStatus>(); }

cteno_status check_precision(const cteno_mesh *m, int32_t precision, bool &f32) {
    if (precision != CTENO_FP64 && precision != CTENO_MIXED) return fail(CTENO_ERR_INVALID, "precision must be FP64 or MIXED");
    if (!(m->dm.precision & precision)) return fail(CTENO_ERR_INVALID, "mesh was uploaded without this precision");
    f32 = precision == CTENO_MIXED;
    return CTENO_OK;
}
}  // namespace

extern "C" cteno_status cteno_sol_create(cteno_ctx *ctx, const cteno_mesh *m, const double *u0, double t0,
                                         cteno_sol **out) {
    if (!ctx || !m || !u0 || !out) return fail(CTENO_ERR_INVALID, "NULL argument");
    HIP_TRY(hipSetDevice(ctx->device));
    auto s = std::make_unique<cteno_sol>();
    s->ctx = ctx;
    s->mesh = m;
    const DeviceMesh &dm = m->dm;
    const size_t bytes = (size_t)dm.Np * dm.nv * sizeof(double);
    for (auto &u : s->U) {
        u = DevBuf(ctx, bytes);
        if (!u.p) return fail(CTENO_ERR_NOMEM, "device allocation failed");
        HIP_TRY(hipMemsetAsync(u.p, 0, bytes, ctx->stream()));
    }
    s->ctrl = DevBuf(ctx, sizeof(Ctrl));
    s->dt_part = DevBuf(ctx, (size_t)dm.dt_parts() * sizeof(double));
    s->status = DevBuf(ctx, sizeof(SolStatus));
    if (!s->ctrl.p || !s->dt_part.p || !s->status.p) return fail(CTENO_ERR_NOMEM, "device allocation failed");
    HIP_TRY(hipMemsetAsync(s->ctrl.p, 0, sizeof(Ctrl), ctx->stream()));
    HIP_TRY(hipHostMalloc((void **)&s->h_ctrl, sizeof(Ctrl), hipHostMallocDefault));
    cteno_sol *raw = s.release();
    cteno_status rc = cteno_sol_set(raw, u0, t0);
    if (rc != CTENO_OK) { cteno_sol_destroy(raw); return rc; }
    *out = raw;
    return CTENO_OK;
}

extern "C" cteno_status cteno_sol_set(cteno_sol *s, const double *u, double t) {
    if (!s || !u) return fail(CTENO_ERR_INVALID, "NULL argument");
    const DeviceMesh &dm = s->mesh->dm;
    hipStream_t st = s->ctx->stream();
    HIP_TRY(hipSetDevice(s->ctx->device));
    DevBuf tmp(s->ctx, (size_t)dm.N * dm.nv * sizeof(double));
    if (!tmp.p) return fail(CTENO_ERR_NOMEM, "device allocation failed");
    HIP_TRY(hipMemcpyAsync(tmp.p, u, (size_t)dm.N * dm.nv * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_user_to_state(dm, tmp.as<double>(), s->U[0].as<double>(), st));
    HIP_TRY(hipMemsetAsync(s->status.p, 0, sizeof(SolStatus), st));
    HIP_TRY(hipStreamSynchronize(st));
    s->t = t;
    return CTENO_OK;
}

extern "C" cteno_status cteno_sol_download(cteno_sol *s, double *u, double *t) {
    if (!s) return fail(CTENO_ERR_INVALID, "sol is NULL");
    const DeviceMesh &dm = s->mesh->dm;
    hipStream_t st = s->ctx->stream();
    HIP_TRY(hipSetDevice(s->ctx->device));
    DevBuf tmp;
    if (u) {
        tmp = DevBuf(s->ctx, (size_t)dm.N * dm.nv * sizeof(double));
        if (!tmp.p) return fail(CTENO_ERR_NOMEM, "device allocation failed");
        HIP_TRY(launch_state_to_user(dm, s->U[0].as<double>(), tmp.as<double>(), st));
        HIP_TRY(hipMemcpyAsync(u, tmp.p, (size_t)dm.N * dm.nv * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    SolStatus h{};
    HIP_TRY(hipMemcpyAsync(&h, s->status.p, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (t) *t = s->t;
    if (h.nonphysical) {
        // reported once: the flag of the stage calls is cleared
        HIP_TRY(hipMemsetAsync(&sol_status(s)->nonphysical, 0, sizeof(int), st));
        HIP_TRY(hipStreamSynchronize(st));
        return fail(CTENO_ERR_NONPHYSICAL, "a stage call met a non-physical face state (density or pressure <= 0, "
                                           "or NaN)");
    }
    return CTENO_OK;
}

extern "C" cteno_status cteno_sol_fallbacks(cteno_sol *s, int64_t *count) {
    if (!s || !count) return fail(CTENO_ERR_INVALID, "NULL argument");
    HIP_TRY(hipSetDevice(s->ctx->device));
    hipStream_t st = s->ctx->stream();
    SolStatus h{};
    HIP_TRY(hipMemcpyAsync(&h, s->status.p, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *count = (int64_t)h.fallbacks;
    return CTENO_OK;
}

extern "C" void cteno_sol_destroy(cteno_sol *s) {
    if (!s) return;
    (void)hipSetDevice(s->ctx->device);
    (void)hipStreamSynchronize(s->ctx->stream());
    delete s;
}

// ---------------------------------------------------------------------------
// stage calls
// ---------------------------------------------------------------------------
extern "C" cteno_status cteno_reconstruct(cteno_ctx *ctx, const cteno_mesh *m, const cteno_sol *sol,
                                          int32_t precision, void *face_vals, uint8_t *delta_out,
                                          const uint8_t *delta_forced) {
    if (!ctx || !m || !sol || !face_vals) return fail(CTENO_ERR_INVALID, "NULL argument");
    if (sol->mesh != m) return fail(CTENO_ERR_INVALID, "solution belongs to another mesh");
    bool f32;
    if (cteno_status rc = check_precision(m, precision, f32)) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    const DeviceMesh &dm = m->dm;
    hipStream_t st = ctx->stream();
    cteno_sol *s = const_cast<cteno_sol *>(sol);
    void *fv = s->fv(f32);
    if (!fv) return fail(CTENO_ERR_NOMEM, "device allocation failed");
    DevBuf dbuf;
    int dmode = 0;
    if (delta_forced || delta_out) {
        dbuf = DevBuf(ctx, (size_t)dm.Np * dm.delta_bytes());
        if (!dbuf.p) return fail(CTENO_ERR_NOMEM, "device allocation failed");
        if (delta_forced) {
            HIP_TRY(launch_delta_from_user(dm, delta_forced, dbuf.as<uint8_t>(), st));
            dmode = 2;
        } else {
            dmode = 1;
        }
    }
    HIP_TRY(timed(ctx, 0, [&] {
        return launch_reconstruct(dm, f32, s->U[0].as<double>(), fv, dbuf.as<uint8_t>(), dmode, nullptr, st,
                                  &sol_status(s)->fallbacks);
    }));
    HIP_TRY(launch_fv_to_user(dm, f32, fv, face_vals, st));
    if (delta_out) HIP_TRY(launch_delta_to_user(dm, dbuf.as<uint8_t>(), delta_out, st));
    HIP_TRY(hipStreamSynchronize(st));   // dbuf is released on return
    return CTENO_OK;
}

extern "C" cteno_status cteno_flux(cteno_ctx *ctx, const cteno_mesh *m, int32_t precision, const void *face_vals,
                                   double t, void *face_flux) {
    if (!ctx || !m || !face_vals || !face_flux) return fail(CTENO_ERR_INVALID, "NULL argument");
    bool f32;
    if (cteno_status rc = check_precision(m, precision, f32)) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    const DeviceMesh &dm = m->dm;
    hipStream_t st = ctx->stream();
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    DevBuf fv(ctx, (size_t)dm.Np * 3 * dm.Nq * dm.nv * es), fo(ctx, (size_t)dm.Np * 3 * dm.nv * es),
        flag(ctx, sizeof(int));
    if (!fv.p || !fo.p || !flag.p) return fail(CTENO_ERR_NOMEM, "device allocation failed");
    HIP_TRY(hipMemsetAsync(flag.p, 0, sizeof(int), st));
    HIP_TRY(launch_fv_from_user(dm, f32, face_vals, fv.p, st));
    FluxLaunch fl;
    fl.mode = 0;
    fl.FV = fv.p;
    fl.flux_out = fo.p;
    fl.t_base = t;
    fl.nonphys = flag.as<int>();
    HIP_TRY(timed(ctx, 1, [&] { return launch_flux(dm, f32, fl, st); }));
    HIP_TRY(launch_flux_to_user(dm, f32, fo.p, face_flux, st));
    int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (bad) return fail(CTENO_ERR_NONPHYSICAL, "non-physical face state (density or pressure <= 0, or NaN)");
    return CTENO_OK;
}

extern "C" cteno_status cteno_flux_noalloc(cteno_ctx *ctx, const cteno_mesh *m, int32_t precision,
                                           const void *face_vals, double t, void *face_flux) {
    if (!ctx || !m || !face_vals || !face_flux) return fail(CTENO_ERR_INVALID, "NULL argument");
    bool f32;
    if (cteno_status rc = check_precision(m, precision, f32)) return rc;
    const DeviceMesh &dm = m->dm;
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    const size_t fv_bytes = (size_t)dm.Np * 3 * dm.Nq * dm.nv * es;
    const size_t fo_bytes = (size_t)dm.Np * 3 * dm.nv * es;
    const size_t fo_off = (fv_bytes + 255) / 256 * 256;
    const size_t flag_off = (fo_off + fo_bytes + 255) / 256 * 256;
    const size_t need = flag_off + 256;
    if (need > kScratchBytes)
        return fail(CTENO_ERR_INVALID, "mesh too large for the fixed scratch: needs " + std::to_string(need) +
                                           " bytes, holds " + std::to_string(kScratchBytes));
    HIP_TRY(hipSetDevice(ctx->device));
    unsigned char *base = (unsigned char *)scratch_device_ptr(ctx->device);
    if (!base) return fail(CTENO_ERR_DEVICE, "fixed scratch not initialised on this device");
    void *fv = base, *fo = base + fo_off;
    unsigned long long *flag = (unsigned long long *)(base + flag_off);
    hipStream_t st = ctx->stream();
    // the flag must start at zero; the buffers are fully written before use
    HIP_TRY(launch_fill_u64(flag, 0ull, 1, st));
    HIP_TRY(launch_fv_from_user(dm, f32, face_vals, fv, st));
    FluxLaunch fl;
    fl.mode = 0;
    fl.FV = fv;
    fl.flux_out = fo;
    fl.t_base = t;
    fl.nonphys = (int *)flag;
    HIP_TRY(launch_flux(dm, f32, fl, st));
    HIP_TRY(launch_flux_to_user(dm, f32, fo, face_flux, st));
    unsigned long long bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (bad) return fail(CTENO_ERR_NONPHYSICAL, "non-physical face state (density or pressure <= 0, or NaN)");
    return CTENO_OK;
}

extern "C" cteno_status cteno_residual(cteno_ctx *ctx, const cteno_mesh *m, const cteno_sol *sol, int32_t precision,
                                       double *resid) {
    if (!ctx || !m || !sol || !resid) return fail(CTENO_ERR_INVALID, "NULL argument");
    if (sol->mesh != m) return fail(CTENO_ERR_INVALID, "solution belongs to another mesh");
    bool f32;
    if (cteno_status rc = check_precision(m, precision, f32)) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    const DeviceMesh &dm = m->dm;
    hipStream_t st = ctx->stream();
    cteno_sol *s = const_cast<cteno_sol *>(sol);
    void *fv = s->fv(f32);
    DevBuf r(ctx, (size_t)dm.Np * dm.nv * sizeof(double));
    if (!fv || !r.p) return fail(CTENO_ERR_NOMEM, "device allocation failed");
    SolStatus *ss = sol_status(s);
    HIP_TRY(hipMemsetAsync(&ss->nonphysical, 0, sizeof(int), st));
    HIP_TRY(timed(ctx, 0, [&] {
        return launch_reconstruct(dm, f32, s->U[0].as<double>(), fv, nullptr, 0, nullptr, st, &ss->fallbacks);
    }));
    FluxLaunch fl;
    fl.mode = 1;
    fl.FV = fv;
    fl.resid = r.as<double>();
    fl.t_base = s->t;
    fl.nonphys = &ss->nonphysical;
    HIP_TRY(timed(ctx, 1, [&] { return launch_flux(dm, f32, fl, st); }));
    HIP_TRY(launch_state_to_user(dm, r.as<double>(), resid, st));
    int bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, &ss->nonphysical, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (bad) {
        HIP_TRY(hipMemsetAsync(&ss->nonphysical, 0, sizeof(int), st));
        HIP_TRY(hipStreamSynchronize(st));
        return fail(CTENO_ERR_NONPHYSICAL, "non-physical face state (density or pressure <= 0, or NaN)");
    }
    return CTENO_OK;
}

namespace {
// the fused stage kernels (degree <= 3, both precisions) unless the context
// asks for the separate reconstruction and flux kernels
bool use_fused(const cteno_ctx *ctx, const DeviceMesh &dm, bool) { return dm.fused && ctx->fused_stage; }

// one SSP-RK3 stage on sol; dt from a device pointer or a host value
hipError_t issue_stage(cteno_ctx *ctx, cteno_sol *s, bool f32, int stage, const double *dt_ptr, double dt_value,
                       Ctrl *ctrl, double *dt_part, hipStream_t st) {
    const DeviceMesh &dm = s->mesh->dm;
    const double *in = s->U[stage].as<double>();    // U^n, U^(1), U^(2)
    double *outU = stage == 2 ? s->U[0].as<double>() : s->U[stage + 1].as<double>();
    void *fv = s->fv(f32);
    const int *done = ctrl ? &ctrl->done : nullptr;
    SolStatus *ss = sol_status(s);
    FluxLaunch fl;
    fl.mode = 2;
    fl.FV = fv;
    fl.Un = s->U[0].as<double>();
    fl.Us = in;
    fl.Uout = outU;
    fl.stage = stage;
    fl.dt_ptr = dt_ptr;
    fl.dt_value = dt_value;
    fl.ctrl = ctrl;
    fl.nonphys = ctrl ? nullptr : &ss->nonphysical;    // a march reports through its control block
    fl.dt_part = dt_part;
    fl.t_base = s->t;
    if (use_fused(ctx, dm, f32)) {
        fl.xpart = s->xpart.as<double>();
        hipError_t e = timed(ctx, 0, [&] { return launch_stage(dm, f32, fl, done, 0, st, &ss->fallbacks); });
        if (e != hipSuccess) return e;
        return timed(ctx, 1, [&] { return launch_stage(dm, f32, fl, done, 1, st, &ss->fallbacks); });
    }
    hipError_t e = timed(ctx, 0, [&] { return launch_reconstruct(dm, f32, in, fv, nullptr, 0, done, st, &ss->fallbacks); });
    if (e != hipSuccess) return e;
    return timed(ctx, 1, [&] { return launch_flux(dm, f32, fl, st); });
}

// the work buffers a stage needs: face values, and the fused stage's partial states
bool stage_buffers(cteno_ctx *ctx, cteno_sol *s, bool f32) {
    if (!s->fv(f32)) return false;
    const DeviceMesh &dm = s->mesh->dm;
    if (use_fused(ctx, dm, f32) && !s->xpart.p) {
        s->xpart = DevBuf(ctx, (size_t)std::max<int64_t>(dm.n_cross, 1) * dm.nv * sizeof(double));
        if (!s->xpart.p) return false;
    }
    return true;
}
}  // namespace

extern "C" cteno_status cteno_rk_stage(cteno_ctx *ctx, const cteno_mesh *m, cteno_sol *sol, int32_t precision,
                                       int32_t stage, double dt) {
    if (!ctx || !m || !sol) return fail(CTENO_ERR_INVALID, "NULL argument");
    if (sol->mesh != m) return fail(CTENO_ERR_INVALID, "solution belongs to another mesh");
    if (stage < 0 || stage > 2) return fail(CTENO_ERR_INVALID, "stage must be 0, 1 or 2");
    bool f32;
    if (cteno_status rc = check_precision(m, precision, f32)) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    if (!stage_buffers(ctx, sol, f32)) return fail(CTENO_ERR_NOMEM, "device allocation failed");
    HIP_TRY(issue_stage(ctx, sol, f32, stage, nullptr, dt, nullptr, nullptr, ctx->stream()));
    if (stage == 2) sol->t += dt;
    return CTENO_OK;
}

// ---------------------------------------------------------------------------
// time march
// ---------------------------------------------------------------------------
namespace {
hipError_t issue_step(cteno_ctx *ctx, cteno_sol *s, bool f32, hipStream_t st) {
    Ctrl *c = s->ctrl.as<Ctrl>();
    double *part = s->dt_part.as<double>();
    const DeviceMesh &dm = s->mesh->dm;
    hipError_t e = launch_control(c, part, use_fused(ctx, dm, f32) ? dm.dt_parts() : dm.blocks(), 0, st);
    for (int stage = 0; stage < 3 && e == hipSuccess; ++stage)
        e = issue_stage(ctx, s, f32, stage, &c->dt, 0.0, c, stage == 2 ? part : nullptr, st);
    return e;
}
}  // namespace

extern "C" cteno_status cteno_solve(cteno_ctx *ctx, const cteno_mesh *m, cteno_sol *s, int32_t precision,
                                    double t_final, int64_t max_steps, double cfl, int32_t use_graph,
                                    int64_t *steps_done) {
    if (!ctx || !m || !s) return fail(CTENO_ERR_INVALID, "NULL argument");
    if (s->mesh != m) return fail(CTENO_ERR_INVALID, "solution belongs to another mesh");
    if (!(cfl > 0) || max_steps < 0) return fail(CTENO_ERR_INVALID, "bad cfl or max_steps");
    bool f32;
    if (cteno_status rc = check_precision(m, precision, f32)) return rc;
    HIP_TRY(hipSetDevice(ctx->device));
    if (!stage_buffers(ctx, s, f32)) return fail(CTENO_ERR_NOMEM, "device allocation failed");
    const DeviceMesh &dm = m->dm;
    hipStream_t st = ctx->stream();
    Ctrl *dc = s->ctrl.as<Ctrl>();
    Ctrl &h = *s->h_ctrl;
    std::memset(&h, 0, sizeof(Ctrl));
    h.t = s->t;
    h.t_final = t_final;
    h.cfl = cfl;
    h.max_steps = max_steps;
    h.dt_cand_bits = 0x7FF0000000000000ull;
    HIP_TRY(hipMemcpyAsync(dc, &h, sizeof(Ctrl), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_dt_partials(dm, f32, s->U[0].as<double>(), s->dt_part.as<double>(), st));
    if (use_fused(ctx, dm, f32) && dm.cross_blocks())    // the second stage kernel's minima: none yet
        HIP_TRY(launch_fill_u64((unsigned long long *)(s->dt_part.as<double>() + dm.blocks()),
                                0x7FF0000000000000ull, (size_t)dm.cross_blocks(), st));

    // graphs need a capturable stream: the context's own stream when the
    // caller uses the null stream
    const bool graph = use_graph && !ctx->timing;
    hipStream_t gs = st;
    hipEvent_t ev = nullptr;
    if (graph && st == nullptr) {
        gs = ctx->own_stream;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(ev, st));
        HIP_TRY(hipStreamWaitEvent(gs, ev, 0));
    }
    hipGraphExec_t &gx = s->graph[f32 ? 1 : 0];
    if (gx && s->graph_fused[f32 ? 1 : 0] != use_fused(ctx, dm, f32)) {   // captured with the other stage kernels
        (void)hipGraphExecDestroy(gx);
        gx = nullptr;
    }
    if (graph && !gx) {
        s->graph_fused[f32 ? 1 : 0] = use_fused(ctx, dm, f32);
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
        hipError_t e = issue_step(ctx, s, f32, gs);
        hipError_t e2 = hipStreamEndCapture(gs, &g);
        if (e != hipSuccess) return fail(CTENO_ERR_DEVICE, std::string("capture: ") + hipGetErrorString(e));
        HIP_TRY(e2);
        HIP_TRY(hipGraphInstantiate(&gx, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
    }
    // steps are issued in chunks between host checks of the done flag; a
    // step issued after the march has reached t_final exits at once on the
    // device.  No more steps than the budget are issued.
    int64_t issued = 0;
    while (issued < max_steps) {
        const int64_t chunk = std::min<int64_t>(16, max_steps - issued);
        for (int64_t k = 0; k < chunk; ++k) {
            if (graph) HIP_TRY(hipGraphLaunch(gx, gs));
            else HIP_TRY(issue_step(ctx, s, f32, gs));
        }
        issued += chunk;
        HIP_TRY(hipMemcpyAsync(&h, dc, sizeof(Ctrl), hipMemcpyDeviceToHost, gs));
        HIP_TRY(hipStreamSynchronize(gs));
        collect_timing(ctx);
        if (h.done) break;
    }
    HIP_TRY(launch_control(dc, nullptr, 0, 1, gs));
    HIP_TRY(hipMemcpyAsync(&h, dc, sizeof(Ctrl), hipMemcpyDeviceToHost, gs));
    HIP_TRY(hipStreamSynchronize(gs));
    if (ev) {
        (void)hipEventDestroy(ev);
    }
    s->t = h.t;
    if (steps_done) *steps_done = h.step;
    if (h.nonphysical) return fail(CTENO_ERR_NONPHYSICAL, "non-physical state (density or pressure <= 0, or NaN)");
    return CTENO_OK;
}

extern "C" cteno_status cteno_count_flips(cteno_ctx *ctx, const cteno_mesh *m, const cteno_sol *sol, int64_t *flips) {
    if (!ctx || !m || !sol || !flips) return fail(CTENO_ERR_INVALID, "NULL argument");
    if (m->dm.precision != CTENO_BOTH) return fail(CTENO_ERR_INVALID, "needs both pseudo-inverse copies (CTENO_BOTH)");
    HIP_TRY(hipSetDevice(ctx->device));
    const DeviceMesh &dm = m->dm;
    hipStream_t st = ctx->stream();
    cteno_sol *s = const_cast<cteno_sol *>(sol);
    DevBuf d64(ctx, (size_t)dm.Np * dm.delta_bytes()), d32(ctx, (size_t)dm.Np * dm.delta_bytes()),
        cnt(ctx, sizeof(unsigned long long));
    void *fv64 = s->fv(false), *fv32 = s->fv(true);
    if (!d64.p || !d32.p || !cnt.p || !fv64 || !fv32) return fail(CTENO_ERR_NOMEM, "device allocation failed");
    HIP_TRY(launch_reconstruct(dm, false, s->U[0].as<double>(), fv64, d64.as<uint8_t>(), 1, nullptr, st));
    HIP_TRY(launch_reconstruct(dm, true, s->U[0].as<double>(), fv32, d32.as<uint8_t>(), 1, nullptr, st));
    HIP_TRY(launch_fill_u64(cnt.as<unsigned long long>(), 0ull, 1, st));
    HIP_TRY(launch_count_diff(dm, d64.as<uint8_t>(), d32.as<uint8_t>(), cnt.as<unsigned long long>(), st));
    unsigned long long c = 0;
    HIP_TRY(hipMemcpyAsync(&c, cnt.p, sizeof(c), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *flips = (int64_t)c;
    return CTENO_OK;
}

extern "C" cteno_status cteno_util_copy(cteno_ctx *ctx, void *dst, const void *src, size_t n_bytes) {
    if (!ctx || !dst || !src || (n_bytes % 16)) return fail(CTENO_ERR_INVALID, "bad copy arguments");
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(launch_copy16(dst, src, n_bytes / 16, ctx->stream()));
    return CTENO_OK;
}

// ---------------------------------------------------------------------------
// serving: continuous batching of independent solves
// ---------------------------------------------------------------------------
namespace {
using Clock = std::chrono::steady_clock;

enum { REQ_QUEUED = 0, REQ_READY = 1, REQ_RUNNING = 2, REQ_DONE = 3, REQ_FAILED = 4 };

struct ServerRequest {
    uint64_t ticket = 0;
    std::vector<double> xy;
    std::vector<int32_t> tri;
    cteno_mesh_desc desc{};
    std::vector<double> u0;
    int32_t n_steps = 0;
    double cfl = 0.3;
    // submitted, host mesh built, upload started (memory reserved), resident
    // on the device, in a batch slot, finished
    Clock::time_point t_submit, t_built, t_admit, t_ready, t_running, t_done;
    int state = REQ_QUEUED;
    HostMesh hm;
    std::string err;
    cteno_status fail_status = CTENO_OK;
    std::vector<double> result;
    double t_end = 0.0;
    int64_t steps = 0;
    int64_t fallbacks = 0;
};

struct ServerSlot {
    std::shared_ptr<ServerRequest> req;
    DeviceMesh dm;
    std::vector<DevBuf> bufs;
    DevBuf U[3], FV, dt_part;
    int ctrl_index = -1;
    int64_t bytes = 0;
};
}  // namespace

// SSP-RK3 steps per tick: one graph launch and one host round trip cover
// this many batched steps (a solve that finishes within a tick idles through
// the rest of it)
constexpr int kStepsPerTick = 4;

struct cteno_server {
    cteno_ctx *ctx = nullptr;
    cteno_scheme scheme{};
    int64_t budget = 0;
    int max_slots = 0;
    int64_t max_blocks = 0;
    hipStream_t stream = nullptr;
    DeviceMesh proto;              // scheme constants shared by every slot
    // device slot table, slot count, control pool
    DevBuf d_table, d_nslots, d_ctrl;
    BatchSlot *h_table = nullptr;
    int *h_nslots = nullptr;
    Ctrl *h_ctrl = nullptr;
    // one captured tick per grid size (powers of two up to max_blocks)
    std::map<int64_t, hipGraphExec_t> graphs;
    // host side
    std::mutex mu;
    std::condition_variable cv_build, cv_upload, cv_sched, cv_done, cv_budget;
    std::deque<std::shared_ptr<ServerRequest>> to_build, built;
    std::deque<std::unique_ptr<ServerSlot>> prepared;   // resident on the device, waiting for a slot
    std::map<uint64_t, std::shared_ptr<ServerRequest>> requests;
    std::vector<std::unique_ptr<ServerSlot>> active;
    std::vector<int> free_ctrl;
    uint64_t next_ticket = 1;
    int64_t bytes_used = 0, peak_bytes = 0;
    int peak_active = 0;
    int64_t ticks = 0, cell_stages = 0, n_submitted = 0, n_finished = 0, fallbacks = 0;
    bool stop = false;
    std::string sched_error;
    std::vector<std::thread> builders, uploaders;
    std::vector<hipStream_t> upload_streams;
    std::thread scheduler;
};

namespace {

// steady and transient device bytes of a slot with N cells
void slot_footprint(const cteno_server *sv, int64_t N, int64_t &steady, int64_t &transient) {
    const int r = sv->scheme.degree;
    const int64_t Np = pad64(N);
    const int64_t E32 = round_up(pinv_entries(r), 4), E64 = round_up(pinv_entries(r), 2);
    const int S = dims_S(r), SP = round_up(S, 4);
    steady = Np * (E32 * 4 + SP * 4 + 1 + 12 * 4 + 8 + 3 * 32 + 3 * kNq * 4 * 4) + N * 4 + ((N + 255) / 256) * 8;
    transient = Np * (E64 * 8 + 6 * 8 + S + 2 * S) + 64;
}

// a request's device state on a builder's stream: mesh arrays and FP64
// precompute, state buffers, the initial state in internal order and its
// time-step partials; synchronises that stream
cteno_status prepare_slot(cteno_server *sv, const std::shared_ptr<ServerRequest> &rq, std::unique_ptr<ServerSlot> &sl,
                          hipStream_t st) {
    sl = std::make_unique<ServerSlot>();
    sl->req = rq;
    cteno_scheme s = sv->scheme;
    s.precision = CTENO_MIXED;
    int64_t bytes = 0;
    cteno_status rc = upload_device_mesh(sv->ctx, st, rq->hm, s, sl->dm, sl->bufs, bytes, false);
    if (rc != CTENO_OK) return rc;
    const DeviceMesh &dm = sl->dm;
    const size_t sb = (size_t)dm.Np * dm.nv * sizeof(double);
    for (auto &u : sl->U) {
        u = DevBuf(sv->ctx, sb);
        if (!u.p) return fail(CTENO_ERR_NOMEM, "device allocation failed");
        HIP_TRY(hipMemsetAsync(u.p, 0, sb, st));
    }
    sl->FV = DevBuf(sv->ctx, (size_t)dm.Np * 3 * kNq * dm.nv * sizeof(float));
    sl->dt_part = DevBuf(sv->ctx, (size_t)dm.blocks() * sizeof(double));
    if (!sl->FV.p || !sl->dt_part.p) return fail(CTENO_ERR_NOMEM, "device allocation failed");
    bytes += (int64_t)(3 * sb + sl->FV.bytes + sl->dt_part.bytes);
    // initial state: caller order -> internal order
    DevBuf tmp(sv->ctx, (size_t)dm.N * dm.nv * sizeof(double));
    if (!tmp.p) return fail(CTENO_ERR_NOMEM, "device allocation failed");
    HIP_TRY(hipMemcpyAsync(tmp.p, rq->u0.data(), (size_t)dm.N * dm.nv * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_user_to_state(dm, tmp.as<double>(), sl->U[0].as<double>(), st));
    HIP_TRY(launch_dt_partials(dm, true, sl->U[0].as<double>(), sl->dt_part.as<double>(), st));
    HIP_TRY(hipStreamSynchronize(st));     // tmp and the host u0 are released after this
    rq->u0.clear();
    rq->u0.shrink_to_fit();
    sl->bytes = bytes;
    return CTENO_OK;
}

void fail_request(cteno_server *sv, ServerRequest &rq, cteno_status rc, const std::string &err) {
    rq.state = REQ_FAILED;
    rq.fail_status = rc;
    rq.err = err;
    rq.t_done = Clock::now();
    rq.hm = HostMesh();
    sv->n_finished++;
    sv->cv_done.notify_all();
}

// A builder thread takes queued requests in arrival order and builds each
// one's host mesh and stencils.
void builder_main(cteno_server *sv, int threads_each) {
    set_builder_threads(threads_each);
    for (;;) {
        std::shared_ptr<ServerRequest> rq;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_build.wait(lk, [&] { return sv->stop || !sv->to_build.empty(); });
            if (sv->to_build.empty()) return;
            rq = sv->to_build.front();
            sv->to_build.pop_front();
        }
        std::string err;
        cteno_status rc = build_host_mesh(rq->desc, sv->scheme, rq->hm, err);
        if (rc == CTENO_OK) {
            int64_t steady = 0, transient = 0;
            slot_footprint(sv, rq->hm.N, steady, transient);
            if (steady + transient > sv->budget) { rc = CTENO_ERR_BUSY; err = "request exceeds the HBM budget"; }
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        rq->t_built = Clock::now();
        if (rc != CTENO_OK) { fail_request(sv, *rq, rc, err); continue; }
        rq->state = REQ_READY;
        sv->built.push_back(rq);
        sv->cv_upload.notify_one();
    }
}

// An upload thread takes built requests in the order they were built, waits
// until the device budget holds the request's steady plus transient
// footprint beside the resident solves, uploads it and runs its FP64
// precompute on its own stream (overlapping the batched ticks), and hands the
// resident solve to the scheduler.
void uploader_main(cteno_server *sv, int index) {
    const bool dev_ok = hipSetDevice(sv->ctx->device) == hipSuccess;
    const hipStream_t st = sv->upload_streams[index];
    for (;;) {
        std::shared_ptr<ServerRequest> rq;
        int64_t reserve = 0;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_upload.wait(lk, [&] { return sv->stop || !sv->built.empty(); });
            if (sv->stop) return;
            rq = sv->built.front();
            sv->built.pop_front();
            if (!dev_ok) { fail_request(sv, *rq, CTENO_ERR_DEVICE, "hipSetDevice failed"); continue; }
            int64_t steady = 0, transient = 0;
            slot_footprint(sv, rq->hm.N, steady, transient);
            reserve = steady + transient;
            sv->cv_budget.wait(lk, [&] { return sv->stop || sv->bytes_used + reserve <= sv->budget; });
            if (sv->stop) return;
            sv->bytes_used += reserve;
            sv->peak_bytes = std::max(sv->peak_bytes, sv->bytes_used);
            rq->t_admit = Clock::now();
        }
        std::unique_ptr<ServerSlot> sl;
        const cteno_status rc = prepare_slot(sv, rq, sl, st);
        const std::string perr = g_err;
        std::lock_guard<std::mutex> lk(sv->mu);
        if (rc != CTENO_OK) {
            sv->bytes_used -= reserve;
            sl.reset();
            fail_request(sv, *rq, rc, perr);
            sv->cv_budget.notify_all();
            continue;
        }
        // the transient precompute buffers are gone: keep what stays resident
        sv->bytes_used += sl->bytes - reserve;
        sv->peak_bytes = std::max(sv->peak_bytes, sv->bytes_used);
        rq->t_ready = Clock::now();
        sv->prepared.push_back(std::move(sl));
        sv->cv_budget.notify_all();
        sv->cv_sched.notify_all();
    }
}

// the result of a finished slot in caller order, into `result` (the
// caller publishes it under the server lock)
cteno_status retire(cteno_server *sv, ServerSlot &sl, std::vector<double> &result) {
    const DeviceMesh &dm = sl.dm;
    DevBuf tmp(sv->ctx, (size_t)dm.N * dm.nv * sizeof(double));
    if (!tmp.p) return fail(CTENO_ERR_NOMEM, "device allocation failed");
    result.resize((size_t)dm.N * dm.nv);
    HIP_TRY(launch_state_to_user(dm, sl.U[0].as<double>(), tmp.as<double>(), sv->stream));
    HIP_TRY(hipMemcpyAsync(result.data(), tmp.p, result.size() * sizeof(double), hipMemcpyDeviceToHost, sv->stream));
    HIP_TRY(hipStreamSynchronize(sv->stream));
    return CTENO_OK;
}

void scheduler_fail(cteno_server *sv, const std::string &m) {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->sched_error = m;
    for (auto &kv : sv->requests)
        if (kv.second->state != REQ_DONE && kv.second->state != REQ_FAILED) {
            kv.second->state = REQ_FAILED;
            kv.second->fail_status = CTENO_ERR_DEVICE;
            kv.second->err = "server stopped: " + m;
            kv.second->t_done = Clock::now();
            sv->n_finished++;
        }
    sv->to_build.clear();
    sv->built.clear();
    sv->stop = true;
    sv->cv_build.notify_all();
    sv->cv_upload.notify_all();
    sv->cv_budget.notify_all();
    sv->cv_done.notify_all();
}

// the captured tick for a grid of `blocks` blocks (captured on first use)
hipGraphExec_t tick_graph(cteno_server *sv, int64_t blocks) {
    auto it = sv->graphs.find(blocks);
    if (it != sv->graphs.end()) return it->second;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(sv->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    hipError_t e = hipSuccess;
    for (int k = 0; k < kStepsPerTick && e == hipSuccess; ++k)
        e = launch_batch_step(sv->proto, sv->d_table.as<BatchSlot>(), sv->d_nslots.as<int>(), sv->max_slots, blocks,
                              sv->stream);
    hipError_t e2 = hipStreamEndCapture(sv->stream, &g);
    hipGraphExec_t x = nullptr;
    if (e == hipSuccess && e2 == hipSuccess && hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) x = nullptr;
    if (g) (void)hipGraphDestroy(g);
    if (x) sv->graphs[blocks] = x;
    return x;
}

void scheduler_main(cteno_server *sv) {
    if (hipSetDevice(sv->ctx->device) != hipSuccess) { scheduler_fail(sv, "hipSetDevice failed"); return; }
    bool dirty = true;
    int64_t grid = 0;
    for (;;) {
        // admissions: resident solves, in the order their uploads finished,
        // while slots are free (no device work: the builders did it)
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            if (sv->active.empty())
                sv->cv_sched.wait(lk, [&] { return sv->stop || !sv->prepared.empty(); });
            if (sv->stop && sv->active.empty()) return;
            while (!sv->stop && !sv->prepared.empty() && (int)sv->active.size() < sv->max_slots) {
                std::unique_ptr<ServerSlot> sl = std::move(sv->prepared.front());
                sv->prepared.pop_front();
                sl->ctrl_index = sv->free_ctrl.back();
                sv->free_ctrl.pop_back();
                Ctrl &c = sv->h_ctrl[sl->ctrl_index];
                c = Ctrl{};
                c.t = 0.0;
                c.t_final = INFINITY;
                c.cfl = sl->req->cfl;
                c.max_steps = sl->req->n_steps;
                // stream-ordered before the next tick and before this entry's read-back
                if (hipMemcpyAsync(sv->d_ctrl.as<Ctrl>() + sl->ctrl_index, &c, sizeof(Ctrl), hipMemcpyHostToDevice,
                                   sv->stream) != hipSuccess) {
                    lk.unlock();
                    scheduler_fail(sv, "control upload failed");
                    return;
                }
                sl->req->state = REQ_RUNNING;
                sl->req->t_running = Clock::now();
                sv->active.push_back(std::move(sl));
                sv->peak_active = std::max(sv->peak_active, (int)sv->active.size());
                dirty = true;
            }
        }
        if (sv->active.empty()) continue;
        if (dirty) {
            int64_t b0 = 0;
            for (size_t k = 0; k < sv->active.size(); ++k) {
                ServerSlot &sl = *sv->active[k];
                BatchSlot &t = sv->h_table[k];
                t.N = sl.dm.N;
                t.block0 = b0;
                t.nblocks = sl.dm.blocks();
                t.slot = sl.dm.slot;
                t.flags = sl.dm.flags;
                t.P = sl.dm.P32;
                t.fr = sl.dm.fr32;
                t.area = sl.dm.area;
                for (int q = 0; q < 3; ++q) t.U[q] = sl.U[q].as<double>();
                t.FV = sl.FV.as<float>();
                t.dt_part = sl.dt_part.as<double>();
                t.ctrl = sv->d_ctrl.as<Ctrl>() + sl.ctrl_index;
                b0 += t.nblocks;
            }
            *sv->h_nslots = (int)sv->active.size();
            if (b0 > sv->max_blocks) { scheduler_fail(sv, "block budget exceeded"); return; }
            // the smallest power-of-two grid that covers the active blocks
            grid = 64;
            while (grid < b0) grid *= 2;
            grid = std::min(grid, sv->max_blocks);
            if (hipMemcpyAsync(sv->d_table.p, sv->h_table, sizeof(BatchSlot) * sv->active.size(),
                               hipMemcpyHostToDevice, sv->stream) != hipSuccess ||
                hipMemcpyAsync(sv->d_nslots.p, sv->h_nslots, sizeof(int), hipMemcpyHostToDevice, sv->stream) !=
                    hipSuccess) {
                scheduler_fail(sv, "slot table upload failed");
                return;
            }
            dirty = false;
        }
        // kStepsPerTick SSP-RK3 steps of every active solve
        hipGraphExec_t gx = tick_graph(sv, grid);
        if (!gx) { scheduler_fail(sv, "tick capture failed"); return; }
        if (hipGraphLaunch(gx, sv->stream) != hipSuccess) { scheduler_fail(sv, "graph launch failed"); return; }
        sv->ticks += kStepsPerTick;
        // read back the control blocks of the active slots
        for (size_t k = 0; k < sv->active.size(); ++k) {
            const int ci = sv->active[k]->ctrl_index;
            if (hipMemcpyAsync(sv->h_ctrl + ci, sv->d_ctrl.as<Ctrl>() + ci, sizeof(Ctrl), hipMemcpyDeviceToHost,
                               sv->stream) != hipSuccess) { scheduler_fail(sv, "control read-back failed"); return; }
        }
        if (hipStreamSynchronize(sv->stream) != hipSuccess) { scheduler_fail(sv, "device error during a step"); return; }
        for (size_t k = 0; k < sv->active.size();) {
            ServerSlot &sl = *sv->active[k];
            const Ctrl &c = sv->h_ctrl[sl.ctrl_index];
            if (!c.done) { ++k; continue; }
            std::vector<double> result;
            const cteno_status rc = c.nonphysical ? CTENO_ERR_NONPHYSICAL : retire(sv, sl, result);
            const std::string err = c.nonphysical ? "non-physical state (density or pressure <= 0, or NaN)" : g_err;
            std::lock_guard<std::mutex> lk(sv->mu);
            ServerRequest &rq = *sl.req;
            rq.steps = c.step;
            rq.t_end = c.t;
            rq.fallbacks = (int64_t)c.fallbacks;
            rq.hm = HostMesh();
            rq.t_done = Clock::now();
            if (rc == CTENO_OK) {
                rq.result = std::move(result);
                rq.state = REQ_DONE;
            } else {
                rq.state = REQ_FAILED;
                rq.fail_status = rc;
                rq.err = err;
            }
            sv->cell_stages += sl.dm.N * 3 * c.step;
            sv->fallbacks += (int64_t)c.fallbacks;
            sv->bytes_used -= sl.bytes;
            sv->free_ctrl.push_back(sl.ctrl_index);
            sv->n_finished++;
            sv->active.erase(sv->active.begin() + k);
            dirty = true;
            sv->cv_budget.notify_all();
            sv->cv_done.notify_all();
        }
    }
}
}  // namespace

extern "C" cteno_status cteno_server_create(cteno_ctx *ctx, const cteno_scheme *scheme, size_t hbm_budget_bytes,
                                            int32_t max_slots, cteno_server **out) {
    if (!ctx || !scheme || !out) return fail(CTENO_ERR_INVALID, "NULL argument");
    if (cteno_status rc = check_scheme(*scheme)) return rc;
    if (scheme->physics != CTENO_EULER) return fail(CTENO_ERR_INVALID, "serving runs the Euler equations");
    if (scheme->degree > 3) return fail(CTENO_ERR_INVALID, "serving runs degree 2 or 3");
    if (scheme->variables != CTENO_VARS_CONSERVED) return fail(CTENO_ERR_INVALID, "serving runs conserved variables");
    if (max_slots < 1 || max_slots > 1024) return fail(CTENO_ERR_INVALID, "max_slots must be 1..1024");
    if (hbm_budget_bytes < (1u << 20)) return fail(CTENO_ERR_INVALID, "budget too small");
    HIP_TRY(hipSetDevice(ctx->device));
    auto sv = std::make_unique<cteno_server>();
    sv->ctx = ctx;
    sv->scheme = *scheme;
    sv->scheme.precision = CTENO_MIXED;
    sv->budget = (int64_t)hbm_budget_bytes;
    sv->max_slots = max_slots;
    // the batched grid covers the most cells the budget can hold, plus one
    // partial block per slot
    int64_t steady, transient;
    slot_footprint(sv.get(), 1 << 20, steady, transient);
    const double per_cell = (double)steady / (1 << 20);
    sv->max_blocks = (int64_t)(sv->budget / per_cell) / 256 + max_slots + 1;
    HIP_TRY(hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking));
    sv->d_table = DevBuf(ctx, sizeof(BatchSlot) * max_slots);
    sv->d_nslots = DevBuf(ctx, sizeof(int));
    sv->d_ctrl = DevBuf(ctx, sizeof(Ctrl) * max_slots);
    if (!sv->d_table.p || !sv->d_nslots.p || !sv->d_ctrl.p) return fail(CTENO_ERR_NOMEM, "device allocation failed");
    HIP_TRY(hipMemsetAsync(sv->d_nslots.p, 0, sizeof(int), sv->stream));
    HIP_TRY(hipMemsetAsync(sv->d_ctrl.p, 0, sizeof(Ctrl) * max_slots, sv->stream));
    HIP_TRY(hipHostMalloc((void **)&sv->h_table, sizeof(BatchSlot) * max_slots, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void **)&sv->h_nslots, sizeof(int), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void **)&sv->h_ctrl, sizeof(Ctrl) * max_slots, hipHostMallocDefault));
    for (int k = max_slots - 1; k >= 0; --k) sv->free_ctrl.push_back(k);
    // scheme constants (tables, linear weights) shared by every slot
    DeviceMesh &p = sv->proto;
    p.r = scheme->degree; p.K = dims_K(p.r); p.S = dims_S(p.r); p.nv = 4; p.physics = CTENO_EULER;
    p.scheme = scheme->scheme; p.gamma_form = scheme->gamma_form; p.precision = CTENO_MIXED;
    p.gamma = scheme->gamma; p.lam1p = scheme->lambda1_prime; p.ct = scheme->c_t; p.eps = scheme->eps;
    p.positivity = scheme->positivity;
    make_ref_tables(p.r, p.tab);
    HIP_TRY(hipStreamSynchronize(sv->stream));
    // several mesh builders, each with a share of the host threads, and two
    // upload threads, each with a stream of its own (default priority)
    constexpr int kUploaders = 2;
    for (int k = 0; k < kUploaders; ++k) {
        hipStream_t us = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&us, hipStreamNonBlocking));
        sv->upload_streams.push_back(us);
    }
    const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
    const int nb = std::max(1, std::min(4, hw / 2));
    cteno_server *raw = sv.release();
    for (int k = 0; k < nb; ++k) raw->builders.emplace_back(builder_main, raw, std::max(1, std::min(hw, 16) / nb));
    for (int k = 0; k < kUploaders; ++k) raw->uploaders.emplace_back(uploader_main, raw, k);
    raw->scheduler = std::thread(scheduler_main, raw);
    *out = raw;
    return CTENO_OK;
}

extern "C" cteno_status cteno_server_submit(cteno_server *sv, const cteno_mesh_desc *desc, const double *u0,
                                            int32_t n_steps, double cfl, uint64_t *ticket) {
    if (!sv || !desc || !u0 || !ticket) return fail(CTENO_ERR_INVALID, "NULL argument");
    if (n_steps < 0 || !(cfl > 0)) return fail(CTENO_ERR_INVALID, "bad n_steps or cfl");
    if (desc->n_cells <= 0 || desc->n_vertices <= 0) return fail(CTENO_ERR_INVALID, "empty mesh");
    for (int k = 0; k < 4; ++k)
        if (desc->bc[k] == CTENO_INFLOW || desc->split_kind[k] != 0)
            return fail(CTENO_ERR_INVALID, "the server takes periodic, wall and transmissive sides only");
    auto rq = std::make_shared<ServerRequest>();
    rq->t_submit = Clock::now();
    rq->xy.assign(desc->xy, desc->xy + 2 * (size_t)desc->n_vertices);
    rq->tri.assign(desc->tri, desc->tri + 3 * (size_t)desc->n_cells);
    rq->desc = *desc;
    rq->desc.xy = rq->xy.data();
    rq->desc.tri = rq->tri.data();
    rq->u0.assign(u0, u0 + 4 * (size_t)desc->n_cells);
    rq->n_steps = n_steps;
    rq->cfl = cfl;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (!sv->sched_error.empty()) return fail(CTENO_ERR_DEVICE, "server stopped: " + sv->sched_error);
    rq->ticket = sv->next_ticket++;
    sv->requests[rq->ticket] = rq;
    sv->to_build.push_back(rq);
    sv->n_submitted++;
    sv->cv_build.notify_one();
    *ticket = rq->ticket;
    return CTENO_OK;
}

extern "C" cteno_status cteno_server_poll(cteno_server *sv, uint64_t ticket, int32_t *state, double *u_out,
                                          int64_t *steps_done, double *latency_s) {
    if (!sv) return fail(CTENO_ERR_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(ticket);
    if (it == sv->requests.end()) return fail(CTENO_ERR_INVALID, "unknown or released ticket");
    ServerRequest &rq = *it->second;
    if (state) *state = rq.state;
    const bool finished = rq.state == REQ_DONE || rq.state == REQ_FAILED;
    if (finished && latency_s) *latency_s = std::chrono::duration<double>(rq.t_done - rq.t_submit).count();
    if (finished && steps_done) *steps_done = rq.steps;
    if (rq.state == REQ_FAILED) {
        g_err = rq.err;
        const cteno_status rc = rq.fail_status == CTENO_OK ? CTENO_ERR_DEVICE : rq.fail_status;
        if (u_out) sv->requests.erase(it);
        return rc;
    }
    if (rq.state == REQ_DONE && u_out) {
        std::memcpy(u_out, rq.result.data(), rq.result.size() * sizeof(double));
        sv->requests.erase(it);
    }
    return CTENO_OK;
}

extern "C" cteno_status cteno_server_drain(cteno_server *sv) {
    if (!sv) return fail(CTENO_ERR_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] { return sv->n_finished >= sv->n_submitted; });
    if (!sv->sched_error.empty()) return fail(CTENO_ERR_DEVICE, "server stopped: " + sv->sched_error);
    return CTENO_OK;
}

extern "C" cteno_status cteno_server_get_stats(cteno_server *sv, cteno_server_stats *st) {
    if (!sv || !st) return fail(CTENO_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    st->submitted = sv->n_submitted;
    st->finished = sv->n_finished;
    st->active = (int32_t)sv->active.size();
    st->peak_active = sv->peak_active;
    st->ticks = sv->ticks;
    st->cell_stages = sv->cell_stages;
    st->bytes_in_use = sv->bytes_used;
    st->peak_bytes = sv->peak_bytes;
    st->budget_bytes = sv->budget;
    st->fallbacks = sv->fallbacks;
    return CTENO_OK;
}

extern "C" cteno_status cteno_server_request_info(cteno_server *sv, uint64_t ticket, cteno_request_info *info) {
    if (!sv || !info) return fail(CTENO_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(ticket);
    if (it == sv->requests.end()) return fail(CTENO_ERR_INVALID, "unknown or released ticket");
    const ServerRequest &rq = *it->second;
    auto sec = [](Clock::time_point a, Clock::time_point b) {
        return (a.time_since_epoch().count() && b.time_since_epoch().count() && b >= a)
                   ? std::chrono::duration<double>(b - a).count() : 0.0;
    };
    *info = cteno_request_info{};
    info->state = rq.state;
    info->status = rq.state == REQ_FAILED ? (rq.fail_status == CTENO_OK ? CTENO_ERR_DEVICE : rq.fail_status) : CTENO_OK;
    info->n_cells = (int64_t)rq.tri.size() / 3;
    info->steps_done = rq.steps;
    info->fallbacks = rq.fallbacks;
    const bool finished = rq.state == REQ_DONE || rq.state == REQ_FAILED;
    info->latency_s = finished ? sec(rq.t_submit, rq.t_done) : 0.0;
    info->build_s = sec(rq.t_submit, rq.t_built);
    info->queue_s = sec(rq.t_built, rq.t_admit) + sec(rq.t_ready, rq.t_running);
    info->admit_s = sec(rq.t_admit, rq.t_ready);
    info->run_s = finished ? sec(rq.t_running, rq.t_done) : 0.0;
    return CTENO_OK;
}

extern "C" void cteno_server_destroy(cteno_server *sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->to_build.clear();
        sv->built.clear();
    }
    sv->cv_build.notify_all();
    sv->cv_upload.notify_all();
    sv->cv_budget.notify_all();
    sv->cv_sched.notify_all();
    for (auto &b : sv->builders)
        if (b.joinable()) b.join();
    for (auto &u : sv->uploaders)
        if (u.joinable()) u.join();
    if (sv->scheduler.joinable()) sv->scheduler.join();
    (void)hipSetDevice(sv->ctx->device);
    (void)hipStreamSynchronize(sv->stream);
    for (hipStream_t us : sv->upload_streams) {
        (void)hipStreamSynchronize(us);
        (void)hipStreamDestroy(us);
    }
    sv->prepared.clear();
    sv->active.clear();
    for (auto &kv : sv->graphs) (void)hipGraphExecDestroy(kv.second);
    if (sv->h_table) (void)hipHostFree(sv->h_table);
    if (sv->h_nslots) (void)hipHostFree(sv->h_nslots);
    if (sv->h_ctrl) (void)hipHostFree(sv->h_ctrl);
    sv->d_table.reset();
    sv->d_nslots.reset();
    sv->d_ctrl.reset();
    (void)hipStreamDestroy(sv->stream);
    delete sv;
}
