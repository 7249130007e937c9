// Host-side mesh and stencil construction (C++17, multi-threaded).
//
// Builds, from a triangle list: periodic vertex welding, counter-clockwise
// cells, faces and their owners, the central stencil of M = 2K cells
// (sec. 2.1) and one compact directional stencil per face inside it (sec.
// 2.3, fig. 1; degree 1 up to cubic, ceil(r/2) above, M_d = 2 K_d cells,
// admissible with at least K_d + 1), then lays everything out for the device in 64-cell
// tiles, optionally in Morton order.
//
// Stencil rule (the paper only names its construction):
//   * centroids c_i = ((x_a + x_b) + x_c) / 3 from the input vertex order;
//   * offsets between cells use the nearest periodic image of the centroid
//     difference; squared distance d2 = dx*dx + dy*dy;
//   * central stencil: layers of vertex neighbours of the cell (layer k+1 =
//     unvisited cells sharing a welded vertex with layer k), taken whole
//     while they fit in M; the first layer that does not fit contributes
//     first the face neighbours, then cells by ascending (d2, cell id);
//   * directional stencil of face f (vertices P_f -> P_f+1 of the CCW cell):
//     central-stencil cells whose offset q satisfies cross(P_f - c, q) >= 0
//     and cross(q, P_f+1 - c) > 0, the face neighbours being assigned to
//     their own faces; the face neighbour first, then up to 3 more by
//     ascending (d2, id); admissible when the face is interior and the
//     stencil holds at least 3 cells.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "cteno_internal.h"

namespace cteno {

namespace {

thread_local int tl_max_threads = 16;

template <class F>
void parallel_for(int64_t n, F &&fn) {
    unsigned hw = std::thread::hardware_concurrency();
    int nt = (int)std::max(1u, std::min(hw, (unsigned)tl_max_threads));
    if (n < 4096) nt = 1;
    if (nt == 1) {
        for (int64_t i = 0; i < n; ++i) fn(i, 0);
        return;
    }
    std::atomic<int64_t> next{0};
    const int64_t chunk = 1024;
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (;;) {
                int64_t b = next.fetch_add(chunk);
                if (b >= n) break;
                int64_t e = std::min(n, b + chunk);
                for (int64_t i = b; i < e; ++i) fn(i, t);
            }
        });
    for (auto &x : th) x.join();
}

inline int nthreads_for(int64_t n) {
    unsigned hw = std::thread::hardware_concurrency();
    int nt = (int)std::max(1u, std::min(hw, (unsigned)tl_max_threads));
    return n < 4096 ? 1 : nt;
}

struct Builder {
    const cteno_mesh_desc &d;
    int N, nvert, r, K, M, S, Kd, Md;
    int per_x, per_y;
    double Lx, Ly;
    std::vector<int32_t> tri;       // CCW-normalised raw vertex ids
    std::vector<double> cx, cy, area;
    std::vector<int32_t> canon;
    std::vector<int32_t> v2c_off, v2c;
    std::vector<int32_t> fnb, fnbf, fbc;   // user order [3N]
    std::vector<int32_t> cen;              // [N][M]
    std::vector<int32_t> dir;              // [N][3][Md]
    std::vector<int32_t> dirn;             // [N][3]
    std::string err;

    Builder(const cteno_mesh_desc &dd, int rr) : d(dd), N(dd.n_cells), nvert(dd.n_vertices), r(rr) {
        K = dims_K(r);
        M = dims_M(r);
        S = dims_S(r);
        Kd = dims_Kd(r);
        Md = dims_Md(r);
        per_x = dd.bc[0] == CTENO_PERIODIC;
        per_y = dd.bc[2] == CTENO_PERIODIC;
        Lx = dd.box[1] - dd.box[0];
        Ly = dd.box[3] - dd.box[2];
    }

    double X(int v) const { return d.xy[2 * (size_t)v]; }
    double Y(int v) const { return d.xy[2 * (size_t)v + 1]; }

    void offset(int i, int j, int &sx, int &sy, double &dx, double &dy) const {
        double x = cx[j] - cx[i], y = cy[j] - cy[i];
        sx = sy = 0;
        if (per_x) {
            if (x > 0.5 * Lx) { x = x - Lx; sx = -1; }
            else if (x < -0.5 * Lx) { x = x + Lx; sx = 1; }
        }
        if (per_y) {
            if (y > 0.5 * Ly) { y = y - Ly; sy = -1; }
            else if (y < -0.5 * Ly) { y = y + Ly; sy = 1; }
        }
        dx = x;
        dy = y;
    }

    bool geometry() {
        tri.assign(d.tri, d.tri + 3 * (size_t)N);
        cx.resize(N);
        cy.resize(N);
        area.resize(N);
        std::atomic<int64_t> bad{-1};
        parallel_for(N, [&](int64_t i, int) {
            const int32_t *t = d.tri + 3 * i;
            for (int k = 0; k < 3; ++k)
                if (t[k] < 0 || t[k] >= nvert) { bad = i; return; }
            cx[i] = (X(t[0]) + X(t[1]) + X(t[2])) / 3.0;
            cy[i] = (Y(t[0]) + Y(t[1]) + Y(t[2])) / 3.0;
            int32_t *u = tri.data() + 3 * i;
            double s = (X(u[1]) - X(u[0])) * (Y(u[2]) - Y(u[0])) - (X(u[2]) - X(u[0])) * (Y(u[1]) - Y(u[0]));
            if (!(s != 0.0) || !std::isfinite(s)) { bad = i; return; }
            if (s < 0) { std::swap(u[1], u[2]); s = -s; }
            area[i] = 0.5 * s;
        });
        if (bad >= 0) { err = "degenerate or invalid triangle " + std::to_string((long long)bad); return false; }
        return true;
    }

    // union-find welding of the two sides of each periodic pair
    bool weld() {
        canon.resize(nvert);
        std::iota(canon.begin(), canon.end(), 0);
        auto root = [&](int a) { while (canon[a] != a) { canon[a] = canon[canon[a]]; a = canon[a]; } return a; };
        double tol = 1e-9 * (std::fabs(Lx) + std::fabs(Ly));
        for (int dirn = 0; dirn < 2; ++dirn) {
            if (!(dirn == 0 ? per_x : per_y)) continue;
            double lo = dirn == 0 ? d.box[0] : d.box[2];
            double hi = dirn == 0 ? d.box[1] : d.box[3];
            std::vector<std::pair<double, int>> A, B;
            for (int v = 0; v < nvert; ++v) {
                double s = d.xy[2 * (size_t)v + dirn], o = d.xy[2 * (size_t)v + 1 - dirn];
                if (std::fabs(s - lo) <= tol) A.push_back({o, v});
                if (std::fabs(s - hi) <= tol) B.push_back({o, v});
            }
            if (A.size() != B.size() || A.empty()) { err = "periodic seam vertices do not match"; return false; }
            std::sort(A.begin(), A.end());
            std::sort(B.begin(), B.end());
            for (size_t k = 0; k < A.size(); ++k) {
                if (std::fabs(A[k].first - B[k].first) > tol) { err = "periodic seam vertices do not match"; return false; }
                int a = root(A[k].second), b = root(B[k].second);
                if (a != b) { if (a < b) canon[b] = a; else canon[a] = b; }
            }
        }
        for (int v = 0; v < nvert; ++v) canon[v] = root(v);
        return true;
    }

    void vertex_cells() {
        v2c_off.assign(nvert + 1, 0);
        for (int64_t i = 0; i < N; ++i)
            for (int k = 0; k < 3; ++k) v2c_off[canon[tri[3 * i + k]] + 1]++;
        for (int v = 0; v < nvert; ++v) v2c_off[v + 1] += v2c_off[v];
        v2c.resize(3 * (size_t)N);
        std::vector<int32_t> fill(nvert, 0);
        for (int64_t i = 0; i < N; ++i)
            for (int k = 0; k < 3; ++k) {
                int v = canon[tri[3 * i + k]];
                v2c[v2c_off[v] + fill[v]++] = (int32_t)i;
            }
    }

    // face neighbours through shared welded edges
    bool faces() {
        fnb.assign(3 * (size_t)N, -1);
        fnbf.assign(3 * (size_t)N, -1);
        fbc.assign(3 * (size_t)N, -1);
        double tol = 1e-9 * (std::fabs(Lx) + std::fabs(Ly));
        std::atomic<int64_t> bad{-1};
        std::atomic<int> why{0};
        parallel_for(N, [&](int64_t i, int) {
            for (int f = 0; f < 3; ++f) {
                int a = canon[tri[3 * i + f]], b = canon[tri[3 * i + (f + 1) % 3]];
                int found = -1, ff = -1, count = 0;
                for (int p = v2c_off[a]; p < v2c_off[a + 1]; ++p) {
                    int j = v2c[p];
                    if (j == i) continue;
                    for (int g = 0; g < 3; ++g) {
                        int ga = canon[tri[3 * (size_t)j + g]], gb = canon[tri[3 * (size_t)j + (g + 1) % 3]];
                        if ((ga == a && gb == b) || (ga == b && gb == a)) { found = j; ff = g; ++count; }
                    }
                }
                if (count > 1) { bad = i; why = 1; return; }
                if (count == 1) {
                    fnb[3 * i + f] = found;
                    fnbf[3 * i + f] = ff;
                } else {
                    int va = tri[3 * i + f], vb = tri[3 * i + (f + 1) % 3];
                    double mx = 0.5 * (X(va) + X(vb)), my = 0.5 * (Y(va) + Y(vb));
                    int side = -1;
                    if (std::fabs(mx - d.box[0]) <= tol) side = 0;
                    else if (std::fabs(mx - d.box[1]) <= tol) side = 1;
                    else if (std::fabs(my - d.box[2]) <= tol) side = 2;
                    else if (std::fabs(my - d.box[3]) <= tol) side = 3;
                    if (side < 0) { bad = i; why = 2; return; }
                    if (d.bc[side] == CTENO_PERIODIC) { bad = i; why = 3; return; }
                    const double along = side < 2 ? my : mx;
                    fbc[3 * i + f] = d.split_kind[side] != 0 && along < d.split_at[side] ? d.split_kind[side]
                                                                                         : d.bc[side];
                }
            }
            for (int f = 0; f < 3; ++f)
                for (int g = f + 1; g < 3; ++g)
                    if (fnb[3 * i + f] >= 0 && fnb[3 * i + f] == fnb[3 * i + g]) { bad = i; why = 4; }
        });
        if (bad >= 0) {
            static const char *msg[] = {"", "edge shared by more than two cells", "open edge not on the box boundary",
                                        "unmatched edge on a periodic side", "two faces share a neighbour (mesh too small)"};
            err = std::string(msg[why.load()]) + " at cell " + std::to_string((long long)bad);
            return false;
        }
        return true;
    }

    // per-thread work space of the stencil search, reused from cell to cell
    // (per-cell heap allocations would serialise the threads on the allocator)
    struct StencilScratch {
        std::vector<int32_t> stamp, vstamp, S_, layer, next;
        std::vector<std::pair<double, int>> rest, cand3[3];
    };

    bool stencils() {
        cen.assign((size_t)N * M, -1);
        dir.assign((size_t)N * 3 * Md, -1);
        dirn.assign((size_t)N * 3, 0);
        int nt = nthreads_for(N);
        std::vector<StencilScratch> scratch(nt);
        std::atomic<int64_t> bad{-1};
        parallel_for(N, [&](int64_t ii, int tid) {
            int i = (int)ii;
            StencilScratch &w = scratch[tid];
            auto &st = w.stamp, &vst = w.vstamp;
            if (st.empty()) st.assign(N, -1);
            if (vst.empty()) vst.assign(nvert, -1);
            auto &S_ = w.S_, &layer = w.layer, &next = w.next;
            S_.clear();
            layer.assign(1, i);
            st[i] = i;
            while ((int)S_.size() < M) {
                next.clear();
                for (int c : layer)
                    for (int k = 0; k < 3; ++k) {
                        int v = canon[tri[3 * (size_t)c + k]];
                        // a vertex expanded for an earlier layer has no unvisited cells
                        if (vst[v] == i) continue;
                        vst[v] = i;
                        for (int p = v2c_off[v]; p < v2c_off[v + 1]; ++p) {
                            int j = v2c[p];
                            if (st[j] == i) continue;
                            st[j] = i;
                            next.push_back(j);
                        }
                    }
                if (next.empty()) { bad = i; return; }
                if (S_.size() + next.size() <= (size_t)M) {
                    S_.insert(S_.end(), next.begin(), next.end());
                    layer = next;
                } else {
                    int need = M - (int)S_.size();
                    auto is_face_nb = [&](int j) {
                        bool isf = false;
                        for (int f = 0; f < 3; ++f) isf |= (fnb[3 * (size_t)i + f] == j);
                        return isf;
                    };
                    for (int j : next)
                        if (need > 0 && is_face_nb(j)) { S_.push_back(j); --need; }
                    // the `need` nearest of the others in (d2, id) order, by
                    // insertion into a short sorted list (once it is full, most
                    // candidates fail the first comparison)
                    auto &best = w.rest;
                    best.resize(std::max(need, 1));
                    int nbest = 0;
                    if (need > 0)
                        for (int j : next) {
                            if (is_face_nb(j)) continue;
                            int sx, sy; double dx, dy;
                            offset(i, j, sx, sy, dx, dy);
                            const std::pair<double, int> x{dx * dx + dy * dy, j};
                            if (nbest == need) {
                                if (!(x < best[need - 1])) continue;
                            } else {
                                ++nbest;
                            }
                            int p = nbest - 1;
                            for (; p > 0 && x < best[p - 1]; --p) best[p] = best[p - 1];
                            best[p] = x;
                        }
                    for (int a = 0; a < nbest; ++a) S_.push_back(best[a].second);
                }
            }
            // ascending ids (insertion sort: at most 54 entries)
            for (size_t a = 1; a < S_.size(); ++a) {
                const int32_t x = S_[a];
                size_t b = a;
                for (; b > 0 && S_[b - 1] > x; --b) S_[b] = S_[b - 1];
                S_[b] = x;
            }
            std::copy(S_.begin(), S_.end(), cen.begin() + (size_t)i * M);
            // sectors
            const int32_t *t = tri.data() + 3 * (size_t)i;
            // the members of each sector other than the face neighbours, with
            // their squared offsets
            double px[3], py[3];                      // vertices relative to the centroid
            for (int f = 0; f < 3; ++f) { px[f] = X(t[f]) - cx[i]; py[f] = Y(t[f]) - cy[i]; }
            for (auto &c : w.cand3) c.clear();
            for (int a = 0; a < M; ++a) {
                const int j = S_[a];
                bool isf = false;
                for (int f = 0; f < 3; ++f) isf |= fnb[3 * (size_t)i + f] == j;
                if (isf) continue;                    // each face neighbour leads its own face's stencil
                int sx, sy; double qx, qy;
                offset(i, j, sx, sy, qx, qy);
                for (int f = 0; f < 3; ++f) {
                    const int g = (f + 1) % 3;
                    double c1 = px[f] * qy - py[f] * qx;
                    double c2 = qx * py[g] - qy * px[g];
                    if (c1 >= 0.0 && c2 > 0.0) { w.cand3[f].push_back({qx * qx + qy * qy, j}); break; }
                }
            }
            for (int f = 0; f < 3; ++f) {
                int nbf = fnb[3 * (size_t)i + f];
                if (nbf < 0) continue;
                auto &cand = w.cand3[f];
                const size_t take = std::min(cand.size(), (size_t)(Md - 1));
                std::partial_sort(cand.begin(), cand.begin() + take, cand.end());
                int32_t *out = dir.data() + ((size_t)i * 3 + f) * Md;
                int n = 0;
                out[n++] = nbf;
                for (size_t a = 0; a < cand.size() && n < Md; ++a) out[n++] = cand[a].second;
                if (n >= Kd + 1) dirn[3 * (size_t)i + f] = n;
                else for (int a = 0; a < Md; ++a) out[a] = -1;
            }
        });
        if (bad >= 0) { err = "mesh too small for a stencil at cell " + std::to_string((long long)bad); return false; }
        return true;
    }
};

uint64_t spread16(uint32_t x) {
    uint64_t v = x & 0xFFFF;
    v = (v | (v << 8)) & 0x00FF00FFull;
    v = (v | (v << 4)) & 0x0F0F0F0Full;
    v = (v | (v << 2)) & 0x33333333ull;
    v = (v | (v << 1)) & 0x55555555ull;
    return v;
}

}  // namespace

void set_builder_threads(int n) { tl_max_threads = std::max(1, std::min(n, 16)); }

cteno_status build_host_mesh(const cteno_mesh_desc &d, const cteno_scheme &s, HostMesh &hm, std::string &err) {
    if (d.n_cells <= 0 || d.n_vertices <= 0 || !d.xy || !d.tri) { err = "empty mesh"; return CTENO_ERR_INVALID; }
    if (d.n_cells >= (1 << 28)) { err = "too many cells (limit 2^28)"; return CTENO_ERR_INVALID; }
    bool inflow = false;
    for (int k = 0; k < 4; ++k) {
        if (d.bc[k] < 0 || d.bc[k] > CTENO_INFLOW || d.split_kind[k] < 0 || d.split_kind[k] > CTENO_INFLOW) {
            err = "bad boundary kind";
            return CTENO_ERR_INVALID;
        }
        if (d.split_kind[k] != 0 && d.bc[k] == CTENO_PERIODIC) {
            err = "a periodic side cannot switch kind";
            return CTENO_ERR_INVALID;
        }
        inflow |= d.bc[k] == CTENO_INFLOW || d.split_kind[k] == CTENO_INFLOW;
    }
    if (inflow && s.physics == CTENO_EULER)
        for (const double *b : {d.behind, d.ahead}) {
            const double p = (s.gamma - 1.0) * (b[3] - 0.5 * (b[1] * b[1] + b[2] * b[2]) / b[0]);
            if (!(b[0] > 0.0) || !(p > 0.0)) { err = "non-physical inflow state"; return CTENO_ERR_INVALID; }
        }
    for (double v : {d.behind[0], d.behind[1], d.behind[2], d.behind[3], d.ahead[0], d.ahead[1], d.ahead[2],
                     d.ahead[3], d.line[0], d.line[1], d.line[2]})
        if (inflow && !std::isfinite(v)) { err = "non-finite inflow data"; return CTENO_ERR_INVALID; }
    if ((d.bc[0] == CTENO_PERIODIC) != (d.bc[1] == CTENO_PERIODIC) ||
        (d.bc[2] == CTENO_PERIODIC) != (d.bc[3] == CTENO_PERIODIC)) {
        err = "periodic sides must come in pairs";
        return CTENO_ERR_INVALID;
    }
    if (!(d.box[1] > d.box[0]) || !(d.box[3] > d.box[2])) { err = "bad box"; return CTENO_ERR_INVALID; }
    if (s.physics == CTENO_ADVECTION)
        for (int k = 0; k < 4; ++k)
            if (d.bc[k] == CTENO_WALL || d.split_kind[k] == CTENO_WALL) {
                err = "walls need the Euler equations";
                return CTENO_ERR_INVALID;
            }

    Builder b(d, s.degree);
    if (!b.geometry()) { err = b.err; return CTENO_ERR_MESH; }
    if (!b.weld()) { err = b.err; return CTENO_ERR_MESH; }
    b.vertex_cells();
    if (!b.faces()) { err = b.err; return CTENO_ERR_MESH; }
    if (!b.stencils()) { err = b.err; return CTENO_ERR_STENCIL; }

    const int N = b.N, M = b.M, S = b.S, K = b.K;
    hm.N = N; hm.r = s.degree; hm.K = K; hm.M = M; hm.S = S;
    hm.Kd = b.Kd; hm.Md = b.Md; hm.Nq = dims_Nq(s.degree);
    hm.nv = s.physics == CTENO_EULER ? 4 : 1;
    hm.per_x = b.per_x; hm.per_y = b.per_y; hm.Lx = b.Lx; hm.Ly = b.Ly;

    // internal order
    hm.perm.resize(N);
    std::iota(hm.perm.begin(), hm.perm.end(), 0);
    if (s.reorder) {
        std::vector<uint64_t> key(N);
        double x0 = d.box[0], y0 = d.box[2];
        double sx = 65535.0 / b.Lx, sy = 65535.0 / b.Ly;
        for (int i = 0; i < N; ++i) {
            double fx = std::min(65535.0, std::max(0.0, (b.cx[i] - x0) * sx));
            double fy = std::min(65535.0, std::max(0.0, (b.cy[i] - y0) * sy));
            key[i] = spread16((uint32_t)fx) | (spread16((uint32_t)fy) << 1);
        }
        std::stable_sort(hm.perm.begin(), hm.perm.end(), [&](int a, int c) { return key[a] < key[c]; });
    }
    hm.iperm.resize(N);
    for (int k = 0; k < N; ++k) hm.iperm[hm.perm[k]] = k;

    // the stencils in caller order move to the host mesh (the slot layout
    // below reads them there)
    hm.cen_user = std::move(b.cen);
    hm.dir_user = std::move(b.dir);
    hm.dirn_user = std::move(b.dirn);

    const int64_t Np = pad64(N);
    const int SP = round_up(S, 4);
    // degree >= 4: slot entries carry the slot's directional stencil
    const bool ho = s.degree >= 4, var_groups = ho_var_groups(s.degree);
    static_assert(kMaxS <= 64, "slot tables fit 64 entries");
    hm.SP = SP;
    // every entry of these is written by the layout below (first touch by
    // its threads)
    hm.slot.resize((size_t)Np * SP);
    hm.slot_flag.resize((size_t)Np * S);
    hm.slot_shift.resize((size_t)Np * 2 * S);
    hm.flags.resize(Np);
    hm.verts.resize((size_t)Np * 6);
    hm.fr64.resize((size_t)Np * 12);
    hm.fr32.resize((size_t)Np * 12);
    hm.area.resize(Np);

    auto put_face = [&](int64_t k, int f, double nx, double ny, double len, uint32_t code) {
        hm.fr64[avix(k, 4 * f + 0, 12, 2)] = nx;
        hm.fr64[avix(k, 4 * f + 1, 12, 2)] = ny;
        hm.fr64[avix(k, 4 * f + 2, 12, 2)] = len;
        uint64_t c64 = code;
        std::memcpy(&hm.fr64[avix(k, 4 * f + 3, 12, 2)], &c64, sizeof c64);
        hm.fr32[avix(k, 4 * f + 0, 12, 4)] = (float)nx;
        hm.fr32[avix(k, 4 * f + 1, 12, 4)] = (float)ny;
        hm.fr32[avix(k, 4 * f + 2, 12, 4)] = (float)len;
        std::memcpy(&hm.fr32[avix(k, 4 * f + 3, 12, 4)], &code, sizeof code);
    };

    // rows of the inflow faces, in internal cell order (no table without
    // inflow sides)
    std::vector<int32_t> inflow_row(inflow ? 3 * (size_t)N : 0, -1);
    int64_t n_inflow = 0;
    if (inflow)
        for (int64_t k = 0; k < N; ++k)
            for (int f = 0; f < 3; ++f)
                if (b.fnb[3 * (size_t)hm.perm[k] + f] < 0 && b.fbc[3 * (size_t)hm.perm[k] + f] == CTENO_INFLOW)
                    inflow_row[3 * k + f] = (int32_t)n_inflow++;
    if (n_inflow > (int64_t)kNbInflowMask) { err = "too many inflow faces"; return CTENO_ERR_INVALID; }
    hm.bface.assign(4 * (size_t)n_inflow, 0.0);
    for (int v = 0; v < 4; ++v) { hm.bst[0][v] = d.behind[v]; hm.bst[1][v] = d.ahead[v]; }
    for (int k = 0; k < 3; ++k) hm.bline[k] = d.line[k];

    // per-thread counts (shared atomic counters made the threads contend for
    // one cache line at every face)
    struct alignas(64) Counts { int64_t faces = 0, bnd = 0; int inad = 0, over = 0; };
    std::vector<Counts> cnt(nthreads_for(Np));
    parallel_for(Np, [&](int64_t k, int tid) {
        Counts &c = cnt[tid];
        if (k >= N) {
            // padding cells: self slots, unit area, boundary faces; never written back
            for (int j = 0; j < SP; ++j)
                hm.slot[avix(k, j, SP, 4)] = (int32_t)(k | (ho ? kSlotNoGroup << kSlotGroupShift : 0u));
            for (int j = 0; j < S; ++j) {
                hm.slot_flag[tix(k, j, S)] = 0;
                hm.slot_shift[tix(k, 2 * j, 2 * S)] = 0;
                hm.slot_shift[tix(k, 2 * j + 1, 2 * S)] = 0;
            }
            hm.flags[k] = 0;
            for (int e = 0; e < 6; ++e) hm.verts[tix(k, e, 6)] = 0.0;
            hm.area[k] = 1.0;
            for (int f = 0; f < 3; ++f) put_face(k, f, 1.0, 0.0, 0.0, kNbBoundary | CTENO_TRANSMISSIVE);
            return;
        }
        const int u = hm.perm[k];
        const int32_t *t = b.tri.data() + 3 * (size_t)u;
        for (int v = 0; v < 3; ++v) {
            hm.verts[tix(k, 2 * v, 6)] = b.X(t[v]);
            hm.verts[tix(k, 2 * v + 1, 6)] = b.Y(t[v]);
        }
        hm.area[k] = b.area[u];
        // slots: sector groups first (fixed groups of M_d slots, or at
        // degrees 4 and 5 one member after the other), then the remaining
        // central cells, then pads
        const int32_t *cen = hm.cen_user.data() + (size_t)u * M;
        const int Md = b.Md;
        const int32_t *dr = hm.dir_user.data() + (size_t)u * 3 * Md;
        const int32_t *dn = hm.dirn_user.data() + (size_t)u * 3;
        static_assert(2 * ((kMaxR + 1) * (kMaxR + 2) / 2 - 1) <= 64, "central stencils fit 64 slots");
        int used[64] = {0};
        int32_t sl[64];
        uint8_t fl[64] = {0};
        uint32_t grp[64];   // degree >= 4: the directional stencil of each slot
        std::fill(sl, sl + S, -1);
        std::fill(grp, grp + 64, kSlotNoGroup);
        uint8_t adm = 0;
        int nd = 0;         // variable groups: slots taken by directional members
        for (int f = 0; f < 3; ++f) {
            if (dn[f] > 0) {
                adm |= (uint8_t)(1 << f);
                for (int a = 0; a < dn[f]; ++a) {
                    // (directional stencils are disjoint subsets of the
                    // central one; a cell that neighbours another across two
                    // faces could break that on a tiny periodic mesh)
                    if (var_groups && nd >= S) { c.over++; break; }
                    const int j = var_groups ? nd++ : f * Md + a;
                    sl[j] = dr[f * Md + a];
                    fl[j] = 3;
                    grp[j] = (uint32_t)f;
                    for (int m = 0; m < M; ++m) if (cen[m] == dr[f * Md + a]) used[m] = 1;
                }
            } else if (b.fnb[3 * (size_t)u + f] >= 0) {
                c.inad++;
            }
        }
        int m = 0;
        for (int j = 0; j < S; ++j) {
            if (sl[j] >= 0) continue;
            while (m < M && used[m]) ++m;
            if (m < M) { sl[j] = cen[m]; fl[j] = 1; used[m] = 1; }
        }
        hm.flags[k] = adm;
        for (int j = 0; j < SP; ++j) {
            const int src = j < S ? sl[j] : -1;
            if (src < 0) {   // pad: the cell itself, zero weight
                hm.slot[avix(k, j, SP, 4)] = (int32_t)(k | (ho ? kSlotNoGroup << kSlotGroupShift : 0u));
                if (j < S) {
                    hm.slot_flag[tix(k, j, S)] = 0;
                    hm.slot_shift[tix(k, 2 * j, 2 * S)] = 0;
                    hm.slot_shift[tix(k, 2 * j + 1, 2 * S)] = 0;
                }
                continue;
            }
            int sx, sy; double dx, dy;
            b.offset(u, src, sx, sy, dx, dy);
            hm.slot[avix(k, j, SP, 4)] = (int32_t)((uint32_t)hm.iperm[src] | (ho ? grp[j] << kSlotGroupShift : 0u));
            hm.slot_flag[tix(k, j, S)] = fl[j];
            hm.slot_shift[tix(k, 2 * j, 2 * S)] = (int8_t)sx;
            hm.slot_shift[tix(k, 2 * j + 1, 2 * S)] = (int8_t)sy;
        }
        // faces
        for (int f = 0; f < 3; ++f) {
            int j = b.fnb[3 * (size_t)u + f];
            // outward normal from an edge a -> b of a CCW triangle: (ey, -ex) / |e|
            auto edge_normal = [&](int cell, int face, double &nx, double &ny, double &len) {
                const int32_t *tt = b.tri.data() + 3 * (size_t)cell;
                int va = tt[face], vb = tt[(face + 1) % 3];
                double ex = b.X(vb) - b.X(va), ey = b.Y(vb) - b.Y(va);
                len = std::sqrt(ex * ex + ey * ey);
                nx = ey / len;
                ny = -ex / len;
            };
            double nx, ny, len;
            uint32_t code;
            if (j < 0) {
                edge_normal(u, f, nx, ny, len);
                code = kNbBoundary | (uint32_t)b.fbc[3 * (size_t)u + f];
                const int32_t row = inflow ? inflow_row[3 * k + f] : -1;
                if (row >= 0) {
                    const int32_t *tt = b.tri.data() + 3 * (size_t)u;
                    const int va = tt[f], vb = tt[(f + 1) % 3];
                    double *e = hm.bface.data() + 4 * (size_t)row;
                    e[0] = b.X(va);
                    e[1] = b.Y(va);
                    e[2] = b.X(vb) - b.X(va);
                    e[3] = b.Y(vb) - b.Y(va);
                    code |= (uint32_t)row << 2;
                }
                c.bnd++;
                c.faces++;
            } else {
                int kj = hm.iperm[j];
                int g = b.fnbf[3 * (size_t)u + f];
                bool owner = k < kj;
                // the face's normal and length come from the owner's edge;
                // the other cell stores the exact negation
                if (owner) edge_normal(u, f, nx, ny, len);
                else { edge_normal(j, g, nx, ny, len); nx = -nx; ny = -ny; }
                code = (uint32_t)kj | ((uint32_t)g << 28) | (owner ? kNbOwner : 0u);
                if (owner) c.faces++;
            }
            put_face(k, f, nx, ny, len, code);
        }
    });
    int64_t nfaces = 0, nbnd = 0;
    int ninad = 0, overfull = 0;
    for (const Counts &c : cnt) { nfaces += c.faces; nbnd += c.bnd; ninad += c.inad; overfull += c.over; }
    hm.n_faces = nfaces;
    hm.n_boundary = nbnd;
    if (overfull) { err = "directional stencils overlap (mesh too small)"; return CTENO_ERR_INVALID; }
    hm.n_inadmissible = ninad;
    return CTENO_OK;
}

// ---------------------------------------------------------------------------
// reference-triangle tables
// ---------------------------------------------------------------------------
namespace {
double fct(int n) { double f = 1; for (int k = 2; k <= n; ++k) f *= k; return f; }
// integral of xi^a eta^b over the reference triangle
double ref_int(int a, int b) { return fct(a) * fct(b) / fct(a + b + 2); }
// n-point Gauss-Legendre rule on [0, 1], points ascending: Newton iteration
// on P_n from the three-term recurrence, weights 2 / ((1 - z^2) P_n'(z)^2)
// on [-1, 1], halved
void gauss_legendre01(int n, double *t, double *w) {
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        {   // derivative at the converged root
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        // z runs from near +1 downwards: t = (1 - z) / 2 ascends
        t[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}
}  // namespace

void make_ref_tables(int r, RefTables &t) {
    std::memset(&t, 0, sizeof t);
    t.K = dims_K(r);
    int k = 0;
    for (int deg = 1; deg <= r; ++deg)
        for (int a = deg; a >= 0; --a) { t.ex[k][0] = a; t.ex[k][1] = deg - a; ++k; }
    for (int q = 0; q < t.K; ++q) t.mean[q] = 2.0 * ref_int(t.ex[q][0], t.ex[q][1]);
    // Gram matrix of the smoothness indicator: sum over multi-indices alpha,
    // 1 <= |alpha| <= r, of int D^alpha psi_k D^alpha psi_l
    for (int p = 0; p < t.K; ++p)
        for (int q = 0; q < t.K; ++q) {
            double g = 0;
            for (int o = 1; o <= r; ++o)
                for (int ax = o; ax >= 0; --ax) {
                    int ay = o - ax;
                    int a1 = t.ex[p][0], b1 = t.ex[p][1], a2 = t.ex[q][0], b2 = t.ex[q][1];
                    if (a1 < ax || b1 < ay || a2 < ax || b2 < ay) continue;
                    double c1 = fct(a1) / fct(a1 - ax) * fct(b1) / fct(b1 - ay);
                    double c2 = fct(a2) / fct(a2 - ax) * fct(b2) / fct(b2 - ay);
                    g += c1 * c2 * ref_int(a1 - ax + a2 - ax, b1 - ay + b2 - ay);
                }
            t.gram[p][q] = g;
        }
    // N_q-point Gauss-Legendre on [0,1]; reference images of the face points
    t.Nq = dims_Nq(r);
    gauss_legendre01(t.Nq, t.gq, t.gw);
    const double *tq = t.gq;
    for (int f = 0; f < 3; ++f)
        for (int q = 0; q < t.Nq; ++q) {
            double xi, eta;
            if (f == 0) { xi = tq[q]; eta = 0.0; }
            else if (f == 1) { xi = 1.0 - tq[q]; eta = tq[q]; }
            else { xi = 0.0; eta = 1.0 - tq[q]; }
            for (int p = 0; p < t.K; ++p)
                t.basis[f][q][p] = std::pow(xi, t.ex[p][0]) * std::pow(eta, t.ex[p][1]) - t.mean[p];
        }
}

}  // namespace cteno
