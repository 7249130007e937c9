/*
 * cteno_oracle.c -- plain, slow, FP64 CPU oracle of the CTENO / CTENOZ
 * finite-volume hot path on unstructured triangles (Ma, Chong, Feng, Zhang,
 * Wang, Zhou, "High-order finite-volume central targeted ENO family scheme
 * for compressible flows in unstructured meshes", arXiv 2312.17042).
 *
 * TEST INFRASTRUCTURE.  This file is used only by the test-suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark.  It shares no
 * code, header, table or constant generator with the GPU library, and the
 * GPU library never calls it.
 *
 * Everything is double precision, plain loops, no fast-math and no FMA
 * contraction (built with -O2 -ffp-contract=off).  Per-cell and per-face
 * loops are independent, so the optional OpenMP loops give bit-identical
 * results for any thread count.
 *
 * What is computed, in the paper's order (section 2):
 *   - the semi-discrete finite-volume form (eq. e1 and the equation after it):
 *     dU_i/dt = -(1/|V_i|) sum_faces sum_q F(U_L, U_R; n) w_q |A|;
 *   - reconstruction (sec. 2.1): affine map of the target cell to the
 *     reference triangle, zero-mean monomial basis phi_k = psi_k - mean(psi_k)
 *     over the reference cell, mean-constrained least squares A a = b with
 *     A_mk = int_{V'_m} phi_k, b_m = |V'_m| (U_m - U_0), solved by
 *     Householder QR (eq. after "QR decomposition ... Householder");
 *   - CWENO decomposition p_opt = sum lambda_s p_s, p_1 = (p_opt - sum
 *     lambda_s p_s)/lambda_1 and lambda_1 = 1 - 1/lambda1', lambda_s =
 *     (1-lambda_1)/(s_t-1) (eqs. e16, e17, e18);
 *   - smoothness indicators SI_s = sum_{q=1..r} int_{V'_0} (D^q p_s)^2 (sec. 2.2);
 *   - CTENO weights (Algorithm 1) and CTENOZ weights (Algorithm 2) with the
 *     cut-off delta_s = [chi_s >= C_T] (eq. e23) and the two-branch final
 *     polynomial (sec. 2.5, 2.6);
 *   - the comparison schemes of sec. 2.3-2.4: CWENO (nonlinear weights
 *     lambda_s / (eps + SI_s)^b with b = 4 and the linear weights of eq.
 *     e18, final polynomial sum_s omega_s p_s with p_1 from eq. e17) and
 *     TENO (the cut-off of eq. e22-e23 with gamma_s = 1/(SI_s + eps)^6 on
 *     the central-stencil polynomial itself, then the same two branches);
 *   - HLLC flux with Roe-averaged wave-speed estimates (sec. 2.7);
 *   - third-order explicit Runge-Kutta in time (sec. 2, Shu-Osher SSP form).
 *
 * Readings where the paper is silent or ambiguous (all shared with the GPU
 * library only as written specification, never as code):
 *   K = (r+1)(r+2)/2 - 1 non-constant basis functions, M = 2K neighbours;
 *   central stencil = vertex-neighbour layers taken whole while they fit,
 *     last layer filled face-neighbours-first then by (squared centroid
 *     distance, cell id);
 *   directional stencils = one per face: the central-stencil cells whose
 *     centroid lies in the cone from the target centroid through that
 *     face's two vertices (face neighbour always assigned to its face),
 *     nearest M_d = 2 K_d of them with the face neighbour first; admissible
 *     when the face is interior and the stencil has >= K_d + 1 cells;
 *     directional degree r_d = 1 for r <= 3 and r_d = ceil(r/2) above
 *     (third-order directional stencils for the fifth-order scheme, Fig. 1);
 *   reference map anchored at the first vertex of the counter-clockwise
 *     normalised triangle; SI multi-indices counted once each;
 *   final polynomial p_1 when delta_1 = 1 (Algorithms 1 and 2); TENO's p_1
 *     is the central-stencil least-squares polynomial (p_opt), CTENO's the
 *     decomposed one of eq. e17;
 *   eps = 1e-12 by default; N_q = ceil((r+1)/2) Gauss-Legendre points;
 *   CTENOZ's gamma_s: literally 1 + tau / (SI_s + eps) by default; as an
 *     option (gamma_form SCALED) 1 + tau / (SI_s + eps)^6, the sixth power
 *     that Algorithm 1's gamma_s carries, which makes the selection
 *     independent of the scale of the indicators (the printed form is not:
 *     tau grows like SI^6, the denominator like SI);
 *   non-physical face states (density or pressure <= 0) are reported as an
 *     error, as the paper has no positivity treatment; an optional fallback
 *     (positivity = 1, not in the paper) replaces all Gauss-point values of
 *     such a cell by its cell average and flags the cell with bit 7.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXR 6
#define OR_MAXK 27
#define OR_MAXM 54
#define OR_MAXNQ 4
#define OR_MAXNV 4

enum { OR_PERIODIC = 0, OR_WALL = 1, OR_TRANSMISSIVE = 2, OR_INFLOW = 3 };
enum { OR_ADVECTION = 0, OR_EULER = 1 };
enum { OR_CTENO = 0, OR_CTENOZ = 1, OR_CWENO = 2, OR_TENO = 3 };
enum { OR_GAMMA_PAPER = 0, OR_GAMMA_LAMBDA = 1, OR_GAMMA_SCALED = 2 };
enum { OR_VARS_CONSERVED = 0, OR_VARS_CHARACTERISTIC = 1 };

static char or_err[512];
static void set_err(const char *m, long a) { snprintf(or_err, sizeof or_err, "%s (%ld)", m, a); }
const char *or_last_error(void) { return or_err; }

/* per-cell precomputed least-squares data (built on first use) */
typedef struct {
    int cen[OR_MAXM];            /* central stencil cell ids */
    signed char csx[OR_MAXM], csy[OR_MAXM];
    int dir[3][OR_MAXM];         /* directional stencil cell ids */
    signed char dsx[3][OR_MAXM], dsy[3][OR_MAXM];
    int dirn[3];                 /* members (0 = inadmissible) */
    /* Householder factors of the central system: A (M x K, column-major),
       v0[j], beta[j], rdiag[j] */
    double qa[OR_MAXM * OR_MAXK], qv0[OR_MAXK], qb[OR_MAXK], qr[OR_MAXK];
    double wc[OR_MAXM];
    double da[3][OR_MAXM * OR_MAXK], dv0[3][OR_MAXK], db[3][OR_MAXK], dr[3][OR_MAXK];
    double wd[3][OR_MAXM];
    int status;                  /* 0 ok, else error code */
} or_cell;

typedef struct {
    int nvert, N;
    double *xy;        /* raw vertex coordinates */
    int *tri;          /* CCW-normalised, raw vertex ids */
    int *canon;        /* canonical vertex id after periodic welding */
    double box[4];
    int bc[4];
    /* prescribed outside states of inflow faces: bs[0] where
       x < bline[0] + bline[1] y + bline[2] t, else bs[1]; a side k may switch
       to kind split_kind[k] (0 = no switch) below split_at[k] */
    double bs[2][OR_MAXNV], bline[3];
    int split_kind[4];
    double split_at[4];
    int per_x, per_y;
    double Lx, Ly;
    int physics, nv;
    double ax, ay, gam;
    int scheme, r, K, M, rd, Kd, Md, Nq, gamma_form, vars;
    int positivity;              /* 1: cell-average fallback for non-physical face states */
    long long n_fallback;        /* cell reconstructions that took the fallback */
    double lam1p, ct, eps;
    int ex[OR_MAXK + 1][2];      /* exponents of psi_k, k = 1..K */
    double gq[OR_MAXNQ], gw[OR_MAXNQ];
    double *cx, *cy, *area;
    int *fnb, *fnbf, *fbc;       /* [3N] */
    double *fnx, *fny, *flen;    /* [3N] */
    int *v2c_off, *v2c;          /* canonical vertex -> cells */
    or_cell **cells;
    int nthreads;
    int **stamp;                 /* per-thread visit stamps */
} or_ctx;

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */
static double fact(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; }

/* integral over the reference triangle {xi,eta >= 0, xi+eta <= 1} of xi^a eta^b */
static double ref_mono(int a, int b) { return fact(a) * fact(b) / fact(a + b + 2); }

static int find_root(int *p, int a) { while (p[a] != a) { p[a] = p[p[a]]; a = p[a]; } return a; }
static void unite(int *p, int a, int b) {
    a = find_root(p, a); b = find_root(p, b);
    if (a == b) return;
    if (a < b) p[b] = a; else p[a] = b;
}

typedef struct { double key; int id; } dkey;
static int cmp_dkey(const void *x, const void *y) {
    const dkey *a = x, *b = y;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->id > b->id) - (a->id < b->id);
}

typedef struct { int a, b, cell, face; } edge_rec;
static int cmp_edge(const void *x, const void *y) {
    const edge_rec *p = x, *q = y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    if (p->cell != q->cell) return p->cell < q->cell ? -1 : 1;
    return p->face - q->face;
}

/* nearest periodic image of the centroid of j seen from the centroid of i:
   returns the integer shifts and the shifted difference vector */
static void image(const or_ctx *c, int i, int j, int *sx, int *sy, double *dx, double *dy) {
    double x = c->cx[j] - c->cx[i], y = c->cy[j] - c->cy[i];
    *sx = 0; *sy = 0;
    if (c->per_x) {
        if (x > 0.5 * c->Lx) { x = x - c->Lx; *sx = -1; }
        else if (x < -0.5 * c->Lx) { x = x + c->Lx; *sx = 1; }
    }
    if (c->per_y) {
        if (y > 0.5 * c->Ly) { y = y - c->Ly; *sy = -1; }
        else if (y < -0.5 * c->Ly) { y = y + c->Ly; *sy = 1; }
    }
    *dx = x; *dy = y;
}

/* ------------------------------------------------------------------ */
/* mesh set-up: welding, geometry, faces                               */
/* ------------------------------------------------------------------ */
typedef struct { double key; int v; } vkey;
static int cmp_vkey(const void *x, const void *y) {
    const vkey *a = x, *b = y;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return a->v - b->v;
}

static int weld(or_ctx *c, int dirn /* 0: x seam, 1: y seam */) {
    double lo = dirn == 0 ? c->box[0] : c->box[2];
    double hi = dirn == 0 ? c->box[1] : c->box[3];
    double L = hi - lo;
    double tol = 1e-9 * (fabs(c->box[1] - c->box[0]) + fabs(c->box[3] - c->box[2]));
    int n = c->nvert;
    vkey *A = malloc(sizeof(vkey) * n), *B = malloc(sizeof(vkey) * n);
    int na = 0, nb = 0;
    for (int v = 0; v < n; ++v) {
        double s = c->xy[2 * v + dirn], o = c->xy[2 * v + 1 - dirn];
        if (fabs(s - lo) <= tol) { A[na].key = o; A[na].v = v; ++na; }
        if (fabs(s - hi) <= tol) { B[nb].key = o; B[nb].v = v; ++nb; }
    }
    (void)L;
    int ok = (na == nb);
    if (ok) {
        qsort(A, na, sizeof(vkey), cmp_vkey);
        qsort(B, nb, sizeof(vkey), cmp_vkey);
        for (int k = 0; k < na; ++k) {
            if (fabs(A[k].key - B[k].key) > tol) { ok = 0; break; }
            unite(c->canon, A[k].v, B[k].v);
        }
    }
    free(A); free(B);
    return ok;
}

static int build_mesh(or_ctx *c) {
    int N = c->N;
    /* counter-clockwise normalisation: swap the 2nd and 3rd vertex when the
       signed area is negative; the first vertex stays first */
    c->cx = malloc(sizeof(double) * N);
    c->cy = malloc(sizeof(double) * N);
    c->area = malloc(sizeof(double) * N);
    for (int i = 0; i < N; ++i) {
        int *t = c->tri + 3 * i;
        double x0 = c->xy[2 * t[0]], y0 = c->xy[2 * t[0] + 1];
        double x1 = c->xy[2 * t[1]], y1 = c->xy[2 * t[1] + 1];
        double x2 = c->xy[2 * t[2]], y2 = c->xy[2 * t[2] + 1];
        double s = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
        if (!(s != 0.0)) { set_err("degenerate triangle", i); return 0; }
        if (s < 0) {
            int tmp = t[1]; t[1] = t[2]; t[2] = tmp;
            s = -s;
        }
        c->area[i] = 0.5 * s;
    }
    /* centroids from the stored (input) vertex order: ((xa + xb) + xc) / 3.
       The CCW swap above keeps the set; recompute from the swapped order
       would change the bits, so the input order is kept in a copy. */
    /* (input order is restored by the caller through or_tri_input) */
    /* periodic welding */
    c->canon = malloc(sizeof(int) * c->nvert);
    for (int v = 0; v < c->nvert; ++v) c->canon[v] = v;
    if (c->per_x && !weld(c, 0)) { set_err("periodic x seam vertices do not match", 0); return 0; }
    if (c->per_y && !weld(c, 1)) { set_err("periodic y seam vertices do not match", 0); return 0; }
    for (int v = 0; v < c->nvert; ++v) c->canon[v] = find_root(c->canon, v);

    /* outward normals and lengths, edge f runs from vertex f to vertex f+1 */
    c->fnx = malloc(sizeof(double) * 3 * N);
    c->fny = malloc(sizeof(double) * 3 * N);
    c->flen = malloc(sizeof(double) * 3 * N);
    for (int i = 0; i < N; ++i) {
        for (int f = 0; f < 3; ++f) {
            int a = c->tri[3 * i + f], b = c->tri[3 * i + (f + 1) % 3];
            double ex = c->xy[2 * b] - c->xy[2 * a], ey = c->xy[2 * b + 1] - c->xy[2 * a + 1];
            double len = sqrt(ex * ex + ey * ey);
            c->flen[3 * i + f] = len;
            c->fnx[3 * i + f] = ey / len;
            c->fny[3 * i + f] = -ex / len;
        }
    }
    /* faces: match edges by their canonical vertex pair */
    edge_rec *E = malloc(sizeof(edge_rec) * 3 * (size_t)N);
    for (int i = 0; i < N; ++i)
        for (int f = 0; f < 3; ++f) {
            int a = c->canon[c->tri[3 * i + f]], b = c->canon[c->tri[3 * i + (f + 1) % 3]];
            edge_rec *e = E + 3 * i + f;
            e->a = a < b ? a : b; e->b = a < b ? b : a; e->cell = i; e->face = f;
        }
    qsort(E, 3 * (size_t)N, sizeof(edge_rec), cmp_edge);
    c->fnb = malloc(sizeof(int) * 3 * N);
    c->fnbf = malloc(sizeof(int) * 3 * N);
    c->fbc = malloc(sizeof(int) * 3 * N);
    double tol = 1e-9 * (fabs(c->box[1] - c->box[0]) + fabs(c->box[3] - c->box[2]));
    for (size_t k = 0; k < 3 * (size_t)N;) {
        size_t m = k + 1;
        while (m < 3 * (size_t)N && E[m].a == E[k].a && E[m].b == E[k].b) ++m;
        if (m - k == 2) {
            int i = E[k].cell, j = E[k + 1].cell;
            if (i == j) { set_err("cell is its own face neighbour (mesh too small)", i); free(E); return 0; }
            c->fnb[3 * i + E[k].face] = j; c->fnbf[3 * i + E[k].face] = E[k + 1].face; c->fbc[3 * i + E[k].face] = -1;
            c->fnb[3 * j + E[k + 1].face] = i; c->fnbf[3 * j + E[k + 1].face] = E[k].face; c->fbc[3 * j + E[k + 1].face] = -1;
        } else if (m - k == 1) {
            int i = E[k].cell, f = E[k].face;
            int a = c->tri[3 * i + f], b = c->tri[3 * i + (f + 1) % 3];
            double mx = 0.5 * (c->xy[2 * a] + c->xy[2 * b]), my = 0.5 * (c->xy[2 * a + 1] + c->xy[2 * b + 1]);
            int side = -1;
            if (fabs(mx - c->box[0]) <= tol) side = 0;
            else if (fabs(mx - c->box[1]) <= tol) side = 1;
            else if (fabs(my - c->box[2]) <= tol) side = 2;
            else if (fabs(my - c->box[3]) <= tol) side = 3;
            if (side < 0) { set_err("open edge not on the box boundary", i); free(E); return 0; }
            if (c->bc[side] == OR_PERIODIC) { set_err("unmatched edge on a periodic side", i); free(E); return 0; }
            int kind = c->bc[side];
            /* coordinate along the side: y on the sides x = const, x on the others */
            double along = side < 2 ? my : mx;
            if (c->split_kind[side] != 0 && along < c->split_at[side]) kind = c->split_kind[side];
            c->fnb[3 * i + f] = -1; c->fnbf[3 * i + f] = -1; c->fbc[3 * i + f] = kind;
        } else {
            set_err("edge shared by more than two cells", E[k].cell); free(E); return 0;
        }
        k = m;
    }
    free(E);
    for (int i = 0; i < N; ++i)
        for (int f = 0; f < 3; ++f)
            for (int g = f + 1; g < 3; ++g)
                if (c->fnb[3 * i + f] >= 0 && c->fnb[3 * i + f] == c->fnb[3 * i + g]) {
                    set_err("two faces share a neighbour (mesh too small)", i); return 0;
                }
    /* canonical vertex -> cell lists */
    c->v2c_off = calloc((size_t)c->nvert + 1, sizeof(int));
    for (int i = 0; i < N; ++i)
        for (int f = 0; f < 3; ++f) c->v2c_off[c->canon[c->tri[3 * i + f]] + 1]++;
    for (int v = 0; v < c->nvert; ++v) c->v2c_off[v + 1] += c->v2c_off[v];
    c->v2c = malloc(sizeof(int) * 3 * (size_t)N);
    int *fill = calloc((size_t)c->nvert, sizeof(int));
    for (int i = 0; i < N; ++i)
        for (int f = 0; f < 3; ++f) {
            int v = c->canon[c->tri[3 * i + f]];
            c->v2c[c->v2c_off[v] + fill[v]++] = i;
        }
    free(fill);
    return 1;
}

/* ------------------------------------------------------------------ */
/* Householder QR least squares (Golub & Van Loan), column-major A     */
/* ------------------------------------------------------------------ */
static int hh_factor(double *A, int m, int n, double *v0, double *beta, double *rdiag) {
    for (int j = 0; j < n; ++j) {
        double *col = A + (size_t)j * m;
        double nrm = 0.0;
        for (int i = j; i < m; ++i) nrm += col[i] * col[i];
        nrm = sqrt(nrm);
        if (nrm == 0.0) return 0;
        double alpha = col[j] > 0 ? -nrm : nrm;
        double vj = col[j] - alpha;            /* v = x - alpha e1 */
        double vv = vj * vj;
        for (int i = j + 1; i < m; ++i) vv += col[i] * col[i];
        double bt = vv > 0 ? 2.0 / vv : 0.0;
        v0[j] = vj; beta[j] = bt; rdiag[j] = alpha;
        for (int k = j + 1; k < n; ++k) {
            double *ck = A + (size_t)k * m;
            double s = vj * ck[j];
            for (int i = j + 1; i < m; ++i) s += col[i] * ck[i];
            s *= bt;
            ck[j] -= s * vj;
            for (int i = j + 1; i < m; ++i) ck[i] -= s * col[i];
        }
    }
    /* reject numerically rank-deficient systems */
    double mx = 0.0;
    for (int j = 0; j < n; ++j) if (fabs(rdiag[j]) > mx) mx = fabs(rdiag[j]);
    for (int j = 0; j < n; ++j) if (fabs(rdiag[j]) <= 1e-12 * mx) return 0;
    return 1;
}

/* x (n) = argmin |A x - b|; b (m) is overwritten */
static void hh_solve(const double *A, int m, int n, const double *v0, const double *beta,
                     const double *rdiag, double *b, double *x) {
    for (int j = 0; j < n; ++j) {
        const double *col = A + (size_t)j * m;
        double s = v0[j] * b[j];
        for (int i = j + 1; i < m; ++i) s += col[i] * b[i];
        s *= beta[j];
        b[j] -= s * v0[j];
        for (int i = j + 1; i < m; ++i) b[i] -= s * col[i];
    }
    for (int j = n - 1; j >= 0; --j) {
        double s = b[j];
        for (int k = j + 1; k < n; ++k) s -= A[(size_t)k * m + j] * x[k];
        x[j] = s / rdiag[j];
    }
}

/* ------------------------------------------------------------------ */
/* reference-space moments                                             */
/* ------------------------------------------------------------------ */
/* integral over the triangle with vertices (X[t], Y[t]) of xi^a eta^b, from
   int_T l0^p l1^q l2^s = 2|T| p! q! s! / (p+q+s+2)!  with xi, eta linear in
   the barycentric coordinates l0, l1, l2 */
static double tri_moment(const double X[3], const double Y[3], double area, int a, int b) {
    double tot = 0.0;
    for (int i0 = 0; i0 <= a; ++i0)
        for (int i1 = 0; i0 + i1 <= a; ++i1) {
            int i2 = a - i0 - i1;
            double ca = fact(a) / (fact(i0) * fact(i1) * fact(i2)) * pow(X[0], i0) * pow(X[1], i1) * pow(X[2], i2);
            for (int k0 = 0; k0 <= b; ++k0)
                for (int k1 = 0; k0 + k1 <= b; ++k1) {
                    int k2 = b - k0 - k1;
                    double cb = fact(b) / (fact(k0) * fact(k1) * fact(k2)) * pow(Y[0], k0) * pow(Y[1], k1) * pow(Y[2], k2);
                    tot += ca * cb * 2.0 * area * fact(i0 + k0) * fact(i1 + k1) * fact(i2 + k2) / fact(a + b + 2);
                }
        }
    return tot;
}

/* physical -> reference coordinates of cell i */
static void to_ref(const or_ctx *c, int i, double x, double y, double *xi, double *eta) {
    const int *t = c->tri + 3 * i;
    double x0 = c->xy[2 * t[0]], y0 = c->xy[2 * t[0] + 1];
    double a = c->xy[2 * t[1]] - x0, b = c->xy[2 * t[2]] - x0;
    double cc = c->xy[2 * t[1] + 1] - y0, d = c->xy[2 * t[2] + 1] - y0;
    double det = a * d - b * cc;
    double px = x - x0, py = y - y0;
    *xi = (d * px - b * py) / det;
    *eta = (-cc * px + a * py) / det;
}

/* mapped vertices and |V'| of cell m (shifted by the periodic image) in the
   reference frame of cell i */
static double mapped_tri(const or_ctx *c, int i, int m, int sx, int sy, double X[3], double Y[3]) {
    for (int k = 0; k < 3; ++k) {
        int v = c->tri[3 * m + k];
        double x = c->xy[2 * v] + sx * c->Lx, y = c->xy[2 * v + 1] + sy * c->Ly;
        to_ref(c, i, x, y, &X[k], &Y[k]);
    }
    return 0.5 * fabs((X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]));
}

/* least-squares matrix rows for a stencil: A_mk = int psi_k - |V'_m| mean(psi_k) */
static int build_ls(const or_ctx *c, int i, int n, const int *ids, const signed char *sx, const signed char *sy,
                    int K, double *A, double *w) {
    for (int m = 0; m < n; ++m) {
        double X[3], Y[3];
        double ar = mapped_tri(c, i, ids[m], sx[m], sy[m], X, Y);
        w[m] = ar;
        for (int k = 1; k <= K; ++k) {
            int a = c->ex[k][0], b = c->ex[k][1];
            double mean = 2.0 * ref_mono(a, b);
            A[(size_t)(k - 1) * n + m] = tri_moment(X, Y, ar, a, b) - ar * mean;
        }
    }
    return 1;
}

/* ------------------------------------------------------------------ */
/* stencils                                                            */
/* ------------------------------------------------------------------ */
static int thread_id(void) {
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

static int build_cell(or_ctx *c, int i, or_cell *pc) {
    int M = c->M, N = c->N;
    int tid = thread_id();
    if (!c->stamp[tid]) {
        c->stamp[tid] = malloc(sizeof(int) * N);
        for (int k = 0; k < N; ++k) c->stamp[tid][k] = -1;
    }
    int *st = c->stamp[tid];
    int S[OR_MAXM]; int nS = 0;
    int front[4096], nf = 1, next[4096];
    front[0] = i; st[i] = i;
    while (nS < M) {
        int nn = 0;
        for (int a = 0; a < nf; ++a) {
            int cell = front[a];
            for (int f = 0; f < 3; ++f) {
                int v = c->canon[c->tri[3 * cell + f]];
                for (int p = c->v2c_off[v]; p < c->v2c_off[v + 1]; ++p) {
                    int j = c->v2c[p];
                    if (st[j] == i) continue;
                    st[j] = i;
                    if (nn >= 4096) return 2;
                    next[nn++] = j;
                }
            }
        }
        if (nn == 0) return 3;      /* mesh exhausted before M cells */
        if (nS + nn <= M) {
            /* the whole layer fits: take it and grow the next layer from it */
            for (int a = 0; a < nn; ++a) { S[nS++] = next[a]; front[a] = next[a]; }
            nf = nn;
        } else {
            /* the last layer: face neighbours first, then by (distance, id) */
            int need = M - nS;
            for (int a = 0; a < nn && need > 0; ++a)
                for (int f = 0; f < 3; ++f)
                    if (next[a] == c->fnb[3 * i + f]) { S[nS++] = next[a]; next[a] = -1; --need; break; }
            dkey dk[4096];
            int nd = 0;
            for (int a = 0; a < nn; ++a) {
                if (next[a] < 0) continue;
                int sx, sy; double dx, dy;
                image(c, i, next[a], &sx, &sy, &dx, &dy);
                dk[nd].key = dx * dx + dy * dy; dk[nd].id = next[a]; ++nd;
            }
            qsort(dk, nd, sizeof(dkey), cmp_dkey);
            for (int a = 0; a < need; ++a) S[nS++] = dk[a].id;
        }
    }
    /* sort the central list by id for a canonical order */
    for (int a = 1; a < nS; ++a) { int v = S[a], b = a - 1; while (b >= 0 && S[b] > v) { S[b + 1] = S[b]; --b; } S[b + 1] = v; }
    for (int a = 0; a < M; ++a) {
        int sx, sy; double dx, dy;
        image(c, i, S[a], &sx, &sy, &dx, &dy);
        pc->cen[a] = S[a]; pc->csx[a] = (signed char)sx; pc->csy[a] = (signed char)sy;
    }
    /* directional stencils: cone of face f from the centroid through vertices f, f+1 */
    const int *t = c->tri + 3 * i;
    int sector[OR_MAXM];
    for (int a = 0; a < M; ++a) {
        int j = S[a], s = -1;
        for (int f = 0; f < 3; ++f) if (c->fnb[3 * i + f] == j) s = f;
        if (s < 0) {
            int sx, sy; double qx, qy;
            image(c, i, j, &sx, &sy, &qx, &qy);
            for (int f = 0; f < 3; ++f) {
                double ux = c->xy[2 * t[f]] - c->cx[i], uy = c->xy[2 * t[f] + 1] - c->cy[i];
                int g = (f + 1) % 3;
                double wx = c->xy[2 * t[g]] - c->cx[i], wy = c->xy[2 * t[g] + 1] - c->cy[i];
                double c1 = ux * qy - uy * qx;      /* cross(u, q) */
                double c2 = qx * wy - qy * wx;      /* cross(q, w) */
                if (c1 >= 0.0 && c2 > 0.0) { s = f; break; }
            }
        }
        sector[a] = s;   /* -1 cannot happen for a point away from the centroid */
    }
    for (int f = 0; f < 3; ++f) {
        pc->dirn[f] = 0;
        int nbf = c->fnb[3 * i + f];
        if (nbf < 0) continue;
        dkey dk[OR_MAXM]; int nd = 0;
        for (int a = 0; a < M; ++a) {
            if (sector[a] != f || S[a] == nbf) continue;
            int sx, sy; double dx, dy;
            image(c, i, S[a], &sx, &sy, &dx, &dy);
            dk[nd].key = dx * dx + dy * dy; dk[nd].id = S[a]; ++nd;
        }
        qsort(dk, nd, sizeof(dkey), cmp_dkey);
        int n = 0;
        pc->dir[f][n++] = nbf;
        for (int a = 0; a < nd && n < c->Md; ++a) pc->dir[f][n++] = dk[a].id;
        if (n >= c->Kd + 1) pc->dirn[f] = n;
        for (int a = 0; a < n; ++a) {
            int sx, sy; double dx, dy;
            image(c, i, pc->dir[f][a], &sx, &sy, &dx, &dy);
            pc->dsx[f][a] = (signed char)sx; pc->dsy[f][a] = (signed char)sy;
        }
    }
    /* least-squares factors */
    build_ls(c, i, M, pc->cen, pc->csx, pc->csy, c->K, pc->qa, pc->wc);
    if (!hh_factor(pc->qa, M, c->K, pc->qv0, pc->qb, pc->qr)) return 4;
    for (int f = 0; f < 3; ++f) {
        if (!pc->dirn[f]) continue;
        build_ls(c, i, pc->dirn[f], pc->dir[f], pc->dsx[f], pc->dsy[f], c->Kd, pc->da[f], pc->wd[f]);
        if (!hh_factor(pc->da[f], pc->dirn[f], c->Kd, pc->dv0[f], pc->db[f], pc->dr[f])) pc->dirn[f] = 0;
    }
    return 0;
}

static or_cell *get_cell(or_ctx *c, int i) {
    if (!c->cells[i]) {
        or_cell *pc = calloc(1, sizeof(or_cell));
        pc->status = build_cell(c, i, pc);
        c->cells[i] = pc;
    }
    return c->cells[i];
}

/* ------------------------------------------------------------------ */
/* polynomial algebra for smoothness indicators (coefficient grids)    */
/* ------------------------------------------------------------------ */
#define PG (2 * OR_MAXR + 1)
/* smoothness indicator of p = sum_k a_k phi_k (constants drop out): every
   multi-index alpha with 1 <= |alpha| <= r once, each derivative squared
   and integrated exactly over the reference triangle */
static double smoothness(const or_ctx *c, const double *a, int K, int r) {
    double P[PG][PG];
    memset(P, 0, sizeof P);
    for (int k = 1; k <= K; ++k) P[c->ex[k][0]][c->ex[k][1]] += a[k - 1];
    double si = 0.0;
    for (int q = 1; q <= r; ++q)
        for (int ax = q; ax >= 0; --ax) {
            int ay = q - ax;
            /* D = d^ax/dxi^ax d^ay/deta^ay p, a polynomial of degree <= r - q */
            double D[PG][PG];
            memset(D, 0, sizeof D);
            for (int i = ax; i <= r; ++i)
                for (int j = ay; i + j <= r; ++j) {
                    double f = 1.0;
                    for (int s = 0; s < ax; ++s) f *= (i - s);
                    for (int s = 0; s < ay; ++s) f *= (j - s);
                    D[i - ax][j - ay] += f * P[i][j];
                }
            /* int_{T_ref} D^2 term by term */
            int dq = r - q;
            for (int i1 = 0; i1 <= dq; ++i1)
                for (int j1 = 0; i1 + j1 <= dq; ++j1)
                    for (int i2 = 0; i2 <= dq; ++i2)
                        for (int j2 = 0; i2 + j2 <= dq; ++j2)
                            si += D[i1][j1] * D[i2][j2] * ref_mono(i1 + i2, j1 + j2);
        }
    return si;
}

/* ------------------------------------------------------------------ */
/* reconstruction of one cell                                          */
/* ------------------------------------------------------------------ */
static double pow6(double x) { double x2 = x * x; return x2 * x2 * x2; }

/* TENO-type selection (Algorithm 1 = CTENO, Algorithm 2 = CTENOZ) for one
   variable.  si[0] is the central (p_1) indicator, si[1..3] the faces; adm
   marks admissible stencils.  Returns the delta bits (bit 0 = central). */
static int teno_select(const or_ctx *c, const double *si, const int *adm, double lam1, double lams) {
    double g[4], sum = 0.0;
    int st = 1;
    for (int s = 1; s < 4; ++s) st += adm[s];
    if (c->scheme == OR_CTENO || c->scheme == OR_TENO) {
        for (int s = 0; s < 4; ++s) {
            if (!adm[s]) continue;
            double lam = (s == 0) ? lam1 : lams;
            g[s] = 1.0 / pow6(si[s] + c->eps);
            if (c->scheme == OR_CTENO && c->gamma_form == OR_GAMMA_LAMBDA) g[s] = lam / pow6(si[s] + c->eps);
        }
    } else {
        double tsum = 0.0;
        for (int s = 1; s < 4; ++s) if (adm[s]) tsum += fabs(si[s] - si[0]);
        double tau = pow6(tsum / (st - 1));
        for (int s = 0; s < 4; ++s) {
            if (!adm[s]) continue;
            if (c->gamma_form == OR_GAMMA_SCALED) g[s] = 1.0 + tau / pow6(si[s] + c->eps);
            else g[s] = 1.0 + tau / (si[s] + c->eps);
        }
    }
    for (int s = 0; s < 4; ++s) if (adm[s]) sum += g[s];
    int bits = 0;
    for (int s = 0; s < 4; ++s) {
        if (!adm[s]) continue;
        double chi = g[s] / sum;
        if (!(chi < c->ct)) bits |= 1 << s;
    }
    return bits;
}

/* CWENO nonlinear weights: omega_s proportional to lambda_s / (eps + SI_s)^4
   over the admissible stencils, normalised to sum 1 */
static void cweno_weights(const or_ctx *c, const double *si, const int *adm, double lam1, double lams, double *w) {
    double g[4] = {0, 0, 0, 0}, sum = 0.0;
    for (int s = 0; s < 4; ++s) {
        if (!adm[s]) continue;
        double e = c->eps + si[s], e2 = e * e;
        g[s] = ((s == 0) ? lam1 : lams) / (e2 * e2);
        sum += g[s];
    }
    for (int s = 0; s < 4; ++s) w[s] = adm[s] ? g[s] / sum : 0.0;
}

/* evaluate p = U0 + sum a_k (psi_k - mean psi_k) at (xi, eta) */
static double poly_eval(const or_ctx *c, double U0, const double *a, int K, double xi, double eta) {
    double v = U0;
    for (int k = 1; k <= K; ++k) {
        int ax = c->ex[k][0], ay = c->ex[k][1];
        v += a[k - 1] * (pow(xi, ax) * pow(eta, ay) - 2.0 * ref_mono(ax, ay));
    }
    return v;
}

/* One reconstructed field: a conserved variable, or one characteristic
   field on one face.  vc[m] are the field's values on the central stencil
   (central-list order), vd[f][m] on the directional stencils, w0 on the
   cell.  Least squares (sec. 2.1), p_1 (eq. e17), smoothness indicators,
   the scheme's selection or weights, and the final coefficients fin[K]
   (p = w0 + sum_k fin_k phi_k).  forced < 0: compute the selection. */
static int reconstruct_field(or_ctx *c, or_cell *pc, const int *adm, int st, double lam1, double lams, double w0,
                             const double *vc, double vd[3][OR_MAXM], int forced, int *bits_out, double *fin) {
    int M = c->M, K = c->K, Kd = c->Kd;
    double b[OR_MAXM], aopt[OR_MAXK], ad[3][OR_MAXK];
    for (int m = 0; m < M; ++m) b[m] = pc->wc[m] * (vc[m] - w0);
    hh_solve(pc->qa, M, K, pc->qv0, pc->qb, pc->qr, b, aopt);
    for (int f = 0; f < 3; ++f) {
        if (!adm[f + 1]) continue;
        int n = pc->dirn[f];
        for (int m = 0; m < n; ++m) b[m] = pc->wd[f][m] * (vd[f][m] - w0);
        hh_solve(pc->da[f], n, Kd, pc->dv0[f], pc->db[f], pc->dr[f], b, ad[f]);
    }
    /* p_1 = (p_opt - sum_s lambda_s p_s) / lambda_1 (eq. e17); with no
       admissible directional stencil the scheme is the linear p_opt.
       TENO keeps the central-stencil polynomial itself. */
    double a1[OR_MAXK];
    for (int k = 0; k < K; ++k) {
        if (st == 1 || c->scheme == OR_TENO) { a1[k] = aopt[k]; continue; }
        double sm = aopt[k];
        if (k < Kd)
            for (int f = 0; f < 3; ++f) if (adm[f + 1]) sm -= lams * ad[f][k];
        a1[k] = sm / lam1;
    }
    int bits;
    if (c->scheme == OR_CWENO) {
        /* every admissible stencil contributes; the selection byte reports
           them, and forced selections do not apply */
        bits = 1 | (adm[1] << 1) | (adm[2] << 2) | (adm[3] << 3);
        if (st == 1) {
            for (int k = 0; k < K; ++k) fin[k] = a1[k];
        } else {
            double si[4] = {0, 0, 0, 0}, w[4];
            si[0] = smoothness(c, a1, K, c->r);
            for (int f = 0; f < 3; ++f) if (adm[f + 1]) si[f + 1] = smoothness(c, ad[f], Kd, c->rd);
            cweno_weights(c, si, adm, lam1, lams, w);
            for (int k = 0; k < K; ++k) {
                double x = w[0] * a1[k];
                if (k < Kd)
                    for (int f = 0; f < 3; ++f) if (adm[f + 1]) x += w[f + 1] * ad[f][k];
                fin[k] = x;
            }
        }
    } else {
        /* TENO-type selection and the two-branch final polynomial */
        if (st == 1) {
            bits = 1;
        } else {
            double si[4] = {0, 0, 0, 0};
            si[0] = smoothness(c, a1, K, c->r);
            for (int f = 0; f < 3; ++f) if (adm[f + 1]) si[f + 1] = smoothness(c, ad[f], Kd, c->rd);
            bits = teno_select(c, si, adm, lam1, lams);
        }
        if (forced >= 0) bits = forced & (1 | (adm[1] << 1) | (adm[2] << 2) | (adm[3] << 3));
        if (bits & 1) {
            for (int k = 0; k < K; ++k) fin[k] = a1[k];
        } else {
            int nd = 0;
            for (int k = 0; k < K; ++k) fin[k] = 0.0;
            for (int f = 0; f < 3; ++f)
                if (bits & (2 << f)) { ++nd; for (int k = 0; k < Kd; ++k) fin[k] += ad[f][k]; }
            if (nd == 0) return 5;   /* impossible by max chi >= 1/s_t > C_T */
            for (int k = 0; k < Kd; ++k) fin[k] /= nd;
        }
    }
    *bits_out = bits;
    return 0;
}

/* the physical Gauss points of face f of cell i in reference coordinates */
static void face_ref_points(const or_ctx *c, int i, int f, double *xi, double *eta) {
    const int *t = c->tri + 3 * i;
    int pa = t[f], pb = t[(f + 1) % 3];
    for (int q = 0; q < c->Nq; ++q) {
        double x = c->xy[2 * pa] + c->gq[q] * (c->xy[2 * pb] - c->xy[2 * pa]);
        double y = c->xy[2 * pa + 1] + c->gq[q] * (c->xy[2 * pb + 1] - c->xy[2 * pa + 1]);
        to_ref(c, i, x, y, xi + q, eta + q);
    }
}

/* Right eigenvectors (columns) of the Jacobian of the Euler flux in the
   direction of the unit normal n at the state U, for the eigenvalues
   u_n - c, u_n, u_n (shear), u_n + c, and the left eigenvectors L = R^-1
   obtained by Gauss-Jordan elimination. */
int or_char_vectors(double g, const double *U, double nx, double ny, double *Rm, double *Lm) {
    double rho = U[0], u = U[1] / rho, v = U[2] / rho;
    double p = (g - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v));
    double cs = sqrt(g * p / rho), H = (U[3] + p) / rho;
    double un = u * nx + v * ny, ut = -u * ny + v * nx;
    double R[4][4] = {{1.0, 1.0, 0.0, 1.0},
                      {u - cs * nx, u, -ny, u + cs * nx},
                      {v - cs * ny, v, nx, v + cs * ny},
                      {H - un * cs, 0.5 * (u * u + v * v), ut, H + un * cs}};
    double A[4][8];
    for (int r = 0; r < 4; ++r)
        for (int k = 0; k < 8; ++k) A[r][k] = k < 4 ? R[r][k] : (k - 4 == r ? 1.0 : 0.0);
    for (int k = 0; k < 4; ++k) {
        int piv = k;
        for (int r = k + 1; r < 4; ++r) if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
        if (A[piv][k] == 0.0) return 1;
        for (int j = 0; j < 8; ++j) { double tmp = A[k][j]; A[k][j] = A[piv][j]; A[piv][j] = tmp; }
        double d = A[k][k];
        for (int j = 0; j < 8; ++j) A[k][j] /= d;
        for (int r = 0; r < 4; ++r) {
            if (r == k) continue;
            double f = A[r][k];
            for (int j = 0; j < 8; ++j) A[r][j] -= f * A[k][j];
        }
    }
    for (int r = 0; r < 4; ++r)
        for (int k = 0; k < 4; ++k) { Rm[r * 4 + k] = R[r][k]; Lm[r * 4 + k] = A[r][k + 4]; }
    return 0;
}

/* reconstructs cell i: face-point values fv[3][Nq][nv] and the selection
   bits: conserved variables dbits[nv], characteristic variables
   dbits[3][nv] (per face and field); forced (may be NULL, same layout)
   overrides the computed selections */
static int reconstruct_cell(or_ctx *c, int i, const double *U, const uint8_t *forced, double *fv,
                            uint8_t *dbits, double *coef_out) {
    /* forced, fv, dbits, coef_out point at this cell's own entries */
    or_cell *pc = get_cell(c, i);
    if (pc->status) return pc->status;
    int N = c->N, M = c->M, K = c->K, nv = c->nv;
    int adm[4] = {1, pc->dirn[0] > 0, pc->dirn[1] > 0, pc->dirn[2] > 0};
    int st = 1 + adm[1] + adm[2] + adm[3];
    double lam1 = 1.0 - 1.0 / c->lam1p;
    double lams = st > 1 ? (1.0 - lam1) / (st - 1) : 0.0;
    double vc[OR_MAXM], vd[3][OR_MAXM], fin[OR_MAXK];
    if (c->vars == OR_VARS_CHARACTERISTIC) {
        /* per face: fields W = L_f U with the eigenvectors of the flux
           Jacobian along the face normal at the cell's average state */
        double U0[OR_MAXNV];
        for (int v = 0; v < nv; ++v) U0[v] = U[(size_t)v * N + i];
        for (int f = 0; f < 3; ++f) {
            double Rm[16], Lm[16];
            if (or_char_vectors(c->gam, U0, c->fnx[3 * i + f], c->fny[3 * i + f], Rm, Lm)) return 6;
            double xi[OR_MAXNQ], eta[OR_MAXNQ], Wq[OR_MAXNQ][4];
            face_ref_points(c, i, f, xi, eta);
            for (int j = 0; j < 4; ++j) {
                double w0 = 0.0;
                for (int v = 0; v < 4; ++v) w0 += Lm[j * 4 + v] * U0[v];
                for (int m = 0; m < M; ++m) {
                    double x = 0.0;
                    for (int v = 0; v < 4; ++v) x += Lm[j * 4 + v] * U[(size_t)v * N + pc->cen[m]];
                    vc[m] = x;
                }
                for (int s2 = 0; s2 < 3; ++s2)
                    for (int m = 0; m < pc->dirn[s2]; ++m) {
                        double x = 0.0;
                        for (int v = 0; v < 4; ++v) x += Lm[j * 4 + v] * U[(size_t)v * N + pc->dir[s2][m]];
                        vd[s2][m] = x;
                    }
                int bits;
                int rc = reconstruct_field(c, pc, adm, st, lam1, lams, w0, vc, vd,
                                           forced ? forced[f * nv + j] : -1, &bits, fin);
                if (rc) return rc;
                if (dbits) dbits[f * nv + j] = (uint8_t)bits;
                for (int q = 0; q < c->Nq; ++q) Wq[q][j] = poly_eval(c, w0, fin, K, xi[q], eta[q]);
            }
            for (int q = 0; q < c->Nq; ++q)
                for (int v = 0; v < 4; ++v) {
                    double x = 0.0;
                    for (int j = 0; j < 4; ++j) x += Rm[v * 4 + j] * Wq[q][j];
                    fv[((size_t)f * c->Nq + q) * nv + v] = x;
                }
        }
    } else {
        for (int v = 0; v < nv; ++v) {
            const double *Uv = U + (size_t)v * N;
            double U0 = Uv[i];
            for (int m = 0; m < M; ++m) vc[m] = Uv[pc->cen[m]];
            for (int s2 = 0; s2 < 3; ++s2)
                for (int m = 0; m < pc->dirn[s2]; ++m) vd[s2][m] = Uv[pc->dir[s2][m]];
            int bits;
            int rc = reconstruct_field(c, pc, adm, st, lam1, lams, U0, vc, vd, forced ? forced[v] : -1, &bits, fin);
            if (rc) return rc;
            if (dbits) dbits[v] = (uint8_t)bits;
            if (coef_out) for (int k = 0; k < K; ++k) coef_out[(size_t)v * K + k] = fin[k];
            for (int f = 0; f < 3; ++f) {
                double xi[OR_MAXNQ], eta[OR_MAXNQ];
                face_ref_points(c, i, f, xi, eta);
                for (int q = 0; q < c->Nq; ++q)
                    fv[((size_t)f * c->Nq + q) * nv + v] = poly_eval(c, U0, fin, K, xi[q], eta[q]);
            }
        }
    }
    /* optional positivity fallback (not in the paper): a cell whose
       reconstructed state is non-physical at any of its Gauss points
       (density or pressure <= 0) uses its cell average at all of them;
       flagged with bit 7.  Without it the flux reports the state. */
    if (c->physics == OR_EULER && c->positivity) {
        int bad = 0;
        for (int p = 0; p < 3 * c->Nq; ++p) {
            const double *W = fv + (size_t)p * nv;
            double pr = (c->gam - 1.0) * (W[3] - 0.5 * (W[1] * W[1] + W[2] * W[2]) / W[0]);
            if (!(W[0] > 0.0) || !(pr > 0.0)) bad = 1;
        }
        if (bad) {
#pragma omp atomic
            c->n_fallback++;
            for (int p = 0; p < 3 * c->Nq; ++p)
                for (int v = 0; v < nv; ++v) fv[(size_t)p * nv + v] = U[(size_t)v * N + i];
            if (dbits) {
                int nb = c->vars == OR_VARS_CHARACTERISTIC ? 3 * nv : nv;
                for (int k = 0; k < nb; ++k) dbits[k] |= 0x80;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* fluxes                                                              */
/* ------------------------------------------------------------------ */
static void euler_normal_flux(double g, const double *U, double nx, double ny, double *F) {
    double rho = U[0], u = U[1] / rho, v = U[2] / rho, E = U[3];
    double p = (g - 1.0) * (E - 0.5 * rho * (u * u + v * v));
    double un = u * nx + v * ny;
    F[0] = rho * un;
    F[1] = rho * u * un + p * nx;
    F[2] = rho * v * un + p * ny;
    F[3] = (E + p) * un;
}

/* HLLC (sec. 2.7) in the face-normal frame: u normal, w tangential velocity */
static int hllc(double g, const double *UL, const double *UR, double nx, double ny, double *F) {
    double rl = UL[0], rr = UR[0];
    double ul = (UL[1] * nx + UL[2] * ny) / rl, wl = (-UL[1] * ny + UL[2] * nx) / rl;
    double ur = (UR[1] * nx + UR[2] * ny) / rr, wr = (-UR[1] * ny + UR[2] * nx) / rr;
    double El = UL[3], Er = UR[3];
    double pl = (g - 1.0) * (El - 0.5 * rl * (ul * ul + wl * wl));
    double pr = (g - 1.0) * (Er - 0.5 * rr * (ur * ur + wr * wr));
    if (!(rl > 0) || !(rr > 0) || !(pl > 0) || !(pr > 0)) return 6;
    double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
    double Hl = (El + pl) / rl, Hr = (Er + pr) / rr;
    double D = sqrt(rr / rl);
    double ut = (ul + ur * D) / (1.0 + D);
    double wt = (wl + wr * D) / (1.0 + D);
    double Ht = (Hl + Hr * D) / (1.0 + D);
    double ct = sqrt((g - 1.0) * (Ht - 0.5 * (ut * ut + wt * wt)));
    double SL = fmin(ul - cl, ut - ct);
    double SR = fmax(ur + cr, ut + ct);
    double SM = (rr * ur * (SR - ur) - rl * ul * (SL - ul) + pl - pr) / (rr * (SR - ur) - rl * (SL - ul));
    double ps = rl * (ul - SL) * (ul - SM) + pl;
    double Fl[4] = {rl * ul, rl * ul * ul + pl, rl * ul * wl, ul * (El + pl)};
    double Fr[4] = {rr * ur, rr * ur * ur + pr, rr * ur * wr, ur * (Er + pr)};
    double Fn[4];
    if (SL > 0) {
        for (int k = 0; k < 4; ++k) Fn[k] = Fl[k];
    } else if (SL <= 0 && 0 < SM) {
        double d = SL - SM;
        double Us[4] = {rl * (SL - ul) / d, ((SL - ul) * rl * ul + ps - pl) / d, (SL - ul) * rl * wl / d,
                        ((SL - ul) * El - pl * ul + ps * SM) / d};
        double Uc[4] = {rl, rl * ul, rl * wl, El};
        for (int k = 0; k < 4; ++k) Fn[k] = Fl[k] + SL * (Us[k] - Uc[k]);
    } else if (SM <= 0 && 0 < SR) {
        double d = SR - SM;
        double Us[4] = {rr * (SR - ur) / d, ((SR - ur) * rr * ur + ps - pr) / d, (SR - ur) * rr * wr / d,
                        ((SR - ur) * Er - pr * ur + ps * SM) / d};
        double Uc[4] = {rr, rr * ur, rr * wr, Er};
        for (int k = 0; k < 4; ++k) Fn[k] = Fr[k] + SR * (Us[k] - Uc[k]);
    } else {  /* S_R <= 0 */
        for (int k = 0; k < 4; ++k) Fn[k] = Fr[k];
    }
    F[0] = Fn[0];
    F[1] = Fn[1] * nx - Fn[2] * ny;
    F[2] = Fn[1] * ny + Fn[2] * nx;
    F[3] = Fn[3];
    return 0;
}

/* HLLC against the mirror image of the inside state (a wall).  The two
   states have opposite normal velocities and equal density, pressure,
   enthalpy and tangential velocity, so the Roe-averaged normal velocity and
   the contact speed S_M are zero, S_R = -S_L, and the star flux reduces to
   the star pressure on the normal: F = (0, p* n_x, p* n_y, 0) with
   p* = p + rho u_n (u_n - S_L), S_L = min(u_n - c, -c~),
   c~^2 = (gamma - 1)(H - w^2 / 2).  Written out so that the mass and energy
   fluxes through a wall are exactly zero, not a rounding residue of the
   star-region formulas. */
static int wall_flux(double g, const double *UL, double nx, double ny, double *F) {
    double r = UL[0];
    double u = (UL[1] * nx + UL[2] * ny) / r, w = (-UL[1] * ny + UL[2] * nx) / r;
    double E = UL[3];
    double p = (g - 1.0) * (E - 0.5 * r * (u * u + w * w));
    if (!(r > 0) || !(p > 0)) return 6;
    double c = sqrt(g * p / r);
    double H = (E + p) / r;
    double ct = sqrt((g - 1.0) * (H - 0.5 * w * w));
    double SL = fmin(u - c, -ct);
    double ps = r * (u - SL) * u + p;
    F[0] = 0.0;
    F[1] = ps * nx;
    F[2] = ps * ny;
    F[3] = 0.0;
    return 0;
}

int or_wall_flux(double g, const double *UL, double nx, double ny, double *F) { return wall_flux(g, UL, nx, ny, F); }

static int point_flux(const or_ctx *c, const double *UL, const double *UR, double nx, double ny, double *F) {
    if (c->physics == OR_ADVECTION) {
        double an = c->ax * nx + c->ay * ny;
        F[0] = an * (an >= 0 ? UL[0] : UR[0]);
        return 0;
    }
    return hllc(c->gam, UL, UR, nx, ny, F);
}

/* outside state of a boundary face at its Gauss point (px, py) and time t:
   wall = mirror image of the inside state (normal momentum reversed),
   transmissive = the inside state, inflow = the prescribed state on the
   point's side of the moving line */
static void ghost(const or_ctx *c, int kind, const double *UL, double nx, double ny, double px, double py, double t,
                  double *UR) {
    if (kind == OR_INFLOW) {
        int behind = px < c->bline[0] + c->bline[1] * py + c->bline[2] * t;
        for (int v = 0; v < c->nv; ++v) UR[v] = c->bs[behind ? 0 : 1][v];
        return;
    }
    for (int v = 0; v < c->nv; ++v) UR[v] = UL[v];
    if (kind == OR_WALL && c->physics == OR_EULER) {
        double mn = UL[1] * nx + UL[2] * ny;
        UR[1] = UL[1] - 2.0 * mn * nx;
        UR[2] = UL[2] - 2.0 * mn * ny;
    }
}

/* position of Gauss point q of face f of cell i (from vertex f to f+1) */
static void gauss_point(const or_ctx *c, int i, int f, int q, double *px, double *py) {
    int a = c->tri[3 * i + f], b = c->tri[3 * i + (f + 1) % 3];
    *px = c->xy[2 * a] + c->gq[q] * (c->xy[2 * b] - c->xy[2 * a]);
    *py = c->xy[2 * a + 1] + c->gq[q] * (c->xy[2 * b + 1] - c->xy[2 * a + 1]);
}

/* outward, quadrature-integrated flux of every cell face: fo[N][3][nv].
   Each interior face is evaluated once, from its lower-numbered cell. */
static int face_fluxes(or_ctx *c, const double *fv, double t, double *fo) {
    int N = c->N, nv = c->nv, Nq = c->Nq;
    int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
    for (int i = 0; i < N; ++i) {
        for (int f = 0; f < 3; ++f) {
            int j = c->fnb[3 * i + f];
            if (j >= 0 && j < i) continue;
            double nx = c->fnx[3 * i + f], ny = c->fny[3 * i + f];
            double acc[OR_MAXNV] = {0, 0, 0, 0};
            for (int q = 0; q < Nq; ++q) {
                const double *UL = fv + (((size_t)i * 3 + f) * Nq + q) * nv;
                double UR[OR_MAXNV], F[OR_MAXNV];
                if (j >= 0) {
                    int g = c->fnbf[3 * i + f];
                    const double *p = fv + (((size_t)j * 3 + g) * Nq + (Nq - 1 - q)) * nv;
                    for (int v = 0; v < nv; ++v) UR[v] = p[v];
                } else if (c->fbc[3 * i + f] == OR_WALL && c->physics == OR_EULER) {
                    err |= wall_flux(c->gam, UL, nx, ny, F);
                    for (int v = 0; v < nv; ++v) acc[v] += c->gw[q] * F[v];
                    continue;
                } else {
                    double px, py;
                    gauss_point(c, i, f, q, &px, &py);
                    ghost(c, c->fbc[3 * i + f], UL, nx, ny, px, py, t, UR);
                }
                err |= point_flux(c, UL, UR, nx, ny, F);
                for (int v = 0; v < nv; ++v) acc[v] += c->gw[q] * F[v];
            }
            for (int v = 0; v < nv; ++v) {
                double val = c->flen[3 * i + f] * acc[v];
                fo[((size_t)i * 3 + f) * nv + v] = val;
                if (j >= 0) fo[((size_t)j * 3 + c->fnbf[3 * i + f]) * nv + v] = -val;
            }
        }
    }
    return err;
}

/* ------------------------------------------------------------------ */
/* public API                                                          */
/* ------------------------------------------------------------------ */
typedef struct {
    int physics; double ax, ay, gamma;
    int scheme, degree, gamma_form;
    double lambda1_prime, c_t, eps;
    int variables;                 /* OR_VARS_CONSERVED | OR_VARS_CHARACTERISTIC */
    int positivity;                /* 1: optional cell-average fallback (not in the paper) */
} or_scheme;

void or_destroy(or_ctx *c) {
    if (!c) return;
    if (c->cells) { for (int i = 0; i < c->N; ++i) free(c->cells[i]); free(c->cells); }
    if (c->stamp) { for (int t = 0; t < c->nthreads; ++t) free(c->stamp[t]); free(c->stamp); }
    free(c->xy); free(c->tri); free(c->canon); free(c->cx); free(c->cy); free(c->area);
    free(c->fnb); free(c->fnbf); free(c->fbc); free(c->fnx); free(c->fny); free(c->flen);
    free(c->v2c_off); free(c->v2c);
    free(c);
}

/* boundary data of inflow faces (see or_ctx) */
typedef struct {
    double behind[4], ahead[4];
    double line[3];
    int split_kind[4];
    double split_at[4];
} or_boundary;

or_ctx *or_create(int nvert, const double *xy, int ncell, const int *tri, const double *box, const int *bc,
                  const or_scheme *sch, const or_boundary *bnd) {
    or_err[0] = 0;
    if (nvert <= 0 || ncell <= 0 || !xy || !tri || !box || !bc || !sch) { set_err("bad arguments", 0); return NULL; }
    if (sch->degree < 1 || sch->degree > OR_MAXR) { set_err("degree must be 1..6", sch->degree); return NULL; }
    or_ctx *c = calloc(1, sizeof(or_ctx));
    c->nvert = nvert; c->N = ncell;
    c->xy = malloc(sizeof(double) * 2 * nvert); memcpy(c->xy, xy, sizeof(double) * 2 * nvert);
    c->tri = malloc(sizeof(int) * 3 * ncell); memcpy(c->tri, tri, sizeof(int) * 3 * ncell);
    for (int k = 0; k < 4; ++k) { c->box[k] = box[k]; c->bc[k] = bc[k]; }
    if ((bc[0] == OR_PERIODIC) != (bc[1] == OR_PERIODIC) || (bc[2] == OR_PERIODIC) != (bc[3] == OR_PERIODIC)) {
        set_err("periodic sides must come in pairs", 0); or_destroy(c); return NULL;
    }
    if (bnd) {
        for (int v = 0; v < OR_MAXNV; ++v) { c->bs[0][v] = bnd->behind[v]; c->bs[1][v] = bnd->ahead[v]; }
        for (int k = 0; k < 3; ++k) c->bline[k] = bnd->line[k];
        for (int k = 0; k < 4; ++k) { c->split_kind[k] = bnd->split_kind[k]; c->split_at[k] = bnd->split_at[k]; }
    }
    for (int k = 0; k < 4; ++k) {
        if (bc[k] < 0 || bc[k] > OR_INFLOW || c->split_kind[k] < 0 || c->split_kind[k] > OR_INFLOW) {
            set_err("bad boundary kind on side", k); or_destroy(c); return NULL;
        }
        if (c->split_kind[k] != 0 && bc[k] == OR_PERIODIC) {
            set_err("a periodic side cannot switch kind", k); or_destroy(c); return NULL;
        }
    }
    c->per_x = bc[0] == OR_PERIODIC; c->per_y = bc[2] == OR_PERIODIC;
    c->Lx = box[1] - box[0]; c->Ly = box[3] - box[2];
    c->physics = sch->physics; c->nv = sch->physics == OR_EULER ? 4 : 1;
    if (sch->physics == OR_ADVECTION)
        for (int k = 0; k < 4; ++k)
            if (bc[k] == OR_WALL || c->split_kind[k] == OR_WALL) {
                set_err("walls need the Euler equations", k); or_destroy(c); return NULL;
            }
    c->ax = sch->ax; c->ay = sch->ay; c->gam = sch->gamma;
    int inflow = 0;
    for (int k = 0; k < 4; ++k) inflow |= bc[k] == OR_INFLOW || c->split_kind[k] == OR_INFLOW;
    if (inflow && c->physics == OR_EULER)
        for (int s = 0; s < 2; ++s) {
            const double *b = c->bs[s];
            double p = (c->gam - 1.0) * (b[3] - 0.5 * (b[1] * b[1] + b[2] * b[2]) / b[0]);
            if (!(b[0] > 0.0) || !(p > 0.0)) { set_err("non-physical inflow state", s); or_destroy(c); return NULL; }
        }
    c->scheme = sch->scheme; c->r = sch->degree; c->gamma_form = sch->gamma_form;
    c->vars = sch->variables;
    c->positivity = sch->positivity;
    if (c->gamma_form == OR_GAMMA_SCALED && c->scheme != OR_CTENOZ) {
        set_err("the scaled gamma form belongs to CTENOZ", c->gamma_form); or_destroy(c); return NULL;
    }
    if (c->vars == OR_VARS_CHARACTERISTIC && c->physics != OR_EULER) {
        set_err("characteristic variables need the Euler equations", 0); or_destroy(c); return NULL;
    }
    c->lam1p = sch->lambda1_prime; c->ct = sch->c_t; c->eps = sch->eps;
    c->K = (c->r + 1) * (c->r + 2) / 2 - 1;
    c->M = 2 * c->K;
    c->rd = c->r <= 3 ? 1 : (c->r + 1) / 2;
    c->Kd = (c->rd + 1) * (c->rd + 2) / 2 - 1;
    c->Md = 2 * c->Kd;
    c->Nq = (c->r + 2) / 2;
    int k = 1;
    for (int d = 1; d <= c->r; ++d)
        for (int a = d; a >= 0; --a) { c->ex[k][0] = a; c->ex[k][1] = d - a; ++k; }
    /* Gauss-Legendre points on [0, 1] (closed forms of the roots of P_Nq on
       [-1, 1], mapped; weights 2 / ((1 - x^2) P'_Nq(x)^2), halved) */
    if (c->Nq == 1) { c->gq[0] = 0.5; c->gw[0] = 1.0; }
    else if (c->Nq == 2) {
        double s = 0.5 / sqrt(3.0);
        c->gq[0] = 0.5 - s; c->gq[1] = 0.5 + s; c->gw[0] = c->gw[1] = 0.5;
    } else if (c->Nq == 3) {
        double x = sqrt(0.6);
        c->gq[0] = 0.5 - 0.5 * x; c->gq[1] = 0.5; c->gq[2] = 0.5 + 0.5 * x;
        c->gw[0] = c->gw[2] = 5.0 / 18.0; c->gw[1] = 8.0 / 18.0;
    } else {
        double x1 = sqrt(3.0 / 7.0 - 2.0 / 7.0 * sqrt(1.2)), x2 = sqrt(3.0 / 7.0 + 2.0 / 7.0 * sqrt(1.2));
        double w1 = (18.0 + sqrt(30.0)) / 36.0, w2 = (18.0 - sqrt(30.0)) / 36.0;
        c->gq[0] = 0.5 - 0.5 * x2; c->gq[1] = 0.5 - 0.5 * x1; c->gq[2] = 0.5 + 0.5 * x1; c->gq[3] = 0.5 + 0.5 * x2;
        c->gw[0] = c->gw[3] = 0.5 * w2; c->gw[1] = c->gw[2] = 0.5 * w1;
    }
    /* centroids from the input vertex order */
    c->cx = NULL;
    double *cx = malloc(sizeof(double) * ncell), *cy = malloc(sizeof(double) * ncell);
    for (int i = 0; i < ncell; ++i) {
        const int *t = tri + 3 * i;
        cx[i] = (xy[2 * t[0]] + xy[2 * t[1]] + xy[2 * t[2]]) / 3.0;
        cy[i] = (xy[2 * t[0] + 1] + xy[2 * t[1] + 1] + xy[2 * t[2] + 1]) / 3.0;
    }
    if (!build_mesh(c)) { free(cx); free(cy); or_destroy(c); return NULL; }
    memcpy(c->cx, cx, sizeof(double) * ncell); memcpy(c->cy, cy, sizeof(double) * ncell);
    free(cx); free(cy);
    c->cells = calloc((size_t)ncell, sizeof(or_cell *));
#ifdef _OPENMP
    /* per-thread stamps for as many threads as a later or_set_threads may start */
    c->nthreads = omp_get_max_threads() > omp_get_num_procs() ? omp_get_max_threads() : omp_get_num_procs();
#else
    c->nthreads = 1;
#endif
    c->stamp = calloc((size_t)c->nthreads, sizeof(int *));
    return c;
}

int or_n_cells(const or_ctx *c) { return c->N; }
int or_dims(const or_ctx *c, int *K, int *M, int *Kd, int *Md, int *Nq, int *nv) {
    *K = c->K; *M = c->M; *Kd = c->Kd; *Md = c->Md; *Nq = c->Nq; *nv = c->nv; return 0;
}

/* builds stencils and least-squares factors for every cell (OpenMP) */
int or_prepare(or_ctx *c) {
    int bad = -1;
#pragma omp parallel for schedule(dynamic, 256)
    for (int i = 0; i < c->N; ++i) {
        or_cell *pc = get_cell(c, i);
        if (pc->status) {
#pragma omp critical
            { if (bad < 0 || i < bad) bad = i; }
        }
    }
    if (bad >= 0) { set_err("stencil or least-squares failure at cell", bad); return c->cells[bad]->status; }
    return 0;
}

int or_geometry(or_ctx *c, double *cxy, double *area, int *fnb, int *fnbf, double *fn) {
    for (int i = 0; i < c->N; ++i) {
        if (cxy) { cxy[2 * i] = c->cx[i]; cxy[2 * i + 1] = c->cy[i]; }
        if (area) area[i] = c->area[i];
        for (int f = 0; f < 3; ++f) {
            if (fnb) fnb[3 * i + f] = c->fnb[3 * i + f];
            if (fnbf) fnbf[3 * i + f] = c->fnbf[3 * i + f];
            if (fn) {
                fn[3 * (3 * i + f)] = c->fnx[3 * i + f];
                fn[3 * (3 * i + f) + 1] = c->fny[3 * i + f];
                fn[3 * (3 * i + f) + 2] = c->flen[3 * i + f];
            }
        }
    }
    return 0;
}

/* stencils of selected cells: cen[n][M], dir[n][3][Md] (-1 padded), dirn[n][3] */
int or_stencils(or_ctx *c, int n, const int *cells, int *cen, int *dir, int *dirn) {
    for (int a = 0; a < n; ++a) {
        int i = cells[a];
        if (i < 0 || i >= c->N) { set_err("cell out of range", i); return 1; }
        or_cell *pc = get_cell(c, i);
        if (pc->status) { set_err("stencil failure at cell", i); return pc->status; }
        for (int m = 0; m < c->M; ++m) cen[(size_t)a * c->M + m] = pc->cen[m];
        for (int f = 0; f < 3; ++f) {
            dirn[a * 3 + f] = pc->dirn[f];
            for (int m = 0; m < c->Md; ++m)
                dir[((size_t)a * 3 + f) * c->Md + m] = m < pc->dirn[f] ? pc->dir[f][m] : -1;
        }
    }
    return 0;
}

/* pseudo-inverses of selected cells, by solving for each weighted unit
   right-hand side: pc[n][K][M] (columns in the order of or_stencils' cen),
   pd[n][3][Kd][Md] (zero for inadmissible / absent members) */
int or_pinv(or_ctx *c, int n, const int *cells, double *pcen, double *pdir) {
    int M = c->M, K = c->K, Kd = c->Kd, Md = c->Md;
    for (int a = 0; a < n; ++a) {
        or_cell *pc = get_cell(c, cells[a]);
        if (pc->status) { set_err("stencil failure at cell", cells[a]); return pc->status; }
        for (int m = 0; m < M; ++m) {
            double b[OR_MAXM] = {0}, x[OR_MAXK];
            b[m] = pc->wc[m];
            hh_solve(pc->qa, M, K, pc->qv0, pc->qb, pc->qr, b, x);
            for (int k = 0; k < K; ++k) pcen[((size_t)a * K + k) * M + m] = x[k];
        }
        for (int f = 0; f < 3; ++f)
            for (int m = 0; m < Md; ++m) {
                double x[OR_MAXK] = {0};
                if (m < pc->dirn[f]) {
                    double b[OR_MAXM] = {0};
                    b[m] = pc->wd[f][m];
                    hh_solve(pc->da[f], pc->dirn[f], Kd, pc->dv0[f], pc->db[f], pc->dr[f], b, x);
                }
                for (int k = 0; k < Kd; ++k) pdir[(((size_t)a * 3 + f) * Kd + k) * Md + m] = x[k];
            }
    }
    return 0;
}

/* least-squares matrix of the central stencil of one cell (K columns,
   rows in or_stencils' order), column-major [K][M]; and its row weights */
int or_ls_matrix(or_ctx *c, int i, double *A, double *w) {
    or_cell *pc = get_cell(c, i);
    if (pc->status) return pc->status;
    build_ls(c, i, c->M, pc->cen, pc->csx, pc->csy, c->K, A, w);
    return 0;
}

/* smoothness indicator of coefficients a[K'] of the first K' basis functions */
double or_smoothness(or_ctx *c, const double *a, int Kp, int r) { return smoothness(c, a, Kp, r); }

/* raw TENO selection for tests: si[4], adm[4] -> delta bits */
int or_select(or_ctx *c, const double *si, const int *adm) {
    int st = 1 + adm[1] + adm[2] + adm[3];
    double lam1 = 1.0 - 1.0 / c->lam1p;
    double lams = st > 1 ? (1.0 - lam1) / (st - 1) : 0.0;
    return teno_select(c, si, adm, lam1, lams);
}

/* CWENO nonlinear weights w[4] for smoothness indicators si[4] and the
   admissibility mask adm[4] (central first) */
int or_cweno_weights(or_ctx *c, const double *si, const int *adm, double *w) {
    int st = 1 + adm[1] + adm[2] + adm[3];
    double lam1 = st > 1 ? 1.0 - 1.0 / c->lam1p : 1.0;
    double lams = st > 1 ? (1.0 - lam1) / (st - 1) : 0.0;
    cweno_weights(c, si, adm, lam1, lams, w);
    return 0;
}

int or_hllc(double g, const double *UL, const double *UR, double nx, double ny, double *F) {
    return hllc(g, UL, UR, nx, ny, F);
}
void or_euler_flux(double g, const double *U, double nx, double ny, double *F) { euler_normal_flux(g, U, nx, ny, F); }

/* reconstruction of all cells: fv[N][3][Nq][nv], delta[N][nv] (characteristic
   variables: [N][3][nv]; may be NULL),
   coef[N][nv][K] (may be NULL), forced[N][nv] (may be NULL) */
int or_reconstruct(or_ctx *c, const double *U, const uint8_t *forced, double *fv, uint8_t *delta, double *coef) {
    int rc = or_prepare(c);
    if (rc) return rc;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int i = 0; i < c->N; ++i) {
        size_t nv = c->nv, nb = c->vars == OR_VARS_CHARACTERISTIC ? 3 * nv : nv;
        bad |= reconstruct_cell(c, i, U, forced ? forced + i * nb : NULL, fv + (size_t)i * 3 * c->Nq * nv,
                                delta ? delta + i * nb : NULL, coef ? coef + i * nv * c->K : NULL);
    }
    if (bad) set_err("reconstruction failure", bad);
    return bad;
}

/* reconstruction of selected cells only: fv[n][3][Nq][nv], delta[n][nv] */
int or_reconstruct_cells(or_ctx *c, const double *U, int n, const int *cells, double *fv, uint8_t *delta) {
    size_t nv = c->nv, Nq = c->Nq, nb = c->vars == OR_VARS_CHARACTERISTIC ? 3 * nv : nv;
    for (int a = 0; a < n; ++a) {
        int i = cells[a];
        if (i < 0 || i >= c->N) { set_err("cell out of range", i); return 1; }
        int rc = reconstruct_cell(c, i, U, NULL, fv + (size_t)a * 3 * Nq * nv, delta ? delta + (size_t)a * nb : NULL, NULL);
        if (rc) { set_err("reconstruction failure at cell", i); return rc; }
    }
    return 0;
}

/* residual of selected cells only: each sampled cell and its face
   neighbours are reconstructed, the three face fluxes formed as in
   face_fluxes (owner = lower cell id), R[n][nv] */
int or_residual_cells(or_ctx *c, const double *U, double t, int n, const int *cells, double *R) {
    int nv = c->nv, Nq = c->Nq;
    size_t per = (size_t)3 * Nq * nv;
    double *own = malloc(sizeof(double) * per), *nbf = malloc(sizeof(double) * per);
    uint8_t dl[3 * OR_MAXNV];
    int rc = 0;
    for (int a = 0; a < n && !rc; ++a) {
        int i = cells[a];
        if (i < 0 || i >= c->N) { rc = 1; set_err("cell out of range", i); break; }
        rc = reconstruct_cell(c, i, U, NULL, own, dl, NULL);
        double acc[OR_MAXNV] = {0, 0, 0, 0};
        for (int f = 0; f < 3 && !rc; ++f) {
            int j = c->fnb[3 * i + f];
            int g = c->fnbf[3 * i + f];
            if (j >= 0) rc = reconstruct_cell(c, j, U, NULL, nbf, dl, NULL);
            if (rc) break;
            /* evaluate from the owner's side exactly as face_fluxes does */
            int owner_is_i = (j < 0) || (i < j);
            int oc = owner_is_i ? i : j, of = owner_is_i ? f : g;
            const double *ofv = owner_is_i ? own : nbf, *xfv = owner_is_i ? nbf : own;
            int xf = owner_is_i ? g : f;
            double nx = c->fnx[3 * oc + of], ny = c->fny[3 * oc + of];
            double facc[OR_MAXNV] = {0, 0, 0, 0};
            for (int q = 0; q < Nq; ++q) {
                const double *UL = ofv + ((size_t)of * Nq + q) * nv;
                double UR[OR_MAXNV], F[OR_MAXNV];
                if (j >= 0) {
                    const double *p = xfv + ((size_t)xf * Nq + (Nq - 1 - q)) * nv;
                    for (int v = 0; v < nv; ++v) UR[v] = p[v];
                } else if (c->fbc[3 * i + f] == OR_WALL && c->physics == OR_EULER) {
                    rc |= wall_flux(c->gam, UL, nx, ny, F);
                    for (int v = 0; v < nv; ++v) facc[v] += c->gw[q] * F[v];
                    continue;
                } else {
                    double px, py;
                    gauss_point(c, i, f, q, &px, &py);
                    ghost(c, c->fbc[3 * i + f], UL, nx, ny, px, py, t, UR);
                }
                rc |= point_flux(c, UL, UR, nx, ny, F);
                for (int v = 0; v < nv; ++v) facc[v] += c->gw[q] * F[v];
            }
            for (int v = 0; v < nv; ++v) {
                double val = c->flen[3 * oc + of] * facc[v];
                acc[v] += owner_is_i ? val : -val;
            }
        }
        for (int v = 0; v < nv; ++v) R[(size_t)a * nv + v] = -acc[v] / c->area[i];
    }
    free(own); free(nbf);
    return rc;
}

int or_face_fluxes(or_ctx *c, const double *fv, double t, double *fo) {
    int rc = face_fluxes(c, fv, t, fo);
    if (rc) set_err("non-physical face state", rc);
    return rc;
}

/* R[nv][N] = -(1/|V_i|) sum_f fo[i][f] */
static void residual_from_fluxes(const or_ctx *c, const double *fo, double *R) {
    int N = c->N, nv = c->nv;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (int v = 0; v < nv; ++v) {
            double s = 0.0;
            for (int f = 0; f < 3; ++f) s += fo[((size_t)i * 3 + f) * nv + v];
            R[(size_t)v * N + i] = -s / c->area[i];
        }
}

typedef struct { double *fv, *fo; uint8_t *delta; } or_work;

static int residual(or_ctx *c, const double *U, double t, double *R, or_work *w) {
    int rc = or_reconstruct(c, U, NULL, w->fv, w->delta, NULL);
    if (rc) return rc;
    rc = or_face_fluxes(c, w->fv, t, w->fo);
    if (rc) return rc;
    residual_from_fluxes(c, w->fo, R);
    return 0;
}

int or_residual(or_ctx *c, const double *U, double t, double *R) {
    size_t N = c->N;
    or_work w;
    w.fv = malloc(sizeof(double) * N * 3 * c->Nq * c->nv);
    w.fo = malloc(sizeof(double) * N * 3 * c->nv);
    w.delta = malloc((size_t)N * 3 * c->nv);
    int rc = residual(c, U, t, R, &w);
    free(w.fv); free(w.fo); free(w.delta);
    return rc;
}

/* minimum over cells of 2|V_i| / sum_f |A_f| s_f, s_f the normal signal speed */
double or_dt_bound(or_ctx *c, const double *U) {
    int N = c->N;
    double best = INFINITY;
    for (int i = 0; i < N; ++i) {
        double sum = 0.0;
        double u = 0, v = 0, a = 0;
        if (c->physics == OR_EULER) {
            double rho = U[i], mx = U[(size_t)N + i], my = U[2 * (size_t)N + i], E = U[3 * (size_t)N + i];
            u = mx / rho; v = my / rho;
            double p = (c->gam - 1.0) * (E - 0.5 * rho * (u * u + v * v));
            a = sqrt(c->gam * p / rho);
        }
        for (int f = 0; f < 3; ++f) {
            double nx = c->fnx[3 * i + f], ny = c->fny[3 * i + f], s;
            if (c->physics == OR_EULER) s = fabs(u * nx + v * ny) + a;
            else s = fabs(c->ax * nx + c->ay * ny);
            sum += c->flen[3 * i + f] * s;
        }
        double d = 2.0 * c->area[i] / sum;
        if (d < best) best = d;
    }
    return best;
}

/* one Shu-Osher SSP-RK3 step of size dt from time t, in place on U[nv][N];
   the three residuals are those of the stage times t, t + dt and t + dt/2 */
int or_rk3_step(or_ctx *c, double *U, double t, double dt) {
    size_t n = (size_t)c->N * c->nv;
    double *U1 = malloc(sizeof(double) * n), *U2 = malloc(sizeof(double) * n), *R = malloc(sizeof(double) * n);
    or_work w;
    w.fv = malloc(sizeof(double) * (size_t)c->N * 3 * c->Nq * c->nv);
    w.fo = malloc(sizeof(double) * (size_t)c->N * 3 * c->nv);
    w.delta = malloc((size_t)c->N * 3 * c->nv);
    int rc = residual(c, U, t, R, &w);
    if (!rc) {
        for (size_t k = 0; k < n; ++k) U1[k] = U[k] + dt * R[k];
        rc = residual(c, U1, t + dt, R, &w);
    }
    if (!rc) {
        for (size_t k = 0; k < n; ++k) U2[k] = 0.75 * U[k] + 0.25 * (U1[k] + dt * R[k]);
        rc = residual(c, U2, t + 0.5 * dt, R, &w);
    }
    if (!rc)
        for (size_t k = 0; k < n; ++k) U[k] = (1.0 / 3.0) * U[k] + (2.0 / 3.0) * (U2[k] + dt * R[k]);
    free(U1); free(U2); free(R); free(w.fv); free(w.fo); free(w.delta);
    return rc;
}

/* march to t_final (or max_steps) with dt = cfl * bound, the last step
   clipped to land on t_final; returns steps taken in *steps and time in *t */
int or_solve(or_ctx *c, double *U, double t0, double t_final, int max_steps, double cfl, int *steps, double *t_out) {
    double t = t0;
    int n = 0;
    int rc = or_prepare(c);
    if (rc) return rc;
    while (t < t_final && n < max_steps) {
        double dt = cfl * or_dt_bound(c, U);
        double tn = t + dt;
        if (dt >= t_final - t) { dt = t_final - t; tn = t_final; }
        rc = or_rk3_step(c, U, t, dt);
        if (rc) break;
        t = tn;
        ++n;
    }
    *steps = n;
    *t_out = t;
    return rc;
}

/* number of cell reconstructions that took the positivity fallback since
   the context was created or the count was reset */
long long or_fallbacks(const or_ctx *c) { return c->n_fallback; }
void or_reset_fallbacks(or_ctx *c) { c->n_fallback = 0; }

/* threads of the OpenMP loops of contexts created from now on (timing only:
   results do not depend on it) */
void or_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
