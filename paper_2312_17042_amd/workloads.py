"""Seeded synthetic workloads: meshes, initial cell averages and exact solutions.

This module is the only code that both the CPU oracle's tests and the GPU
library's tests/bench consume.  It generates inputs and exact reference
solutions; it contains none of the finite-volume method's arithmetic
(no stencils, no least squares, no weights, no fluxes).

Mesh recipe (the paper's meshes are not available, so these stand in for them):
  * an nx x ny grid of rectangles on [x0,x1]x[y0,y1], each split into two
    counter-clockwise triangles along a diagonal picked by one random bit;
  * every interior vertex is moved by an independent uniform offset in
    [-jitter*hx, jitter*hx] x [-jitter*hy, jitter*hy]; boundary vertices stay
    put, so periodic seams keep matching vertices;
  * numpy PCG64 ``default_rng(seed)``; draw order: nx*ny diagonal bits in
    row-major square order (row j outer, column i inner), then two jitter
    draws per interior vertex in row-major vertex order.
Vertices are emitted row-major, (nx+1)*(ny+1) of them (seam vertices are
duplicated, the library/oracle weld them); triangles are emitted in square
order, two per square.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PERIODIC, WALL, TRANSMISSIVE, INFLOW = 0, 1, 2, 3
ADVECTION, EULER = 0, 1


@dataclass
class Boundary:
    """Prescribed outside states of INFLOW faces: `behind` (conserved
    variables) at points with x < line[0] + line[1] y + line[2] t, `ahead`
    elsewhere; a side k switches to kind split_kind[k] (0 = no switch) where
    its coordinate along the side (y on the sides x = const, x on the others)
    is below split_at[k]."""
    behind: tuple = (0.0, 0.0, 0.0, 0.0)
    ahead: tuple = (0.0, 0.0, 0.0, 0.0)
    line: tuple = (0.0, 0.0, 0.0)
    split_kind: tuple = (0, 0, 0, 0)
    split_at: tuple = (0.0, 0.0, 0.0, 0.0)


def constant_inflow(state):
    """One prescribed state on every INFLOW side."""
    st = tuple(float(v) for v in state)
    return Boundary(behind=st, ahead=st)


@dataclass
class Mesh:
    xy: np.ndarray          # float64 [n_vertices, 2]
    tri: np.ndarray         # int32 [n_cells, 3]
    box: tuple              # (x0, x1, y0, y1)
    bc: tuple               # (xmin, xmax, ymin, ymax) boundary kinds
    nx: int
    ny: int
    seed: int
    meta: dict = field(default_factory=dict)
    boundary: Boundary | None = None

    @property
    def n_cells(self) -> int:
        return int(self.tri.shape[0])

    @property
    def h(self) -> float:
        return (self.box[1] - self.box[0]) / self.nx


def split_jitter_mesh(nx, ny, box=(0.0, 1.0, 0.0, 1.0), seed=0, jitter=0.2,
                      bc=(PERIODIC, PERIODIC, PERIODIC, PERIODIC)) -> Mesh:
    x0, x1, y0, y1 = map(float, box)
    hx = (x1 - x0) / nx
    hy = (y1 - y0) / ny
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 2, size=nx * ny)
    n_int = max(nx - 1, 0) * max(ny - 1, 0)
    jit = rng.uniform(-1.0, 1.0, size=(n_int, 2)) * jitter

    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1))
    x = x0 + ii.astype(np.float64) * hx
    y = y0 + jj.astype(np.float64) * hy
    # pin the far edges exactly so the periodic seams match bit-for-bit
    x[:, nx] = x1
    y[ny, :] = y1
    if n_int:
        x[1:ny, 1:nx] += (jit[:, 0] * hx).reshape(ny - 1, nx - 1)
        y[1:ny, 1:nx] += (jit[:, 1] * hy).reshape(ny - 1, nx - 1)
    xy = np.stack([x.ravel(), y.ravel()], axis=1)

    sj, si = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    sj = sj.ravel()
    si = si.ravel()
    v00 = sj * (nx + 1) + si
    v10 = v00 + 1
    v01 = v00 + (nx + 1)
    v11 = v01 + 1
    b = bits.astype(bool)
    t1 = np.where(b[:, None], np.stack([v00, v10, v01], 1), np.stack([v00, v10, v11], 1))
    t2 = np.where(b[:, None], np.stack([v10, v11, v01], 1), np.stack([v00, v11, v01], 1))
    tri = np.stack([t1, t2], axis=1).reshape(-1, 3).astype(np.int32)
    return Mesh(xy=np.ascontiguousarray(xy), tri=np.ascontiguousarray(tri),
                box=(x0, x1, y0, y1), bc=tuple(int(v) for v in bc), nx=nx, ny=ny, seed=seed)


# ----------------------------------------------------------------------------
# quadrature used only to produce exact cell averages of closed-form fields
# ----------------------------------------------------------------------------

def _collapsed_gauss(n):
    """Collapsed (Duffy) Gauss-Legendre rule on the unit reference triangle.

    Returns (xi, eta, w) with sum(w) = 1/2; exact for total degree <= 2n-2.
    """
    g, gw = np.polynomial.legendre.leggauss(n)
    u = 0.5 * (g + 1.0)
    wu = 0.5 * gw
    U, V = np.meshgrid(u, u, indexing="ij")
    WU, WV = np.meshgrid(wu, wu, indexing="ij")
    xi = U.ravel()
    eta = (V * (1.0 - U)).ravel()
    w = (WU * WV * (1.0 - U)).ravel()
    return xi, eta, w


def cell_points(mesh: Mesh, n=6, cells=None):
    """Physical quadrature points and weights (weights sum to 1 per cell)."""
    tri = mesh.tri if cells is None else mesh.tri[cells]
    p0 = mesh.xy[tri[:, 0]]
    p1 = mesh.xy[tri[:, 1]]
    p2 = mesh.xy[tri[:, 2]]
    xi, eta, w = _collapsed_gauss(n)
    X = p0[:, None, 0] + xi[None, :] * (p1[:, None, 0] - p0[:, None, 0]) + eta[None, :] * (p2[:, None, 0] - p0[:, None, 0])
    Y = p0[:, None, 1] + xi[None, :] * (p1[:, None, 1] - p0[:, None, 1]) + eta[None, :] * (p2[:, None, 1] - p0[:, None, 1])
    return X, Y, 2.0 * w


def cell_average(mesh: Mesh, f, n=6, chunk=1 << 20):
    """Cell averages of f(X, Y) -> array [..., npts] (leading dims = variables)."""
    N = mesh.n_cells
    out = None
    for s in range(0, N, chunk):
        idx = np.arange(s, min(N, s + chunk))
        X, Y, w = cell_points(mesh, n, idx)
        vals = np.asarray(f(X, Y))
        avg = (vals * w).sum(axis=-1)
        if out is None:
            out = np.empty(avg.shape[:-1] + (N,), dtype=np.float64)
        out[..., idx] = avg
    return out


def cell_areas(mesh: Mesh):
    p0 = mesh.xy[mesh.tri[:, 0]]
    p1 = mesh.xy[mesh.tri[:, 1]]
    p2 = mesh.xy[mesh.tri[:, 2]]
    return 0.5 * np.abs((p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p2[:, 0] - p0[:, 0]) * (p1[:, 1] - p0[:, 1]))


# ----------------------------------------------------------------------------
# closed-form fields
# ----------------------------------------------------------------------------

def prim_to_cons(rho, u, v, p, gamma=1.4):
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def advection_sine(t=0.0, ax=1.0, ay=1.0):
    def f(X, Y):
        return np.sin(2.0 * np.pi * ((X - ax * t) + (Y - ay * t)))[None]
    return f


def density_wave(t=0.0, gamma=1.4):
    """rho = 1 + 0.2 sin(2 pi (x + y - 2t)), u = v = p = 1 (periodic unit square)."""
    def f(X, Y):
        rho = 1.0 + 0.2 * np.sin(2.0 * np.pi * (X + Y - 2.0 * t))
        one = np.ones_like(X)
        return prim_to_cons(rho, one, one, one, gamma)
    return f


def isentropic_vortex(t=0.0, beta=5.0, center=(5.0, 5.0), L=(10.0, 10.0), vel=(1.0, 1.0), gamma=1.4):
    """Shu's isentropic vortex on a periodic box, carried by the free stream."""
    def f(X, Y):
        xc = center[0] + vel[0] * t
        yc = center[1] + vel[1] * t
        dx = X - xc
        dy = Y - yc
        dx = dx - L[0] * np.round(dx / L[0])
        dy = dy - L[1] * np.round(dy / L[1])
        r2 = dx * dx + dy * dy
        e = np.exp(0.5 * (1.0 - r2))
        u = vel[0] - beta / (2.0 * np.pi) * dy * e
        v = vel[1] + beta / (2.0 * np.pi) * dx * e
        T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * np.pi * np.pi) * e * e
        rho = T ** (1.0 / (gamma - 1.0))
        p = rho * T
        return prim_to_cons(rho, u, v, p, gamma)
    return f


def riemann_x_average(mesh: Mesh, left, right, x_split=0.5, gamma=1.4):
    """Exact cell averages of a piecewise-constant state split at x = x_split.

    left/right are primitive (rho, u, v, p).  The area fraction of each
    triangle lying left of the line is computed by polygon clipping.
    """
    p = mesh.xy[mesh.tri]                      # [N,3,2]
    frac = _left_area_fraction(p, x_split)
    UL = prim_to_cons(*[np.float64(s) for s in left], gamma=gamma)
    UR = prim_to_cons(*[np.float64(s) for s in right], gamma=gamma)
    return UL[:, None] * frac[None, :] + UR[:, None] * (1.0 - frac[None, :])


def _left_area_fraction(p, xs):
    # clip each triangle against x <= xs (Sutherland-Hodgman, vectorised per edge)
    N = p.shape[0]
    area_full = 0.5 * np.abs((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                             - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    inside = p[:, :, 0] <= xs
    frac = np.where(inside.all(1), 1.0, 0.0)
    mixed = np.where(inside.any(1) & ~inside.all(1))[0]
    for c in mixed:
        poly = []
        for k in range(3):
            a = p[c, k]
            b = p[c, (k + 1) % 3]
            ain = a[0] <= xs
            bin_ = b[0] <= xs
            if ain:
                poly.append(a)
            if ain != bin_:
                s = (xs - a[0]) / (b[0] - a[0])
                poly.append(a + s * (b - a))
        poly = np.array(poly)
        xq = poly[:, 0]
        yq = poly[:, 1]
        ar = 0.5 * abs(np.dot(xq, np.roll(yq, -1)) - np.dot(yq, np.roll(xq, -1)))
        frac[c] = ar / area_full[c]
    return frac


# ----------------------------------------------------------------------------
# exact solution of the 1-D Riemann problem (textbook two-rarefaction/shock
# wave curves with a Newton iteration on the star pressure)
# ----------------------------------------------------------------------------

def _wave_curve(p, rho_k, p_k, c_k, g):
    if p > p_k:   # shock
        A = 2.0 / ((g + 1.0) * rho_k)
        B = (g - 1.0) / (g + 1.0) * p_k
        f = (p - p_k) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - p_k) / (B + p))
    else:         # rarefaction
        f = 2.0 * c_k / (g - 1.0) * ((p / p_k) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho_k * c_k) * (p / p_k) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def riemann_star(left, right, g=1.4):
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(200):
        fl, dfl = _wave_curve(p, rl, pl, cl, g)
        fr, dfr = _wave_curve(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-14, p - dp)
        if abs(pn - p) <= 1e-15 * max(1.0, p):
            p = pn
            break
        p = pn
    fl, _ = _wave_curve(p, rl, pl, cl, g)
    fr, _ = _wave_curve(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def riemann_sample(left, right, s, g=1.4):
    """Exact (rho, u, p) at similarity coordinate s = (x - x0)/t, vectorised over s."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = riemann_star(left, right, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    s = np.asarray(s, dtype=np.float64)
    rho = np.empty_like(s)
    u = np.empty_like(s)
    p = np.empty_like(s)
    gm = (g - 1.0) / (g + 1.0)
    # left side of contact
    if ps > pl:
        rls = rl * ((ps / pl + gm) / (gm * ps / pl + 1.0))
        sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
        m = s <= sl
        left_region = [(m, rl, ul, pl)]
        m2 = (s > sl) & (s <= us)
        left_region.append((m2, rls, us, ps))
        fan = None
    else:
        rls = rl * (ps / pl) ** (1.0 / g)
        cls_ = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
        shl = ul - cl
        stl = us - cls_
        left_region = [(s <= shl, rl, ul, pl), ((s > stl) & (s <= us), rls, us, ps)]
        fan = ((s > shl) & (s <= stl))
    for m, a, b, c in left_region:
        rho[m] = a
        u[m] = b
        p[m] = c
    if fan is not None and fan.any():
        ss = s[fan]
        cc = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * cl) * (ul - ss)
        rho[fan] = rl * cc ** (2.0 / (g - 1.0))
        u[fan] = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * ul + ss)
        p[fan] = pl * cc ** (2.0 * g / (g - 1.0))
    # right side of contact
    if ps > pr:
        rrs = rr * ((ps / pr + gm) / (gm * ps / pr + 1.0))
        sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
        regs = [((s > us) & (s < sr), rrs, us, ps), (s >= sr, rr, ur, pr)]
        fan = None
    else:
        rrs = rr * (ps / pr) ** (1.0 / g)
        crs = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
        shr = ur + cr
        str_ = us + crs
        regs = [((s > us) & (s < str_), rrs, us, ps), (s >= shr, rr, ur, pr)]
        fan = (s >= str_) & (s < shr)
    for m, a, b, c in regs:
        rho[m] = a
        u[m] = b
        p[m] = c
    if fan is not None and fan.any():
        ss = s[fan]
        cc = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * cr) * (ur - ss)
        rho[fan] = rr * cc ** (2.0 / (g - 1.0))
        u[fan] = 2.0 / (g + 1.0) * (-cr + (g - 1.0) / 2.0 * ur + ss)
        p[fan] = pr * cc ** (2.0 * g / (g - 1.0))
    return rho, u, p


def sod_exact(t, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), x0=0.5, gamma=1.4):
    """Exact field of the x-split Riemann problem (rho,u,p) at time t > 0."""
    def f(X, Y):
        s = (X - x0) / t
        rho, u, p = riemann_sample(left, right, s.ravel(), gamma)
        rho = rho.reshape(X.shape)
        u = u.reshape(X.shape)
        p = p.reshape(X.shape)
        return prim_to_cons(rho, u, np.zeros_like(u), p, gamma)
    return f


# ----------------------------------------------------------------------------
# the configured workloads
# ----------------------------------------------------------------------------

def advection_case(n=20, seed=1):
    """Scalar advection of sin(2 pi (x+y)) with a=(1,1) on the periodic unit square."""
    m = split_jitter_mesh(n, n, (0.0, 1.0, 0.0, 1.0), seed=seed)
    u0 = cell_average(m, advection_sine(0.0))
    return m, u0


def vortex_case(n=200, seed=2, beta=5.0, center=(5.0, 5.0), L=10.0, gamma=1.4, quad=6):
    """Isentropic vortex on the periodic [0,L]^2 box (n x n squares, 2n^2 cells)."""
    m = split_jitter_mesh(n, n, (0.0, L, 0.0, L), seed=seed)
    u0 = cell_average(m, isentropic_vortex(0.0, beta, center, (L, L), gamma=gamma), n=quad)
    return m, u0


def sod_case(nx=1600, ny=400, seed=3, left=(1.0, 0.0, 0.0, 1.0), right=(0.125, 0.0, 0.0, 0.1),
             gamma=1.4, Ly=0.25, prescribed=False):
    """x-split Riemann problem on [0,1]x[0,Ly], walls in y, transmissive in x.
    prescribed=True holds the left and right states on the x sides instead
    (far-field sides, split by the line x = 0.5): exact until the first wave
    reaches a side (t = 0.28 for the standard Sod states), and needed for
    runs of thousands of steps, where a transmissive side next to the gas at
    rest lets a boundary mode grow from rounding."""
    side = INFLOW if prescribed else TRANSMISSIVE
    m = split_jitter_mesh(nx, ny, (0.0, 1.0, 0.0, Ly), seed=seed, bc=(side, side, WALL, WALL))
    if prescribed:
        m.boundary = Boundary(behind=tuple(float(v) for v in prim_to_cons(*left, gamma)),
                              ahead=tuple(float(v) for v in prim_to_cons(*right, gamma)), line=(0.5, 0.0, 0.0))
    u0 = riemann_x_average(m, left, right, 0.5, gamma)
    return m, u0


def density_wave_case(n=20, seed=11, gamma=1.4):
    m = split_jitter_mesh(n, n, (0.0, 1.0, 0.0, 1.0), seed=seed)
    u0 = cell_average(m, density_wave(0.0, gamma))
    return m, u0


def shock_density(gamma=1.4):
    """Shock-density wave interaction (sec. 3.1.2): a Mach 3 shock at x = -4
    moving into rho = 1 + 0.2 sin(5x), u = 0, p = 1."""
    def f(X, Y):
        left = X < -4.0
        rho = np.where(left, 3.857143, 1.0 + 0.2 * np.sin(5.0 * X))
        u = np.where(left, 2.629369, 0.0)
        p = np.where(left, 10.33333, 1.0)
        return prim_to_cons(rho, u, 0.0 * X, p, gamma)
    return f


SHOCK_DENSITY_POST = (3.857143, 2.629369, 10.33333)   # rho, u, p behind the Mach 3 shock


def shock_density_case(nx=200, ny=40, seed=12, gamma=1.4, quad=6, prescribed=True):
    """The shock-density wave on [-5, 5] x [0, 2], walls in y.  Both open
    sides take prescribed far-field states: the post-shock state flowing in
    supersonically at x = -5 and the undisturbed gas at rest at x = 5
    (rho = 1 + 0.2 sin 25, which the shock does not reach by t = 1.8); the
    line x = 0 separates the two.  prescribed=False makes both sides
    transmissive instead.  nx x ny squares, 2 nx ny cells; 200 x 40 gives
    h = 1/20 as in the paper."""
    side = INFLOW if prescribed else TRANSMISSIVE
    m = split_jitter_mesh(nx, ny, (-5.0, 5.0, 0.0, 2.0), seed=seed, bc=(side, side, WALL, WALL))
    rho, u, p = SHOCK_DENSITY_POST
    post = tuple(float(v) for v in prim_to_cons(rho, u, 0.0, p, gamma))
    rest = tuple(float(v) for v in prim_to_cons(1.0 + 0.2 * math.sin(25.0), 0.0, 0.0, 1.0, gamma))
    m.boundary = Boundary(behind=post, ahead=rest, line=(0.0, 0.0, 0.0))
    u0 = cell_average(m, shock_density(gamma), n=quad)
    return m, u0


def triple_point(gamma=1.4):
    """Single-material triple point (sec. 3.5): (rho, u, v, p) = (1, 0, 0, 1)
    for x <= 1; (0.125, 0, 0, 0.1) for x > 1, y > 1.5; (1, 0, 0, 0.1) for
    x > 1, y <= 1.5."""
    def f(X, Y):
        left = X <= 1.0
        top = Y > 1.5
        rho = np.where(left, 1.0, np.where(top, 0.125, 1.0))
        p = np.where(left, 1.0, 0.1)
        return prim_to_cons(rho, 0.0 * X, 0.0 * X, p, gamma)
    return f


def triple_point_case(nx=500, ny=215, seed=14, gamma=1.4, quad=6):
    """The triple-point problem on [0, 7] x [0, 3], walls on every side, to
    t = 5.  nx x ny rectangles; 500 x 215 (215,000 cells, h = 0.014) comes
    nearest the paper's 214,770 triangles with h = 1/67."""
    m = split_jitter_mesh(nx, ny, (0.0, 7.0, 0.0, 3.0), seed=seed, bc=(WALL, WALL, WALL, WALL))
    u0 = cell_average(m, triple_point(gamma), n=quad)
    return m, u0


# double Mach reflection (sec. 3.4): states and the incident shock line as the
# paper gives them (shock foot at x = 0.1667, slope 1.732, Mach 10 into gas at
# rest with unit sound speed, so the foot moves at 10 / sin 60 = 20 / 1.732),
# except the post-shock pressure: the Mach 10 jump gives 116.5, the paper
# prints 116.8333
DMR_PRE = (1.4, 0.0, 0.0, 1.0)
DMR_POST = (8.0, 7.145, -4.125, 116.5)
DMR_LINE = (0.1667, 1.0 / 1.732, 20.0 / 1.732)


def dmr(gamma=1.4):
    """Initial field of the double Mach reflection: post-shock state left of
    the incident shock line, pre-shock state right of it."""
    def f(X, Y):
        behind = X < DMR_LINE[0] + DMR_LINE[1] * Y
        st = [np.where(behind, b, a) for b, a in zip(DMR_POST, DMR_PRE)]
        return prim_to_cons(st[0], st[1], st[2], st[3], gamma)
    return f


def dmr_case(nx=240, ny=60, seed=13, gamma=1.4, quad=6):
    """Double Mach reflection on [0, 4] x [0, 1] to t = 0.2: prescribed
    states on the three open sides from the exact moving incident shock
    (post-shock state behind the line, pre-shock ahead): post-shock inflow at
    x = 0, the gas at rest at x = 4 (the line reaches x = 4 only after
    t = 0.28), the top side across the moving shock; bottom side post-shock
    for x < 0.1667 and a wall beyond.  nx x ny squares (nx = 4 ny keeps them
    square); 860 x 215 and 1196 x 299 come nearest the paper's 369,604 and
    714,138 triangles."""
    m = split_jitter_mesh(nx, ny, (0.0, 4.0, 0.0, 1.0), seed=seed, bc=(INFLOW, INFLOW, WALL, INFLOW))
    post = tuple(float(v) for v in prim_to_cons(*DMR_POST, gamma))
    pre = tuple(float(v) for v in prim_to_cons(*DMR_PRE, gamma))
    m.boundary = Boundary(behind=post, ahead=pre, line=DMR_LINE, split_kind=(0, 0, INFLOW, 0),
                          split_at=(0.0, 0.0, DMR_LINE[0], 0.0))
    u0 = cell_average(m, dmr(gamma), n=quad)
    return m, u0


def x_profile(mesh, u, bins):
    """Area-weighted average of u over x-bins of the box (a 1-D profile of a
    y-independent flow)."""
    c = mesh.xy[mesh.tri].mean(1)[:, 0]
    a = cell_areas(mesh)
    x0, x1 = mesh.box[0], mesh.box[1]
    k = np.clip(((c - x0) / (x1 - x0) * bins).astype(np.int64), 0, bins - 1)
    num = np.bincount(k, weights=u * a, minlength=bins)
    den = np.bincount(k, weights=a, minlength=bins)
    return num / np.maximum(den, 1e-300)


@dataclass
class Request:
    index: int
    arrival_s: float
    kind: str          # "vortex" | "riemann"
    n_target: int
    nx: int
    ny: int
    params: dict


def serving_requests(n_requests=256, rate_hz=10.0, seed=4, lo=2e3, hi=2e5):
    """Poisson arrivals of independent 2-D Euler solves with log-uniform sizes."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        n_star = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        if rng.integers(0, 2) == 0:
            n = max(4, int(round(math.sqrt(n_star / 2.0))))
            params = dict(center=(float(rng.uniform(0, 10)), float(rng.uniform(0, 10))),
                          beta=float(rng.uniform(1.0, 5.0)))
            out.append(Request(k, t, "vortex", n_star, n, n, params))
        else:
            ny = max(2, int(round(math.sqrt(n_star / 8.0))))
            params = dict(rho_l=float(rng.uniform(0.1, 1.0)), rho_r=float(rng.uniform(0.1, 1.0)),
                          p_l=float(rng.uniform(0.1, 1.0)), p_r=float(rng.uniform(0.1, 1.0)))
            out.append(Request(k, t, "riemann", n_star, 4 * ny, ny, params))
    return out


def build_request(req: Request, gamma=1.4, quad=4):
    """Mesh + initial cell averages for one serving request (mesh seed 4000 + index)."""
    seed = 4000 + req.index
    if req.kind == "vortex":
        return vortex_case(req.nx, seed=seed, beta=req.params["beta"], center=req.params["center"], gamma=gamma,
                           quad=quad)
    p = req.params
    return sod_case(req.nx, req.ny, seed=seed, left=(p["rho_l"], 0.0, 0.0, p["p_l"]),
                    right=(p["rho_r"], 0.0, 0.0, p["p_r"]), gamma=gamma)
