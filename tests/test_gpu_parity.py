"""GPU (HIP, gfx950) path against the FP64 CPU oracle, through the C ABI.

Tolerances (normwise per variable, ||gpu - oracle||_inf / ||oracle||_inf):
  FP64 mode: 1e-12 for pseudo-inverses, face values, fluxes, residuals and
             final states; TENO selections (delta bits) identical;
  mixed mode (FP32 reconstruction/weights/fluxes, FP64 state): face values
             5e-6 with the oracle's selections forced, pseudo-inverse FP32
             copies 1e-6, final states 1e-5 of the FP64 run.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2312_17042_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_17042_amd import cteno as T  # noqa: E402


def relerr(g, o):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    return float(np.abs(g - o).max() / max(np.abs(o).max(), 1e-300))


def relerr_var(g, o, axis_v=-1):
    g = np.moveaxis(np.asarray(g, np.float64), axis_v, 0).reshape(np.shape(g)[axis_v], -1)
    o = np.moveaxis(np.asarray(o, np.float64), axis_v, 0).reshape(np.shape(o)[axis_v], -1)
    return max(float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)) for a, b in zip(g, o))


def _evolved(case, steps):
    """A workload advanced by the oracle (cubic CTENO, conserved variables,
    with the positivity fallback, which the initial jump needs)."""
    mesh, u0 = case
    o = O.Oracle.from_mesh(mesh, physics=O.EULER, scheme=O.CTENO, degree=3, lambda1_prime=1e15, positivity=1)
    u, n, _ = o.solve(u0, 10.0, cfl=0.3, max_steps=steps)
    assert n == steps
    return mesh, u


CASES = {
    # name: (workload factory, scheme keywords shared by library and oracle)
    "advection_r2_cteno": (lambda: W.advection_case(20, seed=1),
                           dict(physics=O.ADVECTION, scheme=O.CTENO, degree=2, lambda1_prime=1e15)),
    "vortex_r3_ctenoz": (lambda: W.vortex_case(24, seed=2),
                         dict(physics=O.EULER, scheme=O.CTENOZ, degree=3, lambda1_prime=1e4)),
    # the shock cases run with the optional positivity fallback (their
    # initial jumps reconstruct non-physical states without it:
    # test_positivity_is_reported_without_the_fallback)
    "sod_r3_cteno": (lambda: W.sod_case(48, 12, seed=3),
                     dict(physics=O.EULER, scheme=O.CTENO, degree=3, lambda1_prime=1e15, positivity=1)),
    "vortex_r3_cteno_lambda": (lambda: W.vortex_case(20, seed=5),
                               dict(physics=O.EULER, scheme=O.CTENO, degree=3, lambda1_prime=1e15,
                                    gamma_form=O.GAMMA_LAMBDA)),
    "density_r2_ctenoz": (lambda: W.density_wave_case(12, seed=11),
                          dict(physics=O.EULER, scheme=O.CTENOZ, degree=2, lambda1_prime=1e4)),
    # orders 5 to 7: one lane per (cell, variable), N_q = 3 or 4
    "density_r4_ctenoz": (lambda: W.density_wave_case(12, seed=11),
                          dict(physics=O.EULER, scheme=O.CTENOZ, degree=4, lambda1_prime=1e4)),
    "sod_r4_cteno": (lambda: W.sod_case(48, 12, seed=3),
                     dict(physics=O.EULER, scheme=O.CTENO, degree=4, lambda1_prime=1e15, positivity=1)),
    # degree 5 next to walls: the stencils of boundary faces are
    # inadmissible, so the slots of the remaining stencils start elsewhere
    "sod_r5_cteno": (lambda: W.sod_case(48, 12, seed=3),
                     dict(physics=O.EULER, scheme=O.CTENO, degree=5, lambda1_prime=1e15, positivity=1)),
    "vortex_r5_ctenoz": (lambda: W.vortex_case(20, seed=6),
                         dict(physics=O.EULER, scheme=O.CTENOZ, degree=5, lambda1_prime=1e4)),
    # degree 5 with one lane per cell: the directional sums follow the
    # stencil each slot names (degrees 4 and 5 lay out exactly M slots)
    "advection_r5_cteno": (lambda: W.advection_case(20, seed=1),
                           dict(physics=O.ADVECTION, scheme=O.CTENO, degree=5, lambda1_prime=1e15)),
    "advection_r6_cteno_lambda": (lambda: W.advection_case(20, seed=1),
                                  dict(physics=O.ADVECTION, scheme=O.CTENO, degree=6, lambda1_prime=1e15,
                                       gamma_form=O.GAMMA_LAMBDA)),
    "vortex_r6_ctenoz": (lambda: W.vortex_case(20, seed=7),
                         dict(physics=O.EULER, scheme=O.CTENOZ, degree=6, lambda1_prime=1e4)),
    # the paper's comparison schemes in the same pipeline
    "vortex_r3_cweno": (lambda: W.vortex_case(24, seed=2),
                        dict(physics=O.EULER, scheme=O.CWENO, degree=3, lambda1_prime=1e4)),
    "sod_r3_teno": (lambda: W.sod_case(48, 12, seed=3),
                    dict(physics=O.EULER, scheme=O.TENO, degree=3, lambda1_prime=1e15, positivity=1)),
    "sod_r4_cweno": (lambda: W.sod_case(48, 12, seed=3),
                     dict(physics=O.EULER, scheme=O.CWENO, degree=4, lambda1_prime=1e4, positivity=1)),
    "density_r4_teno": (lambda: W.density_wave_case(12, seed=11),
                        dict(physics=O.EULER, scheme=O.TENO, degree=4, lambda1_prime=1e4)),
    # characteristic variables (selection bytes per face and field).  At t = 0
    # every field of the x-split Riemann data is a scaled copy of one step, so
    # the fields select alike; the Sod cases therefore start from the
    # oracle's state after 20 steps (rarefaction, contact and shock apart),
    # and the data carry a velocity so that no conserved variable is zero.
    "sod_r3_cteno_char": (lambda: _evolved(W.sod_case(48, 12, seed=3, left=(1.0, 0.2, 0.1, 1.0),
                                                      right=(0.125, 0.1, -0.05, 0.1)), 20),
                          dict(physics=O.EULER, scheme=O.CTENO, degree=3, lambda1_prime=1e15,
                               variables=O.CHARACTERISTIC)),
    "vortex_r3_ctenoz_char": (lambda: W.vortex_case(24, seed=2),
                              dict(physics=O.EULER, scheme=O.CTENOZ, degree=3, lambda1_prime=1e4,
                                   variables=O.CHARACTERISTIC)),
    "sod_r4_ctenoz_char": (lambda: _evolved(W.sod_case(48, 12, seed=3, left=(1.0, 0.2, 0.1, 1.0),
                                                       right=(0.125, 0.1, -0.05, 0.1)), 20),
                           dict(physics=O.EULER, scheme=O.CTENOZ, degree=4, lambda1_prime=1e4,
                                variables=O.CHARACTERISTIC, positivity=1)),
    "vortex_r5_cweno_char": (lambda: W.vortex_case(20, seed=6),
                             dict(physics=O.EULER, scheme=O.CWENO, degree=5, lambda1_prime=1e4,
                                  variables=O.CHARACTERISTIC)),
    # prescribed-state sides: the shock-density wave's supersonic inflow and
    # the double Mach reflection's moving incident shock (top side) and
    # switched bottom side (inflow, then wall)
    "shockdensity_r4_cteno": (lambda: W.shock_density_case(40, 8),
                              dict(physics=O.EULER, scheme=O.CTENO, degree=4, lambda1_prime=1e15, positivity=1)),
    "dmr_r4_ctenoz": (lambda: W.dmr_case(48, 12),
                      dict(physics=O.EULER, scheme=O.CTENOZ, degree=4, lambda1_prime=1e15, positivity=1)),
    "dmr_r3_cteno_char": (lambda: W.dmr_case(48, 12),
                          dict(physics=O.EULER, scheme=O.CTENO, degree=3, lambda1_prime=1e15,
                               variables=O.CHARACTERISTIC, positivity=1)),
    # CTENOZ with the scaled reading of Algorithm 2's gamma (gamma_form SCALED)
    "vortex_r3_ctenoz_scaled": (lambda: W.vortex_case(24, seed=2),
                                dict(physics=O.EULER, scheme=O.CTENOZ, degree=3, lambda1_prime=1e4,
                                     gamma_form=O.GAMMA_SCALED)),
    "density_r2_ctenoz_scaled": (lambda: W.density_wave_case(12, seed=11),
                                 dict(physics=O.EULER, scheme=O.CTENOZ, degree=2, lambda1_prime=1e4,
                                      gamma_form=O.GAMMA_SCALED)),
    "sod_r3_ctenoz_scaled_char": (lambda: _evolved(W.sod_case(48, 12, seed=3, left=(1.0, 0.2, 0.1, 1.0),
                                                              right=(0.125, 0.1, -0.05, 0.1)), 20),
                                  dict(physics=O.EULER, scheme=O.CTENOZ, degree=3, lambda1_prime=1e4,
                                       variables=O.CHARACTERISTIC, gamma_form=O.GAMMA_SCALED, positivity=1)),
    "vortex_r5_ctenoz_scaled": (lambda: W.vortex_case(20, seed=6),
                                dict(physics=O.EULER, scheme=O.CTENOZ, degree=5, lambda1_prime=1e4,
                                     gamma_form=O.GAMMA_SCALED)),
}


EPS64 = float(np.finfo(np.float64).eps)


def mixed_tolerance(name, mesh, uo, t):
    """Tolerance of a mixed-precision march against the FP64 oracle: 1e-5
    normwise per variable, or 1% of the oracle's own error against the exact
    solution (vortex cases: the vortex carried by the free stream), whichever
    is larger."""
    tol = 1e-5
    if name.startswith("vortex"):
        exact = W.cell_average(mesh, W.isentropic_vortex(t))
        tol = max(tol, 0.01 * relerr_var(uo, exact, axis_v=0))
    return tol


def flux_scale(mesh, u, cells, gamma=1.4):
    """Per-variable size of the face terms that the residual of a cell sums,
    max over the sampled cells of |physical flux of U_i| x perimeter / area.
    The terms cancel to a residual that can be far smaller (fine meshes,
    smooth flow), so round-off is bounded relative to this scale."""
    xy = mesh.xy[mesh.tri[cells]]
    e = np.roll(xy, -1, axis=1) - xy
    perim = np.hypot(e[..., 0], e[..., 1]).sum(1)
    area = W.cell_areas(mesh)[cells]
    rho, mx, my, E = u[:, cells]
    uu, vv = mx / rho, my / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (uu * uu + vv * vv))
    Fx = np.stack([mx, mx * uu + p, mx * vv, uu * (E + p)])
    Fy = np.stack([my, my * uu, my * vv + p, vv * (E + p)])
    return (np.maximum(np.abs(Fx), np.abs(Fy)) * (perim / area)[None]).max(1)


_cache = {}
_large = {}


@pytest.fixture(scope="module")
def ctx():
    c = T.Context(0)
    yield c
    _cache.clear()
    _large.clear()
    c.close()


def take(t, cells, dim=0):
    """Sampled cells of a device tensor, gathered on the device."""
    idx = torch.from_numpy(np.asarray(cells, np.int64)).to(t.device)
    return t.index_select(dim, idx).cpu().numpy()


LARGE_KW = dict(physics=O.EULER, scheme=O.CTENOZ, degree=3, lambda1_prime=1e4)


def large_case(ctx):
    """The 8M-cell vortex of the throughput benchmark (2000 x 2000 squares,
    seed 5, 3 x 3 collapsed-Gauss cell averages), both precisions resident."""
    if "m" not in _large:
        mesh, u0 = W.vortex_case(2000, seed=5, quad=3)
        _large.update(mesh=mesh, u0=u0, m=T.Mesh.from_workload(ctx, mesh, precision=T.BOTH, **LARGE_KW))
    return _large


def setup_case(ctx, name, precision=T.BOTH):
    key = (name, precision)
    if key not in _cache:
        make, kw = CASES[name]
        mesh, u0 = make()
        o = O.Oracle.from_mesh(mesh, **kw)
        m = T.Mesh.from_workload(ctx, mesh, precision=precision, **kw)
        _cache[key] = (mesh, u0, o, m)
    return _cache[key]


@pytest.mark.parametrize("name", list(CASES))
def test_stencils_and_pinv(ctx, name):
    mesh, u0, o, m = setup_case(ctx, name)
    oc, od, on = o.stencils()
    lc, ld, ln = m.stencils()
    assert np.array_equal(np.sort(oc, 1), lc)
    assert np.array_equal(on, ln)
    cells = np.arange(0, mesh.n_cells, max(1, mesh.n_cells // 97)).astype(np.int32)
    opc, opd = o.pinv(cells)
    gpc, gpd = m.pinv(cells, T.FP64)
    # oracle columns follow its central list; the library's follow the sorted list
    order = np.argsort(oc[cells], axis=1)
    opc_sorted = np.take_along_axis(opc, order[:, None, :], axis=2)
    for a in range(len(cells)):
        # Householder QR is backward stable: the forward error of the
        # pseudo-inverse grows with the condition number of the system, which
        # reaches 1e6 for the degree-6 monomial basis
        tol = max(1e-12, 50 * EPS64 * np.linalg.cond(o.ls_matrix(cells[a])[0]))
        assert relerr(gpc[a], opc_sorted[a]) < tol, (a, tol)
        if np.abs(opd[a]).max() > 0:
            assert relerr(gpd[a], opd[a]) < tol, (a, tol)
        else:
            assert np.abs(gpd[a]).max() == 0
    fpc, fpd = m.pinv(cells, T.MIXED)
    assert relerr(fpc, gpc) < 1e-6 and relerr(fpd, gpd) < 1e-6


@pytest.mark.parametrize("name", list(CASES))
def test_reconstruct_fp64(ctx, name):
    mesh, u0, o, m = setup_case(ctx, name)
    s = T.Solution(m, u0)
    fv, dl = s.reconstruct(T.FP64)
    ofv, odl = o.reconstruct(u0)
    assert np.array_equal(dl.cpu().numpy(), odl), "TENO selections differ"
    assert relerr_var(fv.cpu().numpy(), ofv) < 1e-12
    # forced selections reproduce the same values
    fv2, _ = s.reconstruct(T.FP64, forced=odl)
    assert relerr_var(fv2.cpu().numpy(), ofv) < 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_reconstruct_mixed(ctx, name):
    mesh, u0, o, m = setup_case(ctx, name)
    s = T.Solution(m, u0)
    ofv, odl = o.reconstruct(u0)
    fv, _ = s.reconstruct(T.MIXED, forced=odl)
    assert relerr_var(fv.cpu().numpy(), ofv) < 5e-6
    fv_free, dl = s.reconstruct(T.MIXED)
    # the FP64 selections equal the oracle's (test_reconstruct_fp64), so the
    # FP32-vs-oracle differences are exactly the library's flip count
    flips = int((dl.cpu().numpy() != odl).sum())
    assert flips == s.count_flips()
    same = (dl.cpu().numpy() == odl).reshape(mesh.n_cells, -1).all(axis=1)
    assert relerr_var(fv_free.cpu().numpy()[same], ofv[same]) < 5e-6


@pytest.mark.parametrize("name", list(CASES))
def test_flux_and_residual_fp64(ctx, name):
    mesh, u0, o, m = setup_case(ctx, name)
    ofv, _ = o.reconstruct(u0)
    ofo = o.face_fluxes(ofv)
    gfo = T.flux(m, torch.as_tensor(ofv).cuda(), T.FP64)
    assert relerr_var(gfo.cpu().numpy(), ofo) < 1e-12
    s = T.Solution(m, u0)
    R = s.residual(T.FP64).cpu().numpy()
    oR = o.residual(u0)
    assert relerr_var(R, oR, axis_v=0) < 1e-12


def term_scale(mesh, o, fv, gamma=1.4):
    """Per cell, face and variable, the size of the terms an HLLC / upwind
    flux of the face-point values fv [N][3][Nq][nv] sums: |A| max over the
    Gauss points of (|F_x(U)| + |F_y(U)| + (|v| + c) |U|) for Euler,
    |A| |a| |U| for advection.  FP32 rounding of the inputs and of the
    arithmetic is bounded by a small multiple of eps_32 times this size."""
    g = o.geometry()
    length = g["length"]                                   # [N][3]
    if o.nv == 1:
        t = np.abs(fv[..., 0]).max(2) * np.hypot(1.0, 1.0)
        return (t * length)[..., None]
    rho, mx, my, E = (fv[..., k] for k in range(4))
    u, v = mx / rho, my / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    c = np.sqrt(np.abs(gamma * p / rho))
    sp = np.hypot(u, v) + c
    Fx = np.stack([mx, mx * u + p, mx * v, u * (E + p)], -1)
    Fy = np.stack([my, my * u, my * v + p, v * (E + p)], -1)
    t = np.abs(Fx) + np.abs(Fy) + sp[..., None] * np.abs(fv)
    return t.max(2) * length[..., None]                    # [N][3][nv]


EPS32 = float(np.finfo(np.float32).eps)


@pytest.mark.parametrize("name", list(CASES))
def test_flux_and_residual_mixed(ctx, name):
    """Level 1 in mixed precision against the oracle, element by element.
    Fluxes from the oracle's face values (rounded to FP32 on the way in):
    |F_gpu - F_oracle| <= 50 eps_32 x the size of the flux's terms on both
    sides of the face.  Residuals from the FP32 reconstruction: where a cell
    and its face neighbours select as the oracle does, |R_gpu - R_oracle|
    <= 50 eps_32 x the sum of its face terms / |V|, plus what the 5e-6
    face-value bound of the FP32 reconstruction propagates into them."""
    mesh, u0, o, m = setup_case(ctx, name)
    ofv, odl = o.reconstruct(u0)
    ofo = o.face_fluxes(ofv)
    gfo = T.flux(m, torch.as_tensor(ofv.astype(np.float32)).cuda(), T.MIXED).cpu().numpy()
    own = term_scale(mesh, o, ofv)
    nb = o.geometry()["nbr"]
    nf = o.geometry()["nbr_face"]
    other = np.where((nb >= 0)[..., None], own[np.maximum(nb, 0), np.maximum(nf, 0)], own)
    scale = np.maximum(own, other)
    err = np.abs(gfo - ofo)
    ratio = float((err / (EPS32 * scale.max(axis=(0, 1)))).max())
    assert ratio <= 50, ratio
    s = T.Solution(m, u0)
    R = s.residual(T.MIXED).cpu().numpy().T                # [N][nv]
    oR = o.residual(u0).T
    _, dl = s.reconstruct(T.MIXED)
    agree = (dl.cpu().numpy() == odl).reshape(mesh.n_cells, -1).all(1)
    ok = agree & np.where(nb >= 0, agree[np.maximum(nb, 0)], True).all(1)
    area = W.cell_areas(mesh)
    rscale = (scale.sum(1) / area[:, None])[ok].max(0)
    # face values within 5e-6 of the oracle's (normwise per variable) move a
    # flux by at most about that fraction of its terms
    rtol = (50 * EPS32 + 2 * 5e-6) * rscale
    rerr = np.abs(R - oR)[ok].max(0)
    assert np.all(rerr <= rtol), (rerr, rtol)
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_rk_stages_fp64(ctx, name):
    mesh, u0, o, m = setup_case(ctx, name)
    dt = 0.3 * o.dt_bound(u0)
    s = T.Solution(m, u0)
    for st in range(3):
        s.rk_stage(st, dt, T.FP64)
    ug, t = s.download()
    uo = o.rk3_step(u0, dt)
    assert abs(t - dt) < 1e-15
    assert relerr_var(ug, uo, axis_v=0) < 1e-12


@pytest.mark.parametrize("name", ["advection_r2_cteno", "vortex_r3_ctenoz", "sod_r3_cteno", "sod_r4_cteno",
                                  "vortex_r6_ctenoz", "sod_r3_teno", "sod_r4_cweno", "sod_r3_cteno_char",
                                  "sod_r4_ctenoz_char", "shockdensity_r4_cteno", "dmr_r4_ctenoz",
                                  "dmr_r3_cteno_char"])
def test_solve_fp64_matches_oracle(ctx, name):
    mesh, u0, o, m = setup_case(ctx, name)
    s = T.Solution(m, u0)
    if name.startswith("advection"):
        steps = s.solve(t_final=0.1, cfl=0.3, precision=T.FP64)       # the full advection run
        uo, so, to = o.solve(u0, 0.1, cfl=0.3)
    else:
        steps = s.solve(t_final=10.0, max_steps=12, cfl=0.3, precision=T.FP64)
        uo, so, to = o.solve(u0, 10.0, cfl=0.3, max_steps=12)
    ug, tg = s.download()
    assert steps == so
    assert abs(tg - to) <= 1e-12 * max(1.0, abs(to))
    assert relerr_var(ug, uo, axis_v=0) < 1e-12


@pytest.mark.parametrize("name", ["dmr_r4_ctenoz", "dmr_r3_cteno_char"])
def test_inflow_states_follow_the_time(ctx, name):
    """The top side's prescribed state moves with the incident shock: every
    entry point evaluates it at its own time (flux: the time passed in;
    residual: the solution's; RK stages and marches: t, t + dt, t + dt/2)."""
    mesh, u0, o, m = setup_case(ctx, name)
    t0 = 0.05
    u, _, _ = o.solve(u0, t0, cfl=0.3)
    ofv, _ = o.reconstruct(u)
    for t in (t0, 0.12):
        gfo = T.flux(m, torch.as_tensor(ofv).cuda(), T.FP64, t=t)
        assert relerr_var(gfo.cpu().numpy(), o.face_fluxes(ofv, t)) < 1e-12
    # the state on the top side differs between the two times
    assert np.abs(o.face_fluxes(ofv, t0) - o.face_fluxes(ofv, 0.12)).max() > 1.0
    s = T.Solution(m, u, t0)
    assert relerr_var(s.residual(T.FP64).cpu().numpy(), o.residual(u, t0), axis_v=0) < 1e-12
    dt = 0.3 * o.dt_bound(u)
    for st in range(3):
        s.rk_stage(st, dt, T.FP64)
    ug, tg = s.download()
    assert abs(tg - (t0 + dt)) < 1e-15
    assert relerr_var(ug, o.rk3_step(u, dt, t0), axis_v=0) < 1e-12
    uo, so, to = o.solve(u, 10.0, cfl=0.3, t0=t0, max_steps=10)
    for graph in (True, False):
        s.set(u, t0)
        n = s.solve(t_final=10.0, max_steps=10, cfl=0.3, precision=T.FP64, use_graph=graph)
        ug, tg = s.download()
        assert n == so and abs(tg - to) <= 1e-12
        assert relerr_var(ug, uo, axis_v=0) < 1e-12
    s.set(u, t0)
    s.solve(t_final=10.0, max_steps=10, cfl=0.3, precision=T.MIXED)
    assert relerr_var(s.download()[0], uo, axis_v=0) < 1e-5
    s.close()


def test_graph_replay_equals_direct_launch(ctx):
    mesh, u0, o, m = setup_case(ctx, "vortex_r3_ctenoz")
    a = T.Solution(m, u0)
    b = T.Solution(m, u0)
    for prec in (T.FP64, T.MIXED):
        a.set(u0)
        b.set(u0)
        na = a.solve(t_final=10.0, max_steps=7, precision=prec, use_graph=True)
        nb = b.solve(t_final=10.0, max_steps=7, precision=prec, use_graph=False)
        ua, ta = a.download()
        ub, tb = b.download()
        assert na == nb == 7 and ta == tb
        assert np.array_equal(ua, ub)
        # a second graph solve continues from the same state the same way
        a.solve(t_final=10.0, max_steps=3, precision=prec, use_graph=True)
        b.solve(t_final=10.0, max_steps=3, precision=prec, use_graph=False)
        assert np.array_equal(a.download()[0], b.download()[0])


@pytest.mark.parametrize("graph", [False, True])
def test_degenerate_marches(ctx, graph):
    """A march with no step budget, or one that starts at or past its final
    time, takes no step and leaves state and time bitwise unchanged; a march
    to a final time just ahead takes one step, clipped to land on it."""
    mesh, u0, o, m = setup_case(ctx, "vortex_r3_ctenoz")
    t0 = 0.25
    for prec in (T.FP64, T.MIXED):
        s = T.Solution(m, u0, t0)
        for kw in (dict(t_final=10.0, max_steps=0), dict(t_final=t0), dict(t_final=0.1)):
            assert s.solve(precision=prec, use_graph=graph, **kw) == 0
            u, t = s.download()
            assert t == t0 and np.array_equal(u, u0)
        assert s.solve(t_final=t0 + 1e-9, precision=prec, use_graph=graph) == 1
        u, t = s.download()
        assert t == t0 + 1e-9 and not np.array_equal(u, u0)
        assert np.abs(u - u0).max() <= 1e-6 * np.abs(u0).max()
        s.close()


@pytest.mark.parametrize("prec", [T.FP64, T.MIXED])
def test_conservation_on_gpu(ctx, prec):
    mesh, u0, o, m = setup_case(ctx, "vortex_r3_ctenoz")
    area = W.cell_areas(mesh)
    s = T.Solution(m, u0)
    s.solve(t_final=10.0, max_steps=25, precision=prec)
    u, _ = s.download()
    tot0 = (u0 * area).sum(1)
    tot1 = (u * area).sum(1)
    assert np.abs(tot1 - tot0).max() <= 2e-13 * np.abs(tot0).max()


def test_freestream_on_gpu(ctx):
    mesh = W.split_jitter_mesh(16, 16, seed=9)
    kw = dict(physics=O.EULER, scheme=O.CTENOZ, degree=3, lambda1_prime=1e4)
    m = T.Mesh.from_workload(ctx, mesh, precision=T.BOTH, **kw)
    U = np.tile(np.array([1.3, 0.4, -0.7, 2.9])[:, None], (1, mesh.n_cells))
    s = T.Solution(m, U)
    r64 = s.residual(T.FP64).cpu().numpy()
    r32 = s.residual(T.MIXED).cpu().numpy()
    h = 1.0 / 16
    assert np.abs(r64).max() <= 1e-13 * 3.0 / h
    assert np.abs(r32).max() <= 1e-5 * 3.0 / h


def test_mixed_vs_fp64_solution(ctx):
    mesh, u0, o, m = setup_case(ctx, "vortex_r3_ctenoz")
    a = T.Solution(m, u0)
    b = T.Solution(m, u0)
    a.solve(t_final=10.0, max_steps=20, precision=T.FP64)
    b.solve(t_final=10.0, max_steps=20, precision=T.MIXED)
    ua, _ = a.download()
    ub, _ = b.download()
    assert relerr_var(ub, ua, axis_v=0) < 1e-5


def test_nonphysical_state_is_reported(ctx):
    mesh, u0, o, m = setup_case(ctx, "vortex_r3_ctenoz")
    bad = u0.copy()
    bad[3, 5] = -1.0          # negative total energy -> negative pressure
    s = T.Solution(m, bad)
    with pytest.raises(T.CtenoError) as e:
        s.solve(t_final=10.0, max_steps=3, precision=T.FP64)
    assert e.value.status == T.ERR_NONPHYSICAL


@pytest.mark.parametrize("case,degree", [("vortex", 3), ("sod", 3), ("sod", 4), ("vortex", 5), ("vortex", 6)])
def test_mesh_counts_match_the_oracle(ctx, case, degree):
    """The mesh handle's counts against the oracle's geometry and stencils:
    faces and boundary faces, inadmissible interior faces (directional
    stencil with fewer than K_d + 1 cells), slots per cell (max(M, 3 M_d) up
    to cubic and at degree 6, M at degrees 4 and 5) and, in the caller's
    cell order, the cells with a face to another 256-cell block."""
    if case == "vortex":
        mesh, _ = W.vortex_case(24, seed=2)
    else:
        mesh, _ = W.sod_case(48, 12, seed=3)
    m = T.Mesh.from_workload(ctx, mesh, physics=O.EULER, scheme=O.CTENO, degree=degree, precision=T.BOTH,
                             reorder=0)
    o = O.Oracle.from_mesh(mesh, physics=O.EULER, scheme=O.CTENO, degree=degree)
    nb = o.geometry()["nbr"]
    _, _, cnt = o.stencils()
    info = m.info
    N = mesh.n_cells
    assert info.n_cells == N
    assert info.n_boundary_faces == int((nb < 0).sum())
    assert info.n_faces == int((nb >= 0).sum()) // 2 + int((nb < 0).sum())
    assert info.n_inadmissible == int(((nb >= 0) & (cnt == 0)).sum())
    K = (degree + 1) * (degree + 2) // 2 - 1
    kd = (degree + 1) // 2 if degree >= 4 else 1
    Md = 2 * ((kd + 1) * (kd + 2) // 2 - 1)
    assert info.slots == (2 * K if degree in (4, 5) else max(2 * K, 3 * Md))
    cells = np.arange(N)[:, None]
    cross = ((nb >= 0) & (nb // 256 != cells // 256)).any(axis=1)
    assert info.n_cross_cells == (int(cross.sum()) if degree <= 3 else 0)
    m.close()


@pytest.mark.parametrize("which", ["vortex_80k", "sod_1p28M", "vortex_8M", "vortex_2M_r4", "vortex_2M_r5",
                                   "vortex_2M_r6", "dmr_715k_r4"])
def test_full_size_sampled_parity(ctx, which):
    """Full configured sizes, one reconstruction and residual in the launch
    configuration of the time march; the oracle evaluates sampled cells.
    Besides the configured cases: the 2M-cell vortex of the orders 5-7
    measurement and the double Mach reflection on the larger timing mesh."""
    rng = np.random.default_rng(0)
    if which == "vortex_8M":
        L = large_case(ctx)
        mesh, u0, m, kw = L["mesh"], L["u0"], L["m"], LARGE_KW
    else:
        if which == "vortex_80k":
            mesh, u0 = W.vortex_case(200, seed=2)
            kw = dict(physics=O.EULER, scheme=O.CTENOZ, degree=3, lambda1_prime=1e4)
        elif which.startswith("vortex_2M"):
            mesh, u0 = W.vortex_case(1000, seed=5, quad=3)
            kw = dict(physics=O.EULER, scheme=O.CTENOZ, degree=int(which[-1]), lambda1_prime=1e4)
        elif which == "dmr_715k_r4":
            mesh, u0 = W.dmr_case(1196, 299)
            kw = dict(physics=O.EULER, scheme=O.CTENO, degree=4, lambda1_prime=1e15, positivity=1)
        else:
            mesh, u0 = W.sod_case(1600, 400, seed=3, prescribed=True)
            kw = dict(physics=O.EULER, scheme=O.CTENO, degree=3, lambda1_prime=1e15, positivity=1)
        m = T.Mesh.from_workload(ctx, mesh, precision=T.BOTH, **kw)
    o = O.Oracle.from_mesh(mesh, **kw)
    cells = np.sort(rng.choice(mesh.n_cells, 300, replace=False)).astype(np.int32)
    if which == "sod_1p28M":   # also sample the discontinuity
        cx = mesh.xy[mesh.tri].mean(1)[:, 0]
        near = np.where(np.abs(cx - 0.5) < 2.0 / 1600)[0]
        cells = np.unique(np.concatenate([cells, rng.choice(near, 200, replace=False)])).astype(np.int32)
    if which.startswith("vortex_8M") or which.startswith("vortex_2M"):
        # also sample the vortex core, where the selection varies most
        cx = mesh.xy[mesh.tri].mean(1)
        near = np.where(np.hypot(cx[:, 0] - 5.0, cx[:, 1] - 5.0) < 1.5)[0]
        cells = np.unique(np.concatenate([cells, rng.choice(near, 200, replace=False)])).astype(np.int32)
    if which == "dmr_715k_r4":  # also sample the incident shock and the prescribed sides
        c = mesh.xy[mesh.tri].mean(1)
        shock = np.where(np.abs(c[:, 0] - W.DMR_LINE[0] - W.DMR_LINE[1] * c[:, 1]) < 2.0 / 299)[0]
        side = np.where((c[:, 0] < 1.0 / 299) | (c[:, 0] > 4.0 - 1.0 / 299) | (c[:, 1] > 1.0 - 1.0 / 299))[0]
        cells = np.unique(np.concatenate([cells, rng.choice(shock, 200, replace=False),
                                          rng.choice(side, 100, replace=False)])).astype(np.int32)
    s = T.Solution(m, u0)
    fv, dl = s.reconstruct(T.FP64)
    ofv, odl = o.reconstruct_cells(u0, cells)
    dls = take(dl, cells)
    assert np.array_equal(dls, odl)
    assert relerr_var(take(fv, cells), ofv) < 1e-12
    R = take(s.residual(T.FP64), cells, dim=1).T
    oR = o.residual_cells(u0, cells)
    # 1e-12 of the residual, or FP64 round-off of its face terms (the same
    # form as the mixed-precision residual bound, with the FP64 epsilon)
    err = np.abs(R - oR).max(0)
    tol = np.maximum(1e-12 * np.abs(oR).max(0), 50 * EPS64 * flux_scale(mesh, u0, cells))
    assert np.all(err <= tol), (err, tol)
    fv32, _ = s.reconstruct(T.MIXED, forced=dl.cpu().numpy())
    assert relerr_var(take(fv32, cells), ofv) < 5e-6
    s.close()


def test_large_march_conservation_and_precision(ctx):
    """The benchmark's 8M-cell configuration in its timed launch path (direct
    launches, kernel timing on): 3 SSP-RK3 steps in each precision.  Mass,
    momentum and energy are conserved to FP64 round-off, and the mixed state
    is within 1e-5 (normwise per variable) of the FP64 state."""
    L = large_case(ctx)
    area = W.cell_areas(L["mesh"])
    tot0 = (L["u0"] * area).sum(1)
    out = {}
    for prec in (T.FP64, T.MIXED):
        s = T.Solution(L["m"], L["u0"])
        ctx.set_timing(True)
        n = s.solve(max_steps=3, cfl=0.3, precision=prec, use_graph=False)
        ctx.set_timing(False)
        u, _ = s.download()
        s.close()
        assert n == 3
        tot1 = (u * area).sum(1)
        assert np.abs(tot1 - tot0).max() <= 1e-12 * np.abs(tot0).max()
        out[prec] = u
    assert relerr_var(out[T.MIXED], out[T.FP64], axis_v=0) < 1e-5


@pytest.mark.parametrize("prec", [T.FP64, T.MIXED])
def test_positivity_is_reported_without_the_fallback(ctx, prec):
    """The paper's scheme (positivity = 0): the 48 x 12 Sod start
    reconstructs a negative density in one cut cell.  The oracle raises a
    non-physical face state; the library reports CTENO_ERR_NONPHYSICAL from
    the flux, the residual, the march and (after stage calls) the next
    download -- and marches with the fallback on."""
    mesh, u0 = W.sod_case(48, 12, seed=3)
    kw = dict(physics=O.EULER, scheme=O.CTENO, degree=3, lambda1_prime=1e15)
    o = O.Oracle.from_mesh(mesh, **kw)
    with pytest.raises(O.OracleError):
        o.residual(u0)
    m = T.Mesh.from_workload(ctx, mesh, precision=T.BOTH, **kw)
    s = T.Solution(m, u0)
    ofv, odl = o.reconstruct(u0)          # no fallback: the non-physical values themselves
    fv, dl = s.reconstruct(prec)
    assert not (dl.cpu().numpy() & 0x80).any() and s.fallbacks() == 0
    if prec == T.FP64:
        assert np.array_equal(dl.cpu().numpy(), odl)
        assert relerr_var(fv.cpu().numpy(), ofv) < 1e-12
    dt_ = torch.float64 if prec == T.FP64 else torch.float32
    for call in (lambda: T.flux(m, torch.as_tensor(ofv).to(dt_).cuda(), prec),
                 lambda: s.residual(prec),
                 lambda: s.solve(t_final=10.0, max_steps=3, precision=prec)):
        with pytest.raises(T.CtenoError) as e:
            call()
        assert e.value.status == T.ERR_NONPHYSICAL
    s.set(u0, 0.0)
    dt = 0.3 * o.dt_bound(u0)
    s.rk_stage(0, dt, prec)
    with pytest.raises(T.CtenoError) as e:
        s.download()
    assert e.value.status == T.ERR_NONPHYSICAL
    s.download()                            # reported once
    s.close()
    mp = T.Mesh.from_workload(ctx, mesh, precision=T.BOTH, positivity=1, **kw)
    sp = T.Solution(mp, u0)
    assert sp.solve(t_final=10.0, max_steps=3, precision=prec) == 3
    assert sp.fallbacks() >= 1
    sp.close()


@pytest.mark.parametrize("name", ["sod_r3_cteno", "sod_r4_cteno", "dmr_r4_ctenoz", "dmr_r3_cteno_char",
                                  "shockdensity_r4_cteno"])
def test_fallback_counts_match_oracle(ctx, name):
    """With the fallback on, the library counts the cells (x stages) that
    take it; in FP64 over a 12-step march that is the oracle's count."""
    mesh, u0, _, m = setup_case(ctx, name)
    make, kw = CASES[name]
    o = O.Oracle.from_mesh(mesh, **kw)
    uo, so, _ = o.solve(u0, 10.0, cfl=0.3, max_steps=12)
    s = T.Solution(m, u0)
    assert s.solve(t_final=10.0, max_steps=12, cfl=0.3, precision=T.FP64) == so
    assert s.fallbacks() == o.fallbacks() > 0
    s.set(u0, 0.0)
    s.solve(t_final=10.0, max_steps=12, cfl=0.3, precision=T.MIXED)
    fb32 = s.fallbacks()
    assert abs(fb32 - o.fallbacks()) <= max(2, 0.05 * o.fallbacks()), (fb32, o.fallbacks())
    s.close()


def _chi_of(mesh, kw, cell, var, lo=1e-12, hi=0.2):
    """The oracle's chi of the centre stencil of (cell, var), found as the
    cut-off C_T at which its delta_1 bit turns off (bisection on a log
    scale: delta_1 = 1 iff chi_1 >= C_T).  C_T stays below 1/4 <= 1/s_t,
    so some stencil always passes the cut-off."""
    def bit(ct):
        o = O.Oracle.from_mesh(mesh, c_t=ct, **kw)
        _, d = o.reconstruct_cells(U_FLIP, np.array([cell], np.int32))
        return int(d[0, var] & 1)
    if bit(hi) == 1 or bit(lo) == 0:
        return None
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if bit(mid):
            lo = mid
        else:
            hi = mid
        if hi / lo - 1.0 < 1e-15:
            break
    return lo


U_FLIP = None


def test_flips_are_counted(ctx):
    """Flips exercised on purpose: for a few (cell, variable) pairs of an
    evolved Sod state (10 oracle steps with moving gas, so the centre
    stencil's chi spreads over many decades), C_T is set within FP32
    rounding of the oracle's FP64 chi of the centre stencil, so the FP32
    selection can fall on the other side.  Every library count equals the
    element-wise difference of the FP32 selections from the oracle's, and
    some are non-zero."""
    global U_FLIP
    mesh, u0 = W.sod_case(24, 6, seed=3, left=(1.0, 0.2, 0.1, 1.0), right=(0.125, 0.1, -0.05, 0.1))
    kw = dict(physics=O.EULER, scheme=O.CTENO, degree=3, lambda1_prime=1e15, positivity=1)
    U_FLIP, _, _ = O.Oracle.from_mesh(mesh, **kw).solve(u0, 10.0, cfl=0.3, max_steps=10)
    # (cell, variable) pairs whose centre chi lies between 1e-9 and 0.2
    _, dlo = O.Oracle.from_mesh(mesh, c_t=1e-9, **kw).reconstruct(U_FLIP)
    _, dhi = O.Oracle.from_mesh(mesh, c_t=0.2, **kw).reconstruct(U_FLIP)
    cand = np.argwhere((dlo & 1).astype(bool) & ~(dhi & 1).astype(bool))
    assert len(cand) >= 4
    total = 0
    for i, var in cand[:: max(1, len(cand) // 4)][:4]:
        chi = _chi_of(mesh, kw, int(i), int(var), lo=1e-9)
        assert chi is not None
        # offsets of half a step from chi itself, where the FP64 selections
        # of library and oracle (different rounding orders) could differ
        for k in range(-6, 6):
            ct = chi * (1.0 + (k + 0.5) * 1.5e-7)
            _, od = O.Oracle.from_mesh(mesh, c_t=ct, **kw).reconstruct(U_FLIP)
            mk = T.Mesh.from_workload(ctx, mesh, precision=T.BOTH, c_t=ct, **kw)
            sk = T.Solution(mk, U_FLIP)
            _, d64 = sk.reconstruct(T.FP64)
            assert np.array_equal(d64.cpu().numpy(), od)
            _, d32 = sk.reconstruct(T.MIXED)
            diff = int((d32.cpu().numpy() != od).sum())
            assert diff == sk.count_flips()
            total += diff
            sk.close()
            mk.close()
    assert total > 0


@pytest.mark.parametrize("nx,ny", [(10, 10), (8, 16), (6, 22)])
def test_fused_stage_at_block_edges(ctx, nx, ny):
    """Meshes of 200, 256 and 264 cells: one partial 256-cell block, one
    full block (no cell has a face to another block, so the second fused
    kernel has nothing to do), and a second block of 8 cells.  The fused
    FP64 march equals the separate kernels' and the oracle's to 1e-12."""
    mesh = W.split_jitter_mesh(nx, ny, (0.0, 10.0, 0.0, 10.0), seed=9)
    u0 = W.cell_average(mesh, W.isentropic_vortex(0.0, 5.0, (5.0, 5.0), (10.0, 10.0)), n=4)
    N = mesh.n_cells
    kw = dict(physics=O.EULER, scheme=O.CTENOZ, degree=3, lambda1_prime=1e4)
    m = T.Mesh.from_workload(ctx, mesh, precision=T.BOTH, **kw)
    assert (m.info.n_cross_cells == 0) == (N <= 256)
    o = O.Oracle.from_mesh(mesh, **kw)
    steps = 6
    uo, so, _ = o.solve(u0, 10.0, cfl=0.3, max_steps=steps)
    out = {}
    for fused in (True, False):
        ctx.set_fused_stage(fused)
        try:
            s = T.Solution(m, u0)
            assert s.solve(t_final=10.0, max_steps=steps, cfl=0.3, precision=T.FP64) == so
            out[fused], _ = s.download()
            s.close()
        finally:
            ctx.set_fused_stage(True)
    assert relerr_var(out[True], out[False], axis_v=0) < 1e-12
    assert relerr_var(out[True], uo, axis_v=0) < 1e-12
    m.close()


@pytest.mark.parametrize("name", ["advection_r2_cteno", "vortex_r3_ctenoz", "density_r2_ctenoz", "dmr_r3_cteno_char",
                                  "vortex_r3_ctenoz_scaled"])
def test_fused_stage_matches_split_kernels(ctx, name):
    """Marches of degree <= 3 run the fused stage kernels by default.
    Against the separate reconstruction and flux kernels: the first stage is
    the same to FP64 rounding (the fused kernels sum a cell's in-block faces
    first, and evaluate a face inside a block once, its other cell taking
    the exact negation).  In FP64 the 12-step marches agree with each other
    and with the oracle to 1e-12.  In mixed precision the FP64 rounding
    differences of the state enter the FP32 reconstruction, so the marches
    agree to the mixed-precision tolerance, and each agrees with the oracle
    to it: 1e-5 normwise per variable, or 1% of the oracle's own error
    against the exact solution where that is larger (the scaled CTENOZ
    reading switches stencils at many smooth cells, so FP32 and FP64 take
    different stencils at some of them)."""
    mesh, u0, o, m = setup_case(ctx, name)
    steps = 12
    uo, so, to = o.solve(u0, 10.0, cfl=0.3, max_steps=steps)
    dt = 0.3 * o.dt_bound(u0)
    for prec in (T.FP64, T.MIXED):
        out, stage0 = {}, {}
        for fused in (True, False):
            ctx.set_fused_stage(fused)
            try:
                s = T.Solution(m, u0)
                s.rk_stage(0, dt, prec)
                stage0[fused] = s.download()[0]
                s.set(u0, 0.0)
                assert s.solve(t_final=10.0, max_steps=steps, cfl=0.3, precision=prec) == so
                out[fused], _ = s.download()
                s.close()
            finally:
                ctx.set_fused_stage(True)
        assert relerr_var(stage0[True], stage0[False], axis_v=0) < 1e-13
        tol = 1e-12 if prec == T.FP64 else mixed_tolerance(name, mesh, uo, to)
        assert relerr_var(out[True], out[False], axis_v=0) < tol
        for fused in (True, False):
            assert relerr_var(out[fused], uo, axis_v=0) < tol
