"""The paper's Euler density-wave order study (sec. 3.1.1, Tables 2 and 3)
run on the GPU through the C ABI, orders 3 to 7.

rho = 1 + 0.2 sin(2 pi (x + y)), u = v = p = 1 on the periodic unit square,
our jittered split meshes (2 n^2 cells, not the paper's meshes: orders are
compared, not errors), FP64, lambda1' = 1e15 (Table 3, where CTENO and
CTENOZ coincide and reach design order at every degree).  The time step
scales like h^((r+1)/3) so the third-order time error stays below the
spatial error."""
import math
import os

import numpy as np
import pytest

from paper_2312_17042_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_17042_amd import cteno as T  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_orders.txt")


def _table3():
    rows = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, lam, order, err, first = line.split()
            if float(lam) == 1e15:
                rows[int(name[-1]) - 1] = float(order)    # degree r = order - 1
    return rows


@pytest.fixture(scope="module")
def ctx():
    c = T.Context(0)
    yield c
    c.close()


def density_wave_errors(ctx, r, ns, t_end=0.1, precision=T.FP64):
    errs = []
    for n in ns:
        mesh, u0 = W.density_wave_case(n, seed=11)
        m = T.Mesh.from_workload(ctx, mesh, physics=T.EULER, scheme=T.CTENOZ, degree=r, lambda1_prime=1e15,
                                 precision=T.BOTH)
        s = T.Solution(m, u0)
        cfl = 0.3 * (10.0 / n) ** ((r + 1) / 3.0 - 1.0)
        s.solve(t_final=t_end, cfl=cfl, precision=precision)
        u, t = s.download()
        assert abs(t - t_end) < 1e-12
        ue = W.cell_average(mesh, W.density_wave(t_end))
        errs.append(math.sqrt(((u[0] - ue[0]) ** 2 * W.cell_areas(mesh)).sum()))
        s.close()
        m.close()
    return errs


@pytest.mark.parametrize("r", [2, 3, 4, 5, 6])
def test_density_wave_design_order(ctx, r):
    errs = density_wave_errors(ctx, r, (10, 20, 40, 80))
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    print(f"r={r} L2 errors {['%.3e' % e for e in errs]} orders {['%.2f' % o for o in orders]}")
    assert orders[-1] >= _table3()[r] - 0.3, (orders, _table3()[r])
