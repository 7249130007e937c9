"""The boundary's ownership rules on the GPU: device memory of the library's
handles goes through the caller's allocator (torch's caching allocator in
the Python binding) and comes back on destroy; a process that exits with
live handles (contexts, meshes, solutions, a server with work queued) ends
cleanly."""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

from paper_2312_17042_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2312_17042_amd import cteno as T  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_handles_allocate_through_torch():
    """memory_allocated rises by the mesh's resident bytes on upload (each
    block rounded up to torch's 512-byte granule) and returns after
    destroy; a solution's state and work buffers likewise."""
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated(0)
    ctx = T.Context(0)
    assert ctx.allocator is not None
    mesh, u0 = W.vortex_case(40, seed=2)
    m = T.Mesh.from_workload(ctx, mesh, precision=T.BOTH, physics=T.EULER, scheme=T.CTENOZ, degree=3,
                             lambda1_prime=1e4)
    torch.cuda.synchronize()
    grown = torch.cuda.memory_allocated(0) - base
    dev = int(m.info.device_bytes)
    assert dev <= grown <= dev + 512 * ctx.allocator.allocs, (grown, dev)
    s = T.Solution(m, u0)
    s.solve(t_final=10.0, max_steps=2, precision=T.MIXED)
    assert torch.cuda.memory_allocated(0) > base + dev
    s.close()
    m.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) == base
    ctx.close()
    assert ctx.allocator.allocs == ctx.allocator.frees > 0


def test_hipmalloc_context_still_works():
    ctx = T.Context(0, allocator=None)
    mesh, u0 = W.vortex_case(12, seed=2)
    base = torch.cuda.memory_allocated(0)
    m = T.Mesh.from_workload(ctx, mesh, precision=T.FP64, physics=T.EULER, scheme=T.CTENOZ, degree=3)
    assert torch.cuda.memory_allocated(0) == base
    s = T.Solution(m, u0)
    assert s.solve(t_final=10.0, max_steps=2) == 2
    ctx.close()


def test_exit_with_live_handles_is_clean():
    """A child process leaves a context, a mesh, a solution mid-use and a
    server with queued work to interpreter exit: the binding closes them
    children-first before the runtime goes, and the process exits 0 with
    no finaliser error."""
    code = textwrap.dedent(f"""
        import sys
        sys.path.insert(0, {ROOT!r})
        from paper_2312_17042_amd import cteno as T, workloads as W
        ctx = T.Context(0)
        mesh, u0 = W.vortex_case(16, seed=2)
        m = T.Mesh.from_workload(ctx, mesh, precision=T.BOTH, physics=T.EULER, scheme=T.CTENOZ, degree=3)
        s = T.Solution(m, u0)
        s.solve(t_final=10.0, max_steps=2)
        srv = T.Server(ctx, T.make_scheme(degree=3, precision=T.MIXED), budget_bytes=1 << 28, max_slots=4)
        for k in range(3):
            srv.submit(mesh, u0, 50)
        keep = [ctx, m, s, srv]          # module globals still alive at exit
        print("child ready", flush=True)
    """)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    assert "child ready" in r.stdout
    # and no finaliser raised on the way out
    assert "Traceback" not in r.stderr and "Exception ignored" not in r.stderr, r.stderr[-2000:]
