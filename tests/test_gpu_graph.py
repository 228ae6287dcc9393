"""The hot path captured in a HIP graph (assemble, Dirichlet, evaluate on one
stream; the fused step; the general assembly and evaluation of non-affine Q1
meshes): every replay, with the program's own eager work and
synchronisations in between, gives the eager results bit for bit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2505_02438_amd import api
from paper_2505_02438_amd import inputs as I

from gpu_util import dev, host

pytestmark = pytest.mark.gpu
MAT = api.Material()


@pytest.mark.parametrize("elem", [I.QUAD4, I.HEX8, I.TET10])
def test_graph_replays_equal_eager(elem):
    pr = I.small_problem(elem, seed=41, dims=(30, 20) if elem == I.QUAD4 else None)
    m = pr.mesh
    pat = api.Pattern.from_mesh(m)
    st = torch.cuda.Stream()
    rho, u, mask = dev(pr.rho), dev(pr.u), dev(pr.mask)
    K = torch.empty(pat.nnz, dtype=torch.float64, device="cuda")
    dc = torch.empty(m.n_cells, dtype=torch.float64, device="cuda")
    c = torch.zeros(2, dtype=torch.float64, device="cuda")

    def step():
        pat.assemble(MAT, rho, None, out=K, stream=st)
        pat.apply_dirichlet(mask, K, stream=st)
        pat.evaluate(MAT, rho, u, dc=dc, c=c, stream=st)

    with torch.cuda.stream(st):
        step()  # warm-up on the capture stream: workspace and launch attributes set
    torch.cuda.synchronize()
    ref = (host(K).copy(), host(dc).copy(), host(c).copy())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        step()
    for rep in range(4):
        K.fill_(np.nan)
        dc.fill_(np.nan)
        c.fill_(np.nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(K), ref[0]) and np.array_equal(host(dc), ref[1]), rep
        assert np.array_equal(host(c), ref[2]), rep
        _ = (rho * 2).sum().item()  # eager work between replays


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("elem,renumber", [(I.QUAD4, False), (I.TRI3, False), (I.HEX8, False), (I.TET10, False),
                                           (I.HEX8, True)])
def test_graph_replays_of_the_fused_step(elem, renumber, variant):
    """soptx_step (the bound Dirichlet table; for a renumbered mesh the rank
    tables and the densities read through the rank map) captured in a HIP graph: every replay,
    with eager work between replays, gives the eager results bit for bit,
    with either assembly kernel (forced through the debug hook)."""
    from paper_2505_02438_amd import _lib
    L = _lib.lib()
    assert L.soptx_debug_set_assembly_variant(variant) == 0
    try:
        _fused_step_graph(elem, renumber)
    finally:
        L.soptx_debug_set_assembly_variant(-1)


def _fused_step_graph(elem, renumber):
    pr = I.small_problem(elem, seed=43, dims=(30, 20) if elem == I.QUAD4 else None)
    if renumber:
        pr = I.renumber(pr, 44)
    m = pr.mesh
    pat = api.Pattern.from_mesh(m)
    if renumber:
        assert pat.stats()["n_groups_ranked"] > 0
    bc = api.Dirichlet(pat, pr.mask)
    st = torch.cuda.Stream()
    rho, u = dev(pr.rho), dev(pr.u)
    K = torch.empty(pat.nnz, dtype=torch.float64, device="cuda")
    dc = torch.empty(m.n_cells, dtype=torch.float64, device="cuda")
    c = torch.zeros(2, dtype=torch.float64, device="cuda")

    def step():
        pat.step(MAT, rho, u, bc=bc, K=K, dc=dc, c=c, stream=st)

    with torch.cuda.stream(st):
        step()  # warm-up on the capture stream: workspaces and launch attributes set
    torch.cuda.synchronize()
    ref = (host(K).copy(), host(dc).copy(), host(c).copy())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        step()
    for rep in range(4):
        K.fill_(np.nan)
        dc.fill_(np.nan)
        c.fill_(np.nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(K), ref[0]) and np.array_equal(host(dc), ref[1]), rep
        assert np.array_equal(host(c), ref[2]), rep
        _ = (rho * 2).sum().item()  # eager work between replays


def test_graph_replays_after_the_workspace_grew():
    """A fused step captured on a small mesh (its graph holds the stream's
    workspace address of the compliance partials); then a step on a larger
    mesh on the same stream, which needs a larger workspace; the earlier
    graph's replays still give its eager results bit for bit (the replaced
    workspace is kept, not freed)."""
    pr = I.renumber(I.small_problem(I.HEX8, seed=43, dims=(6, 5, 4)), 44)
    m = pr.mesh
    pat = api.Pattern.from_mesh(m)
    assert pat.stats()["n_groups_ranked"] > 0
    bc = api.Dirichlet(pat, pr.mask)
    st = torch.cuda.Stream()
    rho, u, f = dev(pr.rho), dev(pr.u), dev(pr.f)
    K = torch.empty(pat.nnz, dtype=torch.float64, device="cuda")
    dc = torch.empty(m.n_cells, dtype=torch.float64, device="cuda")
    c = torch.zeros(2, dtype=torch.float64, device="cuda")

    def step():
        pat.step(MAT, rho, u, f, bc=bc, K=K, dc=dc, c=c, stream=st)

    with torch.cuda.stream(st):
        step()
    torch.cuda.synchronize()
    ref = (host(K).copy(), host(dc).copy(), host(c).copy())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        step()
    # a larger mesh on the same stream: more than 2048 energy blocks, so the
    # partials need more than the workspace's first 4096 doubles
    m2 = I.hex_grid(100, 80, 70)
    assert (m2.n_cells + 255) // 256 > 2048
    pat2 = api.Pattern.from_mesh(m2)
    rng = np.random.default_rng(45)
    K2, dc2, c2 = pat2.step(MAT, dev(rng.uniform(0.1, 1.0, m2.n_cells)), dev(rng.standard_normal(pat2.ndof)),
                            dev(rng.standard_normal(pat2.ndof)), stream=st)
    torch.cuda.synchronize()
    assert np.isfinite(host(c2)).all()
    del K2, dc2, c2, pat2
    for rep in range(3):
        K.fill_(np.nan)
        dc.fill_(np.nan)
        c.fill_(np.nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(K), ref[0]) and np.array_equal(host(dc), ref[1]), rep
        assert np.array_equal(host(c), ref[2]), rep
        _ = (rho * 2).sum().item()  # eager work between replays


@pytest.mark.parametrize("elem", [I.QUAD4, I.HEX8])
def test_graph_replays_of_the_general_assembly(elem):
    """soptx_assemble_general on a jittered (non-affine) Q1 mesh, in its
    default form (in LDS on the plan's node groups), then the general
    evaluation, captured in a HIP graph: every replay, with eager work
    between replays, gives the eager results bit for bit."""
    rng = np.random.default_rng(42)
    m0 = I.quad_grid(30, 20) if elem == I.QUAD4 else I.hex_grid(12, 8, 6)
    m = I.jitter_interior(m0, 0.25, rng)
    pat = api.Pattern.from_mesh(m, general=True)
    st = torch.cuda.Stream()
    rho = dev(rng.uniform(0.01, 1.0, m.n_cells))
    u = dev(rng.standard_normal(m.ndof))
    mask = dev((rng.uniform(size=m.ndof) < 0.1).astype(np.uint8))
    K = torch.empty(pat.nnz, dtype=torch.float64, device="cuda")
    dc = torch.empty(m.n_cells, dtype=torch.float64, device="cuda")
    c = torch.zeros(2, dtype=torch.float64, device="cuda")

    def step():
        pat.assemble_general(MAT, rho, mask, out=K, stream=st)
        pat.evaluate_general(MAT, rho, u, dc=dc, c=c, stream=st)

    with torch.cuda.stream(st):
        step()  # warm-up on the capture stream: workspace and launch attributes set
    torch.cuda.synchronize()
    ref = (host(K).copy(), host(dc).copy(), host(c).copy())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        step()
    for rep in range(4):
        K.fill_(np.nan)
        dc.fill_(np.nan)
        c.fill_(np.nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(K), ref[0]) and np.array_equal(host(dc), ref[1]), rep
        assert np.array_equal(host(c), ref[2]), rep
        _ = (rho * 2).sum().item()  # eager work between replays
