"""The allocation-free residual (vcx_residual_noalloc) against the solver's
vcx_residual on the same mesh, physics and state: bit for bit, over two
calls in a row on one device (the second on a smaller mesh, so the scratch
array holds the first call's contents), and against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from cases import make_case, normwise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2201_01291_amd import vcx, workloads as wl  # noqa: E402

# (larger, smaller) pairs in nodes, each on the fused 2D pass, the
# three-kernel 3D path, the second closure option, the multi-species model
# and the MUSCL-Hancock predictor (whose half step takes dt)
PAIRS = [("dd2d-streamer", "dd2d-open-vanleer"), ("euler3d-roe", "euler3d-mach2-hllc-sp2"),
         ("explosion2d", "dd2d-open-closure2"), ("ns2d-sp2-open", "ns3d-sp9"),
         ("euler2d-hancock-hllc", "euler3d-hancock-roe-sp2")]


def _reference(case, precision):
    gm = vcx.Mesh(case.mesh, tile_cells=case.tiles[0], tile_nodes=case.tiles[1])
    phys = case.vcx_phys(precision)
    s = vcx.Solver(gm, phys, case.E)
    s.upload(case.U)
    om = oracle.OracleMesh(case.mesh)
    ph = case.oracle_phys()
    dt = om.timestep(ph, case.U, case.E)
    return gm, phys, dt, s.residual(dt), om, ph


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("big,small", PAIRS)
def test_noalloc_residual_matches_vcx_residual(big, small, precision):
    runs = []
    for name in (big, small):
        case = make_case(name)
        print(f"[noalloc] {name} prec={precision} nn={case.mesh.nnodes}", flush=True)
        runs.append((case, *_reference(case, precision)))
    assert runs[1][0].mesh.nnodes < runs[0][0].mesh.nnodes
    for case, gm, phys, dt, r_ref, om, ph in runs:     # two calls in a row, the second smaller
        U = torch.tensor(case.U, device="cuda", dtype=torch.float64)
        E = None if case.E is None else torch.tensor(case.E, device="cuda", dtype=torch.float64)
        r = vcx.residual_noalloc(gm, phys, U, E, dt)
        torch.cuda.synchronize()
        r = r.cpu().numpy()
        assert np.array_equal(r, r_ref), case.name
        err = normwise(r, om.residual(ph, case.U, case.E, dt), om.flux_scale(ph, case.U, case.E, dt))
        assert err.max() <= (1e-4 if precision else 1e-12), (case.name, err)


def test_noalloc_rejects_meshes_beyond_its_scratch():
    """A mesh whose arrays exceed the fixed scratch is refused before any
    launch (the 2M-tet 3D Euler workload needs several hundred MB)."""
    assert vcx.noalloc_scratch_bytes() == 64 << 20
    m = wl.euler3d_mesh()
    gm = vcx.Mesh(m)
    U = torch.zeros((5, m.nnodes), device="cuda", dtype=torch.float64)
    phys = vcx.physics(flux=vcx.FLUX_ROE, limiter=vcx.LIM_VANLEER)
    with pytest.raises(vcx.VcxError) as e:
        vcx.residual_noalloc(gm, phys, U, None, 0.0)
    assert e.value.code == vcx.E_ARG
