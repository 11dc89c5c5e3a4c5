"""GPU second boundary-closure option (Sec. "Boundary conditions in AVIP"):
the interpolated half-edge fluxes, 0.75 F_i + 0.25 F_j, against the oracle
on the linear-drift pin, and the configurations it is defined for (plane 2D
meshes, one solver at a time)."""
import numpy as np
import pytest

import oracle
from paper_2201_01291_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2201_01291_amd import vcx  # noqa: E402


def _dd(closure, **kw):
    return vcx.physics(model=vcx.MODEL_DRIFT_DIFFUSION, limiter=vcx.LIM_MINMOD, rk_stages=1, nspecies=1,
                       z=[1.0], mu=[1.0], D=[0.0], closure=closure, **kw)


def test_linear_drift_closure_matches_the_oracle_and_differs_from_the_first_option():
    m = wl.tri_rect_mesh(40, 30, 1.0, 0.75, jitter=0.25, seed=4)
    print(f"[case] closure2 linear drift nn={m.nnodes}", flush=True)
    x, y = m.xyz
    u = (1.0 + 0.7 * x - 0.4 * y)[None, :]
    E = np.tile(np.array([0.6, -0.3])[:, None], (1, m.nnodes))
    om = oracle.OracleMesh(m)
    gm = vcx.Mesh(m)
    dt = 1e-3
    res = {}
    for c in (1, 2):
        s = vcx.Solver(gm, _dd(c), E)
        s.upload(u)
        ph = oracle.Phys(model=oracle.DRIFT_DIFFUSION, limiter=oracle.MINMOD, rk=1, nspecies=1, z=[1.0],
                         mu=[1.0], D=[0.0], closure=c)
        ro = om.residual(ph, u, E, dt)
        res[c] = s.residual(dt)
        scale = np.abs(om.flux_scale(ph, u, E, dt)).max()
        err = np.abs(res[c] - ro).max() / scale
        print("closure", c, "residual err", err)
        assert err <= 1e-12
    assert np.abs(res[2] - res[1]).max() > 1e-6 * np.abs(res[1]).max()


def test_second_option_restrictions():
    m2 = wl.tri_rect_mesh(8, 6, 1.0, 0.75)
    m3 = wl.kuhn_tet_mesh(2, 2, 2, periodic=False)
    E3 = np.zeros((3, m3.nnodes))
    with pytest.raises(vcx.VcxError) as e:
        vcx.Solver(vcx.Mesh(m3), _dd(2), E3)
    assert e.value.code == vcx.E_ARG
    ax = wl.tri_rect_mesh(8, 6, 1.0, 0.75, origin=(0.0, 0.0))
    with pytest.raises(vcx.VcxError) as e:
        vcx.Solver(vcx.Mesh(ax, axisymmetric=True), _dd(2), np.zeros((2, ax.nnodes)))
    assert e.value.code == vcx.E_ARG
    with pytest.raises(vcx.VcxError) as e:
        vcx.Solver(vcx.Mesh(m2), _dd(3), np.zeros((2, m2.nnodes)))
    assert e.value.code == vcx.E_ARG
    s = vcx.Solver(vcx.Mesh(m2), _dd(2), np.zeros((2, m2.nnodes)))
    s.upload(np.ones((1, m2.nnodes)))
    with pytest.raises(vcx.VcxError) as e:
        vcx.solve_batch([s], [2], graphs=False)
    assert e.value.code == vcx.E_ARG
