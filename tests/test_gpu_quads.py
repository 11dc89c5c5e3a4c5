"""GPU quadrilateral meshes beyond the per-case parity tests: the
Scharfetter-Gummel exactness on rectangles that the oracle pins, the
drifting heat kernel to its end time, and what quadrilateral meshes are not
offered for (multi-species model, Poisson, batches, the server)."""
import numpy as np
import pytest

import oracle
from cases import make_case
from paper_2201_01291_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2201_01291_amd import vcx  # noqa: E402


def test_sg_residual_of_the_steady_profile_vanishes_on_rectangles():
    V, D, A, B = 3.0, 0.4, 1.0, 0.05
    m = wl.quad_rect_mesh(12, 5, 1.0, 0.5, periodic=(False, True))
    x = m.xyz[0]
    U = (A + B * np.exp(V * x / D))[None, :]
    E = np.vstack([np.full(m.nnodes, V), np.zeros(m.nnodes)])
    s = vcx.Solver(vcx.Mesh(m), vcx.physics(model=vcx.MODEL_DRIFT_DIFFUSION, flux=vcx.FLUX_SG, rk_stages=1,
                                              nspecies=1, z=[1.0], mu=[1.0], D=[D], closure=False), E)
    s.upload(U)
    r = s.residual(1e-4)
    inner = (x > 1e-12) & (x < 1.0 - 1e-12)
    assert np.abs(r[0, inner]).max() <= 1e-12 * V * A * 0.1


@pytest.mark.parametrize("precision", [0, 1])
def test_quad_heat_kernel_matches_the_oracle(precision):
    L, V, D, s0, t_end, nx = 1.0, 1.0, 0.02, 0.08, 0.3, 64
    m = wl.quad_rect_mesh(nx, 3, L, 3.0 * L / nx, periodic=True)
    x = m.xyz[0]
    U = np.exp(-((x - 0.5) / s0) ** 2)[None, :]
    E = np.vstack([np.full(m.nnodes, V), np.zeros(m.nnodes)])
    kw = dict(nspecies=1, z=[1.0], mu=[1.0], D=[D])
    op = oracle.Phys(model=oracle.DRIFT_DIFFUSION, flux=oracle.LLW, limiter=4, rk=2, cfl=0.4, fourier=0.2,
                     closure=0, **kw)
    print(f"[quads] heat kernel prec={precision}", flush=True)
    Uo, to, _, no = oracle.OracleMesh(m).step(op, U, E, nsteps=100000, t_end=t_end)
    s = vcx.Solver(vcx.Mesh(m), vcx.physics(model=vcx.MODEL_DRIFT_DIFFUSION, limiter=vcx.LIM_NONE, rk_stages=2,
                                              cfl=0.4, fourier=0.2, closure=False, precision=precision,
                                              **kw), E)
    s.upload(U)
    tg, _ = s.step(100000, t_end=t_end)
    assert tg == pytest.approx(t_end, abs=1e-14)
    err = np.abs(s.download() - Uo).max() / np.abs(Uo).max()
    print(f"quad heat kernel prec={precision}: {no} steps, err {err}")
    if precision == 0:
        assert s.steps_done() == no and err <= 1e-12
    else:
        assert err <= 1e-4


def test_quad_meshes_outside_their_scope_are_rejected():
    m = wl.quad_rect_mesh(8, 6, 0.01, 0.008, periodic=True)
    gm = vcx.Mesh(m)
    mix = wl.synthetic_mixture(2, seed=1)
    with pytest.raises(vcx.VcxError) as e:
        vcx.Solver(gm, vcx.physics(model=vcx.MODEL_NAVIER_STOKES, nspecies=2, mixture=mix), None)
    assert e.value.code == vcx.E_ARG
    with pytest.raises(vcx.VcxError) as e:
        vcx.Poisson(gm)
    assert e.value.code == vcx.E_ARG
    case = make_case("quad-euler-hllc")
    s = vcx.Solver(vcx.Mesh(case.mesh), case.vcx_phys())
    s.upload(case.U)
    with pytest.raises(vcx.VcxError) as e:
        vcx.solve_batch([s], [1])
    assert e.value.code == vcx.E_ARG
    sv = vcx.Server(hbm_budget=1 << 28)
    with pytest.raises(vcx.VcxError) as e:
        sv.submit(vcx.Mesh(case.mesh), case.vcx_phys(), case.U, None, nsteps=2)
    assert e.value.code == vcx.E_ARG
    sv.close()
    bad = wl.quad_rect_mesh(2, 2)
    bad.xyz[:, 4] += 0.9
    with pytest.raises(vcx.VcxError) as e:
        vcx.Mesh(bad)
    assert e.value.code in (vcx.E_ARG, vcx.E_MESH)
