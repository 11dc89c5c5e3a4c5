"""Pins of the oracle's Scharfetter-Gummel drift-diffusion flux (Sec.
"Scharfetter Gummel scheme"): exponential fitting along each edge, central
across it.

* Along the edge the flux is that of the 1D steady advection-diffusion
  solution through the two nodal values: for nodal values sampled from
  u = A + B exp(V_t x / D) (the steady solutions, flux V_t A) it returns
  exactly V_t A times the edge-parallel area.
* Its limits: D -> 0 is upwinding, V -> 0 the two-point diffusion flux.
* Across the edge it is the central flux (V u_bar - D grad u_bar) . S_perp.
* Scheme level: on a periodic strip a drifting, spreading Gaussian (the 1D
  heat kernel in the moving frame) is reached at second order at moderate
  cell Peclet numbers, and mass is conserved.
"""
import numpy as np
import pytest

import oracle
from paper_2201_01291_amd import workloads as wl


def _edge(rng, nd):
    dx = rng.normal(size=nd)
    h = np.linalg.norm(dx)
    return dx, h, dx / h


@pytest.mark.parametrize("nd", [2, 3])
def test_flux_of_the_steady_exponential_profile_is_exact(nd):
    rng = np.random.default_rng(nd)
    for _ in range(20):
        dx, h, t = _edge(rng, nd)
        Vt = rng.uniform(-5.0, 5.0)
        D = rng.uniform(0.05, 3.0)
        A, B = rng.uniform(0.5, 2.0), rng.uniform(-0.3, 0.3)
        ui, uj = A + B, A + B * np.exp(Vt * h / D)
        c = rng.uniform(0.2, 2.0)
        S = c * dx                                   # all of S along the edge
        V = Vt * t + 0.0 * rng.normal(size=nd)
        F = oracle.sg_flux(ui, uj, V, S, dx, D, rng.normal(size=nd))
        want = Vt * A * (S @ t)
        assert F == pytest.approx(want, rel=1e-11, abs=1e-13 * abs(Vt * A * c * h))


def test_limits_upwind_and_pure_diffusion():
    rng = np.random.default_rng(5)
    for _ in range(20):
        dx, h, t = _edge(rng, 2)
        S = rng.uniform(0.3, 1.5) * dx
        ui, uj = rng.uniform(0.1, 3.0, size=2)
        Vt = rng.uniform(-4.0, 4.0)
        V = Vt * t
        up = (S @ t) * Vt * (ui if Vt >= 0 else uj)
        # D = 0 is upwinding, and small D approaches it
        assert oracle.sg_flux(ui, uj, V, S, dx, 0.0, np.zeros(2)) == pytest.approx(up, rel=1e-14)
        assert oracle.sg_flux(ui, uj, V, S, dx, 1e-9, np.zeros(2)) == pytest.approx(up, rel=1e-6)
        # no drift: two-point diffusion along the edge
        D = rng.uniform(0.1, 2.0)
        diff = -D * (uj - ui) / h * (S @ t)
        assert oracle.sg_flux(ui, uj, np.zeros(2), S, dx, D, np.zeros(2)) == pytest.approx(diff, rel=1e-13)
        # and a tiny drift is continuous with it
        assert oracle.sg_flux(ui, uj, 1e-9 * t, S, dx, D, np.zeros(2)) == pytest.approx(diff, rel=1e-6,
                                                                                        abs=1e-8)


@pytest.mark.parametrize("nd", [2, 3])
def test_flux_across_the_edge_is_central(nd):
    rng = np.random.default_rng(10 + nd)
    for _ in range(20):
        dx, h, t = _edge(rng, nd)
        w = rng.normal(size=nd)
        Sp = w - (w @ t) * t                         # S orthogonal to the edge
        V, g = rng.normal(size=nd), rng.normal(size=nd)
        ui, uj, D = rng.uniform(0.1, 2.0), rng.uniform(0.1, 2.0), rng.uniform(0.1, 2.0)
        F = oracle.sg_flux(ui, uj, V, Sp, dx, D, g)
        assert F == pytest.approx(0.5 * (ui + uj) * (V @ Sp) - D * (g @ Sp), rel=1e-12, abs=1e-14)
        # a general S: the two parts add
        Sa = 0.7 * dx
        Fa = oracle.sg_flux(ui, uj, V, Sa, dx, D, g)
        assert oracle.sg_flux(ui, uj, V, Sa + Sp, dx, D, g) == pytest.approx(F + Fa, rel=1e-12, abs=1e-14)


def _gauss(x, t, V, D, s0, L):
    s2 = s0 * s0 + 4.0 * D * t
    xc = (x - 0.5 * L - V * t + 0.5 * L) % L - 0.5 * L   # distance to the centre, periodic
    return np.sqrt(s0 * s0 / s2) * np.exp(-xc * xc / s2)


def _sg_error(nx, V=1.0, D=0.02, s0=0.08, t_end=0.3, L=1.0):
    m = wl.tri_rect_mesh(nx, 3, L, 3.0 * L / nx, periodic=True)
    x = m.xyz[0]
    U = _gauss(x, 0.0, V, D, s0, L)[None, :]
    E = np.vstack([np.full(m.nnodes, V), np.zeros(m.nnodes)])     # z mu = 1: drift V along x
    ph = oracle.Phys(model=oracle.DRIFT_DIFFUSION, flux=oracle.SG, rk=2, nspecies=1, z=[1.0], mu=[1.0],
                     D=[D], cfl=0.4, fourier=0.2, closure=0)
    om = oracle.OracleMesh(m)
    m0 = om.sums(U)[0]
    Ue, t, *_ = om.step(ph, U, E, nsteps=100000, t_end=t_end)
    assert t == pytest.approx(t_end, abs=1e-14)
    np.testing.assert_allclose(om.sums(Ue)[0], m0, rtol=1e-13)
    return np.abs(Ue[0] - _gauss(x, t_end, V, D, s0, L)).max()


def test_scheme_converges_to_the_drifting_heat_kernel():
    errs = [_sg_error(n) for n in (32, 64, 128)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("SG errors", errs, "orders", rates)
    assert errs[-1] < 5e-3
    assert rates[-1] >= 1.7


def test_sg_differs_from_llw_and_rejects_unknown_schemes():
    m = wl.tri_rect_mesh(12, 5, periodic=True)
    x = m.xyz[0]
    U = (1.0 + np.exp(-((x - 0.5) / 0.1) ** 2))[None, :]
    E = np.vstack([np.full(m.nnodes, 2.0), np.full(m.nnodes, 0.5)])
    base = dict(model=oracle.DRIFT_DIFFUSION, rk=1, nspecies=1, z=[1.0], mu=[1.0], D=[0.05], closure=0)
    om = oracle.OracleMesh(m)
    r_sg = om.residual(oracle.Phys(flux=oracle.SG, **base), U, E, dt=1e-3)
    r_llw = om.residual(oracle.Phys(flux=oracle.LLW, **base), U, E, dt=1e-3)
    assert np.abs(r_sg - r_llw).max() > 1e-3 * np.abs(r_llw).max()
    assert abs(r_sg.sum()) <= 1e-13 * np.abs(r_sg).sum()
    with pytest.raises(oracle.OracleError):
        om.residual(oracle.Phys(flux=1, **base), U, E, dt=1e-3)
