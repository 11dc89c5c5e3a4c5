"""Pins of the oracle's axisymmetric multi-species Navier-Stokes (Sec.
"Geometric source terms", eq. ns_cyl_source_terms): r-weighted convective
and diffusive fluxes, the convective source p and the diffusive source
-2 eta u_r/r - lambda (u_r/r + du_r/dr + du_x/dx) of the radial momentum,
with lambda = -2/3 eta.

The viscous part of a residual is isolated as R(eta) - R(eta = 0): with a
uniform temperature and composition the convective fluxes do not see the
viscosity, and with eta = 0 every diffusive coefficient vanishes.

* A uniform axial stream stays steady.
* Uniform radial expansion u_r = a r: the axisymmetric stress has
  tau_rr = tau_theta_theta, so the r-weighted viscous force on the radial
  momentum, tau_rr A_i, is cancelled exactly by the hoop-stress source
  -tau_theta_theta A_i at every interior node (the velocity is linear, its
  cell gradients exact, and the r-weighted dual faces close:
  int r n dl = (0, A_i)).
* Axial shear u_x = c r: the viscous force on the axial momentum is
  eta c A_i exactly (eta c is the constant shear stress).
* An axial-velocity Gaussian across the axis spreads as the planar radial
  heat kernel (peak decay (s0/s)^2); the scheme converges to it at second
  order through the axis nodes.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle import NAVIER_STOKES
from paper_2201_01291_amd import workloads as wl

LX, R = 0.02, 0.01


def _mesh(nx, nr, jitter=0.0, seed=0):
    return wl.tri_rect_mesh(nx, nr, LX, R, jitter=jitter, seed=seed, periodic=(True, False),
                            origin=(-LX / 2, 0.0))


def _mixture(mu_ref):
    mix = wl.synthetic_mixture(2, seed=5)
    return dataclasses.replace(mix, mu_ref=mu_ref)


def _phys(mu_ref, rk=2):
    mix = _mixture(mu_ref)
    return oracle.Phys(model=NAVIER_STOKES, limiter=2, rk=rk, nspecies=2, closure=1, mixture=mix)


def _state(m, ph, ux, ur, T=600.0, rho=1.1):
    nn = m.nnodes
    P = np.stack([np.full(nn, rho), ux, ur, np.full(nn, T), np.full(nn, 0.3), np.full(nn, 0.7)])
    return oracle.conserved_from_primitive(2, ph, P)


def _viscous_part(m, ux, ur, mu_ref=2e-3):
    om = oracle.OracleMesh(m, axisymmetric=True)
    ph1, ph0 = _phys(mu_ref), _phys(0.0)
    U = _state(m, ph1, ux, ur)
    r1 = om.residual(ph1, U, dt=1e-6)
    r0 = om.residual(ph0, U, dt=1e-6)
    assert np.array_equal(U, _state(m, ph0, ux, ur))
    g = om.geometry()
    interior = np.all(g["Sb"] == 0.0, axis=0)
    eta = mu_ref * (600.0 / _mixture(mu_ref).T_ref) ** 0.7
    return om, r1, r0, interior, g["Vn"], eta


def test_uniform_axial_stream_is_steady():
    m = _mesh(10, 6, jitter=0.2, seed=3)
    om = oracle.OracleMesh(m, axisymmetric=True)
    ph = _phys(2e-3)
    U = _state(m, ph, np.full(m.nnodes, 40.0), np.zeros(m.nnodes))
    r = om.residual(ph, U, dt=1e-6)
    scale = om.flux_scale(ph, U, dt=1e-6)
    assert np.all(np.abs(r) <= 1e-13 * scale.max(axis=1, keepdims=True))
    Ue, *_ = om.step(ph, U, nsteps=4)
    assert np.all(np.abs(Ue - U) <= 1e-13 * np.abs(U).max(axis=1, keepdims=True) + 1e-13 * 40.0 * 1.1)


@pytest.mark.parametrize("jitter", [0.0, 0.25])
def test_radial_expansion_viscous_force_cancels_the_hoop_stress(jitter):
    m = _mesh(9, 7, jitter=jitter, seed=4)
    a = 1.5e3
    r = m.xyz[1]
    om, r1, r0, inner, A, eta = _viscous_part(m, np.zeros(m.nnodes), a * r)
    dv = r1 - r0
    tau = 2.0 / 3.0 * eta * a                    # tau_rr = tau_theta_theta
    scale = tau * A.max()
    print("radial/axial viscous residual at interior nodes",
          np.abs(dv[2, inner]).max() / scale, np.abs(dv[1, inner]).max() / scale)
    assert np.abs(dv[2, inner]).max() <= 1e-10 * scale
    assert np.abs(dv[1, inner]).max() <= 1e-10 * scale
    # the two halves are each of the size tau A: the cancellation is real
    assert np.abs(dv[2, ~inner]).max() > 0.1 * scale


@pytest.mark.parametrize("jitter", [0.0, 0.25])
def test_axial_shear_viscous_force_is_the_shear_stress_times_the_area(jitter):
    m = _mesh(9, 7, jitter=jitter, seed=5)
    c = 2.0e3
    om, r1, r0, inner, A, eta = _viscous_part(m, c * m.xyz[1], np.zeros(m.nnodes))
    dv = r1 - r0
    # residual = outflow - sources: the viscous force eta c A enters with a minus
    want = -eta * c * A
    assert np.allclose(dv[1, inner], want[inner], rtol=1e-10, atol=0)
    assert np.abs(dv[2, inner]).max() <= 1e-10 * eta * c * A.max()


def _gaussian_shear_error(n, s0=2e-3, Rmax=8e-3, mu_ref=0.05):
    """Axial velocity 2 exp(-r^2/s0^2) (m/s) diffusing across the axis: the
    planar radial heat kernel, u = 2 (s0/s)^2 exp(-r^2/s^2) with
    s^2 = s0^2 + 4 nu t, solves the axial momentum equation of this shear
    flow (uniform density and pressure, no x dependence; the viscous heating
    is below 1e-5 of the internal energy).  Run to s^2 = 2 s0^2."""
    h = Rmax / n
    m = wl.tri_rect_mesh(4, n, 4 * h, Rmax, periodic=(True, False), origin=(0.0, 0.0))
    r = m.xyz[1]
    ph = _phys(mu_ref, rk=2)
    ph.fourier = 0.2
    U = _state(m, ph, 2.0 * np.exp(-(r / s0) ** 2), np.zeros(m.nnodes))
    eta = mu_ref * (600.0 / ph.mixture.T_ref) ** 0.7
    nu = eta / 1.1
    t_end = s0 * s0 / (4.0 * nu)
    Ue, t, *_ = oracle.OracleMesh(m, axisymmetric=True).step(ph, U, nsteps=100000, t_end=t_end)
    s2 = s0 * s0 + 4.0 * nu * t
    exact = 2.0 * (s0 * s0 / s2) * np.exp(-r * r / s2)
    near = r <= 0.5 * Rmax
    return np.abs(Ue[1] / Ue[0] - exact)[near].max() / 2.0


def test_gaussian_shear_diffuses_at_the_cylindrical_heat_kernel_rate():
    """The peak of an axial-velocity Gaussian centred on the axis decays as
    (s0/s)^2, the planar radial heat kernel: second-order convergence of
    the r-weighted viscous fluxes through the axis nodes (from about 1.5 at
    32 to 64 cells across the radius)."""
    errs = [_gaussian_shear_error(n) for n in (32, 64)]
    rate = np.log2(errs[0] / errs[1])
    print("Gaussian shear errors", errs, "order", rate)
    # (1.5 at this pair, 1.7 from 64 to 128 cells across the radius)
    assert errs[-1] < 2e-3
    assert rate >= 1.4


def test_axis_nodes_keep_zero_radial_velocity():
    m = _mesh(8, 6, jitter=0.2, seed=6)
    ph = _phys(2e-3)
    r = m.xyz[1]
    U = _state(m, ph, 30.0 + 5.0 * np.sin(2 * np.pi * m.xyz[0] / LX), 1.0e3 * r * (R - r) / R)
    Ue, *_ = oracle.OracleMesh(m, axisymmetric=True).step(ph, U, nsteps=3)
    assert np.all(Ue[2, r == 0.0] == 0.0)
    assert np.abs(Ue[2, r > 0]).max() > 0
