"""Pins of the oracle's axisymmetric drift-diffusion (Sec. "Cylindrical
frames", eq. vertex_centered_flux_axi): fluxes through the revolved dual
faces carry the face's centroid radius (first Pappus-Guldinus theorem), node
volumes are int r dA over the dual region (second theorem), both over 2 pi.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import DRIFT_DIFFUSION, MINMOD
from paper_2201_01291_amd import workloads as wl


def _strip(nx, nr, lx=2.0, R=1.0, jitter=0.0, seed=0, periodic_x=True):
    """(x, r) mesh of [-lx/2, lx/2] x [0, R], periodic in x."""
    return wl.tri_rect_mesh(nx, nr, lx, R, jitter=jitter, seed=seed, periodic=(periodic_x, False),
                            origin=(-lx / 2, 0.0))


def _phys(D=1.0, mu=0.0, rk=1):
    return oracle.Phys(model=DRIFT_DIFFUSION, limiter=MINMOD, rk=rk, nspecies=1, z=[1.0], mu=[mu],
                       D=[D], cfl=0.5, fourier=0.25)


def test_pappus_volumes_integrate_r_over_the_domain():
    m = wl.tri_rect_mesh(7, 5, 1.5, 0.8, jitter=0.25, seed=3, origin=(0.0, 0.3))
    Vp, _ = oracle.OracleMesh(m, axisymmetric=True).axi_geometry()
    r0, r1 = 0.3, 1.1
    assert Vp.sum() == pytest.approx(1.5 * (r1 ** 2 - r0 ** 2) / 2, rel=1e-14)
    assert np.all(Vp > 0)


@pytest.mark.parametrize("jitter", [0.0, 0.25])
def test_uniform_drift_residual_is_the_radial_divergence(jitter):
    """u = 1 drifting with a uniform V: the residual of node i is
    V . (sum of r-weighted dual normals around i) = V_r A_i, with A_i the
    plane dual area (closed revolved dual surface: int r n dl = (0, A_i));
    an axial drift leaves the state unchanged."""
    m = wl.tri_rect_mesh(8, 6, 1.0, 0.9, jitter=jitter, seed=4, origin=(0.0, 0.0))
    om = oracle.OracleMesh(m, axisymmetric=True)
    A = om.geometry()["Vn"]
    U = np.ones((1, m.nnodes))
    for V in ((3.0, 0.0), (0.0, 2.0), (1.0, -0.5)):
        E = np.tile(np.asarray(V)[:, None], (1, m.nnodes))
        r = om.residual(_phys(D=0.0, mu=1.0), U, E, dt=1e-3)
        np.testing.assert_allclose(r[0], V[1] * A, rtol=0, atol=1e-14 * np.abs(A).max())


def _gauss3d(x, r, t, s0, D):
    s2 = s0 * s0 + 4 * D * t
    return (s0 * s0 / s2) ** 1.5 * np.exp(-(x * x + r * r) / s2)


def test_diffusion_converges_to_the_three_dimensional_heat_kernel():
    """A Gaussian centred on the axis spreads as in three dimensions (peak
    decay (s0^2 / s^2)^(3/2)), not as in the plane: second-order
    convergence of the axisymmetric scheme, through the axis nodes."""
    s0, D, T = 0.15, 1.0, 0.005
    errs = []
    for n in (20, 40, 80):
        m = _strip(2 * n, n, jitter=0.1, seed=n)
        om = oracle.OracleMesh(m, axisymmetric=True)
        x, r = m.xyz
        U = _gauss3d(x, r, 0.0, s0, D)[None, :]
        E = np.zeros((2, m.nnodes))
        Un, t, _, _ = om.step(_phys(D=D), U, E, nsteps=100000, t_end=T)
        assert t == pytest.approx(T, abs=1e-15)
        errs.append(np.abs(Un[0] - _gauss3d(x, r, T, s0, D)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print("axisymmetric heat kernel errors", errs, rates)
    assert min(rates) > 1.6 and errs[-1] < 6e-3   # peak 0.385: about 1% at 80 cells per radius
    # the plane scheme on the same mesh follows the 2D kernel instead
    om2 = oracle.OracleMesh(m)
    U2, _, _, _ = om2.step(_phys(D=D), U, E, nsteps=100000, t_end=T)
    assert abs(U2[0].max() - _gauss3d(0, 0, T, s0, D)) > 10 * errs[-1]


def test_conservation_of_the_revolved_total():
    """Without boundary closure (no flux through r = R) the revolved total
    sum_i V_i u_i is conserved to roundoff; the axis carries no flux."""
    m = _strip(30, 15, jitter=0.2, seed=5)
    om = oracle.OracleMesh(m, axisymmetric=True)
    Vp, _ = om.axi_geometry()
    x, r = m.xyz
    U = _gauss3d(x - 0.2, r, 0.0, 0.15, 1.0)[None, :]
    E = np.tile(np.array([3.0, 0.0])[:, None], (1, m.nnodes))   # axial drift, periodic in x
    ph = _phys(D=0.3, mu=1.0)
    ph.closure = False
    s0 = Vp @ U[0]
    Un, _, _, n = om.step(ph, U, E, nsteps=20)
    assert n == 20
    assert abs(Vp @ Un[0] - s0) <= 1e-13 * s0
    so, _ = om.sums(Un)
    assert so[0] == pytest.approx(Vp @ Un[0], rel=1e-13)


def test_axisymmetric_poisson_operator_identities():
    """Sec. "Axisymmetric configuration": the matrix of -lap phi over the
    revolved nodal volumes is not symmetric, but rows and columns sum to
    zero (constants are its null space on both sides); it annihilates
    a + b x away from the outer boundary, and -lap r = -1/r integrates to
    -A_i (int over the revolved volume of 1/r, over 2 pi), axis nodes
    included."""
    m = wl.tri_rect_mesh(10, 8, 2.0, 1.0, jitter=0.2, seed=3, origin=(-1.0, 0.0))
    om = oracle.OracleMesh(m, axisymmetric=True)
    L = om.poisson_matrix()
    one = np.ones(m.nnodes)
    scale = abs(L).max()
    assert abs(L - L.T).max() > 1e-3 * scale
    assert np.abs(L @ one).max() <= 1e-14 * scale and np.abs(L.T @ one).max() <= 1e-14 * scale
    x, r = m.xyz
    outer = om.boundary_measure() > 0          # the axis carries no boundary surface
    A = om.geometry()["Vn"]
    assert np.abs((L @ (0.3 + 2.0 * x))[~outer]).max() <= 1e-14 * scale
    np.testing.assert_allclose((L @ r)[~outer], -A[~outer], rtol=0, atol=1e-14 * scale)


def test_axisymmetric_poisson_converges_to_a_3d_solution():
    """phi = exp(-(x^2 + r^2)/s^2) with q = -lap phi (three-dimensional
    Laplacian), Dirichlet values on x = +-1 and r = 1, nothing imposed on
    the axis: second-order convergence, axis nodes included."""
    s2 = 0.2
    errs = []
    for n in (12, 24, 48):
        m = wl.tri_rect_mesh(2 * n, n, 2.0, 1.0, jitter=0.15, seed=n, origin=(-1.0, 0.0))
        om = oracle.OracleMesh(m, axisymmetric=True)
        x, r = m.xyz
        rho2 = x * x + r * r
        exact = np.exp(-rho2 / s2)
        q = -exact * (4 * rho2 / s2 ** 2 - 6 / s2)
        dirichlet = (np.abs(np.abs(x) - 1) < 1e-12) | (np.abs(r - 1) < 1e-12)
        phi = om.poisson_solve(q, dirichlet=dirichlet, phi_D=exact)
        errs.append(np.abs(phi - exact).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print("axisymmetric Poisson errors", errs, rates)
    assert min(rates) > 1.7 and errs[-1] < 2e-3


def _gas(flux=oracle.HLLC, **kw):
    return oracle.Phys(model=oracle.GAS, flux=flux, limiter=oracle.VANLEER, rk=2, cfl=0.5, **kw)


@pytest.mark.parametrize("flux", [oracle.HLLC, oracle.ROE])
def test_axisymmetric_gas_preserves_a_uniform_axial_stream(flux):
    """Sec. "Geometric source terms": with the pressure source p A_i in the
    radial momentum, a uniform stream along the axis is an exact discrete
    steady state on every node, boundary and axis included (the revolved
    dual surface gives int r n dl = (0, A_i), which the source balances)."""
    m = wl.tri_rect_mesh(10, 6, 2.0, 1.0, jitter=0.25, seed=8, origin=(-1.0, 0.0))
    om = oracle.OracleMesh(m, axisymmetric=True)
    U = wl.conserved_from_primitive(np.ones(m.nnodes), np.vstack([np.full(m.nnodes, 0.7), np.zeros(m.nnodes)]),
                                    np.full(m.nnodes, 1.3), 1.4)
    r = om.residual(_gas(flux), U)
    scale = np.abs(om.flux_scale(_gas(flux), U)).max(axis=1)
    assert np.all(np.abs(r).max(axis=1) <= 1e-14 * scale)


def test_axisymmetric_gas_conserves_mass_axial_momentum_and_energy():
    """Periodic in x, no boundary closure: the revolved totals of mass,
    axial momentum and energy are conserved (the geometric source acts on
    the radial momentum only); the radial velocity stays zero on the axis."""
    m = wl.tri_rect_mesh(24, 10, 2.0, 1.0, jitter=0.2, seed=9, periodic=(True, False), origin=(-1.0, 0.0))
    om = oracle.OracleMesh(m, axisymmetric=True)
    x, r = m.xyz
    rho = 1.0 + 0.3 * np.exp(-(x * x + r * r) / 0.1)
    p = 1.0 + 0.5 * np.exp(-(x * x + r * r) / 0.1)
    U = wl.conserved_from_primitive(rho, np.vstack([0.3 + 0 * x, 0 * x]), p, 1.4)
    ph = _gas()
    ph.closure = False
    Vp, _ = om.axi_geometry()
    s0 = Vp @ U.T
    Un, _, _, n = om.step(ph, U, nsteps=10)
    assert n == 10
    s1 = Vp @ Un.T
    for v in (0, 1, 3):
        assert abs(s1[v] - s0[v]) <= 1e-13 * abs(Vp @ np.abs(U[v]))
    assert np.all(Un[2][r == 0.0] == 0.0)
    assert abs(s1[2]) > 1e-6 * Vp @ np.abs(U[1])    # the radial momentum has a source
