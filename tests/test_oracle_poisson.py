"""Pins of the oracle's Poisson operator and solve.

Paper passages: Sec. "Integrating the Poisson equation" (eq.
poisson_discretization_cartesian, the coefficient a_ij and the remark that
-lap phi is solved), Sec. "Boundary conditions" (Neumann data on the
right-hand side, Dirichlet rows), eq. (poisson).

The matrix S_i . S_k / (V_tau n_d^2) equals the P1 finite-element stiffness
matrix (S_k = -n_d V_tau grad lambda_k), so on a structured right-triangle
grid it is the 5-point stencil and on the Kuhn split of cubes the 7-point
stencil times h: textbook results the tests check against stencils built
from the node coordinates alone.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2201_01291_amd import workloads as wl


def _index(xyz, h, L):
    keys = np.rint(xyz / h).astype(np.int64)
    n = np.rint(np.asarray(L) / h).astype(np.int64)
    return {tuple(int(v) for v in k): i for i, k in enumerate(keys.T)}, n


@pytest.mark.parametrize("nd", [2, 3])
def test_structured_grid_gives_the_finite_difference_stencil(nd):
    if nd == 2:
        m = wl.tri_rect_mesh(8, 8, 1.0, 1.0, periodic=True)
        h, scale = 1.0 / 8, 1.0
    else:
        m = wl.kuhn_tet_mesh(5, 5, 5, 1.0, 1.0, 1.0, periodic=True)
        h, scale = 1.0 / 5, 1.0 / 5
    L = oracle.OracleMesh(m).poisson_matrix().toarray()
    idx, n = _index(m.xyz, h, [1.0] * nd)
    ref = np.zeros_like(L)
    for key, i in idx.items():
        ref[i, i] = 2 * nd * scale
        for d in range(nd):
            for s in (-1, 1):
                nb = list(key)
                nb[d] = (nb[d] + s) % n[d]
                ref[i, idx[tuple(nb)]] -= scale
    np.testing.assert_allclose(L, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("mesh", ["tri-open", "tet-open", "tri-periodic"])
def test_symmetric_zero_row_sums_and_exact_for_linear_fields(mesh):
    if mesh == "tri-open":
        m = wl.tri_rect_mesh(9, 7, 1.0, 0.7, jitter=0.25, seed=3)
    elif mesh == "tet-open":
        m = wl.kuhn_tet_mesh(4, 5, 4, jitter=0.15, seed=2, periodic=False)
    else:
        m = wl.tri_rect_mesh(9, 7, 1.0, 0.7, jitter=0.25, seed=3, periodic=True)
    om = oracle.OracleMesh(m)
    L = om.poisson_matrix()
    assert abs(L - L.T).max() <= 1e-15 * abs(L).max()
    assert np.abs(L @ np.ones(m.nnodes)).max() <= 1e-14 * abs(L).max()
    if m.period is not None:
        return
    # -lap of a linear field vanishes in every interior row; on a boundary
    # row it is the outward flux grad(phi) . S_i^b of the closed dual surface
    g = np.array([0.7, -1.3, 0.4][:m.ndim])
    phi = g @ m.xyz + 0.2
    Sb = om.geometry()["Sb"]
    np.testing.assert_allclose(L @ phi, g @ Sb, rtol=0, atol=1e-13 * np.abs(L).max())


def test_dirichlet_manufactured_solution_converges_at_second_order():
    """-lap phi = 2 pi^2 sin(pi x) sin(pi y), phi = 0 on the boundary of the
    unit square: nodal error O(h^2) on jittered meshes."""
    errs = []
    for n in (12, 24, 48):
        m = wl.tri_rect_mesh(n, n, jitter=0.2, seed=n)
        om = oracle.OracleMesh(m)
        x, y = m.xyz
        exact = np.sin(np.pi * x) * np.sin(np.pi * y)
        bnd = (x < 1e-12) | (x > 1 - 1e-12) | (y < 1e-12) | (y > 1 - 1e-12)
        phi = om.poisson_solve(2 * np.pi ** 2 * exact, dirichlet=bnd, phi_D=np.zeros(m.nnodes))
        assert np.all(phi[bnd] == 0.0)
        errs.append(np.abs(phi - exact).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print("Dirichlet errors", errs, "rates", rates)
    assert errs[-1] < 2e-3 and min(rates) > 1.8


def test_neumann_data_enter_with_the_paper_sign():
    """phi(0) = 0 and grad(phi) . n = -E_n at x = 1 on a strip periodic in y
    with no charge: phi = -E_n x exactly (linear), which fixes the sign and
    the |S_i^b| weight of the Neumann term."""
    m = wl.tri_rect_mesh(10, 4, 1.0, 0.4, jitter=0.2, seed=1, periodic=(False, True))
    om = oracle.OracleMesh(m)
    x = m.xyz[0]
    left, right = x < 1e-12, x > 1 - 1e-12
    En = np.where(right, 3.0, 0.0)
    phi = om.poisson_solve(np.zeros(m.nnodes), dirichlet=left, phi_D=np.zeros(m.nnodes), En=En)
    np.testing.assert_allclose(phi, -3.0 * x, rtol=0, atol=1e-12)
    np.testing.assert_allclose(om.electric_field(phi)[0], 3.0, rtol=0, atol=1e-11)


def test_periodic_mode_with_neutralising_background():
    """Periodic unit square, q = 1 + cos(2 pi x) cos(2 pi y): the uniform part
    is removed (neutralising background), phi -> cos cos / (8 pi^2) with zero
    mean, at second order; E = -grad phi."""
    errs, eerrs = [], []
    for n in (16, 32, 64):
        m = wl.tri_rect_mesh(n, n, jitter=0.2, seed=n, periodic=True)
        om = oracle.OracleMesh(m)
        x, y = m.xyz
        k = 2 * np.pi
        q = 1.0 + np.cos(k * x) * np.cos(k * y)
        phi = om.poisson_solve(q)
        Vn = om.geometry()["Vn"]
        assert abs(Vn @ phi) <= 1e-13 * (Vn @ np.abs(phi))
        exact = np.cos(k * x) * np.cos(k * y) / (2 * k * k)
        errs.append(np.abs(phi - exact).max() / np.abs(exact).max())
        E = om.electric_field(phi)
        Ex = np.sin(k * x) * np.cos(k * y) / (2 * k)
        eerrs.append(np.abs(E[0] - Ex).max() / np.abs(Ex).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print("periodic errors", errs, rates, "field", eerrs)
    assert min(rates) > 1.7 and errs[-1] < 5e-3   # second order (jittered: not superconvergent)
    # the nodal gradient of a jittered mesh is first order in the max norm
    assert all(math.log2(eerrs[i] / eerrs[i + 1]) > 0.9 for i in range(2)) and eerrs[-1] < 0.05
