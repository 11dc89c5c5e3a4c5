"""Pins of the second boundary-closure option (Sec. "Boundary conditions in
AVIP"): in two dimensions the flux through each half of a boundary edge is
interpolated, 0.75 F_i + 0.25 F_j, which is the exact integral of the
linearly interpolated node flux over that half edge."""
import numpy as np
import pytest

import oracle
from oracle import DRIFT_DIFFUSION, GAS, HLLC, MINMOD, VANLEER
from paper_2201_01291_amd import workloads as wl


def _half_edges(m):
    """Boundary half edges (node, other node, outward normal times the half
    length) of a rectangle mesh, built from the coordinates alone."""
    x = m.xyz
    lo, hi = x.min(axis=1), x.max(axis=1)
    on = [np.isclose(x[0], lo[0]), np.isclose(x[0], hi[0]), np.isclose(x[1], lo[1]), np.isclose(x[1], hi[1])]
    normals = [(-1.0, 0.0), (1.0, 0.0), (0.0, -1.0), (0.0, 1.0)]
    out = []
    cells = m.cells
    for c in range(m.ncells):
        v = cells[:, c]
        for a, b in ((v[0], v[1]), (v[1], v[2]), (v[2], v[0])):
            for side, n in zip(on, normals):
                if side[a] and side[b]:
                    L = np.linalg.norm(x[:, b] - x[:, a])
                    for i, j in ((a, b), (b, a)):
                        out.append((i, j, np.asarray(n) * L / 2))
    return out


def test_uniform_state_gives_the_first_option():
    m = wl.tri_rect_mesh(7, 5, 1.0, 0.6, jitter=0.25, seed=2)
    om = oracle.OracleMesh(m)
    U = wl.conserved_from_primitive(np.full(m.nnodes, 1.2), np.vstack([np.full(m.nnodes, 0.4),
                                    np.full(m.nnodes, -0.2)]), np.full(m.nnodes, 0.9), 1.4)
    ph1 = oracle.Phys(model=GAS, flux=HLLC, limiter=VANLEER, rk=2, closure=1)
    ph2 = oracle.Phys(model=GAS, flux=HLLC, limiter=VANLEER, rk=2, closure=2)
    r1, r2 = om.residual(ph1, U), om.residual(ph2, U)
    scale = np.abs(om.flux_scale(ph1, U)).max()
    np.testing.assert_allclose(r2, r1, rtol=0, atol=1e-14 * scale)


def test_linear_flux_is_integrated_exactly_per_node():
    """Uniform drift V of a linear density u, no diffusion: the closure of
    each boundary node equals the integral of u V . n over its half edges
    (two-point Gauss quadrature from the coordinates), which the first
    option only approximates."""
    m = wl.tri_rect_mesh(8, 6, 1.0, 0.75, jitter=0.25, seed=4)
    om = oracle.OracleMesh(m)
    x, y = m.xyz
    u = (1.0 + 0.7 * x - 0.4 * y)[None, :]
    V = np.array([0.6, -0.3])
    E = np.tile(V[:, None], (1, m.nnodes))
    base = dict(model=DRIFT_DIFFUSION, limiter=MINMOD, rk=1, nspecies=1, z=[1.0], mu=[1.0], D=[0.0])
    dt = 1e-3
    r0 = om.residual(oracle.Phys(**base, closure=0), u, E, dt)[0]
    c1 = om.residual(oracle.Phys(**base, closure=1), u, E, dt)[0] - r0
    c2 = om.residual(oracle.Phys(**base, closure=2), u, E, dt)[0] - r0
    exact = np.zeros(m.nnodes)
    g = 0.5 / np.sqrt(3.0)
    for i, j, Sn in _half_edges(m):
        mid = 0.5 * (m.xyz[:, i] + m.xyz[:, j])
        pts = [m.xyz[:, i] + (mid - m.xyz[:, i]) * (0.5 + s) for s in (-g, g)]
        ubar = np.mean([1.0 + 0.7 * p[0] - 0.4 * p[1] for p in pts])
        exact[i] += ubar * (V @ Sn)
    np.testing.assert_allclose(c2, exact, rtol=0, atol=1e-14 * np.abs(exact).max())
    assert np.abs(c1 - exact).max() > 1e-3 * np.abs(exact).max()


def test_second_option_is_two_dimensional_and_planar():
    m3 = wl.kuhn_tet_mesh(2, 2, 2, periodic=False)
    om = oracle.OracleMesh(m3)
    U = wl.conserved_from_primitive(np.ones(m3.nnodes), np.zeros((3, m3.nnodes)), np.ones(m3.nnodes), 1.4)
    with pytest.raises(oracle.OracleError):
        om.residual(oracle.Phys(model=GAS, closure=2), U)
