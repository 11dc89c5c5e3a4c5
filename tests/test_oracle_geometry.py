"""Pins of the oracle's mesh geometry and gradients against closed forms and
an independent geometric construction (not against the oracle's formulas).

Paper passages: Sec. "Nomenclature and notations" (eq. node_normal, nodal
average), Sec. "Integrating the Poisson equation" (cell gradient, the identity
sum_j S_ij = S_i / n_d and the 2D relation n_ij = (n_i - n_j)/6).
"""
import numpy as np
import pytest

import oracle
from paper_2201_01291_amd import workloads as wl


def _meshes():
    return [
        ("tri-jit", wl.tri_rect_mesh(7, 5, 1.3, 0.7, jitter=0.25, seed=1)),
        ("tri-per", wl.tri_rect_mesh(8, 6, 1.0, 0.5, jitter=0.2, seed=2, periodic=True)),
        ("tet-jit", wl.kuhn_tet_mesh(4, 3, 3, 1.0, 0.8, 0.6, jitter=0.15, seed=3, periodic=False)),
        ("tet-per", wl.kuhn_tet_mesh(4, 4, 3, jitter=0.1, seed=4, periodic=True)),
    ]


def _unwrapped_cell_coords(mesh):
    """Cell vertex coordinates unwrapped to the minimum image of vertex 0
    (test-side, from the raw inputs)."""
    X = mesh.xyz[:, mesh.cells]  # [nd][nv][nc]
    if mesh.period is not None:
        L = mesh.period[:, None, None]
        X = X - L * np.round((X - X[:, :1, :]) / L)
    return np.transpose(X, (2, 1, 0))  # [nc][nv][nd]


@pytest.mark.parametrize("name,mesh", _meshes())
def test_node_normals_close_and_volumes(name, mesh):
    om = oracle.OracleMesh(mesh)
    g = om.geometry()
    # a closed simplex surface: sum_k S_k = 0
    scale = np.abs(g["S"]).max()
    assert np.abs(g["S"].sum(axis=1)).max() <= 1e-14 * scale
    # independent volume: |det| / n_d!
    X = _unwrapped_cell_coords(mesh)
    E = X[:, 1:, :] - X[:, :1, :]
    vol = np.abs(np.linalg.det(E)) / (2.0 if mesh.ndim == 2 else 6.0)
    np.testing.assert_allclose(g["Vc"], vol, rtol=1e-12)
    # total volume of the box, twice: cells and median-dual nodal volumes
    box = np.prod(mesh.period) if mesh.period is not None else np.prod(
        mesh.xyz.max(1) - mesh.xyz.min(1))
    assert abs(g["Vc"].sum() - box) <= 1e-13 * box
    assert abs(g["Vn"].sum() - box) <= 1e-13 * box


def _median_dual_face(X, a, b, nd):
    """Area vector of the piece of the median-dual surface of cell X that
    separates vertex a from vertex b, oriented a -> b, built from midpoints
    and centroids (independent construction)."""
    mid = 0.5 * (X[a] + X[b])
    cen = X.mean(axis=0)
    if nd == 2:
        t = cen - mid
        n = np.array([t[1], -t[0]])
        if n @ (X[b] - X[a]) < 0:
            n = -n
        return n
    others = [k for k in range(4) if k not in (a, b)]
    total = np.zeros(3)
    for o in others:
        fc = (X[a] + X[b] + X[o]) / 3.0
        n = 0.5 * np.cross(fc - mid, cen - mid)
        if n @ (X[b] - X[a]) < 0:
            n = -n
        total += n
    return total


@pytest.mark.parametrize("name,mesh", _meshes())
def test_dual_normals_equal_median_dual_faces(name, mesh):
    om = oracle.OracleMesh(mesh)
    Sij, ends = om.edge_normals()
    X = _unwrapped_cell_coords(mesh)
    edges = [(0, 1), (0, 2), (1, 2)] if mesh.nv == 3 else [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    scale = np.abs(Sij).max()
    for c in range(0, mesh.ncells, max(1, mesh.ncells // 40)):
        for e, (a, b) in enumerate(edges):
            ref = _median_dual_face(X[c], a, b, mesh.ndim)
            assert np.abs(Sij[c, e] - ref).max() <= 1e-13 * scale
            assert ends[c, e, 0] == mesh.cells[a, c] and ends[c, e, 1] == mesh.cells[b, c]


@pytest.mark.parametrize("name,mesh", _meshes())
def test_sum_of_dual_normals_is_node_normal_over_nd(name, mesh):
    """The paper's identity sum_{j in tau} S_ij = S_i / n_d (exact for simplices)."""
    om = oracle.OracleMesh(mesh)
    g = om.geometry()
    Sij, _ = om.edge_normals()
    edges = [(0, 1), (0, 2), (1, 2)] if mesh.nv == 3 else [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    acc = np.zeros_like(g["S"])
    for e, (a, b) in enumerate(edges):
        acc[:, a] += Sij[:, e]
        acc[:, b] -= Sij[:, e]
    np.testing.assert_allclose(acc, g["S"] / mesh.ndim, atol=1e-14 * np.abs(g["S"]).max())


@pytest.mark.parametrize("name,mesh", _meshes())
def test_dual_surface_of_every_node_is_closed(name, mesh):
    """sum over cells and edges of +-S_ij plus the boundary normal S_i^b is 0."""
    om = oracle.OracleMesh(mesh)
    g = om.geometry()
    Sij, ends = om.edge_normals()
    acc = np.zeros((mesh.ndim, mesh.nnodes))
    for e in range(Sij.shape[1]):
        for d in range(mesh.ndim):
            np.add.at(acc[d], ends[:, e, 0], Sij[:, e, d])
            np.add.at(acc[d], ends[:, e, 1], -Sij[:, e, d])
    assert np.abs(acc + g["Sb"]).max() <= 1e-14 * np.abs(Sij).max() * 10
    if mesh.period is not None:
        assert np.abs(g["Sb"]).max() == 0.0


def test_2d_relation_one_sixth():
    """2D: n_ij = (n_i - n_j) / 6 on one right triangle, by hand."""
    m = wl.Mesh(np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]), np.array([[0], [1], [2]]), None)
    om = oracle.OracleMesh(m)
    g = om.geometry()
    # S_0 = outward normal of the hypotenuse (1,1); S_1 = (-1,0); S_2 = (0,-1)
    np.testing.assert_allclose(g["S"][0], [[1, 1], [-1, 0], [0, -1]], atol=1e-15)
    Sij, _ = om.edge_normals()
    np.testing.assert_allclose(Sij[0, 0], np.array([2.0, 1.0]) / 6.0, atol=1e-15)
    assert g["Vc"][0] == 0.5
    np.testing.assert_allclose(g["Vn"], [1 / 6, 1 / 6, 1 / 6])


def test_boundary_normals_on_straight_edges():
    nx, ny, lx, ly = 5, 4, 2.0, 1.0
    m = wl.tri_rect_mesh(nx, ny, lx, ly)
    g = oracle.OracleMesh(m).geometry()
    hx, hy = lx / nx, ly / ny
    x, y = m.xyz
    Sb = g["Sb"]
    bottom = (y == 0) & (x > 0) & (x < lx)
    np.testing.assert_allclose(Sb[:, bottom].T, np.tile([0.0, -hx], (bottom.sum(), 1)), atol=1e-15)
    left = (x == 0) & (y > 0) & (y < ly)
    np.testing.assert_allclose(Sb[:, left].T, np.tile([-hy, 0.0], (left.sum(), 1)), atol=1e-15)
    corner = (x == 0) & (y == 0)
    np.testing.assert_allclose(Sb[:, corner].ravel(), [-hy / 2, -hx / 2], atol=1e-15)
    assert np.abs(Sb.sum(axis=1)).max() < 1e-14
    c = oracle.OracleMesh(m).counts()
    assert c["nbfaces"] == 2 * (nx + ny) and c["nbnodes"] == 2 * (nx + ny)


@pytest.mark.parametrize("name,mesh", _meshes())
def test_gradient_exact_for_linear_fields(name, mesh):
    if mesh.period is not None:
        pytest.skip("linear fields are not periodic")
    rng = np.random.default_rng(5)
    coef = rng.normal(size=(3, mesh.ndim))
    off = rng.normal(size=3)
    W = off[:, None] + coef @ mesh.xyz
    G = oracle.OracleMesh(mesh).gradient(W)
    for v in range(3):
        for d in range(mesh.ndim):
            np.testing.assert_allclose(G[v, d], coef[v, d], rtol=0, atol=1e-12 * np.abs(coef).max())


@pytest.mark.parametrize("name,mesh", _meshes())
def test_gradient_of_constant_is_zero(name, mesh):
    W = np.full((2, mesh.nnodes), 3.25)
    G = oracle.OracleMesh(mesh).gradient(W)
    h = mesh.ncells ** (-1.0 / mesh.ndim)
    assert np.abs(G).max() <= 1e-12 * 3.25 / h


def test_gradient_second_order_on_smooth_periodic_field():
    errs = []
    for n in (16, 32):
        m = wl.tri_rect_mesh(n, n, periodic=True)
        x, y = m.xyz
        W = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
        G = oracle.OracleMesh(m).gradient(W[None])
        ex = 2 * np.pi * np.cos(2 * np.pi * x) * np.cos(2 * np.pi * y)
        errs.append(np.abs(G[0, 0] - ex).max())
    assert errs[0] / errs[1] > 3.0  # structured mesh: second order


def test_orientation_and_numbering_do_not_matter():
    m = wl.tri_rect_mesh(6, 5, jitter=0.2, seed=8, periodic=True)
    rng = np.random.default_rng(0)
    W = rng.normal(size=(2, m.nnodes))
    G0 = oracle.OracleMesh(m).gradient(W)
    G1 = oracle.OracleMesh(wl.fix_orientation_free(m)).gradient(W)
    np.testing.assert_allclose(G1, G0, atol=1e-12 * np.abs(G0).max())
    ms, perm = wl.shuffled(m, seed=3)
    G2 = oracle.OracleMesh(ms).gradient(W[:, perm])
    np.testing.assert_allclose(G2, G0[:, :, perm], atol=1e-12 * np.abs(G0).max())


def test_bad_meshes_are_rejected():
    xyz = np.array([[0.0, 1.0, 2.0], [0.0, 0.0, 0.0]])
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleMesh(wl.Mesh(xyz, np.array([[0], [1], [2]]), None))
    assert e.value.code == -2
    xyz = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    with pytest.raises(oracle.OracleError) as e:
        oracle.OracleMesh(wl.Mesh(xyz, np.array([[0], [1], [5]]), None))
    assert e.value.code == -2
