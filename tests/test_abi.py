"""CPU tests of the C ABI library: it loads, exports every symbol declared in
include/vcx.h, and its host-side mesh preprocessing validates meshes and
builds tiles that cover every cell (no device needed)."""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_2201_01291_amd import vcx, workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "vcx.h")).read()
    return sorted(set(re.findall(r"\b(vcx_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared() == sorted(vcx.EXPORTS)


def test_library_exports_every_declared_symbol():
    vcx.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", vcx.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (vcx_[a-z_]+)\b", out))
    missing = [s for s in _declared() if s not in exported]
    assert not missing, missing


@pytest.mark.parametrize("mesh", [
    wl.dd_streamer_mesh(60, 40), wl.sod_tube(50, 5), wl.kuhn_tet_mesh(6, 5, 4, jitter=0.1, seed=1),
    wl.kuhn_tet_mesh(3, 4, 3, jitter=0.1, seed=2, periodic=False)], ids=["dd", "sod", "tet", "tet-open"])
def test_preprocess_matches_oracle_volumes_and_counts(mesh):
    st = vcx.mesh_preprocess(mesh)
    om = oracle.OracleMesh(mesh)
    g = om.geometry()
    assert st["nnodes"] == mesh.nnodes and st["ncells"] == mesh.ncells
    assert st["nfaces"] == mesh.nfaces
    assert st["vol_cells"] == pytest.approx(g["Vc"].sum(), rel=1e-13)
    assert st["vol_nodes"] == pytest.approx(g["Vn"].sum(), rel=1e-13)
    assert st["nbnd"] == om.counts()["nbnodes"]
    assert st["max_tile_cells"] <= (256 if mesh.ndim == 2 else 128)
    # every node is in at least one tile slot, slots are bounded by the incidences
    assert mesh.nnodes <= st["nslots"] <= mesh.ncells * mesh.nv


def test_orientation_and_numbering_do_not_change_volumes():
    m = wl.tri_rect_mesh(12, 9, jitter=0.2, seed=4, periodic=True)
    a = vcx.mesh_preprocess(m)
    b = vcx.mesh_preprocess(wl.fix_orientation_free(m))
    c = vcx.mesh_preprocess(wl.shuffled(m, seed=1)[0])
    assert a["vol_cells"] == pytest.approx(b["vol_cells"], rel=1e-14)
    assert a["vol_cells"] == pytest.approx(c["vol_cells"], rel=1e-14)


def _code(mesh):
    try:
        vcx.mesh_preprocess(mesh)
    except vcx.VcxError as e:
        return e.code
    return 0


def test_invalid_meshes_are_rejected():
    xyz = np.array([[0.0, 1.0, 2.0], [0.0, 0.0, 0.0]])
    assert _code(wl.Mesh(xyz, np.array([[0], [1], [2]]), None)) == vcx.E_MESH       # degenerate
    xyz = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    assert _code(wl.Mesh(xyz, np.array([[0], [1], [7]]), None)) == vcx.E_MESH       # out of range
    assert _code(wl.Mesh(xyz, np.array([[0], [1], [1]]), None)) == vcx.E_MESH       # repeated node
    # a node no cell uses
    xyz4 = np.array([[0.0, 1.0, 0.0, 5.0], [0.0, 0.0, 1.0, 5.0]])
    assert _code(wl.Mesh(xyz4, np.array([[0], [1], [2]]), None)) == vcx.E_MESH
    # three triangles on one edge: non-manifold
    xyz5 = np.array([[0.0, 1.0, 0.5, 0.5, 0.2], [0.0, 0.0, 1.0, -1.0, 0.7]])
    cells = np.array([[0, 1, 0], [1, 0, 1], [2, 3, 4]])
    assert _code(wl.Mesh(xyz5, cells, None)) == vcx.E_MESH
    # wrong arity / dimension
    assert _code(wl.Mesh(np.zeros((1, 3)), np.array([[0], [1]]), None)) == vcx.E_ARG
    bad = wl.Mesh(np.array([[0.0, 1.0, np.nan], [0.0, 0.0, 1.0]]), np.array([[0], [1], [2]]), None)
    assert _code(bad) == vcx.E_ARG


def test_single_cell_mesh_is_accepted():
    m = wl.Mesh(np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]), np.array([[0], [1], [2]]), None)
    st = vcx.mesh_preprocess(m)
    assert st["ntiles"] == 1 and st["nslots"] == 3 and st["nbnd"] == 3
    assert st["vol_cells"] == 0.5


def test_calls_without_a_device_fail_cleanly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(vcx.VcxError) as e:
        vcx.Mesh(wl.sod_tube(10, 3), stream=0)
    assert e.value.code == vcx.E_HIP
