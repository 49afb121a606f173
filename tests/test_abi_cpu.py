"""C-ABI library checks that need no GPU: the library loads, exports every
symbol include/hyb.h declares, and host-side validation (run through
hyb_footprint, which allocates nothing) rejects bad inputs with the
documented status codes."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hyb():
    from paper_1509_01399_amd import build, hyb
    if not os.path.exists(hyb.LIB_PATH):
        build.build()
    hyb.load()
    return hyb


def _declared():
    src = open(os.path.join(ROOT, "include", "hyb.h")).read()
    return sorted(set(re.findall(r"\b(hyb_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported(hyb):
    lib = hyb.load()
    names = _declared()
    assert "hyb_create" in names and "hyb_cg_step" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(hyb.EXPORTS)


def _mesh(hyb, o, C, h):
    from paper_1509_01399_amd import synth
    return hyb.make_mesh(*synth.kuhn_box_mesh(o, C, h))


def test_footprint_valid(hyb):
    g = hyb.make_grid(40)
    b = hyb.hyb_footprint(g, _mesh(hyb, 12, 16, 1 / 40), 2, hyb.make_opts(), 300)
    assert b > 6 * 41 ** 3 * 8


def test_reject_overlap_width(hyb):
    with pytest.raises(hyb.HybError) as e:
        hyb.hyb_footprint(hyb.make_grid(40), _mesh(hyb, 12, 16, 1 / 40), 3, None, 10)
    assert e.value.status == hyb.HYB_E_UNSUPPORTED


def test_reject_mesh_off_grid(hyb):
    from paper_1509_01399_amd import synth
    xyz, tet = synth.kuhn_box_mesh(12, 16, 1 / 40)
    xyz = xyz + 0.3 / 40
    with pytest.raises(hyb.HybError) as e:
        hyb.hyb_footprint(hyb.make_grid(40), hyb.make_mesh(xyz, tet), 2, None, 10)
    assert e.value.status == hyb.HYB_E_MESH


def test_reject_mesh_touching_boundary(hyb):
    with pytest.raises(hyb.HybError) as e:
        hyb.hyb_footprint(hyb.make_grid(20), _mesh(hyb, 0, 8, 1 / 20), 2, None, 10)
    assert e.value.status == hyb.HYB_E_MESH


def test_reject_non_kuhn_tets(hyb):
    from paper_1509_01399_amd import synth
    xyz, tet = synth.kuhn_box_mesh(6, 8, 1 / 20)
    tet = tet.copy()
    tet[0, 3] = tet[0, 2] + 2  # breaks the first tetrahedron
    with pytest.raises(hyb.HybError) as e:
        hyb.hyb_footprint(hyb.make_grid(20), hyb.make_mesh(xyz, tet), 2, None, 10)
    assert e.value.status in (hyb.HYB_E_UNSUPPORTED, hyb.HYB_E_MESH, hyb.HYB_E_ARG)


def test_reject_missing_tet(hyb):
    from paper_1509_01399_amd import synth
    xyz, tet = synth.kuhn_box_mesh(6, 8, 1 / 20)
    tet = tet.copy()
    tet[5] = tet[4]  # duplicate: one cube loses a tetrahedron
    with pytest.raises(hyb.HybError) as e:
        hyb.hyb_footprint(hyb.make_grid(20), hyb.make_mesh(xyz, tet), 2, None, 10)
    assert e.value.status == hyb.HYB_E_MESH


def test_reject_bad_grid(hyb):
    with pytest.raises(hyb.HybError) as e:
        hyb.hyb_footprint(hyb.make_grid(1), None, 2, None, 10)
    assert e.value.status == hyb.HYB_E_ARG
    with pytest.raises(hyb.HybError) as e:
        hyb.hyb_footprint(hyb.make_grid(10, bc=(2, 0, 0, 0, 0, 0)), None, 2, None, 10)
    assert e.value.status == hyb.HYB_E_UNSUPPORTED


def test_permuted_mesh_accepted(hyb):
    """The mesh may list nodes and tetrahedra in any order."""
    from paper_1509_01399_amd import synth
    xyz, tet = synth.kuhn_box_mesh(6, 8, 1 / 20)
    rng = np.random.default_rng(0)
    perm = rng.permutation(len(xyz))
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    xyz2 = xyz[perm]
    tet2 = inv[tet][rng.permutation(len(tet))]
    b = hyb.hyb_footprint(hyb.make_grid(20), hyb.make_mesh(xyz2, tet2.astype(np.int32)), 2, None, 10)
    assert b > 0
