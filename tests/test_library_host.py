"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/mw.h declares, and its host-side topology and overlapping
decomposition equal the oracle's (no device calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

import mw_inputs as mi
from oracle import dd, fem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1607_02573_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libmw.so is not built: run `python -m paper_1607_02573_amd.build`")
    return binding.lib()


def test_exports_every_declared_symbol(L):
    hdr = open(os.path.join(ROOT, "include", "mw.h")).read()
    declared = set(re.findall(r"^\s*(?:mw_status|const char \*)\s*(mw_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(L, name), name
        assert isinstance(getattr(L, name), ctypes._CFuncPtr)


@pytest.mark.parametrize("which", ["cube8", "small_chamber"])
def test_host_topology_matches_oracle(L, which):
    from paper_1607_02573_amd import binding
    w = mi.configs.cube8() if which == "cube8" else mi.configs.small_chamber(0.25e9, n_per_ring=8)
    m = w.mesh
    top = binding.host_topology(m.xyz, m.tet, m.bface, m.btag)
    fp = fem.build(m, w.eps, w.k0, w.beta_imp, w.ports)
    A = fp.A.tocsr()
    A.sort_indices()
    assert top["n"] == fp.n and top["n_edges"] == fp.edges.shape[0]
    assert np.array_equal(top["edge_of_dof"], fp.free)
    assert np.array_equal(top["row_ptr"], A.indptr) and np.array_equal(top["col"], A.indices)


def test_host_topology_is_order_independent(L):
    """Vertex order inside tetrahedra and faces does not change the numbering."""
    from paper_1607_02573_amd import binding
    m = mi.mesh.cube_mesh(3)
    rng = np.random.default_rng(0)
    tet = np.array([rng.permutation(t) for t in m.tet])
    bf = np.array([rng.permutation(f) for f in m.bface])
    a = binding.host_topology(m.xyz, m.tet, m.bface, m.btag)
    b = binding.host_topology(m.xyz, tet, bf, m.btag)
    for k in ("edge_of_dof", "row_ptr", "col"):
        assert np.array_equal(a[k], b[k])


@pytest.mark.parametrize("which,nsub", [("cube8", 8), ("cube8", 5), ("small_chamber", 8)])
def test_host_decomposition_matches_oracle(L, which, nsub):
    from paper_1607_02573_amd import binding
    w = mi.configs.cube8() if which == "cube8" else mi.configs.small_chamber(0.25e9, n_per_ring=8)
    m = w.mesh
    part = mi.partition.rcb(m, nsub)
    dec = binding.host_decomposition(m.xyz, m.tet, m.bface, m.btag, part, nsub, 1)
    fp = fem.build(m, w.eps, w.k0, w.beta_imp, w.ports)
    subs = dd.decompose(fp, part, 1, factor=False)
    for i, s in enumerate(subs):
        # same unknowns and weights; the library numbers zero-weight unknowns first
        o = np.argsort(dec["sub_dof"][i], kind="stable")
        assert np.array_equal(dec["sub_dof"][i][o], s.gdof)
        np.testing.assert_allclose(dec["D"][i][o], s.D, rtol=0, atol=1e-15)
        nz = dec["D"][i] > 0
        lead = int((~nz).sum())
        assert not nz[:lead].any() and nz[lead:].all()
        assert np.all(np.diff(dec["sub_dof"][i][:lead]) > 0) and np.all(np.diff(dec["sub_dof"][i][lead:]) > 0)
    # partition of unity: sum_i R_i^T D_i R_i = I
    tot = np.zeros(fp.n)
    for i in range(nsub):
        np.add.at(tot, dec["sub_dof"][i], dec["D"][i])
    np.testing.assert_allclose(tot, 1.0, atol=1e-15)


def test_host_decomposition_overlap_two(L):
    from paper_1607_02573_amd import binding
    w = mi.configs.cube(4, n_sub=4)
    m = w.mesh
    fp = fem.build(m, w.eps, w.k0, w.beta_imp, w.ports)
    dec = binding.host_decomposition(m.xyz, m.tet, m.bface, m.btag, w.part, 4, 2)
    subs = dd.decompose(fp, w.part, 2, factor=False)
    for i, s in enumerate(subs):
        o = np.argsort(dec["sub_dof"][i], kind="stable")
        assert np.array_equal(dec["sub_dof"][i][o], s.gdof)
        np.testing.assert_allclose(dec["D"][i][o], s.D, atol=1e-15)


def test_host_error_paths(L):
    from paper_1607_02573_amd import binding
    m = mi.mesh.cube_mesh(2)
    bad = m.tet.copy()
    bad[0, 0] = 10_000
    with pytest.raises(binding.MwError) as e:
        binding.host_topology(m.xyz, bad, m.bface, m.btag)
    assert e.value.code == binding.MW_EINVAL
    deg = m.tet.copy()
    deg[0, 1] = deg[0, 0]
    with pytest.raises(binding.MwError):
        binding.host_topology(m.xyz, deg, m.bface, m.btag)
    # an interior face labelled as boundary
    interior = np.array([[m.tet[0, 0], m.tet[0, 1], m.tet[0, 3]]], dtype=np.int32)
    with pytest.raises(binding.MwError):
        binding.host_topology(m.xyz, m.tet, np.r_[m.bface, interior], np.r_[m.btag, 0])
    part = np.zeros(m.nt, dtype=np.int32)
    with pytest.raises(binding.MwError) as e:
        binding.host_decomposition(m.xyz, m.tet, m.bface, m.btag, part, 2, 1)   # part 1 empty
    assert e.value.code == binding.MW_EINVAL


def test_library_missing_fails_loudly(tmp_path, monkeypatch):
    from paper_1607_02573_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(binding.MwLibraryMissing):
        binding.lib()
