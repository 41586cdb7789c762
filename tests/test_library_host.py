"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/mw.h declares, and its host-side topology and overlapping
decomposition equal the oracle's (no device calls)."""
import ctypes
import os
import re

import numpy as np
from scipy.sparse.csgraph import reverse_cuthill_mckee
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


def _envelope(B):
    """Sum over the rows of (row index - first nonzero column), lower part."""
    B = B.tocsr()
    first = np.array([min(B.indices[B.indptr[r]:B.indptr[r + 1]].min(), r) for r in range(B.shape[0])])
    return int(np.sum(np.arange(B.shape[0]) - first))


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
        # same unknowns and weights, in the library's banded local order
        o = np.argsort(dec["sub_dof"][i], kind="stable")
        assert np.array_equal(dec["sub_dof"][i][o], s.gdof)
        np.testing.assert_allclose(dec["D"][i][o], s.D, rtol=0, atol=1e-15)
        # reverse Cuthill-McKee: the envelope of B_i (sum over rows of the
        # distance from the first nonzero to the diagonal) is as small as
        # with scipy's implementation of the same method
        pos = np.searchsorted(s.gdof, dec["sub_dof"][i])
        B = s.B.tocsr()
        rc = reverse_cuthill_mckee(B, symmetric_mode=True)
        assert _envelope(B[pos][:, pos]) <= 1.05 * _envelope(B[rc][:, rc])
    # partition of unity: sum_i R_i^T D_i R_i = I
    tot = np.zeros(fp.n)
    for i in range(nsub):
        np.add.at(tot, dec["sub_dof"][i], dec["D"][i])
    np.testing.assert_allclose(tot, 1.0, atol=1e-15)


def test_factorisation_fills_only_the_envelope(L):
    """The triangular solves and the L D L^T updates skip every product
    outside the envelope of B_i in the library's local order: elimination
    without interchanges (numpy, row by row) leaves L[r, c] = 0 for c left of
    the first coupled column of row r and U[r, c] = 0 above that of column c,
    exactly (George & Liu's envelope theorem)."""
    from paper_1607_02573_amd import binding
    w = mi.configs.cube8()
    m = w.mesh
    part = mi.partition.rcb(m, 8)
    dec = binding.host_decomposition(m.xyz, m.tet, m.bface, m.btag, part, 8, 1)
    fp = fem.build(m, w.eps, w.k0, w.beta_imp, w.ports)
    s = dd.decompose(fp, part, 1, factor=False)[0]
    pos = np.searchsorted(s.gdof, dec["sub_dof"][0])
    F = s.B.tocsr()[pos][:, pos].toarray()
    n = F.shape[0]
    first = np.array([min(np.nonzero(F[r])[0].min(), r) for r in range(n)])
    for k in range(n - 1):
        F[k + 1:, k] /= F[k, k]
        F[k + 1:, k + 1:] -= np.outer(F[k + 1:, k], F[k, k + 1:])
    outside = np.arange(n)[None, :] < first[:, None]       # (r, c) left of row r's envelope
    assert not F[outside].any() and not F.T[outside].any()
    assert outside.sum() > 0.5 * n * (n - 1) / 2            # most of the triangle lies outside


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
    # block least squares: width outside [1, 32], or no S0 with steps > 0
    H = np.zeros((64, 32), dtype=np.complex128)
    with pytest.raises(binding.MwError) as e:
        binding.host_block_lstsq(np.eye(32), H, width=33)
    assert e.value.code == binding.MW_EINVAL
    with pytest.raises(binding.MwError) as e:
        binding.check(L.mw_host_block_lstsq(1, 32, None, binding.ptr(H), 0.0, None, None), True)
    assert e.value.code == binding.MW_EINVAL


def test_library_missing_fails_loudly(tmp_path, monkeypatch):
    from paper_1607_02573_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(binding.MwLibraryMissing):
        binding.lib()


def _block_hessenberg(rng, steps, width=32):
    """Random block upper Hessenberg matrix with upper-triangular
    sub-diagonal blocks; columns and rows beyond `width` in every block are
    padding (identity on the sub-diagonal, zero elsewhere) as the solver
    builds them."""
    q = 32
    H = np.zeros(((steps + 1) * q, steps * q), dtype=np.complex128)
    for j in range(steps):
        for i in range(j + 1):
            blk = rng.normal(size=(q, q)) + 1j * rng.normal(size=(q, q))
            blk[width:, :] = 0
            blk[:, width:] = 0
            H[i * q:(i + 1) * q, j * q:(j + 1) * q] = blk
        R = np.triu(rng.normal(size=(q, q)) + 1j * rng.normal(size=(q, q))) + 4 * np.eye(q)
        R[width:, :] = 0
        R[:, width:] = 0
        R[np.arange(width, q), np.arange(width, q)] = 1
        H[(j + 1) * q:(j + 2) * q, j * q:(j + 1) * q] = R
    S0 = np.triu(rng.normal(size=(q, q)) + 1j * rng.normal(size=(q, q)))
    S0[width:, :] = 0
    S0[:, width:] = 0
    S0[np.arange(width, q), np.arange(width, q)] = 1
    return S0, H


@pytest.mark.parametrize("width", [32, 7])
def test_host_block_least_squares_matches_lstsq(L, width):
    """The library's incremental Householder least squares of block GMRES
    equals a dense least-squares solve after every block column."""
    from paper_1607_02573_amd import binding
    rng = np.random.default_rng(width)
    steps = 4
    S0, H = _block_hessenberg(rng, steps, width)
    res, Y = binding.host_block_lstsq(S0, H, width)
    q = 32
    E = np.zeros(((steps + 1) * q, q), dtype=np.complex128)
    E[:q] = S0
    E[:, width:] = 0
    for j in range(steps):
        Hj = H[:(j + 2) * q, :(j + 1) * q]
        Yj = np.linalg.lstsq(Hj, E[:(j + 2) * q], rcond=None)[0]
        want = np.linalg.norm(E[:(j + 2) * q] - Hj @ Yj, axis=0)
        np.testing.assert_allclose(res[j, :width], want[:width], rtol=1e-9, atol=1e-12 * np.abs(E).max())
    np.testing.assert_allclose(Y[:, :width], Yj[:, :width], rtol=1e-9, atol=1e-10 * np.abs(Yj).max())


def test_host_block_cholesky(L):
    """Cholesky factor R^H R = G, and rank deficiency counted."""
    from paper_1607_02573_amd import binding
    rng = np.random.default_rng(3)
    W = rng.normal(size=(200, 32)) + 1j * rng.normal(size=(200, 32))
    G = W.conj().T @ W
    R, nd = binding.host_block_cholesky(G, 1e-10)
    assert nd == 0
    np.testing.assert_allclose(np.triu(R), R)
    np.testing.assert_allclose(R.conj().T @ R, G, rtol=1e-12, atol=1e-12 * np.abs(G).max())
    # a column dependent up to 1e-9 (below the 1e-7 threshold, near the
    # square root of the unit roundoff that a Gram-based factor resolves)
    # counts as deficient; one 1e-5 away does not
    W2 = W.copy()
    W2[:, 5] = W[:, 2] + 1e-9 * np.linalg.norm(W[:, 2]) * W[:, 9] / np.linalg.norm(W[:, 9])
    _, nd = binding.host_block_cholesky(W2.conj().T @ W2, 1e-7)
    assert nd == 1
    W2[:, 5] = W[:, 2] + 1e-5 * np.linalg.norm(W[:, 2]) * W[:, 9] / np.linalg.norm(W[:, 9])
    _, nd = binding.host_block_cholesky(W2.conj().T @ W2, 1e-7)
    assert nd == 0


@pytest.mark.parametrize("which,nsub", [("cube8", 8), ("cube8", 7), ("small_chamber", 13)])
def test_internal_partition_is_balanced_and_decomposes_like_the_oracle(L, which, nsub):
    """tet_part = NULL: the library's recursive coordinate bisection of the
    centroids.  Every part holds floor(nt/nsub) or one more tetrahedron, the
    parts are geometrically compact (each part's centroid bounding box is far
    smaller than the mesh's), a shuffled vertex order inside the tetrahedra
    gives the same parts, and the overlapping decomposition built on it
    equals the oracle's on the same partition."""
    from paper_1607_02573_amd import binding
    w = mi.configs.cube8() if which == "cube8" else mi.configs.small_chamber(0.25e9, n_per_ring=8)
    m = w.mesh
    part = binding.host_partition(m.xyz, m.tet, m.bface, m.btag, nsub)
    cnt = np.bincount(part, minlength=nsub)
    assert part.min() == 0 and part.max() == nsub - 1
    assert set(cnt.tolist()) <= {m.nt // nsub, m.nt // nsub + 1}
    cen = m.xyz[m.tet].mean(axis=1)
    vol_all = np.prod(cen.max(axis=0) - cen.min(axis=0))
    for i in range(nsub):
        c = cen[part == i]
        assert np.prod(c.max(axis=0) - c.min(axis=0)) < 2.5 * vol_all / nsub
    rng = np.random.default_rng(3)
    tet_sh = np.array([rng.permutation(t) for t in m.tet])
    assert np.array_equal(binding.host_partition(m.xyz, tet_sh, m.bface, m.btag, nsub), part)
    dec = binding.host_decomposition(m.xyz, m.tet, m.bface, m.btag, part, nsub, 1)
    fp = fem.build(m, w.eps, w.k0, w.beta_imp, w.ports)
    for i, s in enumerate(dd.decompose(fp, part, 1, factor=False)):
        o = np.argsort(dec["sub_dof"][i], kind="stable")
        assert np.array_equal(dec["sub_dof"][i][o], s.gdof)
        np.testing.assert_allclose(dec["D"][i][o], s.D, rtol=0, atol=1e-15)
    with pytest.raises(Exception):
        binding.host_partition(m.xyz, m.tet, m.bface, m.btag, m.nt + 1)


def test_banded_factor_storage_holds_the_elimination(L):
    """The banded factor storage (factorisation without interchanges): every
    64-row block stores a column range that contains every nonzero that
    elimination without interchanges (numpy, in the library's local order)
    produces in its rows, at least 64 columns past its diagonal block, and
    the whole storage is far smaller than dense."""
    from paper_1607_02573_amd import binding
    w = mi.configs.cube8()
    m = w.mesh
    fp = fem.build(m, w.eps, w.k0, w.beta_imp, w.ports)
    dec = binding.host_decomposition(m.xyz, m.tet, m.bface, m.btag, w.part, 8, 1)
    subs = dd.decompose(fp, w.part, 1, factor=False)
    for sub in (0, 5):
        dense, band, lo, hi = binding.host_factor_storage(m.xyz, m.tet, m.bface, m.btag, w.part, 8, 1, sub)
        s = subs[sub]
        pos = np.searchsorted(s.gdof, dec["sub_dof"][sub])
        F = s.B.tocsr()[pos][:, pos].toarray()
        n = F.shape[0]
        for k in range(n - 1):
            F[k + 1:, k] /= F[k, k]
            F[k + 1:, k + 1:] -= np.outer(F[k + 1:, k], F[k, k + 1:])
        npad = 64 * len(lo)
        assert npad >= n and len(lo) == (n + 63) // 64
        for b in range(len(lo)):
            rows = F[64 * b:64 * b + 64]
            nzc = np.nonzero(rows.any(axis=0))[0]
            assert lo[b] % 64 == 0 and hi[b] % 64 == 0 or hi[b] == npad
            assert lo[b] <= 64 * b and hi[b] >= min(npad, 64 * b + 128)
            assert nzc.min() >= lo[b] and nzc.max() < hi[b]
    assert band < 0.75 * dense
    # on the larger chamber subdomains the band is a small part of dense storage
    ws = mi.configs.small_chamber(0.25e9, n_per_ring=8, n_sub=8)
    ms = ws.mesh
    dense, band, _, _ = binding.host_factor_storage(ms.xyz, ms.tet, ms.bface, ms.btag, ws.part, 8, 1, 0)
    assert band < 0.4 * dense
