"""Pin of the oracle's local matrices B_i (paper Section 3, equation (ORAS)):
B_i must be the Maxwell operator of T_i^delta taken as a mesh of its own,
with the physical conditions on its faces that lie on the chamber boundary
and the impedance transmission condition i k (E x n).(v x n) on every other
face of its boundary, k = k0 sqrt(Re eps_r) of the tetrahedron that owns the
face.

The expected matrix comes from a different path than oracle/dd.py: the test
finds T_i^delta and its boundary faces itself (Python sets over the
tetrahedra), then calls the whole-problem assembly fem.build on that
sub-mesh, each interface face tagged as an impedance aperture whose beta is
the owner's k (fem.build's +i beta sign and face mass are pinned by the
plane-wave convergence test).  Globally PEC edges are then removed, as
R_i restricts to the free unknowns.  A wrong face set, a wrong sign of the
term, or a different k (complex sqrt(eps), the neighbour's permittivity)
changes entries by O(|k| h) and fails the 1e-14 comparison.  CPU only."""
import numpy as np
import pytest

import mw_inputs as mi
from oracle import dd, fem

FACE_SLOTS = ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3))


class _Aperture:
    """Stand-in port record: fem.build reads only beta from a port."""

    def __init__(self, beta):
        self.beta = complex(beta)


def _overlap_tets(tet, part, i, delta):
    """T_i^delta by vertex adjacency, grown one layer at a time with sets."""
    inside = set(np.nonzero(part == i)[0].tolist())
    for _ in range(delta):
        nodes = {int(v) for t in inside for v in tet[t]}
        inside |= {t for t in range(tet.shape[0]) if any(int(v) in nodes for v in tet[t])}
    return np.array(sorted(inside))


def _expected_local_matrix(w, fp, tets):
    tet = np.sort(w.mesh.tet, axis=1)
    count, owner = {}, {}
    for t in tets:
        for sl in FACE_SLOTS:
            key = tuple(int(tet[t, s]) for s in sl)
            count[key] = count.get(key, 0) + 1
            owner[key] = int(t)
    phys = {tuple(sorted(int(v) for v in f)): int(g) for f, g in zip(w.mesh.bface, w.mesh.btag)}
    faces, tags = [], []
    ports = [_Aperture(p.beta) for p in w.ports]
    for key, c in count.items():
        if c != 1:
            continue
        faces.append(key)
        if key in phys:
            tags.append(phys[key])
        else:
            ports.append(_Aperture(fp.k0 * np.sqrt(w.eps[owner[key]].real)))
            tags.append(len(ports))
    sub = mi.mesh.Mesh(xyz=w.mesh.xyz, tet=tet[tets].astype(np.int32), bface=np.array(faces, dtype=np.int32),
                       btag=np.array(tags, dtype=np.int32), cell_of_tet=np.zeros(len(tets), dtype=np.int32),
                       cell_ijk=np.zeros((1, 3), dtype=np.int32))
    loc = fem.build(sub, w.eps[tets], w.k0, w.beta_imp, ports)
    # local free edges -> global edge -> global free unknown (-1: PEC somewhere)
    gedge = fem.edge_ids(fp.edges, fp.nv, loc.edges[loc.free, 0], loc.edges[loc.free, 1])
    gdof = fp.dof[gedge]
    keep = gdof >= 0
    return gdof[keep], loc.A.tocsr()[keep][:, keep].toarray()


@pytest.mark.parametrize("delta,subs", [(1, (0, 5)), (2, (3,))])
def test_local_matrix_is_the_submesh_operator_with_transmission_faces(delta, subs):
    w = mi.configs.small_chamber(0.25e9, n_per_ring=8, n_sub=8)
    fp = fem.build(w.mesh, w.eps, w.k0, w.beta_imp, w.ports)
    # heterogeneous permittivity (phantom), so the owner of a face matters
    assert np.unique(w.eps.real).size > 100
    got = dd.decompose(fp, w.part, delta, factor=False, subset=list(subs))
    for i, s in zip(subs, got):
        tets = _overlap_tets(np.sort(w.mesh.tet, axis=1), w.part, i, delta)
        np.testing.assert_array_equal(np.sort(s.tets), tets)
        gdof, Bexp = _expected_local_matrix(w, fp, tets)
        assert sorted(gdof.tolist()) == sorted(s.gdof.tolist())
        pos = {int(g): k for k, g in enumerate(s.gdof)}
        perm = np.array([pos[int(g)] for g in gdof])
        Bdd = s.B.toarray()[np.ix_(perm, perm)]
        scale = np.abs(Bexp).max()
        assert np.abs(Bdd - Bexp).max() <= 1e-14 * scale, np.abs(Bdd - Bexp).max() / scale
