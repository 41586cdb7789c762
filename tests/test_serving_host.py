"""CPU tests of the serving inputs and of the admission bookkeeping."""
import numpy as np

import mw_inputs as mi


def test_request_stream_is_seeded_and_shaped():
    a = mi.serving.serving_requests()
    b = mi.serving.serving_requests()
    assert len(a) == 400
    assert [r.t_arrive for r in a] == [r.t_arrive for r in b]
    t = np.array([r.t_arrive for r in a])
    assert np.all(np.diff(t) > 0)
    # Poisson rate 4/s: mean gap 0.25 s within sampling error
    assert abs(np.diff(np.r_[0, t]).mean() - 0.25) < 0.05
    kinds = np.array([r.kind == "gradient" for r in a])
    assert 0.18 < kinds.mean() < 0.32
    for r in a:
        assert r.tx.size == np.unique(r.tx).size
        assert 1 <= r.ncols <= (32 if r.kind == "gradient" else 160)
        assert r.mesh in range(4) and r.version in range(2)
        if r.kind == "gradient":
            assert r.s_meas.shape == (160, r.ncols)
    n = np.array([r.ncols for r in a if r.kind == "solve"])
    # log-uniform on [1, 160]: about half the requests at or below sqrt(161)
    assert 0.35 < (n <= 13).mean() < 0.65


def test_edge_count_of_one_kuhn_cube():
    m = mi.mesh.cube_mesh(1)
    assert mi.serving.count_edges(m.tet) == 19
    m = mi.mesh.cube_mesh(2)
    assert mi.serving.count_edges(m.tet) == 98


def test_admission_bookkeeping():
    from paper_1607_02573_amd.serve import Admission
    a = Admission(budget=1000, base=100)
    a.add_problem("A", factor_bytes=300, slot_bytes=20, bytes_per_col=10, max_cols=16)
    a.add_problem("B", factor_bytes=400, slot_bytes=30, bytes_per_col=20, max_cols=16)
    assert a.total() == 100
    assert a.delta("A", 4) == 300 + 20 + 40
    assert a.fits("A", 4)
    a.admit("A", 4, now=1.0)
    assert a.total() == 100 + 320 + 40
    assert a.delta("A", 2) == 20                     # peak grows by 2 columns
    assert not a.fits("A", 13)                       # slot capacity
    assert a.delta("B", 8) == 430 + 160
    assert not a.fits("B", 8)                        # 460 + 590 > 1000
    assert a.victims("B", 50, busy=set()) == []      # A has open columns
    a.finish("A", 4)
    assert a.total() == 100 + 320                    # workspace freed when idle
    assert a.victims("B", 50, busy=set()) == ["A"]
    assert a.victims("B", 50, busy={"A"}) == []
    a.evicted("A")
    assert a.total() == 100 and a.fits("B", 8)
    assert a.group_cols("B") == min(16, (1000 - 100 - 430) // 20)


def test_dispatch_first_fit_then_eviction():
    """The dispatcher admits in arrival order what fits, and lets the oldest
    blocked group evict idle factors (no GPU: slots are stand-ins)."""
    import threading
    from collections import deque

    from paper_1607_02573_amd.serve import Admission, Group, Outcome, Server

    class Slot:
        def __init__(self):
            self.inbox, self.tags, self.evict = deque(), {}, False

    srv = object.__new__(Server)
    srv.cond = threading.Condition()
    srv.adm = Admission(budget=1000, base=100)
    srv.adm.add_problem((0, 0), 300, 20, 10, 16)
    srv.adm.add_problem((1, 0), 400, 30, 20, 16)
    srv.slots = {(0, 0): Slot(), (1, 0): Slot()}
    mk = mi.serving.Request
    reqs = [mk(0, 0.0, 0, 0, "solve", np.arange(6, dtype=np.int32), np.arange(8, dtype=np.int32)),
            mk(1, 0.1, 1, 0, "solve", np.arange(8, dtype=np.int32), np.arange(8, dtype=np.int32)),
            mk(2, 0.2, 0, 0, "solve", np.arange(3, dtype=np.int32), np.arange(8, dtype=np.int32))]
    srv.outcomes = {r.rid: Outcome(r.rid, r.kind, r.mesh, r.version, r.ncols, r.t_arrive) for r in reqs}
    groups = [Group(r, np.arange(r.ncols)) for r in reqs]
    pending = deque(groups)
    with srv.cond:
        srv._admit(pending, 1.0)
    # request 0 and 2 (problem (0,0)) fit; request 1 needs 430 + 160 more bytes
    assert list(pending) == [groups[1]]
    assert list(srv.slots[(0, 0)].inbox) == [groups[0], groups[2]]
    assert srv.outcomes[0].t_admit == 1.0 and srv.outcomes[1].t_admit < 0
    assert not srv.slots[(0, 0)].evict          # (0,0) is busy: no victim yet
    # both finish; (0,0) idles with its factors resident
    srv.slots[(0, 0)].inbox.clear()
    srv.adm.finish((0, 0), 6)
    srv.adm.finish((0, 0), 3)
    with srv.cond:
        srv._admit(pending, 2.0)
    assert list(pending) == [groups[1]] and srv.slots[(0, 0)].evict
    srv.adm.evicted((0, 0))
    srv.slots[(0, 0)].evict = False
    with srv.cond:
        srv._admit(pending, 3.0)
    assert not pending and list(srv.slots[(1, 0)].inbox) == [groups[1]]
    assert srv.adm.total() == 100 + 430 + 160
