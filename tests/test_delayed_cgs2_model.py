"""CPU model of the Arnoldi recurrence the library's GMRES runs (Gram-Schmidt
applied twice, the second pass of each new vector delayed to the next step,
and with the FP32 basis the next candidate kept unnormalised in memory),
written from the recurrence in numpy, and checked against what any Arnoldi
process must satisfy and against textbook classical Gram-Schmidt applied
twice (right-preconditioned GMRES, Section 6 of the paper; Saad, Iterative
Methods for Sparse Linear Systems, Alg. 6.9 and 9.5):

  * A M^-1 V_m = V_{m+1} H_m and V_{m+1}^H V_{m+1} = I (FP64, to rounding);
  * H_m equals the textbook CGS2 Arnoldi's Hessenberg matrix;
  * keeping the candidate unnormalised (its readers apply 1/||u||) gives the
    same H and V as normalising it in memory, and with a basis stored in
    FP32 both keep the Arnoldi relation and orthogonality at the FP32 level.

This pins the algebra of the delayed recurrence, not the device kernels; the
GPU tests compare the kernels' iteration counts and solutions with the
oracle's textbook GMRES.  CPU only.
"""
import numpy as np
import pytest

RNG = np.random.default_rng(2024)


def _problem(n=240):
    A = np.eye(n) + 0.6 * (RNG.normal(size=(n, n)) + 1j * RNG.normal(size=(n, n))) / np.sqrt(n)
    Minv = np.diag(1.0 / (1.0 + 0.3 * RNG.random(n)))   # a fixed right preconditioner
    r0 = RNG.normal(size=n) + 1j * RNG.normal(size=n)
    return A, Minv, r0


def _round(x, fp32):
    return x.astype(np.complex64).astype(np.complex128) if fp32 else x


def delayed_step(Vp, y, T, H, hprov_prev, beta):
    """One step j = len(Vp) of the delayed CGS2 recurrence.

    Vp: v_0 .. v_{j-1} (rows, orthonormal); y: the candidate of slot j as
    its readers see it (already times 1/||u||); T = op(y) or None (the
    finishing step); H: Hessenberg columns 0 .. j-2 (final); hprov_prev,
    beta: the provisional column j-1 and ||u|| of the previous step.
    The second pass writes y = nu v_j + sum_k a_k v_k.  Returns v_j, the
    final column j-1 (j+1 entries), the provisional column j (j+1 entries)
    and the next candidate u (unnormalised); the last two are None when T
    is None."""
    j = Vp.shape[0]
    a = Vp.conj() @ y
    alpha = np.vdot(y, y).real
    nu = 1.0 if j == 0 else np.sqrt(max(alpha - np.vdot(a, a).real, 0.0))
    col = None
    if j > 0:
        col = np.concatenate([hprov_prev + beta * a, [beta * nu]])
    vj = (y - a @ Vp) / nu
    if T is None:
        return vj, col, None, None
    b = Vp.conj() @ T
    e = (np.vdot(y, T) - np.vdot(a, b)) / nu
    d = np.concatenate([b, [e]])
    Hj = np.zeros((j + 1, j), dtype=np.complex128)   # op v_k = sum_i Hj[i, k] v_i, k < j
    if j > 0:
        Hj[:, : j - 1] = H[: j + 1, : j - 1]
        Hj[:, j - 1] = col
    hprov = (d - Hj @ a) / nu
    u = (T - b @ Vp - e * vj) / nu
    return vj, col, hprov, u


def delayed_arnoldi(op, r0, m, lazy, fp32=False):
    """m steps of the delayed CGS2 Arnoldi process on op = A M^-1.

    Step j applies op to the once-orthogonalised candidate y_j (slot j),
    computes [V_<j, y_j]^H y_j and [V_<j, y_j]^H op(y_j) in one sweep,
    finishes y_j, the final column j-1 of the Hessenberg matrix and the
    provisional column j, then writes v_j and the next candidate u (slot
    j+1) in one sweep.  lazy: u is stored as is and read times 1/||u||;
    else it is stored normalised.  fp32: every slot is stored rounded to
    complex FP32 (all arithmetic FP64)."""
    n = r0.size
    V = np.zeros((m + 1, n), dtype=np.complex128)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    V[0] = _round(r0 / np.linalg.norm(r0), fp32)
    sc, hn2, hprov = 1.0, None, None
    for j in range(m + 1):
        y = V[j] * sc                                  # the candidate as its readers see it
        T = op(y) if j < m else None
        vj, col, hprov_new, u = delayed_step(V[:j], y, T, H, hprov, None if j == 0 else np.sqrt(hn2))
        if j > 0:
            H[: j + 1, j - 1] = col
        if j == m:
            v_last = vj                                 # v_m, implied by the finished candidate
            break
        hprov = hprov_new
        V[j] = _round(vj, fp32)
        us = _round(u, fp32)
        hn2 = np.vdot(us, us).real
        if lazy:
            V[j + 1], sc = us, 1.0 / np.sqrt(hn2)
        else:
            V[j + 1], sc = _round(us / np.sqrt(hn2), fp32), 1.0
    Vm = np.vstack([V[:m], v_last[None, :]])
    return Vm, H


def textbook_arnoldi(op, r0, m):
    """Classical Gram-Schmidt applied twice per step."""
    n = r0.size
    V = np.zeros((m + 1, n), dtype=np.complex128)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    V[0] = r0 / np.linalg.norm(r0)
    for j in range(m):
        w = op(V[j])
        h = V[: j + 1].conj() @ w
        w = w - h @ V[: j + 1]
        h2 = V[: j + 1].conj() @ w
        w = w - h2 @ V[: j + 1]
        H[: j + 1, j] = h + h2
        H[j + 1, j] = np.linalg.norm(w)
        V[j + 1] = w / H[j + 1, j]
    return V, H


@pytest.mark.parametrize("lazy", [False, True])
def test_delayed_recurrence_is_an_arnoldi_process(lazy):
    A, Minv, r0 = _problem()
    op = lambda x: A @ (Minv @ x)   # noqa: E731
    m = 30
    V, H = delayed_arnoldi(op, r0, m, lazy)
    AV = np.stack([op(V[k]) for k in range(m)])
    rel = np.linalg.norm(AV - H.T @ V) / np.linalg.norm(H)
    assert rel <= 1e-13, rel
    orth = np.abs(V.conj() @ V.T - np.eye(m + 1)).max()
    assert orth <= 1e-13, orth
    Vt, Ht = textbook_arnoldi(op, r0, m)
    assert np.abs(H - Ht).max() <= 1e-12 * np.abs(Ht).max()
    assert np.abs(V - Vt).max() <= 1e-12


def test_unnormalised_candidate_changes_nothing_but_rounding():
    A, Minv, r0 = _problem()
    op = lambda x: A @ (Minv @ x)   # noqa: E731
    V0, H0 = delayed_arnoldi(op, r0, 30, lazy=False)
    V1, H1 = delayed_arnoldi(op, r0, 30, lazy=True)
    assert np.abs(H1 - H0).max() <= 1e-14 * np.abs(H0).max()
    assert np.abs(V1 - V0).max() <= 1e-14


@pytest.mark.parametrize("lazy", [False, True])
def test_fp32_basis_keeps_the_relation_at_fp32_level(lazy):
    """A basis stored in FP32, candidate normalised in memory or not: the
    relation and orthogonality hold to a small multiple of the FP32 unit
    roundoff (6e-8), and the two storage forms agree to that level."""
    A, Minv, r0 = _problem()
    op = lambda x: A @ (Minv @ x)   # noqa: E731
    m = 30
    V, H = delayed_arnoldi(op, r0, m, lazy, fp32=True)
    AV = np.stack([op(V[k]) for k in range(m)])
    rel = np.linalg.norm(AV - H.T @ V) / np.linalg.norm(H)
    assert rel <= 1e-6, rel
    orth = np.abs(V.conj() @ V.T - np.eye(m + 1)).max()
    assert orth <= 1e-6, orth
    _, H64 = delayed_arnoldi(op, r0, m, lazy=False)
    assert np.abs(H - H64).max() <= 1e-5 * np.abs(H64).max()


def test_breakdown_column_is_exact_zero():
    """A Krylov space that closes (op has a 3-dimensional invariant subspace
    holding r0): the subdiagonal entry after it vanishes to rounding."""
    n = 50
    Q, _ = np.linalg.qr(RNG.normal(size=(n, n)) + 1j * RNG.normal(size=(n, n)))
    D = np.diag(np.concatenate([[2.0, 3.0, 5.0], 7.0 + RNG.random(n - 3)]))
    A = Q @ D @ Q.conj().T
    r0 = Q[:, :3] @ np.array([1.0, 2.0, 3.0])
    op = lambda x: A @ x   # noqa: E731
    _, H = delayed_arnoldi(op, r0, 3, lazy=True)
    assert abs(H[3, 2]) <= 1e-12 * np.abs(H).max()


def test_one_step_against_an_exact_history():
    """One step from a history whose Arnoldi relation is exact by
    construction, with a candidate far from orthogonal to the basis (second
    pass coefficients of order 0.3, where each term of the step matters):
    v_j, the final column j-1, the provisional column j and the remainder u
    equal their exact values."""
    n, j = 60, 6
    Q, _ = np.linalg.qr(RNG.normal(size=(n, n)) + 1j * RNG.normal(size=(n, n)))
    G = RNG.normal(size=(n, n)) + 1j * RNG.normal(size=(n, n))
    G[:, :j] = np.triu(G[:, :j], -1)                  # op Q_k in span(Q_0..Q_{k+1}) for k < j
    op = lambda x: Q @ (G @ (Q.conj().T @ x))   # noqa: E731
    Vp = Q[:, :j].T
    # previous step: op v_{j-1} = sum_{i<j} hprov_i v_i + beta y, y = nu v_j + sum_k a_k v_k
    a_true = 0.3 * (RNG.normal(size=j) + 1j * RNG.normal(size=j))
    nu_true = 0.8
    beta = abs(G[j, j - 1]) / nu_true
    # pick the candidate so that beta y is op v_{j-1}'s remainder in direction j
    # and a_true in directions < j: y = nu v_j + V a
    ph = G[j, j - 1] / abs(G[j, j - 1])
    v_j = Q[:, j] * ph                                 # a unit vector orthogonal to V_<j
    y = nu_true * v_j + a_true @ Vp
    hprov_prev = G[:j, j - 1] - beta * a_true
    H = np.zeros((j + 1, j), dtype=np.complex128)
    H[: j + 1, : j - 1] = G[: j + 1, : j - 1]
    vj, col, hprov, u = delayed_step(Vp, y, op(y), H, hprov_prev, beta)
    tol = 1e-12 * np.abs(G).max()
    assert np.abs(vj - v_j).max() <= 1e-13
    assert np.abs(col - G[: j + 1, j - 1] * np.concatenate([np.ones(j), [np.conj(ph)]])).max() <= tol
    # exact projections of op v_j onto [V_<j, v_j] and the remainder
    w = op(v_j)
    B = np.vstack([Vp, v_j[None, :]])
    h_exact = B.conj() @ w
    assert np.abs(hprov - h_exact).max() <= tol
    assert np.abs(u - (w - h_exact @ B)).max() <= tol
