"""GPU check of mw_apply_preconditioner_noalloc (the entry point for callers
that cannot allocate): through the C ABI it gives, bit for bit, what
mw_apply_preconditioner gives on the same factors, on two calls in a row
(the second smaller, so stale contents of the shared fixed buffer would
show), for FP32 and FP64 factors, and it refuses sizes beyond its fixed
buffer with MW_EINVAL."""
import numpy as np
import pytest

import mw_inputs as mi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def small():
    from paper_1607_02573_amd import solver
    ctx = solver.Context(0)
    w = mi.configs.small_chamber(0.25e9, n_per_ring=8, n_sub=8)
    P = solver.problem_from_workload(ctx, w)
    yield w, P
    P.close()
    ctx.close()


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_noalloc_apply_equals_allocating_apply(small, prec):
    from paper_1607_02573_amd import binding
    w, P = small
    print(f"[noalloc] {prec}: factor, two calls (9 then 3 columns)", flush=True)
    P.factor(w.part, w.n_sub, 1, prec)
    rng = np.random.default_rng(31)
    for nc in (9, 3):
        V = torch.from_numpy(rng.normal(size=(P.n, nc)) + 1j * rng.normal(size=(P.n, nc))).cuda()
        Z_ref = P.apply_preconditioner(V)
        Z = torch.full_like(V, complex(np.nan, np.nan))
        P.apply_preconditioner_noalloc(V, Z)
        torch.cuda.synchronize()
        assert torch.equal(Z, Z_ref), (prec, nc)
    # more columns than the fixed buffer holds: a clear MW_EINVAL, Z untouched
    esz = 8 if prec == "c64" else 16
    sum_ni = P.info().sum_ni                  # <= the padded sum the buffer must hold
    nbig = binding.NOALLOC_SCRATCH_BYTES // (esz * sum_ni) + 1
    V = torch.zeros((P.n, nbig), dtype=torch.complex128, device="cuda")
    Z = torch.zeros_like(V)
    with pytest.raises(binding.MwError) as e:
        P.apply_preconditioner_noalloc(V, Z)
    assert e.value.code == binding.MW_EINVAL and "fixed buffer" in str(e.value)
