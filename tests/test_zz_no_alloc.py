"""The allocation-free apply (spand_apply_noalloc) against spand_apply.

Two calls in a row on the same device's fixed scratch, the second with a
smaller input (another problem's factor, fewer columns): each must give what
spand_apply gives on the same factor and vectors (the same kernels; columns
are independent, so only the chunking may differ).  A handle of a batch factor
is refused.
"""
import numpy as np
import pytest

from synthetic import laplacian_2d, laplacian_3d, rhs

gpu = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.asfortranarray(a).reshape(-1, order="F").copy()).to("cuda")


@gpu
def test_apply_noalloc_matches_apply_on_two_calls():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_00789_amd import spand
    ctx = spand.Context(0)
    cases = [(laplacian_3d(20), 7, 2, 3), (laplacian_2d(40), 5, 1, 1)]   # second: smaller input
    for p, depth, skip, nrhs in cases:
        print(f"noalloc apply n={p.n} nrhs={nrhs}", flush=True)
        opts = spand.make_opts(depth=depth, skip=skip, eps=1e-2, scheme="SO")
        plan = spand.analyze(p.n, p.rowptr, p.colind, p.coords, opts, ctx)
        fac = ctx.factor(plan, _dev(p.vals), opts)
        x = _dev(rhs(p.n, nrhs, 31 + nrhs))
        y_ref = torch.zeros_like(x)
        y = torch.full_like(x, np.nan)
        ctx.apply(fac, nrhs, x, y_ref)
        ctx.apply_noalloc(fac, nrhs, x, y)
        a, b = y.cpu().numpy(), y_ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(b)
        fac.close()
        plan.close()


@gpu
def test_apply_noalloc_refuses_a_batch_handle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_00789_amd import spand
    ctx = spand.Context(0)
    p, q = laplacian_2d(24), laplacian_2d(20)
    plans = [spand.analyze(r.n, r.rowptr, r.colind, r.coords,
                           spand.make_opts(depth=3, skip=1, eps=1e-2)) for r in (p, q)]
    facs = ctx.factor_batch(plans, [_dev(p.vals), _dev(q.vals)], spand.make_opts(skip=1, eps=1e-2))
    x = _dev(rhs(p.n, 1, 5))
    with pytest.raises(spand.SpandError) as e:
        ctx.apply_noalloc(facs[0], 1, x, torch.zeros_like(x))
    assert e.value.status == -1
