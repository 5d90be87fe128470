"""The allocation-free decision function (gabp_svm_predict_noalloc) against
gabp_svm_predict on the same solved machine: both run the same kernels on
the same staged inputs with the same launch shapes, so the values must agree
bit for bit -- on two calls in a row, the second with fewer queries (the
scratch array keeps the first call's contents), for every precision and Gram
kind.  A call whose working set exceeds the scratch array is refused."""
import numpy as np
import pytest

from paper_0810_1648_amd import gabp, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


CASES = [("covertype", 2000, "mixed", "bf16x6"), ("covertype", 1300, "mixed", "bf16x3"),
         ("letter", 1500, "fp32", "auto"), ("tiny", 700, "fp64", "auto"), ("large", 2600, "mixed", "bf16")]


@pytest.mark.parametrize("name,n,precision,gram", CASES)
def test_noalloc_predict_equals_predict(torch, name, n, precision, gram):
    wl, Xt, _ = inputs.holdout(name, 3000, n=n)
    print(f"[case] noalloc predict {name} N={n} {precision} {gram}", flush=True)
    s = gabp.GabpSVM(gamma=wl.gamma, C=wl.C, lambda_aug=wl.lam, precision=precision, gram=gram,
                     tol_rel=1e-7)
    st = s.solve(torch.from_numpy(wl.X).cuda(), torch.from_numpy(wl.y).cuda())
    assert st == gabp.OK
    for nq in (3000, 517):
        Xq = torch.from_numpy(np.ascontiguousarray(Xt[:nq])).cuda()
        ref = s.predict(Xq)
        out = torch.full((nq,), float("nan"), dtype=torch.float64, device="cuda")
        s.predict_noalloc(Xq, out)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b), float(np.max(np.abs(a - b)))
    s.close()


def test_noalloc_predict_refuses_oversize_and_bad_input(torch):
    wl, Xt, _ = inputs.holdout("covertype", 10, n=1000)
    s = gabp.GabpSVM(gamma=wl.gamma, C=wl.C, lambda_aug=wl.lam)
    # no solve yet: no machine to evaluate
    Xq = torch.from_numpy(Xt).cuda()
    f = torch.empty(10, dtype=torch.float64, device="cuda")
    with pytest.raises(gabp.GabpError) as e:
        s.predict_noalloc(Xq, f)
    assert e.value.status == gabp.E_STATE
    assert s.solve(torch.from_numpy(wl.X).cuda(), torch.from_numpy(wl.y).cuda()) == gabp.OK
    big = torch.zeros((400000, wl.m), dtype=torch.float32, device="cuda")
    fb = torch.empty(400000, dtype=torch.float64, device="cuda")
    with pytest.raises(gabp.GabpError) as e:
        s.predict_noalloc(big, fb)
    assert e.value.status == gabp.E_NOMEM and "scratch" in str(e.value)
    # the handle still works after the refusal
    s.predict_noalloc(Xq, f)
    torch.cuda.synchronize()
    assert np.array_equal(f.cpu().numpy(), s.predict(Xq).cpu().numpy())
    s.close()
