"""Resuming a fit (cox_fit_opts.warm_start = 2): K1 steps, then a resumed call
to max_iter = K2, give bit for bit the coefficients, step counts, objectives
and (from the resumed steps on) the objective trace of one call with
max_iter = K2 -- on the vector path and on the batched matrix-core path, with
lambdas that converge before K1, between K1 and K2, or not at all.  A resume
after any other call on the context, or with other lambdas, is refused."""
import numpy as np
import pytest

import coxsim
import oracle
from tests.gpu_helpers import device_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
import paper_2010_16114_amd as P  # noqa: E402


def _bits(x):
    return np.ascontiguousarray(x).view(np.uint32 if x.dtype == np.float32 else np.uint64)


@pytest.mark.parametrize("storage,B", [("f32", 3), ("fp8", 5), ("fp8", 20), ("int8", 64)])
def test_resume_equals_one_call(storage, B):
    d = coxsim.genotype_problem(3001, 700, 12, 0.6, 6262, days=True)
    cox, M = device_problem(d, storage, ldx=(d.n + 15) // 16 * 16, max_batch=B)
    lm = oracle.lambda_max(M, d.time, d.event)
    lams = lm * np.geomspace(1.01, 0.05, B)
    sigma = 1.0 / (2.0 * oracle.opnorm2(M)[0])
    K1, K2 = 23, 60
    one = cox.fit_path(lams, max_iter=K2, tol=1e-7, lag=10, step=sigma, trace=True)
    part = cox.fit_path(lams, max_iter=K1, tol=1e-7, lag=10, step=sigma)
    rest = cox.fit_path(lams, max_iter=K2, tol=1e-7, lag=10, step=sigma, resume=True, trace=True)
    np.testing.assert_array_equal(_bits(rest[0].cpu().numpy()), _bits(one[0].cpu().numpy()))
    np.testing.assert_array_equal(rest[1], one[1])
    np.testing.assert_array_equal(_bits(rest[2]), _bits(one[2]))
    assert rest[3] == one[3]
    for b in range(B):  # the resumed call records the steps after K1
        k = rest[1][b]
        if part[1][b] == K1:
            np.testing.assert_array_equal(_bits(rest[4][b, K1 + 1 : k + 1]), _bits(one[4][b, K1 + 1 : k + 1]))
    assert (one[1] < K1).any() or B < 5  # some lambda stopped before the interruption (large B)


def test_resume_is_refused_after_other_work():
    d = coxsim.genotype_problem(1500, 300, 6, 0.5, 6363)
    cox, M = device_problem(d, "f32", max_batch=2)
    lams = [0.5 * cox.lambda_max(), 0.2 * cox.lambda_max()]
    cox.fit_path(lams, max_iter=5, tol=0.0, step=1e-3)
    for other in (lambda: cox.loss_grad(torch.zeros((1, d.p), device="cuda")),
                  lambda: cox.opnorm2(maxiter=3)):
        other()
        with pytest.raises(P.CoxError) as ei:
            cox.fit_path(lams, max_iter=10, tol=0.0, step=1e-3, resume=True)
        assert ei.value.status == P.ERR_INVALID_ARG
        cox.fit_path(lams, max_iter=5, tol=0.0, step=1e-3)
    for kw in (dict(lambdas=[lams[0], lams[1] * 0.9]), dict(max_iter=3), dict(step=2e-3)):
        args = dict(lambdas=lams, max_iter=10, tol=0.0, step=1e-3, resume=True)
        args.update(kw)
        with pytest.raises(P.CoxError) as ei:
            cox.fit_path(**args)
        assert ei.value.status == P.ERR_INVALID_ARG
