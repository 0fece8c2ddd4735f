"""The hand-written adjoint behind torch.autograd.Function.

BreslowNLL(eta) = -L(eta) and its backward -r (Section 5.3's (I - P) delta);
CoxLinearNLL(beta) = -L(X~ beta) and its backward -X~' r.  Checked against
torch.autograd.gradcheck (FP64, tiny n), the FP64 oracle, and central finite
differences (h = 1e-3, 20 random unit directions) on the 100,000 x 10,000
genotype workload with times discretised to days (many ties).
"""
import numpy as np
import pytest

import coxsim
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
import paper_2010_16114_amd as P  # noqa: E402


def test_gradcheck_fp64_eta():
    rng = np.random.default_rng(0)
    n = 40
    t = rng.integers(1, 12, n).astype(float)
    e = (rng.random(n) < 0.7).astype(np.int32)
    X = torch.zeros((1, n), device="cuda")  # only the context's order and events are used here
    cox = P.Cox(X, t, e, max_batch=3)
    eta = torch.tensor(rng.standard_normal((3, n)), dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda z: P.BreslowNLL.apply(z, cox), (eta,), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_eta_loss_and_adjoint_against_oracle():
    rng = np.random.default_rng(1)
    n = 5000
    t = rng.integers(1, 300, n).astype(float)
    e = (rng.random(n) < 0.6).astype(np.int32)
    cox = P.Cox(torch.zeros((1, n), device="cuda"), t, e, max_batch=2)
    eta = torch.tensor(2 * rng.standard_normal((2, n)), dtype=torch.float32, device="cuda", requires_grad=True)
    loss = P.BreslowNLL.apply(eta, cox)
    (loss * torch.tensor([1.0, -2.5], device="cuda")).sum().backward()
    g = eta.grad.cpu().numpy()
    for b, w in ((0, 1.0), (1, -2.5)):
        L, r = oracle.loglik(eta.detach().cpu().numpy()[b].astype(np.float64), t, e)
        assert float(loss[b]) == pytest.approx(-L, rel=1e-6)
        np.testing.assert_allclose(g[b], -w * r, rtol=0, atol=1e-6 * np.abs(r).max() * abs(w))


@pytest.fixture(scope="module")
def c2():
    d = coxsim.config2()
    X = torch.from_numpy(d.standardized32()).cuda()
    return d, X


def test_c2_linear_fd_and_oracle(c2):
    d, X = c2
    cox = P.Cox(X, d.time, d.event, max_batch=1)
    assert len(np.unique(d.time)) <= 1000  # discretised: ties
    M = oracle.Matrix.genotype(d.G, d.mu, d.s)
    rng = np.random.default_rng(7)
    for beta_np in (np.zeros(d.p), d.beta_true):
        beta = torch.tensor(beta_np, dtype=torch.float32, device="cuda", requires_grad=True)
        loss = P.CoxLinearNLL.apply(beta.view(1, -1), cox)
        loss.sum().backward()
        g = beta.grad.cpu().numpy().astype(np.float64)
        negL, go = oracle.loss_grad(M, d.time, d.event, beta_np.astype(np.float32).astype(np.float64))
        assert float(loss[0]) == pytest.approx(negL, rel=1e-6)
        assert np.abs(g + go).max() <= 1e-5 * np.abs(go).max()
        h = 1e-3
        for _ in range(20):
            v = rng.standard_normal(d.p)
            v /= np.linalg.norm(v)
            bp = torch.tensor((beta_np + h * v)[None], dtype=torch.float32, device="cuda")
            bm = torch.tensor((beta_np - h * v)[None], dtype=torch.float32, device="cuda")
            fp, _ = cox.loss_grad(bp, want_grad=False)
            fm, _ = cox.loss_grad(bm, want_grad=False)
            fd = (fp[0] - fm[0]) / (2 * h)
            dd = float(g @ v)
            assert fd == pytest.approx(dd, rel=1e-3, abs=1e-3 * np.abs(g).max())


def test_c2_breslow_on_eta(c2):
    d, X = c2
    cox = P.Cox(X, d.time, d.event, max_batch=1)
    beta = torch.tensor(d.beta_true[None], dtype=torch.float32, device="cuda")
    eta = (beta @ X).detach().clone().requires_grad_(True)  # (1, n)
    loss = P.BreslowNLL.apply(eta, cox)
    loss.sum().backward()
    L, r = oracle.loglik(eta.detach().cpu().numpy()[0].astype(np.float64), d.time, d.event)
    assert float(loss[0]) == pytest.approx(-L, rel=1e-6)
    np.testing.assert_allclose(eta.grad.cpu().numpy()[0], -r, rtol=0, atol=1e-6 * np.abs(r).max())
