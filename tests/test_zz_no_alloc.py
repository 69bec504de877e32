"""The allocation-free estimator entry point (cr_eval_noalloc) against the
workspace entry point (cr_eval) it mirrors: two calls in a row through the C
ABI, the second with a smaller input, identical bits required (the same
kernels on the same inputs), plus sampled queries against the FP64 oracle.

Every case prints its name, sizes and seed before touching the GPU."""
import sys

import numpy as np
import pytest

from oracle import estimator

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1407_7220_amd as cr
    return cr


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _case(N, n, M, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, size=(N, n))
    y = rng.normal(size=N)
    xi = rng.normal(size=(N, n))
    Q = rng.uniform(-1.5, 1.5, size=(M, n))
    return X, y, xi, Q


def test_noalloc_matches_workspace_entry_point(cr):
    # the second call is smaller: the scratch keeps the first call's planes past its end
    for (N, n, M, seed) in [(6000, 20, 1500, 1), (700, 5, 333, 2)]:
        say("eval_noalloc N=%d n=%d M=%d seed=%d" % (N, n, M, seed))
        X, y, xi, Q = _case(N, n, M, seed)
        Xd, yd, xid, Qd = dev(X), dev(y), dev(xi), dev(Q)
        f_ref, a_ref = cr.evaluate(Xd, yd, xid, Qd)
        f = torch.full((M,), float("nan"), dtype=torch.float64, device="cuda")
        a = torch.full((M,), -1, dtype=torch.int64, device="cuda")
        cr.evaluate_noalloc(Xd, yd, xid, Qd, f, a)
        torch.cuda.synchronize()
        assert torch.equal(f, f_ref)
        assert torch.equal(a, a_ref)
        fo, ao = estimator.evaluate(X, y, xi, Q[:64])
        fh, ah = f[:64].cpu().numpy(), a[:64].cpu().numpy()
        scale = np.abs(y).max() + np.abs(xi).sum(axis=1).max() * 3.0
        assert np.max(np.abs(fh - fo)) <= 1e-12 * scale
        np.testing.assert_array_equal(ah, ao)


def test_noalloc_without_arg_and_size_limit(cr):
    say("eval_noalloc arg=None N=4096 n=3 M=100, and the largest n=20 size")
    X, y, xi, Q = _case(4096, 3, 100, 3)
    Xd, yd, xid, Qd = dev(X), dev(y), dev(xi), dev(Q)
    f_ref, _ = cr.evaluate(Xd, yd, xid, Qd, with_arg=False)
    f = torch.empty(100, dtype=torch.float64, device="cuda")
    cr.evaluate_noalloc(Xd, yd, xid, Qd, f, None)
    torch.cuda.synchronize()
    assert torch.equal(f, f_ref)
    # 174752 planes at n = 20 fill the 32 MiB scratch exactly
    N = 174752
    X, y, xi, Q = _case(N, 20, 96, 4)
    Xd, yd, xid, Qd = dev(X), dev(y), dev(xi), dev(Q)
    f = torch.empty(96, dtype=torch.float64, device="cuda")
    a = torch.empty(96, dtype=torch.int64, device="cuda")
    cr.evaluate_noalloc(Xd, yd, xid, Qd, f, a)
    f_ref, a_ref = cr.evaluate(Xd, yd, xid, Qd)
    torch.cuda.synchronize()
    assert torch.equal(f, f_ref) and torch.equal(a, a_ref)
