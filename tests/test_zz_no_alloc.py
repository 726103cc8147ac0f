"""life_dsc_noalloc (workspace in the library's static device array, no
allocation) against life_dsc through the C ABI: two calls in a row on different
plans, the second with a smaller problem, bitwise equal outputs; both within
1e-5 of the FP64 oracle; a plan whose workspace exceeds the static array is
rejected with LIFE_ERANGE."""
import numpy as np
import pytest

import oracle
import synth
from conftest import connectome, relerr

torch = pytest.importorskip("torch")
from paper_1905_06234_amd import life  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    life.load()
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float32).ravel())).to(dev)


def test_noalloc_matches_dsc_twice(dev):
    big = connectome("mid")
    small = synth.random_coo(33, 70, 150, 60, 700, seed=3)
    for c in (big, small):            # the second call: a smaller problem on the same static array
        print(f"[noalloc] nnz={c.nnz} n_theta={c.n_theta}", flush=True)
        plan = life.Plan.from_connectome(c)
        rng = np.random.default_rng(c.nnz)
        w = rng.random(c.n_fascicles).astype(np.float32)
        D, wd = _t(c.D, dev), _t(w, dev)
        ref = plan.dsc(D, wd).clone()
        y = torch.full((plan.n_signal,), float("nan"), dtype=torch.float32, device=dev)
        plan.dsc_noalloc(D, wd, y)
        torch.cuda.synchronize()
        assert torch.equal(y, ref)
        op = oracle.Operator.from_connectome(c)
        assert relerr(y.cpu().double().numpy(), op.dsc(w)) <= 1e-5
        plan.close()


def test_noalloc_rejects_oversized_workspace(dev):
    nf = (64 << 20) // 4 + 1          # weights alone exceed the 64 MiB array
    plan = life.Plan(16, 8, 4, nf, np.array([0, 1], np.int16), np.array([0, 3], np.int32),
                     np.array([0, nf - 1], np.int32), np.array([0.5, 1.0], np.float32))
    D = torch.zeros(16 * 8, dtype=torch.float32, device=dev)
    w = torch.ones(nf, dtype=torch.float32, device=dev)
    y = torch.zeros(16 * 4, dtype=torch.float32, device=dev)
    with pytest.raises(life.LifeError) as e:
        plan.dsc_noalloc(D, w, y)
    assert e.value.status == 2
    plan.dsc(D, w, y)                   # the ordinary call still serves it
    torch.cuda.synchronize()
    plan.close()
