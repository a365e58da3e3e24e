"""Fast-cadence autocorrelations: selective dump and zeroing of the selected
inputs' autocorrelation cells while every other cell integrates on."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def rand4(rng, T, F, N):
    re = rng.integers(-8, 8, size=(T, F, N)).astype(np.int8)
    im = rng.integers(-8, 8, size=(T, F, N)).astype(np.int8)
    return synth.pack4(re, im)


def diag(n):
    return np.array([i * (i + 1) // 2 + i for i in range(n)])


@pytest.mark.parametrize("N,engine", [(64, 0), (40, 0), (128, 1)])
def test_fast_autos_dump_and_reset(torch_cuda, oracle_lib, N, engine):
    from paper_1411_3751_amd import Correlator
    torch = torch_cuda
    print("case fast autos N=%d engine=%d" % (N, engine), flush=True)
    rng = np.random.default_rng(40 + N)
    F, T = 4, 256
    sel = [3, 10, N - 1]
    gulps = [rand4(rng, T, F, N) for _ in range(5)]
    V = [oracle_lib.correlate(g, 4) for g in gulps]   # int64 [F][tri][2] per gulp
    d = diag(N)
    with Correlator([dict(n_inputs=N, n_chans=F, n_time=T, engine=engine)]) as c:
        c.set_fast_autos(sel)
        assert not c.dump_fast_autos(reset=False)[0].cpu().numpy().any()  # nothing yet
        for g in gulps[:3]:
            c.correlate([torch.from_numpy(g).cuda()])
        fast1 = c.dump_fast_autos(reset=True)[0].cpu().numpy()
        want1 = sum(V[:3])[:, d[sel], 0]
        assert np.array_equal(fast1, want1)
        for g in gulps[3:]:
            c.correlate([torch.from_numpy(g).cuda()])
        fast2 = c.dump_fast_autos(reset=False)[0].cpu().numpy()
        assert np.array_equal(fast2, sum(V[3:])[:, d[sel], 0])
        full = c.dump(reset=True)[0].cpu().numpy()
    want = sum(V).copy()
    want[:, d[sel], 0] = sum(V[3:])[:, d[sel], 0]    # selected autos since their reset
    assert np.array_equal(full, oracle_lib.narrow(want))
    assert not full[:, d, 1].any()                     # Im V_ii = 0 everywhere


def test_fast_autos_errors(torch_cuda):
    from paper_1411_3751_amd import Correlator, XengError
    from paper_1411_3751_amd.xeng import XENG_EINVAL
    with Correlator([dict(n_inputs=16, n_chans=2, n_time=64)]) as c:
        with pytest.raises(XengError) as ei:
            c.set_fast_autos([16])
        assert ei.value.code == XENG_EINVAL
        c.set_fast_autos([])           # clearing the selection is allowed
        assert c.dump_fast_autos(reset=True) == [None]
