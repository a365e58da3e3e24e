"""C-ABI behaviour that needs the HIP runtime and a device: errors and bounds."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_invalid_arguments(torch_cuda):
    from paper_1411_3751_amd import Correlator, XengError
    from paper_1411_3751_amd.xeng import XENG_EINVAL
    for bad in [dict(n_inputs=0, n_chans=1, n_time=1), dict(n_inputs=4, n_chans=0, n_time=1),
                dict(n_inputs=4, n_chans=1, n_time=0), dict(n_inputs=4, n_chans=1, n_time=8, in_bits=6),
                dict(n_inputs=4, n_chans=1, n_time=8, engine=7),
                dict(n_inputs=4, n_chans=1, n_time=8, in_bits=8, engine=1),
                dict(n_inputs=40, n_chans=1, n_time=8, in_bits=4, engine=1)]:
        with pytest.raises(XengError) as ei:
            Correlator([bad])
        assert ei.value.code == XENG_EINVAL


def test_exactness_bound_refused_before_launch(torch_cuda):
    from paper_1411_3751_amd import Correlator, XengError
    from paper_1411_3751_amd.xeng import XENG_ERANGE
    torch = torch_cuda
    T = 30000
    x = torch.zeros((T, 1, 4, 2), dtype=torch.int8, device="cuda")
    with Correlator([dict(n_inputs=4, n_chans=1, n_time=T, in_bits=8)]) as c:
        assert c.max_dump_samples() == 65535
        c.correlate([x])
        c.correlate([x])
        with pytest.raises(XengError) as ei:
            c.correlate([x])  # 90000 > 65535
        assert ei.value.code == XENG_ERANGE
        assert c.samples_since_dump() == 2 * T
        c.dump(reset=True)
        c.correlate([x])
        assert c.samples_since_dump() == T


def test_shape_checks_and_null(torch_cuda):
    from paper_1411_3751_amd import Correlator
    torch = torch_cuda
    with Correlator([dict(n_inputs=8, n_chans=2, n_time=16)]) as c:
        with pytest.raises(ValueError):
            c.correlate([torch.zeros((16, 2, 9), dtype=torch.uint8, device="cuda")])
        plan = c.plan()
        assert plan["subarrays"][0]["n_inputs"] == 8
