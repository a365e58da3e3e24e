"""Batched subarrays of uneven N: autotuned kernel choices, one persistent
launch per engine and input width, and whole-step HIP-graph replays, all
bit-exact against the oracle."""
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


SMALL = [(64, 8, 512), (128, 4, 300), (40, 3, 200), (96, 2, 130)]  # (N, F, T)


def test_graph_replays_match_oracle(torch_cuda, oracle_lib):
    # replays read refilled buffers; eager work and syncs between replays
    from paper_1411_3751_amd import Correlator
    torch = torch_cuda
    print("case graph replays", flush=True)
    rng = np.random.default_rng(31)
    subs = [dict(n_inputs=N, n_chans=F, n_time=T) for (N, F, T) in SMALL]
    dev = [torch.empty((T, F, N), dtype=torch.uint8, device="cuda") for (N, F, T) in SMALL]
    out = [torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device="cuda")
           for (N, F, T) in SMALL]
    with Correlator(subs) as c:
        with c.capture(dev, out) as g:
            for rep in range(3):
                host = [rand4(rng, T, F, N) for (N, F, T) in SMALL]
                for d, h in zip(dev, host):
                    d.copy_(torch.from_numpy(h))
                torch.cuda.synchronize()
                g.launch()
                torch.cuda.synchronize()
                for (N, F, T), h, o in zip(SMALL, host, out):
                    want = oracle_lib.narrow(oracle_lib.correlate(h, 4))
                    assert np.array_equal(o.cpu().numpy(), want), (rep, N)
        # the context is left reset: an eager step after the graph starts from zero
        h = [rand4(rng, T, F, N) for (N, F, T) in SMALL]
        c.correlate([torch.from_numpy(x).cuda() for x in h])
        for (N, F, T), x, o in zip(SMALL, h, c.dump()):
            assert np.array_equal(o.cpu().numpy(), oracle_lib.narrow(oracle_lib.correlate(x, 4)))


def test_graph_needs_reset_context(torch_cuda):
    from paper_1411_3751_amd import Correlator, XengError
    from paper_1411_3751_amd.xeng import XENG_EINVAL
    torch = torch_cuda
    x = torch.zeros((64, 2, 16), dtype=torch.uint8, device="cuda")
    o = torch.empty((2, 136, 2), dtype=torch.int32, device="cuda")
    with Correlator([dict(n_inputs=16, n_chans=2, n_time=64)]) as c:
        c.correlate([x])
        with pytest.raises(XengError) as ei:
            c.capture([x], [o])
        assert ei.value.code == XENG_EINVAL


def test_autotune_choices_stay_exact_and_are_cached(torch_cuda, oracle_lib):
    from paper_1411_3751_amd import Correlator
    torch = torch_cuda
    print("case autotune", flush=True)
    rng = np.random.default_rng(32)
    shapes = [(64, 16, 1024), (48, 4, 700), (256, 3, 500)]
    subs = [dict(n_inputs=N, n_chans=F, n_time=T) for (N, F, T) in shapes]
    host = [rand4(rng, T, F, N) for (N, F, T) in shapes]
    dev = [torch.from_numpy(h).cuda() for h in host]
    with Correlator(subs) as c:
        c.correlate(dev)
        c.autotune(dev, reps=2)   # discards the sums above
        assert c.samples_since_dump() == 0
        plan = c.plan()
        assert plan["tuned"] is True
        c.correlate(dev)
        c.correlate(dev)
        outs = [o.cpu().numpy() for o in c.dump()]
    for (N, F, T), h, o in zip(shapes, host, outs):
        assert np.array_equal(o, oracle_lib.narrow(oracle_lib.correlate(h, 4) * 2)), N
    with Correlator(subs) as c2:
        assert c2.plan()["tuned"] is True
        assert [s["kernel"] for s in c2.plan()["subarrays"]] == \
            [s["kernel"] for s in plan["subarrays"]]

def test_graph_survives_autotune(torch_cuda, oracle_lib):
    # autotuning replans the context (new tile lists); a graph captured before
    # keeps the lists it was captured with and still replays exactly
    from paper_1411_3751_amd import Correlator
    torch = torch_cuda
    print("case graph then autotune", flush=True)
    rng = np.random.default_rng(34)
    shapes = [(64, 8, 512), (128, 4, 300)]
    subs = [dict(n_inputs=N, n_chans=F, n_time=T) for (N, F, T) in shapes]
    dev = [torch.empty((T, F, N), dtype=torch.uint8, device="cuda") for (N, F, T) in shapes]
    out = [torch.empty((F, N * (N + 1) // 2, 2), dtype=torch.int32, device="cuda")
           for (N, F, T) in shapes]
    with Correlator(subs) as c:
        with c.capture(dev, out) as g:
            host = [rand4(rng, T, F, N) for (N, F, T) in shapes]
            for d, h in zip(dev, host):
                d.copy_(torch.from_numpy(h))
            torch.cuda.synchronize()
            c.autotune(dev, reps=1)
            torch.cuda.synchronize()
            for rep in range(2):
                g.launch()
                torch.cuda.synchronize()
                for (N, F, T), h, o in zip(shapes, host, out):
                    want = oracle_lib.narrow(oracle_lib.correlate(h, 4))
                    assert np.array_equal(o.cpu().numpy(), want), (rep, N)


def test_second_process_starts_tuned(torch_cuda, tmp_path):
    # this process autotunes with XENG_TUNING_FILE set (the cache is written
    # to the file); a fresh process with the same setting creates a context of
    # the same shapes and starts with the same choices, marked tuned
    import json
    import os
    import subprocess
    import sys
    from paper_1411_3751_amd import Correlator
    torch = torch_cuda
    path = str(tmp_path / "tuning.json")
    shapes = [(64, 40, 2048), (256, 12, 2048), (144, 6, 1000)]
    subs = [dict(n_inputs=N, n_chans=F, n_time=T) for N, F, T in shapes]
    rng = np.random.default_rng(4242)
    dev = [torch.from_numpy(rng.integers(0, 256, size=(T, F, N), dtype=np.uint8)).cuda()
           for N, F, T in shapes]
    os.environ["XENG_TUNING_FILE"] = path
    try:
        with Correlator(subs) as c:
            c.autotune(dev, reps=1)
            plan = c.plan()
    finally:
        del os.environ["XENG_TUNING_FILE"]
    picks = [s["kernel"] for s in plan["subarrays"]]
    print("process 1 picks", picks, flush=True)
    doc = json.load(open(path))
    assert doc["format"] == "xeng-tuning"
    # (earlier tests of this process may have tuned other shape lists)
    mine = [b for b in doc["batches"] if b["shapes"] == [[N, F, T, 4, 0] for N, F, T in shapes]]
    assert len(mine) == 1 and [k for k, _ in mine[0]["kernels"]] == picks
    code = ("import json; from paper_1411_3751_amd import Correlator\n"
            "subs = %r\n"
            "with Correlator(subs) as c:\n"
            "    p = c.plan()\n"
            "print(json.dumps({'tuned': p['tuned'], 'picks': [s['kernel'] for s in p['subarrays']],"
            " 'wg': p['workgroups_per_cu'], 'order': p['schedule_order']}))\n" % subs)
    env = dict(os.environ, XENG_TUNING_FILE=path)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=300, cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.returncode == 0, out.stderr[-2000:]
    got = json.loads(out.stdout.strip().splitlines()[-1])
    print("process 2", got, flush=True)
    assert got["tuned"] is True
    assert got["picks"] == picks
    assert got["wg"] == plan["workgroups_per_cu"] and got["order"] == plan["schedule_order"]
