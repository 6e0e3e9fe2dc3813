"""One plan executed from several host threads at once, each on its own
stream (the C interface allows concurrent execute calls on a plan; its
device tables are made by whichever call comes first): every result equals
the same call made alone afterwards bit for bit, and the oracle."""
import threading

import numpy as np
import pytest

import oracle
from gpu_util import abs_sum, check_float, torch_dtype

pytestmark = pytest.mark.gpu

NCHANS, NDM, NSAMP, STEP = 96, 72, 5000, 0.35
F_TOP, DF, TSAMP = 150.0, 0.1953125 * 4, 327.68e-6
THREADS, REPEATS = 4, 3


@pytest.fixture(scope="module")
def dd(device):
    from paper_1111_6399_amd import dedisp
    return dedisp


def inputs(dtype, m, seed):
    rng = np.random.default_rng(seed)
    shape = (NCHANS, NSAMP + m)
    if dtype == "u8":
        return rng.integers(0, 256, size=shape, dtype=np.uint8)
    x = rng.standard_normal(shape).astype(np.float32)
    return x.astype(np.float16) if dtype == "f16" else x


@pytest.mark.parametrize("dtype", ["f32", "f16", "u8"])
def test_concurrent_execute_on_streams(dd, dtype):
    import torch

    dms = np.arange(NDM) * STEP
    sh, m = oracle.shift_table(NCHANS, F_TOP, DF, TSAMP, dms)
    plan = dd.Plan(NCHANS, F_TOP, DF, TSAMP, dms, dtype)  # no device tables yet
    assert plan.max_shift == m
    print("concurrent execute: %s, %d threads, plan variant %d" % (dtype, THREADS, plan.variant), flush=True)
    xs = [inputs(dtype, m, 100 + i) for i in range(THREADS)]
    dev_in = [torch.from_numpy(x).to("cuda") for x in xs]
    odt = torch.int32 if dtype == "u8" else torch.float32
    outs = [torch.full((NDM, NSAMP), -3, dtype=odt, device="cuda") for _ in range(THREADS)]
    streams = [torch.cuda.Stream() for _ in range(THREADS)]
    torch.cuda.synchronize()
    start = threading.Barrier(THREADS)
    errors = []

    def work(i):
        try:
            start.wait()
            for _ in range(REPEATS):
                plan.execute(dev_in[i], outs[i], NSAMP, streams[i].cuda_stream)
            streams[i].synchronize()
        except Exception as e:  # reported by the test thread below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(THREADS)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not errors, errors
    torch.cuda.synchronize()

    for i in range(THREADS):
        alone = torch.empty_like(outs[i])
        plan.execute(dev_in[i], alone, NSAMP, torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert torch.equal(alone, outs[i]), "thread %d differs from the same call alone" % i
    got = outs[0].cpu().numpy()
    want = oracle.dedisperse(xs[0], sh, NSAMP)
    if dtype == "u8":
        assert np.array_equal(got, want)
    else:
        check_float(got, want, abs_sum(xs[0], sh, NSAMP))
