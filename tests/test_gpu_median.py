"""GPU parity of the running-median de-reddening (Sec. 5.2) against the
oracle: bit-exact, since the median is one of the samples and the difference
is one FP32 subtraction (the oracle's FP64 difference of two FP32 values,
rounded to FP32)."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2004_03701_amd as ffa  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = ffa.ffa_create(0)
    yield c
    ffa.ffa_destroy(c)


def expected(x32, window):
    _, med = oracle.running_median(x32.astype(np.float64), window)
    return (x32.astype(np.float64) - med).astype(np.float32)


def run(ctx, x, window, tdt=torch.float32):
    xd = torch.from_numpy(x).to(device="cuda", dtype=tdt)
    out = ffa.ffa_running_median(ctx, xd, window)
    torch.cuda.synchronize()
    assert ffa.ffa_sync_status(ctx) == ffa.FFA_OK
    return out.cpu().numpy()


@pytest.mark.parametrize("n,window", [(1, 1), (2, 3), (7, 1), (10, 7), (50, 99), (100, 101),
                                      (300, 31), (1000, 257), (5000, 1001), (20000, 4001),
                                      (3000, 5999), (70001, 4097), (200_003, 20001)])
@pytest.mark.parametrize("kind", ["noise", "ties", "const", "ramp", "offset"])
def test_running_median_bit_exact(ctx, n, window, kind):
    print(f"median n={n} window={window} {kind}", flush=True)
    g = np.random.default_rng(n + window)
    if kind == "noise":
        x = g.standard_normal(n).astype(np.float32)
    elif kind == "ties":
        x = g.integers(-3, 4, n).astype(np.float32)
        x[::11] = -0.0  # equal to +0 in the order
    elif kind == "const":
        x = np.full(n, -1.5, np.float32)
    elif kind == "offset":  # every key shares its top digit: the full three-digit selection
        x = (100.0 + g.standard_normal(n)).astype(np.float32)
    else:
        x = np.cumsum(g.uniform(0, 1, n)).astype(np.float32)
    assert np.array_equal(run(ctx, x, window), expected(x, window))


def test_running_median_workload2_full_size(ctx):
    # the 9,375,000-sample red-noise series of workload 2 at its 5 s window
    # (78,125 samples of 64 us)
    x, cfg, _ = synth.workload2()
    assert cfg.median_window == 78125 and x.size == 9_375_000
    print("median workload 2, 9,375,000 samples, window 78,125", flush=True)
    assert np.array_equal(run(ctx, x, cfg.median_window), expected(x, cfg.median_window))


@pytest.mark.parametrize("tdt", [torch.bfloat16, torch.float16])
def test_running_median_16bit_input(ctx, tdt):
    x = np.random.default_rng(9).standard_normal(100_000).astype(np.float32)
    xq = torch.from_numpy(x).to(tdt).to(torch.float32).numpy()  # what the kernel reads
    assert np.array_equal(run(ctx, x, 1001, tdt), expected(xq, 1001))


@pytest.mark.parametrize("tdt,odt", [(torch.bfloat16, ffa.FFA_BF16), (torch.float16, ffa.FFA_F16)])
def test_running_median_16bit_output(ctx, tdt, odt):
    # the de-reddened series in a 16-bit storage type: the FP32 difference
    # rounded to nearest even
    x = np.random.default_rng(10).standard_normal(100_000).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    out = ffa.ffa_running_median(ctx, xd, 1001, out_dtype=odt)
    torch.cuda.synchronize()
    want = torch.from_numpy(expected(x, 1001)).to(tdt)
    assert torch.equal(out.cpu().view(torch.int16), want.view(torch.int16))


def test_running_median_impulse_passes_unchanged(ctx):
    # Sec. 5.2: a constant impulse narrower than half the window is left
    # intact by x - median
    n, window = 50_000, 2001
    x = np.full(n, 3.0, np.float32)
    x[20000:21000] += 7.0  # 1000 < 2001 / 2
    y = run(ctx, x, window)
    want = np.zeros(n, np.float32)
    want[20000:21000] = 7.0
    assert np.array_equal(y, want)


def test_running_median_argument_errors(ctx):
    x = torch.zeros(100, device="cuda")
    for w in (0, 2, -3):
        with pytest.raises(ffa.FFAError) as e:
            ffa.ffa_running_median(ctx, x, w)
        assert e.value.status == ffa.FFA_ERR_INVALID_ARG
