"""Accuracy of the device elementary functions used by the ionic models
(exp, expm1, log; double and single precision) against extended-precision
host values (numpy longdouble, 64-bit significand on x86), plus their
special cases."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -52   # one ulp at 1 in double
U32 = 2.0 ** -23


@pytest.fixture(scope="module")
def E():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2401_01745_amd import emrkc
    emrkc.lib()
    return emrkc


def dev_eval(E, fn, x, precision="fp64"):
    import torch
    y = E.emrkc_eval_elementary(fn, torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda(), precision)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def samples(seed, lo, hi, n=200_000):
    return np.random.default_rng(seed).uniform(lo, hi, n)


def ref(fn, x):
    xl = x.astype(np.longdouble)
    return {"exp": np.exp, "expm1": np.expm1, "log": np.log}[fn](xl)


def rel_err(y, r):
    return np.abs((y.astype(np.longdouble) - r) / r).astype(np.float64)


def test_exp_double(E):
    x = np.concatenate([samples(1, -700, 700), samples(2, -1, 1), samples(3, -30, 30)])
    assert rel_err(dev_eval(E, "exp", x), ref("exp", x)).max() <= 2 * U64


def test_expm1_double(E):
    rng = np.random.default_rng(4)
    tiny = 10.0 ** rng.uniform(-300, -1, 100_000) * np.where(rng.uniform(size=100_000) < 0.5, -1, 1)
    x = np.concatenate([samples(5, -60, 10), samples(6, -0.4, 0.4), tiny, samples(7, -700, 700)])
    assert rel_err(dev_eval(E, "expm1", x), ref("expm1", x)).max() <= 4 * U64


def test_log_double(E):
    rng = np.random.default_rng(8)
    x = np.concatenate([10.0 ** rng.uniform(-300, 300, 200_000), samples(9, 0.5, 2.0),
                        1.0 + samples(10, -1e-6, 1e-6, 50_000), 10.0 ** rng.uniform(-320, -308, 1000)])
    x = x[x != 1.0]
    assert rel_err(dev_eval(E, "log", x), ref("log", x)).max() <= 4 * U64


def test_double_special_cases(E):
    inf, nan = np.inf, np.nan
    y = dev_eval(E, "exp", np.array([0.0, -746.0, 710.0, nan, -1e6, 1e6]))
    assert y[0] == 1.0 and y[1] == 0.0 and y[2] == inf and np.isnan(y[3]) and y[4] == 0.0 and y[5] == inf
    y = dev_eval(E, "expm1", np.array([0.0, -40.0, -800.0, 800.0, 1e-310, nan]))
    assert y[0] == 0.0 and y[1] == -1.0 and y[2] == -1.0 and y[3] == inf and y[4] == 1e-310 and np.isnan(y[5])
    y = dev_eval(E, "log", np.array([1.0, 0.0, -1.0, inf, nan, 5e-324, 2.0]))
    assert y[0] == 0.0 and y[1] == -inf and np.isnan(y[2]) and y[3] == inf and np.isnan(y[4])
    assert abs(y[5] - float(np.log(np.longdouble(5e-324)))) <= 4 * U64 * 745
    assert abs(y[6] - 0.6931471805599453) <= U64


def test_single_precision_forms(E):
    # exp and log: the native exp2/log2 paths, whose error grows with |x log2 e|
    x = samples(11, -80, 80).astype(np.float32).astype(np.float64)
    e = rel_err(dev_eval(E, "exp", x, "mixed"), ref("exp", x))
    assert (e <= 4 * U32 * (1 + np.abs(x))).all()
    x = samples(12, -60, 10).astype(np.float32).astype(np.float64)
    x = np.concatenate([x, (10.0 ** samples(13, -30, -1, 50_000)).astype(np.float32).astype(np.float64)])
    assert rel_err(dev_eval(E, "expm1", x, "mixed"), ref("expm1", x)).max() <= 4 * U32
    x = (10.0 ** samples(14, -30, 30)).astype(np.float32).astype(np.float64)
    y, r = dev_eval(E, "log", x, "mixed"), ref("log", x)
    assert (np.abs(y - r.astype(np.float64)) <= 4 * U32 * np.maximum(1.0, np.abs(r.astype(np.float64)))).all()


def test_rejects_bad_arguments(E):
    from paper_2401_01745_amd.emrkc import lib, EMRKC_EINVAL
    assert lib().emrkc_eval_elementary(3, 0, None, None, 0, None) == EMRKC_EINVAL
    assert lib().emrkc_eval_elementary(0, 7, None, None, 0, None) == EMRKC_EINVAL
    assert lib().emrkc_eval_elementary(0, 0, None, None, 5, None) == EMRKC_EINVAL
    assert lib().emrkc_eval_elementary(0, 0, None, None, 0, None) == 0
