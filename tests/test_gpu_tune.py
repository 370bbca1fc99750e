"""GPU tests of the autotuner (hidft_autotune and HIDFT_SCHED_TUNED)."""
import sys

import numpy as np
import pytest

import oracle
from workloads import homogeneous_support, rng_for, sample_values

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
native = pytest.importorskip("paper_2211_15299_amd.native")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    native.tune_clear()
    yield
    native.tune_clear()
    torch.cuda.synchronize()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("s,prec", [(6, native.PREC_FP32), (10, native.PREC_FP32),
                                    (12, native.PREC_FP32), (13, native.PREC_FP32),
                                    (14, native.PREC_FP32), (11, native.PREC_BF16X3),
                                    (14, native.PREC_F16X2)])
def test_autotune_picks_a_valid_variant(s, prec):
    rng = rng_for(2200, s)
    M = 22 if s >= 13 else 20
    sup = homogeneous_support(M, s, rng)
    J = sup.J.tolist()
    plan = native.Plan(M, J)
    k = plan.k
    batch = max(8, (1 << 20) >> s)
    f = sample_values(M, k, batch, rng)
    x = torch.from_numpy(f.astype(np.complex64)).cuda()
    y = torch.empty_like(x)
    _say(f"case s={s} prec={prec} batch={batch}: autotune")
    best, us = plan.autotune_ptr(x.data_ptr(), k, y.data_ptr(), k, batch, precision=prec, reps=3)
    torch.cuda.synchronize()
    _say(f"  best {best} {us:.1f} us")
    assert best.precision == prec and us > 0
    assert best.radix in (16, 32) or (prec != native.PREC_FP32 and best.radix in (0, 16))
    # the output buffer holds the transform
    rows = [0, batch - 1]
    want = oracle.adjoint_coefficients(M, J, plan.samples().tolist(), f[rows])
    got = y.cpu().numpy()[rows].astype(np.complex128)
    assert np.max(oracle.rel_l2(got, want)) <= 1e-5
    # the table holds it, and TUNED runs exactly it
    found = plan.tune_lookup(batch, prec)
    assert found is not None and found.as_tuple() == best.as_tuple()
    a = plan.execute(x, config=best)
    b = plan.execute(x, config=native.ExecConfig(prec, native.SCHED_TUNED, 0, 0))
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # another batch class has no entry: TUNED falls back to the default variant
    small = x[:3]
    assert plan.tune_lookup(3, prec) is None
    c = plan.execute(small, config=native.ExecConfig(prec, native.SCHED_TUNED, 0, 0))
    d = plan.execute(small, config=native.ExecConfig(prec, native.SCHED_DEFAULT, 0, 0))
    torch.cuda.synchronize()
    assert torch.equal(c, d)


def test_tuning_table_survives_save_and_load(tmp_path):
    rng = rng_for(2201, 0)
    M, s, batch = 20, 9, 2048
    plan = native.Plan(M, homogeneous_support(M, s, rng).J.tolist())
    x = torch.from_numpy(sample_values(M, plan.k, batch, rng).astype(np.complex64)).cuda()
    y = torch.empty_like(x)
    best, _ = plan.autotune_ptr(x.data_ptr(), plan.k, y.data_ptr(), plan.k, batch, reps=2)
    path = str(tmp_path / "tune.txt")
    native.tune_save(path)
    native.tune_clear()
    assert plan.tune_lookup(batch) is None
    native.tune_load(path)
    again = plan.tune_lookup(batch)
    assert again is not None and again.as_tuple() == best.as_tuple()
    # the batch class is floor(log2 batch): 2048..4095 share the entry
    assert plan.tune_lookup(4095).as_tuple() == best.as_tuple()
    assert plan.tune_lookup(4096) is None


def test_autotune_errors():
    rng = rng_for(2202, 0)
    plan = native.Plan(16, homogeneous_support(16, 8, rng).J.tolist())
    x = torch.zeros((4, plan.k), dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    for args, kw in [((x.data_ptr(), plan.k, x.data_ptr(), plan.k, 4), {}),    # in place
                     ((x.data_ptr(), plan.k, y.data_ptr(), plan.k, 4), {"reps": 0}),
                     ((x.data_ptr(), plan.k, y.data_ptr(), plan.k, 0), {}),
                     ((x.data_ptr(), plan.k, y.data_ptr(), plan.k, 4), {"precision": 5})]:
        with pytest.raises(native.HiDFTError) as ei:
            plan.autotune_ptr(*args, **kw)
        assert ei.value.status_name == "HIDFT_ERR_INVALID_ARGUMENT"
    tiny = native.Plan(12, homogeneous_support(12, 2, rng).J.tolist())
    with pytest.raises(native.HiDFTError) as ei:
        tiny.autotune_ptr(x.data_ptr(), 4, y.data_ptr(), 4, 4, precision=native.PREC_F16X2)
    assert ei.value.status_name == "HIDFT_ERR_UNSUPPORTED"
    torch.cuda.synchronize()
