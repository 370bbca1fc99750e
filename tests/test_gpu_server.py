"""Request server (continuous batching) on the GPU.

Requests of different (N, J, k) arrive while others are on the device; each
result must equal -- bit for bit -- the result of the same request run alone
through the single-plan path, and agree with the FP64 oracle.
"""
import sys
import threading

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
    yield
    torch.cuda.synchronize()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _supports(n, cfg=5):
    out = []
    for i in range(n):
        rng = rng_for(cfg, i)
        M = int(rng.integers(10, 23))
        s = int(rng.integers(6, min(13, M - 2) + 1))
        sup = homogeneous_support(M, s, rng)
        out.append((M, np.ascontiguousarray(sup.J, dtype=np.uint64)))
    return out


def _alone(M, J, f):
    plan = native.Plan(M, J.tolist())
    x = torch.from_numpy(f).cuda()
    y = plan.execute(x)
    torch.cuda.synchronize()
    r = y[0].cpu().numpy()
    plan.close()
    return r


def test_server_mix_equals_alone_and_oracle():
    sups = _supports(48)
    rng = rng_for(5, 1000)
    n_req = 1500
    which = rng.integers(0, len(sups), size=n_req)
    samples = [sample_values(sups[w][0], len(sups[w][1]), 1, rng) for w in which]
    outs = [np.full(len(sups[w][1]), np.nan, dtype=np.complex64) for w in which]
    srv = native.Server(data_bytes=64 << 20, plan_bytes=16 << 20, slots=3, max_batch=256)
    ids = {}
    for i, w in enumerate(which):
        M, J = sups[w]
        ids[srv.submit(M, J, samples[i][0], outs[i])] = i
        if i % 100 == 0:
            srv.poll()
    srv.drain()
    st = srv.stats()
    _say(f"server: {st}")
    assert st["completed"] == n_req and st["rejected"] == 0
    assert st["batches"] >= 2
    # every request's result, alone vs in the mix: bit-identical
    checked = 0
    for i in range(0, n_req, 7):
        M, J = sups[which[i]]
        alone = _alone(M, J, samples[i])
        assert np.array_equal(alone, outs[i]), i
        checked += 1
    # oracle on a sample
    for i in range(0, n_req, 97):
        M, J = sups[which[i]]
        plan = native.Plan(M, J.tolist(), host_only=True)
        want = oracle.adjoint_coefficients(M, J.tolist(), plan.samples().tolist(),
                                           samples[i][0].astype(np.complex128))
        assert oracle.rel_l2(outs[i].astype(np.complex128), want) <= 1e-5
    _say(f"server: {checked} requests identical alone and in the mix")
    srv.close()


def test_server_admission_errors_and_eviction():
    rng = rng_for(5, 2000)
    # a budget smaller than any plan's tables refuses every support at submit
    tiny = native.Server(data_bytes=2 * 16 * 1024 * 2, plan_bytes=1, slots=2, max_batch=8)
    sup = homogeneous_support(10, 6, rng)
    J6 = np.ascontiguousarray(sup.J, dtype=np.uint64)
    with pytest.raises(native.HiDFTError) as ei:
        tiny.submit(10, J6, np.zeros(64, np.complex64), np.zeros(64, np.complex64))
    assert ei.value.status_name == "HIDFT_ERR_OUT_OF_MEMORY"
    tiny.close()
    # budget for about two plans of up to 1024 points
    budget = 2 * (8 * 1023 + 2 * 1024)
    srv = native.Server(data_bytes=2 * 16 * 1024 * 2, plan_bytes=budget, slots=2, max_batch=8)
    # a request larger than one slot's region is rejected
    big = homogeneous_support(16, 12, rng)
    J = np.ascontiguousarray(big.J, dtype=np.uint64)
    f = sample_values(16, len(J), 1, rng)[0]
    out = np.zeros(len(J), dtype=np.complex64)
    with pytest.raises(native.HiDFTError) as ei:
        srv.submit(16, J, f, out)
    assert ei.value.status_name == "HIDFT_ERR_OUT_OF_MEMORY"
    # a non-homogeneous support is rejected at submit
    bad = np.array([1, 2, 4, 8], dtype=np.uint64)
    with pytest.raises(native.HiDFTError) as ei:
        srv.submit(4, bad, np.zeros(4, np.complex64), np.zeros(4, np.complex64))
    assert ei.value.status_name == "HIDFT_ERR_NOT_HOMOGENEOUS"
    # plans are evicted once no request holds them, within the budget
    sups = _supports(12, cfg=6)
    keep = []
    for M, J in sups:
        if len(J) > 1024:
            continue
        f = sample_values(M, len(J), 1, rng)[0]
        o = np.zeros(len(J), dtype=np.complex64)
        keep.append((M, J, f, o))
        srv.submit(M, J, f, o)
        srv.drain()
    st = srv.stats()
    need = sum(8 * (len(J) - 1) + 2 * len(J) for _, J, _, _ in keep)
    assert need > budget and st["plan_evictions"] >= 1, (need, st)
    assert st["plan_bytes_peak"] <= budget and st["plan_bytes_resident"] <= budget, st
    assert st["failed"] == 0 and st["plan_misses"] == len(keep), st
    for M, J, f, o in keep:
        assert np.array_equal(o, _alone(M, J, f[None, :]))
    srv.close()


def test_server_hard_plan_budget_under_load():
    """Four client threads submit, without waiting, 1200 requests over 24
    supports whose plans need about 4.5 times the plan budget.  The device
    bytes counted for plans never exceed the budget (peak reported by the
    server), plans are evicted and recreated, requests wait for plan memory
    instead of failing, and every result equals the request run alone, bit
    for bit."""
    sups = [x for x in _supports(40, cfg=8) if len(x[1]) <= 2048][:24]
    assert len(sups) == 24
    need = [8 * (len(J) - 1) + 2 * len(J) for _, J in sups]
    budget = sum(need) * 2 // 9
    assert max(need) <= budget < sum(need)
    srv = native.Server(data_bytes=16 << 20, plan_bytes=budget, slots=3, max_batch=32)
    results, errors = {}, []

    def client(cid):
        try:
            rng = rng_for(8, 300 + cid)
            for r in range(300):
                w = int(rng.integers(0, len(sups)))
                M, J = sups[w]
                f = sample_values(M, len(J), 1, rng)[0]
                o = np.full(len(J), np.nan, dtype=np.complex64)
                rid = srv.submit(M, J, f, o)
                results[(cid, r)] = (w, f, o, rid)
        except Exception as e:  # pragma: no cover
            errors.append(e)

    th = [threading.Thread(target=client, args=(c,)) for c in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    srv.drain()
    st = srv.stats()
    _say(f"budget {budget} B (working set {sum(need)} B): {st}")
    assert not errors
    assert st["completed"] == 1200 and st["failed"] == 0 and st["rejected"] == 0, st
    assert st["plan_bytes_peak"] <= budget, st
    assert st["plan_evictions"] > 0 and st["plan_misses"] > len(sups), st
    statuses = []
    while True:
        res = srv.poll()
        if len(res) == 0:
            break
        statuses.extend(res["status"].tolist())
    assert statuses and all(x == 0 for x in statuses)
    alone = {}
    for key in list(results)[::5]:
        w, f, o, _ = results[key]
        if w not in alone:
            alone[w] = {}
        M, J = sups[w]
        assert np.array_equal(o, _alone(M, J, f[None, :])), key
    srv.close()


def test_server_submit_many():
    """One call submits a burst of requests (one refused in the middle);
    each accepted request completes with the result of the request alone."""
    sups = _supports(6, cfg=9)
    rng = rng_for(9, 77)
    srv = native.Server(data_bytes=32 << 20, plan_bytes=16 << 20, slots=2, max_batch=64)
    recs = np.zeros(9, dtype=native.REQUEST_DTYPE)
    keep = []
    for i in range(9):
        M, J = sups[i % len(sups)]
        f = sample_values(M, len(J), 1, rng)[0]
        o = np.full(len(J), np.nan, dtype=np.complex64)
        keep.append((M, J, f, o))
        recs[i] = (M, J.ctypes.data, len(J), f.ctypes.data, o.ctypes.data)
    bad = np.array([1, 2, 4, 8], dtype=np.uint64)
    recs[4] = (4, bad.ctypes.data, 4, keep[4][2].ctypes.data, keep[4][3].ctypes.data)
    ids, sts = srv.submit_many(recs)
    assert sts[4] == 5 and ids[4] == 0               # HIDFT_ERR_NOT_HOMOGENEOUS
    assert all(sts[i] == 0 and ids[i] > 0 for i in range(9) if i != 4)
    acc = [int(ids[i]) for i in range(9) if i != 4]
    assert acc == sorted(acc) and len(set(acc)) == len(acc)  # ids in submission order
    srv.drain()
    for i, (M, J, f, o) in enumerate(keep):
        if i != 4:
            assert np.array_equal(o, _alone(M, J, f[None, :])), i
    # the same burst again, every plan now resident, with a NULL support in it
    for _, _, _, o in keep:
        o[:] = np.nan
    recs[7]["J"] = 0
    ids2, sts2 = srv.submit_many(recs)
    assert sts2[4] == 5 and sts2[7] == 1 and ids2[4] == 0 and ids2[7] == 0  # INVALID_ARGUMENT
    assert all(sts2[i] == 0 and ids2[i] > max(acc) for i in range(9) if i not in (4, 7))
    srv.drain()
    for i, (M, J, f, o) in enumerate(keep):
        if i not in (4, 7):
            assert np.array_equal(o, _alone(M, J, f[None, :])), i
    assert np.isnan(keep[7][3]).all()
    srv.close()


@pytest.mark.parametrize("s", [0, 5, 9, 12, 13, 14])
def test_server_single_request_batches(s):
    """A batch of up to four requests runs as one block per request with the
    descriptors passed with the launch (no table read): narrow sizes on the
    first quarter block, 2^13 and 2^14 points on the whole block.  Each
    request is drained before the next, so every batch holds one; each
    equals the request alone, bit for bit, and the FP64 oracle."""
    rng = rng_for(9, 300 + s)
    M = s + 6
    J = np.ascontiguousarray(homogeneous_support(M, s, rng).J, dtype=np.uint64)
    srv = native.Server(data_bytes=8 << 20, plan_bytes=8 << 20, slots=2, max_batch=8)
    plan = native.Plan(M, J.tolist())
    I = plan.samples().tolist()
    for rep in range(3):
        f = sample_values(M, len(J), 1, rng)
        o = np.full(len(J), np.nan, dtype=np.complex64)
        srv.submit(M, J, f[0], o)
        srv.drain()
        res = srv.poll()
        assert len(res) == 1 and res["status"][0] == 0 and res["batch_size"][0] == 1
        want = plan.execute(torch.from_numpy(f).cuda())[0].cpu().numpy()
        assert np.array_equal(o, want), (s, rep)
        ref = oracle.coefficients(M, J.tolist(), f.astype(np.complex128)) if s <= 9 else None
        if ref is not None:
            assert np.max(oracle.rel_l2(o[None, :].astype(np.complex128), ref)) <= 1e-5
    plan.close()
    srv.close()


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_server_few_request_batches(n):
    """n requests of mixed sizes (2^5..2^14 points) in one submit_many call,
    all plans resident: the scheduler takes them as one batch (one block per
    request up to four, the packed launch with tables from five).  Every
    result equals the request alone, bit for bit; repeated with the requests
    rotated."""
    rng = rng_for(9, 400 + n)
    sizes = [14, 5, 13, 9, 12][:n]
    sups = []
    for i, s in enumerate(sizes):
        M = s + 4 + i
        sups.append((M, np.ascontiguousarray(homogeneous_support(M, s, rng_for(9, 410 + i)).J,
                                             dtype=np.uint64)))
    plans = [native.Plan(M, J.tolist()) for M, J in sups]
    srv = native.Server(data_bytes=16 << 20, plan_bytes=16 << 20, slots=2, max_batch=8)
    warm = [np.zeros(len(J), dtype=np.complex64) for _, J in sups]
    warm_out = [np.empty_like(w) for w in warm]  # alive until polled
    for (M, J), w, wo in zip(sups, warm, warm_out):  # make every plan resident
        srv.submit(M, J, w, wo)
        srv.drain()
    srv.poll()
    for rot in range(2):
        order = [(i + rot) % n for i in range(n)]
        recs = np.zeros(n, dtype=native.REQUEST_DTYPE)
        keep = []
        for q, i in enumerate(order):
            M, J = sups[i]
            f = sample_values(M, len(J), 1, rng)[0]
            o = np.full(len(J), np.nan, dtype=np.complex64)
            keep.append((i, f, o))
            recs[q] = (M, J.ctypes.data, len(J), f.ctypes.data, o.ctypes.data)
        ids, sts = srv.submit_many(recs)
        assert (sts == 0).all()
        srv.drain()
        res = srv.poll()
        assert len(res) == n and (res["status"] == 0).all()
        _say(f"n={n} rot={rot}: batch sizes {sorted(set(res['batch_size'].tolist()))}")
        for i, f, o in keep:
            want = plans[i].execute(torch.from_numpy(f[None, :]).cuda())[0].cpu().numpy()
            assert np.array_equal(o, want), (n, rot, i)
    for p in plans:
        p.close()
    srv.close()


def test_server_large_batches_through_copy_helpers():
    """Bursts large enough that a batch's copies (samples in, coefficients
    out) pass the 1 MB at which the scheduler shares them with its helper
    threads: 3 bursts of 240 requests over 8 supports of 2^11..2^13 points,
    one submit_many each, batches of up to 512.  Every result equals the
    request run alone, bit for bit."""
    rng = rng_for(9, 99)
    sups = []
    for i, s in enumerate([11, 12, 13, 11, 12, 13, 12, 13]):
        M = int(rng.integers(s + 2, 23))
        sups.append((M, np.ascontiguousarray(homogeneous_support(M, s, rng_for(9, 100 + i)).J,
                                             dtype=np.uint64)))
    srv = native.Server(data_bytes=256 << 20, plan_bytes=64 << 20, slots=2, max_batch=512)
    ref_of = {}
    for burst in range(3):
        recs = np.zeros(240, dtype=native.REQUEST_DTYPE)
        keep = []
        for i in range(240):
            M, J = sups[(i + burst) % len(sups)]
            f = sample_values(M, len(J), 1, rng)[0]
            o = np.full(len(J), np.nan, dtype=np.complex64)
            keep.append((M, J, f, o))
            recs[i] = (M, J.ctypes.data, len(J), f.ctypes.data, o.ctypes.data)
        ids, sts = srv.submit_many(recs)
        assert (sts == 0).all() and (ids > 0).all()
        srv.drain()
        st = srv.stats()
        _say(f"burst {burst}: {st['batches']} batches so far")
        for i, (M, J, f, o) in enumerate(keep):
            key = (M, J.ctypes.data)
            if key not in ref_of:
                ref_of[key] = native.Plan(M, J.tolist())
            plan = ref_of[key]
            want = plan.execute(torch.from_numpy(f[None, :]).cuda())[0].cpu().numpy()
            assert np.array_equal(o, want), (burst, i)
    for plan in ref_of.values():
        plan.close()
    srv.close()


def test_server_concurrent_clients():
    sups = _supports(16, cfg=7)
    srv = native.Server(data_bytes=32 << 20, plan_bytes=64 << 20, slots=2, max_batch=64)
    errors = []
    results = {}

    def client(cid):
        try:
            rng = rng_for(7, 100 + cid)
            for r in range(120):
                w = int(rng.integers(0, len(sups)))
                M, J = sups[w]
                f = sample_values(M, len(J), 1, rng)[0]
                o = np.zeros(len(J), dtype=np.complex64)
                srv.submit(M, J, f, o)
                results[(cid, r)] = (w, f, o)
        except Exception as e:  # pragma: no cover
            errors.append(e)

    th = [threading.Thread(target=client, args=(c,)) for c in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    srv.drain()
    assert not errors
    assert srv.stats()["completed"] == 480
    for key in list(results)[::11]:
        w, f, o = results[key]
        M, J = sups[w]
        assert np.array_equal(o, _alone(M, J, f[None, :]))
    srv.close()


def test_serving_configuration_at_full_rate():
    """The serving configuration as measured: Poisson arrivals at 20 000
    requests/s (3 s here), 256 supports with N = 2^10..2^22 and k = 2^6..2^13
    chosen by a Zipf(1.1) law, one sample vector per support.  Every request
    completes; every 50th result, kept in its own buffer, equals the request
    run alone bit for bit; 20 of those (k <= 2048) against the FP64 oracle."""
    import time
    sups = _supports(256)
    vecs = [sample_values(M, len(J), 1, rng_for(5, 5000 + i))[0] for i, (M, J) in enumerate(sups)]
    rng = rng_for(5, 10 ** 6 + 1)
    rate, seconds = 20000.0, 3.0
    n = int(rate * seconds)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n))
    pz = np.arange(1, 257, dtype=np.float64) ** -1.1
    which = rng.choice(256, size=n, p=pz / pz.sum())
    keep = list(range(0, n, 50))
    kept = {i: np.full(len(sups[which[i]][1]), np.nan, dtype=np.complex64) for i in keep}
    pool = np.zeros((4096, 1 << 13), dtype=np.complex64)
    busy = np.zeros(len(pool), dtype=bool)
    slot_of, done = {}, 0
    srv = native.Server(data_bytes=256 << 20, plan_bytes=256 << 20, slots=4, max_batch=1024)
    for (M, J), f in zip(sups, vecs):  # plans resident before the clock starts
        srv.submit(M, J, f, pool[0, :len(J)])
    srv.drain()
    srv.poll()

    def collect(wait_us=0):
        nonlocal done
        res = srv.poll(wait_us)
        for r in res:
            assert int(r["status"]) == 0
            s = slot_of.pop(int(r["id"]))
            if s >= 0:
                busy[s] = False
        done += len(res)

    _say(f"serving at {rate:.0f} requests/s for {seconds} s: {n} requests")
    t0 = time.perf_counter()
    for i in range(n):
        while time.perf_counter() < t0 + arrivals[i]:
            collect()
        M, J = sups[which[i]]
        if i in kept:
            out, s = kept[i], -1
        else:
            s = i % len(pool)
            while busy[s]:
                collect(100)
            out = pool[s, :len(J)]
            busy[s] = True
        rid = srv.submit(M, J, vecs[which[i]], out)
        slot_of[rid] = s
    srv.drain()
    while len(slot_of):
        collect(1000)
    st = srv.stats()
    srv.close()
    assert done == n and st["completed"] >= n and st["rejected"] == 0
    alone = {}
    for i in keep:
        w = int(which[i])
        if w not in alone:
            M, J = sups[w]
            alone[w] = _alone(M, J, vecs[w][None, :])
        assert np.array_equal(kept[i], alone[w]), f"request {i} (support {w}) differs from alone"
    picked = [w for w in sorted(set(int(which[i]) for i in keep)) if len(sups[w][1]) <= 2048][:20]
    for w in picked:
        M, J = sups[w]
        plan = native.Plan(M, J.tolist())
        want = oracle.adjoint_coefficients(M, J.tolist(), plan.samples().tolist(),
                                           vecs[w][None, :].astype(np.complex128))[0]
        plan.close()
        err = np.linalg.norm(alone[w] - want) / np.linalg.norm(want)
        assert err <= 1e-5, (w, err)
    _say(f"{len(keep)} kept results equal alone; {len(picked)} supports against the oracle")
