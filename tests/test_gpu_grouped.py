"""Uneven batch in one persistent launch (grouped execution) against the oracle.

2048 instances, each with its own seeded homogeneous J: N log-uniform over
2^12..2^24, k log-uniform over 2^6..2^14 with k <= N/4, plus composite
supports (direct sums of homogeneous blocks on disjoint bit ranges).  Every
instance is checked bit-for-bit against the single-plan fused path (itself
checked against the oracle), every instance on the energy identity and on
64 seeded coefficient positions against the FP64 oracle (all of them when
k <= 64), and a sample of instances on every coefficient.
"""
import sys

import numpy as np
import pytest

import oracle
from tests.positions import positions_vs_oracle
from workloads import homogeneous_support, rng_for, sample_values, uneven_instances

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


def _instances(n):
    """(M, J list, levels) for n seeded instances of the uneven configuration."""
    return [(M, sup.J.tolist(), sup.levels) for M, sup in uneven_instances(n)]


def _expected_packs(ks, grid):
    """Pack count of the host packer: k >= 2^13 in wide packs of
    1024 / 2^(s-4) slots, whose partial last round of the grid is split until
    it has a pack per block or every pack holds one instance; smaller sizes in
    narrow packs of 256 / 2^max(s-4, 0) slots, split likewise up to 2 per
    block of the grid."""
    sizes = {}
    for k in ks:
        s = int(k).bit_length() - 1
        sizes[s] = sizes.get(s, 0) + 1
    wide, narrow = [], []
    for s in sorted(sizes, reverse=True):
        per = (1024 >> (s - 4)) if s >= 13 else (256 >> max(s - 4, 0))
        n = sizes[s]
        (wide if s >= 13 else narrow).extend(min(per, n - i) for i in range(0, n, per))
    full = len(wide) // grid * grid
    n_wide = len(wide) if full in (0, len(wide)) else full + min(grid, sum(wide[full:]))
    n_narrow = len(narrow) if len(narrow) >= 2 * grid else min(2 * grid, sum(narrow))
    return n_wide + n_narrow


def _energy_rel(c, f, M, k):
    N = float(1 << M)
    return abs(np.sum(np.abs(c) ** 2) - (N * N / k) * np.sum(np.abs(f) ** 2)) / ((N * N / k) * np.sum(np.abs(f) ** 2))


def test_config3_uneven_batch_one_launch():
    insts = _instances(2048)
    plans, xs, ys = [], [], []
    rng = rng_for(3, 99999)
    for M, J, _ in insts:
        plans.append(native.Plan(M, J))
        k = len(J)
        xs.append(torch.from_numpy(sample_values(M, k, 1, rng)[0]).cuda())
        ys.append(torch.full((k,), complex(np.nan, np.nan), dtype=torch.complex64, device="cuda"))
    ks = np.array([p.k for p in plans])
    _say(f"C3: {len(plans)} instances, k from {ks.min()} to {ks.max()}, {ks.sum()} points")
    items = [(p, x.data_ptr(), p.k, y.data_ptr(), p.k, 1) for p, x, y in zip(plans, xs, ys)]
    grp = native.Group(items)
    assert grp.n_instances == 2048
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert grp.n_packs == _expected_packs(ks, cus), (grp.n_packs, _expected_packs(ks, cus))
    grp.execute()
    torch.cuda.synchronize()
    _say(f"C3: {grp.n_packs} packs executed on {cus} blocks")
    got = [y.cpu().numpy().astype(np.complex128) for y in ys]
    # fused single-plan path on each instance: bit-identical
    n_diff = 0
    for p, x, g in zip(plans, xs, got):
        z = p.execute(x)
        torch.cuda.synchronize()
        n_diff += not np.array_equal(z[0].cpu().numpy().astype(np.complex128), g)
    assert n_diff == 0, f"{n_diff} instances differ from the fused path"
    # energy identity on every instance
    worst = max(_energy_rel(g, x.cpu().numpy(), M, len(J)) for g, x, (M, J, _) in zip(got, xs, insts))
    assert worst <= 2e-5, worst
    # oracle on a sample: every instance with k <= 64 plus 40 random others
    pick = [i for i in range(len(insts)) if ks[i] <= 64]
    pick += rng_for(3, 12345).choice(len(insts), 40, replace=False).tolist()
    errs = []
    for i in sorted(set(pick)):
        M, J, levels = insts[i]
        f = xs[i].cpu().numpy().astype(np.complex128)
        I = plans[i].samples().tolist()
        assert I == sorted(oracle.sample_pattern_recursive(M, levels))
        if len(J) <= 2048:
            want = oracle.adjoint_coefficients(M, J, I, f)
            errs.append(float(oracle.rel_l2(got[i], want)))
        else:
            sel = rng_for(3, 777 + i).choice(len(J), 64, replace=False)
            want = oracle.adjoint_coefficients(M, [J[t] for t in sel], I, f, k=len(J))
            errs.append(float(oracle.rel_l2(got[i][sel], want)))
    _say(f"C3: oracle on {len(errs)} instances, rel-L2 max {max(errs):.3e}")
    assert max(errs) <= 1e-5
    # every instance on 64 positions of its own
    prng = rng_for(3, 4242)
    per_inst = []
    for i, (M, J, _) in enumerate(insts):
        f = xs[i].cpu().numpy()[None, :]
        per_inst.append(positions_vs_oracle(M, J, plans[i].samples().tolist(), f,
                                            got[i][None, :], 64, prng)[0])
    _say(f"C3: all {len(insts)} instances on 64 positions each: rel-L2 max {max(per_inst):.3e}")
    assert max(per_inst) <= 1e-5
    grp.close()
    for p in plans:
        p.close()


def test_grouped_mixed_batches_and_ragged_packs():
    """Items with several rows, strides, every size 2^0..2^14, partial packs."""
    rng = rng_for(3, 5000)
    items, refs, bufs = [], [], []
    for s in range(0, 15):
        M = max(s, 1) + int(rng.integers(0, 6))
        sup = homogeneous_support(M, s, rng)
        plan = native.Plan(M, sup.J.tolist())
        k = plan.k
        batch = int(rng.integers(1, 5))
        f = sample_values(M, k, batch, rng)
        ld_in, ld_out = k + int(rng.integers(0, 3)), k + int(rng.integers(0, 3))
        x = torch.zeros((batch, ld_in), dtype=torch.complex64, device="cuda")
        x[:, :k] = torch.from_numpy(f).cuda()
        y = torch.zeros((batch, ld_out), dtype=torch.complex64, device="cuda")
        items.append((plan, x.data_ptr(), ld_in, y.data_ptr(), ld_out, batch))
        bufs.append((plan, x, y, f, M, sup.J.tolist(), k))
    grp = native.Group(items)
    grp.execute()
    grp.execute()  # twice: same result
    torch.cuda.synchronize()
    for plan, x, y, f, M, J, k in bufs:
        got = y[:, :k].cpu().numpy().astype(np.complex128)
        rows = range(f.shape[0]) if k <= 2048 else [0]
        want = oracle.adjoint_coefficients(M, J, plan.samples().tolist(), f[list(rows)])
        err = np.max(oracle.rel_l2(got[list(rows)], want))
        assert err <= 1e-5, (k, err)
    grp.close()


@pytest.mark.parametrize("s,full_rounds,tail_packs,ragged", [(14, 1, 10, 0), (13, 1, 37, 1),
                                                           (12, 1, 0, 0), (8, 0, 44, 17),
                                                           (6, 1, 44, 3)])
def test_grouped_last_round_spreading(s, full_rounds, tail_packs, ragged):
    """The packer's edge cases, one plan with many rows each.  Wide packs
    (a round is one pack per block): a partial last round of single-instance
    packs (2^14 points, nothing to split), and a partial round of 2-instance
    packs split to single ones.  Narrow packs (a round is two packs per
    block): exactly one round (nothing to spread), fewer packs than a round
    (split until every instance has its own), and more than a round (kept
    full).  Pack count as the model says; every row bit-identical to
    hidft_execute."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    rng = rng_for(3, 8000 + s)
    M = s + 6
    plan = native.Plan(M, homogeneous_support(M, s, rng).J.tolist())
    k = plan.k
    per = (1024 >> (s - 4)) if s >= 13 else (256 >> max(s - 4, 0))  # instances per full pack
    round_packs = cus if s >= 13 else 2 * cus
    batch = (full_rounds * round_packs + tail_packs) * per + ragged
    _say(f"case s={s} batch={batch} cus={cus}")
    x = torch.from_numpy(sample_values(M, k, batch, rng)).cuda()
    y = torch.full_like(x, complex(np.nan, np.nan))
    grp = native.Group([(plan, x.data_ptr(), k, y.data_ptr(), k, batch)])
    want_packs = _expected_packs([k] * batch, cus)
    assert grp.n_packs == want_packs, (grp.n_packs, want_packs)
    grp.execute()
    ref = plan.execute(x)
    torch.cuda.synchronize()
    assert torch.equal(y, ref)
    # a second launch finds the narrow-pack queue back at zero
    y.fill_(complex(np.nan, np.nan))
    grp.execute()
    torch.cuda.synchronize()
    assert torch.equal(y, ref)
    grp.close()
    plan.close()


def test_group_argument_errors():
    M, s = 12, 6
    sup = homogeneous_support(M, s, rng_for(3, 6000))
    plan = native.Plan(M, sup.J.tolist())
    x = torch.zeros((2, plan.k), dtype=torch.complex64, device="cuda")
    with pytest.raises(native.HiDFTError):
        native.Group([(plan, x.data_ptr() + 4, plan.k, x.data_ptr(), plan.k, 1)])
    with pytest.raises(native.HiDFTError):
        native.Group([(plan, x.data_ptr(), plan.k - 1, x.data_ptr(), plan.k, 1)])
    with pytest.raises(native.HiDFTError):
        native.Group([])


def test_group_configurations_and_autotune():
    """Every launch configuration of a group (short group first or last, packs
    largest first or alternating) gives each instance exactly the result of
    hidft_execute_config with the same schedule; the order changes nothing.
    More packs than the persistent grid, so the alternating order reorders.
    The autotuner leaves the group in one of the configurations."""
    rng = rng_for(3, 7000)
    sizes = [14] * 200 + [13] * 200 + [12] * 100 + [s for s in range(0, 12) for _ in range(4)]
    plans, xs, ys = [], [], []
    for s in sizes:
        M = max(s, 1) + int(rng.integers(0, 8))
        plan = native.Plan(M, homogeneous_support(M, s, rng).J.tolist())
        plans.append(plan)
        xs.append(torch.from_numpy(sample_values(M, plan.k, 1, rng)[0]).cuda())
        ys.append(torch.empty(plan.k, dtype=torch.complex64, device="cuda"))
    grp = native.Group([(p, x.data_ptr(), p.k, y.data_ptr(), p.k, 1)
                        for p, x, y in zip(plans, xs, ys)])
    assert grp.n_packs > 256
    _say(f"group: {grp.n_instances} instances, {grp.n_packs} packs")
    want = {}
    for sched in (native.SCHED_SHORT_LAST, native.SCHED_SHORT_FIRST):
        out = []
        for p, x in zip(plans, xs):
            z = torch.empty(p.k, dtype=torch.complex64, device="cuda")
            p.execute_ptr(x.data_ptr(), p.k, z.data_ptr(), p.k, 1,
                          config=native.ExecConfig(native.PREC_FP32, sched, 16, 0))
            out.append(z)
        torch.cuda.synchronize()
        want[sched] = [z.cpu().numpy() for z in out]

    def check(sched, what):
        torch.cuda.synchronize()
        bad = sum(not np.array_equal(y.cpu().numpy(), w) for y, w in zip(ys, want[sched]))
        assert bad == 0, f"{what}: {bad} instances differ"

    for sched in (native.SCHED_SHORT_LAST, native.SCHED_SHORT_FIRST):
        for order in (native.GROUP_ORDER_LARGEST_FIRST, native.GROUP_ORDER_ALTERNATE):
            for y in ys:
                y.fill_(complex(np.nan, np.nan))
            grp.set_config(sched, order)
            assert (grp.config().schedule, grp.config().order) == (sched, order)
            grp.execute()
            check(sched, f"schedule {sched}, order {order}")
    cfg, us = grp.autotune(reps=3)
    _say(f"group autotune: schedule {cfg.schedule}, order {cfg.order}, {us:.1f} us")
    assert us > 0 and cfg.schedule in (native.SCHED_SHORT_LAST, native.SCHED_SHORT_FIRST)
    assert (grp.config().schedule, grp.config().order) == (cfg.schedule, cfg.order)
    for y in ys:
        y.fill_(complex(np.nan, np.nan))
    grp.execute()
    check(cfg.schedule, "tuned")
    with pytest.raises(native.HiDFTError):
        grp.set_config(7, 0)
    with pytest.raises(native.HiDFTError):
        grp.set_config(0, 5)
    grp.close()
    for p in plans:
        p.close()
