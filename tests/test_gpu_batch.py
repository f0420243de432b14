"""Batched persistent hipGraph launch: every item bitwise equal to its standalone launch with
the same tile kernel, across several graph replays with eager work in between; latencies are
recorded; items without rows complete at once."""
import numpy as np
import pytest

from paper_2407_00829_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2407_00829_amd import sable  # noqa: E402


def make_items(count, seed=0):
    rng = np.random.default_rng(seed)
    plans, items, refs = [], [], []
    kinds = [sable.SABLE_X_VDIA, sable.SABLE_X_VBR, sable.SABLE_X_CSR]
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(500), np.log(30000))))
        A, x = synth.gen_mixed(1000 + i, n=n, rowlen=float(rng.uniform(4, 20)),
                               pi=rng.dirichlet([1, 1, 1]))
        p = sable.plan_host(A, kinds, sable.SABLE_VBR_TILED,
                            sable.Thresholds(amin_band=256, amin_block=64))
        op = int(rng.integers(0, 2))
        if op == 0:
            sable.sable_plan_set_variant(p, 0, int(rng.choice([0, 1, 2, 8, 9, 10, 5, 12])))
            xd = torch.from_numpy(x).cuda()
            yd = torch.full((n,), float("nan"), device="cuda")
            items.append((0, 1, xd, yd))
        else:
            X = torch.from_numpy(synth.gen_dense_matrix(i, n, 16)).cuda()
            Y = torch.full((n, 16), float("nan"), device="cuda")
            items.append((1, 16, X, Y))
        plans.append(p)
    return plans, items


STREAMED = (0, 1, 2, 8, 9, 10)


def standalone(plans, items):
    """Standalone results with the kernels a batch runs: SpMV items with the plan's streamed
    tile variant (the 256-row streamed tile, variant 0, for any other variant) without the
    far-column pass, SpMM items as planned. A CSR-only plan's SpMV runs the plain kernels, so
    its streamed tile is the plain variant of the same tile height."""
    outs = []
    for p, (op, n, x, y) in zip(plans, items):
        z = torch.empty_like(y)
        if op == 0:
            info = sable.sable_plan_info(p)
            v, fs, pv = info["spmv_variant"], info["far_split"], info["plain_variant"]
            vs = v if v in STREAMED else 0
            sable.sable_plan_set_variant(p, 0, vs)
            sable.sable_plan_set_variant(p, 3, 0)
            sable.sable_plan_set_variant(p, 2, vs if vs < 8 else vs + 2)
            sable.sable_spmv(p, x, z)
            sable.sable_plan_set_variant(p, 0, v)
            sable.sable_plan_set_variant(p, 3, fs)
            sable.sable_plan_set_variant(p, 2, pv)
        else:
            sable.sable_spmm(p, x, z, n)
        outs.append(z)
    torch.cuda.synchronize()
    return outs


def test_batch_bitwise_equal_and_replays():
    plans, items = make_items(24)
    ref = standalone(plans, items)
    b = sable.sable_batch_create(plans, items)
    for rep in range(3):
        for (_, _, _, y) in items:
            y.fill_(float("nan"))  # eager work between replays
        sable.sable_batch_run(b)
        torch.cuda.synchronize()
        for i, ((_, _, _, y), r) in enumerate(zip(items, ref)):
            assert torch.equal(y, r), (rep, i)
        ticks, hz = sable.sable_batch_latencies(b)
        assert hz > 0 and np.all(ticks > 0)
    b.destroy()


def test_batch_with_empty_items():
    plans, items = make_items(6, seed=3)
    E = synth.from_coo(0, 7, [], [], [])
    pe = sable.plan_host(E, [sable.SABLE_X_VDIA, sable.SABLE_X_VBR, sable.SABLE_X_CSR],
                         sable.SABLE_VBR_TILED, sable.Thresholds())
    ye = torch.zeros(0, device="cuda")
    plans = plans[:3] + [pe] + plans[3:]
    items = items[:3] + [(0, 1, torch.zeros(7, device="cuda"), ye)] + items[3:]
    ref = standalone(plans, items)
    b = sable.sable_batch_create(plans, items)
    for rep in range(2):
        sable.sable_batch_run(b)
        torch.cuda.synchronize()
        for i, ((_, _, _, y), r) in enumerate(zip(items, ref)):
            assert torch.equal(y, r), (rep, i)
        ticks, hz = sable.sable_batch_latencies(b)
        assert ticks[3] == 0 and np.all(np.delete(ticks, 3) > 0)
    b.destroy()


def test_batch_rejects_bad_items():
    plans, items = make_items(2, seed=5)
    bad = [(0, 2, items[0][2], items[0][3])] + items[1:]
    with pytest.raises(sable.SableError):
        sable.sable_batch_create(plans, bad)


def test_serving_batch_full_size():
    """The benchmark's serving batch: 256 generated matrices (1e3 - 2e5 rows, SpMV or SpMM
    with 16 right-hand sides), planner-chosen plans; every item bitwise equal to its
    standalone launch, and sampled items against the FP64 oracle."""
    import concurrent.futures as cf

    import oracle
    from paper_2407_00829_amd import planner
    params, mean, std, tau = planner.load_weights(planner.WEIGHTS)
    Pd = torch.from_numpy(params).cuda()
    with cf.ProcessPoolExecutor(8) as ex:
        mats = list(ex.map(synth.gen_c5_matrix, range(256)))
    plans, items = [], []
    for i, (A, kind, op) in enumerate(mats):
        ip, ix, vv = sable.device_csr(A)
        x = torch.from_numpy(synth.gen_dense_vector(i, A.ncols)).cuda()
        y = torch.empty(A.nrows, device="cuda")
        p, _, _, _ = sable.sable_plan_auto(A.nrows, A.ncols, ip, ix, vv, Pd, mean, std, tau, x, y)
        p._src = (ip, ix, vv)
        if op == 0:
            items.append((0, 1, x, torch.full((A.nrows,), float("nan"), device="cuda")))
        else:
            X = torch.from_numpy(synth.gen_dense_matrix(i, A.ncols, 16)).cuda()
            items.append((1, 16, X, torch.full((A.nrows, 16), float("nan"), device="cuda")))
        plans.append(p)
    print(f"[batch] {len(plans)} plans", flush=True)
    ref = standalone(plans, items)
    b = sable.sable_batch_create(plans, items)
    sable.sable_batch_run(b)
    torch.cuda.synchronize()
    for i, ((_, _, _, y), r) in enumerate(zip(items, ref)):
        assert torch.equal(y, r), i
    for i in range(0, 256, 32):
        A, _, op = mats[i]
        _, n, x, y = items[i]
        if op == 0:
            err = oracle.rel_err(y.cpu().numpy(), oracle.spmv(A, x.cpu().numpy()))
            assert err <= 1e-5, (i, err)
        else:
            rows = np.arange(min(A.nrows, 4096))
            err = oracle.rel_err(y.cpu().numpy()[rows], oracle.spmm_rows(A, x.cpu().numpy(), rows))
            assert err <= 1e-4, (i, err)
    b.destroy()
