"""GPU planner kernels against the planner oracle: features, MLP forward, gradients, Adam
training, exhaustive search and the learned-plan entry point."""
import numpy as np
import pytest

from oracle import planner_ref as pr
from paper_2407_00829_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2407_00829_amd import sable  # noqa: E402


@pytest.mark.parametrize("seed", range(4))
def test_features_match_oracle(seed):
    A = synth.gen_random_small(seed, 500 + 97 * seed, 400, 0.02, nbands=3, nblocks=4, block_max=40)
    ip, ix, vv = sable.device_csr(A)
    f = sable.sable_features(A.nrows, A.ncols, ip, ix, vv)
    ref = pr.features(A)
    assert np.allclose(f, ref, rtol=1e-6, atol=1e-7), np.nonzero(~np.isclose(f, ref, rtol=1e-6, atol=1e-7))


def test_features_c1():
    A, _ = synth.gen_c1(0, n=2048)
    ip, ix, vv = sable.device_csr(A)
    f = sable.sable_features(A.nrows, A.ncols, ip, ix, vv)
    assert np.allclose(f, pr.features(A), rtol=1e-6, atol=1e-7)


def norm_rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_forward_and_gradients_match_fp64_oracle():
    rng = np.random.default_rng(3)
    B = 37
    p = pr.init_params(5)
    X = rng.standard_normal((B, pr.NFEAT)).astype(np.float32)
    y = rng.integers(0, pr.NOUT, B).astype(np.int32)
    P = torch.from_numpy(p).cuda()
    Xd = torch.from_numpy(X).cuda()
    L = torch.empty(B, pr.NOUT, device="cuda")
    sable.sable_mlp_forward(P, Xd, L)
    torch.cuda.synchronize()
    assert norm_rel(L.cpu().numpy(), pr.mlp_forward(p, X)) <= 1e-5
    G = torch.zeros_like(P)
    loss = sable.sable_mlp_train_step(P, G, None, None, Xd, torch.from_numpy(y).cuda(),
                                      0.0, 0.9, 0.999, 1e-8, 0)
    rl, rg = pr.mlp_loss_grad(p, X, y)
    assert abs(loss - rl) <= 1e-5 * max(1.0, abs(rl))
    g = G.cpu().numpy()
    ref = pr.unflatten(rg)
    got = pr.unflatten(g)
    for k in ref:
        assert norm_rel(got[k], ref[k]) <= 1e-4, k
    assert np.array_equal(P.cpu().numpy(), p)  # t = 0 leaves parameters untouched


def test_adam_step_matches_reference():
    rng = np.random.default_rng(4)
    p = pr.init_params(6)
    X = rng.standard_normal((16, pr.NFEAT)).astype(np.float32)
    y = rng.integers(0, pr.NOUT, 16).astype(np.int32)
    P = torch.from_numpy(p.copy()).cuda()
    G, M, V = (torch.zeros_like(P) for _ in range(3))
    sable.sable_mlp_train_step(P, G, M, V, torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(),
                               1e-2, 0.9, 0.999, 1e-8, 1)
    _, g = pr.mlp_loss_grad(p, X, y)
    m = 0.1 * g
    v = 0.001 * g * g
    ref = p - 1e-2 * (m / 0.1) / (np.sqrt(v / 0.001) + 1e-8)
    assert norm_rel(P.cpu().numpy(), ref) <= 1e-4


def test_training_learns_separable_labels():
    from paper_2407_00829_amd import planner
    rng = np.random.default_rng(0)
    N = 600
    # one noisy cluster of feature vectors per class (structure types); the same training
    # with the FP64 oracle reaches 100% held-out accuracy
    centres = rng.standard_normal((pr.NOUT, pr.NFEAT))
    y = rng.integers(0, pr.NOUT, N).astype(np.int32)
    X = (centres[y] + 0.8 * rng.standard_normal((N, pr.NFEAT))).astype(np.float32)
    params, mean, std, hist = planner.train(X[:500], y[:500], epochs=40, log=None)
    assert hist[-1] < hist[0] * 0.1
    pred, _ = planner.predict(params, mean, std, X[500:])
    assert np.mean(pred == y[500:]) > 0.9


def test_exhaustive_and_auto_plans():
    A, x = synth.gen_mixed(3, n=20000, rowlen=12.0, pi=np.array([0.4, 0.4, 0.2]))
    ip, ix, vv = sable.device_csr(A)
    xd = torch.from_numpy(x).cuda()
    y = torch.empty(A.nrows, device="cuda")
    p, best, times = sable.sable_plan_exhaustive(A.nrows, A.ncols, ip, ix, vv, xd, y, 5)
    assert best == int(np.argmin(times)) and times.min() > 0
    assert times[1] == times[0] and times[2] == times[0]
    import oracle
    sable.sable_spmv(p, xd, y)
    torch.cuda.synchronize()
    assert oracle.rel_err(y.cpu().numpy(), oracle.spmv(A, x)) <= 1e-5
    params = torch.from_numpy(pr.init_params(2)).cuda()
    mean, std = np.zeros(140, np.float32), np.ones(140, np.float32)
    q, c, conf, fb = sable.sable_plan_auto(A.nrows, A.ncols, ip, ix, vv, params, mean, std, 1.01,
                                           xd, y)
    assert fb and 0 <= c < 15
    q2, c2, conf2, fb2 = sable.sable_plan_auto(A.nrows, A.ncols, ip, ix, vv, params, mean, std, 0.0,
                                               xd, y)
    assert not fb2 and 0 < conf2 <= 1
    f = sable.sable_features(A.nrows, A.ncols, ip, ix, vv)
    assert c2 == int(np.argmax(pr.mlp_forward(pr.init_params(2), f[None, :])))


def test_partition_hash_follows_the_partition():
    """Plans of the 15 classes: equal partition hashes exactly when the exported partitions
    (every format array, owner and slot) are equal, so the exhaustive search may time such
    classes once."""
    A, _ = synth.gen_mixed(5, n=12000, rowlen=10.0, pi=np.array([0.3, 0.5, 0.2]))
    ip, ix, vv = sable.device_csr(A)
    lists = [[3], [1, 3], [2, 3], [1, 2, 3], [2, 1, 3]]
    seen = []
    for li, kinds in enumerate(lists):
        for delta in (500, 700, 900):
            th = sable.Thresholds(delta_band_pm=delta, delta_block_pm=delta)
            p = sable.sable_plan(A.nrows, A.ncols, ip, ix, vv, kinds, sable.SABLE_VBR_TILED, th=th)
            h = sable.sable_plan_info(p)["partition_hash"]
            ex = sable.sable_plan_export(p)
            q = sable.sable_plan(A.nrows, A.ncols, ip, ix, vv, kinds, sable.SABLE_VBR_TILED, th=th)
            assert sable.sable_plan_info(q)["partition_hash"] == h  # deterministic
            seen.append((h, ex))
    keys = [k for k in seen[0][1] if isinstance(seen[0][1][k], np.ndarray)]
    distinct = 0
    for i in range(len(seen)):
        for j in range(i):
            same = all(seen[i][1][k].shape == seen[j][1][k].shape and
                       np.array_equal(seen[i][1][k].view(np.uint8), seen[j][1][k].view(np.uint8))
                       for k in keys)
            assert (seen[i][0] == seen[j][0]) == same, (i, j)
            distinct += not same
    assert distinct > 0
