"""Pins of the planner oracle (no GPU): feature definitions on hand-built matrices, the FP64
MLP gradient against central finite differences and the closed-form softmax CE gradient."""
import numpy as np
import pytest

from oracle import planner_ref as pr
from paper_2407_00829_amd.synth import from_coo, gen_random_small


def test_run_length_bins_closed_form():
    # L = 1 -> bin 0; L = 2 -> 4; L = 3 -> 6; L = 100 -> 4*6 + floor(400/64) - 4 = 26
    assert pr._log_bin(np.array([1, 2, 3, 4, 7, 100, 2 ** 16, 10 ** 6])).tolist() == \
        [0, 4, 6, 8, 11, 26, 63, 63]


def test_single_band_features():
    n = 300
    r = np.arange(10, 110)
    A = from_coo(n, n, r, r + 5, np.ones(r.size))
    f = pr.features(A)
    assert f[26] == 1.0 and f[:64].sum() == 1.0          # one run of length 100
    assert f[134] == 0.0 and f[135] == 1.0                # all on d = 5
    assert f[136] == np.float32(100 / n)
    assert f[137] == np.float32(1 / (2 * n - 1))
    assert f[139] == np.float32((n - 100) / n)


def test_dense_tile_features():
    D = np.zeros((32, 32), np.float32)
    D[0:16, 0:16] = 1.0       # one full tile: bin 63, dense
    D[16, 16] = 1.0           # one tile with a single entry: bin floor(64/256) = 0
    r, c = np.nonzero(D)
    f = pr.features(from_coo(32, 32, r, c, D[r, c]))
    assert f[64 + 63] == np.float32(256 / 257) and f[64 + 0] == np.float32(1 / 257)
    assert f[138] == np.float32(256 / 257)
    assert f[130] == np.float32(np.log1p(16))


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = pr.init_params(1).astype(np.float64)
    X = rng.standard_normal((6, pr.NFEAT))
    y = rng.integers(0, pr.NOUT, 6)
    loss, g = pr.mlp_loss_grad(p, X, y)
    idx = rng.choice(p.size, 300, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        num = (pr.mlp_loss_grad(p + e, X, y)[0] - pr.mlp_loss_grad(p - e, X, y)[0]) / (2 * h)
        assert abs(num - g[k]) <= 1e-6 * max(1.0, abs(g[k]))


def test_ce_gradient_closed_form():
    """dCE/dz = softmax(z) - onehot: with W1, W2 = 0 the logits are b3 and grad b3 is exact."""
    p = np.zeros(pr.NPARAM)
    P = pr.unflatten(p)
    P["b3"] = np.linspace(-1, 1, pr.NOUT)
    p = pr.flatten(P)
    X = np.ones((1, pr.NFEAT))
    loss, g = pr.mlp_loss_grad(p, X, np.array([3]))
    z = P["b3"]
    sm = np.exp(z - z.max()) / np.exp(z - z.max()).sum()
    onehot = np.eye(pr.NOUT)[3]
    assert np.allclose(pr.unflatten(g)["b3"], sm - onehot, atol=1e-15)
    assert np.isclose(loss, -np.log(sm[3]))


@pytest.mark.parametrize("seed", range(3))
def test_features_are_bounded(seed):
    A = gen_random_small(seed, 200, 150, 0.05, nbands=3, nblocks=3, block_max=30)
    f = pr.features(A)
    assert np.isclose(f[:64].sum(), 1.0, atol=1e-6) and np.isclose(f[64:128].sum(), 1.0, atol=1e-6)
    assert np.all(f[:128] >= 0) and np.all(f[134:] <= 1.0 + 1e-6)
