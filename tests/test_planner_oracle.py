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


# ---- forward pass (the checker of the GPU forward kernel and of the planner's choice) ----

def _net(**kw):
    P = pr.unflatten(np.zeros(pr.NPARAM))
    for k, v in kw.items():
        P[k][...] = v
    return P


def test_forward_zero_weights_gives_output_bias():
    """W1 = W2 = W3 = 0: every hidden unit is relu(bias) and contributes nothing, so the
    logits are b3 exactly, whatever the input and the other biases."""
    P = _net(b1=np.linspace(-2, 2, pr.NH), b2=np.linspace(3, -1, pr.NH), b3=np.arange(pr.NOUT) - 7.5)
    X = np.random.default_rng(1).standard_normal((5, pr.NFEAT))
    Z = pr.mlp_forward(pr.flatten(P), X)
    assert np.array_equal(Z, np.tile(P["b3"], (5, 1)))


def test_forward_hand_built_network():
    """Units built by hand so that every piece of the forward pass shows in the logits:
    layer 1 unit 0 = relu(x0), unit 1 = relu(-x0), unit 2 = relu(x1 - 1) (bias b1);
    layer 2 unit 0 = relu(h0 - h1 + 0.25) (b2), unit 1 = relu(h1 - h0), unit 2 = relu(h2),
    unit 3 = relu(2 h0) (W2 is not symmetric, so a transposed W2 changes the result);
    logits: z0 = g0 - g1 (a signed sum), z1 = g1 + g0, z2 = g2 + 0.5 (b3), z3 = g3."""
    W1 = np.zeros((pr.NH, pr.NFEAT))
    W1[0, 0], W1[1, 0], W1[2, 1] = 1.0, -1.0, 1.0
    b1 = np.zeros(pr.NH)
    b1[2] = -1.0
    W2 = np.zeros((pr.NH, pr.NH))
    W2[0, 0], W2[0, 1] = 1.0, -1.0
    W2[1, 1], W2[1, 0] = 1.0, -1.0
    W2[2, 2] = 1.0
    W2[3, 0] = 2.0
    b2 = np.zeros(pr.NH)
    b2[0] = 0.25
    W3 = np.zeros((pr.NOUT, pr.NH))
    W3[0, 0], W3[0, 1] = 1.0, -1.0
    W3[1, 0], W3[1, 1] = 1.0, 1.0
    W3[2, 2] = 1.0
    W3[3, 3] = 1.0
    b3 = np.zeros(pr.NOUT)
    b3[2] = 0.5
    p = pr.flatten(_net(W1=W1, b1=b1, W2=W2, b2=b2, W3=W3, b3=b3))

    def expect(x0, x1):
        h0, h1, h2 = max(x0, 0.0), max(-x0, 0.0), max(x1 - 1.0, 0.0)
        g0, g1, g2, g3 = max(h0 - h1 + 0.25, 0.0), max(h1 - h0, 0.0), max(h2, 0.0), max(2 * h0, 0.0)
        z = np.zeros(pr.NOUT)
        z[0], z[1], z[2], z[3] = g0 - g1, g1 + g0, g2 + 0.5, g3
        return z

    pts = [(-2.5, 3.0), (2.0, 0.5), (0.0, 1.0), (-0.125, -4.0), (0.75, 2.25)]
    X = np.zeros((len(pts), pr.NFEAT))
    for k, (a, b) in enumerate(pts):
        X[k, 0], X[k, 1] = a, b
    Z = pr.mlp_forward(p, X)
    for k, (a, b) in enumerate(pts):
        assert np.array_equal(Z[k], expect(a, b)), (a, b, Z[k][:4], expect(a, b)[:4])
    # x0 = -2.5: z0 = relu(0 - 2.5 + 0.25) - relu(2.5) = -2.5 and z1 = 2.5 (no ReLU drop)
    assert Z[0][0] == -2.5 and Z[0][1] == 2.5 and Z[0][2] == 2.5


def test_forward_rows_are_independent_and_match_training_loss():
    """A batch is its rows evaluated one by one, and the softmax cross-entropy of the forward
    logits equals the loss the training pass computes on the same batch."""
    rng = np.random.default_rng(4)
    p = pr.init_params(3).astype(np.float64)
    p[pr.NPARAM - pr.NOUT:] = rng.standard_normal(pr.NOUT)  # non-zero b3
    X = rng.standard_normal((7, pr.NFEAT))
    y = rng.integers(0, pr.NOUT, 7)
    Z = pr.mlp_forward(p, X)
    for k in range(7):
        assert np.allclose(pr.mlp_forward(p, X[k:k + 1])[0], Z[k], rtol=0, atol=1e-13)
    zs = Z - Z.max(axis=1, keepdims=True)
    ce = np.mean(np.log(np.exp(zs).sum(axis=1)) - zs[np.arange(7), y])
    loss, _ = pr.mlp_loss_grad(p, X, y)
    assert abs(ce - loss) <= 1e-13
