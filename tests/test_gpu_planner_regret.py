"""Live regret of the trained planner (paper_2407_00829_amd/planner_weights.npz) on held-out
matrices: the exhaustive timed search is the yardstick; the learned choice must stay close to it
and beat the fixed default plan on average."""
import numpy as np
import pytest

from paper_2407_00829_amd import planner

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2407_00829_amd import sable  # noqa: E402


def test_learned_plan_regret_and_gain():
    params, mean, std, tau = planner.load_weights(planner.WEIGHTS)
    P = torch.from_numpy(params).cuda()
    regrets, gains = [], []
    for seed in range(100000, 100016):
        _, A, x = planner.make_matrix(seed)
        rec = planner.label_matrix(A, x, reps=20)
        ip, ix, vv = sable.device_csr(A)
        xd = torch.from_numpy(x).cuda()
        y = torch.empty(A.nrows, device="cuda")
        p, c, conf, fb = sable.sable_plan_auto(A.nrows, A.ncols, ip, ix, vv, P, mean, std, 0.0, xd, y)
        assert not fb and 0 <= c < 15
        t = np.array(rec["times"])
        regrets.append(t[c] / t.min() - 1.0)
        gains.append(rec["t_default"] / t[c])
        print(f"  seed {seed}: class {planner.class_name(c)} regret {regrets[-1]:.3f}")
    mean_regret = float(np.mean(regrets))
    gain = float(np.exp(np.mean(np.log(gains))))
    print(f"  mean regret {mean_regret:.4f}, geomean gain over the default plan {gain:.3f}")
    assert mean_regret <= 0.15
    assert gain >= 1.0
