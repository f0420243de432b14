"""Live regret of the trained planner (paper_2407_00829_amd/planner_weights.npz) on held-out
matrices of the planner's generator (n ~ logU[1e4, 1e6], mean row length ~ U[4, 64]; the
first 32 held-out seeds with at least 5e4 rows): each matrix is labelled afresh by the
exhaustive timed search (every class, the plain CSR kernel and the default list timed the
same way inside the library). The shipped policy (the network's
class, the exhaustive search below the stored confidence threshold) must stay within 5% of the
fastest class on average; the network alone must stay within one point of always choosing the
best single class (stored with the weights, chosen on the training labels; on these seeds the
stored labels give 2.5% against 3.9%, and the mean over 32 re-timed matrices carries about a
point of timing noise), and the shipped choice must beat the paper's default list."""
import time

import numpy as np
import pytest

from paper_2407_00829_amd import planner

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2407_00829_amd import sable  # noqa: E402

# The first 32 held-out seeds with n >= 5e4 (products of 10 us and more). Below that (products
# of ~6 us) two timings of one kernel differ by 20% and more from run to run, so a fresh
# labelling of those measures timing noise rather than the choice; the offline evaluation on
# all 200 held-out matrices covers them.
SEEDS = [s for s in range(100000, 100200) if planner.matrix_params(s)[0] >= 5e4][:32]
REPS = 20  # as in the training labels


def test_learned_plan_regret_and_gain():
    params, mean, std, tau = planner.load_weights(planner.WEIGHTS)
    cc = planner.load_const_class(planner.WEIGHTS)
    assert 0 <= cc < planner.NCLASS
    P = torch.from_numpy(params).cuda()
    r_net, r_ship, r_const, g_def, g_plain, fb_count = [], [], [], [], [], 0
    t_auto, t_exh = [], []
    for seed in SEEDS:
        _, A, x = planner.make_matrix(seed)
        rec = planner.label_matrix(A, x, reps=REPS)
        ip, ix, vv = sable.device_csr(A)
        xd = torch.from_numpy(x).cuda()
        y = torch.empty(A.nrows, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p, c, conf, fb = sable.sable_plan_auto(A.nrows, A.ncols, ip, ix, vv, P, mean, std, 0.0, xd, y)
        t_auto.append(time.perf_counter() - t0)
        p.destroy()
        assert not fb and 0 <= c < planner.NCLASS and 0.0 < conf <= 1.0
        if len(t_exh) < 8:  # planning time of the exhaustive search itself (forced fallback)
            t0 = time.perf_counter()
            q, _, _, fq = sable.sable_plan_auto(A.nrows, A.ncols, ip, ix, vv, P, mean, std, 1.01, xd, y)
            t_exh.append(time.perf_counter() - t0)
            q.destroy()
            assert fq
        t = np.array(rec["times"])
        best = int(np.argmin(t))
        shipped = best if conf < tau else c  # below tau the exhaustive search decides
        fb_count += conf < tau
        r_net.append(t[c] / t.min() - 1.0)
        r_ship.append(t[shipped] / t.min() - 1.0)
        r_const.append(t[cc] / t.min() - 1.0)
        g_def.append(rec["t_default"] / t[shipped])
        g_plain.append(rec["t_plain"] / t[shipped])
        print(f"  seed {seed} n={A.nrows}: net {planner.class_name(c)} ({conf:.2f}) regret "
              f"{r_net[-1]:.3f}, shipped {r_ship[-1]:.3f}, {planner.class_name(cc)} {r_const[-1]:.3f}")
    geo = lambda v: float(np.exp(np.mean(np.log(v))))  # noqa: E731
    print(f"  mean regret: shipped {np.mean(r_ship):.4f} (fallback {fb_count}/{len(r_net)}), "
          f"network {np.mean(r_net):.4f}, best single class {np.mean(r_const):.4f}; "
          f"geomean gain over the default list {geo(g_def):.3f}, over plain CSR {geo(g_plain):.3f}")
    ta, te = np.median(t_auto[:len(t_exh)]), np.median(t_exh)
    print(f"  planning time (median of {len(t_exh)}): network {ta * 1e3:.0f} ms, exhaustive search "
          f"{te * 1e3:.0f} ms ({te / ta:.1f}x)")
    assert ta < te
    assert np.mean(r_ship) <= 0.05
    assert np.mean(r_net) <= np.mean(r_const) + 0.01
    assert geo(g_def) >= 1.0
