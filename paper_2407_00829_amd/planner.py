"""Learned planner harness: labels from the exhaustive timed search, GPU training, regret.

The planner replaces the search over extractor lists and delta thresholds with an MLP
140-128-128-15 over structure features (diagonal run-length histogram, 16x16 tile density
histogram, row-length statistics). All numerical work runs in libsable:
  sable_features          features on the GPU
  sable_plan_exhaustive   plans every class, autotunes and times its SpMV, returns the
                          fastest, and times plain CSR and the default list the same way
  sable_mlp_train_step    forward, softmax cross-entropy, backward and Adam on the GPU
  sable_plan_auto         features -> MLP -> plan, exhaustive fallback below tau_conf
This module only generates matrices, stores labels (append-only JSONL, resumable), loops
over training batches and computes the summary statistics.

Usage (GPU; the shipped weights were made this way, with training seeds labelled from 0 up
for as long as the time allowed and the held-out seeds 100000..100199):
  python -m paper_2407_00829_amd.planner label --out labels.jsonl --seeds 100000:100200
  python -m paper_2407_00829_amd.planner label --out labels.jsonl --seeds 0:1000 --max-seconds 1080
  python -m paper_2407_00829_amd.planner train --labels labels.jsonl --train 0:1000 --out w.npz \
      --epochs 500 --tol 0.02 --target 0.03
  python -m paper_2407_00829_amd.planner eval --labels labels.jsonl --test 100000:100200 \
      --train 0:1000 --weights w.npz
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import os
import sys
import time

import numpy as np

from . import synth

CLASS_LISTS = ["CSR", "VDIA+CSR", "VBR+CSR", "VDIA+VBR+CSR", "VBR+VDIA+CSR"]
DELTAS = [500, 700, 900]
NCLASS = 15


def class_name(c: int) -> str:
    return f"{CLASS_LISTS[c // 3]}@{DELTAS[c % 3] / 1000:.1f}"


def matrix_params(seed: int, nmin: float = 1e4, nmax: float = 1e6):
    """Planner matrix: n ~ logU[nmin, nmax], mean row length ~ U[4, 64], proportions ~
    Dirichlet(1,1,1) over band / block / scatter generators."""
    rng = np.random.default_rng(10_000_019 + seed)
    n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    rowlen = float(rng.uniform(4, 64))
    pi = rng.dirichlet([1.0, 1.0, 1.0])
    return n, rowlen, pi


def make_matrix(seed: int):
    n, rowlen, pi = matrix_params(seed)
    A, x = synth.gen_mixed(seed, n=n, rowlen=rowlen, pi=pi)
    return seed, A, x


def _time_ms(fn, torch, reps=10):
    """Median over three rounds of the per-launch average of `reps` back-to-back launches."""
    fn()
    out = []
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b) / reps)
    return float(np.median(out))


def label_matrix(A, x, reps=20) -> dict:
    """Features and the exhaustive search's class times; every time (the 15 classes, the
    plain CSR baseline and the default list) is taken inside the library the same way: the
    plan's kernels autotuned, then the median of three rounds of `reps` launches."""
    import torch

    from . import sable
    ip, ix, vv = sable.device_csr(A)
    f = sable.sable_features(A.nrows, A.ncols, ip, ix, vv)
    xd = torch.from_numpy(x).cuda()
    y = torch.empty(A.nrows, device="cuda")
    p, best, times, ref = sable.sable_plan_exhaustive(A.nrows, A.ncols, ip, ix, vv, xd, y, reps,
                                                      with_refs=True)
    p.destroy()
    return {"features": [float(v) for v in f], "times": [float(t) for t in times],
            "best": int(best), "t_plain": float(ref[0]), "t_default": float(ref[1])}


def build_labels(seeds, path: str, workers: int = 8, reps: int = 20, log=print,
                 max_seconds: float = 0.0) -> int:
    """Label the seeds not yet in `path` (append-only JSONL, resumable); with max_seconds > 0
    stop after the matrix that passes that wall time."""
    done = set()
    if os.path.exists(path):
        with open(path) as fh:
            for line in fh:
                try:
                    done.add(json.loads(line)["seed"])
                except (ValueError, KeyError):
                    continue  # a torn last line from an interrupted run is ignored
    todo = [s for s in seeds if s not in done]
    log(f"[labels] {len(done)} cached, {len(todo)} to do")
    n_new = 0
    t0 = time.time()
    window = 2 * workers  # matrices generated ahead of the GPU (bounded host memory)
    with cf.ProcessPoolExecutor(workers) as ex, open(path, "a") as out:
        pending = [ex.submit(make_matrix, s) for s in todo[:window]]
        nxt = len(pending)
        while pending:
            seed, A, x = pending.pop(0).result()
            if nxt < len(todo):
                pending.append(ex.submit(make_matrix, todo[nxt]))
                nxt += 1
            rec = label_matrix(A, x, reps)
            rec.update(seed=int(seed), n=A.nrows, nnz=A.nnz)
            out.write(json.dumps(rec) + "\n")
            out.flush()
            n_new += 1
            log(f"[labels] {n_new}/{len(todo)} seed {seed} n={A.nrows} nnz={A.nnz} "
                f"best {class_name(rec['best'])} ({time.time() - t0:.0f} s)")
            if max_seconds and time.time() - t0 > max_seconds:
                log("[labels] time budget reached; the rest stays for the next run")
                for f in pending:
                    f.cancel()
                break
    return n_new


def load_labels(path: str, seeds=None):
    recs = []
    with open(path) as fh:
        for line in fh:
            try:
                r = json.loads(line)
            except ValueError:
                continue
            if seeds is None or r["seed"] in seeds:
                recs.append(r)
    recs.sort(key=lambda r: r["seed"])
    return recs


def robust_labels(recs, tol: float = 0.05, rank_recs=None):
    """Training label per matrix: among the classes within `tol` of the fastest measured time,
    the one with the lowest mean regret over `rank_recs` (default: recs). Near-ties are mostly
    timing noise; this maps them to one consistent class instead of a random argmin."""
    T = np.array([r["times"] for r in recs])
    R = T / T.min(axis=1, keepdims=True) - 1.0
    Tr = np.array([r["times"] for r in (rank_recs or recs)])
    Rr = Tr / Tr.min(axis=1, keepdims=True) - 1.0
    rank = np.empty(NCLASS, int)
    rank[np.argsort(Rr.mean(axis=0), kind="stable")] = np.arange(NCLASS)
    return np.where(R <= tol, rank[None, :], NCLASS + 1).argmin(axis=1).astype(np.int32)


def choose_tau(params, mean, std, val_recs, target: float = 0.04) -> float:
    """Smallest confidence threshold (grid 0.0..0.95) whose validation regret <= target."""
    for tau in np.round(np.arange(0.0, 0.96, 0.05), 2):
        if evaluate(params, mean, std, val_recs, float(tau))["regret_mean"] <= target:
            return float(tau)
    return 0.95


def train(X: np.ndarray, y: np.ndarray, epochs: int = 10, batch: int = 64, lr: float = 1e-3,
          seed: int = 0, init=None, log=print):
    """Adam on the GPU (sable_mlp_train_step). Returns params, feature mean, feature std."""
    import torch

    from . import sable
    mean = X.mean(axis=0).astype(np.float32)
    std = X.std(axis=0).astype(np.float32)
    std[std < 1e-6] = 1.0
    Xn = ((X - mean) / std).astype(np.float32)
    if init is None:
        rng = np.random.default_rng(seed)
        parts = []
        for rows, cols in ((128, 140), (128, 128), (15, 128)):
            lim = math.sqrt(6.0 / cols)
            parts.append(rng.uniform(-lim, lim, rows * cols))
            parts.append(np.zeros(rows))
        init = np.concatenate(parts).astype(np.float32)
    P = torch.from_numpy(init.copy()).cuda()
    G = torch.zeros_like(P)
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    Xd = torch.from_numpy(Xn).cuda()
    yd = torch.from_numpy(y.astype(np.int32)).cuda()
    rng = np.random.default_rng(seed + 1)
    t = 0
    hist = []
    for ep in range(epochs):
        perm = rng.permutation(Xn.shape[0])
        tot = 0.0
        for b0 in range(0, perm.size, batch):
            idx = torch.from_numpy(perm[b0:b0 + batch]).cuda()
            t += 1
            loss = sable.sable_mlp_train_step(P, G, M, V, Xd[idx].contiguous(),
                                              yd[idx].contiguous(), lr, 0.9, 0.999, 1e-8, t)
            tot += loss * idx.numel()
        hist.append(tot / perm.size)
        if log and (ep % 50 == 0 or ep == epochs - 1):
            log(f"[train] epoch {ep} loss {hist[-1]:.4f}")
    return P.cpu().numpy(), mean, std, hist


def predict(params, mean, std, X):
    import torch

    from . import sable
    Xn = ((X - mean) / std).astype(np.float32)
    Pd = torch.from_numpy(params).cuda()
    Xd = torch.from_numpy(Xn).cuda()
    L = torch.empty(X.shape[0], NCLASS, device="cuda")
    sable.sable_mlp_forward(Pd, Xd, L)
    torch.cuda.synchronize()
    z = L.cpu().numpy().astype(np.float64)
    z -= z.max(axis=1, keepdims=True)
    pr = np.exp(z)
    pr /= pr.sum(axis=1, keepdims=True)
    return pr.argmax(axis=1), pr.max(axis=1)


def best_constant_class(recs) -> int:
    """The single class with the lowest mean regret over `recs` (the planner's yardstick: one
    fixed choice for every matrix, picked on the training records)."""
    T = np.array([r["times"] for r in recs])
    return int((T / T.min(axis=1, keepdims=True) - 1.0).mean(axis=0).argmin())


def evaluate(params, mean, std, recs, tau_conf: float = 0.0, const_class: int | None = None) -> dict:
    """Regret t(pred)/t(best) - 1 over held-out records; below tau_conf the exhaustive search
    decides (regret 0 for that matrix, counted as a fallback). Gains are geomean speedups of
    the chosen plan over the fixed default plan, over plain CSR and (when const_class is
    given) over always choosing that one class."""
    X = np.array([r["features"] for r in recs], np.float32)
    pred, conf = predict(params, mean, std, X)
    regret, g_def, g_plain, g_const, fb = [], [], [], [], 0
    for r, c, cf_ in zip(recs, pred, conf):
        t = np.array(r["times"])
        if cf_ < tau_conf:
            c = int(np.argmin(t))
            fb += 1
        regret.append(t[c] / t.min() - 1.0)
        g_def.append(r["t_default"] / t[c])
        g_plain.append(r["t_plain"] / t[c])
        if const_class is not None:
            g_const.append(t[const_class] / t[c])
    regret = np.array(regret)
    oracle_best = np.array([np.min(r["times"]) for r in recs])
    geo = lambda v: float(np.exp(np.mean(np.log(v))))  # noqa: E731
    out = {"n": len(recs), "regret_mean": float(regret.mean()),
           "regret_p90": float(np.percentile(regret, 90)),
           "accuracy": float(np.mean([np.argmin(r["times"]) == c for r, c in zip(recs, pred)])),
           "gain_vs_default_geomean": geo(g_def),
           "gain_vs_plain_csr_geomean": geo(g_plain),
           "best_vs_plain_geomean": geo([r["t_plain"] / b for r, b in zip(recs, oracle_best)]),
           "best_vs_default_geomean": geo([r["t_default"] / b for r, b in zip(recs, oracle_best)]),
           "fallback_rate": fb / max(1, len(recs)), "tau_conf": tau_conf}
    if const_class is not None:
        T = np.array([r["times"] for r in recs])
        cr = T[:, const_class] / T.min(axis=1) - 1.0
        out.update(const_class=class_name(const_class), const_regret_mean=float(cr.mean()),
                   const_regret_p90=float(np.percentile(cr, 90)),
                   gain_vs_const_geomean=geo(g_const))
    return out


def save_weights(path, params, mean, std, tau=0.0, const_class=-1):
    np.savez(path, params=params.astype(np.float32), mean=mean.astype(np.float32),
             std=std.astype(np.float32), tau=np.float32(tau), const_class=np.int32(const_class))


def load_weights(path):
    z = np.load(path)
    tau = float(z["tau"]) if "tau" in z else 0.0
    return z["params"], z["mean"], z["std"], tau


def load_const_class(path) -> int:
    """The best single class on the training labels, stored with the weights (-1 if absent)."""
    z = np.load(path)
    return int(z["const_class"]) if "const_class" in z else -1


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "planner_weights.npz")


def _range(s: str):
    a, b = s.split(":")
    return list(range(int(a), int(b)))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("label")
    a.add_argument("--out", required=True)
    a.add_argument("--seeds", required=True)
    a.add_argument("--workers", type=int, default=8)
    a.add_argument("--reps", type=int, default=20)
    a.add_argument("--max-seconds", type=float, default=0.0)
    b = sub.add_parser("train")
    b.add_argument("--labels", required=True)
    b.add_argument("--train", required=True)
    b.add_argument("--out", required=True)
    b.add_argument("--epochs", type=int, default=10)
    b.add_argument("--tol", type=float, default=0.05)
    b.add_argument("--target", type=float, default=0.04)
    c = sub.add_parser("eval")
    c.add_argument("--labels", required=True)
    c.add_argument("--test", required=True)
    c.add_argument("--weights", required=True)
    c.add_argument("--tau", type=float, default=-1.0)
    c.add_argument("--train", default="",
                   help="training seeds: the best constant class is chosen on them")
    args = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    if args.cmd == "label":
        build_labels(_range(args.seeds), args.out, args.workers, args.reps, log, args.max_seconds)
    elif args.cmd == "train":
        recs = load_labels(args.labels, set(_range(args.train)))
        val = [r for i, r in enumerate(recs) if i % 10 == 0]   # 10% validation split
        fit = [r for i, r in enumerate(recs) if i % 10 != 0]
        X = np.array([r["features"] for r in fit], np.float32)
        y = robust_labels(fit, args.tol)
        params, mean, std, hist = train(X, y, epochs=args.epochs, log=log)
        tau = choose_tau(params, mean, std, val, args.target)
        cc = best_constant_class(fit)
        save_weights(args.out, params, mean, std, tau, cc)
        print(json.dumps({"trained_on": len(fit), "validation": len(val), "final_loss": hist[-1],
                          "tau_conf": tau, "const_class": class_name(cc),
                          "val_no_fallback": evaluate(params, mean, std, val, 0.0, cc),
                          "val_with_fallback": evaluate(params, mean, std, val, tau, cc)}))
    else:
        recs = load_labels(args.labels, set(_range(args.test)))
        params, mean, std, tau = load_weights(args.weights)
        if args.tau >= 0:
            tau = args.tau
        cc = best_constant_class(load_labels(args.labels, set(_range(args.train)))
                                 if args.train else recs)
        print(json.dumps({"no_fallback": evaluate(params, mean, std, recs, 0.0, cc),
                          "with_fallback": evaluate(params, mean, std, recs, tau, cc)}))


if __name__ == "__main__":
    main()
