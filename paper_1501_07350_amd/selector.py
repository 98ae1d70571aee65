"""Learned plan selector: data collection, training, evaluation.

The paper tunes its communication method at run time by executing every
candidate during initialization (Sec. 3.2.3) and remarks that model-driven
selection suits single-node tuning.  Here a small network predicts
ln(time) of every candidate plan of a grid from the plan's features, and
the plan with the smallest prediction is chosen without timing anything.

  collect()   times every candidate plan of each grid with the library's
              exhaustive tuner (offt_tune_table) on the GPU
  train()     fits the network with the library's HIP kernels
              (offt_mlp_gradient / offt_mlp_adam); torch only holds memory
  evaluate()  regret of the chosen plans against the measured best

Dataset (gzip JSON lines), one record per grid:
  {"i", "dims": [Na, Nb, Nc], "batch", "dtype": 0 complex128 | 1 complex64,
   "plans": [plan strings, candidate order, heuristic first], "ms": [times]}
Weights (text): see the format in csrc/selector.cpp.
"""
from __future__ import annotations

import ctypes
import gzip
import json
import math
import os
import time

import numpy as np

from . import _lib

HIDDEN = 64


def feature_dim() -> int:
    return _lib.load().offt_feature_dim()


def candidates(dims, batch: int, dtype_code: int):
    """(plan strings, features [n, D]) of the candidate plans of one grid."""
    lib = _lib.load()
    D = feature_dim()
    n = _lib.check(lib.offt_candidates(dims[0], dims[1], dims[2], dtype_code, batch, None, 0, None, 0),
                   "candidates")
    buf = ctypes.create_string_buffer(n * 128)
    feats = np.zeros((n, D), dtype=np.float32)
    _lib.check(lib.offt_candidates(dims[0], dims[1], dims[2], dtype_code, batch, buf, len(buf),
                                   feats.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n), "candidates")
    plans = buf.raw.split(b"\0")[:n]
    return [p.decode() for p in plans], feats


def plan_features(dims, batch: int, dtype_code: int, plans):
    lib = _lib.load()
    out = np.zeros((len(plans), feature_dim()), dtype=np.float32)
    for i, p in enumerate(plans):
        _lib.check(lib.offt_plan_features(dims[0], dims[1], dims[2], dtype_code, batch, p.encode(),
                                          out[i:].ctypes.data_as(ctypes.POINTER(ctypes.c_float))), "features")
    return out


def scores(weights_path: str, feats: np.ndarray) -> np.ndarray:
    """Predicted ln(ms) of each feature row (library host inference)."""
    feats = np.ascontiguousarray(feats, dtype=np.float32)
    out = np.zeros(feats.shape[0], dtype=np.float32)
    _lib.check(_lib.load().offt_selector_scores(str(weights_path).encode(),
                                                feats.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                feats.shape[0], out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "selector scores")
    return out


def choose(weights_path: str, dims, batch: int, dtype_code: int) -> str:
    lib = _lib.load()
    buf = ctypes.create_string_buffer(512)
    _lib.check(lib.offt_selector_choose(dims[0], dims[1], dims[2], dtype_code, batch, str(weights_path).encode(),
                                        buf, len(buf)), "selector choose")
    return buf.value.decode()


# ----------------------------------------------------------------- dataset ----
def read_dataset(path):
    with gzip.open(path, "rt") as f:
        return [json.loads(line) for line in f if line.strip()]


def collect(grids, path, reps: int = 2, log=print, start: int = 0):
    """Time every candidate of each grid (GPU); appends to `path` (gzip JSON
    lines).  grids: [(Na, Nb, Nc, batch, dtype_code)]."""
    import torch

    es = {0: 16, 1: 8}
    need = max(a * b * c * bt * es[dt] for a, b, c, bt, dt in grids)
    buf = torch.empty(need // 8 + 1, dtype=torch.float64, device="cuda")
    buf.zero_()
    stream = torch.cuda.current_stream()
    h = ctypes.c_void_p(int(stream.cuda_stream))
    lib = _lib.load()
    t0 = time.time()
    with gzip.open(path, "at") as f:
        for i, (a, b, c, bt, dt) in enumerate(grids):
            if i < start:
                continue
            plans, _ = candidates((a, b, c), bt, dt)
            times = np.zeros(len(plans), dtype=np.float32)
            ts = time.perf_counter()
            n = _lib.check(lib.offt_tune_table(a, b, c, dt, bt, reps, ctypes.c_void_p(buf.data_ptr()),
                                               buf.numel() * 8, h,
                                               times.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), len(plans)),
                           "tune table")
            tune_s = time.perf_counter() - ts
            assert n == len(plans)
            f.write(json.dumps({"i": i, "dims": [a, b, c], "batch": bt, "dtype": dt, "plans": plans,
                                "ms": [round(float(v), 6) for v in times], "tune_s": round(tune_s, 6)}) + "\n")
            if log and (i + 1) % 100 == 0:
                f.flush()
                log(f"collected {i + 1}/{len(grids)} grids in {time.time() - t0:.1f} s")
    return path


def dataset_arrays(records):
    """Feature matrix, targets ln(ms), and per-grid row ranges."""
    X, T, ranges = [], [], []
    r = 0
    for rec in records:
        f = plan_features(rec["dims"], rec["batch"], rec["dtype"], rec["plans"])
        X.append(f)
        T.append(np.log(np.asarray(rec["ms"], dtype=np.float64)))
        ranges.append((r, r + f.shape[0]))
        r += f.shape[0]
    return np.concatenate(X).astype(np.float32), np.concatenate(T).astype(np.float64), ranges


# --------------------------------------------------------------- training ----
def write_weights(path, mean, std, tmean, tstd, params, hidden=HIDDEN):
    D = mean.size
    with open(path, "w") as f:
        f.write("offt-selector 1\n")
        f.write(f"dims {D} {hidden}\n")
        f.write("mean " + " ".join(f"{v:.9g}" for v in mean) + "\n")
        f.write("std " + " ".join(f"{v:.9g}" for v in std) + "\n")
        f.write(f"target {tmean:.9g} {tstd:.9g}\n")
        f.write(f"params {params.size} " + " ".join(f"{v:.9g}" for v in params) + "\n")


class Network:
    """Device network of the library (offt_mlp_*); torch holds the buffers."""

    def __init__(self, D, H=HIDDEN, max_batch=256, params=None, seed=1501):
        self.lib = _lib.load()
        self.D, self.H = D, H
        self.P = self.lib.offt_mlp_nparams(D, H)
        p = None
        if params is not None:
            params = np.ascontiguousarray(params, dtype=np.float32)
            p = params.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self.h = self.lib.offt_mlp_create(D, H, max_batch, p, seed)
        if not self.h:
            raise _lib.OfftError(_lib.last_error(), "offt_mlp_create")

    def params(self):
        out = np.zeros(self.P, dtype=np.float32)
        _lib.check(self.lib.offt_mlp_get_params(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def forward(self, X, idx=None, out=None):
        import torch
        B = X.shape[0] if idx is None else idx.numel()
        out = torch.empty(B, dtype=torch.float32, device="cuda") if out is None else out
        _lib.check(self.lib.offt_mlp_forward(self.h, ctypes.c_void_p(X.data_ptr()),
                                             ctypes.c_void_p(idx.data_ptr() if idx is not None else 0), B,
                                             ctypes.c_void_p(out.data_ptr()),
                                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), "forward")
        return out

    def gradient(self, X, T, idx, grad, loss=None):
        import torch
        B = idx.numel() if idx is not None else X.shape[0]
        _lib.check(self.lib.offt_mlp_gradient(self.h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                                              ctypes.c_void_p(idx.data_ptr() if idx is not None else 0), B,
                                              ctypes.c_void_p(grad.data_ptr()),
                                              ctypes.c_void_p(loss.data_ptr() if loss is not None else 0),
                                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), "gradient")

    def adam(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        import torch
        _lib.check(self.lib.offt_mlp_adam(self.h, ctypes.c_void_p(grad.data_ptr()), lr, beta1, beta2, eps,
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), "adam")

    def close(self):
        if getattr(self, "h", None):
            self.lib.offt_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def train(records, weights_path, epochs=60, batch=256, lr=1e-3, seed=1501, log=print):
    """Fit the network on the training records with the library's kernels."""
    import torch

    X, T, _ = dataset_arrays(records)
    mean = X.mean(axis=0).astype(np.float64)
    std = X.std(axis=0).astype(np.float64)
    std[std < 1e-6] = 1.0
    tmean, tstd = float(T.mean()), float(T.std())
    Xs = ((X - mean) / std).astype(np.float32)
    Ts = ((T - tmean) / tstd).astype(np.float32)
    Xd = torch.from_numpy(Xs).cuda()
    Td = torch.from_numpy(Ts).cuda()
    net = Network(X.shape[1], HIDDEN, batch, seed=seed)
    grad = torch.zeros(net.P, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed)
    n = Xs.shape[0]
    history = []
    t0 = time.time()
    for ep in range(epochs):
        perm = rng.permutation(n).astype(np.int32)
        idx_all = torch.from_numpy(perm).cuda()
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            idx = idx_all[b0:b0 + batch]
            net.gradient(Xd, Td, idx, grad, loss)
            net.adam(grad, lr=lr)
            if (b0 // batch) % 16 == 0:
                tot += float(loss.item())
                cnt += 1
        history.append(tot / max(cnt, 1))
        if log and (ep + 1) % 10 == 0:
            log(f"epoch {ep + 1}: training loss (standardised ln time) {history[-1]:.4f}")
    torch.cuda.synchronize()
    params = net.params()
    write_weights(weights_path, mean, std, tmean, tstd, params)
    net.close()
    return {"epochs": epochs, "loss_history": history, "train_seconds": time.time() - t0,
            "rows": int(n)}


# -------------------------------------------------------------- evaluation ----
def evaluate(records, weights_path, reps: int = 2):
    """Per-grid regret t(chosen)/t(best) - 1 of the learned choice and of the
    heuristic plan (candidate 0), and the cost of each way of choosing."""
    reg_learned, reg_heur, speedup, sel_us, exhaustive_ms = [], [], [], [], []
    for rec in records:
        ms = np.asarray(rec["ms"], dtype=np.float64)
        feats = plan_features(rec["dims"], rec["batch"], rec["dtype"], rec["plans"])
        pred = scores(weights_path, feats)
        k = int(np.argmin(pred))
        # cost of choosing with the library's own path (candidates, features,
        # host inference; weights cached after the first call)
        choose(weights_path, rec["dims"], rec["batch"], rec["dtype"])
        t0 = time.perf_counter()
        choose(weights_path, rec["dims"], rec["batch"], rec["dtype"])
        sel_us.append((time.perf_counter() - t0) * 1e6)
        best = ms.min()
        reg_learned.append(ms[k] / best - 1.0)
        reg_heur.append(ms[0] / best - 1.0)
        speedup.append(ms[0] / ms[k])
        # wall time the exhaustive tuner spent on this grid (all candidates, warm-up + timed runs)
        exhaustive_ms.append(1e3 * rec["tune_s"] if "tune_s" in rec else float(ms.sum()) * (1 + reps))
    rl, rh = np.array(reg_learned), np.array(reg_heur)

    def stats(a):
        return {"mean": float(a.mean()), "median": float(np.median(a)), "p90": float(np.percentile(a, 90)),
                "max": float(a.max())}
    return {"grids": len(records), "regret_learned": stats(rl), "regret_heuristic": stats(rh),
            "speedup_learned_over_heuristic_geomean": float(np.exp(np.mean(np.log(speedup)))),
            "learned_picks_best_fraction": float(np.mean(rl <= 1e-12)),
            "selection_us_mean": float(np.mean(sel_us)),
            "exhaustive_tuning_ms_mean": float(np.mean(exhaustive_ms))}


def evaluate_against_tuner(records, weights_path, count: int = 100, steps: int = 5, log=print):
    """Regret of the learned choice against the library's exhaustive tuner
    (offt_plan_ex with OFFT_TUNE_EXHAUSTIVE, which searches every kernel and
    width per axis, both tile orders and access modes, then every pass order)
    rather than against the best of the selector's own candidate list: on the
    first `count` held-out grids, the learned plan, the heuristic plan and
    the exhaustively tuned plan are each timed as whole forward transforms
    in the same session (one warm-up, then the median of `steps` samples, each
    enough back-to-back executions to cover about 1 ms, HIP events).
    Also the tuner's own time per grid.  GPU."""
    import torch

    from . import Plan

    def timed(plan, x, y, inner):
        h = int(torch.cuda.current_stream().cuda_stream)
        plan.exec_ptr(-1, x.data_ptr(), y.data_ptr(), h)
        ts = []
        for _ in range(steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(inner):
                plan.exec_ptr(-1, x.data_ptr(), y.data_ptr(), h)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / inner)
        return float(np.median(ts))

    reg_l, reg_h, tune_s, per_grid = [], [], [], []
    for j, rec in enumerate(records[:count]):
        dims, bt = tuple(rec["dims"]), rec["batch"]
        dt = torch.complex128 if rec["dtype"] == 0 else torch.complex64
        x = torch.randn((bt,) + dims, dtype=dt, device="cuda")
        y = torch.empty_like(x)
        learned = choose(weights_path, dims, bt, rec["dtype"])
        t0 = time.perf_counter()
        ex = Plan(dims, dtype=dt, batch=bt, tune="exhaustive")
        tune_s.append(time.perf_counter() - t0)
        pl = Plan(dims, dtype=dt, batch=bt, tune="forced", forced_plan=learned)
        ph = Plan(dims, dtype=dt, batch=bt)
        # back-to-back executions per timed sample, enough to cover ~1 ms, so
        # that small grids are not timed at the resolution of one launch
        inner = max(1, min(200, int(math.ceil(1.0 / max(timed(ex, x, y, 1), 1e-3)))))
        t_ex, t_l, t_h = timed(ex, x, y, inner), timed(pl, x, y, inner), timed(ph, x, y, inner)
        reg_l.append(t_l / t_ex - 1.0)
        reg_h.append(t_h / t_ex - 1.0)
        per_grid.append({"dims": list(dims), "batch": bt, "dtype": rec["dtype"], "ms_tuner": round(t_ex, 5),
                         "ms_learned": round(t_l, 5), "ms_heuristic": round(t_h, 5)})
        for q in (ex, pl, ph):
            q.close()
        del x, y
        if log and (j + 1) % 20 == 0:
            log(f"tuner comparison {j + 1}/{min(count, len(records))}")
    torch.cuda.empty_cache()

    def stats(a):
        a = np.asarray(a)
        return {"mean": float(a.mean()), "median": float(np.median(a)), "p90": float(np.percentile(a, 90)),
                "max": float(a.max()), "min": float(a.min())}
    return {"grids": len(reg_l), "regret_learned_vs_tuner": stats(reg_l), "regret_heuristic_vs_tuner": stats(reg_h),
            "tuner_seconds_mean": float(np.mean(tune_s)), "per_grid": per_grid,
            "note": "negative regret: the plan was faster than the tuner's choice in this timing"}


# --------------------------------------------------------------------- CLI ----
DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
DATASET = os.path.join(DATA_DIR, "selector_timings_mi355x.jsonl.gz")
WEIGHTS = os.path.join(DATA_DIR, "selector_weights.txt")
REPORT = os.path.join(DATA_DIR, "selector_report.json")
N_TRAIN, N_HELDOUT = 2000, 200


def split(records):
    """Training records (the first N_TRAIN seeded grids) and held-out ones."""
    train_r = [r for r in records if r["i"] < N_TRAIN]
    held = [r for r in records if r["i"] >= N_TRAIN]
    return train_r, held


def main(argv=None):
    import argparse
    import sys

    ap = argparse.ArgumentParser(prog="python -m paper_1501_07350_amd.selector")
    ap.add_argument("steps", nargs="+", choices=["collect", "train", "evaluate", "evaluate_tuner"])
    ap.add_argument("--dataset", default=DATASET)
    ap.add_argument("--weights", default=WEIGHTS)
    ap.add_argument("--report", default=REPORT)
    ap.add_argument("--count", type=int, default=N_TRAIN + N_HELDOUT)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--tuner-grids", type=int, default=100)
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import synth

    os.makedirs(os.path.dirname(args.dataset), exist_ok=True)
    report = {}
    if "collect" in args.steps:
        grids = synth.selector_grids(args.count)
        done = len(read_dataset(args.dataset)) if os.path.exists(args.dataset) else 0
        t0 = time.time()
        collect(grids, args.dataset, start=done, log=lambda m: print(m, flush=True))
        report["collect_seconds"] = time.time() - t0
    records = read_dataset(args.dataset)
    train_r, held = split(records)
    if "train" in args.steps:
        info = train(train_r, args.weights, epochs=args.epochs, log=lambda m: print(m, flush=True))
        report["train"] = {k: v for k, v in info.items() if k != "loss_history"}
        report["train"]["final_loss"] = info["loss_history"][-1]
    if "evaluate" in args.steps:
        report["heldout"] = evaluate(held, args.weights)
        report["train_set"] = evaluate(train_r[:200], args.weights)
        print(json.dumps(report["heldout"]), flush=True)
    if "evaluate_tuner" in args.steps:
        report["heldout_vs_exhaustive_tuner"] = evaluate_against_tuner(held, args.weights, args.tuner_grids,
                                                                        log=lambda m: print(m, flush=True))
        print(json.dumps(report["heldout_vs_exhaustive_tuner"]), flush=True)
    if report:
        # the heuristic's contiguous-axis rule for complex64 was chosen on all
        # 2200 grids of the data set, the held-out ones included
        report["heuristic_rules_fitted_on"] = "all grids of the data set (training and held-out)"
    if report:
        old = {}
        if os.path.exists(args.report):
            with open(args.report) as f:
                old = json.load(f)
        old.update(report)
        with open(args.report, "w") as f:
            json.dump(old, f, indent=1)


if __name__ == "__main__":
    main()
