"""Schedule selection from timings the method generates itself.

For every contraction C = A (x) B of a training set this collects the 32
scale-free features of the pair (``Context.features``) and the time of every
SpGEMM schedule (``Context.autotune``, the exhaustive tuner).  The selector
MLP is trained on the GPU (``Context.selector_train``) against per-matrix
centred log2 times, so it ranks schedules rather than predicting absolute
times; selection is the arg-min of its output.  Evaluation reports, per
contraction, the regret of the pick against the exhaustive tuner's best
(T_pick / T_best - 1) and the gain over one fixed schedule
(T_fixed / T_pick).  Tuning parameters over a set of candidate
decompositions is how the paper's framework chooses among its own
algorithms (Section 5.1); learning that choice is the automatic
performance-model adjustment it names as future work (Section 7).
"""

from typing import Dict, List, Tuple

import numpy as np

from . import NUM_SCHEDULES


def collect(ctx, semiring: str, A, B, reps: int = 3) -> Tuple[np.ndarray, np.ndarray]:
    """(features[32], median ms of every schedule) for C = A (x) B."""
    feat = ctx.features(semiring, A, B)
    _, times = ctx.autotune(semiring, A, B, reps=reps)
    return feat, times


def targets(times: np.ndarray) -> np.ndarray:
    """Per-contraction centred log2 times (the regression target)."""
    lt = np.log2(np.maximum(np.asarray(times, dtype=np.float64), 1e-6))
    return (lt - lt.mean(axis=1, keepdims=True)).astype(np.float32)


def best_fixed(times: np.ndarray) -> int:
    """The single schedule with the smallest geometric-mean time."""
    return int(np.argmin(np.log(np.maximum(np.asarray(times, dtype=np.float64), 1e-6)).mean(axis=0)))


def train(ctx, X: np.ndarray, times: np.ndarray, epochs: int = 400, batch: int = 128, lr: float = 1e-3,
          seed: int = 0) -> float:
    """Train the context's selector; returns the final training loss."""
    return ctx.selector_train(np.asarray(X, dtype=np.float32), targets(times), epochs=epochs, batch=batch, lr=lr,
                              seed=seed)


def evaluate(ctx, X: np.ndarray, times: np.ndarray, fixed: int) -> Dict[str, object]:
    """Regret and gain of the context's selector on (X, times)."""
    times = np.asarray(times, dtype=np.float64)
    picks = np.array([ctx.select(x) for x in np.asarray(X, dtype=np.float32)], dtype=np.int64)
    rows = np.arange(times.shape[0])
    t_pick = times[rows, picks]
    t_best = times.min(axis=1)
    regret = t_pick / t_best - 1.0
    gain = times[:, fixed] / t_pick
    return {"picks": picks.tolist(), "regret": regret.tolist(), "gain": gain.tolist(),
            "mean_regret": float(regret.mean()), "max_regret": float(regret.max()),
            "fixed_regret": float((times[:, fixed] / t_best - 1.0).mean()),
            "total_gain": float(times[:, fixed].sum() / t_pick.sum()), "hits": int((picks == times.argmin(1)).sum())}


__all__: List[str] = ["collect", "targets", "best_fixed", "train", "evaluate", "NUM_SCHEDULES"]
