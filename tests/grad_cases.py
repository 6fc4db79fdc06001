"""Cases of the device gradient of the free energy, shared by the CPU check of
their conditioning and by the GPU parity tests.

Each case fixes the workload, the mean sequence (seed and scale of
workloads.random_V) and the call index.  The gradient is discontinuous where
an indicator flips (a collision, the CVaR bound test, tail membership), and
the device computes in FP32, so each case is chosen well away from every such
jump for the samples that carry weight: obstacle margins >= 1e-3 m, relative
gap between the n_tail-th and the next risk cost >= 1e-4, relative distance of
CVaR from C_u >= 1e-4, and normalised track radius >= 0.25 (the conditioning
of the Sampson distance)."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2209_12842_amd import workloads as W

CASES = [
    dict(name="c1", kw=dict(lam=50.0), vseed=4, step=1),
    dict(name="c1", kw=dict(K=512, T=24, M=32, lam=20.0, eta=0.3), vseed=4, step=2),
    dict(name="c1", kw=dict(K=300, T=17, M=12, lam=30.0, B=2.5, C_u=20.0), vseed=4, step=1),
    dict(name="c1", kw=dict(K=256, T=20, M=16, lam=40.0, noise_kind=1), vseed=4, step=1),
    dict(name="c1", kw=dict(K=256, T=20, M=16, lam=40.0, noise_kind=2, jump_prob=0.1, jump_size=0.45), vseed=4,
         step=1),
    dict(name="p0", kw=dict(K=512, M=32, lam=5.0), vseed=4, step=4, vscale=(0.5, 0.2)),
    dict(name="c2", kw=dict(K=512, T=50, M=16, lam=100.0, c_bdry=1.0), vseed=4, step=1),
    # tails sorted across waves: M = 128 (one exchange stage through LDS), M = 256 with risk scaling (three)
    dict(name="c1", kw=dict(K=256, T=20, M=128, lam=10.0), vseed=4, step=2),
    dict(name="c1", kw=dict(K=256, T=16, M=256, lam=5.0, B=0.5), vseed=4, step=1),
    # horizons shorter than the recomputed rollouts' four-step load ring
    dict(name="c1", kw=dict(K=64, T=3, M=16, lam=30.0), vseed=4, step=1),
    dict(name="c1", kw=dict(K=64, T=2, M=16, lam=30.0), vseed=4, step=1),
    dict(name="c4", kw=dict(lam=50.0), vseed=4, step=1),
]

IDS = ["%s-%s" % (c["name"], "-".join("%s=%s" % kv for kv in sorted(c["kw"].items()))) for c in CASES]

MARGIN = 1e-3
TAIL_GAP = 1e-4
CU_GAP = 1e-4
COND_MIN = 0.25
W_MIN = 1e-7


def inputs(case):
    w = W.make_world(case["name"], **case["kw"])
    V = W.random_V(int(w["params"]["T"]), case["vseed"], scale=case.get("vscale", (1.0, 0.2)))
    return w, V


def conditioning(p, obs, x0, V, step) -> dict:
    """Distances of the weighted samples from every jump of the gradient."""
    o = oracle.step(p, obs, x0, V, step)
    M = int(p["M"])
    B = float(np.float32(p["B"]))
    nt = oracle.tail_size(float(np.float32(p["alpha"])), M)[1]
    wk = o["w_hat"] > W_MIN
    L = o["L"][wk]
    mu = L.mean(axis=1, keepdims=True)
    srt = -np.sort(-(B * (L - mu) + mu), axis=1)
    if nt < M:
        gap = (srt[:, nt - 1] - srt[:, nt]) / np.maximum(np.abs(srt[:, nt - 1]), 1.0)
    else:
        gap = np.ones(1)
    Cu = float(np.float32(p["C_u"]))
    cv = o["cvar"][wk]
    return dict(n_weighted=int(wk.sum()), nom_margin=float(o["nom_margin"][wk].min()),
                obs_margin=float(o["obs_margin"][wk].min()), nom_cond=float(o["nom_cond"][wk].min()),
                obs_cond=float(o["obs_cond"][wk].min()), tail_gap=float(gap.min()),
                cu_gap=float((np.abs(cv - Cu) / np.maximum(np.abs(cv), 1.0)).min()), oracle=o)


def well_conditioned(c: dict) -> bool:
    return (c["nom_margin"] >= MARGIN and c["obs_margin"] >= MARGIN and c["tail_gap"] >= TAIL_GAP
            and c["cu_gap"] >= CU_GAP and c["nom_cond"] >= COND_MIN and c["obs_cond"] >= COND_MIN)
