"""Trains the ghost-probability network of the final selection (Sec. 4.4) on
synthetic truth and writes its weights to paper_2606_14480_amd/ghost_nn.json.

The paper prints the network's inputs and layer sizes but not its weights, so
they are learned here once and then used as a fixed parameter by both the
library and the oracle.  Inputs come from the oracle: the VELO-seed pairs
that pass the preselection and the chi2_match cut, with their eight inputs.
Labels come from the generator's truth: a pair is true when 70 % or more of
its seed's hits belong to one particle and the VELO state is that particle's;
every other pair is a ghost.  Training events are drawn from an event range
(first event 1,000,000) that no test or benchmark uses.

Run from the repository root:  python oracle/train_ghost_nn.py
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2606_14480_amd import events as ev  # noqa: E402

OUT = os.path.join(ROOT, "paper_2606_14480_amd", "ghost_nn.json")
FIRST_EVENT = 1_000_000
N_EVENTS = 3000
MAJORITY = 0.7


def pairs_and_labels(batch, res):
    """Every surviving pair of every event: inputs [n, 8] and ghost labels."""
    feats, ghost = [], []
    t = batch.truth
    for e in range(batch.n_events):
        seeds = res.event_seeds(e)
        v0, v1 = int(batch.velo_off[e]), int(batch.velo_off[e + 1])
        velo = {"x": batch.velo_x[v0:v1], "y": batch.velo_y[v0:v1], "z": batch.velo_z[v0:v1],
                "tx": batch.velo_tx[v0:v1], "ty": batch.velo_ty[v0:v1]}
        pairs = orc.match_pairs(seeds, velo)
        if len(pairs) == 0:
            continue
        t0, t1 = int(t["track_off"][e]), int(t["track_off"][e + 1])
        th = t["hits"][t0:t1]
        owner = {int(h): k for k, row in enumerate(th) for h in row if h >= 0}
        # the particle each seed belongs to (-1: none reaches the majority)
        seed_trk = np.full(len(seeds), -1, np.int64)
        for i, sd in enumerate(seeds):
            ids = [int(h) for h in sd["id"] if h >= 0]
            own = [owner.get(h, -1) for h in ids]
            ks, cs = np.unique([o for o in own if o >= 0], return_counts=True) if ids else ([], [])
            if len(ks) and cs.max() >= MAJORITY * len(ids):
                seed_trk[i] = ks[int(np.argmax(cs))]
        velo_of = t["velo"][t0:t1]
        for p in pairs:
            k = seed_trk[p["seed_idx"]]
            true = k >= 0 and int(velo_of[k]) == int(p["velo_idx"])
            feats.append(p["f"])
            ghost.append(0.0 if true else 1.0)
    return np.asarray(feats, np.float64), np.asarray(ghost, np.float64)


def train(X, y, seed=0, epochs=3000):
    import torch
    torch.manual_seed(seed)
    torch.set_num_threads(8)
    mean = X.mean(0)
    scale = X.std(0)
    scale[scale == 0] = 1.0
    Xt = torch.tensor((X - mean) / scale, dtype=torch.float64)
    yt = torch.tensor(y, dtype=torch.float64)
    net = torch.nn.Sequential(torch.nn.Linear(8, 32), torch.nn.ReLU(), torch.nn.Linear(32, 1))
    net = net.double()
    opt = torch.optim.Adam(net.parameters(), lr=1e-2)
    lossf = torch.nn.BCEWithLogitsLoss()
    for it in range(epochs):
        opt.zero_grad()
        loss = lossf(net(Xt).squeeze(1), yt)
        loss.backward()
        opt.step()
        if it == epochs // 2:
            for g in opt.param_groups:
                g["lr"] = 2e-3
    w = {"mean": mean.tolist(), "scale": scale.tolist(),
         "w1": net[0].weight.detach().numpy().tolist(), "b1": net[0].bias.detach().numpy().tolist(),
         "w2": net[2].weight.detach().numpy()[0].tolist(), "b2": float(net[2].bias.detach()[0])}
    return w, float(loss.detach())


def main():
    cfg = ev.config(2, n_events=N_EVENTS, first_event=FIRST_EVENT)
    batch = ev.generate_parallel(cfg, 8)
    res = orc.run(batch, threads=8, margins=False)
    X, y = pairs_and_labels(batch, res)
    n = len(y)
    rng = np.random.default_rng(1)
    perm = rng.permutation(n)
    tr, te = perm[: int(0.8 * n)], perm[int(0.8 * n):]
    w, loss = train(X[tr], y[tr])
    p = orc.default_params(final_sel=1, ghost_nn=w)
    gp = np.array([orc.ghost_prob(p, X[i]) for i in te])
    cut = p.ghost_cut
    keep = gp < cut
    info = {"events": f"min-bias generator, events {FIRST_EVENT}..{FIRST_EVENT + N_EVENTS - 1}",
            "pairs": int(n), "ghost_fraction": float(y.mean()), "train_loss": loss,
            "held_out_true_kept": float(keep[y[te] == 0].mean()),
            "held_out_ghost_kept": float(keep[y[te] == 1].mean())}
    out = dict(w, **{"inputs": ["z_match", "dx", "dy", "dtx", "dty", "chi2_match", "eta_velo",
                                "n_hits_scifi"], "hidden": "relu", "output": "logistic",
                     "training": info})
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(info))


if __name__ == "__main__":
    main()
