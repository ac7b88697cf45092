"""Train the learned Newton seed on the GPU and write its weights.

The training and held-out pairs are files written by the oracle's pair
script (oracle-labelled closest points, the configuration of the learned
seed: shapes of the polydisperse suspension, uniform orientations and
centre directions, gaps log-uniform in [1e-4, 1] of the smallest
semi-axis):

    python -m oracle.seed_pairs --seed 1 --m 2097152 --out TRAIN.npz
    python -m oracle.seed_pairs --seed 2 --m 262144 --out HELDOUT.npz
    python -m paper_1308_6482_amd.train_seed --train TRAIN.npz --heldout HELDOUT.npz \\
        --out paper_1308_6482_amd/data/seed_weights.npz

This script reads the files only (the oracle is not imported); the network
is trained by the library's BF16 MFMA kernels (lub_mlp_train, Adam) and the
weights, the loss per epoch, the held-out loss and the wall time are written
to the output file (and a JSON record beside it).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "seed_weights.npz")


def load_pairs(path):
    from paper_1308_6482_amd import seed_data as S
    z = np.load(path)
    P = {k: z[k] for k in z.files}
    ok = P["status"] == 0
    P = {k: v[ok] for k, v in P.items()}
    F = S.labelled_features(P)
    return F["X"], F["T"], int((~ok).sum())


def train(train_path, heldout_path, epochs=8, batch=4096, lr=2e-3, lr_decay=0.75, seed=1):
    import torch
    from paper_1308_6482_amd import lub as L
    X, T, dropped = load_pairs(train_path)
    Xh, Th, _ = load_pairs(heldout_path)
    lb = L.Lub((100.0, 100.0, 100.0), (1, 1, 1),
               dict(mu=1 / 6, delta_n=0.67, delta_t=0.5, delta_r=0.25), 10.0)
    L.lub_mlp_init(lb.h, seed)
    Xd, Td = torch.as_tensor(X).cuda(), torch.as_tensor(T).cuda()
    m = (X.shape[0] // batch) * batch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = L.lub_mlp_train(lb.h, Xd[:m].contiguous(), Td[:m].contiguous(), epochs=epochs,
                             batch=batch, lr=lr, lr_decay=lr_decay)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mh = (Xh.shape[0] // 64) * 64
    held, _ = L.lub_mlp_grad(lb.h, torch.as_tensor(Xh[:mh]).cuda(),
                             torch.as_tensor(Th[:mh]).cuda())
    theta = L.lub_mlp_get_weights(lb.h)
    lb.close()
    rec = dict(train_pairs=int(m), train_pairs_dropped=dropped, heldout_pairs=int(mh),
               epochs=epochs, batch=batch, lr=lr, lr_decay=lr_decay, init_seed=seed,
               epoch_loss=[float(v) for v in losses], heldout_loss=float(held),
               train_s=t1 - t0, labels="oracle closest points (ref_place_pairs)",
               device=torch.cuda.get_device_name(0))
    return theta, rec


def load_weights(path=WEIGHTS):
    """The committed weights and their training record, or (None, None)."""
    if not os.path.exists(path):
        return None, None
    z = np.load(path)
    rec = json.loads(str(z["record"])) if "record" in z.files else {}
    return z["theta"].astype(np.float32), rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", required=True)
    ap.add_argument("--heldout", required=True)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--epochs", type=int, default=8)
    a = ap.parse_args()
    theta, rec = train(a.train, a.heldout, epochs=a.epochs)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    np.savez(a.out, theta=theta, record=json.dumps(rec))
    with open(os.path.splitext(a.out)[0] + ".json", "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
