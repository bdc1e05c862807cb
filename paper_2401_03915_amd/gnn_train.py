"""Training driver of the learned warm start (the network itself and its
forward, loss and backward passes run in the library's device kernels:
``tls_gnn_loss_grad``; this script only feeds instances and takes Adam
steps on the 7-8 thousand weights).

Recipe: layered-elasticity instances (48^3 nodes, 512 boxes of 6^3 nodes,
overlap 1; slab thickness uniform in {2..8}, random phase; seeds 100..),
each set up in FP64 with nev = 20 so that its eq. gevpsvd eigenvectors are
exact to 1e-9 and serve as targets; Adam (lr 2e-3, betas 0.9 / 0.999) on the
mean loss over all subdomains of all instances.

    python -m paper_2401_03915_amd.gnn_train --out weights.txt [--instances 4]
        [--steps 2000] [--c-out 32] [--nev 20]

Writes the weights as text (one float per line after '#' header lines) and
prints one JSON line per 20 steps.
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

# weights trained by this script with its defaults (see the file's header lines)
TRAINED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "gnn_layered_elasticity_c32.txt")


def init_weights(c_out: int, seed: int) -> np.ndarray:
    """Uniform in +-sqrt(3 / fan_in) per block (variance 1 / fan_in)."""
    from . import _lib
    rng = np.random.default_rng(seed)
    parts = []
    cin = _lib.GNN_FEATURES
    for _ in range(_lib.GNN_LAYERS):
        for _ in range(2):  # Theta, Phi
            a = np.sqrt(3.0 / (2 * cin))
            parts.append(rng.uniform(-a, a, cin * _lib.GNN_HIDDEN))
        parts.append(np.zeros(_lib.GNN_HIDDEN))
        cin = _lib.GNN_HIDDEN
    a = np.sqrt(3.0 / _lib.GNN_HIDDEN)
    parts.append(rng.uniform(-a, a, _lib.GNN_HIDDEN * c_out))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == _lib.gnn_n_weights(c_out)
    return w


def save_weights(path: str, w: np.ndarray, c_out: int, header: dict) -> None:
    with open(path, "w") as f:
        f.write(f"# c_out {c_out}\n")
        for k, v in header.items():
            f.write(f"# {k}: {v}\n")
        for x in w:
            f.write(f"{float(x):.9g}\n")


def load_weights(path: str) -> tuple[np.ndarray, int]:
    c_out = None
    vals = []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                if line.startswith("# c_out"):
                    c_out = int(line.split()[2])
                continue
            if line.strip():
                vals.append(float(line))
    w = np.asarray(vals, dtype=np.float32)
    from . import _lib
    if c_out is None or _lib.gnn_n_weights(c_out) != w.size:
        raise ValueError(f"{path}: not a weight file of this network")
    return w, c_out


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--instances", type=int, default=4)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--c-out", type=int, default=32)
    ap.add_argument("--nev", type=int, default=20)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--nodes", type=int, default=48)
    ap.add_argument("--seed", type=int, default=100)
    args = ap.parse_args()
    import paper_2401_03915_amd as tls
    from workloads import elasticity_training_instances

    ctxs = []
    t0 = time.time()
    for seed, thick, phase, A, part, nparts in elasticity_training_instances(args.instances, args.seed, args.nodes):
        pc = tls.Preconditioner(A, part, 1, args.nev, precision=0, gnn_train=1)
        ctxs.append(pc)
        print(json.dumps({"instance": seed, "thick": thick, "phase": phase, "n": A.shape[0], "parts": nparts,
                          "setup_s": round(time.time() - t0, 2)}), flush=True)
    w = init_weights(args.c_out, args.seed)
    m = np.zeros_like(w, dtype=np.float64)
    v = np.zeros_like(w, dtype=np.float64)
    b1, b2, eps = 0.9, 0.999, 1e-8
    w64 = w.astype(np.float64)
    history = []
    for step in range(1, args.steps + 1):
        g = np.zeros(w.size)
        L = 0.0
        for pc in ctxs:
            loss, grad = pc.gnn_loss_grad(w64.astype(np.float32), args.c_out)
            L += loss / len(ctxs)
            g += grad.astype(np.float64) / len(ctxs)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        mh = m / (1 - b1 ** step)
        vh = v / (1 - b2 ** step)
        w64 -= args.lr * mh / (np.sqrt(vh) + eps)
        history.append(L)
        if step % 20 == 0 or step == 1:
            print(json.dumps({"step": step, "loss": round(L, 6), "t_s": round(time.time() - t0, 1)}), flush=True)
    save_weights(args.out, w64.astype(np.float32), args.c_out,
                 {"recipe": f"layered elasticity {args.nodes}^3 nodes, instances {args.instances} from seed "
                            f"{args.seed}, nev {args.nev}, FP64 targets, Adam lr {args.lr}, {args.steps} steps",
                  "final_loss": f"{history[-1]:.6f}", "initial_loss": f"{history[0]:.6f}"})
    for pc in ctxs:
        pc.close()


if __name__ == "__main__":
    main()
