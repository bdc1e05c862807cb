"""Writes tests/golden/oracle_fullsize.json: what the FP64 oracle itself
computes on the full-size benchmark configurations (its own coarse space,
its own Krylov run from x0 = 0 to the 1e-8 relative residual): n_C, the
iteration count, the true relative residual, and the wall times of its
setup and solve with the number of worker processes and the CPU model.

Only oracle/ and workloads/ are called. Usage (takes minutes per config):
    python tests/golden/make_oracle_fullsize.py [cfg ...]
Configs already in the file are kept unless named again.
"""

import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import pool  # noqa: E402
from workloads import make_config  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_fullsize.json")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def run(cfg: int) -> dict:
    p = make_config(cfg)
    comp = "ras_deflated" if cfg == 6 else "additive"
    t0 = time.time()
    with pool.Pool(p.A, p.part, p.overlap, p.nev, spd=p.spd) as pl:
        t1 = time.time()
        _, it, rr = pl.solve(p.b, 1e-8, composition=comp)
        t2 = time.time()
        return {"n": int(p.A.shape[0]), "n_parts": int(p.n_parts), "overlap": p.overlap, "nev": p.nev,
                "composition": comp, "krylov": "pcg" if p.spd and comp == "additive" else "fgmres(30)",
                "n_coarse": int(pl.n_coarse), "iterations": int(it), "relres": float(rr),
                "setup_s": round(t1 - t0, 2), "solve_s": round(t2 - t1, 2), "workers": pl.workers,
                "cpu": cpu_model()}


def main(cfgs):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {
        "about": "The FP64 oracle's own results on the full-size configurations (oracle.pool over "
                 "worker processes; b, seeds and partitions from workloads.make_config). Written by "
                 "tests/golden/make_oracle_fullsize.py; nothing here comes from the GPU library.",
        "configs": {}}
    for cfg in cfgs:
        print(f"cfg{cfg} ...", flush=True)
        data["configs"][str(cfg)] = run(cfg)
        print(json.dumps(data["configs"][str(cfg)]), flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [2, 3, 4, 5, 6])
