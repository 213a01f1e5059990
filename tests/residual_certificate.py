"""Oracle residual certificate of a D_W solve over every site (test
infrastructure).

||b - D_W x||_2 / ||b||_2 per right-hand side, computed by the FP64 oracle
(``oracle.solver.wilson_residual_slab``) on t-slabs in parallel child
processes, so a 32^3 x 64 lattice at N_v = 12 (4.8 GB per FP64 field) is
certified in seconds rather than minutes.  The fields are handed over as .npy
files which each child memory-maps; the children are plain ``python``
processes that import numpy and the oracle only (they never touch the GPU).

Run as a script, this module is one such child:

    python tests/residual_certificate.py U.npy B.npy X.npy M0 T0 T1

and prints one JSON line {"rr": [...], "bb": [...]} with the per-column
squared norms of the residual and of b over the slices T0 <= t < T1.
"""
from __future__ import annotations

import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MAX_WORKERS = 16


def worker_count() -> int:
    """Host cores this process may use, at most 16 (the CPU share of one GPU)."""
    return max(1, min(MAX_WORKERS, len(os.sched_getaffinity(0))))


def slabs(nt: int, parts: int):
    """[t0, t1) ranges covering 0 .. nt - 1 in ``parts`` nearly equal pieces."""
    parts = max(1, min(parts, nt))
    edges = [nt * k // parts for k in range(parts + 1)]
    return [(a, b) for a, b in zip(edges[:-1], edges[1:]) if b > a]


def certify(u_path: str, b_path: str, x_path: str, m0: float, workers: int | None = None) -> np.ndarray:
    """Per-column ||b - D_W x|| / ||b|| over the whole lattice of the saved fields."""
    nt = np.load(u_path, mmap_mode="r").shape[0]
    procs = []
    for t0, t1 in slabs(nt, workers or worker_count()):
        cmd = [sys.executable, os.path.abspath(__file__), u_path, b_path, x_path, repr(float(m0)), str(t0), str(t1)]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                                      env=dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1")))
    rr = bb = 0.0
    errors = []
    for p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            errors.append(f"rc {p.returncode}: {err[-2000:]}")
            continue
        res = json.loads(out.strip().splitlines()[-1])
        rr = rr + np.asarray(res["rr"])
        bb = bb + np.asarray(res["bb"])
    if errors:
        raise RuntimeError("residual worker failed: " + " | ".join(errors))
    return np.sqrt(rr / bb)


def _main(argv):
    sys.path.insert(0, ROOT)
    from oracle import solver
    u_path, b_path, x_path, m0, t0, t1 = argv
    V = np.load(u_path, mmap_mode="r")
    b = np.load(b_path, mmap_mode="r")
    x = np.load(x_path, mmap_mode="r")
    rr, bb = solver.wilson_residual_slab(V, b, x, float(m0), int(t0), int(t1))
    print(json.dumps({"rr": rr.tolist(), "bb": bb.tolist()}), flush=True)


if __name__ == "__main__":
    _main(sys.argv[1:])
