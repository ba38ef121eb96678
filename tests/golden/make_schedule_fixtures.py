"""Write the stored oracle trajectories that the long-schedule GPU parity tests compare against.

Runs the FP64 oracle (oracle/spg_ref.py, nothing else) over the reweighting schedule of a
workload drawn by the seeded generator (paper_1905_13408_amd/synth.py) and stores, at chosen
iterations of every round, the iterate on a fixed sample of voxels together with full-map
norms; after each reweight (eq 11) the sampled weights u and v; and at the end of each round
the smoothed and unsmoothed objectives (eq 31 with eq 14) and the relative fixed-point
residual.  The GPU tests regenerate the same inputs with the same generator and compare the
HIP path's iterates on the same voxels.

Sample: half uniform over the grid, half uniform over the voxels where the truth map exceeds
a tenth of its maximum (the support of the density), drawn from a seeded stream that depends
only on the workload, so the estimate of the relative L2 error is not dominated by empty
solvent voxels.

  python tests/golden/make_schedule_fixtures.py NAME [NAME ...]

NAME is one of the keys of CASES below; each writes tests/golden/sched_NAME.npz.  Oracle time
on 8 host cores: 128^3 about 2 minutes, 256^3 (300 iterations) about 35 minutes, 512^3 about
50 s per iteration.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import spg_ref as O  # noqa: E402
from paper_1905_13408_amd import synth  # noqa: E402

N_SAMPLE = 8192

# name -> (workload, per-round iteration counts, iterations at which the iterate is sampled)
CASES = {
    # the 64^3 and 128^3 scaled reweighting workloads, full 3 x 100 schedule
    "scaled128_3x100": (synth.scaled_config((128, 128, 128)), [100, 100, 100], [1, 10, 50, 100]),
    # the 256^3 reweighting workload, full 3 x 100 schedule
    "reweight256_3x100": (2, [100, 100, 100], [1, 10, 50, 100]),
    # the 512^3 precision workload: 10 iterations, a reweight, 10 more
    "precision512_10r10": (3, [10, 10], [1, 5, 10]),
    # the 512^3 precision workload, full 3 x 100 schedule
    "precision512_3x100": (3, [100, 100, 100], [1, 10, 50, 100]),
}


def input_digest(vol) -> str:
    """SHA-256 of the generator's float32 / complex64 arrays, so a test can tell that it drew
    the same inputs."""
    h = hashlib.sha256()
    for a in (vol.w, vol.b, vol.x_true):
        h.update(np.ascontiguousarray(a).view(np.uint8))
    return h.hexdigest()


def sample_indices(x_true: np.ndarray, seed_words) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence(list(seed_words) + [515]))
    flat = x_true.ravel()
    n = flat.size
    uni = rng.integers(0, n, size=N_SAMPLE // 2)
    sup = np.flatnonzero(flat > 0.1 * float(flat.max()))
    pick = sup[rng.integers(0, sup.size, size=N_SAMPLE - N_SAMPLE // 2)] if sup.size else uni
    return np.unique(np.concatenate([uni, pick])).astype(np.int64)


def run_case(name: str) -> str:
    cfg, counts, ckpts = CASES[name]
    vol, c = synth.make_config(cfg)
    seed_words = [int(c.get("seed", 0)), int(c.get("config_id", cfg if isinstance(cfg, int) else 100))]
    idx = sample_indices(vol.x_true, seed_words)
    p = O.Problem(w=vol.w.astype(np.float64), b=vol.b.astype(np.complex128), lam=c["lam"], mu=c["mu"], eps=c["eps"])
    store = {"idx": idx}
    rows = []
    t0 = time.perf_counter()

    def cb(r, k, x, pr):
        if k == 1 and r > 0:
            store[f"u_r{r}"] = pr.u.ravel()[idx].copy()
            store[f"v_r{r}"] = pr.v.ravel()[idx].copy()
        if k in ckpts or k == counts[r]:
            store[f"x_r{r}_k{k}"] = x.ravel()[idx].copy()
            rows.append([r, k, float(np.linalg.norm(x)), float(np.sum(np.abs(x)))])
        if k == counts[r]:
            fe = O.objective(x, pr)
            f0 = O.objective(x, pr, smoothed=False)
            kkt = O.kkt_residual(x, pr)
            store[f"end_r{r}"] = np.array([fe, f0, kkt])
        print(f"[{name}] round {r + 1} iteration {k}  {time.perf_counter() - t0:.0f} s", flush=True)

    O.solve_schedule(p, len(counts), counts, c["eps1"], c["eps2"], callback=cb)
    meta = {"case": name, "config": {k: (list(v) if isinstance(v, tuple) else v) for k, v in c.items()},
            "counts": counts, "checkpoints": ckpts, "n_sample": int(idx.size), "inputs_sha256": input_digest(vol),
            "oracle_seconds": time.perf_counter() - t0, "fft_workers": O.fft_workers()}
    store["norms"] = np.array(rows)
    store["meta"] = np.array(json.dumps(meta))
    out = os.path.join(HERE, f"sched_{name}.npz")
    np.savez_compressed(out, **store)
    return out


if __name__ == "__main__":
    for nm in sys.argv[1:]:
        print(run_case(nm), flush=True)
