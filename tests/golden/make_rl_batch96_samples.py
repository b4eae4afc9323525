"""Writes rl_batch96_samples.txt: the FP64 oracle's Richardson-Lucy estimate of the
batched 96-volume workload after 50 iterations (the workload's own count) for the
first and the last volume of every shape class, at seeded sample voxels, with the
flux of each of those volumes after every iteration's sum (last value stored).

Only the seeded input generator and oracle/ are used.  Run from the repository
root:

    python tests/golden/make_rl_batch96_samples.py

(a few minutes on 8 host cores).
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2510_14143_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rl_batch96_samples.txt")
COUNT = 96
N_ITER = 50
N_SAMPLES = 512  # per volume
SAMPLE_SEED = 96


def chosen_volumes(shapes):
    """Indices of the first and the last volume of every shape class."""
    first, last = {}, {}
    for v, s in enumerate(shapes):
        first.setdefault(s, v)
        last[s] = v
    return sorted(set(first.values()) | set(last.values()))


def main():
    vols = synth.make_batch(COUNT)
    shapes = [v["shape"] for v in vols]
    pick = chosen_volumes(shapes)
    rng = np.random.default_rng(SAMPLE_SEED)
    t0 = time.time()
    rows = []
    fluxes = {}
    for v in pick:
        c = vols[v]
        n = int(np.prod(c["shape"]))
        flat = np.sort(rng.choice(n, size=min(N_SAMPLES, n), replace=False))
        pts = np.stack(np.unravel_index(flat, c["shape"]), axis=1)
        u, f, _ = oracle.rl(c["d"], c["psf"], c["u0"], N_ITER)
        fluxes[v] = float(f[-1])
        for p in pts:
            rows.append((v, int(p[0]), int(p[1]), int(p[2]), float(u[tuple(p)])))
        print(f"volume {v} {c['shape']} after {time.time() - t0:.0f} s", flush=True)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle (oracle.rl) estimates of the batched workload\n")
        f.write(f"# (paper_2510_14143_amd.synth.make_batch({COUNT}): uneven volumes, each with its\n")
        f.write("# own Gaussian PSF, periodic boundary) after "
                f"{N_ITER} Richardson-Lucy iterations from\n")
        f.write("# their initial estimates: the first and last volume of every shape class, at\n")
        f.write(f"# {N_SAMPLES} voxels per volume drawn with numpy default_rng({SAMPLE_SEED}).\n")
        f.write("# Written by tests/golden/make_rl_batch96_samples.py.\n")
        for v in pick:
            f.write(f"# flux {v} {fluxes[v]!r}\n")
        f.write(f"# columns: volume z y x u_{N_ITER}\n")
        for r in rows:
            f.write(f"{r[0]} {r[1]} {r[2]} {r[3]} {r[4]!r}\n")
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
