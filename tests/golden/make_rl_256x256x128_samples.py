"""Writes rl_256x256x128_samples.txt: the FP64 oracle's Richardson-Lucy estimate of
the 256x256x128 widefield-like workload after 50 and after 100 iterations (the
workload's own iteration count), at seeded sample voxels.

The oracle needs about a second per iteration on this volume, so 100 iterations
are too slow for the test suite; the values are stored once.  Only the seeded
input generator and oracle/ are used.  Run from the repository root:

    python tests/golden/make_rl_256x256x128_samples.py

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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rl_256x256x128_samples.txt")
N_SAMPLES = 4096
SAMPLE_SEED = 256
CHECKPOINTS = (50, 100)


def sample_points(shape, n, seed):
    """n distinct voxels, uniformly at random (seeded)."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(int(np.prod(shape)), size=n, replace=False)
    flat.sort()
    return np.stack(np.unravel_index(flat, shape), axis=1)


def main():
    c = synth.make_config(1)
    shape = c["shape"]
    pts = sample_points(shape, N_SAMPLES, SAMPLE_SEED)
    idx = tuple(pts.T)
    u = c["u0"]
    done = 0
    cols, flux = [], []
    t0 = time.time()
    for n in CHECKPOINTS:
        # RL depends only on the current estimate, so n iterations continue from
        # the estimate after `done`
        u, f, _ = oracle.rl(c["d"], c["psf"], u, n - done)
        done = n
        cols.append(u[idx].copy())
        flux.append(float(f[-1]))
        print(f"{n} iterations after {time.time() - t0:.0f} s", flush=True)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle (oracle.rl) estimate of the 256x256x128 widefield-like workload\n")
        f.write("# (paper_2510_14143_amd.synth.make_config(1): Gaussian PSF sigma (2, 2, 5),\n")
        f.write("# periodic boundary) after 50 and 100 Richardson-Lucy iterations from its\n")
        f.write(f"# initial estimate, at {N_SAMPLES} voxels drawn with numpy "
                f"default_rng({SAMPLE_SEED}).\n")
        f.write("# Written by tests/golden/make_rl_256x256x128_samples.py.\n")
        f.write(f"# flux: {flux[0]!r} {flux[1]!r}\n")
        f.write("# columns: z y x u_50 u_100\n")
        for p, a, b in zip(pts, cols[0], cols[1]):
            f.write(f"{int(p[0])} {int(p[1])} {int(p[2])} {float(a)!r} {float(b)!r}\n")
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
