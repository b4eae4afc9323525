"""Writes rl_512x512x256_samples.txt: the FP64 oracle's Richardson-Lucy estimate of
the 512x512x256 organoid-scale workload after 10 and after 50 iterations, at
seeded sample voxels.

The full-size oracle takes tens of seconds per iteration, too slow for the test
suite, so its values are stored once.  Only the seeded input generator and
oracle/ are used.  Run from the repository root:

    python tests/golden/make_rl_512x512x256_samples.py

(about 40 s per iteration on 8 host cores; 50 iterations in all).
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2510_14143_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rl_512x512x256_samples.txt")
N_SAMPLES = 2048
SAMPLE_SEED = 512
CHECKPOINTS = (10, 50)


def sample_points(shape, n, seed):
    """n distinct voxels, uniformly at random (seeded)."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(int(np.prod(shape)), size=n, replace=False)
    flat.sort()
    return np.stack(np.unravel_index(flat, shape), axis=1)


def main():
    c = synth.make_config(2)
    shape = c["shape"]
    pts = sample_points(shape, N_SAMPLES, SAMPLE_SEED)
    idx = tuple(pts.T)
    u = c["u0"]
    done = 0
    cols = []
    t0 = time.time()
    for n in CHECKPOINTS:
        # RL depends only on the current estimate, so n iterations continue from
        # the estimate after `done`
        u = oracle.rl(c["d"], c["psf"], u, n - done)[0]
        done = n
        cols.append(u[idx].copy())
        print(f"{n} iterations after {time.time() - t0:.0f} s", flush=True)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle (oracle.rl) estimate of the 512x512x256 organoid-scale workload\n")
        f.write("# (paper_2510_14143_amd.synth.make_config(2): Gaussian PSF sigma (2.5, 2.5, 6),\n")
        f.write("# periodic boundary) after 10 and 50 Richardson-Lucy iterations from its initial\n")
        f.write(f"# estimate, at {N_SAMPLES} voxels drawn with numpy default_rng({SAMPLE_SEED}).\n")
        f.write("# Written by tests/golden/make_rl_512x512x256_samples.py.\n")
        f.write("# columns: z y x u_10 u_50\n")
        for p, a, b in zip(pts, cols[0], cols[1]):
            f.write(f"{int(p[0])} {int(p[1])} {int(p[2])} {float(a)!r} {float(b)!r}\n")
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
