"""Writes rl_paper_shape_samples.txt: the FP64 oracle's Richardson-Lucy estimate of
the volume of the paper's stack shape, 30x2160x2560 (Z, Y, X), after 1 and 2
iterations, at seeded sample voxels, with a convolution of the observed volume at
a few voxels.

Only the seeded input generator and oracle/ are used.  Run from the repository
root:

    python tests/golden/make_rl_paper_shape_samples.py

(several minutes and about 25 GB of memory on 8 host cores).
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2510_14143_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rl_paper_shape_samples.txt")
N_SAMPLES = 2048
SAMPLE_SEED = 2560


def main():
    t0 = time.time()
    c = synth.make_paper_shape()
    shape = c["shape"]
    print(f"inputs after {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(SAMPLE_SEED)
    flat = np.sort(rng.choice(int(np.prod(shape)), size=N_SAMPLES, replace=False))
    pts = np.stack(np.unravel_index(flat, shape), axis=1)
    idx = tuple(pts.T)
    u1, f1, _ = oracle.rl(c["d"], c["psf"], c["u0"], 1)
    print(f"1 iteration after {time.time() - t0:.0f} s", flush=True)
    u2, f2, _ = oracle.rl(c["d"], c["psf"], u1, 1)
    print(f"2 iterations after {time.time() - t0:.0f} s", flush=True)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle (oracle.rl) estimate of the volume of the paper's stack shape\n")
        f.write("# (paper_2510_14143_amd.synth.make_paper_shape(): 30x2160x2560, Gaussian PSF\n")
        f.write("# sigma (2, 2, 2.5) of the volume's shape, periodic boundary) after 1 and 2\n")
        f.write(f"# Richardson-Lucy iterations from its initial estimate, at {N_SAMPLES} voxels\n")
        f.write(f"# drawn with numpy default_rng({SAMPLE_SEED}).\n")
        f.write("# Written by tests/golden/make_rl_paper_shape_samples.py.\n")
        f.write(f"# flux: {float(f1[-1])!r} {float(f2[-1])!r}\n")
        f.write("# columns: z y x u_1 u_2\n")
        for p, a, b in zip(pts, u1[idx], u2[idx]):
            f.write(f"{int(p[0])} {int(p[1])} {int(p[2])} {float(a)!r} {float(b)!r}\n")
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main()
