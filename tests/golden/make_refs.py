"""Write the oracle references of the reduced-size, full-step-count parity cases.

Each case runs a benchmark workload's generator at a smaller mesh for the step count of its
configuration, through the FP64 oracle only (``oracle.scheme.step``, ``oracle.burgers.step``), and stores the initial state
and the final state in ``tests/golden/<name>.npz``. The GPU parity tests load both and compare the
library's result element by element. Run from the repository root:

    python tests/golden/make_refs.py [name ...]

(about 1-5 minutes per case on one core).
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle.burgers as BG  # noqa: E402
import oracle.scheme as S  # noqa: E402
from paper_2101_01231_amd import inputs as I  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# name: (workload generator at reduced size, steps of the configuration)
CASES = {
    "rotation64_m4_20steps": (lambda: I.rotation_2d(n=64, M=4), 20),
    "adv3d12_m3_20steps": (lambda: I.advection_3d(n=12, M=3), 20),
    "adv2d32_m3_100steps": (lambda: I.advection_2d(n=32, M=3), 100),
    # a mesh the brick kernels tile (16 x 4 x 4 bricks)
    "adv3d16x8x8_m3_20steps": (lambda: I.advection_3d(M=3, shape=(16, 8, 8)), 20),
    # Burgers (Newton prediction): the benchmark's initial state and cfl on a 12^2 mesh, to t = 1/6
    "burgers2d12_m3_20steps": (lambda: I.burgers(d=2, n=12, M=3), 20),
}


def make(name):
    gen, steps = CASES[name]
    wl = gen()
    t0 = time.time()
    if wl.velocity[0] == "burgers":
        ref = BG.step(BG.BurgersProblem(d=wl.d, n=wl.n, M=wl.M), wl.q0, wl.dt, steps)
    else:
        ref = S.step(S.Problem(d=wl.d, n=wl.n, M=wl.M, velocity=wl.velocity), wl.q0, wl.dt, steps)
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, q0=wl.q0, ref=ref, dt=np.float64(wl.dt), steps=np.int64(steps), d=np.int64(wl.d),
                        n=np.array(wl.n, dtype=np.int64), M=np.int64(wl.M),
                        velocity_kind=np.array(wl.velocity[0]), velocity=np.array(wl.velocity[1], dtype=np.float64))
    print(f"{name}: {steps} steps in {time.time() - t0:.0f} s -> {path}", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(CASES)):
        make(name)
