"""Writes dune400_order2_1000steps.npz: the oracle's second-order variant
(MUSCL-minmod reconstruction, Heun's method) on the periodic 2D Grass dune
(the benchmark's bump on [0, 1000]^2 m at 400 x 400 cells, A_g = 1e-3,
m_g = 3, CFL 0.5) after 250 and 1000 CFL steps.  Calls only the oracle and
the seeded workload generator; the GPU parity test compares the library's
run with these values.

Run from the repository root:  python tests/golden/make_dune400_order2_1000steps.py
(about ten minutes on one core)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

STEPS = (250, 1000)


def main():
    h, hu, hv, zb, dx, dy = W.dune2d(400, 400)
    o = O.Oracle2D(h, hu, hv, zb, dx, dy,
                   O.Params(law=O.LAW_GRASS, A_g=1e-3, m_g=3.0, order=2), (O.BC(),) * 4)
    out = {}
    done = 0
    for k, n in enumerate(STEPS):
        o.step(n - done, 0.5)
        done = n
        for name, a in zip(("h", "hu", "hv", "zb"), o.state):
            out[f"{name}{k}"] = a.copy()
        out[f"t{k}"] = o.t
        out[f"dt_last{k}"] = o.dt_last
        print(f"{n} steps: t = {o.t}", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dune400_order2_1000steps.npz")
    np.savez_compressed(path, steps=np.array(STEPS), **out)
    print(path)


if __name__ == "__main__":
    main()
