"""Writes dune1d_t10000.npz: the oracle's state of the 1D Grass dune
(1000 cells on [0, 1000] m, periodic, A_g = 1e-3, m_g = 3, CFL 0.5) at
T = 10000 s.  Calls only the oracle and the seeded workload generator; the
GPU parity test compares the library's run with these values.

Run from the repository root:  python tests/golden/make_dune1d_t10000.py
(about 1.5 minutes on one core)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

T_END = 10000.0


def main():
    h, hu, zb, dx = W.dune1d(1000)
    o = O.Oracle1D(h, hu, zb, dx, O.Params(law=O.LAW_GRASS, A_g=1e-3, m_g=3.0),
                   (O.BC(), O.BC()))
    while o.t < T_END:                       # one step per call: nsteps counts real steps
        o.step(1, 0.5, T_END)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dune1d_t10000.npz")
    np.savez(out, h=o.h, hu=o.hu, zb=o.z, t=o.t, nsteps=o.nsteps, dt_last=o.dt_last)
    print(out, o.nsteps, o.t)


if __name__ == "__main__":
    main()
