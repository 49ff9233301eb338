"""Writes antidune1d_t50.npz: the oracle's states of the paper's 1D antidune
(subsection "1D antidune evolution": J = 2400 cells on a 24 m channel,
parabolic bump on [8, 12] m, q0 = 1.7 m^2/s, supercritical Bernoulli depth
with h0 = 0.5 m at the inflow, Grass A_g = 1e-3, m_g = 3; inflow (0.5, 1.7)
through the west side, free outflow through the east side; CFL 0.5) at the
times of the paper's figure: 6, 10, 15, 30 and 50 s.  Calls only the
oracle and the seeded workload generator; the GPU parity test compares the
library's run with these values.

Run from the repository root:  python tests/golden/make_antidune1d_t50.py
(a few minutes on one core)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

TIMES = (6.0, 10.0, 15.0, 30.0, 50.0)


def main():
    h, hu, zb, dx = W.antidune1d(2400)
    o = O.Oracle1D(h, hu, zb, dx, O.Params(law=O.LAW_GRASS, A_g=1e-3, m_g=3.0),
                   (O.BC(O.BC_INFLOW, 0.5, 1.7, 0.0), O.BC(O.BC_FREE)))
    out = {}
    for k, t_end in enumerate(TIMES):
        while o.t < t_end:                   # one step per call: nsteps counts real steps
            o.step(1, 0.5, t_end)
        out[f"h{k}"] = o.h.copy()
        out[f"hu{k}"] = o.hu.copy()
        out[f"zb{k}"] = o.z.copy()
        out[f"nsteps{k}"] = o.nsteps
        out[f"dt_last{k}"] = o.dt_last
        print(f"t = {o.t}: {o.nsteps} steps", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "antidune1d_t50.npz")
    np.savez_compressed(path, times=np.array(TIMES), **out)
    print(path)


if __name__ == "__main__":
    main()
