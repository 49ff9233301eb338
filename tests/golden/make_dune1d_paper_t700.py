"""Writes dune1d_paper_t700.npz: the oracle's states of the paper's 1D dune
(subsection "1D dune evolution": J = 2000 cells on [0, 1000] m, the bed
0.1 + sin^2(pi (x - 300)/200) on [300, 500] m, h = 10 - z_b, hu = 10,
Grass A_g = 1, m_g = 3, periodic; CFL 0.5) at 100, 350 and 700 s, with the
paper's first-order scheme (prefix o1_) and with the second-order variant
(prefix o2_).  Calls only the oracle and the seeded workload generator; the
GPU parity test compares the library's runs with these values.

Run from the repository root:  python tests/golden/make_dune1d_paper_t700.py
(about two minutes on one core)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

TIMES = (100.0, 350.0, 700.0)


def main():
    out = {}
    for order in (1, 2):
        h, hu, zb, dx = W.dune1d(2000)
        o = O.Oracle1D(h, hu, zb, dx, O.Params(law=O.LAW_GRASS, A_g=1.0, m_g=3.0, order=order),
                       (O.BC(O.BC_PERIODIC), O.BC(O.BC_PERIODIC)))
        for k, t_end in enumerate(TIMES):
            while o.t < t_end:               # one step per call: nsteps counts real steps
                o.step(1, 0.5, t_end)
            pre = f"o{order}_"
            out[pre + f"h{k}"] = o.h.copy()
            out[pre + f"hu{k}"] = o.hu.copy()
            out[pre + f"zb{k}"] = o.z.copy()
            out[pre + f"nsteps{k}"] = o.nsteps
            out[pre + f"dt_last{k}"] = o.dt_last
            print(f"order {order}, t = {o.t}: {o.nsteps} steps", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dune1d_paper_t700.npz")
    np.savez_compressed(path, times=np.array(TIMES), **out)
    print(path)


if __name__ == "__main__":
    main()
