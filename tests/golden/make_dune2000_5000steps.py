"""Writes dune2000_5000steps.npz: samples of the oracle's state of the
periodic 2D Grass dune (2000 x 2000 cells on [0, 1000]^2 m, bump
sin^2 sin^2 on [300, 500] x [400, 600], h = 10 - z_b, hu = 10, hv = 0,
A_g = 1e-3, m_g = 3, CFL 0.5) after 500 and after 5000 steps, the
benchmarked run's length.  Stored per snapshot: the time, the last dt,
three 32 x 32 windows (the bump's upstream slope, its crest, a cell far
from it) and every 50th cell in each direction, of each field, with each
field's sum and largest magnitude and the largest momentum magnitude.

The steps are the oracle's own (oracle.scheme.fluxes_2d, dt_from_speeds,
update_2d, in the order Oracle2D.step applies them), evaluated on eight
row strips at a time in threads: each strip carries one halo row on each
side (so its interior interfaces are those of the whole grid), the time
step comes from the maximum over all strips, and every operation is
elementwise or an exact maximum, so the result is bitwise that of
Oracle2D.step on the whole grid (--check compares the two on a small grid).
Calls only the oracle and the seeded workload generator.

Run from the repository root:
  python tests/golden/make_dune2000_5000steps.py          (about an hour on 8 cores)
  python tests/golden/make_dune2000_5000steps.py --check"""
import argparse
import os
import sys
import time
import types
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402
from oracle.scheme import dt_from_speeds, fluxes_2d, update_2d  # noqa: E402

SNAPSHOTS = (500, 5000)
# (row, column) of the lower-left cell of each 32 x 32 window
WINDOWS = ((984, 680), (984, 784), (200, 1500))
STRIDE = 50
PARAMS = O.Params(law=O.LAW_GRASS, A_g=1e-3, m_g=3.0)
# periodic in x; the strips' own halo rows stand in for the y neighbours
STRIP_BCS = (O.BC(), O.BC(), O.BC(O.BC_FREE), O.BC(O.BC_FREE))


class StripStepper:
    """Oracle2D.step on a periodic grid, evaluated strip by strip."""

    def __init__(self, state, dx, dy, params, nstrips, workers):
        self.h, self.hu, self.hv, self.z = (np.array(a) for a in state)
        self.dx, self.dy, self.p = dx, dy, params
        ny = self.h.shape[0]
        self.bounds = [(k * ny // nstrips, (k + 1) * ny // nstrips) for k in range(nstrips)]
        self.pool = ThreadPoolExecutor(workers)
        self.t = 0.0
        self.nsteps = 0
        self.dt_last = 0.0

    def _fluxes(self, b):
        j0, j1 = b
        rows = np.arange(j0 - 1, j1 + 1) % self.h.shape[0]      # one halo row each side
        X, Y = fluxes_2d(self.h[rows], self.hu[rows], self.hv[rows], self.z[rows], self.p,
                         STRIP_BCS)
        m = j1 - j0
        # interior rows 1..m of the strip: x-interfaces of those rows, and the
        # y-interfaces below and above each of them
        Xi = types.SimpleNamespace(**{k: getattr(X, k)[1:m + 1] for k in
                                      ("Fh", "FhuL", "FhuR", "Fht", "Fz", "speed", "err")})
        Yi = types.SimpleNamespace(**{k: getattr(Y, k)[1:m + 2] for k in
                                      ("Fh", "FhuL", "FhuR", "Fht", "Fz", "speed", "err")})
        return Xi, Yi

    def step(self, cfl):
        res = list(self.pool.map(self._fluxes, self.bounds))
        for X, Y in res:
            if np.any(X.err) or np.any(Y.err):
                raise RuntimeError(f"oracle interface error at step {self.nsteps}")
        Sx = max(float(np.max(X.speed)) for X, _ in res)
        Sy = max(float(np.max(Y.speed)) for _, Y in res)
        dt = float(dt_from_speeds(Sx, Sy, self.dx, self.dy, cfl))

        def upd(args):
            (j0, j1), (X, Y) = args
            sl = slice(j0, j1)
            return update_2d(self.h[sl], self.hu[sl], self.hv[sl], self.z[sl], X, Y, dt,
                             self.dx, self.dy)

        new = list(self.pool.map(upd, zip(self.bounds, res)))
        self.h, self.hu, self.hv, self.z = (np.concatenate([n[f] for n in new]) for f in range(4))
        for a in (self.h, self.hu, self.hv, self.z):
            if not np.all(np.isfinite(a)):
                raise RuntimeError("non-finite state")
        self.t = self.t + dt
        self.nsteps += 1
        self.dt_last = dt

    @property
    def state(self):
        return self.h, self.hu, self.hv, self.z


def check():
    """The strip evaluation equals Oracle2D.step bitwise on a small grid."""
    h, hu, hv, zb, dx, dy = W.dune2d(120, 96)
    hv = 0.3 * zb
    ref = O.Oracle2D(h, hu, hv, zb, dx, dy, PARAMS, (O.BC(),) * 4)
    s = StripStepper((h, hu, hv, zb), dx, dy, PARAMS, 8, 8)
    for _ in range(20):
        ref.step(1, 0.5)
        s.step(0.5)
    assert s.t == ref.t and s.dt_last == ref.dt_last
    for a, b in zip(s.state, ref.state):
        assert np.array_equal(a, b)
    print("strip evaluation equals Oracle2D.step bitwise (120 x 96, 20 steps)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--check", action="store_true")
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    if args.check:
        check()
        return
    check()
    h, hu, hv, zb, dx, dy = W.dune2d(2000, 2000)
    s = StripStepper((h, hu, hv, zb), dx, dy, PARAMS, 16, args.workers)
    out = {"windows": np.array(WINDOWS), "stride": STRIDE}
    t0 = time.time()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "dune2000_5000steps.npz")
    for k, n in enumerate(SNAPSHOTS):
        while s.nsteps < n:
            s.step(0.5)
            if s.nsteps % 100 == 0:
                print(f"{s.nsteps} steps, t = {s.t}, {time.time() - t0:.0f} s", flush=True)
        h_, hu_, hv_, z_ = s.state
        for f, a in zip(("h", "hu", "hv", "zb"), s.state):
            for w, (j, i) in enumerate(WINDOWS):
                out[f"{f}_w{w}_s{k}"] = a[j:j + 32, i:i + 32].copy()
            out[f"{f}_strided_s{k}"] = a[::STRIDE, ::STRIDE].copy()
            out[f"{f}_sum_s{k}"] = float(np.sum(a))
            out[f"{f}_absmax_s{k}"] = float(np.max(np.abs(a)))
        out[f"mom_max_s{k}"] = float(np.max(np.hypot(hu_, hv_)))
        out[f"t_s{k}"] = s.t
        out[f"dt_last_s{k}"] = s.dt_last
        out[f"nsteps_s{k}"] = s.nsteps
        print(f"snapshot {k}: {s.nsteps} steps, t = {s.t}", flush=True)
    np.savez_compressed(path, **out)
    print(path)


if __name__ == "__main__":
    main()
