"""The benchmarked 2D run at its full length: the periodic 2D Grass dune,
2000 x 2000 cells on [0, 1000]^2 m, A_g = 1e-3, m_g = 3, CFL 0.5, in the
launch configuration the benchmark times (default path, automatic tile
split), for 5000 steps.  Windows and a strided sample of every field after
500 and 5000 steps, the time and the last time step, and the sums of h and
z_b are compared with the oracle's run stored in
tests/golden/dune2000_5000steps.npz (written by make_dune2000_5000steps.py
in the same folder, from the oracle alone).  Tolerance 1e-12 relative per
field (momentum components against the largest momentum magnitude).

The second-order variant on the same dune at 400 x 400 cells, 250 and 1000
CFL steps, every cell against the oracle's run stored in
tests/golden/dune400_order2_1000steps.npz (make_dune400_order2_1000steps.py),
at the same tolerance; the transverse momentum (3 % of the momentum
magnitude) is held to 1e-11 against its own maximum: on the oracle alone, a
1e-15 relative perturbation of the initial depth moves it by 2.0e-12 of its
maximum after 250 steps and 7.5e-13 after 1000."""
import os

import numpy as np
import pytest

import workloads as W
from gpu_helpers import assert_fields_close

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def sve(gpu_lib):
    return gpu_lib


def sample_errors(fields, ref, k):
    """Relative errors of the stored samples of snapshot k: each field
    against its own largest magnitude, the momentum components against the
    largest momentum magnitude (the frame of gpu_helpers.field_errors)."""
    wins = ref["windows"]
    stride = int(ref["stride"])
    out = {}
    for f, a in zip(("h", "hu", "hv", "zb"), fields):
        scale = float(ref[f"mom_max_s{k}"]) if f in ("hu", "hv") else float(ref[f"{f}_absmax_s{k}"])
        err = 0.0
        for w, (j, i) in enumerate(wins):
            err = max(err, float(np.max(np.abs(a[j:j + 32, i:i + 32] - ref[f"{f}_w{w}_s{k}"]))))
        err = max(err, float(np.max(np.abs(a[::stride, ::stride] - ref[f"{f}_strided_s{k}"]))))
        out[f] = err / scale
    return out


def test_dune2000_5000_steps_against_stored_oracle(sve):
    ref = np.load(os.path.join(GOLDEN, "dune2000_5000steps.npz"))
    h, hu, hv, zb, dx, dy = W.dune2d(2000, 2000)
    p = sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0)
    s = sve.Solver(h, hu, zb, hv, lx=1000.0, ly=1000.0, params=p,
                   bcs=[sve.BC(sve.BC_PERIODIC)] * 4)
    done = 0
    for k in range(2):
        n = int(ref[f"nsteps_s{k}"])
        s.step(n - done, 0.5)
        done = n
        fields, t, dtl, ns = s.get_state()
        assert ns == n
        assert t == pytest.approx(float(ref[f"t_s{k}"]), rel=TOL64)
        assert dtl == pytest.approx(float(ref[f"dt_last_s{k}"]), rel=TOL64)
        errs = sample_errors(fields, ref, k)
        assert max(errs.values()) <= TOL64, (n, errs)
        for f, a in zip(("h", "zb"), (fields[0], fields[3])):
            s0 = float(ref[f"{f}_sum_s{k}"])
            assert abs(float(np.sum(a)) - s0) <= 1e-13 * abs(s0)
    s.close()


def test_dune400_order2_1000_steps_against_stored_oracle(sve):
    ref = np.load(os.path.join(GOLDEN, "dune400_order2_1000steps.npz"))
    h, hu, hv, zb, dx, dy = W.dune2d(400, 400)
    p = sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0, order=2)
    s = sve.Solver(h, hu, zb, hv, lx=1000.0, ly=1000.0, params=p,
                   bcs=[sve.BC(sve.BC_PERIODIC)] * 4)
    done = 0
    for k, n in enumerate(ref["steps"]):
        s.step(int(n) - done, 0.5)
        done = int(n)
        fields, t, dtl, ns = s.get_state()
        assert ns == n
        assert t == pytest.approx(float(ref[f"t{k}"]), rel=TOL64)
        assert dtl == pytest.approx(float(ref[f"dt_last{k}"]), rel=TOL64)
        assert_fields_close(fields, tuple(ref[f"{f}{k}"] for f in ("h", "hu", "hv", "zb")), TOL64,
                            own_tol=1e-11)
        assert abs(float(np.sum(fields[3])) - float(np.sum(zb))) <= 1e-13 * float(np.sum(zb))
    s.close()
