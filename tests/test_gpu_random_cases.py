"""Seeded random configurations against the oracle.  2D (200 cases): grid
shapes from 1 to 200 cells per side (tile edges, ragged tiles, single rows
and columns), boundary kinds per direction (periodic pairs, or free /
inflow on each side), closure family, interface problem, order, storage,
momentum friction, tile height and CFL number drawn per case; smooth random
states (subcritical flow over a random bed).  1D (60 cases): 1 to 3000
cells (around the workgroup width of the LDS-resident kernel and its size
limit), periodic or inflow / free, the three closure families, both
interface problems and orders, storage, friction, the resident, split or
one-pass path.  FP64 at 1e-12, float32 storage at 1e-5 against the
oracle's emulation; the time to 1e-12.  A case the oracle rejects must fail at the same step.  Beyond
the stability bound (60 cases at CFL numbers 1.2 to 3) the tolerance
follows the oracle's own spread under a last-bit change of the input."""
import numpy as np
import pytest

import oracle as O
from gpu_helpers import assert_fields_close, field_errors, to_oracle_bcs, to_oracle_params

pytestmark = pytest.mark.gpu

N_CASES = 200


@pytest.fixture(scope="module")
def sve(gpu_lib):
    return gpu_lib


def smooth(rng, ny, nx, amp):
    """A smooth random field: a few low Fourier modes."""
    y = (np.arange(ny) + 0.5)[:, None] / max(ny, 1)
    x = (np.arange(nx) + 0.5)[None, :] / max(nx, 1)
    f = np.zeros((ny, nx))
    for _ in range(4):
        kx, ky = rng.integers(0, 3, 2)
        ph = rng.uniform(0, 2 * np.pi)
        f += rng.uniform(-1, 1) * np.cos(2 * np.pi * (kx * x + ky * y) + ph)
    return amp * f / 4.0


def draw(sve, seed):
    rng = np.random.default_rng(1000 + seed)
    nx = int(rng.choice([1, 2, 3, 7, 59, 60, 61, 62, 63, 64, 121, 130, 200]))
    ny = int(rng.choice([1, 2, 3, 5, 8, 9, 17, 33, 64, 150]))
    dx = float(rng.uniform(2.0, 10.0))
    dy = float(rng.uniform(2.0, 10.0))
    zb = 0.3 + smooth(rng, ny, nx, 0.3)
    h = 2.0 + smooth(rng, ny, nx, 0.4) - (zb - 0.3)
    u = 0.8 + smooth(rng, ny, nx, 0.5)
    v = smooth(rng, ny, nx, 0.4)
    bcs = []
    for pair in range(2):
        if rng.uniform() < 0.5:
            bcs += [sve.BC(sve.BC_PERIODIC)] * 2
        else:
            for _ in range(2):
                if rng.uniform() < 0.4:
                    bcs.append(sve.BC(sve.BC_INFLOW, 2.0, 1.6 if pair == 0 else 0.2,
                                      0.1 if pair == 0 else 1.2))
                else:
                    bcs.append(sve.BC(sve.BC_FREE))
    closure = rng.choice(["grass3", "grassm", "mpm", "nielsen"])
    common = dict(reconstruction=int(rng.integers(0, 2)), order=int(rng.integers(1, 3)),
                  momentum_friction=int(rng.uniform() < 0.3))
    if closure == "grass3":
        p = sve.Params(law=sve.LAW_GRASS, A_g=float(rng.uniform(0.01, 0.1)), m_g=3.0,
                       friction=sve.FRIC_MANNING, fric_coef=0.03, **common)
    elif closure == "grassm":
        p = sve.Params(law=sve.LAW_GRASS, A_g=float(rng.uniform(0.01, 0.1)),
                       m_g=float(rng.uniform(1.5, 4.0)), friction=sve.FRIC_DARCY,
                       fric_coef=0.05, **common)
    elif closure == "mpm":
        p = sve.Params(law=sve.LAW_MPM, friction=sve.FRIC_STRICKLER, fric_coef=40.0, d_s=1e-3,
                       s=2.65, tau_cr=0.05, **common)
    else:
        p = sve.Params(law=sve.LAW_NIELSEN, friction=sve.FRIC_DARCY, fric_coef=0.05,
                       d_s=1e-3, s=2.65, tau_cr=0.05, **common)
    storage = "fp32" if rng.uniform() < 0.25 else "fp64"
    rows = int(rng.choice([0, 0, 1, 2, 3, 5, 16]))
    cfl = float(rng.uniform(0.2, 0.5))
    steps = int(rng.integers(3, 16))
    return dict(h=h, hu=h * u, hv=h * v, zb=zb, dx=dx, dy=dy, bcs=bcs, p=p, storage=storage,
                rows=rows, cfl=cfl, steps=steps)


@pytest.mark.parametrize("seed", range(N_CASES))
def test_random_configuration(sve, seed):
    c = draw(sve, seed)
    ny, nx = c["h"].shape
    s = sve.Solver(c["h"], c["hu"], c["zb"], c["hv"], lx=c["dx"] * nx, ly=c["dy"] * ny,
                   params=c["p"], bcs=c["bcs"], storage=c["storage"])
    s.set_tile_rows(c["rows"])
    o = O.Oracle2D(c["h"], c["hu"], c["hv"], c["zb"], c["dx"], c["dy"], to_oracle_params(c["p"]),
                   to_oracle_bcs(c["bcs"]), storage=c["storage"])
    try:
        with np.errstate(all="ignore"):
            o.step(c["steps"], c["cfl"])
        oracle_error = None
    except O.OracleError as e:
        oracle_error = e
    if oracle_error is not None:
        # the library fails at the same step and keeps the state before it
        with pytest.raises(sve.SveError):
            s.step(c["steps"], c["cfl"])
        f, t, dtl, ns = s.get_state()
        s.close()
        assert ns == oracle_error.step
        return
    s.step(c["steps"], c["cfl"])
    f, t, dtl, ns = s.get_state()
    s.close()
    assert ns == c["steps"]
    assert t == pytest.approx(o.t, rel=1e-12)
    assert_fields_close(f, o.state, 1e-12 if c["storage"] == "fp64" else 1e-5)


def draw1d(sve, seed):
    rng = np.random.default_rng(5000 + seed)
    nx = int(rng.choice([1, 2, 3, 59, 60, 61, 64, 65, 1000, 1023, 1024, 1025, 2000, 2922, 3000]))
    dx = float(rng.uniform(0.5, 10.0))
    zb = 0.3 + smooth(rng, 1, nx, 0.3)[0]
    h = 2.0 + smooth(rng, 1, nx, 0.4)[0] - (zb - 0.3)
    u = 0.8 + smooth(rng, 1, nx, 0.5)[0]
    if rng.uniform() < 0.5:
        bcs = [sve.BC(sve.BC_PERIODIC)] * 2
    else:
        bcs = [sve.BC(sve.BC_INFLOW, 2.0, 1.6, 0.0) if rng.uniform() < 0.5 else sve.BC(sve.BC_FREE),
               sve.BC(sve.BC_FREE)]
    closure = rng.choice(["grass3", "grassm", "mpm"])
    common = dict(reconstruction=int(rng.integers(0, 2)), order=int(rng.integers(1, 3)),
                  momentum_friction=int(rng.uniform() < 0.3))
    if closure == "grass3":
        p = sve.Params(law=sve.LAW_GRASS, A_g=float(rng.uniform(0.01, 0.1)), m_g=3.0,
                       friction=sve.FRIC_MANNING, fric_coef=0.03, **common)
    elif closure == "grassm":
        p = sve.Params(law=sve.LAW_GRASS, A_g=float(rng.uniform(0.01, 0.1)),
                       m_g=float(rng.uniform(1.5, 4.0)), friction=sve.FRIC_DARCY,
                       fric_coef=0.05, **common)
    else:
        p = sve.Params(law=sve.LAW_MPM, friction=sve.FRIC_STRICKLER, fric_coef=40.0, d_s=1e-3,
                       s=2.65, tau_cr=0.05, **common)
    storage = "fp32" if rng.uniform() < 0.25 else "fp64"
    # first order: the split or the one-pass path on 40 % of the draws
    # (else the default: resident up to its size limit, one-pass beyond)
    pick = rng.uniform() if p.order == 1 else 1.0
    path = "SPLIT" if pick < 0.2 else "FUSED" if pick < 0.4 else None
    return dict(h=h, hu=h * u, zb=zb, dx=dx, bcs=bcs, p=p, storage=storage, path=path,
                cfl=float(rng.uniform(0.2, 0.5)), steps=int(rng.integers(3, 40)))


@pytest.mark.parametrize("seed", range(60))
def test_random_configuration_1d(sve, seed):
    c = draw1d(sve, seed)
    nx = c["h"].shape[0]
    s = sve.Solver(c["h"], c["hu"], c["zb"], lx=c["dx"] * nx, params=c["p"], bcs=c["bcs"],
                   storage=c["storage"])
    if c["path"]:
        s.set_path(getattr(sve, "PATH_" + c["path"]))
    o = O.Oracle1D(c["h"], c["hu"], c["zb"], c["dx"], to_oracle_params(c["p"]),
                   to_oracle_bcs(c["bcs"]), storage=c["storage"])
    try:
        with np.errstate(all="ignore"):
            o.step(c["steps"], c["cfl"])
        oracle_error = None
    except O.OracleError as e:
        oracle_error = e
    if oracle_error is not None:
        with pytest.raises(sve.SveError):
            s.step(c["steps"], c["cfl"])
        f, t, dtl, ns = s.get_state()
        s.close()
        assert ns == oracle_error.step
        return
    s.step(c["steps"], c["cfl"])
    f, t, dtl, ns = s.get_state()
    s.close()
    assert ns == c["steps"]
    assert t == pytest.approx(o.t, rel=1e-12)
    assert_fields_close(f, o.state, 1e-12 if c["storage"] == "fp64" else 1e-5,
                        names=("h", "hu", "z"))


# Beyond the stability bound (CFL numbers from 1.2 to 3) the scheme
# amplifies every rounding difference from step to step, so no fixed
# tolerance holds: each case runs the oracle twice, on the input and on the
# input with every depth and discharge moved by one part in 2^52, and the
# spread of the two results (field by field, as the comparison measures it)
# scales the tolerance.  The library stays within LARGE_CFL_FACTOR times
# that spread (a wrong term gives differences of order one, not of the
# spread).  Where both oracle runs meet a non-positive depth or a
# non-finite value at the same step, the library stops at that step too
# and keeps the state before it.
LARGE_CFL_FACTOR = 10.0


def _oracle_until_failure(make, steps, cfl):
    """(failing step or None, state before it or the final state, time)."""
    o = make()
    for k in range(steps):
        before, t_before = o.state, o.t
        try:
            with np.errstate(all="ignore"):
                o.step(1, cfl)
        except O.OracleError:
            return k, before, t_before
    return None, o.state, o.t


def _nudge(a, rng):
    return a * (1.0 + 2.0**-52 * rng.choice([-1.0, 1.0], a.shape))


def _check_large_cfl(sve, s, make, h, hu, steps, cfl, tol, names, seed):
    fa, state_a, t_a = _oracle_until_failure(lambda: make(h, hu), steps, cfl)
    rng = np.random.default_rng(seed)
    fb, state_b, t_b = _oracle_until_failure(lambda: make(_nudge(h, rng), _nudge(hu, rng)),
                                             steps, cfl)
    try:
        s.step(steps, cfl)
        raised = False
    except sve.SveError:
        raised = True
    f, t, dtl, ns = s.get_state()
    s.close()
    assert raised == (ns != steps)
    if fa != fb:
        # the failing step itself is decided by rounding: the library fails
        # at one of the two steps, or runs through if one of them does
        assert ns in {steps if x is None else x for x in (fa, fb)}
        return
    assert ns == (steps if fa is None else fa)
    spread = field_errors(state_b, state_a, names)
    scale = max(v for k, v in spread.items() if k != "hv_share")
    ftol = max(tol, LARGE_CFL_FACTOR * scale)
    assert t == pytest.approx(t_a, rel=max(1e-12, LARGE_CFL_FACTOR * abs(t_b - t_a) / t_a))
    assert_fields_close(f, state_a, ftol, names=names, own_tol=ftol)


@pytest.mark.parametrize("seed", range(40))
def test_random_configuration_large_cfl(sve, seed):
    c = draw(sve, 10000 + seed)
    cfl = float(np.random.default_rng(seed).uniform(1.2, 3.0))
    ny, nx = c["h"].shape
    s = sve.Solver(c["h"], c["hu"], c["zb"], c["hv"], lx=c["dx"] * nx, ly=c["dy"] * ny,
                   params=c["p"], bcs=c["bcs"], storage=c["storage"])
    P, B = to_oracle_params(c["p"]), to_oracle_bcs(c["bcs"])

    def make(h, hu):
        return O.Oracle2D(h, hu, c["hv"], c["zb"], c["dx"], c["dy"], P, B, storage=c["storage"])

    _check_large_cfl(sve, s, make, c["h"], c["hu"], 30, cfl,
                     1e-12 if c["storage"] == "fp64" else 1e-5, ("h", "hu", "hv", "z"), seed)


@pytest.mark.parametrize("seed", range(20))
def test_random_configuration_large_cfl_1d(sve, seed):
    c = draw1d(sve, 10000 + seed)
    cfl = float(np.random.default_rng(seed).uniform(1.2, 3.0))
    nx = c["h"].shape[0]
    s = sve.Solver(c["h"], c["hu"], c["zb"], lx=c["dx"] * nx, params=c["p"], bcs=c["bcs"],
                   storage=c["storage"])
    if c["path"]:
        s.set_path(getattr(sve, "PATH_" + c["path"]))
    P, B = to_oracle_params(c["p"]), to_oracle_bcs(c["bcs"])

    def make(h, hu):
        return O.Oracle1D(h, hu, c["zb"], c["dx"], P, B, storage=c["storage"])

    _check_large_cfl(sve, s, make, c["h"], c["hu"], 60, cfl,
                     1e-12 if c["storage"] == "fp64" else 1e-5, ("h", "hu", "z"), seed)
