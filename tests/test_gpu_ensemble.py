"""Batched ensemble on the GPU: every member matches the oracle run alone
(1e-12) and the single-grid path run member by member; queue and grid
schedules and every tile height agree; the autotuner leaves the states
unchanged."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_helpers import assert_fields_close

pytestmark = pytest.mark.gpu

PER = (O.BC(),) * 4


@pytest.fixture(scope="module")
def sve(gpu_lib):
    return gpu_lib


def members():
    spec = [(64, 64, 3e-3, 3.0, 0.8), (96, 70, 1e-2, 1.7, 0.6), (130, 95, 5e-4, 1.0, 1.0),
            (61, 122, 2e-3, 2.5, 0.7), (200, 64, 4e-3, 4.0, 0.9), (33, 40, 8e-3, 3.3, 0.5)]
    out = []
    for nx, ny, ag, mg, amp in spec:
        h, hu, hv, zb, dx, dy = W.dune2d(nx, ny, amplitude=amp)
        hv = hv + 0.2 * zb
        out.append(dict(h=h, hu=hu, hv=hv, zb=zb, lx=1000.0, ly=1000.0, A_g=ag, m_g=mg))
    return out


def oracle_run(m, nsteps):
    ny, nx = m["h"].shape
    o = O.Oracle2D(m["h"], m["hu"], m["hv"], m["zb"], m["lx"] / nx, m["ly"] / ny,
                   O.Params(law=O.LAW_GRASS, A_g=m["A_g"], m_g=m["m_g"]), PER)
    o.step(nsteps, 0.5)
    return o


@pytest.mark.parametrize("mode,rows", [(0, 16), (1, 16), (0, 8), (1, 32), (0, 128), (1, 96)])
def test_ensemble_members_match_oracle(sve, mode, rows):
    from paper_1307_0491_amd.ensemble import Ensemble
    ms = members()
    e = Ensemble(ms)
    e.set_schedule(rows, mode)
    e.step(12, 0.5)
    e.step(8, 0.5)                        # a second graph and a new step base
    for i, m in enumerate(ms):
        fields, t, ns = e.get(i)
        o = oracle_run(m, 20)
        assert ns == 20
        assert t == pytest.approx(o.t, rel=1e-12)
        assert_fields_close(fields, o.state, 1e-12)
    e.close()


def test_ensemble_equals_sequential_single_grid_path(sve):
    from paper_1307_0491_amd.ensemble import Ensemble
    ms = members()
    a = Ensemble(ms)
    b = Ensemble(ms)
    a.step(15, 0.5)
    b.step_sequential(15, 0.5)
    for i in range(len(ms)):
        fa, ta, _ = a.get(i)
        fb, tb, _ = b.get(i)
        assert ta == pytest.approx(tb, rel=1e-14)
        assert_fields_close(fa, fb, 1e-14)
    a.close()
    b.close()


def test_autotune_keeps_state(sve):
    from paper_1307_0491_amd.ensemble import Ensemble
    ms = members()
    e = Ensemble(ms)
    e.step(5, 0.5)
    before = [e.get(i) for i in range(len(ms))]
    rows, mode = e.autotune(3, 0.5)
    assert rows in (8, 16, 32, 48, 64, 96, 128) and mode in (0, 1)
    after = [e.get(i) for i in range(len(ms))]
    for (fa, ta, na), (fb, tb, nb) in zip(before, after):
        assert ta == tb and na == nb
        for x, y in zip(fa, fb):
            assert np.array_equal(x, y)
    e.step(5, 0.5)
    for i, m in enumerate(ms):
        fields, t, ns = e.get(i)
        o = oracle_run(m, 10)
        assert_fields_close(fields, o.state, 1e-12)
    e.close()


def test_member_failure_is_isolated(sve):
    from paper_1307_0491_amd.ensemble import Ensemble
    ms = members()[:3]
    ms[1] = dict(ms[1])
    e = Ensemble(ms)
    e.step(3, 0.5)
    good1, t1, _ = e.get(1)
    with pytest.raises(sve.SveError):
        e.step(200, 60.0)                 # far beyond the CFL limit: members fail
    for i in range(3):
        f, t, n = e.get(i)
        for a in f:
            assert np.all(np.isfinite(a))
        assert np.all(f[0] > 0)
    e.close()


def test_invalid_members_are_rejected(sve):
    """Members outside what the ensemble supports are refused at creation
    with SVE_ERR_ARG: exponent outside [1, 4], a non-positive depth, an
    empty grid, a non-Grass law."""
    from paper_1307_0491_amd.ensemble import Ensemble
    base = members()[:2]
    bad = []
    m = dict(base[0]); m["m_g"] = 0.5; bad.append((m, None))
    m = dict(base[0]); m["m_g"] = 4.5; bad.append((m, None))
    m = dict(base[0]); m["h"] = m["h"].copy(); m["h"][3, 5] = 0.0; bad.append((m, None))
    m = dict(base[0]); m["h"] = m["h"][:, :0]; m["hu"] = m["hu"][:, :0]
    m["hv"] = m["hv"][:, :0]; m["zb"] = m["zb"][:, :0]; bad.append((m, None))
    bad.append((dict(base[0]), sve.Params(law=sve.LAW_MPM, friction=sve.FRIC_STRICKLER,
                                          fric_coef=40.0, d_s=1e-3, s=2.65, tau_cr=0.05)))
    for m, p in bad:
        with pytest.raises(sve.SveError) as e:
            Ensemble([base[1], m], params=p)
        assert e.value.code == -1


def test_single_member_ensemble(sve):
    """An ensemble of one member equals the oracle run alone."""
    from paper_1307_0491_amd.ensemble import Ensemble
    m = members()[3]
    e = Ensemble([m])
    e.step(25, 0.5)
    f, t, n = e.get(0)
    e.close()
    o = oracle_run(m, 25)
    assert n == 25
    assert t == pytest.approx(o.t, rel=1e-12)
    assert_fields_close(f, o.state, 1e-12)



def test_schedule_round_trip_replays_a_fresh_graph(sve):
    """Changing the tile height rebuilds the tile list; a graph captured
    with the old list must not be replayed afterwards.  Steps at 16 rows,
    then 32, then 16 again with the same step count (the graph key of the
    first capture) still match the oracle on every member."""
    from paper_1307_0491_amd.ensemble import Ensemble
    ms = members()
    for mode in (0, 1):
        e = Ensemble(ms)
        e.set_schedule(16, mode)
        e.step(4, 0.5)
        e.set_schedule(32, mode)
        e.set_schedule(16, mode)
        e.step(4, 0.5)
        e.set_schedule(32, mode)
        e.step(4, 0.5)
        for i, m in enumerate(ms):
            fields, t, ns = e.get(i)
            o = oracle_run(m, 12)
            assert ns == 12
            assert t == pytest.approx(o.t, rel=1e-12)
            assert_fields_close(fields, o.state, 1e-12)
        e.close()


def test_autotune_failure_rewinds_error_state(sve):
    """A member that fails inside an autotune probe (CFL far beyond the
    limit) makes autotune return its code, and leaves the ensemble as it
    was before the probe: every member reports its pre-probe state and step
    count, and later valid steps still match the oracle."""
    from paper_1307_0491_amd.ensemble import Ensemble
    ms = members()[:3]
    e = Ensemble(ms)
    e.step(3, 0.5)
    before = [e.get(i) for i in range(3)]
    with pytest.raises(sve.SveError):
        e.autotune(40, 60.0)
    for (fa, ta, na), i in zip(before, range(3)):
        fb, tb, nb = e.get(i)
        assert nb == na == 3 and tb == ta
        for x, y in zip(fa, fb):
            assert np.array_equal(x, y)
    e.step(4, 0.5)
    for i, m in enumerate(ms):
        fields, t, ns = e.get(i)
        o = oracle_run(m, 7)
        assert ns == 7
        assert_fields_close(fields, o.state, 1e-12)
    e.close()
