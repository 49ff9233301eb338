"""Parity at the full sizes of the benchmarked workloads, in the launch
configuration the benchmark times (default path, automatic tile split).

  * 1D Grass dune, 1000 cells on [0, 1000] m, periodic, CFL 0.5, to
    T = 10000 s (about 218 000 steps): against the oracle's final state stored
    in tests/golden/dune1d_t10000.npz (written by make_dune1d_t10000.py in
    the same folder, from the oracle alone);
  * 2D Grass dune, 2000 x 2000 cells, periodic, CFL 0.5: three steps against
    the oracle on the full grid;
  * 2D Meyer-Peter & Mueller channel, 8192 x 2048 cells on 4000 x 1000 m,
    Strickler K_s = 40, inflow (h 0.5, hu 2) / free boundaries: two steps on
    the full grid, FP64 storage (1e-12) and FP32 storage against the oracle's
    FP32-storage emulation (1e-5);
  * the 256-member ensemble (sides 256 .. 1024, batched, autotuned): three
    members of different sizes against the oracle run alone;
  * a 12288 x 12288 dune (151 M cells, 4.8 GB per state buffer, input and
    output through device memory): two CFL steps; a window against the
    oracle run on that window with the same two time steps, and the sums of
    h and z_b conserved to rounding;
  * the paper's 2D bump at its own size (4000 x 4000 cells, inflow through
    the west side, free flow elsewhere, Grass A_g = 1, m_g = 3): 24 CFL
    steps; three windows (on the bump, at the inflow side, at the free
    north-east corner) against the oracle run on each window, with a halo
    wider than the steps' reach and the library's time steps;
  * the paper's 1D antidune at its own size (2400 cells, inflow / free
    outflow) to T = 50 s: the states at 6, 10, 15, 30 and 50 s against the
    oracle's stored in tests/golden/antidune1d_t50.npz, and the crest
    moving upstream;
  * the paper's 1D dune at its own size and coupling (2000 cells, Grass
    A_g = 1, periodic) to T = 700 s, with the paper's first-order scheme and
    with the second-order variant: the states at 100, 350 and 700 s against
    the oracle's stored in tests/golden/dune1d_paper_t700.npz;
  * the 1024 x 1024 adjoint (2000 fixed-dt steps, sqrt(N) checkpoints):
    directional derivatives of the bed-misfit loss with respect to the
    initial bed and the A_g field against central differences of the
    library's own forward run (agreement 1e-6 relative).
"""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_helpers import assert_fields_close

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def sve(gpu_lib):
    return gpu_lib


def test_dune1d_to_t10000_against_stored_oracle(sve):
    ref = np.load(os.path.join(GOLDEN, "dune1d_t10000.npz"))
    h, hu, zb, dx = W.dune1d(1000)
    s = sve.Solver(h, hu, zb, lx=1000.0, params=sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0),
                   bcs=[sve.BC(sve.BC_PERIODIC)] * 2)
    # exactly the oracle's number of real steps: the last one must be the
    # step clipped to land on T
    t = s.step(int(ref["nsteps"]), 0.5, 10000.0)
    (gh, ghu, gz), t2, dtl, ns = s.get_state()
    s.close()
    assert t == 10000.0 and float(ref["t"]) == 10000.0
    assert ns == int(ref["nsteps"])
    assert dtl == pytest.approx(float(ref["dt_last"]), rel=1e-9)
    assert_fields_close((gh, ghu, gz), (ref["h"], ref["hu"], ref["zb"]), TOL64,
                        names=("h", "hu", "z"))


def test_dune2000_full_grid(sve):
    h, hu, hv, zb, dx, dy = W.dune2d(2000, 2000)
    p = sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0)
    s = sve.Solver(h, hu, zb, hv, lx=1000.0, ly=1000.0, params=p,
                   bcs=[sve.BC(sve.BC_PERIODIC)] * 4)
    s.step(3, 0.5)
    fields, t, dtl, ns = s.get_state()
    s.close()
    o = O.Oracle2D(h, hu, hv, zb, dx, dy, O.Params(law=O.LAW_GRASS, A_g=1e-3, m_g=3.0),
                   (O.BC(),) * 4)
    o.step(3, 0.5)
    assert ns == 3
    assert t == pytest.approx(o.t, rel=TOL64)
    assert dtl == pytest.approx(o.dt_last, rel=TOL64)
    assert_fields_close(fields, o.state, TOL64)


@pytest.mark.parametrize("storage,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_mpm_channel_8192x2048_full_grid(sve, storage, tol):
    h, hu, hv, zb, dx, dy = W.mpm_channel()
    ny, nx = h.shape
    assert (ny, nx) == (2048, 8192)
    p = sve.Params(law=sve.LAW_MPM, friction=sve.FRIC_STRICKLER, fric_coef=40.0, d_s=1e-3,
                   s=2.65, tau_cr=0.05)
    bcs = [sve.BC(sve.BC_INFLOW, 0.5, 2.0, 0.0), sve.BC(sve.BC_FREE), sve.BC(sve.BC_FREE),
           sve.BC(sve.BC_FREE)]
    s = sve.Solver(h, hu, zb, hv, lx=4000.0, ly=1000.0, params=p, bcs=bcs, storage=storage)
    s.step(2, 0.5)
    fields, t, dtl, ns = s.get_state()
    s.close()
    po = O.Params(law=O.LAW_MPM, friction=O.FRIC_STRICKLER, fric_coef=40.0, d_s=1e-3, s=2.65,
                  tau_cr=0.05)
    obcs = (O.BC(O.BC_INFLOW, 0.5, 2.0, 0.0), O.BC(O.BC_FREE), O.BC(O.BC_FREE),
            O.BC(O.BC_FREE))
    o = O.Oracle2D(h, hu, hv, zb, dx, dy, po, obcs, storage=storage)
    o.step(2, 0.5)
    assert t == pytest.approx(o.t, rel=TOL64)       # dt from the state as stored
    assert_fields_close(fields, o.state, tol)
    if storage == "fp32":
        for a in fields:
            assert np.array_equal(a, a.astype(np.float32).astype(np.float64))


def test_ensemble_256_members_sampled(sve):
    from paper_1307_0491_amd.ensemble import Ensemble
    draw = W.ensemble_draw(256)
    members = []
    for m in draw:
        h, hu, hv, zb, dx, dy = W.ensemble_member_state(m)
        members.append(dict(h=h, hu=hu, hv=hv, zb=zb, lx=1000.0, ly=1000.0, A_g=m.Ag, m_g=m.mg))
    e = Ensemble(members)
    e.autotune(2, 0.5)
    e.step(2, 0.5)
    sizes = np.array([m.n for m in draw])
    picks = [int(np.argmin(sizes)), int(np.argmax(sizes)),
             int(np.flatnonzero(sizes == 512)[0])]
    for i in picks:
        m = members[i]
        fields, t, ns = e.get(i)
        n = draw[i].n
        o = O.Oracle2D(m["h"], m["hu"], m["hv"], m["zb"], 1000.0 / n, 1000.0 / n,
                       O.Params(law=O.LAW_GRASS, A_g=m["A_g"], m_g=m["m_g"]), (O.BC(),) * 4)
        o.step(2, 0.5)
        assert ns == 2
        assert t == pytest.approx(o.t, rel=TOL64)
        assert_fields_close(fields, o.state, TOL64)
    e.close()


def test_large_grid_window_and_conservation(sve):
    import torch
    n = 12288
    h, hu, hv, zb, dx, dy = W.dune2d(n, n)
    p = sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0)
    dev = [torch.tensor(a, device="cuda") for a in (h, hu, zb, hv)]
    s = sve.Solver(dev[0], dev[1], dev[2], dev[3], lx=1000.0, ly=1000.0, params=p,
                   bcs=[sve.BC(sve.BC_PERIODIC)] * 4)
    sums0 = [float(torch.sum(d)) for d in (dev[0], dev[2])]
    del dev
    dts = []
    for _ in range(2):
        s.step(1, 0.5)
        dts.append(s.get_state_torch()[2])
    (gh, ghu, ghv, gz), t, dtl, ns = s.get_state_torch()
    s.close()
    assert ns == 2 and t == pytest.approx(sum(dts), rel=TOL64)
    # conservation on the periodic grid (telescoping fluxes)
    for g, s0 in ((gh, sums0[0]), (gz, sums0[1])):
        assert abs(float(torch.sum(g)) - s0) <= 1e-13 * abs(s0)
    # a 48 x 48 window on the bump's steepest slope (x ~ 350 m, y ~ 500 m),
    # plus two halo cells per side (the stencil reaches one cell per step):
    # the oracle on the window with the same time steps matches the interior
    j0, i0, w, hw = 6120, 4280, 48, 2
    sl = (slice(j0 - hw, j0 + w + hw), slice(i0 - hw, i0 + w + hw))
    o = O.Oracle2D(h[sl], hu[sl], hv[sl], zb[sl], dx, dy,
                   O.Params(law=O.LAW_GRASS, A_g=1e-3, m_g=3.0), (O.BC(O.BC_FREE),) * 4)
    for dt in dts:
        o.step_fixed_dt(1, dt)
    inner = (slice(j0, j0 + w), slice(i0, i0 + w))
    got = [g[inner].cpu().numpy() for g in (gh, ghu, ghv, gz)]
    ref = [a[hw:hw + w, hw:hw + w] for a in o.state]
    assert np.ptp(zb[inner]) > 0.01                    # the window sees the bump
    assert_fields_close(got, ref, TOL64)


def test_adjoint_1024_directional_derivatives(sve):
    import torch
    from paper_1307_0491_amd.adjoint import AdjointRun
    n, steps = 1024, 2000
    h, hu, hv, zb, dx, dy = W.dune2d(n, n)
    ag_true = W.adjoint_ag_field(n, n)
    ag0 = np.full((n, n), 1e-3)
    p = sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0)
    bcs = [sve.BC(sve.BC_PERIODIC)] * 4

    def solver(z, ag):
        return sve.Solver(h, hu, z, hv, lx=1000.0, ly=1000.0, params=p, bcs=bcs, Ag=ag)

    s = solver(zb, ag0)
    s.step(1, 0.5)
    dt = 0.9 * s.get_state()[2]
    s.close()

    def final_bed(z, ag):
        s = solver(z, ag)
        s.step_fixed_dt(steps, dt)
        zT = s.get_state()[0][3]
        s.close()
        return zT

    z_target = final_bed(zb, ag_true)

    def loss(z, ag):
        return 0.5 * np.sum((final_bed(z, ag) - z_target) ** 2)

    s = solver(zb, ag0)
    run = AdjointRun(s)
    run.forward(steps, dt)
    zT = s.get_state()[0][3]
    gT = np.zeros((4, n, n))
    gT[3] = zT - z_target
    g0, gAg = run.backward(torch.tensor(gT, device="cuda"))
    g0, gAg = g0.cpu().numpy(), gAg.cpu().numpy()
    s.close()
    assert np.all(np.isfinite(g0)) and np.all(np.isfinite(gAg))

    dA = 0.3e-3 * W.smooth_field(n, n, 1000.0, 1000.0, 50.0, seed=5)
    dz = 0.05 * W.smooth_field(n, n, 1000.0, 1000.0, 50.0, seed=6)
    for name, grad, d, shift in (("A_g", gAg, dA, lambda e: (zb, ag0 + e * dA)),
                                 ("z_b", g0[3], dz, lambda e: (zb + e * dz, ag0))):
        adj = float(np.sum(grad * d))
        fd = {}
        for eps in (1e-3, 5e-4):
            fd[eps] = (loss(*shift(eps)) - loss(*shift(-eps))) / (2.0 * eps)
        # the two step sizes agree (central differences: error ~ eps^2)
        assert abs(fd[1e-3] - fd[5e-4]) <= 4e-6 * abs(fd[5e-4]), (name, fd)
        assert abs(adj - fd[5e-4]) <= 1e-6 * abs(fd[5e-4]), (name, adj, fd)


def test_paper_bump_4000_windows(sve):
    n, nsteps, halo, w = 4000, 24, 26, 48
    h, hu, hv, zb, dx, dy = W.dune2d(n, n, base=0.1)
    p = sve.Params(law=sve.LAW_GRASS, A_g=1.0, m_g=3.0)
    bcs = [sve.BC(sve.BC_INFLOW, 9.9, 10.0, 0.0), sve.BC(sve.BC_FREE), sve.BC(sve.BC_FREE),
           sve.BC(sve.BC_FREE)]
    s = sve.Solver(h, hu, zb, hv, lx=1000.0, ly=1000.0, params=p, bcs=bcs)
    dts = []
    for _ in range(nsteps):
        s.step(1, 0.5)
        dts.append(s.times()[1])
    (gh, ghu, ghv, gz), t, dtl, ns = s.get_state()
    s.close()
    assert ns == nsteps and t == pytest.approx(sum(dts), rel=TOL64)
    po = O.Params(law=O.LAW_GRASS, A_g=1.0, m_g=3.0)
    free = O.BC(O.BC_FREE)
    inflow = O.BC(O.BC_INFLOW, 9.9, 10.0, 0.0)
    # (first row, first column) of the w x w window checked, and the rows /
    # columns of the oracle's domain around it (the grid's own boundary
    # where the window touches it, else a halo beyond the steps' reach)
    cases = {
        "bump": ((1950, 1250), (1950 - halo, 1950 + w + halo), (1250 - halo, 1250 + w + halo),
                 (free,) * 4),
        "inflow": ((2000, 0), (2000 - halo, 2000 + w + halo), (0, w + halo),
                   (inflow, free, free, free)),
        "corner": ((n - w, n - w), (n - w - halo, n), (n - w - halo, n), (free,) * 4),
    }
    for name, ((j0, i0), (ja, jb), (ia, ib), obcs) in cases.items():
        sl = (slice(ja, jb), slice(ia, ib))
        o = O.Oracle2D(h[sl], hu[sl], hv[sl], zb[sl], dx, dy, po, obcs)
        for dt in dts:
            o.step_fixed_dt(1, dt)
        inner = (slice(j0, j0 + w), slice(i0, i0 + w))
        oin = (slice(j0 - ja, j0 - ja + w), slice(i0 - ia, i0 - ia + w))
        got = [g[inner] for g in (gh, ghu, ghv, gz)]
        ref = [a[oin] for a in o.state]
        assert_fields_close(got, ref, TOL64)
        if name == "bump":
            assert np.max(np.abs(ref[3] - zb[inner])) > 1e-4       # the bed moved
            assert np.max(np.abs(ref[2])) > 1e-6                   # flow around the bump


def test_antidune_2400_to_t50_against_stored_oracle(sve):
    ref = np.load(os.path.join(GOLDEN, "antidune1d_t50.npz"))
    h, hu, zb, dx = W.antidune1d(2400)
    s = sve.Solver(h, hu, zb, lx=24.0, params=sve.Params(law=sve.LAW_GRASS, A_g=1e-3, m_g=3.0),
                   bcs=[sve.BC(sve.BC_INFLOW, 0.5, 1.7, 0.0), sve.BC(sve.BC_FREE)])
    x = (np.arange(2400) + 0.5) * dx
    crest = [x[np.argmax(zb)]]
    done = 0
    for k, t_end in enumerate(ref["times"]):
        n = int(ref[f"nsteps{k}"])
        # exactly the oracle's number of real steps, the last one clipped to
        # land on the snapshot time
        t = s.step(n - done, 0.5, float(t_end))
        done = n
        (gh, ghu, gz), t2, dtl, ns = s.get_state()
        assert t == float(t_end) and ns == n
        assert dtl == pytest.approx(float(ref[f"dt_last{k}"]), rel=1e-9)
        assert_fields_close((gh, ghu, gz), (ref[f"h{k}"], ref[f"hu{k}"], ref[f"zb{k}"]), TOL64,
                            names=("h", "hu", "z"))
        crest.append(x[np.argmax(gz)])
    s.close()
    # the antidune travels upstream (section "1D antidune evolution"): the
    # crest of the GPU state moves toward the inflow between snapshots
    assert all(b < a for a, b in zip(crest[:-1], crest[1:])), crest


@pytest.mark.parametrize("order", [1, 2])
def test_paper_dune1d_to_t700_against_stored_oracle(sve, order):
    """First order at 1e-12.  The second-order variant amplifies rounding on
    this strongly coupled dune (A_g = 1): on the oracle alone a 1e-15
    relative perturbation of the initial depth grows to 7.6e-12 in z_b by
    100 s and 1.0e-11 by 350 s (first order: below 2e-14 throughout), so its
    states are compared at 1e-10, ten times that sensitivity."""
    tol = TOL64 if order == 1 else 1e-10
    ref = np.load(os.path.join(GOLDEN, "dune1d_paper_t700.npz"))
    h, hu, zb, dx = W.dune1d(2000)
    s = sve.Solver(h, hu, zb, lx=1000.0,
                   params=sve.Params(law=sve.LAW_GRASS, A_g=1.0, m_g=3.0, order=order),
                   bcs=[sve.BC(sve.BC_PERIODIC)] * 2)
    done = 0
    pre = f"o{order}_"
    for k, t_end in enumerate(ref["times"]):
        n = int(ref[pre + f"nsteps{k}"])
        t = s.step(n - done, 0.5, float(t_end))
        done = n
        (gh, ghu, gz), t2, dtl, ns = s.get_state()
        assert t == float(t_end) and ns == n
        assert dtl == pytest.approx(float(ref[pre + f"dt_last{k}"]), rel=1e-9)
        assert_fields_close((gh, ghu, gz), (ref[pre + f"h{k}"], ref[pre + f"hu{k}"],
                                            ref[pre + f"zb{k}"]), tol,
                            names=("h", "hu", "z"))
    s.close()
    # sediment is conserved and the dune has moved downstream of its start
    assert abs(gz.sum() - zb.sum()) < 1e-11 * zb.sum()
    x = (np.arange(2000) + 0.5) * dx
    assert x[np.argmax(gz)] > x[np.argmax(zb)] + 100.0
