"""The allocation-free entry point (sve_step_dev_noalloc) against the
context entry points (sve_init_state_dev + sve_step + sve_get_state_dev)
on the same inputs: two calls in a row, the second on a smaller grid, must
give the same states, times and time steps, element for element; both also
match the oracle at 1e-12.  A step error leaves the last completed state in
the output arrays, as the context keeps it."""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_helpers import assert_fields_close, to_oracle_bcs, to_oracle_params

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def sve(gpu_lib):
    return gpu_lib


def dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def noalloc_run(sve, case, params, bcs, n, cfl, t_end=0.0, t0=0.0):
    """n steps through sve_step_dev_noalloc; returns (fields, t, dt_last, rc)."""
    import torch
    from paper_1307_0491_amd import _lib
    from paper_1307_0491_amd.solver import _bcs_to_c
    lib = _lib.load()
    ny, nx = case["h"].shape
    ins = [dev(case[k]) for k in ("h", "hu", "hv", "zb")]
    outs = [torch.full_like(ins[0], np.nan) for _ in range(4)]
    t = ctypes.c_double(t0)
    dtl = ctypes.c_double(-1.0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.sve_step_dev_noalloc(nx, ny, float(case["lx"]), float(case["ly"]),
                                  ctypes.byref(params.to_c()), _bcs_to_c(bcs),
                                  *[ptr(a) for a in ins], *[ptr(a) for a in outs], int(n),
                                  float(cfl), float(t_end), ctypes.byref(t), ctypes.byref(dtl),
                                  stream)
    torch.cuda.synchronize()
    return tuple(o.cpu().numpy() for o in outs), t.value, dtl.value, rc


def context_run(sve, case, params, bcs, n, cfl, t_end=0.0):
    ins = [dev(case[k]) for k in ("h", "hu", "zb", "hv")]
    s = sve.Solver(ins[0], ins[1], ins[2], ins[3], lx=case["lx"], ly=case["ly"], params=params,
                   bcs=bcs)
    rc = 0
    try:
        s.step(n, cfl, t_end)
    except sve.SveError as e:
        rc = e.code
    fields, t, dtl, ns = s.get_state()
    s.close()
    return fields, t, dtl, ns, rc


def cases(sve):
    a = W.dune2d(300, 170)
    first = dict(h=a[0], hu=a[1], hv=a[2] + 0.3 * a[3], zb=a[3], lx=1000.0, ly=1000.0)
    lx, ly = 4000.0 * 130 / 8192, 1000.0 * 75 / 2048
    b = W.mpm_channel(130, 75, lx=lx, ly=ly)
    second = dict(h=b[0], hu=b[1], hv=b[2], zb=b[3], lx=lx, ly=ly)
    free = sve.BC(sve.BC_FREE)
    return [
        (first, sve.Params(law=sve.LAW_GRASS, A_g=0.02, m_g=3.0), [sve.BC(sve.BC_PERIODIC)] * 4,
         25),
        (second, sve.Params(law=sve.LAW_MPM, friction=sve.FRIC_STRICKLER, fric_coef=40.0,
                            d_s=1e-3, s=2.65, tau_cr=0.05),
         [sve.BC(sve.BC_INFLOW, 0.5, 2.0, 0.0), free, free, free], 12),
    ]


def test_two_calls_match_the_context_entry_points(sve):
    for case, params, bcs, n in cases(sve):
        f_na, t_na, dtl_na, rc = noalloc_run(sve, case, params, bcs, n, 0.5)
        assert rc == 0
        f_cx, t_cx, dtl_cx, ns, rc_cx = context_run(sve, case, params, bcs, n, 0.5)
        assert rc_cx == 0 and ns == n
        assert t_na == t_cx and dtl_na == dtl_cx
        for a, b in zip(f_na, f_cx):
            assert np.array_equal(a, b)
        ny, nx = case["h"].shape
        o = O.Oracle2D(case["h"], case["hu"], case["hv"], case["zb"], case["lx"] / nx,
                       case["ly"] / ny, to_oracle_params(params), to_oracle_bcs(bcs))
        o.step(n, 0.5)
        assert t_na == pytest.approx(o.t, rel=TOL64)
        assert_fields_close(f_na, o.state, TOL64)


def test_odd_even_zero_steps_and_t_end(sve):
    case, params, bcs, _ = cases(sve)[0]
    for n in (0, 1, 2, 7):
        f_na, t_na, dtl_na, rc = noalloc_run(sve, case, params, bcs, n, 0.5)
        f_cx, t_cx, dtl_cx, ns, rc_cx = context_run(sve, case, params, bcs, n, 0.5)
        assert rc == 0 and t_na == t_cx
        if n > 0:
            assert dtl_na == dtl_cx
        for a, b in zip(f_na, f_cx):
            assert np.array_equal(a, b)
    # a run clipped at t_end inside the call
    f_na, t_na, _, rc = noalloc_run(sve, case, params, bcs, 40, 0.5, t_end=0.1)
    f_cx, t_cx, _, _, _ = context_run(sve, case, params, bcs, 40, 0.5, t_end=0.1)
    assert rc == 0 and t_na == t_cx == 0.1
    for a, b in zip(f_na, f_cx):
        assert np.array_equal(a, b)


def test_step_error_keeps_last_completed_state(sve):
    """CFL far beyond the limit: the call reports the step error, with the
    state and time of the last step that completed, as the context does."""
    case, params, bcs, _ = cases(sve)[0]
    f_na, t_na, _, rc = noalloc_run(sve, case, params, bcs, 50, 60.0)
    f_cx, t_cx, _, ns, rc_cx = context_run(sve, case, params, bcs, 50, 60.0)
    assert rc < 0 and rc == rc_cx
    assert t_na == t_cx
    for a, b in zip(f_na, f_cx):
        assert np.array_equal(a, b)
        assert np.all(np.isfinite(a))


def test_invalid_arguments_are_rejected(sve):
    case, params, bcs, _ = cases(sve)[0]
    bad = dict(case)
    bad["h"] = case["h"].copy()
    bad["h"][3, 4] = -1.0
    assert noalloc_run(sve, bad, params, bcs, 3, 0.5)[3] == -1
    assert noalloc_run(sve, case, params, bcs, 3, -0.5)[3] == -1
    assert noalloc_run(sve, case, params, bcs, -1, 0.5)[3] == -1
    # the variants the entry point does not run
    import dataclasses
    for change in (dict(reconstruction=1), dict(order=2)):
        assert noalloc_run(sve, case, dataclasses.replace(params, **change), bcs, 3, 0.5)[3] == -1
