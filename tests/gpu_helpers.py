"""Shared helpers of the GPU parity tests: oracle runs and comparisons."""
import numpy as np

import oracle as O
import workloads as W


def rel_linf(a, b):
    """max |a - b| / max |b| (0 when both are zero)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b))
    num = np.max(np.abs(a - b))
    if den == 0.0:
        return num
    return num / den


def to_oracle_params(p):
    return O.Params(law=p.law, g=p.g, A_g=p.A_g, m_g=p.m_g, friction=p.friction,
                    fric_coef=p.fric_coef, d_s=p.d_s, s=p.s, tau_cr=p.tau_cr,
                    momentum_friction=p.momentum_friction)


def to_oracle_bcs(bcs):
    return tuple(O.BC(b.kind, b.h, b.hu, b.hv) for b in bcs)


def dune2d_case(nx, ny):
    h, hu, hv, zb, dx, dy = W.dune2d(nx, ny)
    return dict(h=h, hu=hu, hv=hv, zb=zb, lx=1000.0, ly=1000.0)


def mpm_case(nx, ny):
    lx = 4000.0 * nx / 8192
    ly = 1000.0 * ny / 2048
    h, hu, hv, zb, dx, dy = W.mpm_channel(nx, ny, lx=lx, ly=ly)
    return dict(h=h, hu=hu, hv=hv, zb=zb, lx=lx, ly=ly)


def assert_fields_close(gpu_fields, ora_fields, tol, names=("h", "hu", "hv", "z")):
    for name, g, o in zip(names, gpu_fields, ora_fields):
        err = rel_linf(g, o)
        assert err <= tol, f"{name}: rel Linf {err:.3e} > {tol:.1e}"
