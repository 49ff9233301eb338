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
                    momentum_friction=p.momentum_friction,
                    reconstruction=p.reconstruction, order=p.order)


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


# Every comparison made by assert_fields_close, for the parity report that
# conftest.py writes when SVE_PARITY_REPORT names a file.
RECORDS = []
CURRENT_TEST = None


def field_errors(gpu_fields, ora_fields, names=("h", "hu", "hv", "z")):
    """Relative L-infinity error per field.  Depth and bed are measured
    against their own maximum; the two momentum components against the
    largest momentum magnitude max |(hu, hv)| (they are components of one
    vector: the transverse one starts at zero and stays small, so its own
    maximum is no scale for the rounding of the momentum arithmetic).
    The transverse momentum is also measured against its own maximum
    ("hv_own"), with "hv_share" = max |hv| / max |(hu, hv)|."""
    d = dict(zip(names, ora_fields))
    if "hv" in d:
        mom = float(np.max(np.hypot(d["hu"], d["hv"])))
    else:
        mom = float(np.max(np.abs(d["hu"])))
    errs = {}
    for name, g, o in zip(names, gpu_fields, ora_fields):
        if name in ("hu", "hv"):
            num = float(np.max(np.abs(np.asarray(g) - np.asarray(o))))
            errs[name] = num / mom if mom > 0 else num
            if name == "hv":
                own = float(np.max(np.abs(o)))
                errs["hv_own"] = num / own if own > 0 else num
                errs["hv_share"] = own / mom if mom > 0 else 0.0
        else:
            errs[name] = rel_linf(g, o)
    return errs


# Where the transverse momentum reaches this share of the momentum
# magnitude, its error is also held to the parity tolerance against its own
# maximum (1e-12 in FP64, 1e-5 with float32 storage; comparisons between two
# GPU paths at tighter tolerances use 1e-12 there).
HV_OWN_SHARE = 1e-2
HV_OWN_TOL_FLOOR = 1e-12


def assert_fields_close(gpu_fields, ora_fields, tol, names=("h", "hu", "hv", "z"),
                        own_tol=None):
    """own_tol: tolerance of hv against its own maximum (default: the parity
    tolerance, at least HV_OWN_TOL_FLOOR); a test that loosens it states the
    oracle's own sensitivity that justifies it."""
    errs = field_errors(gpu_fields, ora_fields, names)
    RECORDS.append(dict(errs, tol=tol, test=CURRENT_TEST))
    msg = ", ".join(f"{k} {v:.3e}" for k, v in errs.items())
    for name in names:
        assert errs[name] <= tol, f"{name}: rel Linf {errs[name]:.3e} > {tol:.1e} ({msg})"
    if "hv" in errs and errs["hv_share"] >= HV_OWN_SHARE:
        if own_tol is None:
            own_tol = max(tol, HV_OWN_TOL_FLOOR)
        assert errs["hv_own"] <= own_tol, \
            f"hv against its own maximum: {errs['hv_own']:.3e} > {own_tol:.1e} ({msg})"
