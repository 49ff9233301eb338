"""Plain FP64 CPU oracle of the Saint-Venant--Exner relaxation scheme.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may use it.  It shares no code with the HIP
path; the only module both sides read is the seeded input generator
``workloads``, which holds no arithmetic of the scheme.

The oracle follows the paper's method step by step:
  * model: the coupled shallow-water/Exner system (eq. "bedload system")
    with the Grass law (eq. "bedload Grass") or the threshold laws
    (eqs. "MPM" ... "Camenen") fed by the Darcy-Weisbach or Manning
    friction slope (section "Bedload modelling");
  * relaxation system (eqs. "relaxh" ... "relaxqs"), sub-characteristic
    bounds (eq. "ab"), lambda = 0 projection and homogeneous Riemann
    problem per interface, cell average (section "Numerical method");
  * 2D by the method of lines on a structured mesh (section
    "Parallelization");
  * the well-balanced (hydrostatic reconstruction) and second-order
    (MUSCL and Heun, ``oracle.second_order``) variants that the paper
    names as future work.
The explicit Riemann solution of the relaxation system is not printed in
the paper; ``oracle.riemann`` derives it from the relaxation system's jump
conditions (the derivation and the readings of silent points are listed in
that module's docstring).

Every routine works on float64 arrays and, unchanged, on complex128 arrays
for complex-step tangents (comparisons and max/min/abs use real parts).
"""
from .closures import (LAW_GRASS, LAW_MPM, LAW_FLVB, LAW_NIELSEN,
                       LAW_RIBBERINK, LAW_CAMENEN, FRIC_STRICKLER,
                       FRIC_MANNING, FRIC_DARCY, Params, closure)
from .riemann import (B_FLOOR, CellState, InterfaceResult, interface_solve,
                      ERR_POSITIVITY, ERR_ORDER, ERR_NONFINITE)
from .scheme import (BC_PERIODIC, BC_FREE, BC_INFLOW, BC, Oracle1D, Oracle2D,
                     OracleError)

__all__ = [
    "LAW_GRASS", "LAW_MPM", "LAW_FLVB", "LAW_NIELSEN", "LAW_RIBBERINK",
    "LAW_CAMENEN", "FRIC_STRICKLER", "FRIC_MANNING", "FRIC_DARCY", "Params",
    "closure", "B_FLOOR", "CellState", "InterfaceResult", "interface_solve",
    "ERR_POSITIVITY", "ERR_ORDER", "ERR_NONFINITE", "BC_PERIODIC", "BC_FREE",
    "BC_INFLOW", "BC", "Oracle1D", "Oracle2D", "OracleError",
]
