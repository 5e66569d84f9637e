"""Pins of the derivative the reverse-mode tests compare against: the complex-step
derivative of the oracle's 2D operator with flags and speeds frozen (Section 2.2; for
Euler the characteristic limiter and HWENO reconstruction of Remark 4).  Complex step
gives J d = Im F(U + i h d) / h to round-off for a function that is real-analytic in U;
here it is checked against central differences, whose error must fall like h^2 until
round-off takes over: a wrong branch (a non-analytic abs, a complex square root taken on
the wrong sheet, a conjugation inside the eigenvector inverse) would break the agreement."""
import numpy as np
import pytest

import hweno_inputs as hi
from oracle.scheme2d import Scheme2D


def shock_vortex(n, seed=0):
    prm = hi.euler_shock_vortex_params(seed)
    return hi.project_2d(hi.euler_shock_vortex_func(prm), 0.0, 1.0, 0.0, 1.0, n, n, nq=5)


@pytest.mark.parametrize("eq,tc,bc", [("euler", "kxrcf", "periodic"), ("euler", "all", "periodic"),
                                      ("burgers", "all", "periodic"),
                                      ("euler", "kxrcf", ("transmissive", "reflective")),
                                      ("euler", "all", ("reflective", "transmissive")),
                                      ("burgers", "kxrcf", ("transmissive", "transmissive")),
                                      ("euler", "kxrcf", "step"), ("euler", "all", "step"),
                                      ("euler", "kxrcf", "dmr")])
def test_complex_step_matches_central_differences(eq, tc, bc):
    """The wall cases: meshes with transmissive and reflective sides, where the ghost
    cells mirror the cells beside the side (the moment normal to it, and at a reflective
    side the normal momentum, negated).  The step cases: the forward step's inflow, outflow,
    walls and solid cells (Example 3.11; solid cells must get a zero derivative).  The
    double Mach reflection case: its prescribed, wall and outflow ghosts (Example 3.10)."""
    n = 10
    t = 0.0
    if bc == "dmr":
        nx, ny, t = 14, 7, 0.002
        o = Scheme2D(eq, nx, ny, 0.0, 1.0, 0.0, 0.5, ng_edge=2, tc_mode=tc, bc=bc)
        U = hi.euler_dmr_state(nx, ny, 1.0 / 14, 5)
    elif bc == "step":
        nx, ny, si, sj = 18, 10, 7, 3
        o = Scheme2D(eq, nx, ny, 0.0, 1.8, 0.0, 1.0, ng_edge=2, tc_mode=tc, bc=bc,
                     step_corner=(0.7, 0.3))
        assert o.step_ij == (si, sj)
        U = hi.euler_step_state(nx, ny, si, sj, 7)
    elif eq == "euler" and bc != "periodic":
        U = hi.euler_wall_state(n, n, 7)
    elif eq == "euler":
        U = shock_vortex(n)
    else:
        kl, a, phi = hi.burgers_modes_params(5000)
        U = hi.project_2d(hi.burgers_modes_func(kl, a, phi), 0.0, 4.0, 0.0, 4.0, n, n, nq=5)
        U[1:] += 0.02 * np.random.default_rng(3).normal(size=U[1:].shape)
    if bc not in ("step", "dmr"):
        o = Scheme2D(eq, n, n, ng_edge=2, tc_mode=tc, bc=bc)
    _, info = o.operator(U, t=t)
    T = info["T"].astype(bool)
    assert T.any()
    al = o.alphas(U)
    F = lambda X: o.operator(X, alphas=al, T_fixed=T, t=t)[0]
    d = np.random.default_rng(0).normal(size=U.shape)
    d[1:] /= 12.0
    cs = F(U + 1e-30j * d).imag / 1e-30
    errs = []
    for h in (1e-4, 1e-5, 1e-6):
        fd = (F(U + h * d) - F(U - h * d)) / (2.0 * h)
        errs.append(np.abs(fd - cs).max() / np.abs(cs).max())
    # second-order convergence of the differences towards the complex-step value
    assert 30.0 < errs[0] / errs[1] < 300.0, errs
    assert 30.0 < errs[1] / errs[2] < 300.0, errs
    assert errs[2] < 1e-4, errs
    if bc == "step":
        assert np.array_equal(cs[:, :, o.solid], 0 * cs[:, :, o.solid])
        # nor does L depend on the solid cells' values
        e = np.zeros_like(U)
        e[:, :, o.solid] = d[:, :, o.solid]
        assert np.abs(F(U + 1e-30j * e).imag).max() == 0.0
