"""Plain, slow, FP64 CPU oracle of one projection time step (test infrastructure).

This package is test infrastructure only.  It exists to check the GPU library
against the paper's statement of the scheme; the library never imports,
links or calls it, and it shares no code with the library.  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark use it.

It follows Sections 2.1-2.2 of Korhonen et al., "A GPU-accelerated
computational fluid dynamics solver for assessing shear-driven indoor airflow
and virus transmission by scale-resolved simulations" (arXiv 2204.02107):
numpy float64, periodic shifts with ``np.roll`` and ``numpy.fft.rfftn`` /
``irfftn`` for the Poisson solve.  Arrays have shape (nz, ny, nx) (x fastest);
axis a = 0, 1, 2 means x, y, z.

Parity status: everything here is pinned by the tests under ``tests/test_oracle_*.py`` (closed forms,
invariants, brute-force loops on tiny grids, dense linear algebra).  The
immersed-boundary iteration on masked grids is pinned iterate by iterate
against the same iteration written with dense difference matrices built from
the cell indices and a dense pseudo-inverse, and its fixed point against a
dense solve of the masked pressure equation.
"""
from .ops import (shift, ddx, div, grad, lap, conv_skew, conv_scalar, lap_masked,
                  delta6, filter6, poisson_symbol, poisson_solve, ib_rhs)
from .step import OracleParams, OracleState, Oracle, momentum_rhs, scalar_rhs

__all__ = [
    "shift", "ddx", "div", "grad", "lap", "conv_skew", "conv_scalar", "lap_masked",
    "delta6", "filter6", "poisson_symbol", "poisson_solve", "ib_rhs",
    "OracleParams", "OracleState", "Oracle", "momentum_rhs", "scalar_rhs",
]
