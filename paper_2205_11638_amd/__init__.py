"""MI355X-native Lagrange-decomposition dual solver for binary programs.

The hot path (decision-diagram min-marginals, generalized min-marginal
averaging, the dual lower bound and its adjoint) runs in the HIP kernels of
``libdd.so``; this package only binds it.  Build it with
``python -m paper_2205_11638_amd.build``.
"""
from .binding import Batch, DDError, Instance, compile_row, gap_integral, lib  # noqa: F401
