"""Seeded synthetic draws for the random cone programs of Sect. 6 (random
cone programs).

This package holds only random draws (cone sizes, the vector z, the sparse
pattern and values of A, x*, and the parametric family's theta and B). It
contains none of the solver's arithmetic: turning a draw into problem data
(s* = Pi_K(z), y* = s* - z, b = A x* + s*, c = -A^T y*) needs a cone
projection, and each consumer (the CPU oracle, the GPU library) does that
with its own projection.
"""

from .random_cone import (  # noqa: F401
    ConeSpec,
    Draw,
    draw_instance,
    draw_lp,
    draw_socp,
    draw_mixed,
    draw_batch_member,
    draw_parametric_family,
    draw_theta,
    sample_sparse_pattern,
)
from .structured import Program, lasso, logreg, portfolio, rpca  # noqa: F401,E402
