"""MI355X-native mixed-precision column interpolative decomposition.

A ~= A(:, J) P with P = [I  T] Z^T, T = R11^{-1} R12, from a rank-k
column-pivoted Householder QR (Dunton & Fox, arXiv 2012.00706, Section 1.1 and
Algorithms 1-2).  The numerical work runs in the HIP kernels of libmpid.so;
this package only marshals arguments.
"""
from .api import (  # noqa: F401
    PREC,
    RULE,
    ColumnID,
    ColumnIDResult,
    FactorResult,
    backward,
    colmajor,
    column_id,
    empty_colmajor,
    factor,
    factor_noalloc,
    kcap_of,
    last_profile,
    make_opts,
    SketchIDResult,
    reconstruct,
    round_,
    sketch,
    sketch_id,
    solve_T,
    workspace_size,
)
from ._lib import C, MpidError, load  # noqa: F401
from .batched import (  # noqa: F401
    BatchedID,
    BatchItemResult,
    LockstepID,
    autotune,
    factor_batched,
    factor_lockstep,
)
