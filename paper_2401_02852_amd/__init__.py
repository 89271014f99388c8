"""qnae: MI355X-native statevector simulation of depth-p QAOA on k-NAE-SAT.

Thin Python binding (argument marshalling only) over the C ABI of
``libqnae.so`` (see ``include/qnae.h``). Every step of the computation runs in
the library's HIP kernels; PyTorch provides device memory and streams. There
is no fallback: without the built library every call raises.
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    PreparedBatch,
    PreparedCostBuild,
    QNAEError,
    Context,
    Result,
    Server,
    autotune_batched,
    build_cost_diagonal,
    build_cost_diagonal_z2,
    build_cost_diagonals,
    default_context,
    library_path,
    load_library,
    qaoa_grad,
    qaoa_grad_batched,
    qaoa_run,
    qaoa_run_batched,
    qaoa_run_noalloc,
    qaoa_run_z2,
    sample,
)
from .autograd import QAOAFunction  # noqa: F401
from .pretrain import running_time  # noqa: F401
