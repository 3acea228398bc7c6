"""Seven-League (7L) large-step SDE simulation on AMD MI355X (gfx950).

The compute path is libsl7.so (hand-written HIP kernels + C++ host runtime,
C ABI in include/sl7.h).  This package only marshals arguments: torch
tensors serve as device buffers and streams.
"""
from ._lib import (BF16, CIR, F16, F32, F64, GBM, OU, PWL32, PWL64, RELU, SOFTPLUS,  # noqa: F401
                   Sl7Error)
from .api import (Mlp, PRECISIONS, Problem, SL7Adjoint, SL7TrainLoss, adjoint, autotune,  # noqa: F401
                  autotune_batched, eval_H, gh_nodes, labels, pwl_compile, simulate,
                  simulate_batched, simulate_cdc, simulate_noalloc, stats_from_tensor, train, train_grad)
