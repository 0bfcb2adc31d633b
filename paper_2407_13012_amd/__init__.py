"""QAOA statevector simulation on one AMD Instinct MI355X (gfx950).

Thin ctypes binding over ``libqaoa.so`` (C ABI in ``include/qaoa.h``): the
functions below carry the C names and only marshal arguments; every step of
the computation runs in the library's HIP kernels.  PyTorch is used for device
memory (output tensors) and streams only.  If the shared library has not been
built the binding raises at load time; there is no CPU fallback.
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    QAOA_C128,
    QAOA_C64,
    QaoaError,
    LbfgsOptions,
    QaoaHandle,
    QaoaBatch,
    QaoaMpnn,
    Allocator,
    qaoa_set_allocator,
    torch_allocator,
    use_torch_allocator,
    MpnnAdam,
    qaoa_mpnn_create,
    qaoa_mpnn_destroy,
    qaoa_mpnn_get_params,
    qaoa_mpnn_loss_grad,
    qaoa_mpnn_num_params,
    qaoa_mpnn_predict,
    qaoa_mpnn_set_params,
    qaoa_mpnn_train_step,
    BatchOptions,
    batch_options,
    qaoa_batch_create,
    qaoa_batch_destroy,
    qaoa_batch_run,
    qaoa_batch_timeline,
    library_path,
    load_library,
    qaoa_cost_diagonal,
    qaoa_cost_extrema,
    qaoa_gradient_noalloc,
    qaoa_gradient_from_state,
    qaoa_create_maxcut,
    qaoa_create_poly,
    qaoa_create_qubo,
    qaoa_destroy,
    qaoa_evaluate,
    qaoa_expectation,
    qaoa_get_info,
    qaoa_gradient,
    qaoa_last_error_message,
    qaoa_lbfgs_minimize,
    qaoa_optimize,
    qaoa_pass_plan,
    qaoa_profile_enable,
    qaoa_profile_read,
    qaoa_sample,
    qaoa_statevector,
    qaoa_status_string,
)

__all__ = [name for name in dir() if name.startswith("qaoa_")] + [
    "QaoaHandle", "QaoaBatch", "QaoaMpnn", "Allocator", "torch_allocator", "use_torch_allocator", "MpnnAdam", "BatchOptions", "batch_options", "QaoaError", "QAOA_C128", "QAOA_C64", "load_library", "library_path"]
