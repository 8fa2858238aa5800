"""MI355X-native multigroup, time-dependent Monte Carlo particle tracker.

The tracking runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in include/mcdc.h (libmcdc_hip.so, built in-tree).  This package
is the thin Python binding: the same entry-point names, PyTorch tensors for
device memory and the stream, and nothing else.
"""
from ._binding import (MCDCError, MLP, Problem, lib, mcdc_mlp_create,  # noqa: F401
                       mcdc_problem_create, mcdc_problem_destroy, mcdc_problem_tally_shape,
                       mcdc_run, mcdc_run_batched, mcdc_run_eigenvalue, mcdc_set_weight_windows)
