"""Python binding of libhpeps, the MI355X PEPS einsumsvd / boundary-contraction
library (arguments marshalling only: every step runs in the HIP kernels of
``csrc/``).  PyTorch provides device memory and the stream.

The library must have been built (``python -m paper_2006_15234_amd.build`` or
``__graft_entry__.build()``); importing the functions that need it raises
``RuntimeError`` when ``libhpeps.so`` is missing.  There is no CPU fallback.
"""
from ._ffi import (  # noqa: F401
    ABSORB_CARRY, ABSORB_LEFT, ABSORB_NONE, ABSORB_RIGHT, ABSORB_SQRT, F32, F64, C128, L2R, R2L,
    HpepsError, Context, EsvdOpts, lib_path, load_library, symbols,
)
from .api import (  # noqa: F401
    einsumsvd, einsumsvd_batched, einsumsvd_backward, einsumsvd_autograd, einsumsvd_zipup, einsumsvd_pair, einsumsvd_pair_backward, einsumsvd_pair_autograd,
    peps_norm, peps_amplitude, peps_amplitudes, boundary_contract_row, peps_energy, peps_energy_uncached,
    peps_trotter_expectation, peps_norm_backward, peps_energy_backward,
    peps_energy_autograd,
    apply_one_site_gate, apply_two_site_gate, ItePlan, CircuitPlan, get_info, workspace_peak, sketch, make_opts, profile_start, profile_stop,
    profile_read, profile_by_shape, autotune_enable, autotune_export, autotune_import, autotune_save,
    autotune_load,
)
