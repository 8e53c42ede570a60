"""qFlex-style random-circuit amplitude contraction for AMD MI355X (gfx950).

The computation runs in the HIP library libqfmi.so (C-ABI: include/qfmi.h); this package
is its thin Python binding.  Build the library with `python -m paper_1905_00444_amd.build`.
"""
from .api import Context, Circuit, Plan, PRECISIONS, cgemm, permute, time_cgemm, time_permute  # noqa: F401
from .api import profile_enable, profile_read, read_circuit_text  # noqa: F401
from .api import split_bf16, split_f16, cgemm_presplit, time_cgemm_presplit  # noqa: F401
from .api import autotune, tuned_variant, amplitudes, time_ceiling  # noqa: F401
