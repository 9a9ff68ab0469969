"""MI355X (gfx950) permanents: Gray-code BB/FG (Glynn) and Ryser sweeps in HIP.

The computation lives in libpermhip.so (C ABI: include/permhip.h); this
package is its Python binding plus a torch.autograd.Function wrapper.
"""
from .permhip import (  # noqa: F401
    PermhipError,
    Plan,
    boson_probs,
    boson_probs_grad,
    boson_sample,
    sample_inputs,
    fp64_peak,
    lib,
    perm,
    perm_batched,
    perm_chunk_log2,
    perm_combine,
    perm_partial,
    gray_terms,
    perm_grad,
    perm_row_minors,
    perm_ryser_paired,
    version,
)
from . import segments  # noqa: F401
from .autograd import BosonProbsFn, PermFn, boson_probabilities, permanent  # noqa: F401
