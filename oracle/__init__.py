"""Exact CPU oracle for the permanent path.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_1606_05836_amd``) never imports it and shares no code with it.
"""
from .exact import (  # noqa: F401
    gray,
    delta_of_word,
    to_gaussian_integers,
    perm_brute_int,
    ryser_subsets_int,
    ryser_paired_int,
    ryser_gray_raw,
    glynn_direct_raw,
    glynn_gray_raw,
    glynn_gray_int,
    perm_exact,
    to_complex,
    rel_err,
    minor,
    minor_perm_exact,
    certify_int_exact,
)
from .pool import perm_exact_parallel, glynn_raw_parallel, host_cores, split_range  # noqa: F401
from .boson import (  # noqa: F401
    gather_u_st,
    occupation_factorials,
    prob_exact,
    perm_multiplicity,
    prob_multiplicity,
)
from .sampler import (  # noqa: F401
    columns_of_inputs,
    step_weights,
    choose,
    sample_exact,
    sampler_distribution,
)
