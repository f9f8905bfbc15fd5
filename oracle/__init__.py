"""Python access to the FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark import this package.  The product library never does.
"""
from .oracle import (  # noqa: F401
    Process, EventInfo, build, lib, philox4x32_10, event_k53, bin_from_k53,
    vegas_map, vegas_refine, massless_volume, phase_space, cuts, pdf_xf,
    colour_matrix, orderings, partial_amplitudes, me2_sum, me2_sum_hel,
    me2_sum_fullcolour, event_weight, event_weight_y, integrate, combine,
    neumaier_sum, ttx_dweight_dmt_analytic, n_dims, all_helicities,
    unweight_uniform, unweight, lab_event, event_weights, colour_lc, me2_sum_lc,
    colour_count, colour_config, colour_factors, me2_sum_colour_config,
    flow_count, flow_code, flow_weight, flow_total, flow_config, flow_factors, me2_sum_colour_flow, me2_sum_sampled,
    hel_count, hel_config, me2_hel, colour_matrix_relabel, dressed_amplitude, pdf_xq, me2_qqbar_ttx,
    qqbar_ttxg_diagrams, qqbar_ttxg_colour, me2_qqbar_ttxg,
    qqbar_ttxgg_terms, qqbar_ttxgg_colour, qqbar_ttxgg_colour_matrix, me2_qqbar_ttxgg,
)
