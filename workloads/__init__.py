"""Seeded synthetic inputs for FCTN completion, shared by the oracle-side and
GPU-side tests and by bench.py.

This package holds input generation only: ground-truth tensors, Bernoulli
masks, observed tensors, the N(0, 1) initial factors (also the counter-based
seeded stream the library draws them from when given no factors) and the
N(0, 1) draws for rank growth.  It performs none of
the completion method's arithmetic (no sub-networks, Gram products, solves
or X updates) and imports neither the oracle nor the GPU library.
"""

from .generators import (  # noqa: F401
    CONFIGS, Problem, make_problem, init_factors, bernoulli_mask,
    factor_shapes_of, lowrank_order3, lowrank_order5, color_image, video, multispectral,
    multitemporal, serving_requests, rank_growth_draws, seeded_normal_factors,
)
