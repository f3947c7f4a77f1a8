"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package holds no part of the evaluation method: it only draws random
template genotypes (heap-ordered symbol strings) and synthetic datasets.
Encoding, evaluation, fitness and gradients live on two independent sides
(the HIP library and the CPU oracle) and neither is imported from here.
"""
from .configs import CONFIGS, LADDER, Config, get_config  # noqa: F401
from .data import make_dataset  # noqa: F401
from .population import sample_population, gom_variants, template_size  # noqa: F401
