"""Seeded synthetic fragment generators shared by the tests, the benchmark and
the oracle's golden-value script.

This package holds input generation only: orbital energies, density-fitted
electron-repulsion blocks and amplitudes of the shapes the paper's embedded
clusters have.  None of the (T) arithmetic lives here.
"""

from .fragments import (  # noqa: F401
    Fragment,
    make_fragment,
    workload_fragment,
    batch_shapes,
    ov_factors,
    df_factors,
    mp2_inputs,
    WORKLOADS,
)
