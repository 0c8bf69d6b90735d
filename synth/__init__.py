"""Seeded synthetic inputs shared by the oracle-side tests and the HIP-side tests and bench.

This package holds input synthesis only: smooth analytic vector fields made of
sources, sinks and vortices, per-point spread, ensemble members, isovalue picks
and request streams.  It contains none of the method's arithmetic (no
finite-difference divergence, no Gaussian propagation, no level-crossing
probability), so neither side of a parity test can borrow the other's maths
through it.
"""

from .fields import (  # noqa: F401
    SEED_BASE,
    Feature,
    gen_features,
    mean_field,
    analytic_divergence,
    quantile_isovalues,
    smooth_std_map,
    gen_moments,
    gen_moments_3d,
    analytic_divergence_3d,
    gen_ensemble,
    config_c1,
    config_c2,
    config_c3,
    config_c3_low_spread,
    config_c4,
    batch_sizes,
    request_stream,
)
