"""FP64 CPU oracle for the probabilistic local-divergence path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
package: only the test suite, the smoke check and the benchmark's CPU-baseline
leg use it.  It shares no code with the HIP library (no kernels, headers,
helpers, tables or constants) and never imports it.

The oracle is written from the paper (Ouermi et al., "Efficient Probabilistic
Visualization of Local Divergence of 2D Vector Fields with Independent Gaussian
Uncertainty"): plain, slow, obviously correct numpy in float64.  The 3D
extension (pdiv_oracle3d) follows the paper's stated future work.
"""

from .pdiv_oracle import (  # noqa: F401
    moments,
    fd_divergence,
    speed_gradient,
    speed_gradient_moments,
    divergence_gaussian,
    divergence_gaussian_f32,
    vertex_probs,
    lcp,
    philox4x32_10,
    box_muller,
    mc_sample_field,
    mc_lcp,
    mc_lcp_rows,
    mc_lcp_vertex,
    marching_squares,
    marching_squares_row_counts,
    spaghetti,
)
from .pdiv_oracle3d import (  # noqa: F401
    divergence_gaussian_3d,
    divergence_gaussian_3d_f32,
    fd_divergence_3d,
    lcp_3d,
    crossed_3d,
    mc_lcp_3d,
    mc_lcp_3d_vertex,
)
