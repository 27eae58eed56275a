"""FP64 CPU oracle of the HyRF render step (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  The product path never imports it.
"""
from .hyrf_oracle import *  # noqa: F401,F403
