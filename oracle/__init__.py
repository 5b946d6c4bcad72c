"""FP64 CPU oracle for the SRP-map hot path of Dietzen, De Sena and van
Waterschoot, "Scalable-Complexity Steered Response Power based on Low-Rank and
Sparse Interpolation" (arXiv 2306.08514).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it, and this
package imports nothing from the product.

Parity status per function is listed in the module docstring of
``oracle.srp``.
"""

from .srp import *  # noqa: F401,F403
