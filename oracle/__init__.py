"""FP64 CPU oracle of the 1D Maxwell-Bloch hot path.

Test infrastructure only: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product library never imports, links or calls
anything here, and nothing here imports the product library.
"""
from .mb_oracle import Oracle, run  # noqa: F401
