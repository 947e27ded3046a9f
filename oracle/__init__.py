"""FP64 CPU oracle of the IFU datacube forward model and its adjoint.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package. The product path (the HIP library and its Python binding) never imports,
links or calls anything here, and nothing here imports the product path.
"""
from .rubix_oracle import *  # noqa: F401,F403
