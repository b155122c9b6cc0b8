"""CPU oracle for the block-space gasket map and the passes it feeds.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark.  The HIP library and its Python binding
never import it, and it imports nothing from them.
"""
from .oracle import *  # noqa: F401,F403
