"""Shared helpers for tests that use the HIP library."""
import os

from paper_2510_18136_amd import nsfrb


def ensure_built():
    """Load libnsfrb.so, building it first only if it is absent."""
    if not os.path.exists(nsfrb.LIB_PATH):
        from paper_2510_18136_amd import build
        build.build()
    return nsfrb.lib()
