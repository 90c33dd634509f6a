"""The repository's build entry point compiles the HIP library for gfx950
and the C oracle, and loads the binding it built (no GPU needed)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_build_entry_point():
    sys.path.insert(0, ROOT)
    import __graft_entry__
    __graft_entry__.build()
    from paper_2212_11878_amd import mpcd
    assert os.path.exists(mpcd.LIB_PATH)
    assert mpcd.mpcd_abi_version() == mpcd.ABI_VERSION
