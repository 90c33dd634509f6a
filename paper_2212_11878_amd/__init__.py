"""MI355X-native Stochastic Rotation Dynamics (MPCD) step.

The compute path is the HIP library ``libmpcd.so`` (sources in ``csrc/``,
C ABI in ``include/mpcd.h``); ``mpcd`` is its ctypes binding.  Importing this
package loads nothing: ``from paper_2212_11878_amd import mpcd`` loads the
library and fails loudly if it has not been built.
"""
__all__ = ["mpcd", "inputs", "serve"]
