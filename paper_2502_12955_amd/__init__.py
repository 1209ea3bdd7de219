"""MI355X-native multi-component Shan-Chen lattice Boltzmann hot path (CooLBM, arXiv 2502.12955).

The solver lives in the HIP/C-ABI library ``libmclbm.so`` (sources under
``csrc/``, declarations in ``include/mclbm.h``); ``mclbm`` is its thin ctypes
binding.  ``inputs`` generates seeded synthetic workloads.  Importing the
package does not load the GPU library; ``mclbm.load()`` does, and fails
loudly when it is missing.
"""
__all__ = ["inputs", "mclbm"]
