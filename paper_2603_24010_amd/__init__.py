"""MI355X-native circuit-coupled 1D electrostatic PIC step (arXiv 2603.24010).

The compute path is the HIP library ``libgapsim.so`` (C ABI declared in
``include/gapsim.h``); ``gapsim`` is its thin ctypes binding.  Importing this
package loads nothing: ``workloads`` (seeded inputs) stays usable without a GPU.
"""
__all__ = ["gapsim", "workloads"]
