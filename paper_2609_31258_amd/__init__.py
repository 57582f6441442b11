"""MI355X-native ion-pack propagation (MuCITE time step) on HIP/gfx950.

The compute path lives in the HIP shared library built from ``csrc/``;
``paper_2609_31258_amd.mucite`` is its thin ctypes binding.  Importing the
package does not load the library: the binding loads it on first use and
raises if it has not been built.
"""
__all__ = ["synth"]
