"""MI355X-native reduced-order material point method.

The compute path is the HIP library ``libmpmrom.so`` (sources in ``csrc/``,
C-ABI declared in ``include/mpmrom.h``); ``binding`` exposes its entry
points to Python with argument marshalling only.  ``scenes`` generates the
seeded synthetic inputs.  Importing the package does not load the library.
"""
__all__ = ["binding", "scenes"]
