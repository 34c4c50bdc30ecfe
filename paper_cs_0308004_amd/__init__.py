"""MI355X-native DPG (distribute-probe-gather) record retrieval.

The compute path lives in the HIP library ``libdpg.so`` (sources under
``csrc/``, C-ABI declared in ``include/dpg.h``); :mod:`.dpg` is the thin ctypes
binding over it and :mod:`.synth` makes seeded synthetic inputs.  Importing this
package loads nothing: the binding loads the library on first use and raises if
it has not been built.
"""

__all__ = ["dpg", "synth"]
