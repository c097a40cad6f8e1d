"""MI355X-native batched scene placement (Sceniris-style hot path).

The compute path is the C-ABI library ``libscn.so`` (hand-written HIP for
gfx950, declared in ``include/scn.h``); :mod:`paper_2512_16896_amd.scn` is
its thin ctypes binding.  :mod:`paper_2512_16896_amd.scenegen` draws seeded
synthetic inputs.
"""
