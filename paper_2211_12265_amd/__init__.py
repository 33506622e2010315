"""MI355X-native batched CRYSTALS-Dilithium (round-3 parameter sets 2/3/5).

The hot path (Keccak sponges, NTT/INTT, A*y, rounding and hints, the Sign
rejection loop) is hand-written HIP for gfx950 in ``csrc/`` and reached
through the C-ABI library ``libdil.so`` declared in ``include/dil.h``.
``dilithium`` is the thin ctypes binding; torch only provides device memory
and streams.
"""
