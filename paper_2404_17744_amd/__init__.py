"""MI355X-native THC second-order-exchange (SOX) self-energy.

``thcsox``  -- ctypes binding of the HIP library libthcsox (include/thcsox.h).
``synth``   -- seeded synthetic inputs shared with the test oracle.
"""
__all__ = ["thcsox", "synth"]
