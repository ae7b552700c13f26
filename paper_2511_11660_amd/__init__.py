"""MI355X-native static-timing hot path (Elmore RC, NLDM, levelized AT/slew
forward, RAT/slack backward, WNS/TNS) behind the C ABI in ``include/sta.h``.

``sta`` is the ctypes binding of ``libsta.so``; ``synth`` generates seeded
synthetic designs.
"""
