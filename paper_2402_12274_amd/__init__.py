"""MI355X-native datatype flatten and pack/unpack engine.

``paper_2402_12274_amd.mdt`` is the ctypes binding of ``libmdt.so`` (the
C ABI declared in ``include/mdt.h``); importing it loads the library and
fails loudly if it has not been built.  ``inputs`` holds the seeded
synthetic input descriptions.
"""
