"""libsortrace: MI355X (gfx950) adaptive merge sort behind a C ABI.

``paper_1609_04471_amd.sortrace`` is the thin ctypes binding of
``libsortrace.so`` (hand-written HIP kernels; see ``csrc/``).  Nothing is
imported eagerly, so the input generators in ``inputs`` load without a GPU.
"""
