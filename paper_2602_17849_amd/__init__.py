"""MI355X-native Quad Length Code (QLC) codec for e4m3 byte streams.

The codec itself is the HIP library ``libqlc.so`` (built from ``csrc/``);
``qlc`` is its thin Python binding and ``datagen`` the seeded synthetic
workload generator.  Importing the package loads nothing: the library is
opened on first use by ``paper_2602_17849_amd.qlc``.
"""
