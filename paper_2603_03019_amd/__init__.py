"""MI355X-native solver for the spatial hypercube queueing model.

The solver is the Conditional Probability Update iteration of the paper
(Algorithm 1 over the birth-death reformulation of Proposition 1), run by
hand-written HIP kernels behind the C ABI of ``include/hq.h``.

* ``paper_2603_03019_amd.hq``        — ctypes binding of libhq.so (same names as the C ABI)
* ``paper_2603_03019_amd.instances`` — seeded synthetic deployments
* ``paper_2603_03019_amd.build``     — in-tree hipcc build of libhq.so

Importing this package loads nothing; ``hq.load()`` opens the library.
"""
