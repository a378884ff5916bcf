"""CPU FP64 oracle for the hypercube solver — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and the
two share no code (the seeded instance generator is the only common module,
and it holds none of the solver's arithmetic).

* ``oracle.cpu``   — ctypes wrapper of ``hq_oracle.c`` (Algorithm 1, FP64).
* ``oracle.exact`` — independent exact solvers used to pin the oracle:
  dense / sparse direct solves of the balance equations (1)-(2) with Q built
  per source state, and textbook closed forms (Erlang loss, ordered hunting).
"""
