"""CPU oracle for the QS^3 hot path (arXiv 2107.00872): XXZ H.v in the fixed-N_down
and momentum bases, (thick-restart) Lanczos, observables, S^-_q and the
continued-fraction S(q, omega).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute
anything under ``oracle/``.  The HIP library never does, and this package never
imports the library: the two share no code, headers, tables or helpers.  The
only common inputs are the seeded arrays written by ``workloads.py``.

Conventions (each function cites the passage of the paper it follows):
  * sites are numbered 1..N and states are ascending down-spin tuples
    n = (n_1 < ... < n_{N_down}) as in Sec. 3.1; ranks are a = 1..C(N, N_down)
    as in Eq. (a_of_n).  ``to0``/``from0`` convert to the 0-based rank the
    library uses (rank0 = a - 1, site0 = r - 1).
  * floating point is float64 / complex128 throughout.

Readings of passages that are garbled, ambiguous or silent are marked
``READING:`` where they are applied.

Parity unpinned (no value fixed by the paper or by mathematics to check
against): the float32-matvec variant beyond its stated error bound, the
thick-restart restart counts and intermediate Ritz values, eigenvector gauge
inside degenerate eigenspaces (only projectors and observables are compared),
and the random-lattice generator of the serving stream.
"""
