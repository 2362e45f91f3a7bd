"""Plain, slow FP64 CPU oracle for the hybrid purification/sampling method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP library.

Modules (each function cites the passage of Chen & Stoudenmire,
arXiv:1910.09142, that it follows):

* ``model``   spin-1 operators, the two-leg ladder Hamiltonian, the
  closed-form Trotter gate, the hybrid MPS site layout and the Trotter
  update list.
* ``exact``   exact diagonalisation and dense (state-vector) Trotter
  products: the plain definitions the MPS path must reproduce.
* ``philox``  the Philox4x64-10 counter-based generator (Salmon et al.,
  SC'11), used for the initial product states and the collapse draws.
* ``mps``     the MPS state, two-site Trotter updates with truncated SVD,
  measurement and the sequential projective collapse.
* ``hybrid``  the Markov chain of the hybrid METTS-ancilla algorithm.
* ``observables``  long-range correlators and the susceptibility estimator.

Parity status (what pins each function, or "parity unpinned") is listed in
each module header.
"""
