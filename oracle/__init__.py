"""Plain FP64 CPU oracle for noisy many-particle continuous-time quantum walks.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path (no kernels, headers, helpers or constant tables) and imports nothing
from the product package.

What it computes (Piccinini et al., arXiv:1612.00746):

* ``basis``        -- many-particle basis of a 1-D chain (Sec. 2, the N^m
                      Hilbert space; symmetric sector for bosons).
* ``hamiltonian``  -- sparse FP64 H with deterministic + stochastic entries
                      on the diagonal and between neighbours (Eq. 1).
* ``propagate``    -- exact diagonalisation (Eqs. 3-4, Alg. 1), the Taylor
                      series of the evolution operator (Eqs. 5-7, Alg. 3) and
                      classical RK4 (Alg. 2).
* ``observables``  -- diagonal of the ensemble-averaged density matrix
                      (Eq. 2 and the post-processing stage of Algs. 1-3):
                      site occupations and the pair correlation.
* ``gradients``    -- derivative of an ensemble-averaged diagonal observable
                      with respect to the baseline hoppings / on-site
                      energies, by central finite differences and by the
                      Daleckii-Krein formula on the eigen-decomposition.  The
                      paper does not differentiate; this is a reference for
                      an extension of the method.
* ``telegraph``    -- switching (telegraph) hopping noise: the documented
                      counter-based sign process and the step-by-step
                      evolution with H rebuilt every step (Eq. 1, time
                      dependent).
* ``graph``        -- one particle on a general graph or q-dimensional
                      lattice (Sec. 2): bonds of the lattice and H from a
                      bond list.

Every function is FP64 and written for clarity, not speed.  Pins that tie the
oracle to closed forms, textbook routines and invariants live in
``tests/test_oracle_*.py``.
"""

from . import basis, hamiltonian, propagate, observables, gradients  # noqa: F401
