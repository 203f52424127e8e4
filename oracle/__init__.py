"""Plain FP64 CPU oracle for the finite-temperature DQMC sweep of the
half-filled honeycomb Hubbard model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library under
``paper_2609_14668_amd/`` and its Python binding) imports, links or runs
anything from this package; only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code,
tables or helpers with the HIP path: the lattice, hopping matrix, propagators,
Green's function, updates and observables are computed here from their
definitions with dense NumPy/SciPy linear algebra.

Modules
-------
lattice   honeycomb torus, dense hopping matrix K (Gauge-I / Gauge-II, twists),
          f(k) and the (shifted) momentum grid.             [Sec. II A, III C]
dqmc      dense propagators B_l, UDV-stabilised G, sequential Sherman-Morrison
          sweep over both spins, replay mode, Wick observables. [Sec. II B-C, III B]
tau       time-displaced G(tau,0), G(0,tau) from the block-cyclic inverse, the
          per-configuration <H_I(tau) H_I(0)> by Wick's theorem, and the
          integrals giving dD/dU and chi_F.                  [Sec. II C]
exact     U=0 closed forms, brute-force HS enumeration and Fock-space exact
          diagonalisation of the Trotterised partition function (also its
          time-displaced interaction correlator on small clusters).
stats     binning errors and integrated autocorrelation time.
philox    Philox4x32-10 counter-based generator (Salmon et al., SC'11),
          implemented from its published definition.

Parity status: every function is pinned by a test in ``tests/`` marked
``not gpu`` (closed forms, brute force, exact diagonalisation, known-answer
vectors, extended-precision inversion) except where a module header says
"parity unpinned".
"""
