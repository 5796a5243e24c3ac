"""Test infrastructure: a plain, slow CPU oracle of the chromodynamic MRT
lattice Boltzmann scheme of Spendlove, Xu, Halliday, Schenkel and Halliday,
"Chromodynamic multi-relaxation time lattice Boltzmann scheme for fluids with
density difference" (arXiv 2005.04642).

Nothing in the product path may import this package. Only the test-suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code with the HIP path.

Modules
-------
lattice   D2Q9 constants (float and exact-rational forms).
chromo    whole-lattice FP64 sweeps of one time step, in the paper's order.
brute     per-site scalar loops for tiny lattices (independent second copy of
          streaming, recolouring, stencils and the closed-form reconstruction).
analytic  semi-analytic reference flows (App. C, App. D) and Laplace's law.

Every function cites the passage of the paper it follows. Parts with no pin
other than agreement with the HIP path are marked "parity unpinned".
"""
