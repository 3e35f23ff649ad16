"""Plain, slow, FP64 CPU oracle of the local volume-conserving phase-field lattice
Boltzmann model (Xiong, Wang & Liu, arXiv 2505.10899).

TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import it.
The HIP library never calls it, and it shares no code with the HIP library: it
takes case parameters and initial fields from the neutral ``workloads`` module and
does every step of the method itself, in numpy, in the order of the paper's Sect. 3.

Parity pins: see ``tests/test_oracle_*.py``.  Every function here is pinned by at
least one closed form, invariant, special case or brute-force check, except where a
docstring says "parity unpinned".
"""
from .lattice import D2Q9, D3Q19, Lattice, lattice_for
from .model import Model, observables_from_phi, observables_by_labels, derived_observables

__all__ = ["D2Q9", "D3Q19", "Lattice", "lattice_for", "Model", "observables_from_phi",
           "derived_observables", "observables_by_labels"]
