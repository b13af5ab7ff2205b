"""FP64 CPU oracle of the pseudo-vector lattice-BGK Maxwell scheme.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg; the product path never loads it.
"""
