"""MI355X-native stochastic estimation of fermion-determinant ratios
det(D'^+ D') / det(D^+ D) for the Wilson-Dirac operator, its Dirichlet
domain blocks and the domain-decomposition Schur complement (Leder,
Finkenrath, Knechtli, "Fermions as global correction in lattice QCD").

The compute path is the HIP library ``libwdr.so`` (C ABI in
``include/wdr.h``); ``paper_1112_1243_amd.wdr`` is its thin Python binding.
Importing this package loads nothing; ``synth`` generates seeded inputs.
"""
