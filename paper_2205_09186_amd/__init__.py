"""gfx950 (MI355X) implementation of the chemical-potential multiphase lattice
Boltzmann step with accurate difference schemes (Qin et al., arXiv 2205.09186).

The compute path is the HIP library ``liblbm.so`` behind the C ABI of
``include/lbm.h``; ``paper_2205_09186_amd.lbm`` is its Python binding and
``paper_2205_09186_amd.inputs`` the seeded synthetic initial states.
"""
