"""MI355X-native MRT lattice Boltzmann kinetic model for combustion (arXiv:1411.6697)."""
