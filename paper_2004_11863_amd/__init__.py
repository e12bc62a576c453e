"""MI355X-native two-level lattice-Boltzmann hot path (gfx950 HIP kernels
behind a C ABI), after Astoul et al., arXiv:2004.11863."""
