"""MI355X-native colour-gradient lattice Boltzmann step with reaction-limited evaporation
(arXiv:2412.14859).  The compute path is the HIP library libcgevap.so behind the C-ABI
declared in include/cgevap.h; `paper_2412_14859_amd.cgevap` is its Python binding."""
