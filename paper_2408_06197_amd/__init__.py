"""MI355X (gfx950) engine for Lancelot's encrypted pairwise squared distances
(arXiv 2408.06197): RNS-CKKS with hand-written HIP kernels behind a C ABI
(include/lancelot.h).  ``lancelot`` is the ctypes binding; ``build`` compiles
the library in-tree."""
