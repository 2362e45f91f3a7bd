"""MI355X (gfx950) library for the hot path of the hybrid purification /
sampling method for thermal quantum systems (Chen & Stoudenmire,
arXiv:1910.09142): Trotter evolution of the hybrid METTS-ancilla MPS with
truncated Jacobi SVDs, measurement and projective collapse, all in HIP
kernels behind the C ABI of include/hmps.h.  ``hmps`` is the ctypes
binding, ``workloads`` the synthetic ladder inputs, ``build`` the hipcc
build of libhmps.so."""
