"""MI355X (gfx950) engine for the chi(2) split-step Fourier z-loop of BRAHMS
(arXiv 2609.08384).  The compute path is the HIP library libbrahms.so behind
the C ABI of include/brahms.h; `brahms` is its Python binding and `inputs`
builds seeded synthetic workloads."""
