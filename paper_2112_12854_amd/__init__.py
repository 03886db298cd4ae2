"""MI355X-native explicit monodomain step (Del Corso, Verzicco, Viola,
arXiv 2112.12854): tetrahedral cell-centred FV diffusion + TP06 / CRN /
Stewart cell models, as HIP kernels behind the C ABI of include/ep.h.

Modules: ep (binding of libep.so), meshgen (seeded synthetic workloads),
build (compiles libep.so)."""
