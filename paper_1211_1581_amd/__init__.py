"""MI355X-native CSR SpMV and conjugate-gradient library (gfx950 HIP kernels
behind a C ABI).  ``paper_1211_1581_amd.spcg`` is the binding; ``inputs``
builds seeded synthetic workloads."""
