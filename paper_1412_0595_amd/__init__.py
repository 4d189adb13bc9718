"""MI355X-native spiking-network timestep: Traub-Miles HH integration, spike
compaction and CSR spike propagation as hand-written HIP kernels for gfx950,
behind a C ABI (include/snn.h)."""
