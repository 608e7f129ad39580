"""MI355X-native MTTKRP / TTMc library (Deinsum's local multilinear kernels)."""
