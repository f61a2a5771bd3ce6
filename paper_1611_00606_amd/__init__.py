"""MI355X-native H/S generation for FLAPW (complex FP64, gfx950 HIP kernels)."""
