"""MI355X-native SG-Splatting rasteriser: HIP kernels behind a C-ABI."""
