"""MI355X-native PCF Learned Sort: HIP kernels for gfx950 behind a C ABI."""
