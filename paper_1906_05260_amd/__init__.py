"""MI355X-native VIPER rod-solver hot path (hand-written HIP for gfx950 behind a C ABI)."""
