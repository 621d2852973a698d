"""MI355X-native batched non-holonomic trajectory optimizer (gfx950 HIP behind a C-ABI)."""
