"""MI355X-native per-particle ADM1 reaction step (HIP for gfx950)."""
