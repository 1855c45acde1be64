"""MI355X-native hot path of an explicit electromagnetic PIC step (HIP, gfx950)."""
