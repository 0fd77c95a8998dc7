"""MI355X-native GAVIS visibility-field path (placeholder; filled below)."""
