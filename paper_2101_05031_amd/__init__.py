"""MI355X-native convolution-surface lattice slicer (placeholder; binding added with the native library)."""
