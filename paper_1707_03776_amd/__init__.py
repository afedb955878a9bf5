"""MI355X-native FFT library (placeholder: the binding is filled in with the HIP library)."""
