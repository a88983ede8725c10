"""MI355X additive-FFT multiplier for long binary polynomials (placeholder; the
binding is added with the HIP library)."""
