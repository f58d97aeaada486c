"""MI355X-native FFT nonlinear-stencil American option pricing (arXiv 2303.02317)."""
